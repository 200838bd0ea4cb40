// Context setup: dipole list, FFT plans and twiddles, the Fourier-transformed interaction tensor
// (stored for one octant only: every component is even or odd along each axis), work buffers,
// and the host side of the interaction-matrix product.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "matvec_kernels.hpp"

namespace dda {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
const char *last_error() { return g_last_error.c_str(); }

dda_status device_alloc(void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        set_error(std::string("hipMalloc of ") + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? DDA_ENOMEM : DDA_EHIP;
    }
    return DDA_OK;
}

// ------------------------------------------------------------------------ plans
static bool five_smooth(int L) {
    if (L < 1) return false;
    for (int p : {2, 3, 5})
        while (L % p == 0) L /= p;
    return L == 1;
}

// Padded length of an axis of n cells: at least 2n - 1 (the circulant embedding of the Toeplitz
// interaction), 5-smooth, with at most 64 threads per line in the z pass (one column of three
// lines per block; zmul_tpl); a length with compile-time specialized kernels is preferred when it
// costs at most 25 % more than the smallest admissible one.
static bool admissible(int L) {
    if (!five_smooth(L)) return false;
    const FftPlan p = make_plan(L, kMaxRadixZ, false);
    return p.npass > 0 && zmul_tpl(p) <= 64;
}
static int smallest_pad(int n) {
    int L = std::max(1, 2 * n - 1);
    while (!admissible(L)) ++L;
#define DDA_SPEC_ITEM(S) S,
    static const int spec[] = {DDA_SPECIALIZED_LENGTHS(DDA_SPEC_ITEM)};
#undef DDA_SPEC_ITEM
    for (int S : spec)
        if (S >= L) {
            if (4 * S <= 5 * L) L = S;
            break;
        }
    return L;
}

// the padded length dda_setup chooses for an axis of n cells
int default_pad(int n) { return smallest_pad(n); }

// lines per block (a power of two, returned as its log2): up to DDA_MAX_THREADS threads,
// preferably a whole number of waves, LDS within DDA_LDS_CAP
static int pick_lines_log2(int tpl, int line_bytes, int ndim, int want, int maxt = DDA_MAX_THREADS) {
    int nl = want > 0 ? want : std::max(1, maxt / tpl);
    if (want <= 0) nl = std::min(nl, std::max(ndim, 1));
    int l = 0;
    while ((2 << l) <= nl) ++l;  // round down to a power of two
    if (want <= 0)
        while ((((1 << l) * tpl) % 64) != 0 && ((2 << l) * tpl) <= maxt) ++l;  // whole waves if possible
    while (l > 0 && (((1 << l) * tpl) > maxt || (size_t)(1 << l) * line_bytes > DDA_LDS_CAP)) --l;
    return l;
}

// --------------------------------------------------------------------- kernels
__device__ __forceinline__ void comp_ab(int comp, int &a, int &b) {
    const int A[6] = {0, 0, 0, 1, 1, 2}, B[6] = {0, 1, 2, 1, 2, 2};
    a = A[comp];
    b = B[comp];
}

// displacement of circulant index i on an axis of n cells padded to L, or INT_MIN if unused
__device__ __forceinline__ int disp(int i, int n, int L) {
    if (i < n) return i;
    if (i > L - n) return i - L;
    return -0x40000000;
}

__global__ void k_gfill(double2 *__restrict__ buf, int comp, int nx, int ny, int nz, int Lx, int Ly, int Lz,
                        double k) {
    const size_t total = (size_t)Lx * Ly * Lz;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int ix = (int)(e % Lx);
    const int iy = (int)((e / Lx) % Ly);
    const int iz = (int)(e / ((size_t)Lx * Ly));
    const int dx = disp(ix, nx, Lx), dy = disp(iy, ny, Ly), dz = disp(iz, nz, Lz);
    double2 out = make_double2(0.0, 0.0);
    if (dx > -0x40000000 && dy > -0x40000000 && dz > -0x40000000 && (dx | dy | dz) != 0) {
        // G = exp(ikr)/r^3 [ (k^2 r^2 - 1 + i kr) delta_ab + (3 - k^2 r^2 - 3 i kr) rh_a rh_b ]
        const double fx = dx, fy = dy, fz = dz;
        const double r2 = fx * fx + fy * fy + fz * fz;
        const double r = sqrt(r2);
        const double kr = k * r;
        double sn, cs;
        sincos(kr, &sn, &cs);
        const double inv_r3 = 1.0 / (r2 * r);
        int a, b;
        comp_ab(comp, a, b);
        const double ra = (a == 0 ? fx : a == 1 ? fy : fz) / r;
        const double rb = (b == 0 ? fx : b == 1 ? fy : fz) / r;
        const double rr = ra * rb;
        const double dlt = (a == b) ? 1.0 : 0.0;
        const double k2r2 = kr * kr;
        const double qre = (k2r2 - 1.0) * dlt + (3.0 - k2r2) * rr;
        const double qim = kr * dlt - 3.0 * kr * rr;
        out.x = inv_r3 * (cs * qre - sn * qim);
        out.y = inv_r3 * (sn * qre + cs * qim);
    }
    buf[e] = out;
}

__global__ void __launch_bounds__(DDA_MAX_THREADS) k_fft_axis(double2 *__restrict__ buf, int nu, int nv, long su, long sv,
                                                   long sp, FftPlan pl, const double2 *__restrict__ twall,
                                                   int NL, int lanes_over_lines) {
    using C = double2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const C *tw = twall + pl.tw_off;
    const int L = pl.L, TPL = pl.tpl, S = lds_line_stride(L);
    const int utiles = (nu + NL - 1) / NL;
    const int u0 = (blockIdx.x % utiles) * NL;
    const int v = blockIdx.x / utiles;
    const int t = threadIdx.x;
    const int gline = lanes_over_lines ? t % NL : t / TPL;
    const int gj = lanes_over_lines ? t / NL : t % TPL;
    const bool ok = u0 + gline < nu;
    C *base = buf + (size_t)(ok ? u0 + gline : 0) * su + (size_t)v * sv;
    {
        const int R0 = pl.radix[0];
        for (int jb = gj; jb < L / R0; jb += TPL) {
            C a[kMaxRadix];
            load_rt<-1, kMaxRadix>(a, R0, jb, L, 1, tw,
                                   [&](int i) -> C { return ok ? base[(size_t)i * sp] : czero<C>(); });
            C *ln = lds + gline * S;
            store_rt<kMaxRadix>(a, R0, jb, 1, [&](int i, C val) { ln[pidx(i)] = val; });
        }
    }
    __syncthreads();
    lds_passes<-1, kMaxRadix, 0, false>(lds + (t / TPL) * S, pl, 1, pl.npass - 1, t % TPL, tw);
    if (pl.npass >= 2) {
        const int p = pl.npass - 1, Rp = pl.radix[p], Ns = pl.ns[p];
        for (int jb = gj; jb < L / Rp; jb += TPL) {
            C a[kMaxRadix];
            const C *ln = lds + gline * S;
            load_rt<-1, kMaxRadix>(a, Rp, jb, L, Ns, tw, [&](int i) { return ln[pidx(i)]; });
            if (ok) store_rt<kMaxRadix>(a, Rp, jb, Ns, [&](int i, C val) { base[(size_t)i * sp] = val; });
        }
    } else if (ok) {
        for (int i = gj; i < L; i += TPL) base[(size_t)i * sp] = lds[gline * S + pidx(i)];
    }
}

__global__ void k_gextract(const double2 *__restrict__ buf, double2 *__restrict__ Gh, int comp, int Lx, int Ly,
                           int Lz) {
    const int hx = Lx / 2 + 1, hy = Ly / 2 + 1, hz = Lz / 2 + 1;
    const size_t total = (size_t)hx * hy * hz;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int kz = (int)(e % hz);
    const int kx = (int)((e / hz) % hx);
    const int ky = (int)(e / ((size_t)hz * hx));
    // [ky][kx][comp][kz]
    Gh[(((size_t)ky * hx + kx) * 6 + comp) * hz + kz] = buf[((size_t)kz * Ly + ky) * Lx + kx];
}

__global__ void k_to_f32(const double2 *__restrict__ a, float2 *__restrict__ b, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

// ------------------------------------------------------------------- host side
void launch_to_f32(const double2 *a, float2 *b, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
}

static void alpha_of(int pol, double kd, const dda_beam &b, double mr, double mi, double &re, double &im);

void polarizability(const Ctx &c, const dda_beam &b, double &re, double &im) {
    if (wrapped(c)) {
        re = 1.0;
        im = 0.0;
        return;
    }
    polarizability_of(c, b, c.m_re, c.m_im, re, im);
}

void polarizability_comp(const Ctx &c, const dda_beam &b, double mr, double mi, int comp, double &re, double &im) {
    if (c.polarizability != DDA_POL_CLDR) {
        polarizability_of(c, b, mr, mi, re, im);
        return;
    }
    // CLDR (Gutkowicz-Krusin & Draine 2004): LDR's S replaced by a_comp^2, polarization-free
    dda_beam t = b;
    for (int a = 0; a < 3; ++a) {
        t.pol_re[a] = a == comp ? 1.0 : 0.0;
        t.pol_im[a] = 0.0;
    }
    // LDR with e = the unit vector of the component gives S = a_comp^2
    alpha_of(DDA_POL_LDR, c.kd, t, mr, mi, re, im);
}

void polarizability_of(const Ctx &c, const dda_beam &b, double mr, double mi, double &re, double &im) {
    alpha_of(c.polarizability == DDA_POL_CLDR ? DDA_POL_LDR : c.polarizability, c.kd, b, mr, mi, re, im);
}

static void alpha_of(int pol, double kd, const dda_beam &b, double mr, double mi, double &re, double &im) {
    // Clausius-Mossotti for a unit cube: (3/4pi)(m^2-1)/(m^2+2)
    const double m2r = mr * mr - mi * mi, m2i = 2 * mr * mi;
    const double nr = m2r - 1, ni = m2i, dr = m2r + 2, di = m2i;
    const double den = dr * dr + di * di;
    const double f = 3.0 / (4.0 * M_PI);
    const double cmr = f * (nr * dr + ni * di) / den, cmi = f * (ni * dr - nr * di) / den;
    if (pol == DDA_POL_CM) {
        re = cmr;
        im = cmi;
        return;
    }
    if (pol == DDA_POL_RR) {
        // radiative-reaction correction (Draine 1988): 1/alpha = 1/alpha_CM - (2/3) i k^3
        const double k = kd;
        const double cm2 = cmr * cmr + cmi * cmi;
        const double ir = cmr / cm2, ii = -cmi / cm2 - (2.0 / 3.0) * k * k * k;
        const double n2 = ir * ir + ii * ii;
        re = ir / n2;
        im = -ii / n2;
        return;
    }
    // LDR (Draine & Goodman 1993): 1/alpha = 1/alpha_CM + (b1 + m^2 b2 + m^2 b3 S) k^2 - (2/3) i k^3
    const double b1 = -1.8915316, b2 = 0.1648469, b3 = -1.7700004;
    double S = 0;
    for (int a = 0; a < 3; ++a) S += b.prop[a] * b.prop[a] * (b.pol_re[a] * b.pol_re[a] + b.pol_im[a] * b.pol_im[a]);
    const double k = kd;
    const double cm2 = cmr * cmr + cmi * cmi;
    double ir = cmr / cm2, ii = -cmi / cm2;  // 1/alpha_CM
    const double tr = b1 + m2r * b2 + m2r * b3 * S, ti = m2i * b2 + m2i * b3 * S;
    ir += tr * k * k;
    ii += ti * k * k - (2.0 / 3.0) * k * k * k;
    const double n2 = ir * ir + ii * ii;
    re = ir / n2;
    im = -ii / n2;
}

// whether nl lines per block (a power of two) fit the x (axis 0) or y (axis 1) pass of precision R
template <typename R> bool tiles_valid(const Ctx &c, int axis, int nl) {
    if (nl < 1 || (nl & (nl - 1))) return false;
    const FftPlan &p = axis == 0 ? c.pxf : c.pyf;
    const int L = axis == 0 ? c.Lx : c.Ly;
    return nl * p.tpl <= max_threads<R>() && (size_t)nl * lds_line_stride(L) * sizeof(cplx<R>) <= DDA_LDS_CAP;
}
template bool tiles_valid<double>(const Ctx &, int, int);
template bool tiles_valid<float>(const Ctx &, int, int);

template <typename R> static void free_work(Work<R> &w) {
    (void)hipFree(w.B1);
    (void)hipFree(w.B2);
    (void)hipFree(w.scale);
    (void)hipFree(w.dots);
    w = Work<R>{};
}

template <typename R> dda_status ensure_work(Ctx &c, int nrhs) {
    Work<R> &w = work_of<R>(c);
    if (w.nrhs >= nrhs) return DDA_OK;
    DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
    free_work(w);
    const size_t nc = (size_t)3 * nrhs;
    dda_status st;
    if ((st = device_alloc((void **)&w.B1, nc * c.nz * (size_t)c.Lx * row_pitch(c.ny) * sizeof(cplx<R>))) != DDA_OK) return st;
    if ((st = device_alloc((void **)&w.B2, nc * row_pitch(c.nz) * (size_t)c.Lx * c.Ly * sizeof(cplx<R>))) != DDA_OK) return st;
    if ((st = device_alloc((void **)&w.scale, (size_t)nrhs * sizeof(cplx<R>))) != DDA_OK) return st;
    w.ndots = max_dots_per_rhs(c) * nrhs;  // enough for any tile schedule (the tuner may change it)
    if ((st = device_alloc((void **)&w.dots, w.ndots * sizeof(cplx<R>))) != DDA_OK) return st;
    w.nrhs = nrhs;
    return DDA_OK;
}
template dda_status ensure_work<double>(Ctx &, int);
template dda_status ensure_work<float>(Ctx &, int);

template <typename R>
dda_status matvec_launch(Ctx &c, const cplx<R> *x, cplx<R> *y, int nrhs, const double *are, const double *aim,
                         bool want_dots, hipStream_t s) {
    dda_status st = ensure_work<R>(c, nrhs);
    if (st != DDA_OK) return st;
    Work<R> &w = work_of<R>(c);
    std::vector<cplx<R>> sc(nrhs);
    const double inv = 1.0 / ((double)c.Lx * c.Ly * c.Lz);
    for (int r = 0; r < nrhs; ++r) sc[r] = mk<cplx<R>>((R)(are[r] * inv), (R)(aim[r] * inv));
    DDA_HIP_CHECK(hipMemcpyAsync(w.scale, sc.data(), nrhs * sizeof(cplx<R>), hipMemcpyHostToDevice, s));
    DDA_HIP_CHECK(hipStreamSynchronize(s));  // the host staging vector goes out of scope
    return matvec_device<R>(c, x, y, nrhs, w.scale, want_dots ? w.dots : nullptr, s, nullptr, nullptr);
}
template dda_status matvec_launch<double>(Ctx &, const double2 *, double2 *, int, const double *, const double *, bool,
                                          hipStream_t);
template dda_status matvec_launch<float>(Ctx &, const float2 *, float2 *, int, const double *, const double *, bool,
                                         hipStream_t);

void destroy(Ctx *c);

// Rows whose non-void cells form one run x0 <= x < x1 (or none) need no cell-map lookups in the x
// passes: {x0 | x1 << 16, first dipole} per (y, z) row, x0 = 0xFFFF for a row of several runs.
static std::vector<int2> row_runs(const int32_t *gmap, int nx, int ny, int nz) {
    std::vector<int2> rows((size_t)ny * nz);
    for (size_t row = 0; row < rows.size(); ++row) {
        const int32_t *g = gmap + row * nx;
        int x0 = -1, x1 = -1, runs = 0;
        for (int xx = 0; xx < nx; ++xx)
            if (g[xx] >= 0 && (xx == 0 || g[xx - 1] < 0)) {
                ++runs;
                x0 = xx;
            }
        if (runs == 1) {
            x1 = x0;
            while (x1 < nx && g[x1] >= 0) ++x1;
            rows[row] = make_int2(x0 | (x1 << 16), g[x0]);
        } else {
            rows[row] = make_int2(runs == 0 ? 0 : 0xFFFF, 0);
        }
    }
    return rows;
}

// A batch of homogeneous particles that share the padded grid, the wavenumber and the
// polarizability prescription, as one context whose right-hand sides are the particles: each
// particle sits at the origin corner of the batch grid (the largest extent per axis), keeps its own
// dipole order (the grid's linear order restricted to its mask, the same in both grids) and its own
// cell map, and is padded to the largest dipole count.  The product of a right-hand side then
// couples only that particle's dipoles; the tensor, twiddle tables, plans and tile schedule are
// those of the member whose grid is the batch grid (borrowed, not copied).  Returns DDA_ENOTSUP when
// the members do not qualify or no member spans the batch grid.
dda_status pack_setup(Ctx *const *members, int n, Ctx **out) {
    *out = nullptr;
    if (n < 1) return DDA_EINVAL;
    const Ctx &m0 = *members[0];
    int box[3] = {0, 0, 0};
    int64_t nmax = 0;
    for (int i = 0; i < n; ++i) {
        const Ctx &m = *members[i];
        if (m.Lx != m0.Lx || m.Ly != m0.Ly || m.Lz != m0.Lz || m.kd != m0.kd || m.polarizability != m0.polarizability ||
            wrapped(m) || (m.ghat32 == nullptr) != (m0.ghat32 == nullptr))
            return DDA_ENOTSUP;
        box[0] = std::max(box[0], m.nx);
        box[1] = std::max(box[1], m.ny);
        box[2] = std::max(box[2], m.nz);
        nmax = std::max(nmax, m.N);
    }
    const Ctx *donor = nullptr;
    for (int i = 0; i < n && !donor; ++i)
        if (members[i]->nx == box[0] && members[i]->ny == box[1] && members[i]->nz == box[2]) donor = members[i];
    if (!donor) return DDA_ENOTSUP;
    Ctx *c = new (std::nothrow) Ctx();
    if (!c) return DDA_ENOMEM;
    c->nx = box[0];
    c->ny = box[1];
    c->nz = box[2];
    c->Lx = donor->Lx;
    c->Ly = donor->Ly;
    c->Lz = donor->Lz;
    c->N = nmax;
    c->m_re = donor->m_re;
    c->m_im = donor->m_im;
    c->kd = donor->kd;
    c->polarizability = donor->polarizability;
    c->tl64 = donor->tl64;
    c->tl32 = donor->tl32;
    c->nc_z = donor->nc_z;
    c->pxf = donor->pxf;
    c->pxi = donor->pxi;
    c->pyf = donor->pyf;
    c->pyi = donor->pyi;
    c->pzf = donor->pzf;
    c->pzi = donor->pzi;
    c->borrowed = true;
    c->ghat = donor->ghat;
    c->ghat32 = donor->ghat32;
    c->tw64 = donor->tw64;
    c->tw32 = donor->tw32;
    const size_t ncell = (size_t)box[0] * box[1] * box[2], nrow = (size_t)box[1] * box[2];
    c->gmap_stride = ncell;
    c->rows_stride = nrow;
    dda_status st = DDA_OK;
    std::vector<int32_t> gmap(ncell * n, -1);
    std::vector<int2> rows(nrow * n);
    for (int i = 0; i < n; ++i) {
        const Ctx &m = *members[i];
        int32_t *g = gmap.data() + ncell * i;
        for (size_t d = 0; d < m.lin_host.size(); ++d) {
            const int l = m.lin_host[d];
            const int x = l % m.nx, y = (l / m.nx) % m.ny, z = l / (m.nx * m.ny);
            g[((size_t)z * box[1] + y) * box[0] + x] = (int32_t)d;
        }
        const std::vector<int2> r = row_runs(g, box[0], box[1], box[2]);
        std::copy(r.begin(), r.end(), rows.begin() + nrow * i);
    }
    if (hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) {
        set_error("dda_solve_many: stream creation failed");
        c->own_stream = nullptr;
        st = DDA_EHIP;
        goto fail;
    }
    c->stream = c->own_stream;
    if ((st = device_alloc((void **)&c->gmap, gmap.size() * sizeof(int32_t))) != DDA_OK) goto fail;
    if ((st = device_alloc((void **)&c->rows, rows.size() * sizeof(int2))) != DDA_OK) goto fail;
    {
        hipError_t e = hipMemcpy(c->gmap, gmap.data(), gmap.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->rows, rows.data(), rows.size() * sizeof(int2), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            set_error(std::string("dda_solve_many: upload failed: ") + hipGetErrorString(e));
            st = DDA_EHIP;
            goto fail;
        }
    }
    *out = c;
    return DDA_OK;
fail:
    destroy(c);
    return st;
}

void destroy(Ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->borrowed) {  // a batch of particles: the tensor and twiddles belong to a member
        c->ghat = nullptr;
        c->ghat32 = nullptr;
        c->tw64 = nullptr;
        c->tw32 = nullptr;
    }
    free_work(c->w64);
    free_work(c->w32);
    (void)hipFree(c->snap);
    (void)hipFree(c->dmat);
    (void)hipFree(c->mat_beta);
    (void)hipFree(c->xtmp);
    (void)hipFree(c->gmap);
    (void)hipFree(c->rows);
    (void)hipFree(c->lin);
    (void)hipFree(c->line_start);
    (void)hipFree(c->ghat);
    (void)hipFree(c->ghat32);
    (void)hipFree(c->tw64);
    (void)hipFree(c->tw32);
    (void)hipFree(c->vecs);
    (void)hipFree(c->vecs32);
    (void)hipFree(c->sbuf);
    (void)hipFree(c->red);
    if (c->hbuf) (void)hipHostFree(c->hbuf);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
}

static dda_status build_ghat(Ctx &c) {
    const size_t full = (size_t)c.Lx * c.Ly * c.Lz;
    const size_t oct = (size_t)(c.Lx / 2 + 1) * (c.Ly / 2 + 1) * (c.Lz / 2 + 1);
    dda_status st;
    if ((st = device_alloc((void **)&c.ghat, oct * 6 * sizeof(double2))) != DDA_OK) return st;
    double2 *buf = nullptr;
    if ((st = device_alloc((void **)&buf, full * sizeof(double2))) != DDA_OK) return st;
    hipStream_t s = c.stream;
    const int thr = 256;
    struct Axis { FftPlan pl; int nu, nv; long su, sv, sp; int lol; };
    const long Lx = c.Lx, Ly = c.Ly;
    Axis ax[3] = {{c.pxf, c.Ly, c.Lz, Lx, Lx * Ly, 1, 0},
                  {c.pyf, c.Lx, c.Lz, 1, Lx * Ly, Lx, 1},
                  {c.pzf, c.Lx, c.Ly, 1, Lx, Lx * Ly, 1}};
    int nl[3];
    for (int a = 0; a < 3; ++a)
        nl[a] = 1 << pick_lines_log2(ax[a].pl.tpl, lds_line_stride(ax[a].pl.L) * (int)sizeof(double2), ax[a].nu, 0);
    for (int comp = 0; comp < 6; ++comp) {
        hipLaunchKernelGGL(k_gfill, dim3((unsigned)((full + thr - 1) / thr)), dim3(thr), 0, s, buf, comp, c.nx, c.ny,
                           c.nz, c.Lx, c.Ly, c.Lz, c.kd);
        for (int a = 0; a < 3; ++a) {
            const int utiles = (ax[a].nu + nl[a] - 1) / nl[a];
            const size_t lds = (size_t)nl[a] * lds_line_stride(ax[a].pl.L) * sizeof(double2);
            if (lds > 64 * 1024)
                (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_axis),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            hipLaunchKernelGGL(k_fft_axis, dim3(utiles * ax[a].nv), dim3(nl[a] * ax[a].pl.tpl), lds, s, buf, ax[a].nu,
                               ax[a].nv, ax[a].su, ax[a].sv, ax[a].sp, ax[a].pl, (const double2 *)c.tw64, nl[a],
                               ax[a].lol);
        }
        hipLaunchKernelGGL(k_gextract, dim3((unsigned)((oct + thr - 1) / thr)), dim3(thr), 0, s, buf, c.ghat, comp,
                           c.Lx, c.Ly, c.Lz);
    }
    hipError_t e = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (e != hipSuccess || e2 != hipSuccess) {
        set_error(std::string("tensor build failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        return DDA_EHIP;
    }
    return DDA_OK;
}

dda_status setup(Ctx **out, const int32_t grid[3], const uint8_t *mask, const double m[2], double kd, int32_t pol,
                 const dda_setup_opts *opts, void *stream) {
    if (!out) {
        set_error("dda_setup: out is NULL");
        return DDA_EINVAL;
    }
    *out = nullptr;
    if (!grid || !mask || !m) {
        set_error("dda_setup: grid, mask and m must be non-NULL");
        return DDA_EINVAL;
    }
    for (int a = 0; a < 3; ++a)
        if (grid[a] < 1 || grid[a] > 2048) {
            set_error("dda_setup: grid sizes must be in 1..2048");
            return DDA_EINVAL;
        }
    if (!(kd > 0) || !std::isfinite(kd) || !std::isfinite(m[0]) || !std::isfinite(m[1])) {
        set_error("dda_setup: kd must be > 0 and m finite");
        return DDA_EINVAL;
    }
    if (pol != DDA_POL_LDR && pol != DDA_POL_CM && pol != DDA_POL_RR && pol != DDA_POL_CLDR) {
        set_error("dda_setup: unknown polarizability");
        return DDA_EINVAL;
    }
    Ctx *c = new (std::nothrow) Ctx();
    if (!c) return DDA_ENOMEM;
    c->nx = grid[0];
    c->ny = grid[1];
    c->nz = grid[2];
    c->m_re = m[0];
    c->m_im = m[1];
    c->kd = kd;
    c->polarizability = pol;
    c->stream = (hipStream_t)stream;
    const size_t ncell = (size_t)c->nx * c->ny * c->nz;
    c->mask.assign(mask, mask + ncell);
    std::vector<int32_t> gmap(ncell, -1);
    for (size_t e = 0; e < ncell; ++e)
        if (mask[e]) {
            gmap[e] = (int32_t)c->lin_host.size();
            c->lin_host.push_back((int32_t)e);
        }
    c->N = (int64_t)c->lin_host.size();
    if (c->N == 0) {
        set_error("dda_setup: the mask has no non-void cell");
        delete c;
        return DDA_EINVAL;
    }
    if ((uint64_t)c->N * 3 > 0x7fffffffull) {
        set_error("dda_setup: too many dipoles");
        delete c;
        return DDA_EINVAL;
    }
    int Ls[3];
    const int n[3] = {c->nx, c->ny, c->nz};
    for (int a = 0; a < 3; ++a) {
        const int want = opts ? opts->pad[a] : 0;
        if (want > 0) {
            if (want < 2 * n[a] - 1 || !five_smooth(want) || want > 4096) {
                set_error("dda_setup: padded size must be >= 2n-1, 5-smooth and <= 4096");
                delete c;
                return DDA_EINVAL;
            }
            Ls[a] = want;
        } else {
            Ls[a] = smallest_pad(n[a]);
        }
    }
    c->Lx = Ls[0];
    c->Ly = Ls[1];
    c->Lz = Ls[2];
    // plans and twiddle tables (one table per distinct length)
    std::vector<int> lens;
    for (int a = 0; a < 3; ++a)
        if (std::find(lens.begin(), lens.end(), Ls[a]) == lens.end()) lens.push_back(Ls[a]);
    std::vector<int> offs(lens.size());
    size_t total = 0;
    for (size_t i = 0; i < lens.size(); ++i) {
        offs[i] = (int)total;
        total += lens[i];
    }
    auto off_of = [&](int L) { return offs[std::find(lens.begin(), lens.end(), L) - lens.begin()]; };
    auto plans = [&](int L, int maxr, FftPlan &f, FftPlan &inv) {
        f = make_plan(L, maxr, false);
        inv = make_plan(L, maxr, true);
        f.tw_off = inv.tw_off = off_of(L);
        return f.npass > 0 && inv.npass > 0;
    };
    // the z pass of a multi-mode length (zmul_multi) runs its forward plan sorted largest radix
    // last (and the inverse largest first)
    const bool zflip = zmul_multi(make_plan(c->Lz, kMaxRadixZ, false));
    bool zok = plans(c->Lz, kMaxRadixZ, c->pzf, c->pzi);
    if (zok && zflip) {  // sorted: the forward plan's largest radix last, the inverse's first
        c->pzf = make_plan(c->Lz, kMaxRadixZ, 2);
        c->pzi = make_plan(c->Lz, kMaxRadixZ, 3);
        c->pzf.tw_off = c->pzi.tw_off = off_of(c->Lz);
    }
    if (!plans(c->Lx, kMaxRadix, c->pxf, c->pxi) || !plans(c->Ly, kMaxRadix, c->pyf, c->pyi) || !zok) {
        set_error("dda_setup: unsupported padded size");
        delete c;
        return DDA_EINVAL;
    }
    std::vector<double2> tw(total);
    std::vector<float2> tw32(total);
    for (size_t i = 0; i < lens.size(); ++i)
        for (int mm = 0; mm < lens[i]; ++mm) {
            const long double ang = -2.0L * 3.141592653589793238462643383279502884L * mm / lens[i];
            tw[offs[i] + mm] = make_double2((double)cosl(ang), (double)sinl(ang));
            tw32[offs[i] + mm] = make_float2((float)cosl(ang), (float)sinl(ang));
        }
    const int want_nl = opts ? opts->lines_per_block : 0;
    auto tiles = [&](Tiles &t, int cb, int maxt) {
        // fp32 at the automatic setting: twice the lines, so the transposed side still moves
        // 128-byte runs
        const int want = want_nl > 0 ? want_nl : 0;
        t.lnl_x = pick_lines_log2(c->pxf.tpl, lds_line_stride(c->Lx) * cb, c->ny, want, maxt);
        t.lnl_y = pick_lines_log2(c->pyf.tpl, lds_line_stride(c->Ly) * cb, c->nz, want, maxt);
        t.nl_x = 1 << t.lnl_x;
        t.nl_y = 1 << t.lnl_y;
        return t.nl_x * c->pxf.tpl <= maxt && t.nl_y * c->pyf.tpl <= maxt;
    };
    const bool tiles_ok = tiles(c->tl64, 16, max_threads<double>()) && tiles(c->tl32, 8, max_threads<float>());
    c->nc_z = 1;
    if (3 * zmul_ct(c->pzf) > DDA_ZMUL_THREADS || zmul_lds_elems(c->Lz) * 16 > 160 * 1024 || !tiles_ok) {
        set_error("dda_setup: padded size too large for one workgroup per line");
        delete c;
        return DDA_EINVAL;
    }
    dda_status st;
    if (hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) {
        set_error("dda_setup: stream creation failed");
        c->own_stream = nullptr;
        st = DDA_EHIP;
        goto fail;
    }
    if ((st = device_alloc((void **)&c->gmap, ncell * sizeof(int32_t))) != DDA_OK) goto fail;
    if ((st = device_alloc((void **)&c->rows, (size_t)c->ny * c->nz * sizeof(int2))) != DDA_OK) goto fail;
    if ((st = device_alloc((void **)&c->lin, c->N * sizeof(int32_t))) != DDA_OK) goto fail;
    if ((st = device_alloc((void **)&c->tw64, total * sizeof(double2))) != DDA_OK) goto fail;
    if ((st = device_alloc((void **)&c->tw32, total * sizeof(float2))) != DDA_OK) goto fail;
    {
        const std::vector<int2> rows = row_runs(gmap.data(), c->nx, c->ny, c->nz);
        hipError_t e = hipMemcpy(c->gmap, gmap.data(), ncell * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->rows, rows.data(), rows.size() * sizeof(int2), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->lin, c->lin_host.data(), c->N * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->tw64, tw.data(), total * sizeof(double2), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(c->tw32, tw32.data(), total * sizeof(float2), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            set_error(std::string("dda_setup: upload failed: ") + hipGetErrorString(e));
            st = DDA_EHIP;
            goto fail;
        }
    }
    if ((st = build_ghat(*c)) != DDA_OK) goto fail;
    if (opts && opts->fp32) {
        const size_t n6 = (size_t)(c->Lx / 2 + 1) * (c->Ly / 2 + 1) * (c->Lz / 2 + 1) * 6;
        if ((st = device_alloc((void **)&c->ghat32, n6 * sizeof(float2))) != DDA_OK) goto fail;
        hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n6 + 255) / 256)), dim3(256), 0, c->stream, c->ghat, c->ghat32,
                           n6);
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            set_error(std::string("dda_setup: fp32 tensor: ") + hipGetErrorString(e));
            st = DDA_EHIP;
            goto fail;
        }
    }
    *out = c;
    return DDA_OK;
fail:
    destroy(c);
    return st;
}

}  // namespace dda
