// Scattering read-out from the dipole polarizations P = beta x: extinction and absorption cross
// sections, far-field scattering amplitudes, and the Mueller matrix in a scattering plane
// (the quantities the paper compares with Mie theory, Sec. 3.1).
//
// Far field: F(n) = -i k^3 (I - n n) sum_j P_j exp(-i k n.r_j).  A block takes up to 256
// directions (one per thread) and a range of grid lines (y, z); every thread walks the dipoles
// of each line (read wave-uniformly through the scalar cache), advancing its phase factor along
// x by one multiplication per cell (a direct sincos restarts the recurrence after a gap in the
// line and at the start of every line, so at most nx - 1 products accumulate rounding).
#include <cmath>
#include <string>
#include <vector>

#include "ctx.hpp"

namespace dda {

bool beam_ok(const dda_beam *b);
template <typename R> dda_status beam_field_launch(Ctx &c, const dda_beam &b, cplx<R> *out, double sr, double si,
                                                   hipStream_t st);
void beta_of(const Ctx &c, const dda_beam &bm, double &br, double &bi);

constexpr int kRoThreads = 256;

// partial sums over dipoles: sum Im(conj(E_inc) x) (complex, before the beta factor) and |x|^2
__global__ void __launch_bounds__(kRoThreads) k_xsec(const double2 *__restrict__ x, const int *__restrict__ lin, int N,
                                                     int nx, int ny, int nz, double k, double a0, double a1, double a2,
                                                     double e0r, double e0i, double e1r, double e1i, double e2r,
                                                     double e2i, const double2 *__restrict__ einc,
                                                     double2 *part) {
    __shared__ double2 sh[2 * kRoThreads];
    double2 ex = make_double2(0, 0);  // sum conj(E).x  (complex)
    double xx = 0;
    for (int i = blockIdx.x * kRoThreads + threadIdx.x; i < N; i += gridDim.x * kRoThreads) {
        const int l = lin[i];
        const double px = (l % nx) + 0.5 - 0.5 * nx;
        const double py = ((l / nx) % ny) + 0.5 - 0.5 * ny;
        const double pz = (l / (nx * ny)) + 0.5 - 0.5 * nz;
        double sn = 0, cs = 1;
        if (!einc) sincos(k * (a0 * px + a1 * py + a2 * pz), &sn, &cs);
        // conj(E_c) = conj(e_c) exp(-i phase), or conj(einc[c][i]) for a focused beam
        const double er[3] = {e0r, e1r, e2r}, ei[3] = {e0i, e1i, e2i};
        for (int c = 0; c < 3; ++c) {
            const double2 v = x[(size_t)c * N + i];
            double ur, ui;
            if (einc) {
                const double2 e = einc[(size_t)c * N + i];
                ur = e.x;
                ui = -e.y;
            } else {
                ur = er[c] * cs + ei[c] * sn;   // Re(conj(e) exp(-i ph))
                ui = -er[c] * sn + ei[c] * cs;  // Im
            }
            ex.x += ur * v.x - ui * v.y;
            ex.y += ur * v.y + ui * v.x;
            xx += v.x * v.x + v.y * v.y;
        }
    }
    const int t = threadIdx.x;
    sh[t] = ex;
    sh[kRoThreads + t] = make_double2(xx, 0);
    __syncthreads();
    for (int h = kRoThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            sh[t].x += sh[t + h].x;
            sh[t].y += sh[t + h].y;
            sh[kRoThreads + t].x += sh[kRoThreads + t + h].x;
        }
        __syncthreads();
    }
    if (t == 0) {
        part[2 * blockIdx.x] = sh[0];
        part[2 * blockIdx.x + 1] = sh[kRoThreads];
    }
}

// F partial sums (without the -i k^3 (I - nn) beta factor) for the directions of this block
// (one per lane) over the lines [l0, l1) of chunk blockIdx.y; writes part[(d * nchunk + chunk) * 3 + c].
// Every lane of a wave walks the same dipoles, so their polarizations and cell indices are
// wave-uniform: they come through the scalar data cache into scalar registers, which the fp64
// multiply-adds read directly (no LDS staging, no block barriers).
__global__ void __launch_bounds__(kRoThreads) k_farfield(const double2 *__restrict__ x, const int *__restrict__ lin,
                                                         const int *__restrict__ line_start, int N, int nx, int ny,
                                                         int nz, int lines_per_chunk, const double *__restrict__ dirs,
                                                         int ndir, double k, double2 *__restrict__ part) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = d < ndir;
    const int chunk = blockIdx.y, nchunk = gridDim.y;
    double nxd = 0, nyd = 0, nzd = 0;
    if (active) {
        nxd = dirs[3 * d];
        nyd = dirs[3 * d + 1];
        nzd = dirs[3 * d + 2];
    }
    double sw, cw;
    sincos(-k * nxd, &sw, &cw);  // one-cell step along x
    double2 acc[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    const int nlines = ny * nz;
    const int l0 = chunk * lines_per_chunk;
    const int l1 = min(nlines, l0 + lines_per_chunk);
    const double2 *x1 = x + N, *x2 = x + 2 * (size_t)N;
    for (int L = l0; L < l1; ++L) {
        const int s = line_start[L], e = line_start[L + 1];
        const int base = L * nx;  // lin = base + ix on this line
        const double py = (L % ny) + 0.5 - 0.5 * ny;
        const double pz = (L / ny) + 0.5 - 0.5 * nz;
        double2 ph = make_double2(1, 0);
        int xprev = -2;
        auto step = [&](int ix, double2 v0, double2 v1, double2 v2) {
            if (ix == xprev + 1) {
                ph = make_double2(ph.x * cw - ph.y * sw, ph.x * sw + ph.y * cw);
            } else {
                const double px = ix + 0.5 - 0.5 * nx;
                double sn, cs;
                sincos(-k * (nxd * px + nyd * py + nzd * pz), &sn, &cs);
                ph = make_double2(cs, sn);
            }
            xprev = ix;
            const double2 v[3] = {v0, v1, v2};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                acc[c].x += v[c].x * ph.x - v[c].y * ph.y;
                acc[c].y += v[c].x * ph.y + v[c].y * ph.x;
            }
        };
        int q = s;
        for (; q + 4 <= e; q += 4) {  // four dipoles' loads in flight together
            int ix[4];
            double2 a[4], b[4], cc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ix[u] = lin[q + u] - base;
                a[u] = x[q + u];
                b[u] = x1[q + u];
                cc[u] = x2[q + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) step(ix[u], a[u], b[u], cc[u]);
        }
        for (; q < e; ++q) step(lin[q] - base, x[q], x1[q], x2[q]);
    }
    if (active)
        for (int c = 0; c < 3; ++c) part[((size_t)d * nchunk + chunk) * 3 + c] = acc[c];
}

__global__ void k_ff_sum(const double2 *part, int ndir, int nchunk, double2 *out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;  // (d, c)
    if (e >= ndir * 3) return;
    const int d = e / 3, c = e % 3;
    double2 s = make_double2(0, 0);
    for (int q = 0; q < nchunk; ++q) {
        const double2 v = part[((size_t)d * nchunk + q) * 3 + c];
        s.x += v.x;
        s.y += v.y;
    }
    out[e] = s;
}

static dda_status ensure_red(Ctx &c, size_t elems) {
    if (c.red_elems >= elems) return DDA_OK;
    DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
    (void)hipFree(c.red);
    c.red = nullptr;
    c.red_elems = 0;
    dda_status st = device_alloc((void **)&c.red, elems * sizeof(double2));
    if (st != DDA_OK) return st;
    c.red_elems = elems;
    return DDA_OK;
}

static dda_status ensure_lines(Ctx &c) {
    if (c.line_start) return DDA_OK;
    const int nl = c.ny * c.nz;
    std::vector<int> ls(nl + 1, 0);
    size_t q = 0;
    for (int L = 0; L < nl; ++L) {
        ls[L] = (int)q;
        const size_t base = (size_t)L * c.nx;
        while (q < c.lin_host.size() && (size_t)c.lin_host[q] < base + c.nx) ++q;
    }
    ls[nl] = (int)q;
    dda_status st = device_alloc((void **)&c.line_start, (nl + 1) * sizeof(int));
    if (st != DDA_OK) return st;
    DDA_HIP_CHECK(hipMemcpy(c.line_start, ls.data(), (nl + 1) * sizeof(int), hipMemcpyHostToDevice));
    return DDA_OK;
}

// sum_j x_j exp(-i k n.r_j) for each direction (host [ndir][3] complex), before beta and the projector
static dda_status farfield_sums(Ctx &c, const double2 *x, int ndir, const double *dirs, std::vector<double2> &out) {
    dda_status st;
    if ((st = ensure_lines(c)) != DDA_OK) return st;
    const int nlines = c.ny * c.nz;
    // directions in whole waves, at most four waves a block, blocks as even as the count allows
    const int waves = (ndir + 63) / 64;
    const int dtiles = (waves + kRoThreads / 64 - 1) / (kRoThreads / 64);
    const int bthreads = 64 * ((waves + dtiles - 1) / dtiles);
    // enough chunks to fill the GPU several times over, at least a few lines each
    int nchunk = std::max(1, std::min(nlines, 2048 / std::max(1, dtiles)));
    const int lpc = (nlines + nchunk - 1) / nchunk;
    nchunk = (nlines + lpc - 1) / lpc;
    const size_t npart = (size_t)ndir * nchunk * 3;
    if ((st = ensure_red(c, npart + (size_t)ndir * 3 + (size_t)ndir * 3 / 2 + 4)) != DDA_OK) return st;
    double2 *part = c.red;
    double2 *sums = c.red + npart;
    double *ddirs = (double *)(sums + (size_t)ndir * 3);
    DDA_HIP_CHECK(hipMemcpyAsync(ddirs, dirs, (size_t)ndir * 3 * sizeof(double), hipMemcpyHostToDevice, c.stream));
    hipLaunchKernelGGL(k_farfield, dim3(dtiles, nchunk), dim3(bthreads), 0, c.stream, x, c.lin, c.line_start,
                       (int)c.N, c.nx, c.ny, c.nz, lpc, ddirs, ndir, c.kd, part);
    hipLaunchKernelGGL(k_ff_sum, dim3((ndir * 3 + 255) / 256), dim3(256), 0, c.stream, part, ndir, nchunk, sums);
    DDA_HIP_CHECK(hipGetLastError());
    out.resize((size_t)ndir * 3);
    DDA_HIP_CHECK(hipMemcpyAsync(out.data(), sums, out.size() * sizeof(double2), hipMemcpyDeviceToHost, c.stream));
    DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
    return DDA_OK;
}

// F(n) = -i k^3 beta (I - n n) S
static void finish_farfield(const Ctx &c, const dda_beam &bm, int ndir, const double *dirs,
                            const std::vector<double2> &S, double *F) {
    double br, bi;
    beta_of(c, bm, br, bi);
    const double k3 = c.kd * c.kd * c.kd;
    for (int d = 0; d < ndir; ++d) {
        const double *n = dirs + 3 * d;
        double sr[3], si[3];
        for (int a = 0; a < 3; ++a) {
            sr[a] = br * S[3 * d + a].x - bi * S[3 * d + a].y;
            si[a] = br * S[3 * d + a].y + bi * S[3 * d + a].x;
        }
        const double dr = n[0] * sr[0] + n[1] * sr[1] + n[2] * sr[2];
        const double di = n[0] * si[0] + n[1] * si[1] + n[2] * si[2];
        for (int a = 0; a < 3; ++a) {
            const double pr = sr[a] - n[a] * dr, pi = si[a] - n[a] * di;
            // -i k^3 (pr + i pi) = k^3 (pi - i pr)
            F[(3 * d + a) * 2] = k3 * pi;
            F[(3 * d + a) * 2 + 1] = -k3 * pr;
        }
    }
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on P_n, evaluated by the
// three-term recurrence, from the usual cosine first guesses
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;  // P_0, P_1
            for (int j = 1; j < n; ++j) {
                const double p2 = ((2.0 * j + 1.0) * z * p1 - j * p0) / (j + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);  // P_n'(z)
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) <= 1e-16 * std::max(1.0, std::fabs(z))) break;
        }
        double p0 = 1.0, p1 = z;
        for (int j = 1; j < n; ++j) {
            const double p2 = ((2.0 * j + 1.0) * z * p1 - j * p0) / (j + 1.0);
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// mask invariant under the +90 degree rotation about z: cell (i, j) -> (n-1-j, i)
static bool rot90_symmetric(const Ctx &c) {
    if (c.nx != c.ny) return false;
    const int n = c.nx;
    for (int z = 0; z < c.nz; ++z)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const uint8_t a = c.mask[((size_t)z * n + j) * n + i] != 0;
                const uint8_t b = c.mask[((size_t)z * n + i) * n + (n - 1 - j)] != 0;
                if (a != b) return false;
            }
    return true;
}

}  // namespace dda

using namespace dda;

extern "C" {

dda_status dda_cross_sections(dda_ctx *h, const dda_beam *beam, const void *x, double out[3]) {
    clear_error();
    Ctx *c = cx(h);
    if (!c || !x || !out || !beam_ok(beam)) {
        set_error("dda_cross_sections: NULL argument or beam without unit vectors");
        return DDA_EINVAL;
    }
    const int nb = (int)std::min<int64_t>(1024, (c->N + kRoThreads - 1) / kRoThreads);
    dda_status st;
    if ((st = ensure_red(*c, 2 * (size_t)nb)) != DDA_OK) return st;
    const dda_beam &b = *beam;
    if (wrapped(*c)) {  // the polarizations P = beta x of the materials take the place of x (beta_of gives 1)
        if ((st = material_scale(*c, b, (const double2 *)x, c->xtmp, c->stream)) != DDA_OK) return st;
        x = c->xtmp;
    }
    void *einc = nullptr;  // a focused beam's field at the dipoles
    if (b.w0 > 0) {
        if ((st = device_alloc(&einc, 3 * (size_t)c->N * sizeof(double2))) != DDA_OK) return st;
        if ((st = beam_field_launch<double>(*c, b, (double2 *)einc, 1.0, 0.0, c->stream)) != DDA_OK) {
            (void)hipFree(einc);
            return st;
        }
    }
    hipLaunchKernelGGL(k_xsec, dim3(nb), dim3(kRoThreads), 0, c->stream, (const double2 *)x, c->lin, (int)c->N, c->nx,
                       c->ny, c->nz, c->kd, b.prop[0], b.prop[1], b.prop[2], b.pol_re[0], b.pol_im[0], b.pol_re[1],
                       b.pol_im[1], b.pol_re[2], b.pol_im[2], (const double2 *)einc, c->red);
    const hipError_t le = hipGetLastError();
    if (einc) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(einc);
    }
    DDA_HIP_CHECK(le);
    std::vector<double2> p(2 * (size_t)nb);
    DDA_HIP_CHECK(hipMemcpyAsync(p.data(), c->red, p.size() * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
    DDA_HIP_CHECK(hipStreamSynchronize(c->stream));
    double exr = 0, exi = 0, xx = 0;
    for (int i = 0; i < nb; ++i) {
        exr += p[2 * i].x;
        exi += p[2 * i].y;
        xx += p[2 * i + 1].x;
    }
    double ar, ai, br, bi;
    polarizability(*c, b, ar, ai);
    beta_of(*c, b, br, bi);
    const double k = c->kd;
    // conj(E).P = beta conj(E).x
    const double im_ep = br * exi + bi * exr;
    const double cext = 4.0 * M_PI * k * im_ep;
    const double inv_im = -ai / (ar * ar + ai * ai);  // Im(1/alpha)
    const double w = -inv_im - (2.0 / 3.0) * k * k * k;
    double cabs = 4.0 * M_PI * k * w * (br * br + bi * bi) * xx;
    if (wrapped(*c) && (st = material_cabs(*c, b, (const double2 *)x, cabs)) != DDA_OK) return st;
    out[0] = cext;
    out[1] = cabs;
    out[2] = cext - cabs;
    return DDA_OK;
}

dda_status dda_farfield(dda_ctx *h, const dda_beam *beam, const void *x, int32_t n_dir, const double *dirs,
                        double *F) {
    clear_error();
    Ctx *c = cx(h);
    if (!c || !x || !dirs || !F || n_dir < 1 || !beam_ok(beam)) {
        set_error("dda_farfield: NULL argument, n_dir < 1 or beam without unit vectors");
        return DDA_EINVAL;
    }
    dda_status st;
    if (wrapped(*c)) {
        if ((st = material_scale(*c, *beam, (const double2 *)x, c->xtmp, c->stream)) != DDA_OK) return st;
        x = c->xtmp;
    }
    std::vector<double2> S;
    st = farfield_sums(*c, (const double2 *)x, n_dir, dirs, S);
    if (st != DDA_OK) return st;
    finish_farfield(*c, *beam, n_dir, dirs, S, F);
    return DDA_OK;
}

dda_status dda_asymmetry(dda_ctx *h, const dda_beam *beam, const void *x, int32_t n_theta, int32_t n_phi,
                         double out[2]) {
    clear_error();
    Ctx *c = cx(h);
    if (c && (n_theta <= 0 || n_phi <= 0)) {
        // automatic: |F(n)|^2 is band-limited to Legendre degree 2 k R (R the radius of the grid's
        // circumscribing sphere), so n_theta >= k R + 2 Gauss nodes and n_phi > 2 k R azimuths
        // integrate it (times cos theta) exactly
        const double R = 0.5 * std::sqrt((double)c->nx * c->nx + (double)c->ny * c->ny + (double)c->nz * c->nz);
        const int kr = (int)std::ceil(c->kd * R);
        if (n_theta <= 0) n_theta = kr + 4;
        if (n_phi <= 0) n_phi = 2 * kr + 8;
    }
    if (!c || !x || !out || n_theta < 1 || n_phi < 1 || (int64_t)n_theta * n_phi > (1 << 22) || !beam_ok(beam)) {
        set_error("dda_asymmetry: NULL argument, grid sizes outside 1..2^22 directions or beam without unit vectors");
        return DDA_EINVAL;
    }
    if (wrapped(*c)) {
        const dda_status sc = material_scale(*c, *beam, (const double2 *)x, c->xtmp, c->stream);
        if (sc != DDA_OK) return sc;
        x = c->xtmp;
    }
    // directions n = mu a + sqrt(1 - mu^2) (cos phi e1 + sin phi e2) about the propagation a
    const double *a = beam->prop;
    const double t[3] = {std::fabs(a[0]) < 0.9 ? 1.0 : 0.0, std::fabs(a[0]) < 0.9 ? 0.0 : 1.0, 0.0};
    double e1[3] = {a[1] * t[2] - a[2] * t[1], a[2] * t[0] - a[0] * t[2], a[0] * t[1] - a[1] * t[0]};
    const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (double &v : e1) v /= l1;
    const double e2[3] = {a[1] * e1[2] - a[2] * e1[1], a[2] * e1[0] - a[0] * e1[2], a[0] * e1[1] - a[1] * e1[0]};
    std::vector<double> mu, wmu;
    gauss_legendre(n_theta, mu, wmu);
    const int ndir = n_theta * n_phi;
    std::vector<double> dirs((size_t)ndir * 3), wt(ndir), cs(ndir);
    for (int i = 0; i < n_theta; ++i)
        for (int j = 0; j < n_phi; ++j) {
            const double ph = 2.0 * M_PI * j / n_phi, st = std::sqrt(std::max(0.0, 1.0 - mu[i] * mu[i]));
            const int d = i * n_phi + j;
            for (int q = 0; q < 3; ++q)
                dirs[3 * d + q] = mu[i] * a[q] + st * (std::cos(ph) * e1[q] + std::sin(ph) * e2[q]);
            wt[d] = wmu[i] * 2.0 * M_PI / n_phi;
            cs[d] = mu[i];
        }
    std::vector<double2> S;
    dda_status st = farfield_sums(*c, (const double2 *)x, ndir, dirs.data(), S);
    if (st != DDA_OK) return st;
    std::vector<double> F((size_t)ndir * 6);
    finish_farfield(*c, *beam, ndir, dirs.data(), S, F.data());
    double csca = 0, gs = 0;
    const double k2 = c->kd * c->kd;
    for (int d = 0; d < ndir; ++d) {
        double f2 = 0;
        for (int q = 0; q < 6; ++q) f2 += F[6 * d + q] * F[6 * d + q];
        csca += wt[d] * f2 / k2;
        gs += wt[d] * cs[d] * f2 / k2;
    }
    out[0] = csca;
    out[1] = csca > 0 ? gs / csca : 0.0;
    return DDA_OK;
}

dda_status dda_mueller(dda_ctx *h, const dda_beam *beam, const void *x1, const void *x2, double phi,
                       const double *theta, int32_t n_theta, double *M) {
    clear_error();
    Ctx *c = cx(h);
    if (!c || !x1 || !theta || !M || n_theta < 1 || !beam_ok(beam)) {
        set_error("dda_mueller: NULL argument, n_theta < 1 or beam without unit vectors");
        return DDA_EINVAL;
    }
    if (!x2 && (beam->w0 > 0 || wrapped(*c))) {
        set_error("dda_mueller: the one-polarization shortcut (x2 = NULL) takes plane waves on homogeneous particles "
                  "only");
        return DDA_EINVAL;
    }
    const dda_beam &b = *beam;
    for (int a = 0; a < 3; ++a)
        if (b.pol_im[a] != 0) {
            set_error("dda_mueller: the beam frame needs a real (linear) polarization");
            return DDA_EINVAL;
        }
    // beam frame e1 = pol, e2 = prop x pol, e3 = prop
    double e1[3], e2[3], e3[3];
    for (int a = 0; a < 3; ++a) {
        e1[a] = b.pol_re[a];
        e3[a] = b.prop[a];
    }
    e2[0] = e3[1] * e1[2] - e3[2] * e1[1];
    e2[1] = e3[2] * e1[0] - e3[0] * e1[2];
    e2[2] = e3[0] * e1[1] - e3[1] * e1[0];
    const double cp = std::cos(phi), sp = std::sin(phi);
    std::vector<double> n(3 * (size_t)n_theta), th(3 * (size_t)n_theta), ph(3);
    for (int a = 0; a < 3; ++a) ph[a] = -sp * e1[a] + cp * e2[a];
    for (int i = 0; i < n_theta; ++i) {
        const double st = std::sin(theta[i]), ct = std::cos(theta[i]);
        for (int a = 0; a < 3; ++a) {
            n[3 * i + a] = st * (cp * e1[a] + sp * e2[a]) + ct * e3[a];
            th[3 * i + a] = ct * (cp * e1[a] + sp * e2[a]) - st * e3[a];
        }
    }
    std::vector<double> F1(6 * (size_t)n_theta), F2(6 * (size_t)n_theta);
    dda_status st;
    if (wrapped(*c)) {  // P = beta x of each polarization (the second beam has polarization e2)
        dda_beam bb = b;
        for (int a = 0; a < 3; ++a) bb.pol_re[a] = e2[a];
        double2 *P1 = c->xtmp, *P2 = c->xtmp + 3 * (size_t)c->N;
        if ((st = material_scale(*c, b, (const double2 *)x1, P1, c->stream)) != DDA_OK) return st;
        if ((st = material_scale(*c, bb, (const double2 *)x2, P2, c->stream)) != DDA_OK) return st;
        x1 = P1;
        x2 = P2;
    }
    std::vector<double2> S;
    if ((st = farfield_sums(*c, (const double2 *)x1, n_theta, n.data(), S)) != DDA_OK) return st;
    finish_farfield(*c, b, n_theta, n.data(), S, F1.data());
    dda_beam b2 = b;
    for (int a = 0; a < 3; ++a) b2.pol_re[a] = e2[a];
    if (x2) {
        if ((st = farfield_sums(*c, (const double2 *)x2, n_theta, n.data(), S)) != DDA_OK) return st;
        finish_farfield(*c, b2, n_theta, n.data(), S, F2.data());
    } else {
        // F2(n) = R F1(R^T n), R the +90 degree rotation about e3 (takes e1 to e2); needs e3 = +-z
        if (!(std::fabs(std::fabs(e3[2]) - 1.0) < 1e-12) || !rot90_symmetric(*c)) {
            set_error("dda_mueller: x2 = NULL needs incidence along z and a mask invariant under a 90-degree turn");
            return DDA_ESYMMETRY;
        }
        const double sgn = e3[2] > 0 ? 1.0 : -1.0;  // rotation by +90 degrees about e3
        // R about +z by angle sgn*90: (x, y) -> (-sgn y, sgn x)
        std::vector<double> nr(3 * (size_t)n_theta);
        for (int i = 0; i < n_theta; ++i) {  // R^T n
            const double vx = n[3 * i], vy = n[3 * i + 1], vz = n[3 * i + 2];
            nr[3 * i] = sgn * vy;
            nr[3 * i + 1] = -sgn * vx;
            nr[3 * i + 2] = vz;
        }
        std::vector<double> G(6 * (size_t)n_theta);
        if ((st = farfield_sums(*c, (const double2 *)x1, n_theta, nr.data(), S)) != DDA_OK) return st;
        finish_farfield(*c, b, n_theta, nr.data(), S, G.data());
        for (int i = 0; i < n_theta; ++i)
            for (int part = 0; part < 2; ++part) {
                const double gx = G[(3 * i) * 2 + part], gy = G[(3 * i + 1) * 2 + part], gz = G[(3 * i + 2) * 2 + part];
                F2[(3 * i) * 2 + part] = -sgn * gy;
                F2[(3 * i + 1) * 2 + part] = sgn * gx;
                F2[(3 * i + 2) * 2 + part] = gz;
            }
    }
    for (int i = 0; i < n_theta; ++i) {
        // F_par = cos(phi) F1 + sin(phi) F2, F_perp = sin(phi) F1 - cos(phi) F2
        double Sre[4], Sim[4];  // S1..S4
        double tp_r = 0, tp_i = 0, pp_r = 0, pp_i = 0, tq_r = 0, tq_i = 0, pq_r = 0, pq_i = 0;
        for (int a = 0; a < 3; ++a) {
            const double f1r = F1[(3 * i + a) * 2], f1i = F1[(3 * i + a) * 2 + 1];
            const double f2r = F2[(3 * i + a) * 2], f2i = F2[(3 * i + a) * 2 + 1];
            const double par_r = cp * f1r + sp * f2r, par_i = cp * f1i + sp * f2i;
            const double per_r = sp * f1r - cp * f2r, per_i = sp * f1i - cp * f2i;
            tp_r += th[3 * i + a] * par_r;
            tp_i += th[3 * i + a] * par_i;
            pp_r += ph[a] * par_r;
            pp_i += ph[a] * par_i;
            tq_r += th[3 * i + a] * per_r;
            tq_i += th[3 * i + a] * per_i;
            pq_r += ph[a] * per_r;
            pq_i += ph[a] * per_i;
        }
        // S2 = th.F_par, S4 = -ph.F_par, S3 = th.F_perp, S1 = -ph.F_perp
        Sre[1] = tp_r, Sim[1] = tp_i;
        Sre[3] = -pp_r, Sim[3] = -pp_i;
        Sre[2] = tq_r, Sim[2] = tq_i;
        Sre[0] = -pq_r, Sim[0] = -pq_i;
        auto a2 = [&](int j) { return Sre[j] * Sre[j] + Sim[j] * Sim[j]; };
        // u * conj(v) real and imaginary parts for S_(a+1), S_(b+1)
        auto re = [&](int a, int bb) { return Sre[a] * Sre[bb] + Sim[a] * Sim[bb]; };
        auto im = [&](int a, int bb) { return Sim[a] * Sre[bb] - Sre[a] * Sim[bb]; };
        const double s1 = a2(0), s2 = a2(1), s3 = a2(2), s4 = a2(3);
        double *m = M + 16 * (size_t)i;
        m[0] = 0.5 * (s2 + s1 + s4 + s3);
        m[1] = 0.5 * (s2 - s1 + s4 - s3);
        m[2] = re(1, 2) + re(0, 3);   // Re(S2 S3* + S1 S4*)
        m[3] = im(1, 2) - im(0, 3);   // Im(S2 S3* - S1 S4*)
        m[4] = 0.5 * (s2 - s1 - s4 + s3);
        m[5] = 0.5 * (s2 + s1 - s4 - s3);
        m[6] = re(1, 2) - re(0, 3);   // Re(S2 S3* - S1 S4*)
        m[7] = im(1, 2) + im(0, 3);   // Im(S2 S3* + S1 S4*)
        m[8] = re(1, 3) + re(0, 2);   // Re(S2 S4* + S1 S3*)
        m[9] = re(1, 3) - re(0, 2);   // Re(S2 S4* - S1 S3*)
        m[10] = re(0, 1) + re(2, 3);  // Re(S1 S2* + S3 S4*)
        m[11] = im(1, 0) + im(3, 2);  // Im(S2 S1* + S4 S3*)
        m[12] = im(3, 1) + im(0, 2);  // Im(S4 S2* + S1 S3*)
        m[13] = im(3, 1) - im(0, 2);  // Im(S4 S2* - S1 S3*)
        m[14] = im(0, 1) - im(2, 3);  // Im(S1 S2* - S3 S4*)
        m[15] = re(0, 1) - re(2, 3);  // Re(S1 S2* - S3 S4*)
    }
    return DDA_OK;
}

}  // extern "C"
