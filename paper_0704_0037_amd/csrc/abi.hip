// The C-ABI entry points (include/dda.h) that set up contexts, build right-hand sides and apply
// the interaction matrix.  The solver and the read-out entry points live in solver.hip and
// readout.hip.
#include <algorithm>
#include <array>
#include <cmath>
#include <string>
#include <vector>

#include "ctx.hpp"

namespace dda {
int default_pad(int n);
dda_status setup(Ctx **out, const int32_t grid[3], const uint8_t *mask, const double m[2], double kd, int32_t pol,
                 const dda_setup_opts *opts, void *stream);
void destroy(Ctx *c);
const char *last_error();

// b[c][i] = beta e_c exp(i k a.r_i) for each right-hand side (beta = principal sqrt(alpha))
template <typename R>
__global__ void k_rhs(const int *__restrict__ lin, cplx<R> *__restrict__ b, int N, int nx, int ny, int nz, double k,
                      double a0, double a1, double a2, double e0r, double e0i, double e1r, double e1i, double e2r,
                      double e2i, double br, double bi) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int l = lin[i];
    const double x = (l % nx) + 0.5 - 0.5 * nx;
    const double y = ((l / nx) % ny) + 0.5 - 0.5 * ny;
    const double z = (l / (nx * ny)) + 0.5 - 0.5 * nz;
    double sn, cs;
    sincos(k * (a0 * x + a1 * y + a2 * z), &sn, &cs);
    const double pr = br * cs - bi * sn, pi = br * sn + bi * cs;  // beta * exp(i phase)
    b[i] = mk<cplx<R>>((R)(pr * e0r - pi * e0i), (R)(pr * e0i + pi * e0r));
    b[(size_t)N + i] = mk<cplx<R>>((R)(pr * e1r - pi * e1i), (R)(pr * e1i + pi * e1r));
    b[2 * (size_t)N + i] = mk<cplx<R>>((R)(pr * e2r - pi * e2i), (R)(pr * e2i + pi * e2r));
}

void beta_of(const Ctx &c, const dda_beam &bm, double &br, double &bi) {
    double ar, ai;
    polarizability(c, bm, ar, ai);
    // principal square root
    const double mod = std::hypot(ar, ai);
    br = std::sqrt(0.5 * (mod + ar));
    bi = std::copysign(std::sqrt(0.5 * (mod - ar)), ai);
}

template <typename R> dda_status beam_field_launch(Ctx &c, const dda_beam &b, cplx<R> *out, double sr, double si,
                                                   hipStream_t st);
template <typename R> static dda_status rhs_plane(Ctx &c, const dda_beam &bm, cplx<R> *b, double br, double bi,
                                                  hipStream_t s);

template <typename R> dda_status rhs_launch(Ctx &c, const dda_beam &bm, cplx<R> *b, hipStream_t s) {
    double br, bi;
    beta_of(c, bm, br, bi);
    if (wrapped(c)) {
        // beta of each dipole's material (beta_of gives 1 for an inhomogeneous particle)
        if constexpr (!std::is_same<R, double>::value) {
            set_error("right-hand side: an inhomogeneous particle is solved in double precision only");
            return DDA_ENOTSUP;
        } else {
            dda_status st = bm.w0 > 0 ? beam_field_launch<R>(c, bm, b, 1.0, 0.0, s) : rhs_plane<R>(c, bm, b, 1.0, 0.0, s);
            if (st != DDA_OK) return st;
            return material_scale(c, bm, b, b, s);
        }
    }
    if (bm.w0 > 0) return beam_field_launch<R>(c, bm, b, br, bi, s);
    return rhs_plane<R>(c, bm, b, br, bi, s);
}

template <typename R> static dda_status rhs_plane(Ctx &c, const dda_beam &bm, cplx<R> *b, double br, double bi,
                                                  hipStream_t s) {
    const int N = (int)c.N;
    hipLaunchKernelGGL(k_rhs<R>, dim3((N + 255) / 256), dim3(256), 0, s, c.lin, b, N, c.nx, c.ny, c.nz, c.kd,
                       bm.prop[0], bm.prop[1], bm.prop[2], bm.pol_re[0], bm.pol_im[0], bm.pol_re[1], bm.pol_im[1],
                       bm.pol_re[2], bm.pol_im[2], br, bi);
    DDA_HIP_CHECK(hipGetLastError());
    return DDA_OK;
}
template dda_status rhs_launch<double>(Ctx &, const dda_beam &, double2 *, hipStream_t);
template dda_status rhs_launch<float>(Ctx &, const dda_beam &, float2 *, hipStream_t);

bool beam_ok(const dda_beam *b) {
    if (!b) return false;
    double a2 = 0, e2 = 0;
    for (int i = 0; i < 3; ++i) {
        if (!std::isfinite(b->prop[i]) || !std::isfinite(b->pol_re[i]) || !std::isfinite(b->pol_im[i])) return false;
        a2 += b->prop[i] * b->prop[i];
        e2 += b->pol_re[i] * b->pol_re[i] + b->pol_im[i] * b->pol_im[i];
    }
    if (!(std::fabs(a2 - 1) < 1e-6 && std::fabs(e2 - 1) < 1e-6)) return false;
    if (b->w0 == 0) return true;
    // a focused beam: finite waist and focus, polarization orthogonal to the propagation
    if (!(std::isfinite(b->w0) && b->w0 > 0)) return false;
    double dr = 0, di = 0;
    for (int i = 0; i < 3; ++i) {
        if (!std::isfinite(b->center[i])) return false;
        dr += b->pol_re[i] * b->prop[i];
        di += b->pol_im[i] * b->prop[i];
    }
    return std::fabs(dr) < 1e-6 && std::fabs(di) < 1e-6;
}

}  // namespace dda

using namespace dda;

extern "C" {

dda_status dda_setup(dda_ctx **out, const int32_t grid[3], const uint8_t *mask, const double m[2], double kd,
                     int32_t polarizability, const dda_setup_opts *opts, void *stream) {
    clear_error();
    if (polarizability == DDA_POL_CLDR && opts && opts->fp32) {
        set_error("dda_setup: single-precision products are not available with CLDR");
        if (out) *out = nullptr;
        return DDA_ENOTSUP;
    }
    Ctx *c = nullptr;
    dda_status st = setup(&c, grid, mask, m, kd, polarizability, opts, stream);
    if (st == DDA_OK && (st = material_init(*c, 1, m)) != DDA_OK) {  // CLDR runs the wrapped product
        destroy(c);
        c = nullptr;
    }
    if (out) *out = reinterpret_cast<dda_ctx *>(c);
    return st;
}

dda_status dda_free(dda_ctx *ctx) {
    clear_error();
    destroy(cx(ctx));
    return DDA_OK;
}

int64_t dda_num_dipoles(const dda_ctx *ctx) { return ctx ? cx(ctx)->N : -1; }

dda_status dda_padded_grid(const dda_ctx *ctx, int32_t out[3]) {
    clear_error();
    if (!ctx || !out) {
        set_error("dda_padded_grid: NULL argument");
        return DDA_EINVAL;
    }
    out[0] = cx(ctx)->Lx;
    out[1] = cx(ctx)->Ly;
    out[2] = cx(ctx)->Lz;
    return DDA_OK;
}

dda_status dda_polarizability(const dda_ctx *ctx, const dda_beam *beam, double out[2]) {
    clear_error();
    if (!ctx || !out || !beam_ok(beam)) {
        set_error("dda_polarizability: NULL context/output or beam without unit vectors");
        return DDA_EINVAL;
    }
    if (wrapped(*cx(ctx))) {
        set_error("dda_polarizability: the context has a polarizability per material or per component");
        return DDA_ENOTSUP;
    }
    polarizability(*cx(ctx), *beam, out[0], out[1]);
    return DDA_OK;
}

dda_status dda_rhs(dda_ctx *ctx, const dda_beam *beam, void *b) {
    clear_error();
    if (!ctx || !b || !beam_ok(beam)) {
        set_error("dda_rhs: NULL argument or beam without unit vectors");
        return DDA_EINVAL;
    }
    return rhs_launch<double>(*cx(ctx), *beam, (double2 *)b, cx(ctx)->stream);
}

static dda_status matvec_common(dda_ctx *h, const dda_beam *beams, int32_t n, const void *x, void *y, bool f32) {
    Ctx *ctx = cx(h);
    if (!ctx || !beams || !x || !y || n < 1) {
        set_error("dda_matvec: NULL argument or n_rhs < 1");
        return DDA_EINVAL;
    }
    if (x == y) {
        set_error("dda_matvec: x and y must not overlap");
        return DDA_EINVAL;
    }
    std::vector<double> ar(n), ai(n);
    for (int r = 0; r < n; ++r) {
        if (!beam_ok(&beams[r])) {
            set_error("dda_matvec: beam without unit vectors");
            return DDA_EINVAL;
        }
        polarizability(*ctx, beams[r], ar[r], ai[r]);
    }
    if (f32) {
        if (!ctx->ghat32) {
            set_error("dda_matvec_f32: context built without opts.fp32");
            return DDA_ENOTSUP;
        }
        return matvec_launch<float>(*ctx, (const float2 *)x, (float2 *)y, n, ar.data(), ai.data(), false,
                                    ctx->stream);
    }
    dda_status st = material_prepare(*ctx, beams, n);
    if (st != DDA_OK) return st;
    return matvec_launch<double>(*ctx, (const double2 *)x, (double2 *)y, n, ar.data(), ai.data(), false, ctx->stream);
}

dda_status dda_matvec(dda_ctx *ctx, const dda_beam *beam, const void *x, void *y) {
    clear_error();
    return matvec_common(ctx, beam, 1, x, y, false);
}

dda_status dda_matvec_f32(dda_ctx *ctx, const dda_beam *beam, const void *x, void *y) {
    clear_error();
    return matvec_common(ctx, beam, 1, x, y, true);
}

dda_status dda_matvec_batch(dda_ctx *ctx, const dda_beam *beams, int32_t n_rhs, const void *x, void *y) {
    clear_error();
    return matvec_common(ctx, beams, n_rhs, x, y, false);
}

}  // extern "C"

template <typename R>
static dda_status matvec_timed(Ctx &c, int n, const std::vector<double> &ar, const std::vector<double> &ai,
                               const cplx<R> *x, cplx<R> *y, int reps, float kernel_ms[5], float *total_ms) {
    // first call uploads the scales and settles the work buffers
    if (wrapped(c)) {
        set_error("dda_matvec_timed: homogeneous particles only");
        return DDA_ENOTSUP;
    }
    dda_status st = matvec_launch<R>(c, x, y, n, ar.data(), ai.data(), false, c.stream);
    if (st != DDA_OK) return st;
    Work<R> &w = work_of<R>(c);
    hipEvent_t ev[6];
    for (int i = 0; i < 6; ++i) DDA_HIP_CHECK(hipEventCreate(&ev[i]));
    double acc[5] = {0, 0, 0, 0, 0}, tot = 0;
    for (int r = 0; r < reps && st == DDA_OK; ++r) {
        st = matvec_device<R>(c, x, y, n, w.scale, nullptr, c.stream, nullptr, ev);
        if (st != DDA_OK) break;
        hipError_t e = hipEventSynchronize(ev[5]);
        if (e != hipSuccess) {
            set_error(std::string("dda_matvec_timed: ") + hipGetErrorString(e));
            st = DDA_EHIP;
            break;
        }
        for (int k = 0; k < 5; ++k) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
            acc[k] += ms;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ev[0], ev[5]);
        tot += ms;
    }
    for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
    if (st != DDA_OK) return st;
    for (int k = 0; k < 5; ++k) kernel_ms[k] = (float)(acc[k] / reps);
    *total_ms = (float)(tot / reps);
    return DDA_OK;
}

extern "C" {

dda_status dda_matvec_timed(dda_ctx *h, const dda_beam *beams, int32_t n_rhs, int32_t precision, const void *x,
                            void *y, int32_t reps, float kernel_ms[5], float *total_ms) {
    clear_error();
    Ctx *ctx = cx(h);
    if (!ctx || !beams || n_rhs < 1 || !x || !y || reps < 1 || !kernel_ms || !total_ms || x == y) {
        set_error("dda_matvec_timed: bad argument");
        return DDA_EINVAL;
    }
    if (precision != DDA_FP64 && precision != DDA_FP32_REFINE) {
        set_error("dda_matvec_timed: unknown precision");
        return DDA_EINVAL;
    }
    std::vector<double> ar(n_rhs), ai(n_rhs);
    for (int r = 0; r < n_rhs; ++r) {
        if (!beam_ok(&beams[r])) {
            set_error("dda_matvec_timed: beam without unit vectors");
            return DDA_EINVAL;
        }
        polarizability(*ctx, beams[r], ar[r], ai[r]);
    }
    if (precision == DDA_FP64)
        return matvec_timed<double>(*ctx, n_rhs, ar, ai, (const double2 *)x, (double2 *)y, reps, kernel_ms, total_ms);
    if (!ctx->ghat32) {
        set_error("dda_matvec_timed: context built without opts.fp32");
        return DDA_ENOTSUP;
    }
    return matvec_timed<float>(*ctx, n_rhs, ar, ai, (const float2 *)x, (float2 *)y, reps, kernel_ms, total_ms);
}

}  // extern "C"

namespace dda {
template <typename R> static Tiles &tiles_ref(Ctx &c) { return sizeof(R) == 8 ? c.tl64 : c.tl32; }

static int log2i(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

template <typename R> static void set_tiles(Ctx &c, int nlx, int nly) {
    Tiles &t = tiles_ref<R>(c);
    t.nl_x = nlx;
    t.nl_y = nly;
    t.lnl_x = log2i(nlx);
    t.lnl_y = log2i(nly);
}

// Tile-schedule autotuner: every admissible lines-per-block count of the x and of the y pass is
// timed on products of a batch of n_rhs zero vectors (HIP events around each kernel); each axis
// keeps its fastest.
template <typename R> static dda_status tune(Ctx &c, int nrhs, int reps, int32_t out[2]) {
    const Tiles saved = tiles_ref<R>(c);
    cplx<R> *x = nullptr, *y = nullptr;
    const size_t bytes = (size_t)3 * nrhs * c.N * sizeof(cplx<R>);
    dda_status st = device_alloc((void **)&x, bytes);
    if (st == DDA_OK) st = device_alloc((void **)&y, bytes);
    if (st == DDA_OK && hipMemsetAsync(x, 0, bytes, c.stream) != hipSuccess) st = DDA_EHIP;
    std::vector<double> ar(nrhs, 0.0), ai(nrhs, 0.0);
    double best_x = 1e300, best_y = 1e300;
    int nlx = saved.nl_x, nly = saved.nl_y;
    for (int nl = 1; nl <= 64 && st == DDA_OK; nl *= 2) {
        const bool okx = tiles_valid<R>(c, 0, nl) && nl <= std::max(1, c.ny);
        const bool oky = tiles_valid<R>(c, 1, nl) && nl <= std::max(1, c.nz);
        if (!okx && !oky) continue;
        set_tiles<R>(c, okx ? nl : saved.nl_x, oky ? nl : saved.nl_y);
        float k[5], tot;
        st = matvec_timed<R>(c, nrhs, ar, ai, x, y, reps, k, &tot);
        if (st != DDA_OK) break;
        if (okx && k[0] + k[4] < best_x) best_x = k[0] + k[4], nlx = nl;
        if (oky && k[1] + k[3] < best_y) best_y = k[1] + k[3], nly = nl;
    }
    if (x) (void)hipFree(x);
    if (y) (void)hipFree(y);
    if (st != DDA_OK) {
        tiles_ref<R>(c) = saved;
        return st;
    }
    set_tiles<R>(c, nlx, nly);
    if (out) {
        out[0] = nlx;
        out[1] = nly;
    }
    return DDA_OK;
}
}  // namespace dda

extern "C" {

dda_status dda_tune(dda_ctx *h, int32_t precision, int32_t n_rhs, int32_t reps, int32_t tiles_out[2]) {
    clear_error();
    Ctx *c = cx(h);
    if (!c || reps < 1 || n_rhs < 1 || (precision != DDA_FP64 && precision != DDA_FP32_REFINE)) {
        set_error("dda_tune: NULL context, reps < 1, n_rhs < 1 or unknown precision");
        return DDA_EINVAL;
    }
    if (precision == DDA_FP32_REFINE && !c->ghat32) {
        set_error("dda_tune: context built without opts.fp32");
        return DDA_ENOTSUP;
    }
    return precision == DDA_FP64 ? tune<double>(*c, n_rhs, reps, tiles_out) : tune<float>(*c, n_rhs, reps, tiles_out);
}

dda_status dda_tune_padding(const int32_t grid[3], const uint8_t *mask, const double m[2], double kd,
                            int32_t polarizability, int32_t n_rhs, int32_t reps, int32_t n_cand, int32_t pad_out[3],
                            float *ms_out) {
    clear_error();
    if (!grid || !mask || !m || !pad_out || n_rhs < 1 || reps < 1 || n_cand < 1 || n_cand > 8) {
        set_error("dda_tune_padding: NULL argument, n_rhs < 1, reps < 1 or n_cand outside 1..8");
        return DDA_EINVAL;
    }
#define DDA_SPEC_ITEM(S) S,
    static const int spec[] = {DDA_SPECIALIZED_LENGTHS(DDA_SPEC_ITEM)};
#undef DDA_SPEC_ITEM
    const int nspec = (int)(sizeof(spec) / sizeof(spec[0]));
    // candidates: the default choice of dda_setup, then the k-th specialized length at or above
    // 2n - 1 on every axis, k = 0 .. n_cand - 1 (each padding once)
    std::vector<std::array<int, 3>> cand{{default_pad(grid[0]), default_pad(grid[1]), default_pad(grid[2])}};
    for (int k = 0; k < n_cand; ++k) {
        std::array<int, 3> c3{};
        bool ok = true;
        for (int a = 0; a < 3 && ok; ++a) {
            int rank = -1;
            for (int i = 0; i < nspec && rank < k; ++i)
                if (spec[i] >= 2 * grid[a] - 1) {
                    ++rank;
                    if (rank == k) c3[a] = spec[i];
                }
            ok = rank == k;
        }
        if (ok && std::find(cand.begin(), cand.end(), c3) == cand.end()) cand.push_back(c3);
    }
    float best = 3.4e38f;
    int best_pad[3] = {0, 0, 0};
    std::string why;
    for (const auto &c3 : cand) {
        dda_setup_opts o{};
        for (int a = 0; a < 3; ++a) o.pad[a] = c3[a];
        Ctx *c = nullptr;
        dda_status st = setup(&c, grid, mask, m, kd, polarizability, &o, nullptr);
        if (st == DDA_EINVAL) {  // a padding these kernels do not run (e.g. too many threads per line)
            why = last_error();
            clear_error();
            continue;
        }
        if (st != DDA_OK) return st;
        if (wrapped(*c)) {
            destroy(c);
            set_error("dda_tune_padding: homogeneous particles only");
            return DDA_ENOTSUP;
        }
        int32_t tiles[2];
        st = tune<double>(*c, n_rhs, reps, tiles);
        double2 *x = nullptr, *y = nullptr;
        const size_t bytes = (size_t)3 * n_rhs * c->N * sizeof(double2);
        if (st == DDA_OK) st = device_alloc((void **)&x, bytes);
        if (st == DDA_OK) st = device_alloc((void **)&y, bytes);
        if (st == DDA_OK && hipMemset(x, 0, bytes) != hipSuccess) st = DDA_EHIP;
        float k[5], tot = 0;
        std::vector<double> ar(n_rhs, 0.0), ai(n_rhs, 0.0);
        if (st == DDA_OK) st = matvec_timed<double>(*c, n_rhs, ar, ai, x, y, reps, k, &tot);
        if (x) (void)hipFree(x);
        if (y) (void)hipFree(y);
        const int L[3] = {c->Lx, c->Ly, c->Lz};
        destroy(c);
        if (st != DDA_OK) return st;
        if (tot < best) {
            best = tot;
            for (int a = 0; a < 3; ++a) best_pad[a] = L[a];
        }
    }
    if (best_pad[0] == 0) {
        set_error("dda_tune_padding: no candidate padding could be set up: " + why);
        return DDA_EINVAL;
    }
    for (int a = 0; a < 3; ++a) pad_out[a] = best_pad[a];
    if (ms_out) *ms_out = best;
    return DDA_OK;
}

dda_status dda_get_tiles(const dda_ctx *h, int32_t precision, int32_t tiles[2]) {
    clear_error();
    const Ctx *c = cx(h);
    if (!c || !tiles || (precision != DDA_FP64 && precision != DDA_FP32_REFINE)) {
        set_error("dda_get_tiles: bad argument");
        return DDA_EINVAL;
    }
    const Tiles &t = precision == DDA_FP64 ? c->tl64 : c->tl32;
    tiles[0] = t.nl_x;
    tiles[1] = t.nl_y;
    return DDA_OK;
}

dda_status dda_set_tiles(dda_ctx *h, int32_t precision, const int32_t tiles[2]) {
    clear_error();
    Ctx *c = cx(h);
    if (!c || !tiles || (precision != DDA_FP64 && precision != DDA_FP32_REFINE)) {
        set_error("dda_set_tiles: bad argument");
        return DDA_EINVAL;
    }
    const bool f64 = precision == DDA_FP64;
    const bool ok = f64 ? tiles_valid<double>(*c, 0, tiles[0]) && tiles_valid<double>(*c, 1, tiles[1])
                        : tiles_valid<float>(*c, 0, tiles[0]) && tiles_valid<float>(*c, 1, tiles[1]);
    if (!ok) {
        set_error("dda_set_tiles: lines per block must be powers of two within the block and LDS limits");
        return DDA_EINVAL;
    }
    DDA_HIP_CHECK(hipStreamSynchronize(c->stream));
    if (f64) set_tiles<double>(*c, tiles[0], tiles[1]);
    else set_tiles<float>(*c, tiles[0], tiles[1]);
    return DDA_OK;
}

const char *dda_strerror(dda_status s) {
    switch (s) {
        case DDA_OK: return "ok";
        case DDA_EINVAL: return "invalid argument";
        case DDA_ENOMEM: return "out of device memory";
        case DDA_EHIP: return "HIP runtime error";
        case DDA_ENOTCONV: return "not converged";
        case DDA_EBREAKDOWN: return "Krylov breakdown";
        case DDA_ESYMMETRY: return "particle lacks the symmetry the read-out needs";
        case DDA_ENOTSUP: return "not supported";
    }
    return "unknown status";
}

const char *dda_last_error(void) { return last_error(); }

}  // extern "C"
