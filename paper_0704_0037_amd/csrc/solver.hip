// Iterative solvers of eq. 3 on the device: complex-symmetric QMR (one interaction-matrix
// product per iteration) and Bi-CGSTAB (two), the two of the paper's four solvers its runs use
// besides Bi-CG (Sec. 2, Sec. 3.1), plus single-precision inner solves inside double-precision
// iterative refinement.
//
// Every right-hand side of a batch carries its own scalar state on the device; the host only
// launches kernels and reads the per-RHS "done" flags every few iterations.  A right-hand side
// that has converged (or broken down) turns every later kernel of its batch into a no-op, so
// over-launching past convergence never changes its iterate.
//
// Vectors are [nrhs][3N] complex (component-major per RHS).  Reductions are per-block partial
// sums in double precision, summed in a fixed order by one block per right-hand side, so results
// are bitwise reproducible run to run.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "ctx.hpp"

namespace dda {

template <typename R> dda_status rhs_launch(Ctx &c, const dda_beam &bm, cplx<R> *b, hipStream_t s);
dda_status pack_setup(Ctx *const *members, int n, Ctx **out);
void destroy(Ctx *c);
bool beam_ok(const dda_beam *b);
void launch_to_f32(const double2 *a, float2 *b, size_t n, hipStream_t s);

enum { ST_RUN = 0, ST_CONV = 1, ST_MAXIT = 2, ST_BREAK = 3 };
constexpr double kBreakdown = 1e-12;  // |v^T v| below this for unit v: Lanczos breakdown
constexpr int kVecThreads = 256;

struct SolveState {
    // QMR
    double rho, gamma_prev, theta_prev, bnorm, res, c2, tol, snorm;
    double2 eps, delta, beta, eta, cp;
    // Bi-CGSTAB
    double2 rho_b, rho_old, alpha, omega, beta_b;
    int iter, status, maxit, pending, half, first, stop_after, pad1;  // stop_after: at the limit, end this iteration
};

// ------------------------------------------------------------------ small helpers
__device__ __forceinline__ double2 dmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ double2 ddiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double dabs(double2 a) { return hypot(a.x, a.y); }
__device__ __forceinline__ bool dfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }

template <typename R> __device__ __forceinline__ double2 up(cplx<R> a) { return make_double2((double)a.x, (double)a.y); }
template <typename R> __device__ __forceinline__ cplx<R> dn(double2 a) { return mk<cplx<R>>((R)a.x, (R)a.y); }

// sum K double2 values over the block (LDS tree, deterministic); result valid in thread 0
template <int K> __device__ __forceinline__ void block_reduce(double2 (&v)[K], double2 *sh) {
    const int t = threadIdx.x;
    for (int k = 0; k < K; ++k) sh[k * kVecThreads + t] = v[k];
    __syncthreads();
    for (int h = kVecThreads / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int k = 0; k < K; ++k) {
                double2 a = sh[k * kVecThreads + t], b = sh[k * kVecThreads + t + h];
                sh[k * kVecThreads + t] = make_double2(a.x + b.x, a.y + b.y);
            }
        __syncthreads();
    }
    if (t == 0)
        for (int k = 0; k < K; ++k) v[k] = sh[k * kVecThreads];
}

// sum partials [nb][K] of one right-hand side into out[K]; every thread of the block gets them
template <int K> __device__ __forceinline__ void sum_partials(const double2 *p, int nb, double2 (&out)[K], double2 *sh) {
    double2 v[K];
    for (int k = 0; k < K; ++k) v[k] = make_double2(0, 0);
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
        for (int k = 0; k < K; ++k) {
            v[k].x += p[b * 4 + k].x;
            v[k].y += p[b * 4 + k].y;
        }
    block_reduce<K>(v, sh);
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < K; ++k) sh[k] = v[k];
    __syncthreads();
    for (int k = 0; k < K; ++k) out[k] = sh[k];
    __syncthreads();
}

#define VEC_LOOP(n3) for (size_t i = (size_t)blockIdx.x * kVecThreads + threadIdx.x; i < (n3); i += (size_t)gridDim.x * kVecThreads)

// ============================================================================ QMR
// r = b - Ax0 (Ax0 given) or b; vt = r; x zeroed when there is no initial guess.
// partials: (|b|^2, |vt|^2), vt^T vt
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_qmr_init(const cplx<R> *b, const cplx<R> *ax, cplx<R> *x, cplx<R> *r,
                                                          cplx<R> *vt, size_t n3, double2 *part, int zero_x) {
    __shared__ double2 sh[2 * kVecThreads];
    const int rhs = blockIdx.y;
    const size_t off = (size_t)rhs * n3;
    double2 acc[2] = {make_double2(0, 0), make_double2(0, 0)};
    VEC_LOOP(n3) {
        const cplx<R> bi = b[off + i];
        cplx<R> ri = bi;
        if (ax) ri = csub(bi, ax[off + i]);
        if (zero_x) x[off + i] = czero<cplx<R>>();
        r[off + i] = ri;
        vt[off + i] = ri;
        const double2 bd = up<R>(bi), rd = up<R>(ri);
        acc[0].x += bd.x * bd.x + bd.y * bd.y;
        acc[0].y += rd.x * rd.x + rd.y * rd.y;
        acc[1].x += rd.x * rd.x - rd.y * rd.y;  // bilinear r^T r
        acc[1].y += 2 * rd.x * rd.y;
    }
    block_reduce<2>(acc, sh);
    if (threadIdx.x == 0) {
        double2 *p = part + ((size_t)rhs * gridDim.x + blockIdx.x) * 4;
        p[0] = acc[0];
        p[1] = acc[1];
    }
}

__global__ void k_qmr_scal_init(SolveState *st, int *done, const double2 *part, int nb, double *hist, int hcap) {
    __shared__ double2 sh[2 * kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;  // excluded from this solve by the caller
    double2 s[2];
    sum_partials<2>(part + (size_t)rhs * nb * 4, nb, s, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    S.bnorm = sqrt(s[0].x);
    S.rho = sqrt(s[0].y);
    S.res = S.bnorm > 0 ? S.rho / S.bnorm : 0.0;
    S.gamma_prev = 1.0;
    S.theta_prev = 0.0;
    S.eta = make_double2(-1.0, 0.0);
    S.iter = 0;
    S.pending = 0;
    S.first = 1;
    S.status = ST_RUN;
    if (hist && hcap > 0) hist[(size_t)rhs * hcap] = S.res;
    if (S.res < S.tol || S.bnorm == 0.0) {
        S.status = ST_CONV;
        done[rhs] = 1;
        return;
    }
    const double r2 = S.rho * S.rho;
    S.delta = make_double2(s[1].x / r2, s[1].y / r2);  // v^T v with v = vt / rho
    if (dabs(S.delta) < kBreakdown || !dfinite(S.delta)) {
        S.status = ST_BREAK;
        done[rhs] = 1;
        return;
    }
    S.cp = make_double2(0, 0);
    done[rhs] = 0;
}

// first iteration: p = vt / rho
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_qmr_p0(const SolveState *st, const int *done, const cplx<R> *vt,
                                                        cplx<R> *p, size_t n3) {
    const int rhs = blockIdx.y;
    if (done[rhs]) return;
    const size_t off = (size_t)rhs * n3;
    const R inv = (R)(1.0 / st[rhs].rho);
    VEC_LOOP(n3) p[off + i] = cscale(vt[off + i], inv);
}

// eps = p^T A p from the matvec epilogue partials; beta = eps / delta
template <typename R>
__global__ void k_qmr_scal_eps(SolveState *st, int *done, const cplx<R> *dots, int ndots) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;
    double2 v[1] = {make_double2(0, 0)};
    for (int b = threadIdx.x; b < ndots; b += blockDim.x) {
        const double2 d = up<R>(dots[(size_t)rhs * ndots + b]);
        v[0].x += d.x;
        v[0].y += d.y;
    }
    block_reduce<1>(v, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    S.eps = v[0];
    if ((S.eps.x == 0 && S.eps.y == 0) || !dfinite(S.eps)) {
        S.status = ST_BREAK;
        done[rhs] = 1;
        return;
    }
    S.beta = ddiv(S.eps, S.delta);
}

// vt = pt - (beta / rho) vt; partials |vt|^2, vt^T vt
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_qmr_vt(const SolveState *st, const int *done, const cplx<R> *pt,
                                                        cplx<R> *vt, size_t n3, double2 *part) {
    __shared__ double2 sh[2 * kVecThreads];
    const int rhs = blockIdx.y;
    if (done[rhs]) return;
    const size_t off = (size_t)rhs * n3;
    const SolveState &S = st[rhs];
    const cplx<R> c = dn<R>(make_double2(S.beta.x / S.rho, S.beta.y / S.rho));
    double2 acc[2] = {make_double2(0, 0), make_double2(0, 0)};
    VEC_LOOP(n3) {
        const cplx<R> v = csub(pt[off + i], cmul(c, vt[off + i]));
        vt[off + i] = v;
        const double2 d = up<R>(v);
        acc[0].x += d.x * d.x + d.y * d.y;
        acc[1].x += d.x * d.x - d.y * d.y;
        acc[1].y += 2 * d.x * d.y;
    }
    block_reduce<2>(acc, sh);
    if (threadIdx.x == 0) {
        double2 *p = part + ((size_t)rhs * gridDim.x + blockIdx.x) * 4;
        p[0] = acc[0];
        p[1] = acc[1];
    }
}

// rho_new, theta, gamma, eta and the coefficients of the update pass
__global__ void k_qmr_scal_2(SolveState *st, int *done, const double2 *part, int nb) {
    __shared__ double2 sh[2 * kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;
    double2 s[2];
    sum_partials<2>(part + (size_t)rhs * nb * 4, nb, s, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    const double rho_new = sqrt(s[0].x);
    const double bmod = dabs(S.beta);
    const double theta = rho_new / (S.gamma_prev * bmod);
    const double gamma = 1.0 / sqrt(1.0 + theta * theta);
    // eta = -eta rho gamma^2 / (beta gamma_prev^2)
    const double f = S.rho * gamma * gamma / (S.gamma_prev * S.gamma_prev);
    const double2 q = ddiv(make_double2(S.eta.x * f, S.eta.y * f), S.beta);
    S.eta = make_double2(-q.x, -q.y);
    S.c2 = (S.theta_prev * gamma) * (S.theta_prev * gamma);
    S.theta_prev = theta;
    S.gamma_prev = gamma;
    S.rho = rho_new;
    if (rho_new == 0.0 || !isfinite(rho_new)) {
        // rho_new = 0: the Krylov space is exhausted; not finite: the Lanczos recurrence has
        // overflowed.  Either way this update is the last one, and the right-hand side stops as
        // converged only if its residual meets tol (else breakdown)
        S.cp = make_double2(0, 0);
        S.pending = rho_new == 0.0 ? 1 : 2;
        return;
    }
    const double r2 = rho_new * rho_new;
    S.delta = make_double2(s[1].x / r2, s[1].y / r2);
    if (dabs(S.delta) < kBreakdown || !dfinite(S.delta)) {
        S.cp = make_double2(0, 0);
        S.pending = 2;  // breakdown after this update
        return;
    }
    // p_next = vt / rho_new - (rho_new delta / eps) p
    S.cp = ddiv(make_double2(rho_new * S.delta.x, rho_new * S.delta.y), S.eps);
}

// d = eta p + c2 d;  s = eta pt + c2 s;  x += d;  r -= s;  p = vt / rho - cp p;  partial |r|^2
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_qmr_update(const SolveState *st, const int *done, cplx<R> *p,
                                                            const cplx<R> *pt, const cplx<R> *vt, cplx<R> *d,
                                                            cplx<R> *s, cplx<R> *x, cplx<R> *r, size_t n3,
                                                            double2 *part) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.y;
    if (done[rhs]) return;
    const size_t off = (size_t)rhs * n3;
    const SolveState &S = st[rhs];
    const cplx<R> eta = dn<R>(S.eta), cp = dn<R>(S.cp);
    const R c2 = (R)S.c2, inv = (R)(S.rho > 0 ? 1.0 / S.rho : 0.0);
    const bool first = S.first;
    double2 acc[1] = {make_double2(0, 0)};
    VEC_LOOP(n3) {
        const cplx<R> pi = p[off + i], pti = pt[off + i];
        cplx<R> di = cmul(eta, pi), si = cmul(eta, pti);
        if (!first) {
            di = cadd(di, cscale(d[off + i], c2));
            si = cadd(si, cscale(s[off + i], c2));
        }
        d[off + i] = di;
        s[off + i] = si;
        x[off + i] = cadd(x[off + i], di);
        const cplx<R> ri = csub(r[off + i], si);
        r[off + i] = ri;
        p[off + i] = csub(cscale(vt[off + i], inv), cmul(cp, pi));
        const double2 rd = up<R>(ri);
        acc[0].x += rd.x * rd.x + rd.y * rd.y;
    }
    block_reduce<1>(acc, sh);
    if (threadIdx.x == 0) part[((size_t)rhs * gridDim.x + blockIdx.x) * 4] = acc[0];
}

__global__ void k_qmr_scal_3(SolveState *st, int *done, const double2 *part, int nb, double *hist, int hcap) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;
    double2 s[1];
    sum_partials<1>(part + (size_t)rhs * nb * 4, nb, s, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    S.first = 0;
    S.iter += 1;
    S.res = sqrt(s[0].x) / S.bnorm;
    if (hist && hcap > 0) hist[(size_t)rhs * hcap + (S.iter < hcap ? S.iter : hcap - 1)] = S.res;
    if (!isfinite(S.res)) {
        S.status = ST_BREAK;
        done[rhs] = 1;
    } else if (S.res < S.tol) {
        S.status = ST_CONV;
        done[rhs] = 1;
    } else if (S.pending != 0) {  // exhausted Krylov space, vanished v^T v or overflow, tol not met
        S.status = ST_BREAK;
        done[rhs] = 1;
    } else if (S.iter >= S.maxit) {
        S.status = ST_MAXIT;
        done[rhs] = 1;
    }
}

// ====================================================================== Bi-CG (complex symmetric)
// One product per iteration on the bilinear form u^T v (Sec. 2: Bi-CG uses the complex symmetry
// of the interaction matrix).  Initialization reuses k_qmr_init with p as its copy of r:
// partials (|b|^2, |r|^2) and r^T r.
__global__ void k_bicg_scal_init(SolveState *st, int *done, const double2 *part, int nb, double *hist, int hcap) {
    __shared__ double2 sh[2 * kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;  // excluded from this solve by the caller
    double2 s[2];
    sum_partials<2>(part + (size_t)rhs * nb * 4, nb, s, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    S.bnorm = sqrt(s[0].x);
    S.res = S.bnorm > 0 ? sqrt(s[0].y) / S.bnorm : 0.0;
    S.rho_b = s[1];  // r^T r
    S.iter = 0;
    S.pending = 0;
    S.status = ST_RUN;
    if (hist && hcap > 0) hist[(size_t)rhs * hcap] = S.res;
    if (S.res < S.tol || S.bnorm == 0.0) {
        S.status = ST_CONV;
        done[rhs] = 1;
        return;
    }
    if (dabs(S.rho_b) < kBreakdown * s[0].y || !dfinite(S.rho_b)) {  // r^T r = 0: no Bi-CG step
        S.status = ST_BREAK;
        done[rhs] = 1;
        return;
    }
    done[rhs] = 0;
}

// eps = p^T A p from the matvec epilogue partials; alpha = rho / eps
template <typename R>
__global__ void k_bicg_scal_alpha(SolveState *st, int *done, const cplx<R> *dots, int ndots) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;
    double2 v[1] = {make_double2(0, 0)};
    for (int b = threadIdx.x; b < ndots; b += blockDim.x) {
        const double2 d = up<R>(dots[(size_t)rhs * ndots + b]);
        v[0].x += d.x;
        v[0].y += d.y;
    }
    block_reduce<1>(v, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    S.eps = v[0];
    if ((S.eps.x == 0 && S.eps.y == 0) || !dfinite(S.eps)) {
        S.status = ST_BREAK;
        done[rhs] = 1;
        return;
    }
    S.alpha = ddiv(S.rho_b, S.eps);
}

// x += alpha p;  r -= alpha q;  partials |r|^2, r^T r
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_bicg_update(const SolveState *st, const int *done,
                                                             const cplx<R> *__restrict__ p, const cplx<R> *__restrict__ q,
                                                             cplx<R> *__restrict__ x, cplx<R> *__restrict__ r, size_t n3,
                                                             double2 *part) {
    __shared__ double2 sh[2 * kVecThreads];
    const int rhs = blockIdx.y;
    if (done[rhs]) return;
    const size_t off = (size_t)rhs * n3;
    const cplx<R> a = dn<R>(st[rhs].alpha);
    double2 acc[2] = {make_double2(0, 0), make_double2(0, 0)};
    VEC_LOOP(n3) {
        x[off + i] = cadd(x[off + i], cmul(a, p[off + i]));
        const cplx<R> ri = csub(r[off + i], cmul(a, q[off + i]));
        r[off + i] = ri;
        const double2 d = up<R>(ri);
        acc[0].x += d.x * d.x + d.y * d.y;
        acc[1].x += d.x * d.x - d.y * d.y;
        acc[1].y += 2 * d.x * d.y;
    }
    block_reduce<2>(acc, sh);
    if (threadIdx.x == 0) {
        double2 *pp = part + ((size_t)rhs * gridDim.x + blockIdx.x) * 4;
        pp[0] = acc[0];
        pp[1] = acc[1];
    }
}

// residual, stopping rule; beta = rho_new / rho
__global__ void k_bicg_scal_2(SolveState *st, int *done, const double2 *part, int nb, double *hist, int hcap) {
    __shared__ double2 sh[2 * kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;
    double2 s[2];
    sum_partials<2>(part + (size_t)rhs * nb * 4, nb, s, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    S.iter += 1;
    S.res = sqrt(s[0].x) / S.bnorm;
    if (hist && hcap > 0) hist[(size_t)rhs * hcap + (S.iter < hcap ? S.iter : hcap - 1)] = S.res;
    if (S.res < S.tol) {
        S.status = ST_CONV;
        done[rhs] = 1;
    } else if (!isfinite(S.res) || dabs(s[1]) < kBreakdown * s[0].x || !dfinite(s[1])) {
        S.status = ST_BREAK;
        done[rhs] = 1;
    } else {
        S.beta_b = ddiv(s[1], S.rho_b);
        S.rho_b = s[1];
        // at the limit the iteration still forms p, so that a continued solve starts from a whole
        // iteration (k_stop_after ends it)
        if (S.iter >= S.maxit) S.stop_after = 1;
    }
}

// end of an iteration: a right-hand side that reached its limit stops here
__global__ void k_stop_after(SolveState *st, int *done, int nrhs) {
    const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
    if (rhs >= nrhs || done[rhs]) return;
    SolveState &S = st[rhs];
    if (S.stop_after) {
        S.stop_after = 0;
        S.status = ST_MAXIT;
        done[rhs] = 1;
    }
}

// p = r + beta p
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_bicg_p(const SolveState *st, const int *done,
                                                        const cplx<R> *__restrict__ r, cplx<R> *__restrict__ p,
                                                        size_t n3) {
    const int rhs = blockIdx.y;
    if (done[rhs]) return;
    const size_t off = (size_t)rhs * n3;
    const cplx<R> b = dn<R>(st[rhs].beta_b);
    VEC_LOOP(n3) p[off + i] = cadd(r[off + i], cmul(b, p[off + i]));
}

// ====================================================================== CGNR
// Conjugate gradients on the normal equations A^H A x = A^H b (Sec. 2's CGNR); A is complex
// symmetric, so A^H v = conj(A conj(v)): the product runs on t = conj(r) and its result d is
// conjugated where it is read.  Two products per iteration; g = ||A^H r||^2.

// r = b - Ax0 (Ax0 given) or b; t = conj(r); x zeroed without a guess; partials (|b|^2, |r|^2)
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_cgnr_init(const cplx<R> *__restrict__ b, const cplx<R> *__restrict__ ax,
                                                           cplx<R> *__restrict__ x, cplx<R> *__restrict__ r,
                                                           cplx<R> *__restrict__ t, size_t n3, double2 *part,
                                                           int zero_x) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.y;
    const size_t off = (size_t)rhs * n3;
    double2 acc[1] = {make_double2(0, 0)};
    VEC_LOOP(n3) {
        const cplx<R> bi = b[off + i];
        const cplx<R> ri = ax ? csub(bi, ax[off + i]) : bi;
        if (zero_x) x[off + i] = czero<cplx<R>>();
        r[off + i] = ri;
        t[off + i] = cconj(ri);
        const double2 bd = up<R>(bi), rd = up<R>(ri);
        acc[0].x += bd.x * bd.x + bd.y * bd.y;
        acc[0].y += rd.x * rd.x + rd.y * rd.y;
    }
    block_reduce<1>(acc, sh);
    if (threadIdx.x == 0) part[((size_t)rhs * gridDim.x + blockIdx.x) * 4] = acc[0];
}

__global__ void k_cgnr_scal_init(SolveState *st, int *done, const double2 *part, int nb, double *hist, int hcap) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;  // excluded from this solve by the caller
    double2 s[1];
    sum_partials<1>(part + (size_t)rhs * nb * 4, nb, s, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    S.bnorm = sqrt(s[0].x);
    S.res = S.bnorm > 0 ? sqrt(s[0].y) / S.bnorm : 0.0;
    S.iter = 0;
    S.pending = 0;
    S.status = ST_RUN;
    if (hist && hcap > 0) hist[(size_t)rhs * hcap] = S.res;
    if (S.res < S.tol || S.bnorm == 0.0) {
        S.status = ST_CONV;
        done[rhs] = 1;
        return;
    }
    done[rhs] = 0;
}

// sum of |v|^2 over a vector into part slot 0 (v = A p, or d = A conj(r) whose conjugate has the
// same norm)
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_cgnr_norm(const int *done, const cplx<R> *__restrict__ v, size_t n3,
                                                           double2 *part) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.y;
    if (done[rhs]) return;
    const size_t off = (size_t)rhs * n3;
    double2 acc[1] = {make_double2(0, 0)};
    VEC_LOOP(n3) {
        const double2 d = up<R>(v[off + i]);
        acc[0].x += d.x * d.x + d.y * d.y;
    }
    block_reduce<1>(acc, sh);
    if (threadIdx.x == 0) part[((size_t)rhs * gridDim.x + blockIdx.x) * 4] = acc[0];
}

// which = 0: g = ||z||^2 of the first direction;  1: alpha = g / ||w||^2;  2: beta = g_new / g
__global__ void k_cgnr_scal(SolveState *st, int *done, const double2 *part, int nb, int which) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;
    double2 s[1];
    sum_partials<1>(part + (size_t)rhs * nb * 4, nb, s, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    const double v = s[0].x;
    if (!(v > 0) || !isfinite(v)) {  // A^H r = 0 or A p = 0 with r != 0
        S.status = ST_BREAK;
        done[rhs] = 1;
        return;
    }
    if (which == 0) {
        S.rho = v;
    } else if (which == 1) {
        S.alpha = make_double2(S.rho / v, 0);
    } else {
        S.beta_b = make_double2(v / S.rho, 0);
        S.rho = v;
    }
}

// p = conj(d) (first direction);  or p = conj(d) + beta p
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_cgnr_p(const SolveState *st, const int *done,
                                                        const cplx<R> *__restrict__ d, cplx<R> *__restrict__ p,
                                                        size_t n3, int first) {
    const int rhs = blockIdx.y;
    if (done[rhs]) return;
    const size_t off = (size_t)rhs * n3;
    const R b = first ? (R)0 : (R)st[rhs].beta_b.x;
    VEC_LOOP(n3) {
        const cplx<R> z = cconj(d[off + i]);
        p[off + i] = first ? z : cadd(z, cscale(p[off + i], b));
    }
}

// x += alpha p;  r -= alpha w;  t = conj(r);  partials |r|^2
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_cgnr_update(const SolveState *st, const int *done,
                                                             const cplx<R> *__restrict__ p, const cplx<R> *__restrict__ w,
                                                             cplx<R> *__restrict__ x, cplx<R> *__restrict__ r,
                                                             cplx<R> *__restrict__ t, size_t n3, double2 *part) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.y;
    if (done[rhs]) return;
    const size_t off = (size_t)rhs * n3;
    const R a = (R)st[rhs].alpha.x;
    double2 acc[1] = {make_double2(0, 0)};
    VEC_LOOP(n3) {
        x[off + i] = cadd(x[off + i], cscale(p[off + i], a));
        const cplx<R> ri = csub(r[off + i], cscale(w[off + i], a));
        r[off + i] = ri;
        t[off + i] = cconj(ri);
        const double2 d = up<R>(ri);
        acc[0].x += d.x * d.x + d.y * d.y;
    }
    block_reduce<1>(acc, sh);
    if (threadIdx.x == 0) part[((size_t)rhs * gridDim.x + blockIdx.x) * 4] = acc[0];
}

// residual and stopping rule after an update
__global__ void k_cgnr_scal_res(SolveState *st, int *done, const double2 *part, int nb, double *hist, int hcap) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;
    double2 s[1];
    sum_partials<1>(part + (size_t)rhs * nb * 4, nb, s, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    S.iter += 1;
    S.res = sqrt(s[0].x) / S.bnorm;
    if (hist && hcap > 0) hist[(size_t)rhs * hcap + (S.iter < hcap ? S.iter : hcap - 1)] = S.res;
    if (S.res < S.tol) {
        S.status = ST_CONV;
        done[rhs] = 1;
    } else if (!isfinite(S.res)) {
        S.status = ST_BREAK;
        done[rhs] = 1;
    } else if (S.iter >= S.maxit) {
        S.stop_after = 1;  // the iteration still forms the next direction (k_stop_after ends it)
    }
}

// ====================================================================== Bi-CGSTAB
// r = b - Ax0 or b; rs = r; partials (|b|^2, |r|^2)
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_bi_init(const cplx<R> *b, const cplx<R> *ax, cplx<R> *x, cplx<R> *r,
                                                         cplx<R> *rs, size_t n3, double2 *part, int zero_x) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.y;
    const size_t off = (size_t)rhs * n3;
    double2 acc[1] = {make_double2(0, 0)};
    VEC_LOOP(n3) {
        const cplx<R> bi = b[off + i];
        cplx<R> ri = bi;
        if (ax) ri = csub(bi, ax[off + i]);
        if (zero_x) x[off + i] = czero<cplx<R>>();
        r[off + i] = ri;
        rs[off + i] = ri;
        const double2 bd = up<R>(bi), rd = up<R>(ri);
        acc[0].x += bd.x * bd.x + bd.y * bd.y;
        acc[0].y += rd.x * rd.x + rd.y * rd.y;
    }
    block_reduce<1>(acc, sh);
    if (threadIdx.x == 0) part[((size_t)rhs * gridDim.x + blockIdx.x) * 4] = acc[0];
}

__global__ void k_bi_scal_init(SolveState *st, int *done, const double2 *part, int nb, double *hist, int hcap) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;
    double2 s[1];
    sum_partials<1>(part + (size_t)rhs * nb * 4, nb, s, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    S.bnorm = sqrt(s[0].x);
    const double rn = sqrt(s[0].y);
    S.res = S.bnorm > 0 ? rn / S.bnorm : 0.0;
    S.rho_b = make_double2(s[0].y, 0.0);  // rs^H r = |r|^2 at the start
    S.rho_old = S.alpha = S.omega = make_double2(1, 0);
    S.iter = 0;
    S.half = 0;
    S.first = 1;
    S.status = ST_RUN;
    if (hist && hcap > 0) hist[(size_t)rhs * hcap] = S.res;
    if (S.res < S.tol || S.bnorm == 0.0) {
        S.status = ST_CONV;
        done[rhs] = 1;
        return;
    }
    done[rhs] = 0;
}

// beta = (rho/rho_old)(alpha/omega); p = r + beta (p - omega v)   (p = r at the first iteration)
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_bi_p(SolveState *st, const int *done, const cplx<R> *r, cplx<R> *p,
                                                      const cplx<R> *v, size_t n3) {
    const int rhs = blockIdx.y;
    if (done[rhs]) return;
    const size_t off = (size_t)rhs * n3;
    const SolveState &S = st[rhs];
    const bool first = S.first;
    const double2 bd = dmul(ddiv(S.rho_b, S.rho_old), ddiv(S.alpha, S.omega));
    const cplx<R> beta = dn<R>(bd), om = dn<R>(S.omega);
    VEC_LOOP(n3) {
        if (first) p[off + i] = r[off + i];
        else p[off + i] = cadd(r[off + i], cmul(beta, csub(p[off + i], cmul(om, v[off + i]))));
    }
}

// partials of u^H w and (optionally) u^H u over one right-hand side
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_bi_dots(const int *done, const cplx<R> *u, const cplx<R> *w,
                                                         size_t n3, double2 *part, int with_uu) {
    __shared__ double2 sh[2 * kVecThreads];
    const int rhs = blockIdx.y;
    if (done[rhs]) return;
    const size_t off = (size_t)rhs * n3;
    double2 acc[2] = {make_double2(0, 0), make_double2(0, 0)};
    VEC_LOOP(n3) {
        const double2 a = up<R>(u[off + i]), b = up<R>(w[off + i]);
        acc[0].x += a.x * b.x + a.y * b.y;  // conj(a) b
        acc[0].y += a.x * b.y - a.y * b.x;
        if (with_uu) acc[1].x += a.x * a.x + a.y * a.y;
    }
    block_reduce<2>(acc, sh);
    if (threadIdx.x == 0) {
        double2 *p = part + ((size_t)rhs * gridDim.x + blockIdx.x) * 4;
        p[0] = acc[0];
        p[1] = acc[1];
    }
}

// alpha = rho / (rs^H v)
__global__ void k_bi_scal_alpha(SolveState *st, int *done, const double2 *part, int nb) {
    __shared__ double2 sh[2 * kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;
    double2 s[2];
    sum_partials<2>(part + (size_t)rhs * nb * 4, nb, s, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    if ((s[0].x == 0 && s[0].y == 0) || !dfinite(s[0])) {
        S.status = ST_BREAK;
        done[rhs] = 1;
        return;
    }
    S.alpha = ddiv(S.rho_b, s[0]);
}

// s = r - alpha v; partial |s|^2
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_bi_s(const SolveState *st, const int *done, const cplx<R> *r,
                                                      const cplx<R> *v, cplx<R> *s, size_t n3, double2 *part) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.y;
    if (done[rhs]) return;
    const size_t off = (size_t)rhs * n3;
    const cplx<R> a = dn<R>(st[rhs].alpha);
    double2 acc[1] = {make_double2(0, 0)};
    VEC_LOOP(n3) {
        const cplx<R> si = csub(r[off + i], cmul(a, v[off + i]));
        s[off + i] = si;
        const double2 d = up<R>(si);
        acc[0].x += d.x * d.x + d.y * d.y;
    }
    block_reduce<1>(acc, sh);
    if (threadIdx.x == 0) part[((size_t)rhs * gridDim.x + blockIdx.x) * 4] = acc[0];
}

__global__ void k_bi_scal_s(SolveState *st, const int *done, const double2 *part, int nb) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;
    double2 s[1];
    sum_partials<1>(part + (size_t)rhs * nb * 4, nb, s, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    S.snorm = sqrt(s[0].x);
    S.half = (S.snorm / S.bnorm < S.tol) ? 1 : 0;
}

// omega = (t^H s) / (t^H t), or 0 when s already met the tolerance
__global__ void k_bi_scal_omega(SolveState *st, int *done, const double2 *part, int nb) {
    __shared__ double2 sh[2 * kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;
    double2 s[2];
    sum_partials<2>(part + (size_t)rhs * nb * 4, nb, s, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    if (S.half) {
        S.omega = make_double2(0, 0);
        return;
    }
    if (s[1].x == 0 || !isfinite(s[1].x)) {
        S.status = ST_BREAK;
        done[rhs] = 1;
        return;
    }
    S.omega = make_double2(s[0].x / s[1].x, s[0].y / s[1].x);
}

// x += alpha p + omega s;  r = s - omega t;  partials |r|^2, rs^H r
template <typename R>
__global__ void __launch_bounds__(kVecThreads) k_bi_x(const SolveState *st, const int *done, const cplx<R> *p,
                                                      const cplx<R> *s, const cplx<R> *t, const cplx<R> *rs,
                                                      cplx<R> *x, cplx<R> *r, size_t n3, double2 *part) {
    __shared__ double2 sh[2 * kVecThreads];
    const int rhs = blockIdx.y;
    if (done[rhs]) return;
    const size_t off = (size_t)rhs * n3;
    const SolveState &S = st[rhs];
    const cplx<R> a = dn<R>(S.alpha), om = dn<R>(S.omega);
    double2 acc[2] = {make_double2(0, 0), make_double2(0, 0)};
    VEC_LOOP(n3) {
        const cplx<R> si = s[off + i];
        x[off + i] = cadd(x[off + i], cadd(cmul(a, p[off + i]), cmul(om, si)));
        const cplx<R> ri = csub(si, cmul(om, t[off + i]));
        r[off + i] = ri;
        const double2 rd = up<R>(ri), q = up<R>(rs[off + i]);
        acc[0].x += rd.x * rd.x + rd.y * rd.y;
        acc[1].x += q.x * rd.x + q.y * rd.y;
        acc[1].y += q.x * rd.y - q.y * rd.x;
    }
    block_reduce<2>(acc, sh);
    if (threadIdx.x == 0) {
        double2 *pp = part + ((size_t)rhs * gridDim.x + blockIdx.x) * 4;
        pp[0] = acc[0];
        pp[1] = acc[1];
    }
}

__global__ void k_bi_scal_end(SolveState *st, int *done, const double2 *part, int nb, double *hist, int hcap) {
    __shared__ double2 sh[2 * kVecThreads];
    const int rhs = blockIdx.x;
    if (done[rhs]) return;
    double2 s[2];
    sum_partials<2>(part + (size_t)rhs * nb * 4, nb, s, sh);
    if (threadIdx.x != 0) return;
    SolveState &S = st[rhs];
    S.first = 0;
    S.iter += 1;
    S.res = S.half ? S.snorm / S.bnorm : sqrt(s[0].x) / S.bnorm;
    if (hist && hcap > 0) hist[(size_t)rhs * hcap + (S.iter < hcap ? S.iter : hcap - 1)] = S.res;
    S.rho_old = S.rho_b;
    S.rho_b = s[1];
    if (S.res < S.tol || S.half) {
        S.status = ST_CONV;
        done[rhs] = 1;
    } else if (!isfinite(S.res) || (S.rho_b.x == 0 && S.rho_b.y == 0) || (S.omega.x == 0 && S.omega.y == 0)) {
        S.status = ST_BREAK;
        done[rhs] = 1;
    } else if (S.iter >= S.maxit) {
        S.status = ST_MAXIT;
        done[rhs] = 1;
    }
}

// ================================================================ refinement helpers
// r64 = b - ax; partial (|r|^2, |b|^2)
__global__ void __launch_bounds__(kVecThreads) k_resid(const double2 *b, const double2 *ax, double2 *r, size_t n3,
                                                       double2 *part) {
    __shared__ double2 sh[kVecThreads];
    const int rhs = blockIdx.y;
    const size_t off = (size_t)rhs * n3;
    double2 acc[1] = {make_double2(0, 0)};
    VEC_LOOP(n3) {
        const double2 bi = b[off + i], ri = make_double2(bi.x - ax[off + i].x, bi.y - ax[off + i].y);
        if (r) r[off + i] = ri;
        acc[0].x += ri.x * ri.x + ri.y * ri.y;
        acc[0].y += bi.x * bi.x + bi.y * bi.y;
    }
    block_reduce<1>(acc, sh);
    if (threadIdx.x == 0) part[((size_t)rhs * gridDim.x + blockIdx.x) * 4] = acc[0];
}

// r32 = r64 * scale[rhs]  (scale = 1/|r|)
__global__ void k_to32(const double2 *r, float2 *r32, size_t n3, const double *scale) {
    const int rhs = blockIdx.y;
    const size_t off = (size_t)rhs * n3;
    const double sc = scale[rhs];
    VEC_LOOP(n3) r32[off + i] = make_float2((float)(r[off + i].x * sc), (float)(r[off + i].y * sc));
}

// x64 += e32 * scale[rhs] (only for right-hand sides still refining)
__global__ void k_addup(double2 *x, const float2 *e, size_t n3, const double *scale, const int *active) {
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t off = (size_t)rhs * n3;
    const double sc = 1.0 / scale[rhs];
    VEC_LOOP(n3) {
        x[off + i].x += (double)e[off + i].x * sc;
        x[off + i].y += (double)e[off + i].y * sc;
    }
}

__global__ void k_sum_part(const double2 *part, int nb, double2 *out) {
    __shared__ double2 sh[kVecThreads];
    double2 s[1];
    sum_partials<1>(part + (size_t)blockIdx.x * nb * 4, nb, s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

__global__ void k_zero(double2 *x, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] = make_double2(0, 0);
}

// ==================================================================== host driver
struct Bufs {
    int nrhs = 0;
    size_t n3 = 0;
    int nb = 0;
    SolveState *st = nullptr;
    int *done = nullptr;
    double2 *part = nullptr;
    double *hist = nullptr;
    int hcap = 0;
    double2 *scratch = nullptr;  // 4 nrhs + 16 entries of small device scratch
};

template <typename R> struct Vecs {
    cplx<R> *b, *r, *vt, *p, *pt, *d, *s, *rs, *v, *t;
};

template <typename R> static cplx<R> *vec_base(Ctx &c);
template <> double2 *vec_base<double>(Ctx &c) { return c.vecs; }
template <> float2 *vec_base<float>(Ctx &c) { return c.vecs32; }

static constexpr int kNumVecs = 9;  // b r vt p pt d s (QMR) / b r rs p v s t (Bi-CGSTAB)

template <typename R> static dda_status ensure_vecs(Ctx &c, int nrhs) {
    const size_t need = (size_t)kNumVecs * nrhs * 3 * c.N;
    size_t &have = std::is_same<R, double>::value ? c.vecs_elems : c.vecs32_elems;
    if (have >= need) return DDA_OK;
    DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
    if (std::is_same<R, double>::value) {
        (void)hipFree(c.vecs);
        c.vecs = nullptr;
        c.vecs_elems = 0;
        dda_status st = device_alloc((void **)&c.vecs, need * sizeof(double2));
        if (st != DDA_OK) return st;
        c.vecs_elems = need;
    } else {
        (void)hipFree(c.vecs32);
        c.vecs32 = nullptr;
        c.vecs32_elems = 0;
        dda_status st = device_alloc((void **)&c.vecs32, need * sizeof(float2));
        if (st != DDA_OK) return st;
        c.vecs32_elems = need;
    }
    return DDA_OK;
}

template <typename R> static Vecs<R> vecs_of(Ctx &c, int nrhs) {
    cplx<R> *base = vec_base<R>(c);
    const size_t L = (size_t)nrhs * 3 * c.N;
    Vecs<R> v;
    v.b = base;
    v.r = base + L;
    v.vt = base + 2 * L;
    v.p = base + 3 * L;
    v.pt = base + 4 * L;
    v.d = base + 5 * L;
    v.s = base + 6 * L;
    v.rs = v.vt;   // Bi-CGSTAB reuses the QMR slots
    v.v = v.pt;
    v.t = v.d;
    return v;
}

// device scales alpha / (Lx Ly Lz) per right-hand side, in the work buffer of precision R
template <typename R> static dda_status upload_scales(Ctx &c, const std::vector<double> &ar, const std::vector<double> &ai) {
    dda_status st = ensure_work<R>(c, (int)ar.size());
    if (st != DDA_OK) return st;
    Work<R> &w = work_of<R>(c);
    std::vector<cplx<R>> sc(ar.size());
    const double inv = 1.0 / ((double)c.Lx * c.Ly * c.Lz);
    for (size_t r = 0; r < ar.size(); ++r) sc[r] = mk<cplx<R>>((R)(ar[r] * inv), (R)(ai[r] * inv));
    DDA_HIP_CHECK(hipMemcpyAsync(w.scale, sc.data(), sc.size() * sizeof(cplx<R>), hipMemcpyHostToDevice, c.stream));
    DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
    return DDA_OK;
}

static dda_status ensure_bufs(Ctx &c, Bufs &B, int nrhs, int hcap) {
    B.nrhs = nrhs;
    B.n3 = (size_t)3 * c.N;
    B.nb = (int)std::min<size_t>(1024, (B.n3 + kVecThreads * 4 - 1) / (kVecThreads * 4));
    if (B.nb < 1) B.nb = 1;
    B.hcap = hcap;
    const size_t bytes = nrhs * sizeof(SolveState) + 256 + nrhs * sizeof(int) * 2 + 256 +
                         (size_t)nrhs * B.nb * 4 * sizeof(double2) + 256 + (size_t)nrhs * hcap * sizeof(double) + 256 +
                         (4 * (size_t)nrhs + 16) * sizeof(double2) + 256;
    if (c.sbuf_bytes < bytes) {
        DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
        (void)hipFree(c.sbuf);
        c.sbuf = nullptr;
        c.sbuf_bytes = 0;
        dda_status st = device_alloc((void **)&c.sbuf, bytes);
        if (st != DDA_OK) return st;
        c.sbuf_bytes = bytes;
    }
    char *p = (char *)c.sbuf;
    auto take = [&](size_t n) {
        char *q = p;
        p += (n + 255) / 256 * 256;
        return q;
    };
    B.st = (SolveState *)take(nrhs * sizeof(SolveState));
    B.done = (int *)take(nrhs * sizeof(int) * 2);
    B.part = (double2 *)take((size_t)nrhs * B.nb * 4 * sizeof(double2));
    B.hist = hcap > 0 ? (double *)take((size_t)nrhs * hcap * sizeof(double)) : nullptr;
    B.scratch = (double2 *)take((4 * (size_t)nrhs + 16) * sizeof(double2));
    const size_t hb = 64 + nrhs * (sizeof(SolveState) + 2 * sizeof(int) + 4 * sizeof(double2));
    if (c.hbuf_bytes < hb) {
        if (c.hbuf) (void)hipHostFree(c.hbuf);
        c.hbuf = nullptr;
        c.hbuf_bytes = 0;
        DDA_HIP_CHECK(hipHostMalloc((void **)&c.hbuf, hb, hipHostMallocDefault));
        c.hbuf_bytes = hb;
    }
    return DDA_OK;
}

// Initial states (tolerance, iteration limit) for every right-hand side.
static dda_status init_states(Ctx &c, Bufs &B, double tol, int maxit, const int *active = nullptr,
                              const double *tols = nullptr) {
    std::vector<SolveState> h(B.nrhs);
    for (int r = 0; r < B.nrhs; ++r) {
        SolveState &s = h[r];
        std::memset(&s, 0, sizeof s);
        s.tol = tols ? tols[r] : tol;
        s.maxit = maxit;
    }
    DDA_HIP_CHECK(hipMemcpyAsync(B.st, h.data(), h.size() * sizeof(SolveState), hipMemcpyHostToDevice, c.stream));
    std::vector<int> d(B.nrhs, 0);
    if (active)
        for (int r = 0; r < B.nrhs; ++r) d[r] = active[r] ? 0 : 1;
    DDA_HIP_CHECK(hipMemcpyAsync(B.done, d.data(), B.nrhs * sizeof(int), hipMemcpyHostToDevice, c.stream));
    DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
    return DDA_OK;
}

// One Krylov solve in flight on a context: its buffers, the chunk of `check_every` iterations it
// launches between convergence checks, and (optionally) that chunk captured once as a hipGraph
// and replayed.  A right-hand side that is done turns every later kernel into a no-op, so
// launching whole chunks past convergence never changes its iterate.
// FNV-1a over the beams of a batch (propagation, polarization, waist, focus): with LDR or CLDR the
// polarizability, and with it the matrix, depends on them, and the right-hand side always does
static uint64_t beams_hash(const dda_beam *beams, int nrhs) {
    uint64_t h = 1469598103934665603ull;
    const unsigned char *b = reinterpret_cast<const unsigned char *>(beams);
    for (size_t i = 0; i < (size_t)nrhs * sizeof(dda_beam); ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}

template <typename R> struct Run {
    Ctx *c = nullptr;
    Bufs B;
    Vecs<R> v{};
    cplx<R> *x = nullptr;
    int solver = DDA_QMR;
    int check_every = 1;
    bool graph = false;
    int chunks = 0;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipEvent_t ev = nullptr;
    bool fin = false;
    bool pending = false;
    bool mixed = false;  // double-precision Krylov vectors, single-precision transforms (R = double)
    double relax_at = 0;  // > 0: double-precision products until every residual is below it, then mixed
    int switch_it = 0;    // iteration of the switch to single-precision products (0: from the start)
    bool snapped = false; // the double-precision state at the switch is saved (c.snap)
    bool rolled = false;  // the single-precision phase stalled and the saved state was restored
    uint64_t beams_h = 0;  // beams_hash of the batch
    double progress = 0;  // seconds between progress lines on stderr (0: none)
    std::chrono::steady_clock::time_point last_report{};
    // stall guard of a mixed run: best relative residual of each right-hand side and the iteration
    // that reached it; a stalled right-hand side is stopped (stalled[r])
    std::vector<double> best;
    std::vector<int> best_it;
    std::vector<char> stalled;
    std::chrono::steady_clock::time_point last_guard{};
};

// A mixed run (single-precision transforms) stalls where the transforms' rounding limits the
// accuracy the Krylov process can reach.  A stalled right-hand side is stopped there and left to
// the double-precision solver, restarted from its iterate (continuing the same recurrence with
// double-precision products converged far more slowly than the restart).  Stall: no halving of
// the residual within as many iterations as the best residual took, and at least kStallMin.
constexpr int kStallMin = 5000;
constexpr double kGuardSeconds = 0.5;  // host-side stall checks at most this often
constexpr double kRelaxSeconds = 0.05;  // host-side checks of the switch to single-precision products
// A relaxed run whose single-precision phase does not halve a residual within this many iterations
// (or a tenth of the iterations before the switch, if more) goes back to the saved state.
constexpr int kRelaxStallMin = 500;

// Save (save = true) or restore the state a solve carries between iterations: the Krylov vectors,
// the iterate, the per-RHS scalar states and done flags.
static dda_status snapshot(Ctx &c, Bufs &B, double2 *vecs, double2 *x, bool save) {
    const size_t L = (size_t)B.nrhs * B.n3;
    const size_t vb = (size_t)7 * L * sizeof(double2), xb = L * sizeof(double2);  // the 7 slots of vecs_of
    const size_t sb = (size_t)B.nrhs * sizeof(SolveState), db = (size_t)B.nrhs * sizeof(int);
    const size_t need = vb + xb + sb + db + 256;
    if (save && c.snap_bytes < need) {
        DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
        (void)hipFree(c.snap);
        c.snap = nullptr;
        c.snap_bytes = 0;
        dda_status st = device_alloc(&c.snap, need);
        if (st != DDA_OK) return st;
        c.snap_bytes = need;
    }
    char *p = static_cast<char *>(c.snap);
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    if (save) {
        DDA_HIP_CHECK(hipMemcpyAsync(p, vecs, vb, k, c.stream));
        DDA_HIP_CHECK(hipMemcpyAsync(p + vb, x, xb, k, c.stream));
        DDA_HIP_CHECK(hipMemcpyAsync(p + vb + xb, B.st, sb, k, c.stream));
        DDA_HIP_CHECK(hipMemcpyAsync(p + vb + xb + sb, B.done, db, k, c.stream));
    } else {
        DDA_HIP_CHECK(hipMemcpyAsync(vecs, p, vb, k, c.stream));
        DDA_HIP_CHECK(hipMemcpyAsync(x, p + vb, xb, k, c.stream));
        DDA_HIP_CHECK(hipMemcpyAsync(B.st, p + vb + xb, sb, k, c.stream));
        DDA_HIP_CHECK(hipMemcpyAsync(B.done, p + vb + xb + sb, db, k, c.stream));
    }
    DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
    return DDA_OK;
}

template <typename R> static void drop_graph(Run<R> &k) {
    if (k.ge) (void)hipGraphExecDestroy(k.ge);
    if (k.g) (void)hipGraphDestroy(k.g);
    k.ge = nullptr;
    k.g = nullptr;
    k.chunks = 0;
}

// Progress lines for long solves: the environment variable DDA_PROGRESS gives the seconds between
// lines (unset or 0: silent).
static double progress_interval() {
    const char *e = std::getenv("DDA_PROGRESS");
    return e ? std::atof(e) : 0.0;
}

// the product a run applies: plain precision R, or double vectors through single-precision
// transforms
template <typename R>
static dda_status run_matvec(Run<R> &k, const cplx<R> *x, cplx<R> *y, cplx<R> *dots, const int *done) {
    Ctx &c = *k.c;
    Work<R> &w = work_of<R>(c);
    if constexpr (std::is_same<R, double>::value)
        if (k.mixed) return matvec_device_mixed(c, x, y, k.B.nrhs, w.scale, dots, c.stream, done);
    return matvec_device<R>(c, x, y, k.B.nrhs, w.scale, dots, c.stream, done);
}

// enqueue `count` solver iterations on the context's stream
template <typename R> static dda_status enqueue_iterations(Run<R> &k, int count) {
    Ctx &c = *k.c;
    Bufs &B = k.B;
    Vecs<R> &v = k.v;
    hipStream_t s = c.stream;
    const dim3 vg(B.nb, B.nrhs), vb(kVecThreads);
    const int nrhs = B.nrhs;
    const size_t n3 = B.n3;
    Work<R> &w = work_of<R>(c);
    const int ndots = (int)(k.mixed ? dots_per_rhs<float>(c) : dots_per_rhs<R>(c));
    cplx<R> *x = k.x;
    dda_status st;
    for (int it = 0; it < count; ++it) {
        if (k.solver == DDA_CGNR) {
            if ((st = run_matvec(k, v.p, v.pt, nullptr, B.done)) != DDA_OK) return st;  // w = A p
            hipLaunchKernelGGL(k_cgnr_norm<R>, vg, vb, 0, s, B.done, v.pt, n3, B.part);
            hipLaunchKernelGGL(k_cgnr_scal, dim3(nrhs), vb, 0, s, B.st, B.done, B.part, B.nb, 1);
            hipLaunchKernelGGL(k_cgnr_update<R>, vg, vb, 0, s, B.st, B.done, v.p, v.pt, x, v.r, v.vt, n3, B.part);
            hipLaunchKernelGGL(k_cgnr_scal_res, dim3(nrhs), vb, 0, s, B.st, B.done, B.part, B.nb, B.hist, B.hcap);
            if ((st = run_matvec(k, v.vt, v.d, nullptr, B.done)) != DDA_OK) return st;  // d = A conj(r)
            hipLaunchKernelGGL(k_cgnr_norm<R>, vg, vb, 0, s, B.done, v.d, n3, B.part);
            hipLaunchKernelGGL(k_cgnr_scal, dim3(nrhs), vb, 0, s, B.st, B.done, B.part, B.nb, 2);
            hipLaunchKernelGGL(k_cgnr_p<R>, vg, vb, 0, s, B.st, B.done, v.d, v.p, n3, 0);
            hipLaunchKernelGGL(k_stop_after, dim3((nrhs + 63) / 64), dim3(64), 0, s, B.st, B.done, nrhs);
        } else if (k.solver == DDA_BICG) {
            if ((st = run_matvec(k, v.p, v.pt, w.dots, B.done)) != DDA_OK) return st;
            hipLaunchKernelGGL(k_bicg_scal_alpha<R>, dim3(nrhs), vb, 0, s, B.st, B.done, w.dots, ndots);
            hipLaunchKernelGGL(k_bicg_update<R>, vg, vb, 0, s, B.st, B.done, v.p, v.pt, x, v.r, n3, B.part);
            hipLaunchKernelGGL(k_bicg_scal_2, dim3(nrhs), vb, 0, s, B.st, B.done, B.part, B.nb, B.hist, B.hcap);
            hipLaunchKernelGGL(k_bicg_p<R>, vg, vb, 0, s, B.st, B.done, v.r, v.p, n3);
            hipLaunchKernelGGL(k_stop_after, dim3((nrhs + 63) / 64), dim3(64), 0, s, B.st, B.done, nrhs);
        } else if (k.solver == DDA_QMR) {
            if ((st = run_matvec(k, v.p, v.pt, w.dots, B.done)) != DDA_OK) return st;
            hipLaunchKernelGGL(k_qmr_scal_eps<R>, dim3(nrhs), vb, 0, s, B.st, B.done, w.dots, ndots);
            hipLaunchKernelGGL(k_qmr_vt<R>, vg, vb, 0, s, B.st, B.done, v.pt, v.vt, n3, B.part);
            hipLaunchKernelGGL(k_qmr_scal_2, dim3(nrhs), vb, 0, s, B.st, B.done, B.part, B.nb);
            hipLaunchKernelGGL(k_qmr_update<R>, vg, vb, 0, s, B.st, B.done, v.p, v.pt, v.vt, v.d, v.s, x, v.r, n3,
                               B.part);
            hipLaunchKernelGGL(k_qmr_scal_3, dim3(nrhs), vb, 0, s, B.st, B.done, B.part, B.nb, B.hist, B.hcap);
        } else {
            hipLaunchKernelGGL(k_bi_p<R>, vg, vb, 0, s, B.st, B.done, v.r, v.p, v.v, n3);
            if ((st = run_matvec(k, v.p, v.v, nullptr, B.done)) != DDA_OK) return st;
            hipLaunchKernelGGL(k_bi_dots<R>, vg, vb, 0, s, B.done, v.rs, v.v, n3, B.part, 0);
            hipLaunchKernelGGL(k_bi_scal_alpha, dim3(nrhs), vb, 0, s, B.st, B.done, B.part, B.nb);
            hipLaunchKernelGGL(k_bi_s<R>, vg, vb, 0, s, B.st, B.done, v.r, v.v, v.s, n3, B.part);
            hipLaunchKernelGGL(k_bi_scal_s, dim3(nrhs), vb, 0, s, B.st, B.done, B.part, B.nb);
            if ((st = run_matvec(k, v.s, v.t, nullptr, B.done)) != DDA_OK) return st;
            hipLaunchKernelGGL(k_bi_dots<R>, vg, vb, 0, s, B.done, v.t, v.s, n3, B.part, 1);
            hipLaunchKernelGGL(k_bi_scal_omega, dim3(nrhs), vb, 0, s, B.st, B.done, B.part, B.nb);
            hipLaunchKernelGGL(k_bi_x<R>, vg, vb, 0, s, B.st, B.done, v.p, v.s, v.t, v.rs, x, v.r, n3, B.part);
            hipLaunchKernelGGL(k_bi_scal_end, dim3(nrhs), vb, 0, s, B.st, B.done, B.part, B.nb, B.hist, B.hcap);
        }
    }
    DDA_HIP_CHECK(hipGetLastError());
    return DDA_OK;
}

// copy the done flags to the pinned host mirror and mark the point to wait for
template <typename R> static dda_status post_check(Run<R> &k) {
    Ctx &c = *k.c;
    DDA_HIP_CHECK(hipMemcpyAsync(c.hbuf, k.B.done, k.B.nrhs * sizeof(int), hipMemcpyDeviceToHost, c.stream));
    DDA_HIP_CHECK(hipEventRecord(k.ev, c.stream));
    k.pending = true;
    return DDA_OK;
}

// initial residual and scalars (x holds the initial guess if have_x0, else it is zeroed)
template <typename R> static dda_status run_begin(Run<R> &k, bool have_x0) {
    Ctx &c = *k.c;
    Bufs &B = k.B;
    Vecs<R> &v = k.v;
    hipStream_t s = c.stream;
    const dim3 vg(B.nb, B.nrhs), vb(kVecThreads);
    const size_t n3 = B.n3;
    Work<R> &w = work_of<R>(c);
    dda_status st;
    DDA_HIP_CHECK(hipEventCreateWithFlags(&k.ev, hipEventDisableTiming));
    k.progress = progress_interval();
    k.last_report = std::chrono::steady_clock::now();
    k.last_guard = k.last_report;
    k.best.assign(B.nrhs, HUGE_VAL);
    k.best_it.assign(B.nrhs, 0);
    k.stalled.assign(B.nrhs, 0);
    if (have_x0) {
        if ((st = run_matvec(k, k.x, v.pt, nullptr, nullptr)) != DDA_OK) return st;
    }
    if (k.solver == DDA_CGNR) {  // r, t = conj(r); d = A t; p = conj(d) = A^H r; g = ||p||^2
        hipLaunchKernelGGL(k_cgnr_init<R>, vg, vb, 0, s, v.b, have_x0 ? v.pt : nullptr, k.x, v.r, v.vt, n3, B.part,
                           have_x0 ? 0 : 1);
        hipLaunchKernelGGL(k_cgnr_scal_init, dim3(B.nrhs), vb, 0, s, B.st, B.done, B.part, B.nb, B.hist, B.hcap);
        if ((st = run_matvec(k, v.vt, v.d, nullptr, B.done)) != DDA_OK) return st;
        hipLaunchKernelGGL(k_cgnr_norm<R>, vg, vb, 0, s, B.done, v.d, n3, B.part);
        hipLaunchKernelGGL(k_cgnr_scal, dim3(B.nrhs), vb, 0, s, B.st, B.done, B.part, B.nb, 0);
        hipLaunchKernelGGL(k_cgnr_p<R>, vg, vb, 0, s, B.st, B.done, v.d, v.p, n3, 1);
    } else if (k.solver == DDA_BICG) {
        hipLaunchKernelGGL(k_qmr_init<R>, vg, vb, 0, s, v.b, have_x0 ? v.pt : nullptr, k.x, v.r, v.p, n3, B.part,
                           have_x0 ? 0 : 1);
        hipLaunchKernelGGL(k_bicg_scal_init, dim3(B.nrhs), vb, 0, s, B.st, B.done, B.part, B.nb, B.hist, B.hcap);
    } else if (k.solver == DDA_QMR) {
        hipLaunchKernelGGL(k_qmr_init<R>, vg, vb, 0, s, v.b, have_x0 ? v.pt : nullptr, k.x, v.r, v.vt, n3, B.part,
                           have_x0 ? 0 : 1);
        hipLaunchKernelGGL(k_qmr_scal_init, dim3(B.nrhs), vb, 0, s, B.st, B.done, B.part, B.nb, B.hist, B.hcap);
        hipLaunchKernelGGL(k_qmr_p0<R>, vg, vb, 0, s, B.st, B.done, v.vt, v.p, n3);
    } else {
        hipLaunchKernelGGL(k_bi_init<R>, vg, vb, 0, s, v.b, have_x0 ? v.pt : nullptr, k.x, v.r, v.rs, n3, B.part,
                           have_x0 ? 0 : 1);
        hipLaunchKernelGGL(k_bi_scal_init, dim3(B.nrhs), vb, 0, s, B.st, B.done, B.part, B.nb, B.hist, B.hcap);
    }
    DDA_HIP_CHECK(hipGetLastError());
    return post_check(k);
}

// continue a run whose vectors and states are already in place (no initialization kernels)
template <typename R> static dda_status run_resume(Run<R> &k) {
    DDA_HIP_CHECK(hipEventCreateWithFlags(&k.ev, hipEventDisableTiming));
    k.progress = progress_interval();
    k.last_report = std::chrono::steady_clock::now();
    k.last_guard = k.last_report;
    k.best.assign(k.B.nrhs, HUGE_VAL);
    k.best_it.assign(k.B.nrhs, 0);
    k.stalled.assign(k.B.nrhs, 0);
    return post_check(k);
}

// launch one chunk of iterations: eagerly the first time, then as a replayed graph if enabled
template <typename R> static dda_status run_issue(Run<R> &k) {
    Ctx &c = *k.c;
    dda_status st;
    if (k.graph && k.chunks > 0) {
        if (!k.ge) {
            DDA_HIP_CHECK(hipStreamBeginCapture(c.stream, hipStreamCaptureModeRelaxed));
            st = enqueue_iterations(k, k.check_every);
            hipError_t e = hipStreamEndCapture(c.stream, &k.g);
            if (st != DDA_OK) return st;
            if (e != hipSuccess) {
                set_error(std::string("solver graph capture: ") + hipGetErrorString(e));
                return DDA_EHIP;
            }
            DDA_HIP_CHECK(hipGraphInstantiate(&k.ge, k.g, nullptr, nullptr, 0));
        }
        DDA_HIP_CHECK(hipGraphLaunch(k.ge, c.stream));
    } else if ((st = enqueue_iterations(k, k.check_every)) != DDA_OK) {
        return st;
    }
    ++k.chunks;
    return post_check(k);
}

static dda_status fetch_states(Ctx &c, Bufs &B, std::vector<SolveState> &h);

template <typename R> static dda_status run_poll(Run<R> &k) {
    if (!k.pending) return DDA_OK;
    DDA_HIP_CHECK(hipEventSynchronize(k.ev));
    k.pending = false;
    const int *hd = (const int *)k.c->hbuf;
    bool all = true;
    for (int r = 0; r < k.B.nrhs; ++r) all = all && hd[r];
    k.fin = all;
    if (k.relax_at > 0 && !k.mixed && !k.fin) {
        const auto now = std::chrono::steady_clock::now();
        if (std::chrono::duration<double>(now - k.last_guard).count() >= kRelaxSeconds) {
            k.last_guard = now;
            std::vector<int> d(hd, hd + k.B.nrhs);
            std::vector<SolveState> h;
            dda_status st = fetch_states(*k.c, k.B, h);  // the stream is idle here
            if (st != DDA_OK) return st;
            double worst = 0;
            for (int r = 0; r < k.B.nrhs; ++r)
                if (!d[r]) worst = std::max(worst, h[r].res);
            if (worst < k.relax_at) {
                // every active right-hand side is below the threshold: the later iterations run the
                // single-precision transforms (a captured chunk is captured again with them); the
                // double-precision state is saved first, to go back to if that phase stalls
                if constexpr (std::is_same<R, double>::value) {
                    if ((st = snapshot(*k.c, k.B, k.c->vecs, k.x, true)) != DDA_OK) return st;
                    k.snapped = true;
                }
                k.mixed = true;
                drop_graph(k);
                int it = 0;
                for (int r = 0; r < k.B.nrhs; ++r) {
                    k.best[r] = h[r].res;
                    k.best_it[r] = h[r].iter;
                    it = std::max(it, h[r].iter);
                }
                k.switch_it = it;
                k.last_guard = now;
            }
        }
    }
    if (k.mixed && !k.fin) {
        const auto now = std::chrono::steady_clock::now();
        if (std::chrono::duration<double>(now - k.last_guard).count() >= kGuardSeconds) {
            k.last_guard = now;
            std::vector<int> d(hd, hd + k.B.nrhs);
            std::vector<SolveState> h;
            dda_status st = fetch_states(*k.c, k.B, h);  // the stream is idle here
            if (st != DDA_OK) return st;
            bool all = true;
            if (k.snapped) {
                // relaxed run: a right-hand side that has not halved its residual within the window
                // sends the whole batch back to the saved double-precision state, for good
                const int window = std::max(kRelaxStallMin, k.switch_it / 10);
                bool stall = false;
                for (int r = 0; r < k.B.nrhs; ++r) {
                    if (d[r]) continue;
                    if (h[r].res < 0.5 * k.best[r]) {
                        k.best[r] = h[r].res;
                        k.best_it[r] = h[r].iter;
                    } else if (h[r].iter - k.best_it[r] > window) {
                        stall = true;
                    }
                }
                if (stall) {
                    if constexpr (std::is_same<R, double>::value)
                        if ((st = snapshot(*k.c, k.B, k.c->vecs, k.x, false)) != DDA_OK) return st;
                    k.mixed = false;
                    k.relax_at = 0;
                    k.snapped = false;
                    k.rolled = true;
                    drop_graph(k);
                    k.fin = false;
                }
            } else {
                for (int r = 0; r < k.B.nrhs; ++r) {
                    if (d[r]) continue;
                    if (h[r].res < 0.5 * k.best[r]) {
                        k.best[r] = h[r].res;
                        k.best_it[r] = h[r].iter;
                    } else if (h[r].iter - k.best_it[r] > std::max(kStallMin, k.best_it[r] - k.switch_it)) {
                        // stop it: its done flag makes every later iteration skip it
                        static const int one = 1;
                        DDA_HIP_CHECK(hipMemcpyAsync(k.B.done + r, &one, sizeof(int), hipMemcpyHostToDevice,
                                                     k.c->stream));
                        DDA_HIP_CHECK(hipStreamSynchronize(k.c->stream));
                        k.stalled[r] = 1;
                        continue;
                    }
                    all = false;
                }
                k.fin = all;
            }
        }
    }
    if (k.progress > 0 && !k.fin) {
        const auto now = std::chrono::steady_clock::now();
        if (std::chrono::duration<double>(now - k.last_report).count() >= k.progress) {
            k.last_report = now;
            std::vector<int> d(hd, hd + k.B.nrhs);
            std::vector<SolveState> h;
            dda_status st = fetch_states(*k.c, k.B, h);  // the stream is idle here
            if (st != DDA_OK) return st;
            for (int r = 0; r < k.B.nrhs; ++r)
                if (!d[r])
                    std::fprintf(stderr, "dda_solve: right-hand side %d: iteration %d, relative residual %.3e\n", r,
                                 h[r].iter, h[r].res);
            std::fflush(stderr);
        }
    }
    return DDA_OK;
}

template <typename R> static void run_end(Run<R> &k) {
    if (k.ge) (void)hipGraphExecDestroy(k.ge);
    if (k.g) (void)hipGraphDestroy(k.g);
    if (k.ev) (void)hipEventDestroy(k.ev);
    k.ge = nullptr;
    k.g = nullptr;
    k.ev = nullptr;
}

// One Krylov solve to completion (x holds the initial guess if have_x0, else it is zeroed; b must
// already be in v.b; on return the states are on the device).
template <typename R>
static dda_status krylov(Ctx &c, Bufs &B, Vecs<R> &v, cplx<R> *x, bool have_x0, int solver, int check_every,
                         bool graph = false) {
    Run<R> k;
    k.c = &c;
    k.B = B;
    k.v = v;
    k.x = x;
    k.solver = solver;
    k.check_every = check_every;
    k.graph = graph;
    dda_status st = run_begin(k, have_x0);
    if (st == DDA_OK) st = run_poll(k);
    while (st == DDA_OK && !k.fin) {
        if ((st = run_issue(k)) != DDA_OK) break;
        st = run_poll(k);
    }
    run_end(k);
    return st;
}

static dda_status fetch_states(Ctx &c, Bufs &B, std::vector<SolveState> &h) {
    h.resize(B.nrhs);
    DDA_HIP_CHECK(hipMemcpyAsync(h.data(), B.st, B.nrhs * sizeof(SolveState), hipMemcpyDeviceToHost, c.stream));
    DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
    return DDA_OK;
}

// |b - A x| / |b| per right-hand side (fp64), using v.pt as scratch
static dda_status true_residual(Ctx &c, Bufs &B, Vecs<double> &v, const double2 *x, double2 *res_r,
                                std::vector<double> &out) {
    dda_status st;
    if ((st = matvec_device<double>(c, x, v.pt, B.nrhs, c.w64.scale, nullptr, c.stream, nullptr)) != DDA_OK)
        return st;
    hipLaunchKernelGGL(k_resid, dim3(B.nb, B.nrhs), dim3(kVecThreads), 0, c.stream, v.b, v.pt, res_r, B.n3, B.part);
    double2 *sums = (double2 *)((char *)c.hbuf + 64);
    double2 *dsum = B.scratch;
    hipLaunchKernelGGL(k_sum_part, dim3(B.nrhs), dim3(kVecThreads), 0, c.stream, B.part, B.nb, dsum);
    DDA_HIP_CHECK(hipMemcpyAsync(sums, dsum, B.nrhs * sizeof(double2), hipMemcpyDeviceToHost, c.stream));
    DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
    out.resize(B.nrhs);
    for (int r = 0; r < B.nrhs; ++r) out[r] = sums[r].y > 0 ? std::sqrt(sums[r].x / sums[r].y) : 0.0;
    return DDA_OK;
}

// Initial-guess check: a right-hand side whose guess does not lower the residual below |b|
// starts from zero instead (b must be in v.b).
static dda_status check_x0(Ctx &c, Bufs &B, Vecs<double> &v, double2 *x, int nrhs) {
    std::vector<double> r0;
    dda_status st = true_residual(c, B, v, x, nullptr, r0);
    if (st != DDA_OK) return st;
    for (int r = 0; r < nrhs; ++r)
        if (!(r0[r] < 1.0)) hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, c.stream, x + (size_t)r * B.n3, B.n3);
    DDA_HIP_CHECK(hipGetLastError());
    return DDA_OK;
}

static dda_status status_of(int s) {
    return s == ST_CONV ? DDA_OK : s == ST_MAXIT ? DDA_ENOTCONV : s == ST_BREAK ? DDA_EBREAKDOWN : DDA_ENOTCONV;
}

// FP64 solve (QMR or Bi-CGSTAB) of all right-hand sides.
static int hist_cap(const dda_solve_info *info, int nrhs) {
    int m = 0;
    if (info)
        for (int r = 0; r < nrhs; ++r) m = std::max(m, info[r].res_hist_cap);
    return m;
}

// fp64 solve, first half: buffers, scales, right-hand sides, initial guess, states, begin
static dda_status prepare_fp64(Ctx &c, Run<double> &k, const dda_beam *beams, int nrhs, double tol,
                               const dda_solve_opts &o, double2 *x, int hcap) {
    dda_status st;
    if ((st = ensure_vecs<double>(c, nrhs)) != DDA_OK) return st;
    if ((st = ensure_bufs(c, k.B, nrhs, hcap)) != DDA_OK) return st;
    std::vector<double> ar(nrhs), ai(nrhs);
    for (int r = 0; r < nrhs; ++r) polarizability(c, beams[r], ar[r], ai[r]);
    if ((st = upload_scales<double>(c, ar, ai)) != DDA_OK) return st;
    if ((st = material_prepare(c, beams, nrhs)) != DDA_OK) return st;
    k.c = &c;
    k.v = vecs_of<double>(c, nrhs);
    k.x = x;
    k.solver = o.solver;
    k.mixed = o.precision == DDA_FP32_PRODUCT;
    k.relax_at = o.precision == DDA_FP32_RELAXED ? (o.relax_at > 0 ? o.relax_at : 100.0 * tol) : 0.0;
    k.switch_it = 0;
    k.beams_h = beams_hash(beams, nrhs);
    if (k.relax_at > 0 && (st = ensure_work<float>(c, nrhs)) != DDA_OK) return st;  // before any capture
    for (int r = 0; r < nrhs; ++r)
        if ((st = rhs_launch<double>(c, beams[r], k.v.b + (size_t)r * k.B.n3, c.stream)) != DDA_OK) return st;
    if (o.x0 && o.x0 != x)
        DDA_HIP_CHECK(hipMemcpyAsync(x, o.x0, (size_t)nrhs * k.B.n3 * sizeof(double2), hipMemcpyDeviceToDevice,
                                     c.stream));
    if (o.x0 && o.x0_check && (st = check_x0(c, k.B, k.v, x, nrhs)) != DDA_OK) return st;
    if ((st = init_states(c, k.B, tol, o.maxit)) != DDA_OK) return st;
    return run_begin(k, o.x0 != nullptr);
}

// fp64 solve, second half: states, true residual, report
static dda_status finish_fp64(Ctx &c, Run<double> &k, int nrhs, const dda_solve_opts &o, dda_solve_info *info,
                              int hcap) {
    dda_status st;
    std::vector<SolveState> h;
    if ((st = fetch_states(c, k.B, h)) != DDA_OK) return st;
    std::vector<double> rt;
    // A x goes to a slot the iteration recomputes before reading it, so that a solve stopped at
    // its limit keeps its state (Bi-CGSTAB carries v = A p in pt into the next iteration; t is
    // recomputed)
    Vecs<double> tv = k.v;
    if (k.solver == DDA_BICGSTAB) tv.pt = k.v.t;
    if ((st = true_residual(c, k.B, tv, k.x, nullptr, rt)) != DDA_OK) return st;
    std::vector<double> hist;
    if (hcap > 0) {
        hist.resize((size_t)nrhs * hcap);
        DDA_HIP_CHECK(hipMemcpyAsync(hist.data(), k.B.hist, hist.size() * sizeof(double), hipMemcpyDeviceToHost,
                                     c.stream));
        DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
    }
    dda_status ret = DDA_OK;
    c.resume_nrhs = 0;  // continuable: a double-precision run with a right-hand side at its limit
    for (int r = 0; r < nrhs; ++r)
        if (!k.mixed && h[r].status == ST_MAXIT) {
            c.resume_nrhs = nrhs;
            c.resume_solver = o.solver;
            c.resume_beams = k.beams_h;
        }
    for (int r = 0; r < nrhs; ++r) {
        const dda_status sr = status_of(h[r].status);
        if (ret == DDA_OK && sr != DDA_OK) ret = sr;
        if (!info) continue;
        info[r].status = sr;
        info[r].iters = h[r].iter;
        const int per_run = o.solver == DDA_BICGSTAB ? 2 * h[r].iter - (h[r].half ? 1 : 0)
                            : o.solver == DDA_CGNR   ? 2 * h[r].iter + (h[r].status == ST_MAXIT ? 1 : 0)  // a limit stop ends with A^H r
                                                     : h[r].iter;
        info[r].matvecs = per_run + (o.x0 ? 1 + (o.x0_check ? 1 : 0) : 0);
        info[r].outer = (k.stalled.size() > (size_t)r && k.stalled[r]) || k.rolled ? 1 : 0;
        info[r].res_rec = h[r].res;
        info[r].res_true = rt[r];
        if (hcap > 0 && info[r].res_hist && info[r].res_hist_cap > 0) {
            const int n = std::min(info[r].res_hist_cap, h[r].iter + 1);
            for (int q = 0; q < n; ++q) info[r].res_hist[q] = hist[(size_t)r * hcap + q];
            info[r].res_hist_len = n;
        } else {
            info[r].res_hist_len = 0;
        }
    }
    return ret;
}

// continue the context's stopped solve (opts.resume): right-hand sides that hit the iteration
// limit get opts.maxit more iterations and the new tol; the others stay as they ended
static dda_status prepare_resume(Ctx &c, Run<double> &k, const dda_beam *beams, int nrhs, double tol,
                                 const dda_solve_opts &o, double2 *x) {
    if (c.resume_nrhs != nrhs || c.resume_solver != o.solver || o.precision != DDA_FP64 || o.x0) {
        set_error("dda_solve: nothing to resume for this batch size, method and precision (double precision, "
                  "no initial guess)");
        return DDA_EINVAL;
    }
    if (c.resume_beams != beams_hash(beams, nrhs)) {
        set_error("dda_solve: resume needs the beams of the stopped solve (they define its right-hand sides and, "
                  "for LDR and CLDR, its matrix)");
        return DDA_EINVAL;
    }
    dda_status st;
    if ((st = ensure_vecs<double>(c, nrhs)) != DDA_OK) return st;
    if ((st = ensure_bufs(c, k.B, nrhs, 0)) != DDA_OK) return st;  // the states stay where they are
    std::vector<double> ar(nrhs), ai(nrhs);
    for (int r = 0; r < nrhs; ++r) polarizability(c, beams[r], ar[r], ai[r]);
    if ((st = upload_scales<double>(c, ar, ai)) != DDA_OK) return st;
    if ((st = material_prepare(c, beams, nrhs)) != DDA_OK) return st;
    k.c = &c;
    k.v = vecs_of<double>(c, nrhs);
    k.x = x;
    k.solver = o.solver;
    k.mixed = false;
    k.beams_h = c.resume_beams;
    std::vector<SolveState> h;
    if ((st = fetch_states(c, k.B, h)) != DDA_OK) return st;
    std::vector<int> d(nrhs);
    for (int r = 0; r < nrhs; ++r) {
        d[r] = 1;
        if (h[r].status == ST_MAXIT) {
            h[r].status = ST_RUN;
            h[r].maxit = h[r].iter + o.maxit;
            h[r].tol = tol;
            d[r] = 0;
        }
    }
    DDA_HIP_CHECK(hipMemcpyAsync(k.B.st, h.data(), nrhs * sizeof(SolveState), hipMemcpyHostToDevice, c.stream));
    DDA_HIP_CHECK(hipMemcpyAsync(k.B.done, d.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, c.stream));
    DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
    return run_resume(k);
}

static dda_status solve_fp64(Ctx &c, const dda_beam *beams, int nrhs, double tol, const dda_solve_opts &o,
                             double2 *x, dda_solve_info *info, int check_every, bool graph) {
    const int hcap = o.resume ? 0 : hist_cap(info, nrhs);  // a continued solve keeps no history
    Run<double> k;
    k.check_every = check_every;
    k.graph = graph;
    dda_status st = o.resume ? prepare_resume(c, k, beams, nrhs, tol, o, x)
                             : prepare_fp64(c, k, beams, nrhs, tol, o, x, hcap);
    if (st == DDA_OK) st = run_poll(k);
    while (st == DDA_OK && !k.fin) {
        if ((st = run_issue(k)) != DDA_OK) break;
        st = run_poll(k);
    }
    run_end(k);
    if (st != DDA_OK) return st;
    return finish_fp64(c, k, nrhs, o, info, hcap);
}

// Double-precision Krylov iteration whose products run their transforms and tensor multiply in
// single precision, to max(tol, 1e-6) (below that the single-precision products' rounding makes
// the residual stagnate); a right-hand side whose true (double-precision) residual then misses
// tol is finished by the double-precision solver, started from that iterate when it lowers the
// residual below |b| and from zero otherwise.
static dda_status solve_products32(Ctx &c, const dda_beam *beams, int nrhs, double tol, const dda_solve_opts &o,
                                   double2 *x, dda_solve_info *info, int check_every, bool graph) {
    if (!c.ghat32) {
        set_error("dda_solve: DDA_FP32_PRODUCT and DDA_FP32_RELAXED need a context set up with opts.fp32");
        return DDA_ENOTSUP;
    }
    std::vector<dda_solve_info> first(nrhs);
    for (int r = 0; r < nrhs; ++r) {
        first[r] = dda_solve_info{};
        if (info) {
            first[r].res_hist = info[r].res_hist;
            first[r].res_hist_cap = info[r].res_hist_cap;
        }
    }
    const double kProductFloor = 1e-6;
    dda_status st = solve_fp64(c, beams, nrhs, std::max(tol, kProductFloor), o, x, first.data(), check_every, graph);
    if (st != DDA_OK && st != DDA_ENOTCONV && st != DDA_EBREAKDOWN) return st;
    bool again = false;
    for (int r = 0; r < nrhs; ++r) again = again || !(first[r].res_true < tol);
    std::vector<dda_solve_info> second(nrhs);
    if (again) {
        dda_solve_opts o2 = o;
        o2.precision = DDA_FP64;
        o2.x0 = x;
        o2.x0_check = 1;
        for (auto &i : second) i = dda_solve_info{};
        st = solve_fp64(c, beams, nrhs, tol, o2, x, second.data(), check_every, graph);
        if (st != DDA_OK && st != DDA_ENOTCONV && st != DDA_EBREAKDOWN) return st;
    }
    dda_status ret = DDA_OK;
    for (int r = 0; r < nrhs; ++r) {
        const dda_solve_info &f = again ? second[r] : first[r];
        if (ret == DDA_OK && f.status != DDA_OK) ret = (dda_status)f.status;
        if (!info) continue;
        info[r].status = f.status;
        info[r].iters = first[r].iters + (again ? second[r].iters : 0);
        info[r].matvecs = first[r].matvecs + (again ? second[r].matvecs : 0);
        info[r].outer = again || first[r].outer ? 1 : 0;
        info[r].res_rec = f.res_rec;
        info[r].res_true = f.res_true;
        info[r].res_hist_len = first[r].res_hist_len;
    }
    return ret;
}

// Iterative refinement: outer fp64 residual and update, inner fp32 QMR to inner_tol.
static dda_status solve_refine(Ctx &c, const dda_beam *beams, int nrhs, double tol, const dda_solve_opts &o,
                               double2 *x, dda_solve_info *info, int check_every, bool graph) {
    dda_status st;
    if (!c.ghat32) {
        const size_t n6 = (size_t)(c.Lx / 2 + 1) * (c.Ly / 2 + 1) * (c.Lz / 2 + 1) * 6;
        if ((st = device_alloc((void **)&c.ghat32, n6 * sizeof(float2))) != DDA_OK) return st;
        launch_to_f32(c.ghat, c.ghat32, n6, c.stream);
    }
    Bufs B;
    if ((st = ensure_vecs<double>(c, nrhs)) != DDA_OK) return st;
    if ((st = ensure_vecs<float>(c, nrhs)) != DDA_OK) return st;
    if ((st = ensure_bufs(c, B, nrhs, 0)) != DDA_OK) return st;
    std::vector<double> ar(nrhs), ai(nrhs);
    for (int r = 0; r < nrhs; ++r) polarizability(c, beams[r], ar[r], ai[r]);
    if ((st = upload_scales<double>(c, ar, ai)) != DDA_OK) return st;
    if ((st = upload_scales<float>(c, ar, ai)) != DDA_OK) return st;
    Vecs<double> v = vecs_of<double>(c, nrhs);
    Vecs<float> v32 = vecs_of<float>(c, nrhs);
    // spare slot 7 of the vector pools: inner fp32 solution and outer fp64 residual
    float2 *e32 = vec_base<float>(c) + (size_t)7 * nrhs * B.n3;
    double2 *r64 = vec_base<double>(c) + (size_t)7 * nrhs * B.n3;
    for (int r = 0; r < nrhs; ++r)
        if ((st = rhs_launch<double>(c, beams[r], v.b + (size_t)r * B.n3, c.stream)) != DDA_OK) return st;
    if (o.x0 && o.x0 != x)
        DDA_HIP_CHECK(hipMemcpyAsync(x, o.x0, (size_t)nrhs * B.n3 * sizeof(double2), hipMemcpyDeviceToDevice, c.stream));
    if (!o.x0) hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, c.stream, x, (size_t)nrhs * B.n3);
    if (o.x0 && o.x0_check && (st = check_x0(c, B, v, x, nrhs)) != DDA_OK) return st;
    // inner tolerance: as given, else what brings each right-hand side to the outer tolerance in
    // one inner solve (half of tol / current residual), floored where single precision stalls
    const double kInnerFloor = 1e-5;
    std::vector<double> inner_tols(nrhs, 1e-2);
    std::vector<int> iters(nrhs, 0), mvs(nrhs, 0), outer(nrhs, 0), active(nrhs, 1);
    std::vector<double> res(nrhs, 1.0), scale(nrhs, 1.0);
    std::vector<int> stat(nrhs, ST_RUN);
    double *dscale = (double *)B.scratch;           // nrhs doubles
    int *dactive = (int *)(B.scratch + nrhs);       // nrhs ints
    double2 *dsum = B.scratch + 2 * nrhs;           // nrhs sums
    const int max_outer = 30;
    for (int k = 0; k <= max_outer; ++k) {
        // outer residual in fp64
        if ((st = matvec_device<double>(c, x, v.pt, nrhs, c.w64.scale, nullptr, c.stream, nullptr)) != DDA_OK)
            return st;
        hipLaunchKernelGGL(k_resid, dim3(B.nb, nrhs), dim3(kVecThreads), 0, c.stream, v.b, v.pt, r64, B.n3, B.part);
        hipLaunchKernelGGL(k_sum_part, dim3(nrhs), dim3(kVecThreads), 0, c.stream, B.part, B.nb, dsum);
        double2 *hs = (double2 *)((char *)c.hbuf + 64);
        DDA_HIP_CHECK(hipMemcpyAsync(hs, dsum, nrhs * sizeof(double2), hipMemcpyDeviceToHost, c.stream));
        DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
        bool any = false;
        for (int r = 0; r < nrhs; ++r) {
            mvs[r] += 1;
            if (!active[r]) continue;
            const double rn = std::sqrt(hs[r].x), bn = std::sqrt(hs[r].y);
            res[r] = bn > 0 ? rn / bn : 0.0;
            if (res[r] < tol || bn == 0) {
                active[r] = 0;
                stat[r] = ST_CONV;
            } else if (k == max_outer || iters[r] >= o.maxit) {
                active[r] = 0;
                stat[r] = ST_MAXIT;
            } else {
                scale[r] = 1.0 / rn;
                outer[r] += 1;
                any = true;
                inner_tols[r] = o.inner_tol > 0 ? o.inner_tol : std::min(0.5, std::max(0.5 * tol / res[r], kInnerFloor));
            }
        }
        if (!any) break;
        DDA_HIP_CHECK(hipMemcpyAsync(dscale, scale.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c.stream));
        DDA_HIP_CHECK(hipMemcpyAsync(dactive, active.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, c.stream));
        hipLaunchKernelGGL(k_to32, dim3(B.nb, nrhs), dim3(kVecThreads), 0, c.stream, r64, v32.b, B.n3, dscale);
        // inner fp32 QMR (inactive right-hand sides start as done)
        if ((st = init_states(c, B, 0.0, std::max(1, o.maxit), active.data(), inner_tols.data())) != DDA_OK) return st;
        if ((st = krylov<float>(c, B, v32, e32, false, DDA_QMR, check_every, graph)) != DDA_OK) return st;
        std::vector<SolveState> h;
        if ((st = fetch_states(c, B, h)) != DDA_OK) return st;
        for (int r = 0; r < nrhs; ++r)
            if (active[r]) {
                iters[r] += h[r].iter;
                mvs[r] += h[r].iter;
                if (h[r].status == ST_BREAK && h[r].iter == 0) {
                    active[r] = 0;
                    stat[r] = ST_BREAK;
                }
            }
        DDA_HIP_CHECK(hipMemcpyAsync(dactive, active.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, c.stream));
        hipLaunchKernelGGL(k_addup, dim3(B.nb, nrhs), dim3(kVecThreads), 0, c.stream, x, e32, B.n3, dscale, dactive);
        DDA_HIP_CHECK(hipGetLastError());
    }
    std::vector<double> rt;
    if ((st = true_residual(c, B, v, x, nullptr, rt)) != DDA_OK) return st;
    dda_status ret = DDA_OK;
    for (int r = 0; r < nrhs; ++r) {
        const dda_status sr = status_of(stat[r]);
        if (ret == DDA_OK && sr != DDA_OK) ret = sr;
        if (!info) continue;
        info[r].status = sr;
        info[r].iters = iters[r];
        info[r].matvecs = mvs[r];
        info[r].outer = outer[r];
        info[r].res_rec = res[r];
        info[r].res_true = rt[r];
        info[r].res_hist_len = 0;
    }
    return ret;
}

}  // namespace dda

using namespace dda;

// Runs a solve on the context's own stream, ordered after the caller's stream, and restores it.
namespace dda {
struct StreamSwap {
    Ctx &c;
    hipStream_t user;
    bool ok = false;
    explicit StreamSwap(Ctx &cc) : c(cc), user(cc.stream) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return;
        ok = hipEventRecord(e, user) == hipSuccess && hipStreamWaitEvent(c.own_stream, e, 0) == hipSuccess;
        (void)hipEventDestroy(e);
        if (ok) c.stream = c.own_stream;
    }
    ~StreamSwap() {
        if (ok) (void)hipStreamSynchronize(c.own_stream);
        c.stream = user;
    }
};

static dda_status check_opts(const dda_solve_opts *opts, dda_solve_opts &o) {
    o = dda_solve_opts{};
    if (opts) o = *opts;
    if (o.maxit <= 0) o.maxit = 100000;
    if (o.solver != DDA_QMR && o.solver != DDA_BICGSTAB && o.solver != DDA_BICG && o.solver != DDA_CGNR) {
        set_error("dda_solve: unknown solver");
        return DDA_EINVAL;
    }
    if (o.precision != DDA_FP64 && o.precision != DDA_FP32_REFINE && o.precision != DDA_FP32_PRODUCT &&
        o.precision != DDA_FP32_RELAXED) {
        set_error("dda_solve: unknown precision");
        return DDA_EINVAL;
    }
    if (o.precision == DDA_FP32_REFINE && o.solver != DDA_QMR) {
        set_error("dda_solve: the refined single-precision solve uses QMR only");
        return DDA_ENOTSUP;
    }
    if (o.resume && (o.precision != DDA_FP64 || o.x0)) {
        set_error("dda_solve: resume continues a double-precision solve without an initial guess");
        return DDA_EINVAL;
    }
    if (o.on_breakdown != DDA_BREAKDOWN_REPORT && o.on_breakdown != DDA_BREAKDOWN_RECOVER) {
        set_error("dda_solve: unknown breakdown policy");
        return DDA_EINVAL;
    }
    return DDA_OK;
}

// host-side convergence check cadence and graph use: big problems check every iteration (the
// check is cheap next to an iteration); small ones launch chunks, replayed as a graph
static void cadence(const Ctx &c, int nrhs, const dda_solve_opts &o, int &check, bool &graph) {
    const int64_t work = c.N * (int64_t)nrhs;
    check = o.check_every > 0 ? o.check_every : work > 2000000 ? 1 : work > 100000 ? 4 : 16;
    graph = o.graph > 0 || (o.graph == 0 && work <= 2000000);
}
}  // namespace dda

namespace dda {
static dda_status solve_with(Ctx &c, const dda_beam *beams, int nrhs, double tol, const dda_solve_opts &o,
                             double2 *x, dda_solve_info *info, int check, bool graph) {
    if (o.precision == DDA_FP64) return solve_fp64(c, beams, nrhs, tol, o, x, info, check, graph);
    if (o.precision == DDA_FP32_REFINE) return solve_refine(c, beams, nrhs, tol, o, x, info, check, graph);
    return solve_products32(c, beams, nrhs, tol, o, x, info, check, graph);
}

// Breakdown recovery (DDA_BREAKDOWN_RECOVER): every right-hand side that stopped on a QMR or Bi-CG
// breakdown is solved again, alone, from its current iterate: the same method restarted on the
// current residual (new Lanczos vectors) at most twice, Bi-CGSTAB after that or at once when the
// breakdown came before the first step (the bilinear form b^T b of the start vector vanishes, and
// so it would again).  The refined single-precision form recovers in double precision.
static dda_status recover_breakdowns(Ctx &c, const dda_beam *beams, int nrhs, double tol,
                                     const dda_solve_opts &o, double2 *x, dda_solve_info *inf, int check,
                                     bool graph) {
    const size_t n3 = (size_t)3 * c.N;
    for (int r = 0; r < nrhs; ++r) {
        int restarts = 0, last_iters = inf[r].iters;
        bool stab = o.solver == DDA_BICGSTAB;
        while (inf[r].status == DDA_EBREAKDOWN && !stab) {
            stab = last_iters == 0 || restarts >= 2;
            dda_solve_opts s = o;
            s.solver = stab ? DDA_BICGSTAB : o.solver;
            s.precision = o.precision == DDA_FP32_REFINE ? DDA_FP64 : o.precision;
            s.x0 = x + r * n3;  // the solve starts from, and overwrites, the current iterate
            s.x0_check = 0;
            s.maxit = o.maxit - inf[r].iters;
            if (s.maxit <= 0) {
                inf[r].status = DDA_ENOTCONV;
                break;
            }
            dda_solve_info si{};
            if (inf[r].res_hist && inf[r].res_hist_cap > inf[r].res_hist_len) {
                si.res_hist = inf[r].res_hist + inf[r].res_hist_len;
                si.res_hist_cap = inf[r].res_hist_cap - inf[r].res_hist_len;
            }
            const dda_status st = solve_with(c, beams + r, 1, tol, s, x + r * n3, &si, check, graph);
            if (st != DDA_OK && st != DDA_ENOTCONV && st != DDA_EBREAKDOWN) return st;
            inf[r].status = si.status;
            inf[r].iters += si.iters;
            inf[r].matvecs += si.matvecs;
            inf[r].outer += si.outer;
            inf[r].res_rec = si.res_rec;
            inf[r].res_true = si.res_true;
            inf[r].res_hist_len += si.res_hist_len;
            last_iters = si.iters;
            if (!stab) ++restarts;
        }
    }
    return DDA_OK;
}
}  // namespace dda

namespace dda {
// Checkpoint file: header, the per-RHS solver states, the iterate x, the Krylov vectors.  Written
// and read by the same library build (the header carries the state size as a check).
struct CkptHeader {
    char magic[8];
    int32_t version, nrhs, solver, state_bytes;
    int64_t N, vec_elems;
    uint64_t particle;  // particle_hash of the context that wrote it
    uint64_t beams;     // beams_hash of the stopped solve
};

// FNV-1a over what defines the interaction matrix: grid, mask (materials), refractive indices, kd
// and the polarizability prescription
static uint64_t particle_hash(const Ctx &c) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](const void *p, size_t n) {
        const unsigned char *b = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    };
    const int32_t g[5] = {c.nx, c.ny, c.nz, c.polarizability, c.nmat};
    mix(g, sizeof g);
    mix(c.mask.data(), c.mask.size());
    mix(&c.kd, sizeof c.kd);
    mix(&c.m_re, sizeof c.m_re);
    mix(&c.m_im, sizeof c.m_im);
    for (size_t i = 0; i < c.mat_re.size(); ++i) {
        mix(&c.mat_re[i], sizeof(double));
        mix(&c.mat_im[i], sizeof(double));
    }
    return h;
}
static const char kCkptMagic[8] = {'D', 'D', 'A', 'C', 'K', 'P', 'T', '3'};

static dda_status ckpt_io(FILE *f, void *dev, size_t bytes, bool write, hipStream_t s) {
    std::vector<char> buf(std::min<size_t>(bytes, (size_t)64 << 20));
    for (size_t off = 0; off < bytes; off += buf.size()) {
        const size_t n = std::min(buf.size(), bytes - off);
        if (write) {
            DDA_HIP_CHECK(hipMemcpyAsync(buf.data(), (char *)dev + off, n, hipMemcpyDeviceToHost, s));
            DDA_HIP_CHECK(hipStreamSynchronize(s));
            if (std::fwrite(buf.data(), 1, n, f) != n) {
                set_error("dda_checkpoint_save: write failed");
                return DDA_EINVAL;
            }
        } else {
            if (std::fread(buf.data(), 1, n, f) != n) {
                set_error("dda_checkpoint_load: file too short");
                return DDA_EINVAL;
            }
            DDA_HIP_CHECK(hipMemcpyAsync((char *)dev + off, buf.data(), n, hipMemcpyHostToDevice, s));
            DDA_HIP_CHECK(hipStreamSynchronize(s));
        }
    }
    return DDA_OK;
}
}  // namespace dda

extern "C" dda_status dda_checkpoint_save(dda_ctx *h, const void *x, const char *path) {
    clear_error();
    Ctx *c = cx(h);
    if (!c || !x || !path) {
        set_error("dda_checkpoint_save: NULL argument");
        return DDA_EINVAL;
    }
    if (c->resume_nrhs <= 0) {
        set_error("dda_checkpoint_save: the context holds no double-precision solve stopped at its limit");
        return DDA_EINVAL;
    }
    const int nrhs = c->resume_nrhs;
    Bufs B;
    dda_status st = ensure_bufs(*c, B, nrhs, 0);  // the layout of the stopped solve's states
    if (st != DDA_OK) return st;
    CkptHeader hd{};
    std::memcpy(hd.magic, kCkptMagic, 8);
    hd.version = 3;
    hd.particle = particle_hash(*c);
    hd.beams = c->resume_beams;
    hd.nrhs = nrhs;
    hd.solver = c->resume_solver;
    hd.state_bytes = (int32_t)(nrhs * sizeof(SolveState));
    hd.N = c->N;
    hd.vec_elems = (int64_t)kNumVecs * nrhs * 3 * c->N;
    FILE *f = std::fopen(path, "wb");
    if (!f) {
        set_error(std::string("dda_checkpoint_save: cannot open ") + path);
        return DDA_EINVAL;
    }
    if (std::fwrite(&hd, sizeof hd, 1, f) != 1) {
        set_error("dda_checkpoint_save: write failed");
        st = DDA_EINVAL;
    }
    if (st == DDA_OK) st = ckpt_io(f, B.st, hd.state_bytes, true, c->stream);
    if (st == DDA_OK) st = ckpt_io(f, const_cast<void *>(x), (size_t)nrhs * 3 * c->N * sizeof(double2), true, c->stream);
    if (st == DDA_OK) st = ckpt_io(f, c->vecs, (size_t)hd.vec_elems * sizeof(double2), true, c->stream);
    if (std::fclose(f) != 0 && st == DDA_OK) {
        set_error("dda_checkpoint_save: closing the file failed");
        st = DDA_EINVAL;
    }
    return st;
}

extern "C" dda_status dda_checkpoint_load(dda_ctx *h, void *x, const char *path) {
    clear_error();
    Ctx *c = cx(h);
    if (!c || !x || !path) {
        set_error("dda_checkpoint_load: NULL argument");
        return DDA_EINVAL;
    }
    FILE *f = std::fopen(path, "rb");
    if (!f) {
        set_error(std::string("dda_checkpoint_load: cannot open ") + path);
        return DDA_EINVAL;
    }
    CkptHeader hd{};
    dda_status st = DDA_OK;
    if (std::fread(&hd, sizeof hd, 1, f) != 1 || std::memcmp(hd.magic, kCkptMagic, 8) != 0 || hd.version != 3 ||
        hd.particle != particle_hash(*c) ||
        hd.nrhs < 1 || hd.N != c->N || hd.state_bytes != (int32_t)(hd.nrhs * sizeof(SolveState)) ||
        hd.vec_elems != (int64_t)kNumVecs * hd.nrhs * 3 * c->N ||
        (hd.solver != DDA_QMR && hd.solver != DDA_BICGSTAB && hd.solver != DDA_BICG && hd.solver != DDA_CGNR)) {
        set_error("dda_checkpoint_load: not a checkpoint of this library for this particle");
        st = DDA_EINVAL;
    }
    Bufs B;
    if (st == DDA_OK) st = ensure_vecs<double>(*c, hd.nrhs);
    if (st == DDA_OK) st = ensure_bufs(*c, B, hd.nrhs, 0);
    if (st == DDA_OK) st = ckpt_io(f, B.st, hd.state_bytes, false, c->stream);
    if (st == DDA_OK) st = ckpt_io(f, x, (size_t)hd.nrhs * 3 * c->N * sizeof(double2), false, c->stream);
    if (st == DDA_OK) st = ckpt_io(f, c->vecs, (size_t)hd.vec_elems * sizeof(double2), false, c->stream);
    std::fclose(f);
    c->resume_nrhs = st == DDA_OK ? hd.nrhs : 0;
    c->resume_solver = hd.solver;
    c->resume_beams = hd.beams;
    return st;
}

extern "C" dda_status dda_solve(dda_ctx *h, const dda_beam *beams, int32_t n_rhs, double tol,
                                const dda_solve_opts *opts, void *x_out, dda_solve_info *info) {
    clear_error();
    Ctx *c = cx(h);
    if (!c || !beams || !x_out || n_rhs < 1 || !(tol > 0)) {
        set_error("dda_solve: NULL argument, n_rhs < 1 or tol <= 0");
        return DDA_EINVAL;
    }
    for (int r = 0; r < n_rhs; ++r)
        if (!beam_ok(&beams[r])) {
            set_error("dda_solve: beam without unit vectors");
            return DDA_EINVAL;
        }
    dda_solve_opts o;
    dda_status st = check_opts(opts, o);
    if (st != DDA_OK) return st;
    if (wrapped(*c) && o.precision != DDA_FP64) {
        set_error("dda_solve: an inhomogeneous particle is solved in DDA_FP64 only");
        return DDA_ENOTSUP;
    }
    int check;
    bool graph;
    cadence(*c, n_rhs, o, check, graph);
    const auto t0 = std::chrono::steady_clock::now();
    {
        StreamSwap sw(*c);
        if (!sw.ok) {
            set_error("dda_solve: could not order the solve after the caller's stream");
            return DDA_EHIP;
        }
        // the breakdown recovery needs the per-RHS report even when the caller passes none
        std::vector<dda_solve_info> own;
        dda_solve_info *inf = info;
        if (!inf && o.on_breakdown == DDA_BREAKDOWN_RECOVER) {
            own.assign(n_rhs, dda_solve_info{});
            inf = own.data();
        }
        if (!o.resume) c->resume_nrhs = 0;  // any other solve overwrites the stopped state
        st = solve_with(*c, beams, n_rhs, tol, o, (double2 *)x_out, inf, check, graph);
        if ((st == DDA_EBREAKDOWN || st == DDA_ENOTCONV) && o.on_breakdown == DDA_BREAKDOWN_RECOVER) {
            st = recover_breakdowns(*c, beams, n_rhs, tol, o, (double2 *)x_out, inf, check, graph);
            for (int r = 0; r < n_rhs && st == DDA_OK; ++r)
                if (inf[r].status != DDA_OK) st = (dda_status)inf[r].status;
        }
    }
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info)
        for (int r = 0; r < n_rhs; ++r) info[r].t_solve_s = dt;
    if (st == DDA_ENOTCONV)
        set_error("dda_solve: a right-hand side did not reach tol within maxit (per-RHS status in info)");
    if (st == DDA_EBREAKDOWN)
        set_error("dda_solve: QMR breakdown for a right-hand side (per-RHS status in info)");
    return st;
}

namespace dda {
// A batch of particles packed on one grid (pack_setup): right-hand side q is particle members[q]
// with beam beams[q].  Vectors are [P][3][N] with N the largest dipole count; the entries beyond a
// particle's own dipoles are zero in b and in the zero initial guess, and stay zero (its product
// writes only that particle's dipoles, and every vector update maps zero to zero).
static dda_status prepare_pack(Ctx &pk, Run<double> &k, Ctx *const *members, const dda_beam *beams, int P, double tol,
                               const dda_solve_opts &o, int hcap) {
    dda_status st;
    if ((st = ensure_vecs<double>(pk, P)) != DDA_OK) return st;
    if ((st = ensure_bufs(pk, k.B, P, hcap)) != DDA_OK) return st;
    std::vector<double> ar(P), ai(P);
    for (int q = 0; q < P; ++q) polarizability(*members[q], beams[q], ar[q], ai[q]);
    if ((st = upload_scales<double>(pk, ar, ai)) != DDA_OK) return st;
    const size_t n3 = k.B.n3, L = (size_t)P * n3;
    if (pk.xtmp_rows < P) {
        (void)hipFree(pk.xtmp);
        pk.xtmp = nullptr;
        pk.xtmp_rows = 0;
        if ((st = device_alloc((void **)&pk.xtmp, L * sizeof(double2))) != DDA_OK) return st;
        pk.xtmp_rows = P;
    }
    Vecs<double> v = vecs_of<double>(pk, P);
    DDA_HIP_CHECK(hipMemsetAsync(pk.vecs, 0, 7 * L * sizeof(double2), pk.stream));
    DDA_HIP_CHECK(hipMemsetAsync(pk.xtmp, 0, L * sizeof(double2), pk.stream));
    for (int q = 0; q < P; ++q) {
        // b of the particle in its own layout [3][N_q], then into the batch layout [3][N]
        double2 *tmp = v.pt + (size_t)q * n3;
        if ((st = rhs_launch<double>(*members[q], beams[q], tmp, pk.stream)) != DDA_OK) return st;
        const size_t nq = (size_t)members[q]->N;
        DDA_HIP_CHECK(hipMemcpy2DAsync(v.b + (size_t)q * n3, pk.N * sizeof(double2), tmp, nq * sizeof(double2),
                                       nq * sizeof(double2), 3, hipMemcpyDeviceToDevice, pk.stream));
        DDA_HIP_CHECK(hipMemsetAsync(tmp, 0, n3 * sizeof(double2), pk.stream));
    }
    k.c = &pk;
    k.v = v;
    k.x = pk.xtmp;
    k.solver = o.solver;
    k.mixed = o.precision == DDA_FP32_PRODUCT;
    k.beams_h = 0;
    if ((st = init_states(pk, k.B, tol, o.maxit)) != DDA_OK) return st;
    return run_begin(k, false);
}
}  // namespace dda

extern "C" dda_status dda_solve_many(dda_ctx *const *ctxs, int32_t n_ctx, const dda_beam *beams, double tol,
                                     const dda_solve_opts *opts, void *const *x_out, dda_solve_info *info) {
    clear_error();
    if (!ctxs || !beams || !x_out || n_ctx < 1 || !(tol > 0)) {
        set_error("dda_solve_many: NULL argument, n_ctx < 1 or tol <= 0");
        return DDA_EINVAL;
    }
    for (int i = 0; i < n_ctx; ++i) {
        if (!ctxs[i] || !x_out[i] || !beam_ok(&beams[i])) {
            set_error("dda_solve_many: NULL context/output or beam without unit vectors");
            return DDA_EINVAL;
        }
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) {
                set_error("dda_solve_many: a context appears twice");
                return DDA_EINVAL;
            }
    }
    dda_solve_opts o;
    dda_status st = check_opts(opts, o);
    if (st != DDA_OK) return st;
    if ((o.precision != DDA_FP64 && o.precision != DDA_FP32_PRODUCT) || o.x0) {
        set_error("dda_solve_many: DDA_FP64 or DDA_FP32_PRODUCT, without an initial guess");
        return DDA_ENOTSUP;
    }
    const bool mixed = o.precision == DDA_FP32_PRODUCT;
    for (int i = 0; i < n_ctx && mixed; ++i)
        if (!cx(ctxs[i])->ghat32) {
            set_error("dda_solve_many: DDA_FP32_PRODUCT needs contexts set up with opts.fp32");
            return DDA_ENOTSUP;
        }
    const double tol_run = mixed ? std::max(tol, 1e-6) : tol;  // single-precision products stall below 1e-6
    std::vector<dda_solve_info> local(n_ctx);
    for (int i = 0; i < n_ctx; ++i) {
        local[i] = dda_solve_info{};
        if (info) {
            local[i].res_hist = info[i].res_hist;
            local[i].res_hist_cap = info[i].res_hist_cap;
        }
    }
    const auto t0 = std::chrono::steady_clock::now();
    // groups of particles packed into one batch: same padded grid, kd and prescription, homogeneous
    std::vector<std::vector<int>> groups;
    std::vector<int> in_pack(n_ctx, -1);
    if (o.pack > 0) {
        for (int i = 0; i < n_ctx; ++i) {
            const Ctx &c = *cx(ctxs[i]);
            if (wrapped(c)) continue;
            int g = -1;
            for (size_t j = 0; j < groups.size() && g < 0; ++j) {
                const Ctx &h = *cx(ctxs[groups[j][0]]);
                if (h.Lx == c.Lx && h.Ly == c.Ly && h.Lz == c.Lz && h.kd == c.kd && h.polarizability == c.polarizability)
                    g = (int)j;
            }
            if (g < 0) {
                groups.push_back({i});
            } else {
                groups[g].push_back(i);
            }
        }
    }
    std::vector<Ctx *> packs;
    std::vector<std::vector<int>> pack_members;
    for (const auto &g : groups) {
        if (g.size() < 2) continue;
        std::vector<Ctx *> mem;
        for (int i : g) mem.push_back(cx(ctxs[i]));
        Ctx *pk = nullptr;
        const dda_status ps = pack_setup(mem.data(), (int)mem.size(), &pk);
        if (ps == DDA_ENOTSUP) continue;  // no member spans the group's grid: solved one by one
        if (ps != DDA_OK) {
            st = ps;
            break;
        }
        for (int i : g) in_pack[i] = (int)packs.size();
        packs.push_back(pk);
        pack_members.push_back(g);
    }
    std::vector<std::unique_ptr<StreamSwap>> sw;
    std::vector<Run<double>> runs(n_ctx);
    std::vector<int> hcaps(n_ctx);
    for (int i = 0; i < n_ctx && st == DDA_OK; ++i) {
        if (in_pack[i] >= 0) continue;
        Ctx &c = *cx(ctxs[i]);
        sw.emplace_back(new StreamSwap(c));
        if (!sw.back()->ok) {
            set_error("dda_solve_many: could not order a solve after the caller's stream");
            st = DDA_EHIP;
            break;
        }
        int check;
        bool graph;
        cadence(c, 1, o, check, graph);
        runs[i].check_every = check;
        runs[i].graph = graph;
        hcaps[i] = hist_cap(&local[i], 1);
        st = prepare_fp64(c, runs[i], &beams[i], 1, tol_run, o, (double2 *)x_out[i], hcaps[i]);
    }
    const int np = (int)packs.size();
    std::vector<Run<double>> pruns(np);
    std::vector<int> phcaps(np, 0);
    for (int g = 0; g < np && st == DDA_OK; ++g) {
        Ctx &pk = *packs[g];
        const std::vector<int> &mem = pack_members[g];
        const int P = (int)mem.size();
        std::vector<Ctx *> mc(P);
        std::vector<dda_beam> mb(P);
        for (int q = 0; q < P; ++q) {
            mc[q] = cx(ctxs[mem[q]]);
            mb[q] = beams[mem[q]];
            phcaps[g] = std::max(phcaps[g], hist_cap(&local[mem[q]], 1));
            // the batch's stream runs after the work already queued on each member's stream
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess ||
                hipEventRecord(e, mc[q]->stream) != hipSuccess || hipStreamWaitEvent(pk.stream, e, 0) != hipSuccess) {
                set_error("dda_solve_many: could not order a batch after the callers' streams");
                st = DDA_EHIP;
            }
            (void)hipEventDestroy(e);
        }
        if (st != DDA_OK) break;
        int check;
        bool graph;
        cadence(pk, P, o, check, graph);
        // a batch advances in step with the others from the host: checking it every iteration would
        // leave the GPU waiting on the host between its iterations, and the iterations past a right-
        // hand side's convergence cost nothing (its kernels return at once), so it replays captured
        // chunks of at least 4 iterations unless told otherwise
        if (o.check_every <= 0) check = std::max(check, 4);
        if (o.graph == 0) graph = true;
        pruns[g].check_every = check;
        pruns[g].graph = graph;
        st = prepare_pack(pk, pruns[g], mc.data(), mb.data(), P, tol_run, o, phcaps[g]);
    }
    // the batches and the remaining particles advance concurrently, each on its own stream
    bool busy = st == DDA_OK;
    while (busy && st == DDA_OK) {
        busy = false;
        for (int i = 0; i < n_ctx && st == DDA_OK; ++i)
            if (in_pack[i] < 0) st = run_poll(runs[i]);
        for (int g = 0; g < np && st == DDA_OK; ++g) st = run_poll(pruns[g]);
        for (int i = 0; i < n_ctx && st == DDA_OK; ++i)
            if (in_pack[i] < 0 && !runs[i].fin) {
                busy = true;
                st = run_issue(runs[i]);
            }
        for (int g = 0; g < np && st == DDA_OK; ++g)
            if (!pruns[g].fin) {
                busy = true;
                st = run_issue(pruns[g]);
            }
    }
    dda_status ret = st;
    for (int i = 0; i < n_ctx; ++i) {
        if (in_pack[i] >= 0) continue;
        run_end(runs[i]);
        if (ret == DDA_OK || ret == DDA_ENOTCONV || ret == DDA_EBREAKDOWN) {
            const dda_status si = finish_fp64(*cx(ctxs[i]), runs[i], 1, o, &local[i], hcaps[i]);
            if (si == DDA_EHIP || si == DDA_ENOMEM) ret = si;
            else if (ret == DDA_OK && si != DDA_OK) ret = si;
        }
    }
    for (int g = 0; g < np; ++g) {
        run_end(pruns[g]);
        Ctx &pk = *packs[g];
        const std::vector<int> &mem = pack_members[g];
        const int P = (int)mem.size();
        if (ret == DDA_OK || ret == DDA_ENOTCONV || ret == DDA_EBREAKDOWN) {
            std::vector<dda_solve_info> pin(P);
            for (int q = 0; q < P; ++q) pin[q] = local[mem[q]];
            dda_status si = finish_fp64(pk, pruns[g], P, o, pin.data(), phcaps[g]);
            for (int q = 0; q < P && si == DDA_OK; ++q) {
                const Ctx &m = *cx(ctxs[mem[q]]);
                const hipError_t e = hipMemcpy2DAsync(x_out[mem[q]], m.N * sizeof(double2), pk.xtmp + (size_t)q * 3 * pk.N,
                                                      pk.N * sizeof(double2), m.N * sizeof(double2), 3,
                                                      hipMemcpyDeviceToDevice, pk.stream);
                if (e != hipSuccess) {
                    set_error(std::string("dda_solve_many: ") + hipGetErrorString(e));
                    si = DDA_EHIP;
                }
            }
            if (si == DDA_OK && hipStreamSynchronize(pk.stream) != hipSuccess) si = DDA_EHIP;
            for (int q = 0; q < P; ++q) local[mem[q]] = pin[q];
            if (si == DDA_EHIP || si == DDA_ENOMEM) ret = si;
            else if (ret == DDA_OK && si != DDA_OK) ret = si;
        }
        destroy(packs[g]);
    }
    // single-precision products: particles whose true residual missed tol are finished in double
    // precision from their iterate (one after another; the remaining work is short)
    if (mixed && (ret == DDA_OK || ret == DDA_ENOTCONV || ret == DDA_EBREAKDOWN)) {
        ret = DDA_OK;
        for (int i = 0; i < n_ctx; ++i) {
            if (local[i].res_true < tol) {
                if (ret == DDA_OK && local[i].status != DDA_OK) ret = (dda_status)local[i].status;
                continue;
            }
            Ctx &c = *cx(ctxs[i]);
            dda_solve_opts o2 = o;
            o2.precision = DDA_FP64;
            o2.x0 = x_out[i];
            o2.x0_check = 1;
            dda_solve_info f = dda_solve_info{};
            int check;
            bool graph;
            cadence(c, 1, o2, check, graph);
            // a packed particle has no stream of its own yet: run it on its context's stream
            std::unique_ptr<StreamSwap> own;
            if (in_pack[i] >= 0) {
                own.reset(new StreamSwap(c));
                if (!own->ok) {
                    set_error("dda_solve_many: could not order a solve after the caller's stream");
                    ret = DDA_EHIP;
                    break;
                }
            }
            const dda_status si = solve_fp64(c, &beams[i], 1, tol, o2, (double2 *)x_out[i], &f, check, graph);
            if (si == DDA_EHIP || si == DDA_ENOMEM) {
                ret = si;
                break;
            }
            local[i].status = f.status;
            local[i].iters += f.iters;
            local[i].matvecs += f.matvecs;
            local[i].outer = 1;
            local[i].res_rec = f.res_rec;
            local[i].res_true = f.res_true;
            if (ret == DDA_OK && f.status != DDA_OK) ret = (dda_status)f.status;
        }
    }
    if (info)
        for (int i = 0; i < n_ctx; ++i) {
            double *hp = info[i].res_hist;
            const int hc = info[i].res_hist_cap;
            info[i] = local[i];
            info[i].res_hist = hp;
            info[i].res_hist_cap = hc;
        }
    sw.clear();
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info)
        for (int i = 0; i < n_ctx; ++i) info[i].t_solve_s = dt;
    if (ret == DDA_ENOTCONV)
        set_error("dda_solve_many: a particle did not reach tol within maxit (per-particle status in info)");
    if (ret == DDA_EBREAKDOWN)
        set_error("dda_solve_many: QMR breakdown for a particle (per-particle status in info)");
    return ret;
}
