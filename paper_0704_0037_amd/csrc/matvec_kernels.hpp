// Kernels of the interaction-matrix product y = A x (eq. 3) by zero-padded 3-D FFTs.
//
// The 3-D transform is done as 1-D transforms along x, y and z with the data re-laid between
// passes so that every pass reads and writes long contiguous runs.  Zero input is never read
// (forward passes only touch the n_a non-void planes of each axis) and unused output is never
// written (inverse passes keep only indices < n_a), as the paper's program does (Sec. 2).
// The Fourier-space multiply by the 6-component symmetric tensor is fused between the forward
// and inverse z transforms, inside registers.
//
// Layouts (c = rhs*3 + component, ncomp = 3*nrhs):
//   compact vectors x, y     [c][N]                       (component-major)
//   gmap                     [nz][ny][nx] int32: dipole index or -1 (void)
//   B1 (after x pass)        [c][nz][Lx][ny]              y fastest
//   B2 (after y pass)        [Ly][Lx][c][nz]              z fastest: a (kx, ky) column is contiguous
//   Ghat octant              [Ly/2+1][Lx/2+1][Lz/2+1][6]  components xx, xy, xz, yy, yz, zz
#pragma once

#include "fft.hpp"

namespace dda {

constexpr int kMaxRadix = 8;    // x and y passes (radix 16 costs more registers than it saves passes)
constexpr int kMaxRadixZ = 8;   // the fused z pass keeps three components in registers

// component signs under k -> L - k along each axis: xy, xz flip with x; xy, yz with y; xz, yz with z
__device__ __forceinline__ void ghat_load(const double2 *g, double2 *G, double sxy, double sxz, double syz) {
    G[0] = g[0];
    G[1] = cscale(g[1], sxy);
    G[2] = cscale(g[2], sxz);
    G[3] = g[3];
    G[4] = cscale(g[4], syz);
    G[5] = g[5];
}
__device__ __forceinline__ void ghat_load(const float2 *g, float2 *G, float sxy, float sxz, float syz) {
    G[0] = g[0];
    G[1] = cscale(g[1], sxy);
    G[2] = cscale(g[2], sxz);
    G[3] = g[3];
    G[4] = cscale(g[4], syz);
    G[5] = g[5];
}

// ---------------------------------------------------------------- K1: forward x pass
// Block: component c, plane z, NL consecutive lines y.  Gathers x from the compact vector
// (zero for void cells and for the padding), transforms along x, writes B1[c][z][kx][y].
template <typename R>
__global__ void __launch_bounds__(DDA_MAX_THREADS) k_fwd_x(const int *__restrict__ gmap, const cplx<R> *__restrict__ x,
                                                cplx<R> *__restrict__ B1, int nx, int ny, int nz, int N,
                                                FftPlan pl, const cplx<R> *__restrict__ twall, int NL) {
    using C = cplx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const C *tw = twall + pl.tw_off;
    const int L = pl.L, TPL = pl.tpl, S = lds_line_stride(L);
    const int ytiles = (ny + NL - 1) / NL;
    int b = blockIdx.x;
    const int y0 = (b % ytiles) * NL;
    b /= ytiles;
    const int z = b % nz;
    const int c = b / nz;
    const int t = threadIdx.x;
    const C *xc = x + (size_t)c * N;
    {   // pass 0 from global, lines along lanes' j (x contiguous)
        const int line = t / TPL, j = t % TPL, y = y0 + line;
        const int R0 = pl.radix[0];
        if (j < L / R0) {
            const int *grow = gmap + ((size_t)z * ny + (y < ny ? y : 0)) * nx;
            const bool yok = y < ny;
            C a[kMaxRadix];
            load_rt<-1, kMaxRadix>(a, R0, j, L, 1, tw, [&](int i) -> C {
                if (yok && i < nx) {
                    const int id = grow[i];
                    if (id >= 0) return xc[id];
                }
                return czero<C>();
            });
            C *ln = lds + line * S;
            store_rt<kMaxRadix>(a, R0, j, 1, [&](int i, C v) { ln[pidx(i)] = v; });
        }
    }
    __syncthreads();
    lds_passes<-1, kMaxRadix>(lds + (t / TPL) * S, pl, 1, pl.npass - 1, t % TPL, tw);
    C *dstc = B1 + ((size_t)c * nz + z) * (size_t)L * ny;
    if (pl.npass >= 2) {  // last pass to global, lanes over lines (y contiguous in B1)
        const int line = t % NL, j = t / NL, y = y0 + line;
        const int p = pl.npass - 1, Rp = pl.radix[p], Ns = pl.ns[p];
        if (j < L / Rp) {
            C a[kMaxRadix];
            const C *ln = lds + line * S;
            load_rt<-1, kMaxRadix>(a, Rp, j, L, Ns, tw, [&](int i) { return ln[pidx(i)]; });
            if (y < ny) store_rt<kMaxRadix>(a, Rp, j, Ns, [&](int i, C v) { dstc[(size_t)i * ny + y] = v; });
        }
    } else {
        for (int e = t; e < NL * L; e += blockDim.x) {
            const int line = e % NL, i = e / NL, y = y0 + line;
            if (y < ny) dstc[(size_t)i * ny + y] = lds[line * S + pidx(i)];
        }
    }
}

// ---------------------------------------------------------------- K2: forward y pass
// Block: component c, column kx, NL consecutive planes z.  Reads B1 lines along y (n_y
// nonzero entries), transforms, writes B2[ky][kx][c][z].
template <typename R>
__global__ void __launch_bounds__(DDA_MAX_THREADS) k_fwd_y(const cplx<R> *__restrict__ B1, cplx<R> *__restrict__ B2, int ny,
                                                int nz, int Lx, int ncomp, FftPlan pl,
                                                const cplx<R> *__restrict__ twall, int NL) {
    using C = cplx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const C *tw = twall + pl.tw_off;
    const int L = pl.L, TPL = pl.tpl, S = lds_line_stride(L);
    const int ztiles = (nz + NL - 1) / NL;
    int b = blockIdx.x;
    const int z0 = (b % ztiles) * NL;
    b /= ztiles;
    const int kx = b % Lx;
    const int c = b / Lx;
    const int t = threadIdx.x;
    {
        const int line = t / TPL, j = t % TPL, z = z0 + line;
        const int R0 = pl.radix[0];
        if (j < L / R0) {
            const bool zok = z < nz;
            const C *src = B1 + (((size_t)c * nz + (zok ? z : 0)) * Lx + kx) * ny;
            C a[kMaxRadix];
            load_rt<-1, kMaxRadix>(a, R0, j, L, 1, tw,
                                   [&](int i) -> C { return (zok && i < ny) ? src[i] : czero<C>(); });
            C *ln = lds + line * S;
            store_rt<kMaxRadix>(a, R0, j, 1, [&](int i, C v) { ln[pidx(i)] = v; });
        }
    }
    __syncthreads();
    lds_passes<-1, kMaxRadix>(lds + (t / TPL) * S, pl, 1, pl.npass - 1, t % TPL, tw);
    const size_t kystride = (size_t)Lx * ncomp * nz;
    C *dst = B2 + ((size_t)kx * ncomp + c) * nz;
    if (pl.npass >= 2) {
        const int line = t % NL, j = t / NL, z = z0 + line;
        const int p = pl.npass - 1, Rp = pl.radix[p], Ns = pl.ns[p];
        if (j < L / Rp) {
            C a[kMaxRadix];
            const C *ln = lds + line * S;
            load_rt<-1, kMaxRadix>(a, Rp, j, L, Ns, tw, [&](int i) { return ln[pidx(i)]; });
            if (z < nz) store_rt<kMaxRadix>(a, Rp, j, Ns, [&](int i, C v) { dst[(size_t)i * kystride + z] = v; });
        }
    } else {
        for (int e = t; e < NL * L; e += blockDim.x) {
            const int line = e % NL, i = e / NL, z = z0 + line;
            if (z < nz) dst[(size_t)i * kystride + z] = lds[line * S + pidx(i)];
        }
    }
}

// ------------------------------------------------- K3: forward z, tensor multiply, inverse z
// Block: NC columns (kx, ky) of one right-hand side; a thread owns butterfly j of all three
// components of its column, so the last forward pass leaves X(kz) for the three components in
// the same registers that the first inverse pass (the reversed radix order) consumes.
template <typename R>
__device__ __forceinline__ void ghat_mul3(cplx<R> (*a)[kMaxRadixZ], int Rr, int j, int q, int Lz,
                                          const cplx<R> *__restrict__ gcol, R sx, R sy) {
    using C = cplx<R>;
    const int hz = Lz / 2;
#pragma unroll
    for (int r = 0; r < kMaxRadixZ; ++r) {
        if (r < Rr) {
            const int kz = j + r * q;
            const int kzo = kz <= hz ? kz : Lz - kz;
            const R sz = kz <= hz ? (R)1 : (R)-1;
            C G[6];
            ghat_load(gcol + (size_t)kzo * 6, G, sx * sy, sx * sz, sy * sz);
            const C X = a[0][r], Y = a[1][r], Z = a[2][r];
            a[0][r] = cadd(cadd(cmul(G[0], X), cmul(G[1], Y)), cmul(G[2], Z));
            a[1][r] = cadd(cadd(cmul(G[1], X), cmul(G[3], Y)), cmul(G[4], Z));
            a[2][r] = cadd(cadd(cmul(G[2], X), cmul(G[4], Y)), cmul(G[5], Z));
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(DDA_MAX_THREADS) k_zmul(cplx<R> *__restrict__ B2, const cplx<R> *__restrict__ Gh, int nz,
                                               int Lx, int Ly, int ncomp, FftPlan pf, FftPlan pi,
                                               const cplx<R> *__restrict__ twall, int NC) {
    using C = cplx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const C *tw = twall + pf.tw_off;
    const int L = pf.L, TPL = pf.tpl, S = lds_line_stride(L);
    const int t = threadIdx.x;
    const int col = t / TPL, j = t % TPL;
    const int cidx = blockIdx.x * NC + col;
    const int rhs = blockIdx.y;
    const bool colok = cidx < Lx * Ly;
    const int kx = colok ? cidx % Lx : 0, ky = colok ? cidx / Lx : 0;
    const int hx = Lx / 2, hy = Ly / 2;
    const int kxo = kx <= hx ? kx : Lx - kx, kyo = ky <= hy ? ky : Ly - ky;
    const R sx = kx <= hx ? (R)1 : (R)-1, sy = ky <= hy ? (R)1 : (R)-1;
    const C *gcol = Gh + ((size_t)kyo * (hx + 1) + kxo) * (size_t)(L / 2 + 1) * 6;
    C *colp = B2 + ((size_t)cidx * ncomp + rhs * 3) * nz;  // three components, nz each
    C *ln[3] = {lds + (col * 3 + 0) * S, lds + (col * 3 + 1) * S, lds + (col * 3 + 2) * S};
    C a[3][kMaxRadixZ];
    const int np = pf.npass;
    // ---- forward pass 0 from global
    const int R0 = pf.radix[0];
    if (j < L / R0) {
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            const C *src = colp + (size_t)cc * nz;
            load_rt<-1, kMaxRadixZ>(a[cc], R0, j, L, 1, tw,
                                    [&](int i) -> C { return (colok && i < nz) ? src[i] : czero<C>(); });
        }
    }
    if (np >= 2) {
        if (j < L / R0) {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                store_rt<kMaxRadixZ>(a[cc], R0, j, 1, [&](int i, C v) { ln[cc][pidx(i)] = v; });
        }
        __syncthreads();
        for (int p = 1; p < np - 1; ++p) {  // middle forward passes, in place
            const int Rp = pf.radix[p], Ns = pf.ns[p];
            const bool act = j < L / Rp;
            if (act) {
#pragma unroll
                for (int cc = 0; cc < 3; ++cc)
                    load_rt<-1, kMaxRadixZ>(a[cc], Rp, j, L, Ns, tw, [&](int i) { return ln[cc][pidx(i)]; });
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int cc = 0; cc < 3; ++cc)
                    store_rt<kMaxRadixZ>(a[cc], Rp, j, Ns, [&](int i, C v) { ln[cc][pidx(i)] = v; });
            }
            __syncthreads();
        }
        const int Rl = pf.radix[np - 1], Nl = pf.ns[np - 1];
        if (j < L / Rl) {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                load_rt<-1, kMaxRadixZ>(a[cc], Rl, j, L, Nl, tw, [&](int i) { return ln[cc][pidx(i)]; });
        }
    }
    // ---- multiply by the tensor at kz = j + r * L/Rl
    const int Rl = pf.radix[np - 1];
    const bool actl = j < L / Rl;
    if (actl && colok) ghat_mul3<R>(a, Rl, j, L / Rl, L, gcol, sx, sy);
    // ---- inverse pass 0 on the same registers (pi.radix[0] == Rl, Ns = 1)
    if (actl) {
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) regs_rt<+1, kMaxRadixZ>(a[cc], Rl, j, L, 1, tw);
    }
    if (np >= 2) {
        __syncthreads();  // all forward reads of LDS are done
        if (actl) {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                store_rt<kMaxRadixZ>(a[cc], Rl, j, 1, [&](int i, C v) { ln[cc][pidx(i)] = v; });
        }
        __syncthreads();
        for (int p = 1; p < np - 1; ++p) {
            const int Rp = pi.radix[p], Ns = pi.ns[p];
            const bool act = j < L / Rp;
            if (act) {
#pragma unroll
                for (int cc = 0; cc < 3; ++cc)
                    load_rt<+1, kMaxRadixZ>(a[cc], Rp, j, L, Ns, tw, [&](int i) { return ln[cc][pidx(i)]; });
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int cc = 0; cc < 3; ++cc)
                    store_rt<kMaxRadixZ>(a[cc], Rp, j, Ns, [&](int i, C v) { ln[cc][pidx(i)] = v; });
            }
            __syncthreads();
        }
        const int Rq = pi.radix[np - 1], Nq = pi.ns[np - 1];
        if (j < L / Rq) {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                load_rt<+1, kMaxRadixZ>(a[cc], Rq, j, L, Nq, tw, [&](int i) { return ln[cc][pidx(i)]; });
            if (colok) {
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    C *dst = colp + (size_t)cc * nz;
                    store_rt<kMaxRadixZ>(a[cc], Rq, j, Nq, [&](int i, C v) {
                        if (i < nz) dst[i] = v;
                    });
                }
            }
        }
    } else if (actl && colok) {  // single pass: inverse output straight to global
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            C *dst = colp + (size_t)cc * nz;
            store_rt<kMaxRadixZ>(a[cc], Rl, j, 1, [&](int i, C v) {
                if (i < nz) dst[i] = v;
            });
        }
    }
}

// ---------------------------------------------------------------- K4: inverse y pass
// Block: component c, column kx, NL consecutive planes z.  Reads B2 along ky (all Ly entries),
// inverse transform, keeps y < ny, writes B1[c][z][kx][y].
template <typename R>
__global__ void __launch_bounds__(DDA_MAX_THREADS) k_inv_y(const cplx<R> *__restrict__ B2, cplx<R> *__restrict__ B1, int ny,
                                                int nz, int Lx, int ncomp, FftPlan pl,
                                                const cplx<R> *__restrict__ twall, int NL) {
    using C = cplx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const C *tw = twall + pl.tw_off;
    const int L = pl.L, TPL = pl.tpl, S = lds_line_stride(L);
    const int ztiles = (nz + NL - 1) / NL;
    int b = blockIdx.x;
    const int z0 = (b % ztiles) * NL;
    b /= ztiles;
    const int kx = b % Lx;
    const int c = b / Lx;
    const int t = threadIdx.x;
    const size_t kystride = (size_t)Lx * ncomp * nz;
    const C *src = B2 + ((size_t)kx * ncomp + c) * nz;
    {   // pass 0 from global, lanes over lines (z contiguous in B2)
        const int line = t % NL, j = t / NL, z = z0 + line;
        const int R0 = pl.radix[0];
        if (j < L / R0) {
            const bool zok = z < nz;
            C a[kMaxRadix];
            load_rt<+1, kMaxRadix>(a, R0, j, L, 1, tw,
                                   [&](int i) -> C { return zok ? src[(size_t)i * kystride + z] : czero<C>(); });
            C *ln = lds + line * S;
            store_rt<kMaxRadix>(a, R0, j, 1, [&](int i, C v) { ln[pidx(i)] = v; });
        }
    }
    __syncthreads();
    lds_passes<+1, kMaxRadix>(lds + (t / TPL) * S, pl, 1, pl.npass - 1, t % TPL, tw);
    const int line = t / TPL, j = t % TPL, z = z0 + line;
    C *dst = B1 + (((size_t)c * nz + (z < nz ? z : 0)) * Lx + kx) * ny;
    if (pl.npass >= 2) {
        const int p = pl.npass - 1, Rp = pl.radix[p], Ns = pl.ns[p];
        if (j < L / Rp) {
            C a[kMaxRadix];
            const C *ln = lds + line * S;
            load_rt<+1, kMaxRadix>(a, Rp, j, L, Ns, tw, [&](int i) { return ln[pidx(i)]; });
            if (z < nz) store_rt<kMaxRadix>(a, Rp, j, Ns, [&](int i, C v) {
                if (i < ny) dst[i] = v;
            });
        }
    } else if (z < nz) {
        for (int i = j; i < ny; i += TPL) dst[i] = lds[line * S + pidx(i)];
    }
}

// ----------------------------------------------- K5: inverse x pass, unpad, y = x - s * conv
// Block: component c, plane z, NL consecutive lines y.  Reads B1 along kx, inverse transform,
// keeps x < nx at non-void cells: y = x - scale[rhs] * v with scale = alpha / (Lx Ly Lz).
// Optionally accumulates the bilinear dot sum x_i y_i of the block into dots[blockIdx.x].
template <typename R>
__device__ __forceinline__ cplx<R> block_sum(cplx<R> v, cplx<R> *scratch) {
    // deterministic tree over LDS; works for any block size (blocks need not be whole waves)
    using C = cplx<R>;
    const int t = threadIdx.x, n = blockDim.x;
    __syncthreads();
    scratch[t] = v;
    __syncthreads();
    int h = 1;
    while (h < n) h <<= 1;
    for (h >>= 1; h > 0; h >>= 1) {
        if (t < h && t + h < n) scratch[t] = cadd(scratch[t], scratch[t + h]);
        __syncthreads();
    }
    return scratch[0];  // valid in every thread
}

template <typename R>
__global__ void __launch_bounds__(DDA_MAX_THREADS) k_inv_x(const int *__restrict__ gmap, const cplx<R> *__restrict__ B1,
                                                const cplx<R> *__restrict__ xin, cplx<R> *__restrict__ yout,
                                                int nx, int ny, int nz, int N, FftPlan pl,
                                                const cplx<R> *__restrict__ twall, int NL,
                                                const cplx<R> *__restrict__ scale, cplx<R> *__restrict__ dots) {
    using C = cplx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const C *tw = twall + pl.tw_off;
    const int L = pl.L, TPL = pl.tpl, S = lds_line_stride(L);
    const int ytiles = (ny + NL - 1) / NL;
    int b = blockIdx.x;
    const int y0 = (b % ytiles) * NL;
    b /= ytiles;
    const int z = b % nz;
    const int c = b / nz;
    const int t = threadIdx.x;
    const C *src = B1 + ((size_t)c * nz + z) * (size_t)L * ny;
    {   // pass 0 from global, lanes over lines (y contiguous in B1)
        const int line = t % NL, j = t / NL, y = y0 + line;
        const int R0 = pl.radix[0];
        if (j < L / R0) {
            const bool yok = y < ny;
            C a[kMaxRadix];
            load_rt<+1, kMaxRadix>(a, R0, j, L, 1, tw,
                                   [&](int i) -> C { return yok ? src[(size_t)i * ny + y] : czero<C>(); });
            C *ln = lds + line * S;
            store_rt<kMaxRadix>(a, R0, j, 1, [&](int i, C v) { ln[pidx(i)] = v; });
        }
    }
    __syncthreads();
    lds_passes<+1, kMaxRadix>(lds + (t / TPL) * S, pl, 1, pl.npass - 1, t % TPL, tw);
    const int line = t / TPL, j = t % TPL, y = y0 + line;
    const C sc = scale[c / 3];
    const C *xc = xin + (size_t)c * N;
    C *yc = yout + (size_t)c * N;
    const int *grow = gmap + ((size_t)z * ny + (y < ny ? y : 0)) * nx;
    C acc = czero<C>();
    auto emit = [&](int i, C v) {
        if (y < ny && i < nx) {
            const int id = grow[i];
            if (id >= 0) {
                const C xv = xc[id];
                const C out = csub(xv, cmul(sc, v));
                yc[id] = out;
                acc = cadd(acc, cmul(xv, out));
            }
        }
    };
    if (pl.npass >= 2) {
        const int p = pl.npass - 1, Rp = pl.radix[p], Ns = pl.ns[p];
        if (j < L / Rp) {
            C a[kMaxRadix];
            const C *ln = lds + line * S;
            load_rt<+1, kMaxRadix>(a, Rp, j, L, Ns, tw, [&](int i) { return ln[pidx(i)]; });
            store_rt<kMaxRadix>(a, Rp, j, Ns, emit);
        }
    } else {
        for (int i = j; i < nx; i += TPL) emit(i, lds[line * S + pidx(i)]);
    }
    if (dots) {
        C s = block_sum<R>(acc, lds);  // LDS reused as scratch: all FFT reads are done
        if (t == 0) dots[blockIdx.x] = s;
    }
}

// ------------------------------------------------------------- Fourier-space tensor build
// Fill a full L grid with one component (mu, nu) of the Green's tensor at the circulant
// displacement of each grid point; the self term and the never-used middle indices are 0.
__global__ void k_gfill(double2 *__restrict__ buf, int comp, int nx, int ny, int nz, int Lx, int Ly, int Lz,
                        double k);

// Full (unpruned) in-place 1-D FFT along one axis of an Lx*Ly*Lz grid.  Lines are (u, v) with
// base u*su + v*sv, point stride sp; a block takes NL consecutive u.  lanes_over_lines selects
// the coalesced mapping for strided axes.
__global__ void k_fft_axis(double2 *__restrict__ buf, int nu, int nv, long su, long sv, long sp, FftPlan pl,
                           const double2 *__restrict__ twall, int NL, int lanes_over_lines);

// Copy the octant 0 <= k <= L/2 of one transformed component into the tensor array.
__global__ void k_gextract(const double2 *__restrict__ buf, double2 *__restrict__ Gh, int comp, int Lx, int Ly,
                           int Lz);

}  // namespace dda
