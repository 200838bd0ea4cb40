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
//   Ghat octant              [Ly/2+1][Lx/2+1][6][Lz/2+1]  components xx, xy, xz, yy, yz, zz; a column's
//                            six kz-runs are contiguous so a wave's tensor loads are unit-stride
#pragma once

#include <type_traits>

#include "fft.hpp"

namespace dda {

constexpr int kMaxRadix = 8;    // x and y passes (radix 16 costs more registers than it saves passes)
constexpr int kMaxRadixZ = 8;   // the fused z pass keeps three components in registers

// ---------------------------------------------------------------- K1: forward x pass
// Block: component c, plane z, NL consecutive lines y.  Gathers x from the compact vector
// (zero for void cells and for the padding), transforms along x, writes B1[c][z][kx][y].
// RX: precision of the input vector (the transform runs in R; a double vector may feed a single-
// precision transform)
// rows: per (y, z) row of the grid, {x0 | x1 << 16, first dipole} when the row's non-void cells are
// the single run x0 <= x < x1 (dipole indices then follow from x without a lookup), x0 = 0xFFFF
// when they are not (the cell map gmap is used)
__device__ __forceinline__ bool row_run(const int2 *__restrict__ rows, int row, int &x0, int &x1, int &id0) {
    const int2 rr = rows[row];
    x0 = rr.x & 0xFFFF;
    x1 = (rr.x >> 16) & 0xFFFF;
    id0 = rr.y;
    return x0 != 0xFFFF;
}

// Workgroups go to the eight XCDs round-robin by index.  The x and y passes renumber them so that
// each XCD runs one contiguous range of the logical block order: the neighbouring tiles that read
// or write neighbouring segments of the same rows then share an L2 (0: hardware order).
#ifndef DDA_XCD_REMAP
#define DDA_XCD_REMAP 1
#endif
__device__ __forceinline__ int xcd_block() {
#if DDA_XCD_REMAP
    const int G = gridDim.x, b = blockIdx.x, q = G >> 3, r = G & 7, x = b & 7, i = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
#else
    return blockIdx.x;
#endif
}

template <typename R, int LC, typename RX = R>
__global__ void __launch_bounds__(max_threads<R>()) k_fwd_x(const int *__restrict__ gmap, const int2 *__restrict__ rows,
                                                size_t gstride, size_t rstride, const cplx<RX> *__restrict__ x,
                                                cplx<R> *__restrict__ B1, int nx, int ny, int nz, int N,
                                                FftPlan pl_rt, const cplx<R> *__restrict__ twall, int lnl,
                                                const int *__restrict__ done) {
    using C = cplx<R>;
    const FftPlan pl = plan_of<LC, kMaxRadix, false>(pl_rt);
    const int NL = 1 << lnl;
    const int NP = pl.npass, R0 = pl.radix[0], RL = pl.radix[NP - 1], NSL = pl.ns[NP - 1];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const C *tw = twall + pl_rt.tw_off;
    const int L = pl.L, TPL = pl.tpl, S = lds_line_stride(L);
    const int ytiles = (ny + NL - 1) >> lnl;
    int b = xcd_block();
    const int y0 = (b % ytiles) * NL;
    b /= ytiles;
    const int z = b % nz;
    const int c = b / nz;
    if (done && done[c / 3]) return;  // this right-hand side has converged
    // a batch of particles (right-hand sides with their own dipoles on a common grid): this one's maps
    gmap += (size_t)(c / 3) * gstride;
    rows += (size_t)(c / 3) * rstride;
    const int t = threadIdx.x;
    const cplx<RX> *xc = x + (size_t)c * N;
    {   // pass 0 from global, lines along lanes' j (x contiguous)
        const int line = t / TPL, j = t % TPL, y = y0 + line;
        const int *grow = gmap + ((size_t)z * ny + (y < ny ? y : 0)) * nx;
        const bool yok = y < ny;
        int rx0, rx1, id0;
        const bool run = row_run(rows, z * ny + (y < ny ? y : 0), rx0, rx1, id0);
        for (int jb = j; jb < L / R0; jb += TPL) {
            C a[kMaxRadix];
            if (run)
                load_rt<-1, kMaxRadix, true>(a, R0, jb, L, 1, tw, [&](int i) -> C {
                    return (yok && i >= rx0 && i < rx1) ? ccast<C>(xc[id0 + i - rx0]) : czero<C>();
                });
            else
                load_rt<-1, kMaxRadix, true>(a, R0, jb, L, 1, tw, [&](int i) -> C {
                    if (yok && i < nx) {
                        const int id = grow[i];
                        if (id >= 0) return ccast<C>(xc[id]);
                    }
                    return czero<C>();
                });
            C *ln = lds + line * S;
            store_rt<kMaxRadix>(a, R0, jb, 1, [&](int i, C v) { ln[pidx(i)] = v; });
        }
    }
    constexpr bool W = wave_lines<LC, kMaxRadix>();
    lds_sync<W>();
    lds_passes<-1, kMaxRadix, LC, false>(lds + (t / TPL) * S, pl_rt, 1, NP - 1, t % TPL, tw);
    if constexpr (W) __syncthreads();  // the store mapping below crosses waves
    const int nyp = row_pitch(ny);
    C *dstc = B1 + ((size_t)c * nz + z) * (size_t)L * nyp;
    if (NP >= 2) {  // last pass to global, lanes over lines (y contiguous in B1)
        const int line = t & (NL - 1), j = t >> lnl, y = y0 + line;
        const int Rp = RL, Ns = NSL;
        for (int jb = j; jb < L / Rp; jb += TPL) {
            C a[kMaxRadix];
            const C *ln = lds + line * S;
            load_rt<-1, kMaxRadix>(a, Rp, jb, L, Ns, tw, [&](int i) { return ln[pidx(i)]; });
            if (y < ny) store_rt<kMaxRadix>(a, Rp, jb, Ns, [&](int i, C v) { st_stream(&dstc[(size_t)i * nyp + y], v); });
        }
    } else {
        for (int e = t; e < NL * L; e += blockDim.x) {
            const int line = e & (NL - 1), i = e >> lnl, y = y0 + line;
            if (y < ny) dstc[(size_t)i * nyp + y] = lds[line * S + pidx(i)];
        }
    }
}

// ---------------------------------------------------------------- K2: forward y pass
// Block: component c, column kx, NL consecutive planes z.  Reads B1 lines along y (n_y
// nonzero entries), transforms, writes B2[ky][kx][c][z].
template <typename R, int LC>
__global__ void __launch_bounds__(max_threads<R>()) k_fwd_y(const cplx<R> *__restrict__ B1, cplx<R> *__restrict__ B2, int ny,
                                                int nz, int Lx, int ncomp, FftPlan pl_rt,
                                                const cplx<R> *__restrict__ twall, int lnl,
                                                const int *__restrict__ done) {
    using C = cplx<R>;
    const FftPlan pl = plan_of<LC, kMaxRadix, false>(pl_rt);
    const int NL = 1 << lnl;
    const int NP = pl.npass, R0 = pl.radix[0], RL = pl.radix[NP - 1], NSL = pl.ns[NP - 1];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const C *tw = twall + pl_rt.tw_off;
    const int L = pl.L, TPL = pl.tpl, S = lds_line_stride(L);
    const int ztiles = (nz + NL - 1) >> lnl;
    int b = xcd_block();
    const int z0 = (b % ztiles) * NL;
    b /= ztiles;
    const int kx = b % Lx;
    const int c = b / Lx;
    if (done && done[c / 3]) return;
    const int t = threadIdx.x;
    {
        const int line = t / TPL, j = t % TPL, z = z0 + line;
        const bool zok = z < nz;
        const C *src = B1 + (((size_t)c * nz + (zok ? z : 0)) * Lx + kx) * row_pitch(ny);
        for (int jb = j; jb < L / R0; jb += TPL) {
            C a[kMaxRadix];
            load_rt<-1, kMaxRadix, true>(a, R0, jb, L, 1, tw,
                                   [&](int i) -> C { return (zok && i < ny) ? ld_stream(&src[i]) : czero<C>(); });
            C *ln = lds + line * S;
            store_rt<kMaxRadix>(a, R0, jb, 1, [&](int i, C v) { ln[pidx(i)] = v; });
        }
    }
    constexpr bool W = wave_lines<LC, kMaxRadix>();
    lds_sync<W>();
    lds_passes<-1, kMaxRadix, LC, false>(lds + (t / TPL) * S, pl_rt, 1, NP - 1, t % TPL, tw);
    if constexpr (W) __syncthreads();  // the store mapping below crosses waves
    const int nzp = row_pitch(nz);
#if DDA_B2_COLMAJOR
    const size_t kystride = (size_t)nzp;
    C *dst = B2 + ((size_t)kx * ncomp + c) * (size_t)L * nzp;
#else
    const size_t kystride = (size_t)Lx * ncomp * nzp;
    C *dst = B2 + ((size_t)kx * ncomp + c) * nzp;
#endif
    if (NP >= 2) {
        const int line = t & (NL - 1), j = t >> lnl, z = z0 + line;
        const int Rp = RL, Ns = NSL;
        for (int jb = j; jb < L / Rp; jb += TPL) {
            C a[kMaxRadix];
            const C *ln = lds + line * S;
            load_rt<-1, kMaxRadix>(a, Rp, jb, L, Ns, tw, [&](int i) { return ln[pidx(i)]; });
            if (z < nz) store_rt<kMaxRadix>(a, Rp, jb, Ns, [&](int i, C v) { st_stream(&dst[(size_t)i * kystride + z], v); });
        }
    } else {
        for (int e = t; e < NL * L; e += blockDim.x) {
            const int line = e & (NL - 1), i = e >> lnl, z = z0 + line;
            if (z < nz) dst[(size_t)i * kystride + z] = lds[line * S + pidx(i)];
        }
    }
}

// ------------------------------------------------- K3: forward z, tensor multiply, inverse z
// The (up to) four columns (kx, ky) with kx in {kxo, Lx - kxo}, ky in {kyo, Ly - kyo} share one
// octant column (kxo, kyo) of the tensor.  A block owns one octant column: it stages the column's
// six kz-runs in LDS once and then runs, for every right-hand side, its mirror columns through
// the z pass, zmul_slots of them side by side per round.  The tensor is read once per batch.
//
// Within a column, thread (comp, j) owns butterfly j of the line of one component (one wave per
// line at L = 512).  After the forward passes the three transformed lines sit in LDS in natural
// order; each thread then forms component `comp` of Ghat(k) X(k) at the frequencies k = j + r L/R0
// that the first inverse pass (radix R0, the forward plan reversed) needs from it, straight into
// registers.
template <typename R, int LC>
__global__ void __launch_bounds__(DDA_ZMUL_THREADS, DDA_ZMUL_WAVES_PER_EU) k_zmul(cplx<R> *__restrict__ B2, const cplx<R> *__restrict__ Gh,
                                                          int nz, int Lx, int Ly, int nrhs, FftPlan pf_rt,
                                                          FftPlan pi_rt, const cplx<R> *__restrict__ twall,
                                                          const int *__restrict__ done) {
    using C = cplx<R>;
    // multi-mode lengths run the forward plan sorted with its largest radix last and the inverse
    // sorted largest first, so the multiply and the passes next to it keep one butterfly per thread
    constexpr bool FLIP = LC > 0 && zmul_multi(make_plan(LC, kMaxRadixZ, false));
    constexpr int FO = FLIP ? 2 : 0, IO = FLIP ? 3 : 1;  // plan orders (make_plan) of the two transforms
    const FftPlan pf = plan_of<LC, kMaxRadixZ, FO>(pf_rt);
    const FftPlan pi = plan_of<LC, kMaxRadixZ, IO>(pi_rt);
    const int NPZ = pf.npass, RQ = pi.radix[NPZ - 1], NQ = pi.ns[NPZ - 1];
    // one butterfly per thread in every pass, or (MB) L / (largest radix) threads per line with
    // several butterflies per thread in the passes of smaller radix
    const bool MB = zmul_multi(pf);
    const int L = pf.L, TPL = zmul_tpl(pf), S = lds_line_stride(L);
    const int np = pf.npass;
    const int R0 = pf.radix[0];
    const int Ri = pi.radix[0];  // == pf.radix[np - 1]
    const int qi = L / Ri;
    // XCD-aware block order: neighbouring octant columns run on the same XCD
    const int per_xcd = gridDim.x / 8;
    const int oct = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int hx = Lx / 2, hy = Ly / 2, hz = L / 2, hz1 = hz + 1;
    const int nzp = row_pitch(nz);
    if (oct >= (hx + 1) * (hy + 1)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const C *tw = twall + pf_rt.tw_off;
    const int t = threadIdx.x;
    const int CT = zmul_ct(pf), LW = zmul_lanes(pf), SL = zmul_slots(pf);
    const int comp = t / CT, u = t % CT, lslot = u / LW, jj = u % LW;  // component, column slot, lane
    const int j0 = jj < TPL ? jj : L;  // lanes past TPL take no butterfly
    const int kxo = oct % (hx + 1), kyo = oct / (hx + 1);
    const int nmx = (kxo == 0 || 2 * kxo == Lx) ? 1 : 2;  // distinct x mirrors of this column
    const int nmy = (kyo == 0 || 2 * kyo == Ly) ? 1 : 2;
    C *gsh = lds;                            // [6][hz1] tensor runs of this octant column
    C *lcol = lds + 6 * hz1 + lslot * 3 * S;  // [3][S] the three component lines of this slot
    {
        const C *gcol = Gh + (size_t)oct * 6 * hz1;
        for (int e = t; e < 6 * hz1; e += blockDim.x) gsh[e] = gcol[e];
    }
    // all-radix-8 lengths: the twiddle bases of every pass staged after the lines (no global
    // twiddle loads inside the rounds)
    constexpr bool TWL = LC > 0 && all_radix8(LC, kMaxRadixZ);
    C *tws = lds + 6 * hz1 + SL * 3 * S;
    if constexpr (TWL) {
        for (int e = t; e < LC / 8; e += blockDim.x) tws[e] = tw[e];
        __syncthreads();
    }
    const auto twp0 = [&] {
        if constexpr (TWL) return TwStaged<C>{tws, tw};
        else return tw;
    }();
    C *ln = lcol + comp * S;
    constexpr bool W = LC > 0 && 64 % zmul_lanes(make_plan(LC, kMaxRadixZ, false)) == 0;  // a line within one wave
    const int ngroups = 4 / SL;
    const bool act = j0 < qi;
    // G[comp][d] for d = x, y, z: row comp of the symmetric tensor is (xx,xy,xz), (xy,yy,yz), (xz,yz,zz)
    const int g0 = comp == 0 ? 0 : comp == 1 ? 1 : 2;
    const int g1 = comp == 0 ? 1 : comp == 1 ? 3 : 4;
    const int g2 = comp == 0 ? 2 : comp == 1 ? 4 : 5;
    // rounds q = rhs * ngroups + grp; a round is skipped when its right-hand side has converged or
    // its group holds no distinct column
    const int Q = nrhs * ngroups;
    auto next_round = [&](int q) {
        for (; q < Q; ++q) {
            const int rhs = q / ngroups, slot0 = (q % ngroups) * SL;
            if (done && done[rhs]) continue;
            if (((slot0 & 1) && nmx == 1) || ((slot0 & 2) && nmy == 1)) continue;
            break;
        }
        return q;
    };
    const int q0 = L / R0;
    for (int q = next_round(0); q < Q; q = next_round(q + 1)) {
        const int rhs = q / ngroups, grp = q % ngroups;
        {
            // several butterflies per thread: the butterfly index and the twiddle table are opaque
            // to the compiler from round to round, so the many per-thread LDS addresses and twiddle
            // loads are formed inside each round instead of being held in registers across rounds
            // (which spills)
            auto twp = twp0;
            int j = j0;
            if (MB) {
                if constexpr (!TWL) __asm__ volatile("" : "+s"(twp));
                __asm__ volatile("" : "+v"(j));
            }
            const int slot = grp * SL + lslot;  // mirror 0..3 of the octant column
            const bool mxs = slot & 1, mys = slot & 2;
            const bool ok = (!mxs || nmx == 2) && (!mys || nmy == 2);  // slot holds a distinct column
            const int kx = mxs ? Lx - kxo : kxo, ky = mys ? Ly - kyo : kyo;
#if DDA_B2_COLMAJOR
            C *line = B2 + (((size_t)(ok ? kx : 0) * (3 * nrhs) + rhs * 3 + comp) * Ly + (ok ? ky : 0)) * nzp;
#else
            C *line = B2 + (((size_t)(ok ? ky : 0) * Lx + (ok ? kx : 0)) * (3 * nrhs) + rhs * 3 + comp) * nzp;
#endif
            for (int jb = j; jb < q0; jb += TPL) {
                C a[kMaxRadixZ];
                load_rt<-1, kMaxRadixZ, true>(a, R0, jb, L, 1, twp,
                                        [&](int i) -> C { return (ok && i < nz) ? ld_stream(&line[i]) : czero<C>(); });
                store_rt<kMaxRadixZ>(a, R0, jb, 1, [&](int i, C v) { ln[pidx(i)] = v; });
            }
            lds_sync<W>();
            // LDS passes [p0, p1) of the forward (inverse) plan, one or several butterflies per thread
            auto fpasses = [&](int p0, int p1) {
                if (MB) lds_passes<-1, kMaxRadixZ, LC, FO, false, true>(ln, pf_rt, p0, p1, j, twp);
                else lds_passes<-1, kMaxRadixZ, LC, FO, true>(ln, pf_rt, p0, p1, j, twp);
            };
            auto ipasses = [&](int p0, int p1) {
                if (MB) lds_passes<+1, kMaxRadixZ, LC, IO, false, true>(ln, pi_rt, p0, p1, j, twp);
                else lds_passes<+1, kMaxRadixZ, LC, IO, true>(ln, pi_rt, p0, p1, j, twp);
            };
            // own-component path (double precision): all forward passes but the last through LDS;
            // the last one keeps this thread's outputs (its own component at kz = j + r qi) in
            // registers and also stores them, in natural order, for the two other components
            constexpr bool OWN = DDA_ZMUL_OWN && sizeof(R) == 8;
            C a[kMaxRadixZ];
            if constexpr (OWN) {
                if (np >= 2) {
                    fpasses(1, np - 1);
                    const int NsL = L / Ri;  // Ns of the last forward pass
                    if (act) load_rt<-1, kMaxRadixZ>(a, Ri, j, L, NsL, twp, [&](int i) { return ln[pidx(i)]; });
                    lds_sync<W>();
                    if (act) store_rt<kMaxRadixZ>(a, Ri, j, NsL, [&](int i, C v) { ln[pidx(i)] = v; });
                } else if (act) {
#pragma unroll
                    for (int r = 0; r < kMaxRadixZ; ++r) a[r] = ln[pidx(j + r * qi)];
                }
                __syncthreads();  // the multiply reads the other two lines and the staged tensor
            } else {
                fpasses(1, np);  // natural order in LDS afterwards
                if constexpr (W) __syncthreads();  // the multiply reads all three lines and the staged tensor
            }
            if (act) {
                // signs under the mirrors: a component is odd along an axis when exactly one of its
                // indices is that axis; the z-odd ones (xz, yz) pick up sz
                const R sx = mxs ? (R)-1 : (R)1, sy = mys ? (R)-1 : (R)1;
                const R s0 = comp == 0 ? (R)1 : comp == 1 ? sx * sy : sx;
                const R s1 = comp == 0 ? sx * sy : comp == 1 ? (R)1 : sy;
                const R s2 = comp == 0 ? sx : comp == 1 ? sy : (R)1;
                auto mul = [&](auto radix_tag) {
                    constexpr int RI = decltype(radix_tag)::value;
                    // one code path per component (a wave holds one component when its lines do
                    // not straddle waves); on the own-component path each reads only the two
                    // other lines
                    auto rows = [&](auto comp_tag) {
                        constexpr int CP = decltype(comp_tag)::value;
#pragma unroll
                        for (int r = 0; r < RI; ++r) {
                            const int kz = j + r * qi;
                            const bool lo = kz <= hz;
                            const R sz = lo ? (R)1 : (R)-1;
                            const C *g = gsh + (lo ? kz : L - kz);
                            const C G0 = cscale(g[g0 * hz1], CP == 2 ? s0 * sz : s0);
                            const C G1 = cscale(g[g1 * hz1], CP == 2 ? s1 * sz : s1);
                            const C G2 = cscale(g[g2 * hz1], CP == 2 ? s2 : s2 * sz);
                            const int p = pidx(kz);
                            const C X = OWN && CP == 0 ? a[r] : lcol[p];
                            const C Y = OWN && CP == 1 ? a[r] : lcol[S + p];
                            const C Z = OWN && CP == 2 ? a[r] : lcol[2 * S + p];
                            a[r] = cadd(cadd(cmul(G0, X), cmul(G1, Y)), cmul(G2, Z));
                        }
                    };
                    if (comp == 0) rows(std::integral_constant<int, 0>{});
                    else if (comp == 1) rows(std::integral_constant<int, 1>{});
                    else rows(std::integral_constant<int, 2>{});
                    dftR<+1, RI>(a);
                };
                switch (Ri) {
                    case 1: mul(std::integral_constant<int, 1>{}); break;
                    case 2: mul(std::integral_constant<int, 2>{}); break;
                    case 3: mul(std::integral_constant<int, 3>{}); break;
                    case 4: mul(std::integral_constant<int, 4>{}); break;
                    case 5: mul(std::integral_constant<int, 5>{}); break;
                    case 6: mul(std::integral_constant<int, 6>{}); break;
                    default: mul(std::integral_constant<int, 8>{}); break;
                }
            }
            __syncthreads();  // every thread has read the three transformed lines
            if (np == 1) {
                if (act && ok) store_rt<kMaxRadixZ>(a, Ri, j, 1, [&](int i, C v) { if (i < nz) st_stream(&line[i], v); });
            } else {
                if (act) store_rt<kMaxRadixZ>(a, Ri, j, 1, [&](int i, C v) { ln[pidx(i)] = v; });
                lds_sync<W>();
                ipasses(1, np - 1);
                for (int jb = j; jb < L / RQ; jb += TPL) {
                    load_rt<+1, kMaxRadixZ>(a, RQ, jb, L, NQ, twp, [&](int i) { return ln[pidx(i)]; });
                    if (ok) store_rt<kMaxRadixZ>(a, RQ, jb, NQ, [&](int i, C v) { if (i < nz) st_stream(&line[i], v); });
                }
            }
            lds_sync<W>();  // the slot's lines are rewritten by the next round
        }
    }
}

// LDS elements of the z-pass block: the tensor column, zmul_slots slots of three lines and,
// for all-radix-8 lengths, the staged twiddle bases
__host__ __device__ constexpr size_t zmul_lds_elems(int Lz) {
    return (size_t)6 * (Lz / 2 + 1) + (size_t)zmul_slots(make_plan(Lz, kMaxRadixZ, false)) * 3 * lds_line_stride(Lz) +
           (all_radix8(Lz, kMaxRadixZ) ? (size_t)Lz / 8 : 0);
}

// ---------------------------------------------------------------- K4: inverse y pass
// Block: component c, column kx, NL consecutive planes z.  Reads B2 along ky (all Ly entries),
// inverse transform, keeps y < ny, writes B1[c][z][kx][y].
template <typename R, int LC>
__global__ void __launch_bounds__(max_threads<R>()) k_inv_y(const cplx<R> *__restrict__ B2, cplx<R> *__restrict__ B1, int ny,
                                                int nz, int Lx, int ncomp, FftPlan pl_rt,
                                                const cplx<R> *__restrict__ twall, int lnl,
                                                const int *__restrict__ done) {
    using C = cplx<R>;
    const FftPlan pl = plan_of<LC, kMaxRadix, true>(pl_rt);
    const int NL = 1 << lnl;
    const int NP = pl.npass, R0 = pl.radix[0], RL = pl.radix[NP - 1], NSL = pl.ns[NP - 1];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const C *tw = twall + pl_rt.tw_off;
    const int L = pl.L, TPL = pl.tpl, S = lds_line_stride(L);
    const int ztiles = (nz + NL - 1) >> lnl;
    int b = xcd_block();
    const int z0 = (b % ztiles) * NL;
    b /= ztiles;
    const int kx = b % Lx;
    const int c = b / Lx;
    if (done && done[c / 3]) return;
    const int t = threadIdx.x;
    const int nzp = row_pitch(nz);
#if DDA_B2_COLMAJOR
    const size_t kystride = (size_t)nzp;
    const C *src = B2 + ((size_t)kx * ncomp + c) * (size_t)L * nzp;
#else
    const size_t kystride = (size_t)Lx * ncomp * nzp;
    const C *src = B2 + ((size_t)kx * ncomp + c) * nzp;
#endif
    {   // pass 0 from global, lanes over lines (z contiguous in B2)
        const int line = t & (NL - 1), j = t >> lnl, z = z0 + line;
        const bool zok = z < nz;
        for (int jb = j; jb < L / R0; jb += TPL) {
            C a[kMaxRadix];
            load_rt<+1, kMaxRadix>(a, R0, jb, L, 1, tw,
                                   [&](int i) -> C { return zok ? ld_stream(&src[(size_t)i * kystride + z]) : czero<C>(); });
            C *ln = lds + line * S;
            store_rt<kMaxRadix>(a, R0, jb, 1, [&](int i, C v) { ln[pidx(i)] = v; });
        }
    }
    __syncthreads();
    lds_passes<+1, kMaxRadix, LC, true>(lds + (t / TPL) * S, pl_rt, 1, NP - 1, t % TPL, tw);
    const int line = t / TPL, j = t % TPL, z = z0 + line;
    C *dst = B1 + (((size_t)c * nz + (z < nz ? z : 0)) * Lx + kx) * row_pitch(ny);
    if (NP >= 2) {
        const int Rp = RL, Ns = NSL;
        for (int jb = j; jb < L / Rp; jb += TPL) {
            C a[kMaxRadix];
            const C *ln = lds + line * S;
            load_rt<+1, kMaxRadix>(a, Rp, jb, L, Ns, tw, [&](int i) { return ln[pidx(i)]; });
            if (z < nz) store_rt<kMaxRadix>(a, Rp, jb, Ns, [&](int i, C v) {
                if (i < ny) st_stream(&dst[i], v);
            });
        }
    } else if (z < nz) {
        for (int i = j; i < ny; i += TPL) dst[i] = lds[line * S + pidx(i)];
    }
}

// ----------------------------------------------- K5: inverse x pass, unpad, y = x - s * conv
// Block: component c, plane z, NL consecutive lines y.  Reads B1 along kx, inverse transform,
// keeps x < nx at non-void cells: y = x - scale[rhs] * v with scale = alpha / (Lx Ly Lz).
// Optionally accumulates the bilinear dot sum x_i y_i of the block into dots[b], b the logical block
// index (right-hand side major, so that each right-hand side owns one contiguous range).
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

// RX: precision of x, y, the scale and the dots (the transform runs in R; with R = float and
// RX = double the epilogue y = x - s v and the dot sums are formed in double)
template <typename R, int LC, typename RX = R>
__global__ void __launch_bounds__(max_threads<R>()) k_inv_x(const int *__restrict__ gmap, const int2 *__restrict__ rows,
                                                size_t gstride, size_t rstride, const cplx<R> *__restrict__ B1,
                                                const cplx<RX> *__restrict__ xin, cplx<RX> *__restrict__ yout,
                                                int nx, int ny, int nz, int N, FftPlan pl_rt,
                                                const cplx<R> *__restrict__ twall, int lnl,
                                                const cplx<RX> *__restrict__ scale, cplx<RX> *__restrict__ dots,
                                                const int *__restrict__ done) {
    using C = cplx<R>;
    using CX = cplx<RX>;
    const FftPlan pl = plan_of<LC, kMaxRadix, true>(pl_rt);
    const int NL = 1 << lnl;
    const int NP = pl.npass, R0 = pl.radix[0], RL = pl.radix[NP - 1], NSL = pl.ns[NP - 1];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const C *tw = twall + pl_rt.tw_off;
    const int L = pl.L, TPL = pl.tpl, S = lds_line_stride(L);
    const int ytiles = (ny + NL - 1) >> lnl;
    const int blk = xcd_block();  // logical block: dot partials are grouped by right-hand side in this order
    int b = blk;
    const int y0 = (b % ytiles) * NL;
    b /= ytiles;
    const int z = b % nz;
    const int c = b / nz;
    if (done && done[c / 3]) return;
    gmap += (size_t)(c / 3) * gstride;
    rows += (size_t)(c / 3) * rstride;
    const int t = threadIdx.x;
    const int nyp = row_pitch(ny);
    const C *src = B1 + ((size_t)c * nz + z) * (size_t)L * nyp;
    {   // pass 0 from global, lanes over lines (y contiguous in B1)
        const int line = t & (NL - 1), j = t >> lnl, y = y0 + line;
        const bool yok = y < ny;
        for (int jb = j; jb < L / R0; jb += TPL) {
            C a[kMaxRadix];
            load_rt<+1, kMaxRadix>(a, R0, jb, L, 1, tw,
                                   [&](int i) -> C { return yok ? ld_stream(&src[(size_t)i * nyp + y]) : czero<C>(); });
            C *ln = lds + line * S;
            store_rt<kMaxRadix>(a, R0, jb, 1, [&](int i, C v) { ln[pidx(i)] = v; });
        }
    }
    __syncthreads();
    lds_passes<+1, kMaxRadix, LC, true>(lds + (t / TPL) * S, pl_rt, 1, NP - 1, t % TPL, tw);
    const int line = t / TPL, j = t % TPL, y = y0 + line;
    const CX sc = scale[c / 3];
    const CX *xc = xin + (size_t)c * N;
    CX *yc = yout + (size_t)c * N;
    const int *grow = gmap + ((size_t)z * ny + (y < ny ? y : 0)) * nx;
    int rx0, rx1, id0;
    const bool run = row_run(rows, z * ny + (y < ny ? y : 0), rx0, rx1, id0);
    CX acc = czero<CX>();
    auto emit = [&](int i, C v) {
        if (y < ny && i < nx) {
            const int id = run ? (i >= rx0 && i < rx1 ? id0 + i - rx0 : -1) : grow[i];
            if (id >= 0) {
                const CX xv = xc[id];
                const CX out = csub(xv, cmul(sc, ccast<CX>(v)));
                st_stream(&yc[id], out);
                acc = cadd(acc, cmul(xv, out));
            }
        }
    };
    if (NP >= 2) {
        const int Rp = RL, Ns = NSL;
        for (int jb = j; jb < L / Rp; jb += TPL) {
            C a[kMaxRadix];
            const C *ln = lds + line * S;
            load_rt<+1, kMaxRadix>(a, Rp, jb, L, Ns, tw, [&](int i) { return ln[pidx(i)]; });
            store_rt<kMaxRadix>(a, Rp, jb, Ns, emit);
        }
    } else {
        for (int i = j; i < nx; i += TPL) emit(i, lds[line * S + pidx(i)]);
    }
    if (dots) {
        CX s = block_sum<RX>(acc, reinterpret_cast<CX *>(lds));  // LDS reused as scratch: all FFT reads are done
        if (t == 0) dots[blk] = s;
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
