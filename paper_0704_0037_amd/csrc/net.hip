// Learned initial guess: a 4-level 3-D convolutional network that maps a particle (mask,
// refractive index, kd, incident field) on a G^3 box to the exciting field's deviation from the
// incident field, and the kernels that train it.  Weights are bfloat16 with fp32 masters,
// activations and stored gradients bfloat16, all products accumulate in fp32 on the matrix cores
// (v_mfma_f32_16x16x32_bf16).
//
// Network (channels-last tensors [batch][z][y][x][c], G a multiple of 8):
//   e0 = relu(conv(f, W0) + b0)            G      16 -> 16
//   e1 = relu(conv(pool(e0), W1) + b1)     G/2    16 -> 32
//   e2 = relu(conv(pool(e1), W2) + b2)     G/4    32 -> 48
//   e3 = relu(conv(pool(e2), W3) + b3)     G/8    48 -> 64
//   d2 = relu(conv(up(e3), W4) + b4 + e2)  G/4    64 -> 48
//   d1 = relu(conv(up(d2), W5) + b5 + e1)  G/2    48 -> 32
//   d0 = relu(conv(up(d1), W6) + b6 + e0)  G      32 -> 16
//   out = conv(d0, W7) + b7                G      16 -> 16(6)
// conv is a 3x3x3 zero-padded cross-correlation, W[t][co][ci] with tap t = 9(dz+1)+3(dy+1)+(dx+1);
// pool is the 2x2x2 mean, up the nearest-neighbour doubling (read through the index map inside
// the convolution, never stored).  Channel counts in parentheses are the real ones; the rest is
// zero padding to multiples of 16.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.hpp"

namespace dda {
void beta_of(const Ctx &c, const dda_beam &bm, double &br, double &bi);
bool beam_ok(const dda_beam *b);
}  // namespace dda

namespace dnet {
using dda::set_error;

typedef uint16_t bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kLayers = 8;
constexpr int kIn = 16, kOut = 6;
// real input / output channels, padded channels, level, input kind (0 plain, 1 pool, 2 up)
struct LayerDef {
    int cin, cout, pcin, pcout, level, kind;
};
constexpr LayerDef kDefs[kLayers] = {
    {kIn, 16, 16, 16, 0, 0}, {16, 32, 16, 32, 1, 1}, {32, 48, 32, 48, 2, 1}, {48, 64, 48, 64, 3, 1},
    {64, 48, 64, 48, 2, 2},  {48, 32, 48, 32, 1, 2}, {32, 16, 32, 16, 0, 2}, {16, kOut, 16, 16, 0, 0},
};

__host__ __device__ inline float bf2f(bf16 h) {
    union {
        uint32_t u;
        float f;
    } v;
    v.u = (uint32_t)h << 16;
    return v.f;
}
__host__ __device__ inline bf16 f2bf(float f) {  // round to nearest even (finite inputs)
    union {
        uint32_t u;
        float f;
    } v;
    v.f = f;
    const uint32_t u = v.u + 0x7FFFu + ((v.u >> 16) & 1u);
    return (bf16)(u >> 16);
}

union Frag {
    uint4 u;
    bf16x8 v;
};

// ------------------------------------------------------------------ convolution (implicit GEMM)
// out[m][n] = sum_{t, c} in[m + off_t][c] W[t][n][c] (+ bias[n] + skip[m][n], relu, x [y > 0]).
// One wave computes 16 voxels x COUT channels: K runs over (tap, channel) in steps of 32, A rows
// are voxels (8 consecutive channels of one shifted voxel per lane), B columns output channels.
// UP: the input lives on the half grid and is read at (z/2, y/2, x/2).
template <int CIN, int COUT, bool UP>
__global__ void __launch_bounds__(256) k_conv(const bf16 *__restrict__ in, const bf16 *__restrict__ W,
                                              const float *__restrict__ bias, const bf16 *__restrict__ skip,
                                              const bf16 *__restrict__ ymask, int relu, bf16 *__restrict__ out16,
                                              float *__restrict__ out32, int out_stride, int out_valid, int g,
                                              int nvox) {
    constexpr int NT = COUT / 16;
    constexpr int KCH = (27 * CIN + 31) / 32;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = (blockIdx.x * 4 + wave) * 16;
    if (m0 >= nvox) return;
    const int ma = m0 + (lane & 15);  // this lane's A row (voxel)
    const int kg = lane >> 4;
    const bool mok = ma < nvox;
    const int g3 = g * g * g;
    const int b = ma / g3, r = ma % g3;
    const int z = r / (g * g), y = (r / g) % g, x = r % g;
    const int gi = UP ? g / 2 : g;
    const size_t in_base = (size_t)b * gi * gi * gi;
    f32x4 acc[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[n] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < KCH; ++kc) {
        const int k0 = kc * 32 + kg * 8;
        const int t = k0 / CIN, c0 = k0 % CIN;
        Frag a;
        a.u = make_uint4(0, 0, 0, 0);
        if (t < 27 && mok) {
            const int zz = z + t / 9 - 1, yy = y + (t / 3) % 3 - 1, xx = x + t % 3 - 1;
            if (zz >= 0 && zz < g && yy >= 0 && yy < g && xx >= 0 && xx < g) {
                const size_t v = UP ? in_base + ((size_t)(zz >> 1) * gi + (yy >> 1)) * gi + (xx >> 1)
                                    : in_base + ((size_t)zz * g + yy) * g + xx;
                a.u = *reinterpret_cast<const uint4 *>(in + v * CIN + c0);
            }
        }
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            Frag w;
            w.u = make_uint4(0, 0, 0, 0);
            if (t < 27) w.u = *reinterpret_cast<const uint4 *>(W + ((size_t)t * COUT + n * 16 + (lane & 15)) * CIN + c0);
            acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, w.v, acc[n], 0, 0, 0);
        }
    }
    // D layout: lane holds rows 4*(lane/16) + i, column lane % 16 of each 16 x 16 tile
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int co = n * 16 + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = m0 + kg * 4 + i;
            if (m >= nvox) continue;
            float v = acc[n][i];
            if (bias) v += bias[co];
            if (skip) v += bf2f(skip[(size_t)m * COUT + co]);
            if (relu) v = fmaxf(v, 0.f);
            if (ymask && !(bf2f(ymask[(size_t)m * COUT + co]) > 0.f)) v = 0.f;
            if (out32) {
                if (co < out_valid) out32[(size_t)m * out_stride + co] = v;
            } else {
                out16[(size_t)m * COUT + co] = f2bf(v);
            }
        }
    }
}

// ------------------------------------------------------------------ weight gradient
// part[blk][t][co][ci] = sum over the block's voxels m of g[m][co] in[m + off_t][ci], tap t =
// blockIdx.y; the voxel range is split in chunks of `chunk`.  Tiles of 32 voxels are staged in LDS
// transposed ([channel][voxel]) so that both MFMA operands read 8 consecutive voxels.  The
// centre-tap blocks also write the bias partials sum g[m][co].
template <int CIN, int COUT, bool UP>
__global__ void __launch_bounds__(256) k_wgrad(const bf16 *__restrict__ gr, const bf16 *__restrict__ in, int g,
                                               int nvox, int chunk, float *__restrict__ part,
                                               float *__restrict__ bpart) {
    constexpr int TM = COUT / 16, TN = CIN / 16, NTILE = TM * TN;
    constexpr int PER = (NTILE + 3) / 4;
    constexpr int SK = 40;  // LDS row stride (elements): 32 voxels + 8 pad, rows 16-byte aligned
    __shared__ __align__(16) bf16 gT[COUT * SK];
    __shared__ __align__(16) bf16 xT[CIN * SK];
    const int t = blockIdx.y;
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int v0 = blockIdx.x * chunk, v1 = min(nvox, v0 + chunk);
    const int g3 = g * g * g, gi = UP ? g / 2 : g;
    f32x4 acc[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) acc[p] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    for (int vs = v0; vs < v1; vs += 32) {
        for (int e = threadIdx.x; e < 32 * (COUT / 8); e += 256) {
            const int vi = e / (COUT / 8), cg = e % (COUT / 8);
            const int m = vs + vi;
            Frag f;
            f.u = make_uint4(0, 0, 0, 0);
            if (m < v1) f.u = *reinterpret_cast<const uint4 *>(gr + (size_t)m * COUT + cg * 8);
            const bf16 *h = reinterpret_cast<const bf16 *>(&f.u);
#pragma unroll
            for (int q = 0; q < 8; ++q) gT[(cg * 8 + q) * SK + vi] = h[q];
        }
        for (int e = threadIdx.x; e < 32 * (CIN / 8); e += 256) {
            const int vi = e / (CIN / 8), cg = e % (CIN / 8);
            const int m = vs + vi;
            Frag f;
            f.u = make_uint4(0, 0, 0, 0);
            if (m < v1) {
                const int b = m / g3, r = m % g3;
                const int zz = r / (g * g) + dz, yy = (r / g) % g + dy, xx = r % g + dx;
                if (zz >= 0 && zz < g && yy >= 0 && yy < g && xx >= 0 && xx < g) {
                    const size_t v = UP ? ((size_t)b * gi * gi * gi + ((size_t)(zz >> 1) * gi + (yy >> 1)) * gi + (xx >> 1))
                                        : ((size_t)b * g3 + ((size_t)zz * g + yy) * g + xx);
                    f.u = *reinterpret_cast<const uint4 *>(in + v * CIN + cg * 8);
                }
            }
            const bf16 *h = reinterpret_cast<const bf16 *>(&f.u);
#pragma unroll
            for (int q = 0; q < 8; ++q) xT[(cg * 8 + q) * SK + vi] = h[q];
        }
        __syncthreads();
        if (t == 13 && threadIdx.x < COUT)
            for (int vi = 0; vi < 32; ++vi) bsum += bf2f(gT[threadIdx.x * SK + vi]);
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int tile = wave + 4 * p;
            if (tile < NTILE) {
                const int tm = tile / TN, tn = tile % TN;
                Frag a, b;
                a.u = *reinterpret_cast<const uint4 *>(&gT[(tm * 16 + (lane & 15)) * SK + (lane >> 4) * 8]);
                b.u = *reinterpret_cast<const uint4 *>(&xT[(tn * 16 + (lane & 15)) * SK + (lane >> 4) * 8]);
                acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc[p], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    float *dst = part + ((size_t)blockIdx.x * 27 + t) * COUT * CIN;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int tile = wave + 4 * p;
        if (tile < NTILE) {
            const int tm = tile / TN, tn = tile % TN;
            const int ci = tn * 16 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) dst[(size_t)(tm * 16 + (lane >> 4) * 4 + i) * CIN + ci] = acc[p][i];
        }
    }
    if (t == 13 && threadIdx.x < COUT) bpart[(size_t)blockIdx.x * COUT + threadIdx.x] = bsum;
}

// canonical gradient of one layer = the sum of the block partials (fixed order), real channels only
__global__ void k_wgrad_reduce(const float *__restrict__ part, const float *__restrict__ bpart, int nblk, int pco,
                               int pci, int co_r, int ci_r, float *__restrict__ gw, float *__restrict__ gb) {
    const int nw = 27 * co_r * ci_r;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nw) {
        const int t = e / (co_r * ci_r), co = (e / ci_r) % co_r, ci = e % ci_r;
        const size_t src = ((size_t)t * pco + co) * pci + ci, stride = (size_t)27 * pco * pci;
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += part[b * stride + src];
        gw[e] = s;
    } else if (e < nw + co_r) {
        const int co = e - nw;
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += bpart[(size_t)b * pco + co];
        gb[co] = s;
    }
}

// ------------------------------------------------------------------ pooling and its adjoints
__global__ void k_pool(const bf16 *__restrict__ in, bf16 *__restrict__ out, int go, int C, int nvo) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nvo * C) return;
    const int c = e % C, m = e / C;
    const int g3 = go * go * go, b = m / g3, r = m % g3;
    const int z = r / (go * go), y = (r / go) % go, x = r % go;
    const int gi = 2 * go;
    float s = 0.f;
    for (int q = 0; q < 8; ++q) {
        const size_t v = (size_t)b * gi * gi * gi + ((size_t)(2 * z + (q >> 2)) * gi + 2 * y + ((q >> 1) & 1)) * gi +
                         2 * x + (q & 1);
        s += bf2f(in[v * C + c]);
    }
    out[e] = f2bf(s * 0.125f);
}

// g[parent] = (sum of the 8 children of gf) x [y > 0]  (adjoint of up, then relu mask)
__global__ void k_up_adj_mask(const bf16 *__restrict__ gf, const bf16 *__restrict__ y, bf16 *__restrict__ g, int gc,
                              int C, int nvc) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nvc * C) return;
    const int c = e % C, m = e / C;
    const int g3 = gc * gc * gc, b = m / g3, r = m % g3;
    const int z = r / (gc * gc), yy = (r / gc) % gc, x = r % gc;
    const int gf3 = 8 * g3, gfs = 2 * gc;
    float s = 0.f;
    for (int q = 0; q < 8; ++q) {
        const size_t v = (size_t)b * gf3 + ((size_t)(2 * z + (q >> 2)) * gfs + 2 * yy + ((q >> 1) & 1)) * gfs + 2 * x + (q & 1);
        s += bf2f(gf[v * C + c]);
    }
    const bf16 h = f2bf(s);
    g[e] = bf2f(y[e]) > 0.f ? h : (bf16)0;
}

// g[child] = (gskip[child] + gp[parent] / 8) x [y > 0]  (adjoint of pool plus the skip path)
__global__ void k_pool_adj_add_mask(const bf16 *__restrict__ gp, const bf16 *__restrict__ gskip,
                                    const bf16 *__restrict__ y, bf16 *__restrict__ g, int gf, int C, int nvf) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nvf * C) return;
    const int c = e % C, m = e / C;
    const int g3 = gf * gf * gf, b = m / g3, r = m % g3;
    const int z = r / (gf * gf), yy = (r / gf) % gf, x = r % gf;
    const int gc = gf / 2;
    const size_t par = (size_t)b * gc * gc * gc + ((size_t)(z >> 1) * gc + (yy >> 1)) * gc + (x >> 1);
    const float s = bf2f(gskip[e]) + 0.125f * bf2f(gp[par * C + c]);
    const bf16 h = f2bf(s);
    g[e] = bf2f(y[e]) > 0.f ? h : (bf16)0;
}

// ------------------------------------------------------------------ loss
constexpr int kLossThreads = 256;

// per block: sum over masked voxels of sum_c (out - tgt)^2, and the number of masked voxels
__global__ void __launch_bounds__(kLossThreads) k_loss_part(const float *__restrict__ out, const float *__restrict__ tgt,
                                                            const bf16 *__restrict__ feat, int nvox,
                                                            double *__restrict__ part) {
    __shared__ double s0[kLossThreads], s1[kLossThreads];
    double a = 0, n = 0;
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < nvox; m += gridDim.x * blockDim.x) {
        if (bf2f(feat[(size_t)m * 16]) > 0.f) {
            n += 1;
            for (int c = 0; c < kOut; ++c) {
                const double d = (double)out[(size_t)m * kOut + c] - (double)tgt[(size_t)m * kOut + c];
                a += d * d;
            }
        }
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = n;
    __syncthreads();
    for (int h = kLossThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            s0[threadIdx.x] += s0[threadIdx.x + h];
            s1[threadIdx.x] += s1[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

__global__ void k_loss_fin(const double *__restrict__ part, int nb, double *__restrict__ res) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0, n = 0;
    for (int b = 0; b < nb; ++b) {
        a += part[2 * b];
        n += part[2 * b + 1];
    }
    res[0] = n > 0 ? a / n : 0.0;
    res[1] = n;
}

// gradient of the loss w.r.t. the output, bf16 [nvox][16] (padded channels zero)
__global__ void k_out_grad(const float *__restrict__ out, const float *__restrict__ tgt, const bf16 *__restrict__ feat,
                           int nvox, const double *__restrict__ res, bf16 *__restrict__ g) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nvox * 16) return;
    const int m = e / 16, c = e % 16;
    float v = 0.f;
    if (c < kOut && bf2f(feat[(size_t)m * 16]) > 0.f && res[1] > 0)
        v = (float)(2.0 * ((double)out[(size_t)m * kOut + c] - (double)tgt[(size_t)m * kOut + c]) / res[1]);
    g[e] = f2bf(v);
}

// ------------------------------------------------------------------ optimizer and weight copies
__global__ void k_adam(float *__restrict__ p, float *__restrict__ m1, float *__restrict__ m2,
                       const float *__restrict__ g, int n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    p[i] -= lr * (a / bc1) / (sqrtf(b / bc2) + eps);
}

// padded bf16 copies of one layer: W[t][co][ci], the flipped transpose WT[t][ci][co] = W[26-t][co][ci]
// (the backward-data convolution), and the padded fp32 bias
__global__ void k_refresh(const float *__restrict__ pw, const float *__restrict__ pb, int co_r, int ci_r, int pco,
                          int pci, bf16 *__restrict__ W, bf16 *__restrict__ WT, float *__restrict__ bias) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < 27 * pco * pci) {
        const int t = e / (pco * pci), co = (e / pci) % pco, ci = e % pci;
        const float v = (co < co_r && ci < ci_r) ? pw[((size_t)t * co_r + co) * ci_r + ci] : 0.f;
        const bf16 h = f2bf(v);
        W[e] = h;
        WT[((size_t)(26 - t) * pci + ci) * pco + co] = h;
    }
    if (e < pco) bias[e] = e < co_r ? pb[e] : 0.f;
}

// ------------------------------------------------------------------ DDA <-> network grid
struct BeamArgs {
    double a[3], er[3], ei[3], br, bi;
};

__device__ inline void box_cell(int v, int G, int &X, int &Y, int &Z) {
    X = v % G;
    Y = (v / G) % G;
    Z = v / (G * G);
}

// features of one particle: 0 mask, 1 (Re m - 1) mask, 2 Im m mask, 3 kd, 4..9 Re/Im E_inc(x, y, z),
// 10..15 Re/Im (m^2 - 1) E_inc mask
__global__ void k_features(const int *__restrict__ gmap, int nx, int ny, int nz, int G, double mre, double mim,
                           double kd, BeamArgs bm, bf16 *__restrict__ f) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= G * G * G) return;
    int X, Y, Z;
    box_cell(v, G, X, Y, Z);
    const int ox = (G - nx) / 2, oy = (G - ny) / 2, oz = (G - nz) / 2;
    const int x = X - ox, y = Y - oy, z = Z - oz;
    const bool in = x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz &&
                    gmap[((size_t)z * ny + y) * nx + x] >= 0;
    const double rx = x + 0.5 - 0.5 * nx, ry = y + 0.5 - 0.5 * ny, rz = z + 0.5 - 0.5 * nz;
    double sn, cs;
    sincos(kd * (bm.a[0] * rx + bm.a[1] * ry + bm.a[2] * rz), &sn, &cs);
    bf16 *o = f + (size_t)v * 16;
    const float mk = in ? 1.f : 0.f;
    o[0] = f2bf(mk);
    o[1] = f2bf((float)((mre - 1.0) * mk));
    o[2] = f2bf((float)(mim * mk));
    o[3] = f2bf((float)kd);
    const double qr = mre * mre - mim * mim - 1.0, qi = 2.0 * mre * mim;  // m^2 - 1
    for (int c = 0; c < 3; ++c) {
        const double er = bm.er[c] * cs - bm.ei[c] * sn, ei = bm.er[c] * sn + bm.ei[c] * cs;
        o[4 + 2 * c] = f2bf((float)er);
        o[5 + 2 * c] = f2bf((float)ei);
        o[10 + 2 * c] = f2bf((float)((qr * er - qi * ei) * mk));
        o[11 + 2 * c] = f2bf((float)((qr * ei + qi * er) * mk));
    }
}

__global__ void k_zero_f32(float *__restrict__ p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.f;
}

// target at the dipoles: Re/Im of x / beta - E_inc
__global__ void k_target(const int *__restrict__ lin, int N, int nx, int ny, int nz, int G, double kd, BeamArgs bm,
                         const double2 *__restrict__ x, float *__restrict__ tgt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int l = lin[j];
    const int cx = l % nx, cy = (l / nx) % ny, cz = l / (nx * ny);
    const double rx = cx + 0.5 - 0.5 * nx, ry = cy + 0.5 - 0.5 * ny, rz = cz + 0.5 - 0.5 * nz;
    double sn, cs;
    sincos(kd * (bm.a[0] * rx + bm.a[1] * ry + bm.a[2] * rz), &sn, &cs);
    const int v = ((cz + (G - nz) / 2) * G + cy + (G - ny) / 2) * G + cx + (G - nx) / 2;
    const double den = bm.br * bm.br + bm.bi * bm.bi;
    for (int c = 0; c < 3; ++c) {
        const double2 xv = x[(size_t)c * N + j];
        const double qr = (xv.x * bm.br + xv.y * bm.bi) / den, qi = (xv.y * bm.br - xv.x * bm.bi) / den;  // x / beta
        tgt[(size_t)v * kOut + 2 * c] = (float)(qr - (bm.er[c] * cs - bm.ei[c] * sn));
        tgt[(size_t)v * kOut + 2 * c + 1] = (float)(qi - (bm.er[c] * sn + bm.ei[c] * cs));
    }
}

// x0 = beta (E_inc + delta) at the dipoles
__global__ void k_guess(const int *__restrict__ lin, int N, int nx, int ny, int nz, int G, double kd, BeamArgs bm,
                        const float *__restrict__ out, double2 *__restrict__ x0) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int l = lin[j];
    const int cx = l % nx, cy = (l / nx) % ny, cz = l / (nx * ny);
    const double rx = cx + 0.5 - 0.5 * nx, ry = cy + 0.5 - 0.5 * ny, rz = cz + 0.5 - 0.5 * nz;
    double sn, cs;
    sincos(kd * (bm.a[0] * rx + bm.a[1] * ry + bm.a[2] * rz), &sn, &cs);
    const int v = ((cz + (G - nz) / 2) * G + cy + (G - ny) / 2) * G + cx + (G - nx) / 2;
    for (int c = 0; c < 3; ++c) {
        const double er = bm.er[c] * cs - bm.ei[c] * sn + out[(size_t)v * kOut + 2 * c];
        const double ei = bm.er[c] * sn + bm.ei[c] * cs + out[(size_t)v * kOut + 2 * c + 1];
        x0[(size_t)c * N + j] = make_double2(bm.br * er - bm.bi * ei, bm.br * ei + bm.bi * er);
    }
}

// ------------------------------------------------------------------ the network object
struct Net {
    int G = 0, maxb = 0;
    hipStream_t stream = nullptr;
    int64_t nparams = 0;
    int64_t off_w[kLayers], off_b[kLayers];
    float *params = nullptr, *m1 = nullptr, *m2 = nullptr, *grad = nullptr;
    bf16 *W[kLayers], *WT[kLayers];
    float *bias[kLayers];
    int64_t step = 0;
    // activations (bf16) and backward tensors
    bf16 *e[4] = {}, *p[3] = {}, *d[3] = {};  // d[0] = d0, d[1] = d1, d[2] = d2
    float *out = nullptr;
    bf16 *gout = nullptr, *gl[8] = {}, *gtmp = nullptr;
    float *part = nullptr, *bpart = nullptr;
    size_t part_elems = 0, bpart_elems = 0;
    double *lpart = nullptr, *lres = nullptr, *lhost = nullptr;
    std::vector<void *> allocs;
};

constexpr int kLossBlocks = 256;

static int side(const Net &n, int level) { return n.G >> level; }
static size_t vox(const Net &n, int level, int batch) {
    const size_t g = (size_t)side(n, level);
    return (size_t)batch * g * g * g;
}

static dda_status dalloc(Net &n, void **p, size_t bytes) {
    dda_status st = dda::device_alloc(p, bytes);
    if (st == DDA_OK) n.allocs.push_back(*p);
    return st;
}

static void destroy(Net *n) {
    if (!n) return;
    for (void *p : n->allocs) (void)hipFree(p);
    if (n->lhost) (void)hipHostFree(n->lhost);
    delete n;
}

static int chunk_of(size_t nvox) {
    size_t c = (nvox + 127) / 128;
    c = (c + 31) / 32 * 32;
    return (int)std::max<size_t>(c, 32);
}

#define DNET_CHECK(x)                                                          \
    do {                                                                       \
        hipError_t e_ = (x);                                                   \
        if (e_ != hipSuccess) {                                                \
            set_error(std::string("dda_net: ") + hipGetErrorString(e_));       \
            return DDA_EHIP;                                                   \
        }                                                                      \
    } while (0)

static dda_status refresh(Net &n) {
    for (int l = 0; l < kLayers; ++l) {
        const LayerDef &d = kDefs[l];
        const int tot = 27 * d.pcout * d.pcin;
        hipLaunchKernelGGL(k_refresh, dim3((tot + 255) / 256), dim3(256), 0, n.stream, n.params + n.off_w[l],
                           n.params + n.off_b[l], d.cout, d.cin, d.pcout, d.pcin, n.W[l], n.WT[l], n.bias[l]);
    }
    DNET_CHECK(hipGetLastError());
    return DDA_OK;
}

// one convolution launch; (cin, cout, up) picks the instantiation
static dda_status conv(Net &n, int cin, int cout, bool upm, const bf16 *in, const bf16 *W, const float *bias,
                       const bf16 *skip, const bf16 *ymask, int relu, bf16 *o16, float *o32, int ostride, int ovalid,
                       int g, size_t nv) {
    const dim3 grid((unsigned)((nv + 63) / 64)), blk(256);
    hipStream_t s = n.stream;
    const int nvi = (int)nv;
#define DNET_CONV(CI, CO, UPM)                                                                                  \
    if (cin == CI && cout == CO && upm == UPM) {                                                                \
        hipLaunchKernelGGL((k_conv<CI, CO, UPM>), grid, blk, 0, s, in, W, bias, skip, ymask, relu, o16, o32,    \
                           ostride, ovalid, g, nvi);                                                            \
        DNET_CHECK(hipGetLastError());                                                                          \
        return DDA_OK;                                                                                          \
    }
    DNET_CONV(16, 16, false)
    DNET_CONV(16, 32, false)
    DNET_CONV(32, 48, false)
    DNET_CONV(48, 64, false)
    DNET_CONV(64, 48, true)
    DNET_CONV(48, 32, true)
    DNET_CONV(32, 16, true)
    DNET_CONV(32, 16, false)
    DNET_CONV(48, 32, false)
    DNET_CONV(64, 48, false)
#undef DNET_CONV
    set_error("dda_net: no convolution instantiated for these channels");
    return DDA_ENOTSUP;
}

static dda_status wgrad(Net &n, int l, const bf16 *g, const bf16 *in, int gside, size_t nv) {
    const LayerDef &d = kDefs[l];
    const int chunk = chunk_of(nv);
    const int nblk = (int)((nv + chunk - 1) / chunk);
    if ((size_t)nblk * 27 * d.pcout * d.pcin > n.part_elems || (size_t)nblk * d.pcout > n.bpart_elems) {
        set_error("dda_net: gradient partial buffer too small");
        return DDA_EINVAL;
    }
    const dim3 grid(nblk, 27), blk(256);
    hipStream_t s = n.stream;
    const int nvi = (int)nv;
    bool done = false;
#define DNET_WG(CI, CO, UPM)                                                                                     \
    if (!done && d.pcin == CI && d.pcout == CO && (d.kind == 2) == UPM) {                                        \
        hipLaunchKernelGGL((k_wgrad<CI, CO, UPM>), grid, blk, 0, s, g, in, gside, nvi, chunk, n.part, n.bpart); \
        done = true;                                                                                             \
    }
    DNET_WG(16, 16, false)
    DNET_WG(16, 32, false)
    DNET_WG(32, 48, false)
    DNET_WG(48, 64, false)
    DNET_WG(64, 48, true)
    DNET_WG(48, 32, true)
    DNET_WG(32, 16, true)
#undef DNET_WG
    if (!done) {
        set_error("dda_net: no weight-gradient kernel for this layer");
        return DDA_ENOTSUP;
    }
    const int tot = 27 * d.cout * d.cin + d.cout;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((tot + 255) / 256), dim3(256), 0, s, n.part, n.bpart, nblk, d.pcout,
                       d.pcin, d.cout, d.cin, n.grad + n.off_w[l], n.grad + n.off_b[l]);
    DNET_CHECK(hipGetLastError());
    return DDA_OK;
}

static dda_status forward(Net &n, const bf16 *feat, int B) {
    dda_status st;
    const int G = n.G;
    // encoder
    if ((st = conv(n, 16, 16, false, feat, n.W[0], n.bias[0], nullptr, nullptr, 1, n.e[0], nullptr, 0, 0, G,
                   vox(n, 0, B))) != DDA_OK)
        return st;
    for (int l = 1; l <= 3; ++l) {
        const LayerDef &d = kDefs[l];
        const size_t nv = vox(n, l, B);
        hipLaunchKernelGGL(k_pool, dim3((unsigned)((nv * d.pcin + 255) / 256)), dim3(256), 0, n.stream, n.e[l - 1],
                           n.p[l - 1], side(n, l), d.pcin, (int)nv);
        if ((st = conv(n, d.pcin, d.pcout, false, n.p[l - 1], n.W[l], n.bias[l], nullptr, nullptr, 1, n.e[l], nullptr,
                       0, 0, side(n, l), nv)) != DDA_OK)
            return st;
    }
    // decoder: d2 (level 2) from e3, d1 from d2, d0 from d1
    const bf16 *src = n.e[3];
    for (int l = 4; l <= 6; ++l) {
        const LayerDef &d = kDefs[l];
        const int lev = d.level;
        if ((st = conv(n, d.pcin, d.pcout, true, src, n.W[l], n.bias[l], n.e[lev], nullptr, 1, n.d[lev], nullptr, 0, 0,
                       side(n, lev), vox(n, lev, B))) != DDA_OK)
            return st;
        src = n.d[lev];
    }
    return conv(n, 16, 16, false, n.d[0], n.W[7], n.bias[7], nullptr, nullptr, 0, nullptr, n.out, kOut, kOut, G,
                vox(n, 0, B));
}

// loss, then gradients of every layer into n.grad (canonical layout)
static dda_status backward(Net &n, const bf16 *feat, const float *tgt, int B) {
    dda_status st;
    hipStream_t s = n.stream;
    const int G = n.G;
    const size_t nv0 = vox(n, 0, B);
    hipLaunchKernelGGL(k_loss_part, dim3(kLossBlocks), dim3(kLossThreads), 0, s, n.out, tgt, feat, (int)nv0, n.lpart);
    hipLaunchKernelGGL(k_loss_fin, dim3(1), dim3(64), 0, s, n.lpart, kLossBlocks, n.lres);
    hipLaunchKernelGGL(k_out_grad, dim3((unsigned)((nv0 * 16 + 255) / 256)), dim3(256), 0, s, n.out, tgt, feat,
                       (int)nv0, n.lres, n.gout);
    DNET_CHECK(hipGetLastError());
    // gl[l]: gradient at the pre-activation of layer l (relu mask applied)
    // layer 7 (head): input d0
    if ((st = wgrad(n, 7, n.gout, n.d[0], G, nv0)) != DDA_OK) return st;
    if ((st = conv(n, 16, 16, false, n.gout, n.WT[7], nullptr, nullptr, n.d[0], 0, n.gl[6], nullptr, 0, 0, G, nv0)) !=
        DDA_OK)
        return st;
    // decoder layers 6, 5, 4: input up(d1), up(d2), up(e3)
    const bf16 *dec_in[7] = {nullptr, nullptr, nullptr, nullptr, n.e[3], n.d[2], n.d[1]};
    for (int l = 6; l >= 4; --l) {
        const LayerDef &d = kDefs[l];
        const int lev = d.level;
        const size_t nv = vox(n, lev, B), nvc = vox(n, lev + 1, B);
        if ((st = wgrad(n, l, n.gl[l], dec_in[l], side(n, lev), nv)) != DDA_OK) return st;
        // input gradient on this level's grid (channels pcin), then the adjoint of up onto the coarse grid
        if ((st = conv(n, d.pcout, d.pcin, false, n.gl[l], n.WT[l], nullptr, nullptr, nullptr, 0, n.gtmp, nullptr, 0,
                       0, side(n, lev), nv)) != DDA_OK)
            return st;
        const bf16 *ycoarse = l == 4 ? n.e[3] : n.d[lev + 1];
        hipLaunchKernelGGL(k_up_adj_mask, dim3((unsigned)((nvc * d.pcin + 255) / 256)), dim3(256), 0, s, n.gtmp,
                           ycoarse, n.gl[l - 1], side(n, lev + 1), d.pcin, (int)nvc);
    }
    // encoder layers 3, 2, 1: input pool(e2), pool(e1), pool(e0); e_l also feeds the skip of layer 6 - l... (l-1 level)
    for (int l = 3; l >= 1; --l) {
        const LayerDef &d = kDefs[l];
        const int lev = d.level;
        const size_t nv = vox(n, lev, B), nvf = vox(n, lev - 1, B);
        if ((st = wgrad(n, l, n.gl[l], n.p[l - 1], side(n, lev), nv)) != DDA_OK) return st;
        if ((st = conv(n, d.pcout, d.pcin, false, n.gl[l], n.WT[l], nullptr, nullptr, nullptr, 0, n.gtmp, nullptr, 0,
                       0, side(n, lev), nv)) != DDA_OK)
            return st;
        // e_{lev-1} is the skip input of the decoder layer on level lev-1: layer 7 - lev
        const bf16 *gskip = n.gl[7 - lev];
        hipLaunchKernelGGL(k_pool_adj_add_mask, dim3((unsigned)((nvf * d.pcin + 255) / 256)), dim3(256), 0, s, n.gtmp,
                           gskip, n.e[lev - 1], n.gl[l - 1], side(n, lev - 1), d.pcin, (int)nvf);
    }
    if ((st = wgrad(n, 0, n.gl[0], feat, G, nv0)) != DDA_OK) return st;
    DNET_CHECK(hipGetLastError());
    return DDA_OK;
}

}  // namespace dnet

using namespace dnet;

static dnet::Net *nx_(dda_net *h) { return reinterpret_cast<dnet::Net *>(h); }

extern "C" {

int64_t dda_net_num_params(void) {
    int64_t n = 0;
    for (int l = 0; l < kLayers; ++l) n += 27 * kDefs[l].cin * kDefs[l].cout + kDefs[l].cout;
    return n;
}

dda_status dda_net_create(dda_net **out, int32_t grid, int32_t max_batch, const float *params, void *stream) {
    dda::clear_error();
    if (!out || !params || grid < 8 || grid % 8 || max_batch < 1 || grid > 256 ||
        (int64_t)max_batch * grid * grid * grid * 64 > (int64_t)1 << 31) {
        set_error("dda_net_create: NULL argument, grid not a multiple of 8 in [8, 256], or batch too large");
        return DDA_EINVAL;
    }
    *out = nullptr;
    Net *n = new Net();
    n->G = grid;
    n->maxb = max_batch;
    n->stream = (hipStream_t)stream;
    int64_t o = 0;
    for (int l = 0; l < kLayers; ++l) {
        n->off_w[l] = o;
        o += 27 * kDefs[l].cin * kDefs[l].cout;
        n->off_b[l] = o;
        o += kDefs[l].cout;
    }
    n->nparams = o;
    dda_status st = DDA_OK;
    auto A = [&](void **p, size_t bytes) {
        if (st == DDA_OK) st = dalloc(*n, p, bytes);
    };
    const size_t P = (size_t)o * sizeof(float);
    A((void **)&n->params, P);
    A((void **)&n->m1, P);
    A((void **)&n->m2, P);
    A((void **)&n->grad, P);
    for (int l = 0; l < kLayers; ++l) {
        const size_t w = (size_t)27 * kDefs[l].pcin * kDefs[l].pcout * sizeof(bf16);
        A((void **)&n->W[l], w);
        A((void **)&n->WT[l], w);
        A((void **)&n->bias[l], kDefs[l].pcout * sizeof(float));
    }
    const int B = max_batch;
    A((void **)&n->e[0], vox(*n, 0, B) * 16 * sizeof(bf16));
    A((void **)&n->e[1], vox(*n, 1, B) * 32 * sizeof(bf16));
    A((void **)&n->e[2], vox(*n, 2, B) * 48 * sizeof(bf16));
    A((void **)&n->e[3], vox(*n, 3, B) * 64 * sizeof(bf16));
    A((void **)&n->p[0], vox(*n, 1, B) * 16 * sizeof(bf16));
    A((void **)&n->p[1], vox(*n, 2, B) * 32 * sizeof(bf16));
    A((void **)&n->p[2], vox(*n, 3, B) * 48 * sizeof(bf16));
    A((void **)&n->d[0], vox(*n, 0, B) * 16 * sizeof(bf16));
    A((void **)&n->d[1], vox(*n, 1, B) * 32 * sizeof(bf16));
    A((void **)&n->d[2], vox(*n, 2, B) * 48 * sizeof(bf16));
    A((void **)&n->out, vox(*n, 0, B) * kOut * sizeof(float));
    A((void **)&n->gout, vox(*n, 0, B) * 16 * sizeof(bf16));
    for (int l = 0; l < kLayers - 1; ++l)
        A((void **)&n->gl[l], vox(*n, kDefs[l].level, B) * kDefs[l].pcout * sizeof(bf16));
    // largest input-gradient tensor: level-l grid with that layer's input channels
    size_t gt = 0, pe = 0, be = 0;
    for (int l = 0; l < kLayers; ++l) {
        const size_t nv = vox(*n, kDefs[l].level, B);
        gt = std::max(gt, nv * kDefs[l].pcin);
        const size_t nblk = (nv + chunk_of(nv) - 1) / chunk_of(nv);
        pe = std::max(pe, nblk * 27 * kDefs[l].pcin * kDefs[l].pcout);
        be = std::max(be, nblk * kDefs[l].pcout);
    }
    A((void **)&n->gtmp, gt * sizeof(bf16));
    A((void **)&n->part, pe * sizeof(float));
    A((void **)&n->bpart, be * sizeof(float));
    n->part_elems = pe;
    n->bpart_elems = be;
    A((void **)&n->lpart, 2 * kLossBlocks * sizeof(double));
    A((void **)&n->lres, 2 * sizeof(double));
    if (st == DDA_OK && hipHostMalloc((void **)&n->lhost, 2 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        n->lhost = nullptr;
        set_error("dda_net_create: pinned host allocation failed");
        st = DDA_ENOMEM;
    }
    if (st == DDA_OK) st = dda_net_set_params(reinterpret_cast<dda_net *>(n), params);
    if (st != DDA_OK) {
        destroy(n);
        return st;
    }
    *out = reinterpret_cast<dda_net *>(n);
    return DDA_OK;
}

dda_status dda_net_free(dda_net *h) {
    dda::clear_error();
    Net *n = nx_(h);
    if (!n) return DDA_OK;
    (void)hipStreamSynchronize(n->stream);
    destroy(n);
    return DDA_OK;
}

dda_status dda_net_set_params(dda_net *h, const float *params) {
    dda::clear_error();
    Net *n = nx_(h);
    if (!n || !params) {
        set_error("dda_net_set_params: NULL argument");
        return DDA_EINVAL;
    }
    const size_t P = (size_t)n->nparams * sizeof(float);
    DNET_CHECK(hipMemcpyAsync(n->params, params, P, hipMemcpyHostToDevice, n->stream));
    hipLaunchKernelGGL(k_zero_f32, dim3(256), dim3(256), 0, n->stream, n->m1, (size_t)n->nparams);
    hipLaunchKernelGGL(k_zero_f32, dim3(256), dim3(256), 0, n->stream, n->m2, (size_t)n->nparams);
    n->step = 0;
    dda_status st = refresh(*n);
    if (st != DDA_OK) return st;
    DNET_CHECK(hipStreamSynchronize(n->stream));
    return DDA_OK;
}

dda_status dda_net_get_params(dda_net *h, float *params) {
    dda::clear_error();
    Net *n = nx_(h);
    if (!n || !params) {
        set_error("dda_net_get_params: NULL argument");
        return DDA_EINVAL;
    }
    DNET_CHECK(hipMemcpyAsync(params, n->params, (size_t)n->nparams * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    DNET_CHECK(hipStreamSynchronize(n->stream));
    return DDA_OK;
}

static BeamArgs beam_args(const dda_beam &b, double br, double bi) {
    BeamArgs a;
    for (int i = 0; i < 3; ++i) {
        a.a[i] = b.prop[i];
        a.er[i] = b.pol_re[i];
        a.ei[i] = b.pol_im[i];
    }
    a.br = br;
    a.bi = bi;
    return a;
}

static bool fits(const Net &n, const dda::Ctx &c) { return c.nx <= n.G && c.ny <= n.G && c.nz <= n.G; }

dda_status dda_net_features(dda_net *h, dda_ctx *ch, const dda_beam *beam, void *feat) {
    dda::clear_error();
    Net *n = nx_(h);
    dda::Ctx *c = dda::cx(ch);
    if (!n || !c || !feat || !dda::beam_ok(beam) || beam->w0 > 0 || dda::wrapped(*c) || !fits(*n, *c)) {
        set_error("dda_net_features: NULL argument, bad or focused beam (plane waves only), inhomogeneous particle, "
                  "or particle grid larger than the network's");
        return DDA_EINVAL;
    }
    const int G = n->G, nv = G * G * G;
    hipLaunchKernelGGL(k_features, dim3((nv + 255) / 256), dim3(256), 0, n->stream, c->gmap, c->nx, c->ny, c->nz, G,
                       c->m_re, c->m_im, c->kd, beam_args(*beam, 0, 0), (bf16 *)feat);
    DNET_CHECK(hipGetLastError());
    return DDA_OK;
}

dda_status dda_net_target(dda_net *h, dda_ctx *ch, const dda_beam *beam, const void *x, void *tgt) {
    dda::clear_error();
    Net *n = nx_(h);
    dda::Ctx *c = dda::cx(ch);
    if (!n || !c || !x || !tgt || !dda::beam_ok(beam) || beam->w0 > 0 || dda::wrapped(*c) || !fits(*n, *c)) {
        set_error("dda_net_target: NULL argument, bad or focused beam (plane waves only), inhomogeneous particle, "
                  "or particle grid larger than the network's");
        return DDA_EINVAL;
    }
    double br, bi;
    dda::beta_of(*c, *beam, br, bi);
    const int G = n->G;
    hipLaunchKernelGGL(k_zero_f32, dim3(256), dim3(256), 0, n->stream, (float *)tgt, (size_t)G * G * G * kOut);
    const int N = (int)c->N;
    hipLaunchKernelGGL(k_target, dim3((N + 255) / 256), dim3(256), 0, n->stream, c->lin, N, c->nx, c->ny, c->nz, G,
                       c->kd, beam_args(*beam, br, bi), (const double2 *)x, (float *)tgt);
    DNET_CHECK(hipGetLastError());
    return DDA_OK;
}

dda_status dda_net_forward(dda_net *h, const void *feat, int32_t batch, void *out) {
    dda::clear_error();
    Net *n = nx_(h);
    if (!n || !feat || !out || batch < 1 || batch > n->maxb) {
        set_error("dda_net_forward: NULL argument or batch outside [1, max_batch]");
        return DDA_EINVAL;
    }
    dda_status st = forward(*n, (const bf16 *)feat, batch);
    if (st != DDA_OK) return st;
    DNET_CHECK(hipMemcpyAsync(out, n->out, vox(*n, 0, batch) * kOut * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    return DDA_OK;
}

static dda_status loss_grad(Net &n, const void *feat, const void *tgt, int batch, double *loss) {
    dda_status st = forward(n, (const bf16 *)feat, batch);
    if (st != DDA_OK) return st;
    if ((st = backward(n, (const bf16 *)feat, (const float *)tgt, batch)) != DDA_OK) return st;
    DNET_CHECK(hipMemcpyAsync(n.lhost, n.lres, 2 * sizeof(double), hipMemcpyDeviceToHost, n.stream));
    DNET_CHECK(hipStreamSynchronize(n.stream));
    if (loss) *loss = n.lhost[0];
    return DDA_OK;
}

dda_status dda_net_grad(dda_net *h, const void *feat, const void *tgt, int32_t batch, double *loss, float *grad) {
    dda::clear_error();
    Net *n = nx_(h);
    if (!n || !feat || !tgt || batch < 1 || batch > n->maxb) {
        set_error("dda_net_grad: NULL argument or batch outside [1, max_batch]");
        return DDA_EINVAL;
    }
    dda_status st = loss_grad(*n, feat, tgt, batch, loss);
    if (st != DDA_OK) return st;
    if (grad) {
        DNET_CHECK(hipMemcpyAsync(grad, n->grad, (size_t)n->nparams * sizeof(float), hipMemcpyDeviceToHost, n->stream));
        DNET_CHECK(hipStreamSynchronize(n->stream));
    }
    return DDA_OK;
}

dda_status dda_net_train_step(dda_net *h, const void *feat, const void *tgt, int32_t batch, double lr, double *loss) {
    dda::clear_error();
    Net *n = nx_(h);
    if (!n || !feat || !tgt || batch < 1 || batch > n->maxb || !(lr > 0)) {
        set_error("dda_net_train_step: NULL argument, batch outside [1, max_batch] or lr <= 0");
        return DDA_EINVAL;
    }
    dda_status st = loss_grad(*n, feat, tgt, batch, loss);
    if (st != DDA_OK) return st;
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = 1.f - std::pow(b1, (float)n->step), bc2 = 1.f - std::pow(b2, (float)n->step);
    const int P = (int)n->nparams;
    hipLaunchKernelGGL(k_adam, dim3((P + 255) / 256), dim3(256), 0, n->stream, n->params, n->m1, n->m2, n->grad, P,
                       (float)lr, b1, b2, 1e-8f, bc1, bc2);
    DNET_CHECK(hipGetLastError());
    return refresh(*n);
}

dda_status dda_guess(dda_ctx *ch, dda_net *h, const dda_beam *beams, int32_t n_rhs, const void *feat, void *x0) {
    dda::clear_error();
    Net *n = nx_(h);
    dda::Ctx *c = dda::cx(ch);
    if (!n || !c || !beams || !feat || !x0 || n_rhs < 1 || n_rhs > n->maxb || dda::wrapped(*c) || !fits(*n, *c)) {
        set_error("dda_guess: NULL argument, n_rhs outside [1, max_batch], inhomogeneous particle, or particle larger "
                  "than the network's grid");
        return DDA_EINVAL;
    }
    for (int r = 0; r < n_rhs; ++r)
        if (!dda::beam_ok(&beams[r]) || beams[r].w0 > 0) {
            set_error("dda_guess: beam without unit vectors, or a focused beam (plane waves only)");
            return DDA_EINVAL;
        }
    dda_status st = forward(*n, (const bf16 *)feat, n_rhs);
    if (st != DDA_OK) return st;
    const int G = n->G, N = (int)c->N;
    for (int r = 0; r < n_rhs; ++r) {
        double br, bi;
        dda::beta_of(*c, beams[r], br, bi);
        hipLaunchKernelGGL(k_guess, dim3((N + 255) / 256), dim3(256), 0, n->stream, c->lin, N, c->nx, c->ny, c->nz, G,
                           c->kd, beam_args(beams[r], br, bi), n->out + (size_t)r * G * G * G * kOut,
                           (double2 *)x0 + (size_t)r * 3 * N);
    }
    DNET_CHECK(hipGetLastError());
    return DDA_OK;
}

}  // extern "C"
