// Inhomogeneous particles: a refractive index per material (eq. 1 holds with a different
// polarizability alpha_i at every dipole; the symmetrized system of eqs. 2-3 has
// A = I - B G B, B = diag(beta_i), beta_i = sqrt(alpha_i), right-hand side beta_i E_inc,i and
// P_i = beta_i x_i).  The product is the homogeneous one with unit polarizability, wrapped:
//   x' = B x;  y' = x' - G x' (the unit product);  y = x - B (x' - y')
// so the transform kernels stay as they are; the two wrapping passes read and write five vectors.
// The wrapping pass also forms the bilinear partials x^T y that the solvers take from the product.
#include <cmath>
#include <string>
#include <vector>

#include "ctx.hpp"

namespace dda {

dda_status matvec_device_unit(Ctx &c, const double2 *x, double2 *y, int nrhs, const double2 *scale, hipStream_t s,
                              const int *done, hipEvent_t *ev);
dda_status setup(Ctx **out, const int32_t grid[3], const uint8_t *mask, const double m[2], double kd, int32_t pol,
                 const dda_setup_opts *opts, void *stream);
void destroy(Ctx *c);

constexpr int kMatThreads = 256;
constexpr int kMatBlocks = 1024;

__device__ inline double2 cm(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// xo[r][q][i] = beta[r][mat_i][q] x[r][q][i] per right-hand side (grid: blocks x nrhs)
__global__ void __launch_bounds__(kMatThreads) k_mat_scale(const double2 *x, double2 *xo,  // may alias
                                                           const uint8_t *__restrict__ mat,
                                                           const double2 *__restrict__ beta, int nmat, int64_t N,
                                                           const int *done) {
    const int r = blockIdx.y;
    if (done && done[r]) return;
    const size_t n3 = 3 * (size_t)N, off = (size_t)r * n3;
    const double2 *bt = beta + (size_t)r * nmat * 3;
    for (size_t e = (size_t)blockIdx.x * kMatThreads + threadIdx.x; e < n3; e += (size_t)gridDim.x * kMatThreads)
        xo[off + e] = cm(bt[3 * mat[e % N] + e / N], x[off + e]);
}

// y = x - beta (xs - y) in place of y, and per-block bilinear partials x^T y into dots[r][0..ndots)
// (blocks beyond the grid's are zero)
__global__ void __launch_bounds__(kMatThreads) k_mat_post(const double2 *__restrict__ x,
                                                          const double2 *__restrict__ xs, double2 *__restrict__ y,
                                                          const uint8_t *__restrict__ mat,
                                                          const double2 *__restrict__ beta, int nmat, int64_t N,
                                                          double2 *dots, int ndots, const int *done) {
    __shared__ double2 sh[kMatThreads];
    const int r = blockIdx.y;
    if (done && done[r]) return;
    const size_t n3 = 3 * (size_t)N, off = (size_t)r * n3;
    const double2 *bt = beta + (size_t)r * nmat * 3;
    double2 acc = make_double2(0, 0);
    for (size_t e = (size_t)blockIdx.x * kMatThreads + threadIdx.x; e < n3; e += (size_t)gridDim.x * kMatThreads) {
        const double2 xv = x[off + e], d = xs[off + e], yv = y[off + e];
        const double2 b = cm(bt[3 * mat[e % N] + e / N], make_double2(d.x - yv.x, d.y - yv.y));
        const double2 o = make_double2(xv.x - b.x, xv.y - b.y);
        y[off + e] = o;
        const double2 p = cm(xv, o);
        acc.x += p.x;
        acc.y += p.y;
    }
    if (!dots) return;
    const int t = threadIdx.x;
    sh[t] = acc;
    __syncthreads();
    for (int h = kMatThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            sh[t].x += sh[t + h].x;
            sh[t].y += sh[t + h].y;
        }
        __syncthreads();
    }
    double2 *dr = dots + (size_t)r * ndots;
    if (t == 0) dr[blockIdx.x] = sh[0];
    for (int j = gridDim.x + blockIdx.x * kMatThreads + t; j < ndots; j += gridDim.x * kMatThreads)
        dr[j] = make_double2(0, 0);
}

// per-block partial sum of |P_q|^2 over the dipoles of material m (component q)
__global__ void __launch_bounds__(kMatThreads) k_mat_norm(const double2 *__restrict__ P,
                                                          const uint8_t *__restrict__ mat, int m, int q, int64_t N,
                                                          double *part) {
    __shared__ double sh[kMatThreads];
    double acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * kMatThreads + threadIdx.x; i < N; i += (int64_t)gridDim.x * kMatThreads)
        if (mat[i] == m) {
            const double2 v = P[(size_t)q * N + i];
            acc += v.x * v.x + v.y * v.y;
        }
    const int t = threadIdx.x;
    sh[t] = acc;
    __syncthreads();
    for (int h = kMatThreads / 2; h > 0; h >>= 1) {
        if (t < h) sh[t] += sh[t + h];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = sh[0];
}

static int mat_blocks(int64_t N) { return (int)std::min<int64_t>(kMatBlocks, (3 * N + kMatThreads - 1) / kMatThreads); }

// beta of every material and component for a beam (principal square roots), [nmat][3]
static void material_betas(const Ctx &c, const dda_beam &b, double2 *out) {
    for (int m = 0; m < c.nmat; ++m)
        for (int q = 0; q < 3; ++q) {
            double ar, ai;
            polarizability_comp(c, b, c.mat_re[m], c.mat_im[m], q, ar, ai);
            const double mod = std::hypot(ar, ai);
            out[3 * m + q] = make_double2(std::sqrt(0.5 * (mod + ar)), std::copysign(std::sqrt(0.5 * (mod - ar)), ai));
        }
}

// table rows (the last row, index rows, serves single-beam scaling) and scaled-vector rows
static dda_status ensure_material_bufs(Ctx &c, int rows, int xrows) {
    if (rows > c.mat_beta_rows) {
        (void)hipFree(c.mat_beta);
        c.mat_beta = nullptr;
        c.mat_beta_rows = 0;
        dda_status st = device_alloc((void **)&c.mat_beta, (size_t)(rows + 1) * c.nmat * 3 * sizeof(double2));
        if (st != DDA_OK) return st;
        c.mat_beta_rows = rows;
    }
    if (xrows > c.xtmp_rows) {
        (void)hipFree(c.xtmp);
        c.xtmp = nullptr;
        c.xtmp_rows = 0;
        dda_status st = device_alloc((void **)&c.xtmp, (size_t)xrows * 3 * c.N * sizeof(double2));
        if (st != DDA_OK) return st;
        c.xtmp_rows = xrows;
    }
    return DDA_OK;
}

dda_status material_prepare(Ctx &c, const dda_beam *beams, int n) {
    if (!wrapped(c)) return DDA_OK;
    dda_status st = ensure_material_bufs(c, n, std::max(n, 2));
    if (st != DDA_OK) return st;
    std::vector<double2> t((size_t)n * c.nmat * 3);
    for (int r = 0; r < n; ++r) material_betas(c, beams[r], t.data() + (size_t)r * c.nmat * 3);
    DDA_HIP_CHECK(hipMemcpyAsync(c.mat_beta, t.data(), t.size() * sizeof(double2), hipMemcpyHostToDevice, c.stream));
    DDA_HIP_CHECK(hipStreamSynchronize(c.stream));
    return DDA_OK;
}

dda_status material_scale(Ctx &c, const dda_beam &b, const double2 *x, double2 *P, hipStream_t s) {
    dda_status st = ensure_material_bufs(c, 1, 2);
    if (st != DDA_OK) return st;
    std::vector<double2> t((size_t)c.nmat * 3);
    material_betas(c, b, t.data());
    double2 *row = c.mat_beta + (size_t)c.mat_beta_rows * c.nmat * 3;
    DDA_HIP_CHECK(hipMemcpyAsync(row, t.data(), t.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_mat_scale, dim3(mat_blocks(c.N), 1), dim3(kMatThreads), 0, s, x, P, c.dmat, row, c.nmat, c.N,
                       nullptr);
    DDA_HIP_CHECK(hipGetLastError());
    DDA_HIP_CHECK(hipStreamSynchronize(s));
    return DDA_OK;
}

dda_status material_cabs(Ctx &c, const dda_beam &b, const double2 *P, double &cabs) {
    const int nb = (int)std::min<int64_t>(kMatBlocks, (c.N + kMatThreads - 1) / kMatThreads);
    double *part = nullptr;
    dda_status st = device_alloc((void **)&part, (size_t)nb * sizeof(double));
    if (st != DDA_OK) return st;
    std::vector<double> h(nb);
    const double k = c.kd;
    cabs = 0;
    hipError_t he = hipSuccess;
    for (int mq = 0; mq < 3 * c.nmat && he == hipSuccess; ++mq) {
        const int m = mq / 3, q = mq % 3;
        hipLaunchKernelGGL(k_mat_norm, dim3(nb), dim3(kMatThreads), 0, c.stream, P, c.dmat, m, q, c.N, part);
        he = hipGetLastError();
        if (he == hipSuccess) he = hipMemcpyAsync(h.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, c.stream);
        if (he == hipSuccess) he = hipStreamSynchronize(c.stream);
        double s = 0;
        for (int i = 0; i < nb; ++i) s += h[i];
        double ar, ai;
        polarizability_comp(c, b, c.mat_re[m], c.mat_im[m], q, ar, ai);
        const double a2 = ar * ar + ai * ai;
        if (a2 > 0) cabs += 4.0 * M_PI * k * (ai / a2 - (2.0 / 3.0) * k * k * k) * s;  // -Im(1/alpha) = Im(alpha)/|alpha|^2
    }
    (void)hipFree(part);
    if (he != hipSuccess) {
        set_error(std::string("material_cabs: ") + hipGetErrorString(he));
        return DDA_EHIP;
    }
    return DDA_OK;
}

dda_status material_init(Ctx &c, int n_mat, const double *m) {
    if (n_mat <= 1 && c.polarizability != DDA_POL_CLDR) return DDA_OK;
    c.nmat = n_mat;
    c.mat_re.resize(n_mat);
    c.mat_im.resize(n_mat);
    for (int i = 0; i < n_mat; ++i) {
        c.mat_re[i] = m[2 * i];
        c.mat_im[i] = m[2 * i + 1];
    }
    std::vector<uint8_t> mt(c.N);
    for (int64_t i = 0; i < c.N; ++i) mt[i] = n_mat > 1 ? (uint8_t)(c.mask[c.lin_host[i]] - 1) : 0;
    dda_status st = device_alloc((void **)&c.dmat, mt.size());
    if (st != DDA_OK) return st;
    const hipError_t he = hipMemcpy(c.dmat, mt.data(), mt.size(), hipMemcpyHostToDevice);
    if (he != hipSuccess) {
        set_error(std::string("material set-up: ") + hipGetErrorString(he));
        return DDA_EHIP;
    }
    return ensure_material_bufs(c, 1, 2);
}

dda_status matvec_materials(Ctx &c, const double2 *x, double2 *y, int nrhs, const double2 *scale, double2 *dots,
                            hipStream_t s, const int *done, hipEvent_t *ev) {
    if (x == y || nrhs > c.mat_beta_rows || nrhs > c.xtmp_rows) {
        set_error("matvec (inhomogeneous particle): x and y must differ, and the materials' table must cover the "
                  "batch (material_prepare)");
        return DDA_EINVAL;
    }
    // one dot partial per block: the grid stays within the partials the solvers read per RHS
    const int ndots = (int)dots_per_rhs<double>(c);
    const dim3 g(std::max(1, std::min(mat_blocks(c.N), ndots)), nrhs);
    hipLaunchKernelGGL(k_mat_scale, g, dim3(kMatThreads), 0, s, x, c.xtmp, c.dmat, c.mat_beta, c.nmat, c.N, done);
    DDA_HIP_CHECK(hipGetLastError());
    dda_status st = matvec_device_unit(c, c.xtmp, y, nrhs, scale, s, done, ev);
    if (st != DDA_OK) return st;
    hipLaunchKernelGGL(k_mat_post, g, dim3(kMatThreads), 0, s, x, c.xtmp, y, c.dmat, c.mat_beta, c.nmat, c.N, dots,
                       ndots, done);
    DDA_HIP_CHECK(hipGetLastError());
    return DDA_OK;
}

}  // namespace dda

using namespace dda;

extern "C" dda_status dda_setup_materials(dda_ctx **out, const int32_t grid[3], const uint8_t *mask, int32_t n_mat,
                                          const double *m, double kd, int32_t polarizability,
                                          const dda_setup_opts *opts, void *stream) {
    clear_error();
    if (out) *out = nullptr;
    if (!out || !grid || !mask || !m || n_mat < 1 || n_mat > 255 || grid[0] < 1 || grid[1] < 1 || grid[2] < 1) {
        set_error("dda_setup_materials: NULL argument, n_mat outside 1..255 or an empty grid");
        return DDA_EINVAL;
    }
    const size_t ncell = (size_t)grid[0] * grid[1] * grid[2];
    for (size_t e = 0; e < ncell; ++e)
        if (mask[e] > n_mat) {
            set_error("dda_setup_materials: a mask value exceeds n_mat");
            return DDA_EINVAL;
        }
    for (int i = 0; i < 2 * n_mat; ++i)
        if (!std::isfinite(m[i])) {
            set_error("dda_setup_materials: non-finite refractive index");
            return DDA_EINVAL;
        }
    if ((n_mat > 1 || polarizability == DDA_POL_CLDR) && opts && opts->fp32) {
        set_error("dda_setup_materials: single-precision products are not available for inhomogeneous particles "
                  "or CLDR");
        return DDA_ENOTSUP;
    }
    Ctx *c = nullptr;
    dda_status st = setup(&c, grid, mask, m, kd, polarizability, opts, stream);
    if (st != DDA_OK) return st;
    if ((st = material_init(*c, n_mat, m)) != DDA_OK) {
        destroy(c);
        return st;
    }
    *out = reinterpret_cast<dda_ctx *>(c);
    return DDA_OK;
}
