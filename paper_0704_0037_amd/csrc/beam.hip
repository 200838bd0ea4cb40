// Focused (Gaussian) incident beams (Sec. 2: the paper's program can illuminate the particle with
// tightly focused Gaussian beams; it does not give their field).  The beam is the superposition
// of propagating plane waves with a Gaussian angular spectrum:
//   E(r) = (w0^2 / 4 pi) int_{|q| < k} exp(-w0^2 |q|^2 / 4) (e - (e.k^) k^) exp(i k k^.(r - c)) d^2q,
// k^ = (q + sqrt(k^2 - |q|^2) a) / k for transverse wavevectors q.  Every term is a transverse
// plane wave, so the field solves Maxwell's equations exactly; its paraxial limit is the Gaussian
// beam of waist radius w0 focused at c, and w0 -> infinity gives the plane wave e exp(i k a.(r - c)).
// With |q| = k sin t: Gauss-Legendre in t on [0, t_max], sin t_max = min(1, 12 / (k w0)) (the
// spectrum is below 3e-16 beyond), n_t = ceil(k sin(t_max) r_max) + 24 nodes, and the periodic
// trapezoid rule on n_phi = 2 ceil(k sin(t_max) r_max) + 16 azimuths, r_max = max |r_i - c| over
// the dipoles.  The host builds the node table (direction k^ and weighted polarization vector
// per node); one thread per dipole sums the plane waves with the table staged through LDS.
#include <cmath>
#include <vector>

#include "ctx.hpp"

namespace dda {

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);

constexpr int kBeamThreads = 256;
constexpr int kNodeDoubles = 9;  // k^ (3), weighted (e - (e.k^) k^) (3 complex)
constexpr int64_t kMaxBeamNodes = 1 << 20;

// out[c][i] = s * E_c(r_i) for the node table tab [M][9]
template <typename R>
__global__ void __launch_bounds__(kBeamThreads) k_beam_field(const int *__restrict__ lin, cplx<R> *__restrict__ out,
                                                             int N, int nx, int ny, int nz, double k, double cx,
                                                             double cy, double cz, const double *__restrict__ tab,
                                                             int M, double sr, double si) {
    __shared__ double t[kBeamThreads * kNodeDoubles];
    const int i = blockIdx.x * kBeamThreads + threadIdx.x;
    double x = 0, y = 0, z = 0;
    if (i < N) {
        const int l = lin[i];
        x = (l % nx) + 0.5 - 0.5 * nx - cx;
        y = ((l / nx) % ny) + 0.5 - 0.5 * ny - cy;
        z = (l / (nx * ny)) + 0.5 - 0.5 * nz - cz;
    }
    double ar[3] = {0, 0, 0}, ai[3] = {0, 0, 0};
    for (int m0 = 0; m0 < M; m0 += kBeamThreads) {
        const int cnt = min(kBeamThreads, M - m0);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt * kNodeDoubles; q += kBeamThreads) t[q] = tab[(size_t)m0 * kNodeDoubles + q];
        __syncthreads();
        for (int m = 0; m < cnt; ++m) {
            const double *n = t + m * kNodeDoubles;
            double sn, cs;
            sincos(k * (n[0] * x + n[1] * y + n[2] * z), &sn, &cs);
            for (int c = 0; c < 3; ++c) {
                const double vr = n[3 + 2 * c], vi = n[4 + 2 * c];
                ar[c] += vr * cs - vi * sn;
                ai[c] += vr * sn + vi * cs;
            }
        }
    }
    if (i >= N) return;
    for (int c = 0; c < 3; ++c)
        out[(size_t)c * N + i] = mk<cplx<R>>((R)(sr * ar[c] - si * ai[c]), (R)(sr * ai[c] + si * ar[c]));
}

// node table of the beam's angular spectrum for this particle (see the file comment)
static dda_status beam_nodes(const Ctx &c, const dda_beam &b, std::vector<double> &tab, int &M) {
    const double k = c.kd, w0 = b.w0;
    const double a[3] = {b.prop[0], b.prop[1], b.prop[2]};
    // e1: the real (else imaginary) part of the polarization, made transverse; e2 = a x e1
    double e1[3], n2 = 0;
    for (int q = 0; q < 3; ++q) n2 += b.pol_re[q] * b.pol_re[q];
    const double *src = n2 > 1e-16 ? b.pol_re : b.pol_im;
    double d = 0;
    for (int q = 0; q < 3; ++q) d += src[q] * a[q];
    double nn = 0;
    for (int q = 0; q < 3; ++q) {
        e1[q] = src[q] - d * a[q];
        nn += e1[q] * e1[q];
    }
    nn = std::sqrt(nn);
    for (int q = 0; q < 3; ++q) e1[q] /= nn;
    const double e2[3] = {a[1] * e1[2] - a[2] * e1[1], a[2] * e1[0] - a[0] * e1[2], a[0] * e1[1] - a[1] * e1[0]};
    // r_max over the dipoles
    double r2 = 0;
    for (int z = 0; z < c.nz; ++z)
        for (int y = 0; y < c.ny; ++y)
            for (int x = 0; x < c.nx; ++x) {
                if (!c.mask[((size_t)z * c.ny + y) * c.nx + x]) continue;
                const double px = x + 0.5 - 0.5 * c.nx - b.center[0], py = y + 0.5 - 0.5 * c.ny - b.center[1],
                             pz = z + 0.5 - 0.5 * c.nz - b.center[2];
                r2 = std::max(r2, px * px + py * py + pz * pz);
            }
    const double st = std::min(1.0, 12.0 / (k * w0));
    const double t_max = std::asin(st);
    const int64_t kr = (int64_t)std::ceil(k * st * std::sqrt(r2));
    const int64_t n_t = kr + 24, n_phi = 2 * kr + 16;
    if (n_t * n_phi > kMaxBeamNodes) {
        set_error("focused beam: the angular-spectrum quadrature would need more than 2^20 nodes (particle too large "
                  "for its waist)");
        return DDA_EINVAL;
    }
    std::vector<double> gx, gw;
    gauss_legendre((int)n_t, gx, gw);
    M = (int)(n_t * n_phi);
    tab.assign((size_t)M * kNodeDoubles, 0.0);
    const double pre = w0 * w0 / (4.0 * M_PI) * (2.0 * M_PI / n_phi) * k * k;
    size_t o = 0;
    for (int64_t it = 0; it < n_t; ++it) {
        const double t = 0.5 * t_max * (gx[it] + 1.0), wt = 0.5 * t_max * gw[it];
        const double s = std::sin(t), cs = std::cos(t);
        const double wgt = pre * wt * std::exp(-0.25 * (w0 * k * s) * (w0 * k * s)) * s * cs;
        for (int64_t ip = 0; ip < n_phi; ++ip) {
            const double ph = 2.0 * M_PI * ip / n_phi, cp = std::cos(ph), sp = std::sin(ph);
            double kh[3];
            for (int q = 0; q < 3; ++q) kh[q] = s * (cp * e1[q] + sp * e2[q]) + cs * a[q];
            double pr = 0, pi = 0;  // e . k^ (bilinear)
            for (int q = 0; q < 3; ++q) {
                pr += b.pol_re[q] * kh[q];
                pi += b.pol_im[q] * kh[q];
            }
            double *n = tab.data() + o;
            for (int q = 0; q < 3; ++q) {
                n[q] = kh[q];
                n[3 + 2 * q] = wgt * (b.pol_re[q] - pr * kh[q]);
                n[4 + 2 * q] = wgt * (b.pol_im[q] - pi * kh[q]);
            }
            o += kNodeDoubles;
        }
    }
    return DDA_OK;
}

// out = s * E_inc at the dipoles for a focused beam (b.w0 > 0), on stream st; returns after the
// launch has finished (the node table is freed)
template <typename R> dda_status beam_field_launch(Ctx &c, const dda_beam &b, cplx<R> *out, double sr, double si,
                                                   hipStream_t st) {
    std::vector<double> tab;
    int M = 0;
    dda_status e = beam_nodes(c, b, tab, M);
    if (e != DDA_OK) return e;
    void *dt = nullptr;
    if ((e = device_alloc(&dt, tab.size() * sizeof(double))) != DDA_OK) return e;
    hipError_t he = hipMemcpyAsync(dt, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, st);
    if (he == hipSuccess) {
        const int N = (int)c.N;
        hipLaunchKernelGGL(k_beam_field<R>, dim3((N + kBeamThreads - 1) / kBeamThreads), dim3(kBeamThreads), 0, st,
                           c.lin, out, N, c.nx, c.ny, c.nz, c.kd, b.center[0], b.center[1], b.center[2],
                           (const double *)dt, M, sr, si);
        he = hipGetLastError();
        if (he == hipSuccess) he = hipStreamSynchronize(st);
    }
    (void)hipFree(dt);
    if (he != hipSuccess) {
        set_error(std::string("focused beam: ") + hipGetErrorString(he));
        return DDA_EHIP;
    }
    return DDA_OK;
}
template dda_status beam_field_launch<double>(Ctx &, const dda_beam &, double2 *, double, double, hipStream_t);
template dda_status beam_field_launch<float>(Ctx &, const dda_beam &, float2 *, double, double, hipStream_t);

}  // namespace dda
