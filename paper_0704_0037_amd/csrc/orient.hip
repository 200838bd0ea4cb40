// Orientation averaging of the cross sections (Sec. 2: the paper's program averages over the
// Euler angles of the particle).  Orientation R = Rz(alpha) Ry(beta) Rz(gamma); alpha only turns
// the scattering plane, so the cross sections need beta and gamma: Romberg integration in
// cos(beta) on 2^n_beta + 1 points and the trapezoid rule on 2^n_gamma points in gamma (periodic).
// Every orientation is solved for both incident polarizations (x and y in the laboratory frame,
// brought into the particle frame by R^T), as batched right-hand sides of dda_solve.
#include <cmath>
#include <string>
#include <vector>

#include "ctx.hpp"

namespace dda {

// Romberg table over samples f[0..2^n] of a function on [a, b]: the value and |R(n,n) - R(n,n-1)|
static void romberg(const std::vector<double> &f, double a, double b, double &value, double &err) {
    const int m = (int)f.size() - 1;
    int n = 0;
    while ((1 << n) < m) ++n;
    std::vector<std::vector<double>> R(n + 1);
    for (int k = 0; k <= n; ++k) {
        const int step = 1 << (n - k);
        double s = 0.5 * (f[0] + f[m]);
        for (int i = step; i < m; i += step) s += f[i];
        R[k].push_back(s * (b - a) / (1 << k));
    }
    for (int j = 1; j <= n; ++j)
        for (int k = j; k <= n; ++k) R[k].push_back(R[k][j - 1] + (R[k][j - 1] - R[k - 1][j - 1]) / (std::pow(4.0, j) - 1.0));
    value = R[n][n];
    err = n >= 1 ? std::fabs(R[n][n] - R[n][n - 1]) : 0.0;
}

}  // namespace dda

using namespace dda;

extern "C" dda_status dda_orientation_average(dda_ctx *h, int32_t n_beta, int32_t n_gamma, double tol,
                                              const dda_solve_opts *opts, double out[4]) {
    clear_error();
    Ctx *c = cx(h);
    if (!c || !out || n_beta < 1 || n_beta > 10 || n_gamma < 0 || n_gamma > 10 || !(tol > 0) || (opts && opts->x0)) {
        set_error("dda_orientation_average: NULL argument, n_beta outside 1..10, n_gamma outside 0..10, tol <= 0 "
                  "or an initial guess");
        return DDA_EINVAL;
    }
    const int nb = (1 << n_beta) + 1, ng = 1 << n_gamma;
    std::vector<dda_beam> beams;
    beams.reserve((size_t)2 * nb * ng);
    for (int i = 0; i < nb; ++i) {
        const double mu = -1.0 + 2.0 * i / (nb - 1);
        const double be = std::acos(std::max(-1.0, std::min(1.0, mu)));
        const double cb = std::cos(be), sb = std::sin(be);
        for (int j = 0; j < ng; ++j) {
            const double ga = 2.0 * M_PI * j / ng, cg = std::cos(ga), sg = std::sin(ga);
            // R = Ry(beta) Rz(gamma) (alpha = 0); the particle-frame beam is R^T applied to the
            // laboratory vectors: row l of R^T is column l of R
            const double R[3][3] = {{cb * cg, -cb * sg, sb}, {sg, cg, 0.0}, {-sb * cg, sb * sg, cb}};
            for (int pol = 0; pol < 2; ++pol) {
                dda_beam bm{};
                for (int q = 0; q < 3; ++q) {
                    bm.prop[q] = R[2][q];         // R^T e_z
                    bm.pol_re[q] = R[pol][q];     // R^T e_x or R^T e_y
                    bm.pol_im[q] = 0.0;
                }
                beams.push_back(bm);
            }
        }
    }
    // solve in batches that fit a modest device buffer
    const size_t per = (size_t)3 * c->N * sizeof(double2);
    const int chunk = (int)std::max<size_t>(2, std::min<size_t>(64, ((size_t)1 << 30) / per)) / 2 * 2;
    void *xbuf = nullptr;
    dda_status st = device_alloc(&xbuf, per * chunk);
    if (st != DDA_OK) return st;
    std::vector<double> cext(beams.size()), cabs(beams.size());
    for (size_t s0 = 0; s0 < beams.size() && st == DDA_OK; s0 += chunk) {
        const int cnt = (int)std::min<size_t>(chunk, beams.size() - s0);
        st = dda_solve(h, beams.data() + s0, cnt, tol, opts, xbuf, nullptr);
        if (st != DDA_OK) break;
        for (int r = 0; r < cnt && st == DDA_OK; ++r) {
            double cs[3];
            st = dda_cross_sections(h, &beams[s0 + r], (const char *)xbuf + per * r, cs);
            cext[s0 + r] = cs[0];
            cabs[s0 + r] = cs[1];
        }
    }
    (void)hipFree(xbuf);
    if (st != DDA_OK) return st;  // the failing call's message stays
    // unpolarized mean over the two polarizations and over gamma, then Romberg in cos(beta)
    std::vector<double> fe(nb), fa(nb);
    for (int i = 0; i < nb; ++i) {
        double se = 0, sa = 0;
        for (int j = 0; j < ng; ++j)
            for (int pol = 0; pol < 2; ++pol) {
                const size_t q = ((size_t)i * ng + j) * 2 + pol;
                se += cext[q];
                sa += cabs[q];
            }
        fe[i] = se / (2.0 * ng);
        fa[i] = sa / (2.0 * ng);
    }
    double ve, ee, va, ea;
    romberg(fe, -1.0, 1.0, ve, ee);
    romberg(fa, -1.0, 1.0, va, ea);
    out[0] = ve / 2.0;
    out[1] = va / 2.0;
    out[2] = (ve - va) / 2.0;
    out[3] = ee / 2.0;
    return DDA_OK;
}
