// Orientation averaging of the cross sections (Sec. 2: the paper's program averages over the
// Euler angles of the particle).  Orientation R = Rz(alpha) Ry(beta) Rz(gamma); alpha only turns
// the scattering plane, so the cross sections need beta and gamma: Romberg integration in
// cos(beta) on 2^n_beta + 1 points and the trapezoid rule on 2^n_gamma points in gamma (periodic).
// Every orientation is solved for both incident polarizations (x and y in the laboratory frame,
// brought into the particle frame by R^T), as batched right-hand sides of dda_solve.  The adaptive
// form doubles the cos(beta) grid (solving only the new points) until Romberg's error estimates
// meet a relative tolerance, as the paper's program integrates adaptively over the angles.  The
// averaged Mueller matrix takes alpha from the scattering planes: turning the particle by alpha
// about the incident direction turns the scattering plane by -alpha, so each orientation's matrix
// is averaged over equispaced planes.
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

// The beams of the orientations (cos(beta) in mus) x (ng equispaced gamma), x and y polarized
// in the laboratory frame, in that order (orientation-major, polarization fastest)
static std::vector<dda_beam> orientation_beams(const std::vector<double> &mus, int ng) {
    std::vector<dda_beam> beams;
    beams.reserve((size_t)2 * mus.size() * ng);
    for (const double mu : mus) {
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
    return beams;
}

// Solve the beams as batched right-hand sides, in chunks of whole polarization pairs that fit a
// modest device buffer; use(s0, cnt, x, per) sees the solutions of beams s0 .. s0 + cnt - 1
// (x: device [cnt][3][N], per bytes each)
template <typename F>
static dda_status solve_in_chunks(dda_ctx *h, Ctx *c, const std::vector<dda_beam> &beams, double tol,
                                  const dda_solve_opts *opts, F &&use) {
    const size_t per = (size_t)3 * c->N * sizeof(double2);
    const int chunk = (int)std::max<size_t>(2, std::min<size_t>(64, ((size_t)1 << 30) / per)) / 2 * 2;
    void *xbuf = nullptr;
    dda_status st = device_alloc(&xbuf, per * chunk);
    if (st != DDA_OK) return st;
    for (size_t s0 = 0; s0 < beams.size() && st == DDA_OK; s0 += chunk) {
        const int cnt = (int)std::min<size_t>(chunk, beams.size() - s0);
        st = dda_solve(h, beams.data() + s0, cnt, tol, opts, xbuf, nullptr);
        if (st == DDA_OK) st = use(s0, cnt, (const char *)xbuf, per);
    }
    (void)hipFree(xbuf);
    return st;  // a failing call's message stays
}

// Mean Cext and Cabs over the ng equispaced gamma and the two incident polarizations at each
// cos(beta) in mus
static dda_status beta_rows(dda_ctx *h, Ctx *c, const std::vector<double> &mus, int ng, double tol,
                            const dda_solve_opts *opts, std::vector<double> &fe, std::vector<double> &fa) {
    const int nb = (int)mus.size();
    const std::vector<dda_beam> beams = orientation_beams(mus, ng);
    std::vector<double> cext(beams.size()), cabs(beams.size());
    dda_status st = solve_in_chunks(h, c, beams, tol, opts, [&](size_t s0, int cnt, const char *x, size_t per) {
        for (int r = 0; r < cnt; ++r) {
            double cs[3];
            const dda_status e = dda_cross_sections(h, &beams[s0 + r], x + per * r, cs);
            if (e != DDA_OK) return e;
            cext[s0 + r] = cs[0];
            cabs[s0 + r] = cs[1];
        }
        return DDA_OK;
    });
    if (st != DDA_OK) return st;
    // unpolarized mean over the two polarizations and over gamma
    fe.assign(nb, 0.0);
    fa.assign(nb, 0.0);
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
    return DDA_OK;
}

// the 2^n + 1 equispaced cos(beta) on [-1, 1] (a point of level n is bitwise the same value at
// every finer level)
static double mu_at(int i, int n) { return -1.0 + 2.0 * i / (1 << n); }

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
    std::vector<double> mus(nb), fe, fa;
    for (int i = 0; i < nb; ++i) mus[i] = mu_at(i, n_beta);
    const dda_status st = beta_rows(h, c, mus, ng, tol, opts, fe, fa);
    if (st != DDA_OK) return st;
    // Romberg in cos(beta)
    double ve, ee, va, ea;
    romberg(fe, -1.0, 1.0, ve, ee);
    romberg(fa, -1.0, 1.0, va, ea);
    out[0] = ve / 2.0;
    out[1] = va / 2.0;
    out[2] = (ve - va) / 2.0;
    out[3] = ee / 2.0;
    return DDA_OK;
}

extern "C" dda_status dda_orientation_average_adaptive(dda_ctx *h, double eps, int32_t n_beta_min,
                                                       int32_t n_beta_max, int32_t n_gamma, double tol,
                                                       const dda_solve_opts *opts, double out[5],
                                                       int32_t *n_beta_used) {
    clear_error();
    Ctx *c = cx(h);
    if (!c || !out || !(eps > 0) || n_beta_min < 1 || n_beta_max < n_beta_min || n_beta_max > 10 || n_gamma < 0 ||
        n_gamma > 10 || !(tol > 0) || (opts && opts->x0)) {
        set_error("dda_orientation_average_adaptive: NULL argument, eps <= 0, not 1 <= n_beta_min <= n_beta_max <= "
                  "10, n_gamma outside 0..10, tol <= 0 or an initial guess");
        return DDA_EINVAL;
    }
    const int ng = 1 << n_gamma;
    int n = n_beta_min;
    std::vector<double> mus((1 << n) + 1), fe, fa;
    for (int i = 0; i <= (1 << n); ++i) mus[i] = mu_at(i, n);
    dda_status st = beta_rows(h, c, mus, ng, tol, opts, fe, fa);
    if (st != DDA_OK) return st;
    for (;;) {
        double ve, ee, va, ea;
        romberg(fe, -1.0, 1.0, ve, ee);
        romberg(fa, -1.0, 1.0, va, ea);
        if ((ee <= eps * std::fabs(ve) && ea <= eps * std::fabs(ve)) || n == n_beta_max) {
            out[0] = ve / 2.0;
            out[1] = va / 2.0;
            out[2] = (ve - va) / 2.0;
            out[3] = ee / 2.0;
            out[4] = ea / 2.0;
            if (n_beta_used) *n_beta_used = n;
            return DDA_OK;
        }
        // next level: only the new midpoints are solved
        ++n;
        std::vector<double> nm, ne, na;
        for (int i = 1; i < (1 << n); i += 2) nm.push_back(mu_at(i, n));
        if ((st = beta_rows(h, c, nm, ng, tol, opts, ne, na)) != DDA_OK) return st;
        std::vector<double> me((1 << n) + 1), ma((1 << n) + 1);
        for (int i = 0; i <= (1 << n); ++i) {
            me[i] = i % 2 ? ne[i / 2] : fe[i / 2];
            ma[i] = i % 2 ? na[i / 2] : fa[i / 2];
        }
        fe.swap(me);
        fa.swap(ma);
    }
}

extern "C" dda_status dda_orientation_average_mueller(dda_ctx *h, int32_t n_beta, int32_t n_gamma, int32_t n_alpha,
                                                      double tol, const dda_solve_opts *opts, const double *theta,
                                                      int32_t n_theta, double *M, double *err) {
    clear_error();
    Ctx *c = cx(h);
    if (!c || !theta || !M || n_theta < 1 || n_theta > (1 << 16) || n_beta < 1 || n_beta > 10 || n_gamma < 0 ||
        n_gamma > 10 || n_alpha < 1 || n_alpha > 1024 || !(tol > 0) || (opts && opts->x0)) {
        set_error("dda_orientation_average_mueller: NULL argument, n_theta outside 1..65536, n_beta outside 1..10, "
                  "n_gamma outside 0..10, n_alpha outside 1..1024, tol <= 0 or an initial guess");
        return DDA_EINVAL;
    }
    const int nb = (1 << n_beta) + 1, ng = 1 << n_gamma;
    std::vector<double> mus(nb);
    for (int i = 0; i < nb; ++i) mus[i] = mu_at(i, n_beta);
    const std::vector<dda_beam> beams = orientation_beams(mus, ng);
    const size_t per_row = (size_t)n_theta * 16;
    std::vector<double> rows((size_t)nb * per_row, 0.0), m1(per_row);
    // every chunk holds whole (x, y) pairs: the pair's solutions give the matrix in any plane
    dda_status st = solve_in_chunks(h, c, beams, tol, opts, [&](size_t s0, int cnt, const char *x, size_t per) {
        for (int r = 0; r < cnt; r += 2) {
            const size_t q = s0 + r, i = q / (2 * (size_t)ng);
            for (int a = 0; a < n_alpha; ++a) {
                const double phi = 2.0 * M_PI * a / n_alpha;
                const dda_status e = dda_mueller(h, &beams[q], x + per * r, x + per * (r + 1), phi, theta, n_theta,
                                                 m1.data());
                if (e != DDA_OK) return e;
                for (size_t t = 0; t < per_row; ++t) rows[i * per_row + t] += m1[t];
            }
        }
        return DDA_OK;
    });
    if (st != DDA_OK) return st;
    // mean over gamma and alpha, then Romberg in cos(beta) element by element
    std::vector<double> f(nb);
    for (size_t t = 0; t < per_row; ++t) {
        for (int i = 0; i < nb; ++i) f[i] = rows[i * per_row + t] / ((double)ng * n_alpha);
        double v, e;
        romberg(f, -1.0, 1.0, v, e);
        M[t] = v / 2.0;
        if (err && t % 16 == 0) err[t / 16] = e / 2.0;
    }
    return DDA_OK;
}
