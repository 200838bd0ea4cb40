/*
 * dda.h — C-ABI of the MI355X (gfx950) discrete-dipole-approximation hot path.
 *
 * The library solves the DDA system of the paper (Yurkin, Maltsev & Hoekstra 2007,
 * Sec. 2, eqs. 1-3) for a particle given as a mask on a cubic dipole grid:
 *
 *     x_i - sum_{j != i} beta_i G_ij beta_j x_j = beta_i E_inc,i ,   P_i = beta_i x_i   (eq. 3)
 *
 * with beta_i^2 = alpha_i the dipole polarizability (LDR by default, Sec. 3.1) and G_ij the
 * free-space Green's tensor.  The interaction-matrix product is applied with zero-padded 3-D
 * FFTs split into 1-D transforms that skip the zero input and the unused output, the Fourier
 * transform of the interaction matrix stored symmetry-reduced (Sec. 2), and every operation
 * other than the FFT touching only the non-void dipoles (Sec. 2).  The iterative solvers are
 * the complex-symmetric QMR (one product per iteration, Sec. 2) and Bi-CGSTAB (Sec. 2), stopped
 * at relative residual norm < tol (default 1e-5, Sec. 2).
 *
 * Units: dipole size d = 1, so kd is the wavenumber; cross sections are in units of d^2.
 * Time dependence exp(-i w t).  Incident amplitude |E0| = 1.
 *
 * Layouts
 *   mask      host uint8  [nz][ny][nx], x fastest, nonzero = material.  The dipole order is the
 *             linear cell index x + nx*(y + ny*z) restricted to the mask; dipole i sits at
 *             (x + 1/2 - nx/2, y + 1/2 - ny/2, z + 1/2 - nz/2).
 *   vectors   device, component-major: complex128 (interleaved re, im doubles) [3][N], or
 *             [n_rhs][3][N] for batches; complex64 for the *_f32 entry points.
 *
 * Ownership: the context owns every device buffer it allocates and frees them in dda_free.
 * Caller vectors are never freed or retained.  Calls on one context are ordered on the
 * context's stream (the one given to dda_setup, or the default stream) and are not
 * thread-safe; separate contexts are independent.
 *
 * Errors: every entry point returns a dda_status; nothing throws or aborts across the ABI.
 * dda_last_error() describes the failure of the calling thread's most recent call ("" after a
 * call that succeeded).
 */
#ifndef DDA_MI355X_H
#define DDA_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dda_ctx dda_ctx;

typedef enum {
    DDA_OK = 0,
    DDA_EINVAL = -1,       /* bad argument (null pointer, empty mask, size out of range, ...) */
    DDA_ENOMEM = -2,       /* device allocation failed */
    DDA_EHIP = -3,         /* a HIP runtime call failed */
    DDA_ENOTCONV = -4,     /* maxit reached before tol; x_out holds the last iterate */
    DDA_EBREAKDOWN = -5,   /* Krylov breakdown (e.g. b^T b = 0 for QMR); x_out holds the last iterate */
    DDA_ESYMMETRY = -6,    /* one-polarization read-out asked for a particle without 90-degree symmetry */
    DDA_ENOTSUP = -7       /* option or combination of options not supported */
} dda_status;

/* Polarizability prescriptions (Sec. 2 lists four; LDR is the one used in Sec. 3).  For a unit
 * cube and wavenumber k: DDA_POL_CM  alpha_CM = (3/4pi)(m^2-1)/(m^2+2) (Clausius-Mossotti);
 * DDA_POL_CLDR  a diagonal tensor (Gutkowicz-Krusin & Draine 2004), independent of the polarization:
 *             1/alpha_jj = 1/alpha_CM + (b1 + m^2 b2 + m^2 b3 a_j^2) k^2 - (2/3) i k^3 with LDR's b;
 *             it runs the product wrapped between per-component scalings (as dda_setup_materials),
 *             in DDA_FP64 only;
 * DDA_POL_RR  1/alpha = 1/alpha_CM - (2/3) i k^3 (radiative-reaction correction);
 * DDA_POL_LDR 1/alpha = 1/alpha_CM + (b1 + m^2 b2 + m^2 b3 S) k^2 - (2/3) i k^3 (lattice
 * dispersion relation, S from the beam). */
enum { DDA_POL_LDR = 0, DDA_POL_CM = 1, DDA_POL_RR = 2, DDA_POL_CLDR = 3 };

/* Iterative solvers (Sec. 2): QMR and Bi-CG use the complex symmetry of the interaction matrix
 * (one product per iteration, bilinear form u^T v); Bi-CGSTAB takes two products per iteration
 * with Hermitian inner products; CGNR is conjugate gradients on A^H A x = A^H b (minimal residual
 * over its Krylov space; two products per iteration, A^H v formed as conj(A conj(v))). */
enum { DDA_QMR = 0, DDA_BICGSTAB = 1, DDA_BICG = 2, DDA_CGNR = 3 };

/* Arithmetic of the solve: plain double precision everywhere (Sec. 2: all floats double), or
 * single-precision FFTs, tensor multiply and inner QMR with double-precision residuals, iterate
 * updates and read-out (iterative refinement). */
/* DDA_FP64: everything in double precision.  DDA_FP32_REFINE: single-precision inner QMR solves
 * (products, vectors, scalars) on the double-precision residual, double-precision residual and
 * update (iterative refinement).  DDA_FP32_PRODUCT: the double-precision solver whose products run
 * the FFTs and the tensor multiply in single precision (x, y and the epilogue in double), to
 * max(tol, 1e-6), or until its residual stalls (no halving within as many iterations as its best
 * value took, at least 5000); a right-hand side whose true residual misses tol afterwards is
 * finished in DDA_FP64 from there (from zero if that iterate is no better than zero).
 * DDA_FP32_RELAXED: DDA_FP32_PRODUCT whose products start in double precision and switch to single
 * precision once the recursive residual of every right-hand side of the batch is below relax_at
 * (default 100 tol): the accuracy a product needs falls as the residual falls (inexact Krylov
 * methods), so the rounding of single-precision transforms, which stalls a strongly scattering
 * particle's solve when it enters at the first iteration, enters here scaled by the residual
 * reached.  Stall guard and double-precision finish as DDA_FP32_PRODUCT. */
enum { DDA_FP64 = 0, DDA_FP32_REFINE = 1, DDA_FP32_PRODUCT = 2, DDA_FP32_RELAXED = 3 };

/* Incident beam in the particle frame: unit propagation vector and complex unit polarization.
 * w0 = 0: the plane wave E_inc(r) = pol * exp(i kd prop.r).
 * w0 > 0: a focused beam of waist radius w0 (units of d) at center (the lattice frame: cell
 * (i, j, l) at (i + 1/2 - nx/2, ...)), the paper's tightly focused Gaussian beams (Sec. 2): the
 * angular spectrum of plane waves
 *   E(r) = (w0^2 / 4 pi) int_{|q| < k} exp(-w0^2 |q|^2 / 4) (pol - (pol.k^) k^) exp(i k k^.(r - center)) d^2q
 * (k^ = (q + sqrt(k^2 - |q|^2) prop) / k), an exact Maxwell solution whose paraxial limit is the
 * Gaussian beam; pol must be orthogonal to prop.  It enters the right-hand side and Cext; the
 * one-polarization Mueller shortcut and the learned guess take plane waves only.  Zero-initialize
 * the struct to get a plane wave. */
typedef struct {
    double prop[3];
    double pol_re[3];
    double pol_im[3];
    double w0;
    double center[3];
} dda_beam;

/* Optional settings of dda_setup (pass NULL for defaults). */
typedef struct {
    int32_t pad[3];        /* padded FFT sizes per axis; 0 = smallest supported size >= 2n-1 */
    int32_t lines_per_block; /* FFT lines per workgroup; 0 = built-in choice */
    int32_t fp32;          /* nonzero: also build the single-precision tensor (DDA_FP32_REFINE, _PRODUCT) */
} dda_setup_opts;

/* Options of dda_solve (pass NULL for defaults). */
typedef struct {
    int32_t solver;        /* DDA_QMR (default), DDA_BICGSTAB, DDA_BICG or DDA_CGNR */
    int32_t precision;     /* DDA_FP64 (default), DDA_FP32_REFINE or DDA_FP32_PRODUCT */
    int32_t maxit;         /* iteration limit; 0 = 100000 */
    int32_t check_every;   /* iterations between host-side convergence checks; 0 = automatic */
    double inner_tol;      /* DDA_FP32_REFINE: relative tolerance of each inner solve; 0 = automatic:
                              half of tol over the current residual, at least 1e-5 */
    const void *x0;        /* device initial guess, same layout as x_out; NULL = zero */
    int32_t graph;         /* iterations replayed as a captured hipGraph: 0 = automatic, 1 = on, -1 = off */
    int32_t x0_check;      /* 1: keep x0 for a right-hand side only if |b - A x0| < |b|, else start from 0 */
    int32_t on_breakdown;  /* DDA_BREAKDOWN_REPORT (default) or DDA_BREAKDOWN_RECOVER, below */
    int32_t resume;        /* 1: continue this context's last double-precision solve, which stopped at
                              its iteration limit (same beams, batch size and solver, else DDA_EINVAL;
                              x_out holding its iterate, or a checkpoint loaded by dda_checkpoint_load): right-hand sides
                              at their limit get maxit more iterations toward tol, exactly as if the
                              solve had not stopped; iters and matvecs count from its start; no
                              residual history */
    double relax_at;       /* DDA_FP32_RELAXED: relative residual below which the products switch to
                              single precision; 0 = 100 tol */
    int32_t pack;          /* dda_solve_many: 1 = particles that share a padded grid are solved as one
                              batch; 0 (default) = each particle on its own stream */
} dda_solve_opts;

/* What dda_solve does when QMR or Bi-CG breaks down for a right-hand side (the paper does not
 * say): DDA_BREAKDOWN_REPORT stops that right-hand side with DDA_EBREAKDOWN and its last iterate.
 * DDA_BREAKDOWN_RECOVER solves it again from its current iterate: the same method restarted (a
 * fresh Lanczos sequence on the current residual) at most twice, then Bi-CGSTAB; a breakdown
 * before the first step (b^T b = 0, e.g. a circularly polarized beam, for which the bilinear form
 * vanishes) goes to Bi-CGSTAB at once.  The attempts share opts.maxit; iters, matvecs and the
 * residual history (concatenated) cover all of them.  Ignored by dda_solve_many. */
enum { DDA_BREAKDOWN_REPORT = 0, DDA_BREAKDOWN_RECOVER = 1 };

/* Per-right-hand-side report of dda_solve. */
typedef struct {
    int32_t status;        /* dda_status of this right-hand side */
    int32_t iters;         /* solver iterations (summed over inner solves for DDA_FP32_REFINE) */
    int32_t matvecs;       /* interaction-matrix products */
    int32_t outer;         /* refinement steps (DDA_FP32_REFINE); 1 if DDA_FP32_PRODUCT switched to
                              double-precision products after its residual stalled or needed the
                              double-precision finish; else 0 */
    double res_rec;        /* relative recursive residual at exit */
    double res_true;       /* relative true residual ||b - A x|| / ||b|| computed once at exit */
    double t_solve_s;      /* wall time of the solve of the whole batch, seconds */
    double *res_hist;      /* optional host buffer for the relative residual per iteration */
    int32_t res_hist_cap;  /* its capacity in doubles (0 = none) */
    int32_t res_hist_len;  /* entries written (initial residual first) */
} dda_solve_info;

/*
 * dda_setup — build a context for one particle (Sec. 2: grid of dipoles, non-void list,
 * polarizability, Fourier transform of the interaction matrix).
 *   out    receives the context (set to NULL on failure)
 *   grid   {nx, ny, nz}, each 1..2048
 *   mask   host uint8 [nz][ny][nx]; at least one nonzero cell
 *   m      {Re m, Im m}, refractive index of the (homogeneous) material
 *   kd     wavenumber times dipole size, > 0
 *   polarizability  DDA_POL_LDR, DDA_POL_CM, DDA_POL_RR or DDA_POL_CLDR
 *   opts   NULL or settings above
 *   stream hipStream_t the context runs on (NULL = default stream)
 * Errors: DDA_EINVAL for bad arguments or an unsupported padded size, DDA_ENOMEM, DDA_EHIP.
 */
dda_status dda_setup(dda_ctx **out, const int32_t grid[3], const uint8_t *mask, const double m[2],
                     double kd, int32_t polarizability, const dda_setup_opts *opts, void *stream);

/*
 * dda_setup_materials — dda_setup for an inhomogeneous particle (eq. 1 takes a polarizability
 * per dipole; the symmetrized system of eqs. 2-3 then has beta_i = sqrt(alpha_i) per dipole):
 * mask values 1..n_mat name each cell's material, m holds {Re m, Im m} of each material
 * ([n_mat][2]); every polarizability prescription applies per material.  n_mat = 1 is dda_setup.
 * With n_mat > 1 the product runs the homogeneous kernels with unit polarizability between a
 * scaling of the vector by each dipole's beta and back (five extra vector passes); solves run in
 * DDA_FP64 only (opts->fp32 is refused with DDA_ENOTSUP), the read-out uses P = beta x and Cabs
 * per material; dda_mueller needs both polarizations, and the learned guess refuses the context.
 * Errors: as dda_setup; DDA_EINVAL for n_mat outside 1..255 or a mask value above n_mat.
 */
dda_status dda_setup_materials(dda_ctx **out, const int32_t grid[3], const uint8_t *mask, int32_t n_mat,
                               const double *m, double kd, int32_t polarizability, const dda_setup_opts *opts,
                               void *stream);

/* Release the context and all device memory it owns.  NULL is accepted. */
dda_status dda_free(dda_ctx *ctx);

/* Number of non-void dipoles N (or -1 for a NULL context). */
int64_t dda_num_dipoles(const dda_ctx *ctx);

/* Padded FFT grid {Lx, Ly, Lz} chosen at setup. */
dda_status dda_padded_grid(const dda_ctx *ctx, int32_t out[3]);

/* Polarizability alpha (host {re, im}) the context uses for this beam (LDR depends on the
 * beam through S = sum_mu (a_mu |e_mu|)^2; Sec. 3.1 names LDR). */
dda_status dda_polarizability(const dda_ctx *ctx, const dda_beam *beam, double out[2]);

/* Right-hand side of eq. 3, b = beta E_inc, written to device complex128 [3][N]. */
dda_status dda_rhs(dda_ctx *ctx, const dda_beam *beam, void *b);

/*
 * dda_matvec — y = A x with A of eq. 2 for the polarizability this beam selects (eq. 3 left side).
 *   x, y   device complex128 [3][N]; must not overlap
 * Errors: DDA_EINVAL (null pointers), DDA_EHIP.
 */
dda_status dda_matvec(dda_ctx *ctx, const dda_beam *beam, const void *x, void *y);

/* dda_matvec_f32 — the same product in single precision (complex64 [3][N]); needs the context
 * built with opts.fp32 != 0, else DDA_ENOTSUP. */
dda_status dda_matvec_f32(dda_ctx *ctx, const dda_beam *beam, const void *x, void *y);

/*
 * dda_matvec_noalloc — dda_matvec for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and the
 * same result bit for bit, with the intermediates of the transforms (and the polarizability scale)
 * in a fixed 128 MiB device array of the library instead of buffers of the context, so the call
 * allocates nothing and makes no allocating library call.  The first call on a device resolves
 * that array's address (hipGetSymbolAddress; make it outside graph capture).  Every call on one
 * device shares the array: calls that overlap on one device (other streams, other threads, other
 * contexts) race and must be ordered by the caller.  Homogeneous contexts only.
 *   x, y   device complex128 [3][N]; must not overlap
 * Errors: DDA_EINVAL (null pointers, overlap, or a particle whose intermediates exceed 128 MiB:
 * 48 (nz Lx ny' + nz' Lx Ly) bytes plus alignment, ny' and nz' being ny and nz rounded up to a
 * multiple of 16), DDA_ENOTSUP (several materials or CLDR),
 * DDA_EHIP.
 */
dda_status dda_matvec_noalloc(dda_ctx *ctx, const dda_beam *beam, const void *x, void *y);

/*
 * dda_matvec_batch — y_r = A_r x_r for n_rhs vectors sharing the particle: one pass over the
 * Fourier-space tensor per batch.  beams[n_rhs]; x, y device complex128 [n_rhs][3][N] (x and y
 * must not overlap).
 */
dda_status dda_matvec_batch(dda_ctx *ctx, const dda_beam *beams, int32_t n_rhs, const void *x, void *y);

/*
 * dda_solve — solve eq. 3 for n_rhs incident beams (Sec. 2 solvers, stopping rule
 * ||r|| / ||b|| < tol on the recursive residual, Sec. 2).
 *   beams   host [n_rhs]
 *   tol     relative residual threshold (> 0)
 *   opts    NULL or options
 *   x_out   device complex128 [n_rhs][3][N]; receives x (P = beta x)
 *   info    host [n_rhs] or NULL
 * Returns DDA_OK if every right-hand side converged, else the first failing status
 * (DDA_ENOTCONV / DDA_EBREAKDOWN); per-RHS statuses are in info.  DDA_EINVAL for bad arguments or
 * options; DDA_ENOTSUP for single precision on a context of several materials or CLDR, or on one
 * built without opts.fp32.
 * With the environment variable DDA_PROGRESS set to a number of seconds, a running solve prints
 * the iteration count and residual of every unconverged right-hand side to stderr that often.
 */
dda_status dda_solve(dda_ctx *ctx, const dda_beam *beams, int32_t n_rhs, double tol,
                     const dda_solve_opts *opts, void *x_out, dda_solve_info *info);

/*
 * dda_checkpoint_save / dda_checkpoint_load — the state of the context's last double-precision
 * solve that stopped at its iteration limit (per right-hand side scalars, iterate, Krylov vectors)
 * to and from a file, to continue it later with opts.resume (the paper's program checkpoints long
 * runs, Sec. 2).  x: device complex128 [n_rhs][3][N], the iterate (read by save, written by load).
 * The file belongs to this library build and the same particle: its header holds a hash of the
 * grid, mask (materials), refractive indices, kd and polarizability prescription, checked on load,
 * and a hash of the stopped solve's beams, which the continuing dda_solve must pass again.
 * Errors: DDA_EINVAL (nothing to save, unreadable or mismatched file), DDA_EHIP.
 */
dda_status dda_checkpoint_save(dda_ctx *ctx, const void *x, const char *path);
dda_status dda_checkpoint_load(dda_ctx *ctx, void *x, const char *path);

/*
 * dda_solve_many — one right-hand side on each of n_ctx particles (contexts), solved together (the
 * paper runs independent orientations or particles as separate simulations, Sec. 2; here they share
 * the GPU): every particle advances on its own stream.  With opts->pack = 1, particles whose
 * contexts share the padded grid, kd and polarizability prescription (homogeneous, not CLDR), one of
 * which spans the others' grid, are packed into one batch instead: each is a right-hand side with
 * its own cell map on the largest grid of the group, so every pass of the product and every solver
 * kernel is one launch over the group (the same sums as each particle's own product, to rounding);
 * a batch runs until its slowest member converges, its converged members' blocks returning at
 * once.  Groups, and particles that fit no group, advance concurrently.  Zero initial guess.
 *   ctxs    host [n_ctx] distinct contexts;  beams  host [n_ctx]
 *   x_out   host [n_ctx] device pointers, each complex128 [3][N_i]
 *   info    host [n_ctx] or NULL
 * opts->precision DDA_FP64 or DDA_FP32_PRODUCT (contexts set up with opts.fp32; particles whose
 * true residual misses tol are finished in double precision one after another).
 * Returns DDA_OK if every particle converged, else the first failing status; DDA_ENOTSUP for
 * DDA_FP32_REFINE or an initial guess.
 */
dda_status dda_solve_many(dda_ctx *const *ctxs, int32_t n_ctx, const dda_beam *beams, double tol,
                          const dda_solve_opts *opts, void *const *x_out, dda_solve_info *info);

/*
 * dda_cross_sections — out = {Cext, Cabs, Csca = Cext - Cabs} in units of d^2 (Sec. 3.1 reports
 * extinction efficiencies; formulas of Draine 1988) from the solution x of beam (device
 * complex128 [3][N]).
 */
dda_status dda_cross_sections(dda_ctx *ctx, const dda_beam *beam, const void *x, double out[3]);

/*
 * dda_farfield — scattering amplitude vectors F(n) = -i k^3 (I - n n) sum_j P_j exp(-i k n.r_j)
 * (far field = exp(ikr)/(-ikr) F) at n_dir unit directions.
 *   dirs   host double [n_dir][3];  F  host complex128 [n_dir][3] (interleaved re, im)
 */
dda_status dda_farfield(dda_ctx *ctx, const dda_beam *beam, const void *x, int32_t n_dir,
                        const double *dirs, double *F);

/*
 * dda_orientation_average — cross sections averaged over particle orientations (the paper's
 * program averages over the Euler angles, Sec. 2).  Orientation R = Rz(alpha) Ry(beta) Rz(gamma);
 * alpha only turns the scattering plane, so the cross sections need beta and gamma: Romberg
 * integration in cos(beta) on 2^n_beta + 1 points, the periodic trapezoid rule on 2^n_gamma points
 * in gamma.  Each orientation is solved for the x and y polarizations of a beam along the
 * laboratory z axis (rotated into the particle frame), as batched right-hand sides of dda_solve.
 *   n_beta 1..10, n_gamma 0..10;  tol, opts as for dda_solve (opts->x0 must be NULL)
 *   out    host {<Cext>, <Cabs>, <Csca>, err}: unpolarized averages (units of d^2) and the Romberg
 *          error estimate of <Cext> (difference of the last two extrapolation columns)
 * Errors: DDA_EINVAL; solver failures are passed on from dda_solve.
 */
dda_status dda_orientation_average(dda_ctx *ctx, int32_t n_beta, int32_t n_gamma, double tol,
                                   const dda_solve_opts *opts, double out[4]);

/*
 * dda_orientation_average_adaptive — the same average with the number of beta values chosen
 * adaptively (the paper's program integrates over the Euler angles by Romberg's method on 2^n + 1
 * points, adaptively, Sec. 2): the cos(beta) grid starts at 2^n_beta_min + 1 points and doubles,
 * solving only the new points, until the Romberg error estimates of <Cext> and <Cabs> are both at
 * most eps <Cext>, or n_beta_max is reached (then the result carries its larger estimates).
 * gamma keeps 2^n_gamma points.
 *   eps > 0; 1 <= n_beta_min <= n_beta_max <= 10; n_gamma 0..10; tol, opts as for dda_solve
 *   (opts->x0 must be NULL)
 *   out          host {<Cext>, <Cabs>, <Csca>, err(<Cext>), err(<Cabs>)}
 *   n_beta_used  host, may be NULL: the level n the result comes from (2^n + 1 beta values)
 * Errors: DDA_EINVAL; solver failures are passed on from dda_solve.
 */
dda_status dda_orientation_average_adaptive(dda_ctx *ctx, double eps, int32_t n_beta_min, int32_t n_beta_max,
                                            int32_t n_gamma, double tol, const dda_solve_opts *opts,
                                            double out[5], int32_t *n_beta_used);

/*
 * dda_orientation_average_mueller — the Mueller matrix (as dda_mueller) averaged over particle
 * orientations (Sec. 2: the Euler angle alpha is averaged through scattering planes, beta and
 * gamma need separate solves).  Turning the particle by alpha about the incident direction turns
 * the scattering plane by -alpha, so each orientation's matrix is averaged over the n_alpha
 * planes phi = 2 pi j / n_alpha; then over the 2^n_gamma equispaced gamma, and Romberg in
 * cos(beta) on 2^n_beta + 1 points, element by element.  Orientations and beams as for
 * dda_orientation_average; the averaged matrix does not depend on the plane.
 *   n_beta 1..10, n_gamma 0..10, n_alpha 1..1024;  tol, opts as for dda_solve (opts->x0 NULL)
 *   theta  host [n_theta] radians, 1 <= n_theta <= 65536
 *   M      host double [n_theta][4][4] row-major (unnormalized, units of d^2 as dda_mueller)
 *   err    host [n_theta] or NULL: Romberg error estimate of the averaged S11 at each angle
 * Errors: DDA_EINVAL; solver and read-out failures are passed on.
 */
dda_status dda_orientation_average_mueller(dda_ctx *ctx, int32_t n_beta, int32_t n_gamma, int32_t n_alpha,
                                           double tol, const dda_solve_opts *opts, const double *theta,
                                           int32_t n_theta, double *M, double *err);

/*
 * dda_asymmetry — out = {Csca, g}: the scattering cross section (units of d^2) and the asymmetry
 * parameter g = <cos theta> from the far field of the solution x (device complex128 [3][N]) of
 * beam, integrated over the sphere of directions: n_theta Gauss-Legendre nodes in cos theta about
 * the propagation direction times n_phi equally spaced azimuths (dCsca/dOmega = |F|^2 / k^2).
 * n_theta or n_phi <= 0: chosen from the band limit of |F|^2 (Legendre degree 2 k R, R the radius
 * of the grid's circumscribing sphere): n_theta = ceil(k R) + 4, n_phi = 2 ceil(k R) + 8.
 * The paper computes g for every sphere (Sec. 3.1) and compares it with Mie theory (Sec. 3.2,
 * Fig. 5) without defining it; this is the usual definition.
 * Errors: DDA_EINVAL for NULL pointers or more than 2^22 directions.
 */
dda_status dda_asymmetry(dda_ctx *ctx, const dda_beam *beam, const void *x, int32_t n_theta, int32_t n_phi,
                         double out[2]);

/*
 * dda_mueller — 4x4 Mueller matrix (Bohren & Huffman eq. 3.16, unnormalized) at n_theta
 * scattering angles in the scattering plane at azimuth phi (Sec. 3.1: all elements in one
 * scattering plane).  The beam frame is e3 = beam->prop, e1 = Re(beam->pol), e2 = e3 x e1;
 * n = sin(theta)(cos(phi) e1 + sin(phi) e2) + cos(theta) e3.
 *   x1     solution for polarization e1 (device complex128 [3][N])
 *   x2     solution for polarization e2, or NULL: then the particle must be invariant under the
 *          90-degree rotation about e3 (checked on the mask; DDA_ESYMMETRY otherwise) and the
 *          second polarization follows from the first (Sec. 3.1: one polarization suffices)
 *   theta  host [n_theta] radians;  M  host double [n_theta][4][4] row-major
 */
dda_status dda_mueller(dda_ctx *ctx, const dda_beam *beam, const void *x1, const void *x2,
                       double phi, const double *theta, int32_t n_theta, double *M);

/*
 * dda_matvec_timed — measurement aid: runs the product of n_rhs vectors (as dda_matvec_batch, or
 * as dda_matvec_f32 per vector when precision = DDA_FP32_REFINE) `reps` times back to back on the
 * context's stream with HIP events around each of its kernels, and returns the mean duration in
 * milliseconds of each kernel launch (kernel_ms[5]: forward x, forward y, z + tensor multiply,
 * inverse y, inverse x) and of a whole product (total_ms).
 *   x, y   device [n_rhs][3][N], complex128 (DDA_FP64) or complex64 (DDA_FP32_REFINE; the context
 *          must have been set up with opts.fp32)
 * Homogeneous contexts only (DDA_ENOTSUP for dda_setup_materials with several materials or
 * CLDR, whose wrapped product runs these same kernels).
 */
dda_status dda_matvec_timed(dda_ctx *ctx, const dda_beam *beams, int32_t n_rhs, int32_t precision,
                            const void *x, void *y, int32_t reps, float kernel_ms[5], float *total_ms);

/*
 * dda_tune — autotuner of the tile schedule of the x and y passes: for the given precision
 * (DDA_FP64 or DDA_FP32_REFINE) it times `reps` products of a batch of n_rhs vectors (the batch
 * size the solves will use) for every admissible number of lines per block (powers of two within
 * the block-size and LDS limits) and keeps, for each axis, the fastest.  tiles_out (optional) receives {lines per block of the x pass, of the y pass}.
 * dda_get_tiles / dda_set_tiles read / impose a schedule (e.g. one cached from an earlier run;
 * DDA_EINVAL for an inadmissible one).  Results of products do not depend on the schedule except
 * through the order of the bilinear-dot partial sums.
 * Homogeneous contexts only (DDA_ENOTSUP otherwise): a schedule tuned on a homogeneous context
 * of the same grid applies unchanged to a wrapped one (dda_set_tiles).
 */
dda_status dda_tune(dda_ctx *ctx, int32_t precision, int32_t n_rhs, int32_t reps, int32_t tiles_out[2]);
dda_status dda_get_tiles(const dda_ctx *ctx, int32_t precision, int32_t tiles[2]);

/*
 * dda_tune_padding — autotuner of the padded grid (any L >= 2n - 1 per axis gives the same product
 * up to rounding, Sec. 2's zero padding): for each candidate, the default choice of dda_setup and
 * the k-th length with compile-time specialized kernels at or above 2n - 1 on every axis
 * (k = 0 .. n_cand - 1), it sets the particle up, tunes its tile schedule for n_rhs vectors
 * (dda_tune), times `reps` double-precision products and keeps the fastest.  Pass pad_out as
 * dda_setup_opts.pad.  Arguments as dda_setup (homogeneous particles); n_cand 1..8; ms_out
 * (optional) receives the winner's product time in milliseconds.  Runs on the default stream;
 * the radix schedule of each length is its compile-time plan.
 * Errors: DDA_EINVAL (bad arguments, or no candidate could be set up), DDA_ENOTSUP, DDA_ENOMEM,
 * DDA_EHIP.
 */
dda_status dda_tune_padding(const int32_t grid[3], const uint8_t *mask, const double m[2], double kd,
                            int32_t polarizability, int32_t n_rhs, int32_t reps, int32_t n_cand, int32_t pad_out[3],
                            float *ms_out);
dda_status dda_set_tiles(dda_ctx *ctx, int32_t precision, const int32_t tiles[2]);

/* ------------------------------------------------------------------ learned initial guess
 * A small 3-D convolutional network supplies QMR's starting vector (the paper's iteration starts
 * from an initial guess it leaves open, Sec. 2; plain QMR from x0 = 0 stays the fallback and the
 * judge of convergence, see dda_solve_opts.x0_check).  The particle is placed at the centre of a
 * G^3 box (G a multiple of 8, each particle grid side <= G).
 *
 * Network, on channels-last tensors [batch][z][y][x][c]:
 *   e0 = relu(conv(f, W0) + b0)         G    16 -> 16     d2 = relu(conv(up(e3), W4) + b4 + e2)  G/4  64 -> 48
 *   e1 = relu(conv(pool(e0), W1) + b1)  G/2  16 -> 32     d1 = relu(conv(up(d2), W5) + b5 + e1)  G/2  48 -> 32
 *   e2 = relu(conv(pool(e1), W2) + b2)  G/4  32 -> 48     d0 = relu(conv(up(d1), W6) + b6 + e0)  G    32 -> 16
 *   e3 = relu(conv(pool(e2), W3) + b3)  G/8  48 -> 64     out = conv(d0, W7) + b7                 G    16 -> 6
 * conv = 3x3x3 zero-padded cross-correlation with W[t][co][ci], t = 9(dz+1) + 3(dy+1) + (dx+1);
 * pool = 2x2x2 mean; up = nearest-neighbour doubling.  Weights are kept as fp32 masters and used as
 * bfloat16; activations and stored gradients are bfloat16; products accumulate in fp32.
 * Parameters (host float32, dda_net_num_params() of them): per layer in order W (27*Cout*Cin,
 * tap-major, then Cout, then Cin) then b (Cout).
 * Features (device bfloat16 [G^3][16]): 0 mask, 1 (Re m - 1) mask, 2 Im m mask, 3 kd, 4..9 Re/Im
 * of E_inc = e exp(i kd a.r) for x, y, z at every box cell (r the particle-frame position of the
 * cell), 10..15 Re/Im of (m^2 - 1) E_inc mask for x, y, z.  Output / target (device float32 [G^3][6]): Re/Im of
 * E_exc - E_inc at the dipoles (E_exc = x / beta, P = beta x, eq. 3); zero elsewhere.
 * Loss: mean over dipole cells of the squared output error summed over the 6 channels.
 */
typedef struct dda_net dda_net;

int64_t dda_net_num_params(void);

/* Network for a G^3 box and batches of up to max_batch particles; params host float32.  Work runs
 * on `stream` (a hipStream_t, NULL = default). */
dda_status dda_net_create(dda_net **out, int32_t grid, int32_t max_batch, const float *params, void *stream);
dda_status dda_net_free(dda_net *net);
/* Replace the parameters (and reset the optimizer state) / read them back (host float32). */
dda_status dda_net_set_params(dda_net *net, const float *params);
dda_status dda_net_get_params(dda_net *net, float *params);

/* Features of the context's particle for one beam into feat (device bfloat16 [G^3][16]). */
dda_status dda_net_features(dda_net *net, dda_ctx *ctx, const dda_beam *beam, void *feat);

/* Training target from a solution x (device complex128 [3][N]) into tgt (device float32 [G^3][6]). */
dda_status dda_net_target(dda_net *net, dda_ctx *ctx, const dda_beam *beam, const void *x, void *tgt);

/* out (device float32 [batch][G^3][6]) = network(feat [batch][G^3][16]). */
dda_status dda_net_forward(dda_net *net, const void *feat, int32_t batch, void *out);

/* Loss of a batch and its gradient (host float32 [num_params] in the parameter layout, or NULL). */
dda_status dda_net_grad(dda_net *net, const void *feat, const void *tgt, int32_t batch, double *loss,
                        float *grad);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on a batch; returns the loss
 * before the step. */
dda_status dda_net_train_step(dda_net *net, const void *feat, const void *tgt, int32_t batch, double lr,
                              double *loss);

/* Initial guesses x0 = beta (E_inc + out) for n_rhs beams on one particle (feat: their features,
 * device bfloat16 [n_rhs][G^3][16]); x0 device complex128 [n_rhs][3][N], ready for
 * dda_solve_opts.x0. */
dda_status dda_guess(dda_ctx *ctx, dda_net *net, const dda_beam *beams, int32_t n_rhs, const void *feat,
                     void *x0);

/* Human-readable name of a status code. */
const char *dda_strerror(dda_status status);

/* Message of the calling thread's most recent call: why it failed, "" if it succeeded (every other
 * entry point clears it on entry). */
const char *dda_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DDA_MI355X_H */
