"""DDA oracle: plain fp64 numpy implementation of what the GPU hot path computes.

TEST INFRASTRUCTURE ONLY.  Used by tests, the smoke check and the benchmark's CPU
baseline; never by the product path.

Conventions (the paper fixes none of these beyond eqs. 1-3; each is a stated reading):
  * Gaussian units, time dependence exp(-i w t), dipole size d = 1, so k stands for kd
    and cross sections come out in units of d^2; incident amplitude |E0| = 1.
  * Dipoles sit at the centres of the non-void cells of a grid centred on the origin;
    the dipole order is the linear cell index x + nx*(y + ny*z) restricted to the mask.
  * A per-dipole vector is an (N, 3) complex array here (the GPU uses [3][N]).

Section/equation references are to the paper unless a literature source is named.
"""
from __future__ import annotations

import math

import numpy as np

# Lattice-dispersion-relation coefficients (Draine & Goodman 1993, the paper's ref. [13];
# the paper names LDR as the polarizability used in all its runs, Sec. 3.1, but does not
# print them).  Pinned by the dispersion relation itself: the k^2 coefficient of the Ewald-
# summed Bloch lattice sum of an infinite cubic lattice (tests/test_oracle_ldr.py).
LDR_B1 = -1.8915316
LDR_B2 = 0.1648469
LDR_B3 = -1.7700004


# ----------------------------------------------------------------------------- lattice
def dipoles(mask):
    """Positions (N, 3) and linear grid indices (N,) of the non-void cells of `mask`.

    `mask` has shape (nz, ny, nx), x fastest.  The paper keeps only non-void dipoles in all
    work except the FFT (Sec. 2); the order here is the grid's linear order.
    pinned by: tests compare counts and positions with brute-force loops on tiny grids.
    """
    mask = np.asarray(mask)
    nz, ny, nx = mask.shape
    lin = np.flatnonzero(mask.reshape(-1))
    ix = lin % nx
    iy = (lin // nx) % ny
    iz = lin // (nx * ny)
    pos = np.stack([ix + 0.5 - nx / 2.0, iy + 0.5 - ny / 2.0, iz + 0.5 - nz / 2.0], axis=1)
    return pos.astype(np.float64), lin.astype(np.int64)


# ---------------------------------------------------------------------- polarizability
def alpha_cm(m):
    """Clausius-Mossotti polarizability of a unit cube: (3/4pi)(m^2-1)/(m^2+2).

    pinned by: alpha = 0 at m = 1; the k -> 0 limit of the LDR polarizability.
    """
    m2 = complex(m) ** 2
    return 3.0 / (4.0 * math.pi) * (m2 - 1.0) / (m2 + 2.0)


def alpha_rr(m, k):
    """Clausius-Mossotti with the radiative-reaction correction (Draine 1988; one of the four
    prescriptions the paper lists, Sec. 2): 1/alpha = 1/alpha_CM - (2/3) i k^3.

    pinned by: the CM limit as k -> 0; a single dipole of real m conserves energy (its extinction
    equals its scattering, computed by the independent double-sum scattering cross section).
    """
    return 1.0 / (1.0 / alpha_cm(m) - (2.0 / 3.0) * 1j * k ** 3)


def ldr_s(prop, pol):
    """S = sum_mu (a_mu |e_mu|)^2 for unit propagation a and unit polarization e.

    Reading: for a complex (e.g. circular) polarization the squared modulus of each
    component is used; for linear polarization this is the usual sum (a_mu e_mu)^2.
    pinned by: test_oracle_ldr.py (the lattice dispersion relation along an axis, S = 0, a face
        diagonal, S = 1/2, and a body diagonal, S = 1/3).
    """
    a = np.asarray(prop, dtype=np.float64)
    e = np.asarray(pol, dtype=np.complex128)
    return float(np.sum(a * a * np.abs(e) ** 2))


def alpha_ldr(m, k, prop, pol):
    """LDR polarizability (Draine & Goodman 1993; the paper uses it for every run, Sec. 3.1).

    1/alpha = 1/alpha_CM + (b1 + m^2 b2 + m^2 b3 S) k^2 - (2/3) i k^3.
    pinned by: the CM limit as k -> 0; Im(1/alpha) = -(2/3) k^3 for real m (radiative
    reaction), which the optical-theorem test checks through the cross sections; the k^2
    coefficient (b1, b2, b3 and S) against the lattice dispersion relation of an infinite cubic
    lattice, its Bloch-mode lattice sum evaluated by Ewald summation (tests/test_oracle_ldr.py).
    """
    m2 = complex(m) ** 2
    S = ldr_s(prop, pol)
    inv = 1.0 / alpha_cm(m) + (LDR_B1 + m2 * LDR_B2 + m2 * LDR_B3 * S) * k * k - (2.0 / 3.0) * 1j * k ** 3
    return 1.0 / inv


def alpha_cldr(m, k, prop):
    """CLDR polarizability (Gutkowicz-Krusin & Draine 2004; one of the prescriptions the paper
    lists, Sec. 2), a diagonal tensor that depends on the propagation direction a only:
    1/alpha_jj = 1/alpha_CM + (b1 + m^2 b2 + m^2 b3 a_j^2) k^2 - (2/3) i k^3, j = x, y, z.
    Returns the three diagonal elements.
    pinned by: the CM limit as k -> 0; for a and the polarization e along lattice axes the
    element along e equals LDR's (a_e = 0 and S = 0); Im(1/alpha_jj) = -(2/3) k^3 for real m; the
    quadratic form on every transverse polarization against the lattice dispersion relation (the
    k^2 coefficient of the Ewald-summed lattice tensor) for a direction off the symmetry axes."""
    m2 = complex(m) ** 2
    a = np.asarray(prop, dtype=np.float64)
    inv = 1.0 / alpha_cm(m) + (LDR_B1 + m2 * LDR_B2 + m2 * LDR_B3 * a * a) * k * k - (2.0 / 3.0) * 1j * k ** 3
    return 1.0 / inv


def beta_of_alpha(alpha):
    """beta with beta*beta = alpha (Sec. 2, text before eq. 2); principal square root.

    pinned by: test_oracle_physics.py::test_inhomogeneous_symmetrized_system_equals_equation_1 and
        test_tensor_polarizability_symmetrized_system_equals_equation_1 (the beta-symmetrized system
        solves eq. 1).
    """
    return np.sqrt(complex(alpha))


def material_alphas(mask, ms, k, prop, pol, polarizability="ldr"):
    """Polarizability of every dipole of an inhomogeneous particle: mask values 1..len(ms) name
    the material of each non-void cell, ms their refractive indices (eq. 1 allows a different
    alpha_i at every dipole; the symmetrized system of eqs. 2-3 then has beta_i = sqrt(alpha_i)).
    Returns (N,) complex in the dipoles' order ((N, 3) diagonal elements for CLDR).
    pinned by: eq. 1 solved directly agrees with the symmetrized system; equal indices give the
    homogeneous particle; a material with m = 1 (alpha = 0 under CM) acts as void cells."""
    _, lin = dipoles(mask)
    mat = np.asarray(mask).reshape(-1)[lin].astype(int) - 1
    per = []
    for m in ms:
        if polarizability == "cm":
            per.append(alpha_cm(m))
        elif polarizability == "rr":
            per.append(alpha_rr(m, k))
        elif polarizability == "cldr":
            per.append(alpha_cldr(m, k, prop))
        else:
            per.append(alpha_ldr(m, k, prop, pol))
    return np.asarray(per, dtype=np.complex128)[mat]  # (N,), or (N, 3) for the tensor CLDR


# ---------------------------------------------------------------------- Green's tensor
def green(r, k):
    """Free-space Green's tensor G(r) of eq. (1): the field at r of a unit dipole at 0.

    G(r) = exp(ikr)/r^3 [k^2 r^2 (I - rr) - (1 - ikr)(I - 3 rr)],  rr = r^ r^ (outer product).
    `r` has shape (..., 3) and must be non-zero; returns (..., 3, 3) complex.
    pinned by: G = (k^2 I + grad grad) exp(ikr)/r checked by finite differences; G = G^T.
    """
    r = np.asarray(r, dtype=np.float64)
    rn = np.sqrt(np.sum(r * r, axis=-1))
    rh = r / rn[..., None]
    rr = rh[..., :, None] * rh[..., None, :]
    eye = np.eye(3)
    kr = np.asarray(k * rn)
    pref = np.exp(1j * kr) / rn ** 3
    t1 = (kr * kr)[..., None, None] * (eye - rr)
    t2 = (1.0 - 1j * kr)[..., None, None] * (eye - 3.0 * rr)
    return pref[..., None, None] * (t1 - t2)


# ------------------------------------------------------------------ interaction matrix
def interaction_matrix(pos, k, beta):
    """Dense A of eq. (2): A_ii = I, A_ij = -beta_i G_ij beta_j, as a (3N, 3N) matrix.

    Row/column index 3*i + mu (dipole i, component mu).  `beta` is a scalar or (N,).
    pinned by: A = A^T exactly; the direct sum below; numpy-FFT convolution on the lattice.
    """
    N = pos.shape[0]
    tensor = np.ndim(beta) == 2  # (N, 3): a diagonal polarizability tensor per dipole (CLDR)
    b = np.asarray(beta, dtype=np.complex128) if tensor else np.broadcast_to(np.asarray(beta, dtype=np.complex128), (N,))
    A = np.zeros((N, 3, N, 3), dtype=np.complex128)
    for i in range(N):
        d = pos[i][None, :] - pos
        d[i] = 1.0  # placeholder, overwritten below
        G = green(d, k)
        G[i] = 0.0
        if tensor:  # A_ij = -diag(beta_i) G_ij diag(beta_j), the product of the betas taken first
            A[i, :, :, :] = -(b[i][:, None, None] * b[None, :, :]) * G.transpose(1, 0, 2)
        else:
            A[i, :, :, :] = -(b[i] * b)[None, :, None] * G.transpose(1, 0, 2)
        A[i, :, i, :] = np.eye(3)
    return A.reshape(3 * N, 3 * N)


def matvec_rows(pos, k, beta, x, rows, chunk=1 << 18):
    """Eq. (3) left-hand side at the dipoles `rows`: y_i = x_i - beta_i sum_{j!=i} G_ij beta_j x_j.

    Direct O(N) sum per row (matrix-free), accumulated over `chunk` dipoles at a time so that
    large particles fit in memory.  x is (N, 3); returns (len(rows), 3).
    pinned by: dense assembly (same rows), numpy-FFT convolution on the lattice.
    """
    N = pos.shape[0]
    b = np.broadcast_to(np.asarray(beta, dtype=np.complex128), (N,))
    out = np.empty((len(rows), 3), dtype=np.complex128)
    for t, i in enumerate(rows):
        s = np.zeros(3, dtype=np.complex128)
        for j0 in range(0, N, chunk):
            j1 = min(N, j0 + chunk)
            d = pos[i][None, :] - pos[j0:j1]
            self_j = i - j0 if j0 <= i < j1 else None
            if self_j is not None:
                d[self_j] = 1.0
            G = green(d, k)
            if self_j is not None:
                G[self_j] = 0.0
            s += np.einsum("jab,jb->a", G, b[j0:j1, None] * x[j0:j1])
        out[t] = x[i] - b[i] * s
    return out


def matvec(pos, k, beta, x, chunk=256):
    """Full direct-sum matvec of eq. (3), processed in row chunks (O(N^2) work).

    pinned by: test_oracle_physics.py::test_direct_sum_equals_dense (row by row) and
        test_direct_sum_equals_library_fft_convolution (numpy FFT convolution on the lattice).
    """
    N = pos.shape[0]
    b = np.broadcast_to(np.asarray(beta, dtype=np.complex128), (N,))
    bx = b[:, None] * x
    y = np.empty_like(x, dtype=np.complex128)
    for s in range(0, N, chunk):
        rows = np.arange(s, min(N, s + chunk))
        ar = np.arange(len(rows))
        d = pos[rows][:, None, :] - pos[None, :, :]
        d[ar, rows] = 1.0          # self pair excluded (j != i in eq. 3)
        G = green(d, k)
        G[ar, rows] = 0.0
        y[rows] = x[rows] - b[rows, None] * np.einsum("ijab,jb->ia", G, bx)
    return y


# ------------------------------------------------------------------- incident field
def incident_field(pos, k, prop, pol, w0=0.0, center=(0.0, 0.0, 0.0)):
    """Incident field at the dipoles (right-hand side of eq. 1): the plane wave
    E_inc(r) = e exp(i k a.r), or for w0 > 0 the focused beam of gaussian_beam_field.

    pinned by: test_oracle_scattering.py::test_single_dipole_is_rayleigh_scatterer (dipole radiation
        pattern of the driven dipole) and test_sphere16_against_mie_and_paper_accuracy (Mie within
        the paper's error envelope).
    """
    if w0 > 0:
        return gaussian_beam_field(pos, k, prop, pol, w0, center)
    a = np.asarray(prop, dtype=np.float64)
    e = np.asarray(pol, dtype=np.complex128)
    ph = np.exp(1j * k * (pos @ a))
    return ph[:, None] * e[None, :]


def gaussian_beam_nodes(k, w0, r_max):
    """Quadrature of the focused beam's angular spectrum over the polar angle t of k^ about the
    axis (|q| = k sin t, so the longitudinal wavenumber k cos t stays smooth up to grazing
    directions): t on [0, t_max], sin t_max = min(1, 12 / (k w0)) (the spectrum exp(-w0^2 |q|^2 / 4)
    is below 3e-16 beyond), Gauss-Legendre with n_t = ceil(k sin(t_max) r_max) + 24 nodes; azimuths
    by the periodic trapezoid rule on n_phi = 2 ceil(k sin(t_max) r_max) + 16 points; r_max bounds
    |r - center| over the dipoles.  Returns (t, weight of t, phi, weight of phi).

    pinned by: test_oracle_physics.py::test_gaussian_beam_quadrature_is_converged and
        test_gaussian_beam_focal_value_closed_form.
    """
    st = min(1.0, 12.0 / (k * w0))
    t_max = math.asin(st)
    kr = int(math.ceil(k * st * r_max))
    n_t, n_phi = kr + 24, 2 * kr + 16
    x, w = np.polynomial.legendre.leggauss(n_t)
    t = 0.5 * t_max * (x + 1.0)
    wt = 0.5 * t_max * w
    phi = 2.0 * math.pi * np.arange(n_phi) / n_phi
    return t, wt, phi, np.full(n_phi, 2.0 * math.pi / n_phi)


def gaussian_beam_field(pos, k, prop, pol, w0, center):
    """A focused beam with waist radius w0 at `center`, propagating along a with polarization e
    (the paper's program can illuminate with tightly focused Gaussian beams, Sec. 2, without
    giving their field): the superposition of propagating plane waves
        E(r) = (w0^2 / 4 pi) int_{|q| < k} exp(-w0^2 |q|^2 / 4) (e - (e.k^) k^) exp(i k k^.(r - c)) d^2q
    over transverse wavevectors q, k^ = (q + sqrt(k^2 - |q|^2) a) / k, i.e. with |q| = k sin t,
    d^2q = k^2 sin t cos t dt dphi.  Each term is a transverse plane wave, so the field solves
    Maxwell's equations exactly; its paraxial limit is the Gaussian beam
    exp(-rho^2 / (w0^2 q)) / q exp(i k z), q = 1 + 2 i z / (k w0^2), and for w0 -> infinity it is
    the plane wave e exp(i k a.(r - c)).  Integrated by gaussian_beam_nodes.
    pinned by: the closed-form value at the focus; divergence-free and Helmholtz by finite
    differences; the plane-wave and paraxial limits; convergence of the quadrature."""
    pos = np.atleast_2d(np.asarray(pos, dtype=np.float64))
    a = np.asarray(prop, dtype=np.float64)
    e = np.asarray(pol, dtype=np.complex128)
    c = np.asarray(center, dtype=np.float64)
    e1 = np.real(e) if np.linalg.norm(np.real(e)) > 1e-8 else np.imag(e)
    e1 = e1 - np.dot(e1, a) * a
    e1 = e1 / np.linalg.norm(e1)
    e2 = np.cross(a, e1)
    rel = pos - c
    r_max = float(np.max(np.linalg.norm(rel, axis=1))) if len(rel) else 0.0
    t, wt, phi, wphi = gaussian_beam_nodes(k, w0, r_max)
    T, PHI = np.meshgrid(t, phi, indexing="ij")
    S, C = np.sin(T), np.cos(T)
    W = np.outer(wt, wphi) * (w0 ** 2 / (4.0 * math.pi)) * np.exp(-0.25 * (w0 * k * S) ** 2) * k * k * S * C
    khat = S[..., None] * (np.cos(PHI)[..., None] * e1 + np.sin(PHI)[..., None] * e2) + C[..., None] * a
    khat = khat.reshape(-1, 3)
    proj = khat @ e  # e . k^ (bilinear)
    vec = W.reshape(-1)[:, None] * (e[None, :] - proj[:, None] * khat)
    ph = np.exp(1j * k * (rel @ khat.T))
    return ph @ vec


def rhs(pos, k, beta, prop, pol, w0=0.0, center=(0.0, 0.0, 0.0)):
    """Right-hand side of eq. (3): b_i = beta_i E_inc,i.

    pinned by: test_oracle_physics.py::test_inhomogeneous_symmetrized_system_equals_equation_1 (b =
        beta E_inc turns eq. 1 into eq. 3).
    """
    N = pos.shape[0]
    if np.ndim(beta) == 2:  # diagonal tensor per dipole
        return np.asarray(beta, dtype=np.complex128) * incident_field(pos, k, prop, pol, w0, center)
    b = np.broadcast_to(np.asarray(beta, dtype=np.complex128), (N,))
    return b[:, None] * incident_field(pos, k, prop, pol, w0, center)


# ---------------------------------------------------------------------------- solvers
def _flat(v):
    """Flat view (bookkeeping, no arithmetic of the method)."""
    return v.reshape(-1)


def qmr(apply_A, b, tol, maxit=100000, x0=None, breakdown_eps=1e-12):
    """Complex-symmetric QMR without look-ahead (Freund 1992, the paper's ref. [16]).

    The paper (Sec. 2) uses QMR and Bi-CG in the form that exploits A = A^T, so one matrix
    product per iteration suffices.  This is the quasi-minimal-residual iteration built on the
    complex-symmetric Lanczos process: Lanczos vectors v scaled to unit Euclidean norm, the
    bilinear form u^T w (no conjugation) in place of an inner product, and the left Lanczos
    vectors equal to the right ones.  Stops when the recursive residual ||r|| / ||b|| < tol
    (the paper's stopping criterion, relative residual norm).

    apply_A maps an (N, 3) array to an (N, 3) array.  Returns (x, info) with info keys
    iters, matvecs, status ('converged' | 'maxit' | 'breakdown'), res_hist (relative recursive
    residual after each iteration, starting with the initial one), res_rec (recursive relative residual at exit).
    pinned by: dense LU on small systems; iterates equal the Lanczos least-squares minimizer.
    """
    shape = b.shape
    bn = np.linalg.norm(_flat(b))
    x = np.zeros(shape, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    nmv = 0
    if x0 is None:
        r = b.astype(np.complex128).copy()
    else:
        r = b - apply_A(x)
        nmv += 1
    hist = [np.linalg.norm(_flat(r)) / bn]
    info = {"iters": 0, "matvecs": nmv, "status": "maxit", "res_hist": hist}
    if hist[-1] < tol:
        info["status"] = "converged"
        info["res_rec"] = hist[-1]
        return x, info

    vt = r.copy()                      # unnormalized Lanczos vector
    rho = np.linalg.norm(_flat(vt))    # its Euclidean norm
    gamma_prev, theta_prev, eta = 1.0, 0.0, -1.0
    eps_prev = None
    p = d = s = None
    for it in range(1, maxit + 1):
        v = vt / rho
        delta = np.dot(_flat(v), _flat(v))          # bilinear v^T v
        if abs(delta) < breakdown_eps:
            info["status"] = "breakdown"
            break
        if it == 1:
            p = v.copy()
        else:
            p = v - (rho * delta / eps_prev) * p
        pt = apply_A(p)
        nmv += 1
        eps = np.dot(_flat(p), _flat(pt))           # bilinear p^T A p
        if eps == 0 or not np.isfinite(eps):
            info["status"] = "breakdown"
            break
        beta = eps / delta
        vt = pt - beta * v
        rho_new = np.linalg.norm(_flat(vt))
        theta = rho_new / (gamma_prev * abs(beta))
        gamma = 1.0 / math.sqrt(1.0 + theta * theta)
        eta = -eta * rho * gamma * gamma / (beta * gamma_prev * gamma_prev)
        c = (theta_prev * gamma) ** 2
        if it == 1:
            d = eta * p
            s = eta * pt
        else:
            d = eta * p + c * d
            s = eta * pt + c * s
        x = x + d
        r = r - s
        rho, gamma_prev, theta_prev, eps_prev = rho_new, gamma, theta, eps
        res = np.linalg.norm(_flat(r)) / bn
        hist.append(res)
        info["iters"] = it
        if res < tol:
            info["status"] = "converged"
            break
        if rho == 0.0:
            info["status"] = "breakdown"
            break
    info["matvecs"] = nmv
    info["res_rec"] = hist[-1]
    return x, info


def bicgstab(apply_A, b, tol, maxit=100000, x0=None):
    """Bi-CGSTAB (van der Vorst 1992; one of the paper's four solvers, Sec. 2).

    Hermitian inner products, shadow residual equal to the initial residual; two matrix
    products per iteration.  Same stopping rule as `qmr`.
    pinned by: dense LU on small systems; agreement with `qmr` on the solution.
    """
    bn = np.linalg.norm(_flat(b))
    x = np.zeros(b.shape, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    nmv = 0
    if x0 is None:
        r = b.astype(np.complex128).copy()
    else:
        r = b - apply_A(x)
        nmv += 1
    hist = [np.linalg.norm(_flat(r)) / bn]
    info = {"iters": 0, "matvecs": nmv, "status": "maxit", "res_hist": hist}
    if hist[-1] < tol:
        info["status"] = "converged"
        info["res_rec"] = hist[-1]
        return x, info
    rs = r.copy()
    rho_old = alpha = omega = 1.0 + 0j
    v = np.zeros_like(r)
    p = np.zeros_like(r)
    for it in range(1, maxit + 1):
        rho = np.vdot(_flat(rs), _flat(r))
        if rho == 0:
            info["status"] = "breakdown"
            break
        beta = (rho / rho_old) * (alpha / omega)
        rho_old = rho
        p = r + beta * (p - omega * v)
        v = apply_A(p)
        nmv += 1
        alpha = rho / np.vdot(_flat(rs), _flat(v))
        s = r - alpha * v
        sn = np.linalg.norm(_flat(s)) / bn
        info["iters"] = it
        if sn < tol:
            x = x + alpha * p
            hist.append(sn)
            info["status"] = "converged"
            break
        t = apply_A(s)
        nmv += 1
        omega = np.vdot(_flat(t), _flat(s)) / np.vdot(_flat(t), _flat(t))
        x = x + alpha * p + omega * s
        r = s - omega * t
        res = np.linalg.norm(_flat(r)) / bn
        hist.append(res)
        if res < tol:
            info["status"] = "converged"
            break
        if omega == 0:
            info["status"] = "breakdown"
            break
    info["matvecs"] = nmv
    info["res_rec"] = hist[-1]
    return x, info


def bicg(apply_A, b, tol, maxit=100000, x0=None):
    """Bi-CG for a complex-symmetric matrix (the paper's Bi-CG, Sec. 2 and its ref. [16]): with
    A^T = A the shadow sequence of Bi-CG equals the conjugate of the primary one, so the method
    needs one product per iteration and runs on the bilinear form u^T v (no conjugation):

        r = b - A x;  p = r;  rho = r^T r
        q = A p;  alpha = rho / p^T q;  x += alpha p;  r -= alpha q
        rho_new = r^T r;  p = r + (rho_new / rho) p

    Same stopping rule as `qmr`; rho = 0 or p^T q = 0 is a breakdown.
    pinned by: dense LU; for a real symmetric positive definite matrix it is conjugate gradients
    (iterates equal scipy's CG step by step); its residuals are conjugate-orthogonal (r_i^T r_j = 0).
    """
    bn = np.linalg.norm(_flat(b))
    x = np.zeros(b.shape, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    nmv = 0
    if x0 is None:
        r = b.astype(np.complex128).copy()
    else:
        r = b - apply_A(x)
        nmv += 1
    hist = [np.linalg.norm(_flat(r)) / bn]
    info = {"iters": 0, "matvecs": nmv, "status": "maxit", "res_hist": hist, "residuals": [r.copy()]}
    if hist[-1] < tol:
        info["status"] = "converged"
        info["res_rec"] = hist[-1]
        return x, info
    p = r.copy()
    rho = np.dot(_flat(r), _flat(r))
    for it in range(1, maxit + 1):
        if rho == 0:
            info["status"] = "breakdown"
            break
        q = apply_A(p)
        nmv += 1
        eps = np.dot(_flat(p), _flat(q))
        if eps == 0:
            info["status"] = "breakdown"
            break
        alpha = rho / eps
        x = x + alpha * p
        r = r - alpha * q
        info["iters"] = it
        res = np.linalg.norm(_flat(r)) / bn
        hist.append(res)
        if len(info["residuals"]) < 16:
            info["residuals"].append(r.copy())
        if res < tol:
            info["status"] = "converged"
            break
        rho_new = np.dot(_flat(r), _flat(r))
        p = r + (rho_new / rho) * p
        rho = rho_new
    info["matvecs"] = nmv
    info["res_rec"] = hist[-1]
    return x, info


def cgnr(apply_A, b, tol, maxit=100000, x0=None):
    """CGNR (the paper's first solver, Sec. 2): conjugate gradients on the normal equations
    A^H A x = A^H b, which minimizes ||b - A x|| over its Krylov space.  A is complex symmetric, so
    A^H v = conj(A conj(v)): two products with A per iteration.

        r = b - A x;  z = A^H r;  p = z;  g = ||z||^2
        w = A p;  alpha = g / ||w||^2;  x += alpha p;  r -= alpha w
        z = A^H r;  g_new = ||z||^2;  p = z + (g_new / g) p

    Same stopping rule as `qmr` on ||r||; g = 0 or w = 0 is a breakdown.
    pinned by: dense LU; its iterates equal scipy's conjugate gradients on A^H A x = A^H b step by
    step; its residual norm never increases.
    """
    def apply_AH(v):
        return np.conj(apply_A(np.conj(v)))

    bn = np.linalg.norm(_flat(b))
    x = np.zeros(b.shape, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    nmv = 0
    if x0 is None:
        r = b.astype(np.complex128).copy()
    else:
        r = b - apply_A(x)
        nmv += 1
    hist = [np.linalg.norm(_flat(r)) / bn]
    info = {"iters": 0, "matvecs": nmv, "status": "maxit", "res_hist": hist}
    if hist[-1] < tol:
        info["status"] = "converged"
        info["res_rec"] = hist[-1]
        return x, info
    z = apply_AH(r)
    nmv += 1
    p = z.copy()
    g = np.vdot(_flat(z), _flat(z)).real
    for it in range(1, maxit + 1):
        if g == 0:
            info["status"] = "breakdown"
            break
        w = apply_A(p)
        nmv += 1
        ww = np.vdot(_flat(w), _flat(w)).real
        if ww == 0:
            info["status"] = "breakdown"
            break
        alpha = g / ww
        x = x + alpha * p
        r = r - alpha * w
        info["iters"] = it
        res = np.linalg.norm(_flat(r)) / bn
        hist.append(res)
        if res < tol:
            info["status"] = "converged"
            break
        z = apply_AH(r)
        nmv += 1
        g_new = np.vdot(_flat(z), _flat(z)).real
        p = z + (g_new / g) * p
        g = g_new
    info["matvecs"] = nmv
    info["res_rec"] = hist[-1]
    return x, info


def solve_dense(pos, k, beta, b):
    """Exact solution of eq. (3) by dense LU (numpy.linalg.solve); for small systems only.

    pinned by: a library routine (numpy.linalg.solve) on the assembled matrix;
        test_oracle_solvers.py checks QMR, Bi-CG, Bi-CGSTAB and CGNR against it.
    """
    A = interaction_matrix(pos, k, beta)
    return np.linalg.solve(A, _flat(b)).reshape(b.shape)


# --------------------------------------------------------------------- cross sections
def cross_sections(pos, k, alpha, P, prop, pol, w0=0.0, center=(0.0, 0.0, 0.0)):
    """Extinction and absorption cross sections from the dipole polarizations P (Draine 1988).

    Cext = 4 pi k sum_i Im(E_inc,i^* . P_i)
    Cabs = 4 pi k sum_i [ -Im(1/alpha_i) - (2/3) k^3 ] |P_i|^2
    Units of d^2.  The paper reports Qext (Sec. 3.1) but does not print these formulas.  For a
    focused beam (w0 > 0) E_inc is its field, normalized to |e| at the focus.
    pinned by: optical theorem Cext = Csca(exact) + Cabs; forward-scattering theorem;
    Cabs = 0 for real m under LDR; agreement with Mie theory.
    """
    E = incident_field(pos, k, prop, pol, w0, center)
    cext = 4.0 * math.pi * k * float(np.sum(np.imag(np.conj(E) * P)))
    if np.ndim(alpha) == 2:  # diagonal tensor per dipole: a weight per component
        w = -np.imag(1.0 / np.asarray(alpha, dtype=np.complex128)) - (2.0 / 3.0) * k ** 3
    else:
        inv = 1.0 / np.broadcast_to(np.asarray(alpha, dtype=np.complex128), (pos.shape[0],))
        w = (-np.imag(inv) - (2.0 / 3.0) * k ** 3)[:, None]
    cabs = 4.0 * math.pi * k * float(np.sum(w * np.abs(P) ** 2))
    return cext, cabs


def csca_exact(pos, k, P):
    """Scattering cross section by the exact double sum over dipole pairs.

    Csca = k^4 sum_ij P_i^H M(r_i - r_j) P_j, M(r) = integral over the unit sphere of
    (I - n n) exp(i k n.r) dOmega = 4 pi [ (2/3 j0 - 1/3 j2)(kr) I + j2(kr) r^ r^ ], M(0) = 8pi/3 I.
    Independent of the far-field route; used only to check the optical theorem.
    pinned by: test_oracle_scattering.py::test_optical_theorem (Cext = Csca + Cabs for the exact
        dense solution).
    """
    N = pos.shape[0]
    tot = 0.0
    for s in range(0, N, 512):
        rows = np.arange(s, min(N, s + 512))
        d = pos[rows][:, None, :] - pos[None, :, :]
        rn = np.sqrt(np.sum(d * d, axis=-1))
        kr = k * rn
        safe = np.where(kr == 0, 1.0, kr)
        j0 = np.sin(safe) / safe
        j1 = np.sin(safe) / safe ** 2 - np.cos(safe) / safe
        j2 = (3.0 / safe ** 2 - 1.0) * j0 - 3.0 * np.cos(safe) / safe ** 2
        j0 = np.where(kr == 0, 1.0, j0)
        j2 = np.where(kr == 0, 0.0, j2)
        rh = d / np.where(rn == 0, 1.0, rn)[..., None]
        c_iso = 4.0 * math.pi * ((2.0 / 3.0) * j0 - (1.0 / 3.0) * j2)
        c_rr = 4.0 * math.pi * j2
        Pj = P[None, :, :]
        iso = np.einsum("ij,ija->ia", c_iso, np.broadcast_to(Pj, d.shape))
        rr = np.einsum("ij,ija,ijb,jb->ia", c_rr, rh, rh, P)
        tot += float(np.real(np.sum(np.conj(P[rows]) * (iso + rr))))
        del j1
    return k ** 4 * tot


# ------------------------------------------------------------------ far field, Mueller
def farfield(pos, k, P, n):
    """Scattering amplitude vector F(n) = -i k^3 (I - n n) sum_j P_j exp(-i k n.r_j).

    The scattered far field is exp(ikr)/(-ikr) F (Bohren & Huffman convention).  `n` is an
    (M, 3) array of unit directions; returns (M, 3).
    pinned by: forward-scattering theorem Cext = (4 pi / k^2) Re(e^* . F(a)); a single dipole
    reproduces Rayleigh scattering in closed form.
    """
    n = np.asarray(n, dtype=np.float64)
    ph = np.exp(-1j * k * (n @ pos.T))      # (M, N)
    s = ph @ P                              # (M, 3)
    s = s - n * np.sum(n * s, axis=1)[:, None]
    return -1j * k ** 3 * s


def sphere_quadrature(prop, n_theta, n_phi):
    """Directions and weights integrating over the unit sphere: Gauss-Legendre in mu = cos(theta)
    about the propagation direction, uniform in phi.  Returns (n (M, 3), w (M,), mu (M,)).

    pinned by:
        test_oracle_physics.py::test_asymmetry_quadrature_reproduces_the_exact_scattering_cross_sect
        ion.
    """
    a = np.asarray(prop, dtype=np.float64)
    a = a / np.linalg.norm(a)
    t = np.array([1.0, 0.0, 0.0]) if abs(a[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(a, t)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(a, e1)
    mu, wmu = np.polynomial.legendre.leggauss(n_theta)
    phi = 2.0 * math.pi * np.arange(n_phi) / n_phi
    M, PH = np.meshgrid(mu, phi, indexing="ij")
    W = np.outer(wmu, np.full(n_phi, 2.0 * math.pi / n_phi))
    st = np.sqrt(1.0 - M ** 2)
    n = (M[..., None] * a + st[..., None] * (np.cos(PH)[..., None] * e1 + np.sin(PH)[..., None] * e2))
    return n.reshape(-1, 3), W.reshape(-1), M.reshape(-1)


def asymmetry(pos, k, P, prop, n_theta, n_phi):
    """Scattering cross section and asymmetry parameter g = <cos theta> by integrating the far field
    over the sphere: dCsca/dOmega = |F|^2 / k^2 (the scattered field is exp(ikr)/(-ikr) F).
    The paper computes g for every sphere (Sec. 3.1) and compares it with Mie theory (Sec. 3.2,
    Fig. 5) without defining it.
    pinned by: Csca equals the exact double sum `csca_exact`; a single dipole scatters with g = 0;
    a sphere's g approaches Mie theory's.
    """
    n, w, mu = sphere_quadrature(prop, n_theta, n_phi)
    F = farfield(pos, k, P, n)
    dc = np.sum(np.abs(F) ** 2, axis=1) / k ** 2
    csca = float(np.sum(w * dc))
    return csca, float(np.sum(w * mu * dc) / csca)


def romberg(fvals, a, b):
    """Romberg integration of samples f(a + i h), i = 0..2^n, h = (b - a) / 2^n: trapezoid sums on
    the nested grids, then Richardson extrapolation.  Returns (integral, |R(n,n) - R(n,n-1)|).
    pinned by: polynomials up to degree 2n + 1 integrate exactly."""
    f = np.asarray(fvals, dtype=np.float64)
    n = int(round(math.log2(len(f) - 1)))
    assert len(f) == 2 ** n + 1
    T = []
    for kk in range(n + 1):
        step = 2 ** (n - kk)
        sub = f[::step]
        h = (b - a) / 2 ** kk
        T.append(h * (np.sum(sub) - 0.5 * (sub[0] + sub[-1])))
    R = [T]
    for j in range(1, n + 1):
        prev = R[-1]
        R.append([prev[i] + (prev[i] - prev[i - 1]) / (4 ** j - 1) for i in range(1, len(prev))])
    best = R[-1][-1]
    err = abs(best - R[-2][-1]) if n >= 1 else float("nan")
    return best, err


def romberg_adaptive(f, a, b, eps, n_min=2, n_max=10):
    """Romberg integration with doubling: f is sampled at a + i h, i = 0..2^n, for n = n_min,
    n_min + 1, ... (a new level evaluates only the new midpoints), until every column's error
    estimate |R(n,n) - R(n,n-1)| is at most eps |R(n,n)| of column 0, or n = n_max.  f maps an
    array of abscissae to an array of rows (one per abscissa).  Returns (integrals per column,
    error estimates per column, n).
    pinned by: closed-form integrals, the level at which polynomials become exact, one evaluation
    per abscissa, the fixed-level rule at the level it stops on."""
    assert 1 <= n_min <= n_max
    n = n_min
    pts = a + (b - a) * np.arange(2 ** n + 1) / 2 ** n
    vals = np.atleast_2d(np.asarray(f(pts), dtype=np.float64).reshape(len(pts), -1))
    while True:
        cols = [romberg(vals[:, q], a, b) for q in range(vals.shape[1])]
        v = np.array([c[0] for c in cols])
        e = np.array([c[1] for c in cols])
        if np.all(e <= eps * abs(v[0])) or n == n_max:
            return v, e, n
        n += 1
        new_idx = np.arange(1, 2 ** n, 2)
        new_vals = np.asarray(f(a + (b - a) * new_idx / 2 ** n), dtype=np.float64).reshape(len(new_idx), -1)
        merged = np.empty((2 ** n + 1, vals.shape[1]))
        merged[0::2] = vals
        merged[1::2] = new_vals
        vals = merged


def _orientation_rows(pos, m, k, mus, n_gamma, polarizability, mask=None):
    """Mean (Cext, Cabs, Csca) over the 2^n_gamma equispaced gamma and the x and y incident
    polarizations, at each cos(beta) in mus.  Orientation R = Ry(beta) Rz(gamma) (alpha = 0); the
    particle-frame beam is R^T applied to the laboratory vectors.

    pinned by: test_oracle_physics.py::test_orientation_average_of_an_isotropic_dipole and
        test_orientation_average_invariant_under_a_lattice_rotation (through orientation_average).
    """
    ng = 2 ** n_gamma
    rows = np.zeros((len(mus), 3))
    for i, mu in enumerate(mus):
        beta_e = math.acos(max(-1.0, min(1.0, mu)))
        c, s = math.cos(beta_e), math.sin(beta_e)
        for j in range(ng):
            gam = 2.0 * math.pi * j / ng
            cg, sg = math.cos(gam), math.sin(gam)
            Ry = np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])
            Rz = np.array([[cg, -sg, 0.0], [sg, cg, 0.0], [0.0, 0.0, 1.0]])
            R = Ry @ Rz
            prop = R.T @ np.array([0.0, 0.0, 1.0])
            for e in (np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])):
                pol = R.T @ e
                if isinstance(m, (list, tuple)):  # several materials: alpha per dipole
                    alpha = material_alphas(mask, m, k, prop, pol, polarizability)
                    bt = np.sqrt(alpha)
                    bx = bt if np.ndim(bt) == 2 else bt[:, None]
                elif polarizability == "cm":
                    alpha = alpha_cm(m)
                    bt = bx = beta_of_alpha(alpha)
                else:
                    alpha = alpha_ldr(m, k, prop, pol)
                    bt = bx = beta_of_alpha(alpha)
                A = interaction_matrix(pos, k, bt)
                b = rhs(pos, k, bt, prop, pol)
                x = np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)
                cext, cabs = cross_sections(pos, k, alpha, bx * x, prop, pol)[:2]
                rows[i] += np.array([cext, cabs, cext - cabs])
    return rows / (2.0 * ng)


def orientation_average(mask, m, k, n_beta, n_gamma, tol=1e-10, polarizability="ldr"):
    """Cross sections averaged over particle orientations (the paper's program averages over the
    Euler angles, Sec. 2).  Orientation R = Rz(alpha) Ry(beta) Rz(gamma); alpha only turns the
    scattering plane, so the cross sections need beta and gamma.  Romberg in cos(beta) on
    2^n_beta + 1 points, the periodic trapezoid rule on 2^n_gamma points in gamma; unpolarized:
    the mean of the x- and y-polarized incident beams, each brought into the particle frame by R^T.
    m may be a list of refractive indices (mask values name the materials).
    Returns ({"Cext", "Cabs", "Csca"} averages, Romberg error estimate of <Cext>).
    pinned by: the Romberg rule on polynomials; a CM single dipole (isotropic) gives its fixed
    value; invariance of the average under a 90-degree lattice rotation of the particle."""
    pos, _ = dipoles(mask)
    nb = 2 ** n_beta + 1
    mus = [-1.0 + 2.0 * i / (nb - 1) for i in range(nb)]
    over_gamma = _orientation_rows(pos, m, k, mus, n_gamma, polarizability, mask)
    out, errs = {}, []
    for q, name in enumerate(("Cext", "Cabs", "Csca")):
        v, e = romberg(over_gamma[:, q], -1.0, 1.0)
        out[name] = v / 2.0
        errs.append(e / 2.0)
    return out, errs[0]


def orientation_average_adaptive(mask, m, k, eps, n_beta_min, n_beta_max, n_gamma, polarizability="ldr"):
    """Orientation average with the number of beta values chosen adaptively (the paper's program
    integrates over the Euler angles by Romberg's method with 2^n + 1 points, adaptively, Sec. 2):
    the cos(beta) grid doubles from 2^n_beta_min + 1 points until the Romberg error estimates of
    <Cext> and <Cabs> are at most eps <Cext>, or n_beta_max is reached; gamma keeps 2^n_gamma
    points (the periodic trapezoid rule).  Returns ({"Cext", "Cabs", "Csca"}, {"Cext", "Cabs"}
    error estimates, n_beta used).
    pinned by: romberg_adaptive's pins and equality with the fixed-level average at the level
    it stops on."""
    pos, _ = dipoles(mask)

    def f(mus):
        return _orientation_rows(pos, m, k, list(mus), n_gamma, polarizability, mask)[:, :2]

    v, e, n = romberg_adaptive(f, -1.0, 1.0, eps, n_beta_min, n_beta_max)
    out = {"Cext": v[0] / 2.0, "Cabs": v[1] / 2.0, "Csca": (v[0] - v[1]) / 2.0}
    return out, {"Cext": e[0] / 2.0, "Cabs": e[1] / 2.0}, n


def orientation_average_mueller(mask, m, k, n_beta, n_gamma, n_alpha, theta, polarizability="ldr"):
    """Mueller matrix averaged over particle orientations (Sec. 2: the average over the Euler
    angle alpha comes from several scattering planes, beta and gamma need separate solves).
    Orientation R = Rz(alpha) Ry(beta) Rz(gamma): turning the particle by alpha about the incident
    direction is the same as turning the scattering plane by -alpha, so for each (beta, gamma) the
    matrix is averaged over the n_alpha equispaced planes phi = 2 pi j / n_alpha (the periodic
    trapezoid rule, the sign of the turn does not matter), over the 2^n_gamma equispaced gamma,
    and integrated by Romberg in cos(beta) on 2^n_beta + 1 points.  The solutions of the x and y
    polarized beams of each orientation give the matrix in every plane.
    Returns ((len(theta), 4, 4) averaged matrix, Romberg error estimate of S11 per angle).
    pinned by: a CM single dipole gives the Rayleigh matrix in closed form; for a particle with a
    mirror plane the eight off-block elements vanish and S21 = S12, S43 = -S34; invariance under a
    lattice rotation of the particle; 2 pi times the integral of S11 sin(theta) / k^2 is <Csca>."""
    pos, _ = dipoles(mask)
    theta = np.asarray(theta, dtype=np.float64)
    nb, ng = 2 ** n_beta + 1, 2 ** n_gamma
    rows = np.zeros((nb, len(theta), 4, 4))
    for i in range(nb):
        mu = -1.0 + 2.0 * i / (nb - 1)
        beta_e = math.acos(max(-1.0, min(1.0, mu)))
        c, s = math.cos(beta_e), math.sin(beta_e)
        for j in range(ng):
            gam = 2.0 * math.pi * j / ng
            cg, sg = math.cos(gam), math.sin(gam)
            Ry = np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])
            Rz = np.array([[cg, -sg, 0.0], [sg, cg, 0.0], [0.0, 0.0, 1.0]])
            R = Ry @ Rz
            prop = R.T @ np.array([0.0, 0.0, 1.0])
            P = []
            for e in (np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])):
                pol = R.T @ e
                alpha = alpha_cm(m) if polarizability == "cm" else alpha_ldr(m, k, prop, pol)
                bt = beta_of_alpha(alpha)
                A = interaction_matrix(pos, k, bt)
                b = rhs(pos, k, bt, prop, pol)
                P.append(bt * np.linalg.solve(A, b.reshape(-1)).reshape(b.shape))
            pol1 = R.T @ np.array([1.0, 0.0, 0.0])
            for a in range(n_alpha):
                rows[i] += mueller(pos, k, prop, pol1, P[0], P[1], theta, 2.0 * math.pi * a / n_alpha)
    rows /= ng * n_alpha
    out = np.zeros((len(theta), 4, 4))
    err = np.zeros(len(theta))
    for t in range(len(theta)):
        for a in range(4):
            for b in range(4):
                v, e = romberg(rows[:, t, a, b], -1.0, 1.0)
                out[t, a, b] = v / 2.0
                if a == 0 and b == 0:
                    err[t] = e / 2.0
    return out, err


def beam_frame(prop, pol):
    """(e1, e2, e3): e3 = propagation, e1 = (real) polarization, e2 = e3 x e1.

    pinned by: test_oracle_scattering.py::test_s11_one_polarization_equals_two and
        test_mueller_formula_equals_the_stokes_transfer_of_the_amplitude_matrix.
    """
    e3 = np.asarray(prop, dtype=np.float64)
    e1 = np.real(np.asarray(pol, dtype=np.complex128))
    e2 = np.cross(e3, e1)
    return e1, e2, e3


def scattering_directions(prop, pol, theta, phi):
    """Directions and unit vectors theta^, phi^ in the scattering plane at azimuth phi.

    pinned by: test_oracle_scattering.py::test_single_dipole_is_rayleigh_scatterer and
        test_symmetry_plane_kills_off_diagonal_blocks.
    """
    e1, e2, e3 = beam_frame(prop, pol)
    th = np.asarray(theta, dtype=np.float64)
    st, ct = np.sin(th), np.cos(th)
    sp, cp = math.sin(phi), math.cos(phi)
    n = np.outer(st * cp, e1) + np.outer(st * sp, e2) + np.outer(ct, e3)
    t_hat = np.outer(ct * cp, e1) + np.outer(ct * sp, e2) - np.outer(st, e3)
    p_hat = np.broadcast_to(-sp * e1 + cp * e2, n.shape)
    return n, t_hat, p_hat


def amplitude_matrix(F1, F2, t_hat, p_hat, phi):
    """S1..S4 (Bohren & Huffman) from far fields F1, F2 of incident polarizations e1, e2.

    Incident parallel/perpendicular to the scattering plane: e_par = cos(phi) e1 + sin(phi) e2,
    e_perp = sin(phi) e1 - cos(phi) e2; by linearity F_par, F_perp follow from F1, F2.
    S2 = theta^.F_par, S4 = -phi^.F_par, S3 = theta^.F_perp, S1 = -phi^.F_perp.
    pinned by: test_oracle_scattering.py::test_mueller_formula_equals_the_stokes_transfer_of_the_amp
        litude_matrix and test_forward_scattering_theorem.
    """
    cp, sp = math.cos(phi), math.sin(phi)
    Fpar = cp * F1 + sp * F2
    Fperp = sp * F1 - cp * F2
    S2 = np.sum(t_hat * Fpar, axis=1)
    S4 = -np.sum(p_hat * Fpar, axis=1)
    S3 = np.sum(t_hat * Fperp, axis=1)
    S1 = -np.sum(p_hat * Fperp, axis=1)
    return S1, S2, S3, S4


def mueller_from_amplitudes(S1, S2, S3, S4):
    """4x4 Mueller matrix from the amplitude matrix (Bohren & Huffman 1983, eq. 3.16).

    Returns (M, 4, 4), unnormalized (S11 = (|S1|^2+|S2|^2+|S3|^2+|S4|^2)/2).
    pinned by: Rayleigh single-dipole closed form; S12 = S21 = -S11 sin^2/(1+cos^2) there.
    """
    a1, a2, a3, a4 = (np.abs(S) ** 2 for S in (S1, S2, S3, S4))
    M = np.empty(S1.shape + (4, 4))
    M[..., 0, 0] = 0.5 * (a2 + a1 + a4 + a3)
    M[..., 0, 1] = 0.5 * (a2 - a1 + a4 - a3)
    M[..., 0, 2] = np.real(S2 * np.conj(S3) + S1 * np.conj(S4))
    M[..., 0, 3] = np.imag(S2 * np.conj(S3) - S1 * np.conj(S4))
    M[..., 1, 0] = 0.5 * (a2 - a1 - a4 + a3)
    M[..., 1, 1] = 0.5 * (a2 + a1 - a4 - a3)
    M[..., 1, 2] = np.real(S2 * np.conj(S3) - S1 * np.conj(S4))
    M[..., 1, 3] = np.imag(S2 * np.conj(S3) + S1 * np.conj(S4))
    M[..., 2, 0] = np.real(S2 * np.conj(S4) + S1 * np.conj(S3))
    M[..., 2, 1] = np.real(S2 * np.conj(S4) - S1 * np.conj(S3))
    M[..., 2, 2] = np.real(S1 * np.conj(S2) + S3 * np.conj(S4))
    M[..., 2, 3] = np.imag(S2 * np.conj(S1) + S4 * np.conj(S3))
    M[..., 3, 0] = np.imag(S4 * np.conj(S2) + S1 * np.conj(S3))
    M[..., 3, 1] = np.imag(S4 * np.conj(S2) - S1 * np.conj(S3))
    M[..., 3, 2] = np.imag(S1 * np.conj(S2) - S3 * np.conj(S4))
    M[..., 3, 3] = np.real(S1 * np.conj(S2) - S3 * np.conj(S4))
    return M


def rotation_about(axis, angle):
    """Rotation matrix by `angle` about the unit vector `axis` (Rodrigues).

    pinned by: test_oracle_physics.py::test_orientation_average_invariant_under_a_lattice_rotation.
    """
    a = np.asarray(axis, dtype=np.float64)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def mueller(pos, k, prop, pol, P1, P2, theta, phi):
    """Mueller matrix in the scattering plane at azimuth phi, from the polarizations P1 (incident
    polarization e1) and P2 (incident polarization e2 = prop x e1).

    If P2 is None, the particle is assumed invariant under a 90-degree rotation about the
    propagation direction (the paper uses the sphere's symmetry to run one polarization only,
    Sec. 3.1): then F2(n) = R F1(R^-1 n) with R the +90-degree rotation taking e1 to e2.
    Returns (len(theta), 4, 4).
    pinned by: test_oracle_scattering.py::test_mueller_formula_equals_the_stokes_transfer_of_the_amp
        litude_matrix (Stokes definitions), test_single_dipole_is_rayleigh_scatterer and
        test_sphere16_against_mie_and_paper_accuracy (every element against Mie).
    """
    n, t_hat, p_hat = scattering_directions(prop, pol, theta, phi)
    F1 = farfield(pos, k, P1, n)
    if P2 is not None:
        F2 = farfield(pos, k, P2, n)
    else:
        R = rotation_about(np.asarray(prop, dtype=np.float64), math.pi / 2)
        F2 = farfield(pos, k, P1, n @ R) @ R.T   # rows: R F1(R^T n)
    S1, S2, S3, S4 = amplitude_matrix(F1, F2, t_hat, p_hat, phi)
    return mueller_from_amplitudes(S1, S2, S3, S4)


def efficiency(C, n_dipoles):
    """Q = C / (pi a_eq^2), a_eq = (3N/4pi)^(1/3) d (volume-equivalent radius, Sec. 3.1).

    pinned by: test_oracle_scattering.py::test_sphere16_against_mie_and_paper_accuracy (Qext against
        Mie within the paper's envelope).
    """
    a_eq = (3.0 * n_dipoles / (4.0 * math.pi)) ** (1.0 / 3.0)
    return C / (math.pi * a_eq * a_eq)


def size_parameter(k, n_dipoles):
    """Volume-equivalent size parameter x = k a_eq.

    pinned by: test_oracle_scattering.py::test_sphere16_against_mie_and_paper_accuracy.
    """
    return k * (3.0 * n_dipoles / (4.0 * math.pi)) ** (1.0 / 3.0)
