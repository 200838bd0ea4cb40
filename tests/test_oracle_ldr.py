"""Pins of the LDR and CLDR polarizabilities against the lattice dispersion relation they come
from (the paper uses LDR for every run, Sec. 3.1, and lists CLDR among its prescriptions, Sec. 2,
without printing either).

An infinite simple cubic lattice (spacing d = 1) of point dipoles with polarizability alpha carries
a Bloch mode P_j = P_0 exp(i q.r_j) without incident field when P_0 / alpha = S(q, k) P_0 with the
lattice sum S(q, k) = sum_{j != 0} G(r_j) exp(i q.r_j) (eq. 1 of the paper with E_inc = 0).  LDR
asks that the lattice propagate transverse waves with the continuum's wavevector q = m k a, so for
a transverse polarization e: 1/alpha = e.S(m k a, k).e.  The sum converges only conditionally; it
is evaluated here by Ewald's split of exp(ikR)/R into a short-range part summed over the lattice
(complementary error functions) and a smooth part summed over the reciprocal lattice (Gaussian
damping), with G = (k^2 + grad grad) exp(ikr)/r applied term by term.  Expanded in k at fixed m,
e.S.e = 4 pi/(m^2 - 1) + 4 pi/3 + (b1 + m^2 b2 + m^2 b3 sum_mu a_mu^2 e_mu^2) k^2 - (2/3) i k^3 + ...
(the first two terms are 1/alpha_CM), which defines LDR's three coefficients; the same expansion
of the full tensor, restricted to its diagonal, is CLDR.

The Ewald sum is checked first on its own: independence of the splitting parameter, and a lossy
wavenumber for which the plain lattice sum converges absolutely.
"""
import math

import numpy as np
import pytest
from scipy.special import erf, erfc

from oracle import dda


def _lattice(nmax):
    r = np.arange(-nmax, nmax + 1)
    return np.array(np.meshgrid(r, r, r, indexing="ij")).reshape(3, -1).T.astype(np.float64)


def lattice_tensor(q, k, eta=2.0, nmax=6):
    """S(q, k) = sum_{j != 0} G(r_j) exp(i q.r_j) on the unit cubic lattice by Ewald summation
    (3 x 3 complex).  k may be complex (Im k > 0)."""
    q = np.asarray(q, dtype=np.float64)
    k = complex(k)
    n = _lattice(nmax)
    # reciprocal-lattice part: 4 pi sum_G F_G (k^2 I - p p), p = q + 2 pi n,
    # F_G = exp(-(p^2 - k^2) / (4 eta^2)) / (p^2 - k^2)
    p = q[None, :] + 2.0 * math.pi * n
    p2 = np.sum(p * p, axis=1)
    F = np.exp(-(p2 - k * k) / (4.0 * eta * eta)) / (p2 - k * k)
    S = 4.0 * math.pi * (k * k * np.sum(F) * np.eye(3) - np.einsum("g,ga,gb->ab", F, p, p))
    # direct-lattice part over j != 0: Hessian and value of the short-range radial function
    # g_s(R) = [exp(ikR) erfc(eta R + ib) + exp(-ikR) erfc(eta R - ib)] / (2R), b = k / (2 eta)
    r = n[np.any(n != 0, axis=1)]
    R = np.linalg.norm(r, axis=1)
    b = k / (2.0 * eta)
    up = np.exp(1j * k * R) * erfc(eta * R + 1j * b)
    um = np.exp(-1j * k * R) * erfc(eta * R - 1j * b)
    w = 2.0 * eta / math.sqrt(math.pi) * np.exp(b * b - eta * eta * R * R)
    U = up + um
    U1 = 1j * k * (up - um) - 2.0 * w
    U2 = -k * k * U + 4.0 * eta * eta * R * w
    g0 = U / (2 * R)
    g1 = U1 / (2 * R) - U / (2 * R * R)
    g2 = U2 / (2 * R) - U1 / (R * R) + U / R ** 3
    rh = r / R[:, None]
    ph = np.exp(1j * (r @ q))
    iso = ph * (k * k * g0 + g1 / R)
    ani = ph * (g2 - g1 / R)
    S += np.sum(iso) * np.eye(3) + np.einsum("j,ja,jb->ab", ani, rh, rh)
    # the j = 0 term minus the singular exp(ikr)/r: -(g_long) with g_long(R) = c0 + c2 R^2 + ...
    e0 = erf(1j * b)
    D = 2.0 / math.sqrt(math.pi) * np.exp(b * b)
    c0 = 1j * k * (1 + e0) + D * eta
    c2 = -(1j * k ** 3 * (1 + e0) + D * (k * k * eta + 2 * eta ** 3)) / 6.0
    S -= (k * k * c0 + 2.0 * c2) * np.eye(3)
    return S


def test_ewald_sum_does_not_depend_on_the_split():
    q, k = np.array([0.1, 0.25, 0.3]), 0.2
    ref = lattice_tensor(q, k, eta=2.0)
    for eta in (1.5, 2.5, 3.0):
        assert np.abs(lattice_tensor(q, k, eta=eta, nmax=7) - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(lattice_tensor(q, k, nmax=9) - ref).max() < 1e-13 * np.abs(ref).max()


def test_ewald_sum_equals_the_plain_sum_for_a_lossy_wavenumber():
    # with Im k > 0 every term decays like exp(-Im k r) and the plain sum converges absolutely
    q, k = np.array([0.3, -0.1, 0.2]), 0.5 + 0.8j
    n = _lattice(30)
    r = n[np.any(n != 0, axis=1)]
    G = dda.green(r, k)   # (M, 3, 3)
    direct = np.einsum("j,jab->ab", np.exp(1j * (r @ q)), G)
    ew = lattice_tensor(q, k)
    assert np.abs(direct - ew).max() < 1e-9 * np.abs(ew).max()


def _coefficient(m, a, e, ks=(0.02, 0.04)):
    """k^2 coefficient of Re e.S(m k a, k).e - 1/alpha_CM, Richardson-extrapolated in k^2."""
    e = np.asarray(e, dtype=np.float64)
    c = []
    for k in ks:
        s = e @ lattice_tensor(m * k * np.asarray(a, dtype=np.float64), k) @ e
        c.append((s.real - (1.0 / dda.alpha_cm(m)).real) / k ** 2)
    r = (ks[1] / ks[0]) ** 2
    return (r * c[0] - c[1]) / (r - 1.0)


_AXIS = ((0.0, 0.0, 1.0), (1.0, 0.0, 0.0))
_FACE = (tuple(np.array([1.0, 1.0, 0.0]) / math.sqrt(2)), tuple(np.array([1.0, -1.0, 0.0]) / math.sqrt(2)))
_BODY = (tuple(np.array([1.0, 1.0, 1.0]) / math.sqrt(3)), tuple(np.array([1.0, -1.0, 0.0]) / math.sqrt(2)))


@pytest.mark.parametrize("m", [1.5, 2.0, 3.0])
@pytest.mark.parametrize("a,e", [_AXIS, _FACE, _BODY])
def test_ldr_is_the_lattice_dispersion_relation(m, a, e):
    """The oracle's LDR (its three coefficients and S) equals the lattice's k^2 coefficient for
    propagation along an axis (S = 0), a face diagonal (S = 1/2) and a body diagonal (S = 1/3):
    a wrong digit in b1..b3 (units of 1e-7 are printed) or a sign slip moves it by >= 1e-6 x m^2."""
    k = 0.05
    ldr = ((1.0 / dda.alpha_ldr(m, k, a, e)).real - (1.0 / dda.alpha_cm(m)).real) / k ** 2
    assert abs(_coefficient(m, a, e) - ldr) < 4e-7 * m * m


def test_ldr_coefficients_solved_from_the_lattice():
    # b1 + m^2 b2 + m^2 S b3 at (m, S) = (1.5, 0), (2, 0), (2, 1/2): three equations
    rows, rhs = [], []
    for m, (a, e), S in ((1.5, _AXIS, 0.0), (2.0, _AXIS, 0.0), (2.0, _FACE, 0.5)):
        rows.append([1.0, m * m, m * m * S])
        rhs.append(_coefficient(m, a, e))
    b = np.linalg.solve(np.array(rows), np.array(rhs))
    assert np.abs(b - np.array([dda.LDR_B1, dda.LDR_B2, dda.LDR_B3])).max() < 1e-6


def test_radiative_term_is_exact_for_the_lattice():
    # Im e.S.e = -(2/3) k^3 for real m (no diffracted orders: |q| > k), the LDR's last term
    for m, k in ((1.5, 0.1), (2.0, 0.3)):
        a, e = np.array(_BODY[0]), np.array(_BODY[1])
        s = e @ lattice_tensor(m * k * a, k) @ e
        assert abs(s.imag + 2.0 / 3.0 * k ** 3) < 1e-13
        assert abs((1.0 / dda.alpha_ldr(m, k, a, e)).imag + 2.0 / 3.0 * k ** 3) < 1e-15


def test_cldr_is_the_diagonal_of_the_lattice_tensor():
    """CLDR: for a direction off every symmetry axis, the quadratic form of 1/alpha_CLDR on every
    transverse polarization has the lattice's k^2 coefficient (the tensor's off-diagonal parts
    vanish on transverse polarizations), where LDR's scalar matches only its own polarization."""
    rng = np.random.default_rng(7)
    a = rng.standard_normal(3)
    a /= np.linalg.norm(a)
    t1 = np.cross(a, [0.0, 0.0, 1.0])
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(a, t1)
    k, m = 0.05, 2.0
    inv_cldr = 1.0 / dda.alpha_cldr(m, k, a)
    for ang in (0.0, 0.7, 2.1):
        e = math.cos(ang) * t1 + math.sin(ang) * t2
        cl = ((e * e) @ inv_cldr).real
        coef = (cl - (1.0 / dda.alpha_cm(m)).real) / k ** 2
        assert abs(_coefficient(m, a, e) - coef) < 4e-7 * m * m
