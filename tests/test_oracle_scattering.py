"""Pins of the oracle's read-out (cross sections, far field, Mueller) and of Mie theory.

Invariants of the discrete system (optical and forward-scattering theorems), closed forms
(Rayleigh dipole), the worked example Bohren & Huffman print for BHMIE, and the accuracy
statements of the paper (tests/golden/)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import dda, mie
from paper_0704_0037_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _solve(n, m, k, prop=(0, 0, 1), pol=(1, 0, 0), mask=None):
    mask = inputs.sphere_mask(n) if mask is None else mask
    pos, _ = dda.dipoles(mask)
    alpha = dda.alpha_ldr(m, k, prop, pol)
    beta = dda.beta_of_alpha(alpha)
    b = dda.rhs(pos, k, beta, prop, pol)
    x = dda.solve_dense(pos, k, beta, b)
    return pos, alpha, beta, x, beta * x


# ----------------------------------------------------------------------- cross sections
@pytest.mark.parametrize("m,k", [(1.5, 0.5), (1.33 + 0.1j, 0.6), (2.0 + 0.5j, 0.4)])
def test_optical_theorem(m, k):
    pos, alpha, beta, x, P = _solve(8, m, k)
    cext, cabs = dda.cross_sections(pos, k, alpha, P, (0, 0, 1), (1, 0, 0))
    csca = dda.csca_exact(pos, k, P)
    assert abs(cext - (csca + cabs)) < 1e-9 * cext
    if complex(m).imag == 0:
        assert abs(cabs) < 1e-12 * cext
    else:
        assert cabs > 0


def test_forward_scattering_theorem():
    pos, alpha, beta, x, P = _solve(8, 1.4 + 0.02j, 0.55)
    cext, _ = dda.cross_sections(pos, 0.55, alpha, P, (0, 0, 1), (1, 0, 0))
    F = dda.farfield(pos, 0.55, P, np.array([[0.0, 0.0, 1.0]]))
    assert abs(4 * math.pi / 0.55 ** 2 * F[0, 0].real - cext) < 1e-12 * cext


def test_single_dipole_is_rayleigh_scatterer():
    """One dipole: P = alpha E, S1 = -i k^3 alpha, S2 = -i k^3 alpha cos(theta)."""
    mask = np.ones((1, 1, 1), dtype=np.uint8)
    pos, _ = dda.dipoles(mask)
    k, m = 0.3, 1.5
    alpha = dda.alpha_ldr(m, k, (0, 0, 1), (1, 0, 0))
    P = alpha * dda.incident_field(pos, k, (0, 0, 1), (1, 0, 0))
    th = np.linspace(0, math.pi, 19)
    M = dda.mueller(pos, k, (0, 0, 1), (1, 0, 0), P, None, th, 0.0)
    a2 = abs(k ** 3 * alpha) ** 2
    c = np.cos(th)
    np.testing.assert_allclose(M[:, 0, 0], a2 * (1 + c * c) / 2, rtol=1e-13)
    np.testing.assert_allclose(M[:, 0, 1], a2 * (c * c - 1) / 2, rtol=0, atol=1e-13 * a2)
    np.testing.assert_allclose(M[:, 2, 2], a2 * c, rtol=0, atol=1e-13 * a2)
    # S44 = S33 and S34 = S43 = 0: the dipole's S1 and S2 are in phase
    np.testing.assert_allclose(M[:, 3, 3], a2 * c, rtol=0, atol=1e-13 * a2)
    np.testing.assert_allclose(M[:, 2, 3], 0.0, rtol=0, atol=1e-13 * a2)
    np.testing.assert_allclose(M[:, 3, 2], 0.0, rtol=0, atol=1e-13 * a2)


def _stokes(Epar, Eperp):
    """Stokes vector of a field from its components parallel and perpendicular to the scattering
    plane, by the definitions of Bohren & Huffman (eq. 2.84): I = |E_par|^2 + |E_perp|^2,
    Q = |E_par|^2 - |E_perp|^2, U = E_par E_perp^* + E_perp E_par^*, V = i (E_par E_perp^* - E_perp E_par^*)."""
    a = Epar * np.conj(Eperp)
    return np.array([abs(Epar) ** 2 + abs(Eperp) ** 2, abs(Epar) ** 2 - abs(Eperp) ** 2,
                     (a + np.conj(a)).real, (1j * (a - np.conj(a))).real])


def test_mueller_formula_equals_the_stokes_transfer_of_the_amplitude_matrix():
    """Every element of the Mueller matrix formula, checked against its meaning: the scattered
    field is (E_par, E_perp)_s = [[S2, S3], [S4, S1]] (E_par, E_perp)_i (Bohren & Huffman eq. 3.12,
    common factor dropped), and the Mueller matrix maps the incident Stokes vector to the scattered
    one.  Four incident states (parallel, perpendicular, +45 degrees, circular) give its four
    columns; generic amplitudes leave no element zero."""
    rng = np.random.default_rng(11)
    S1, S2, S3, S4 = (rng.standard_normal(6) + 1j * rng.standard_normal(6) for _ in range(4))
    M = dda.mueller_from_amplitudes(S1, S2, S3, S4)
    states = [(1.0, 0.0), (0.0, 1.0), (1 / math.sqrt(2), 1 / math.sqrt(2)), (1 / math.sqrt(2), 1j / math.sqrt(2))]
    for q in range(6):
        Si = np.array([_stokes(complex(a), complex(b)) for a, b in states]).T          # columns: incident
        Ss = np.array([_stokes(S2[q] * a + S3[q] * b, S4[q] * a + S1[q] * b) for a, b in states]).T
        ref = Ss @ np.linalg.inv(Si)
        assert np.abs(M[q] - ref).max() < 1e-12 * np.abs(ref).max()


def test_s11_one_polarization_equals_two():
    """Particle symmetric under 90-degree rotation about z: x-pol alone gives the whole matrix."""
    pos, alpha, beta, x1, P1 = _solve(8, 1.5, 0.5, pol=(1, 0, 0))
    _, alpha2, _, x2, P2 = _solve(8, 1.5, 0.5, pol=(0, 1, 0))
    th = np.radians(np.arange(0, 181, 5.0))
    for phi in (0.0, math.pi / 2, 0.3):
        M1 = dda.mueller(pos, 0.5, (0, 0, 1), (1, 0, 0), P1, None, th, phi)
        M2 = dda.mueller(pos, 0.5, (0, 0, 1), (1, 0, 0), P1, P2, th, phi)
        assert np.abs(M1 - M2).max() < 1e-10 * np.abs(M2).max()


def test_symmetry_plane_kills_off_diagonal_blocks():
    pos, alpha, beta, x, P = _solve(8, 1.5, 0.5)
    th = np.radians(np.arange(0, 181, 3.0))
    M = dda.mueller(pos, 0.5, (0, 0, 1), (1, 0, 0), P, None, th, 0.0)
    scale = np.abs(M[:, 0, 0]).max()
    for (i, j) in [(0, 2), (0, 3), (1, 2), (1, 3), (2, 0), (2, 1), (3, 0), (3, 1)]:
        assert np.abs(M[:, i, j]).max() < 1e-10 * scale


# -------------------------------------------------------------------------------- Mie
def test_mie_bhmie_printed_example():
    g = json.load(open(os.path.join(GOLDEN, "bhmie_example.json")))
    inp, pr = g["input"], g["printed"]
    x = 2 * math.pi * inp["radius"] * inp["medium_index"] / inp["wavelength"]
    m = complex(*inp["m"]) / inp["medium_index"]
    qext, qsca, _ = mie.efficiencies(x, m)
    S1, _ = mie.amplitudes(x, m, np.array([math.pi]))
    qback = 4 * abs(S1[0]) ** 2 / x ** 2
    tol = 0.5 * 10 ** (-g["digits"])
    assert abs(qext - pr["Qext"]) <= tol
    assert abs(qsca - pr["Qsca"]) <= tol
    assert abs(qback - pr["Qback"]) <= tol
    assert abs(mie.asymmetry(x, m) - pr["g"]) <= tol


def test_mie_rayleigh_limit():
    for m in (1.5, 1.33 + 0.2j):
        x = 0.01
        pol = (m * m - 1) / (m * m + 2)
        qext, qsca, qabs = mie.efficiencies(x, m)
        assert abs(qsca / (8 / 3 * x ** 4 * abs(pol) ** 2) - 1) < 1e-3
        if complex(m).imag:
            assert abs(qabs / (4 * x * pol.imag) - 1) < 1e-3


def test_mie_energy_and_forward_theorem():
    for x, m in [(3.368, 1.5), (20.0, 1.05), (8.0, 2.0), (5.0, 1.6 + 0.05j)]:
        qext, qsca, qabs = mie.efficiencies(x, m)
        S1, S2 = mie.amplitudes(x, m, np.array([0.0]))
        assert abs(4 / x ** 2 * S1[0].real - qext) < 1e-10 * qext
        assert abs(S1[0] - S2[0]) < 1e-10 * abs(S1[0])
        if complex(m).imag == 0:
            assert abs(qabs) < 1e-10 * qext
        else:
            assert qabs > 0


def test_mie_mueller_rayleigh_limit_and_single_amplitude_pair_identity():
    th = np.radians(np.arange(0.0, 181.0, 5.0))
    c = np.cos(th)
    M = mie.mueller(1e-3, 1.5, th)  # corrections to the dipole are O(x^2)
    s11 = M[:, 0, 0]
    np.testing.assert_allclose(M[:, 0, 1] / s11, -(1 - c * c) / (1 + c * c), rtol=0, atol=1e-6)
    np.testing.assert_allclose(M[:, 2, 2] / s11, 2 * c / (1 + c * c), rtol=0, atol=1e-6)
    np.testing.assert_allclose(M[:, 3, 3], M[:, 2, 2], rtol=0, atol=0)
    assert np.abs(M[:, 2, 3] / s11).max() < 1e-6
    # one amplitude pair: a pure Mueller matrix, S11^2 = S12^2 + S33^2 + S34^2 at every angle
    for x, m in [(3.368, 1.5), (6.0, 1.33 + 0.1j)]:
        M = mie.mueller(x, m, th)
        lhs = M[:, 0, 0] ** 2
        rhs = M[:, 0, 1] ** 2 + M[:, 2, 2] ** 2 + M[:, 2, 3] ** 2
        assert np.abs(lhs - rhs).max() < 1e-12 * lhs.max()
        assert np.abs(M[:, 2, 3] / M[:, 0, 0]).max() > 0.2  # S34 is far from zero here
        # the general amplitude-matrix formula with S3 = S4 = 0 gives the same matrix
        S1, S2 = mie.amplitudes(x, m, th)
        G = dda.mueller_from_amplitudes(S1, S2, np.zeros_like(S1), np.zeros_like(S1))
        assert np.abs(G - M).max() < 1e-12 * M[:, 0, 0].max()


def test_mie_extinction_paradox():
    # geometric-optics limit Qext -> 2, approached like x^(-2/3) (edge term)
    q400 = mie.efficiencies(400.0, 1.33)[0]
    q4000 = mie.efficiencies(4000.0, 1.33)[0]
    assert 2.0 < q400 < 2.0 + 2.5 * 400.0 ** (-2 / 3)
    assert 2.0 < q4000 < 2.0 + 2.5 * 4000.0 ** (-2 / 3)


# ----------------------------------------------------------------------- DDA vs Mie
def test_sphere16_against_mie_and_paper_accuracy():
    """The 16^3 sphere (lambda/(m d) = 10, x < 10) against Mie and the paper's error statements."""
    acc = json.load(open(os.path.join(GOLDEN, "paper_accuracy.json")))
    w = inputs.c1_sphere16()
    pos, _ = dda.dipoles(w.mask)
    k = w.kd
    alpha = dda.alpha_ldr(w.m, k, (0, 0, 1), (1, 0, 0))
    beta = dda.beta_of_alpha(alpha)
    A = dda.interaction_matrix(pos, k, beta)
    b = dda.rhs(pos, k, beta, (0, 0, 1), (1, 0, 0))
    x, info = dda.qmr(lambda v: (A @ v.reshape(-1)).reshape(v.shape), b, w.tol)
    assert info["status"] == "converged"
    P = beta * x
    cext, cabs = dda.cross_sections(pos, k, alpha, P, (0, 0, 1), (1, 0, 0))
    xe = dda.size_parameter(k, len(pos))
    assert xe < 10 and abs(2 * math.pi / (w.m.real * k) - 10) < 0.01
    qext_mie = mie.efficiencies(xe, w.m)[0]
    err_q = abs(dda.efficiency(cext, len(pos)) / qext_mie - 1)
    assert err_q < acc["qext_rel_error_range"]["max"]
    th = np.radians(np.arange(181.0))
    M = dda.mueller(pos, k, (0, 0, 1), (1, 0, 0), P, None, th, 0.0)
    rel = M[:, 0, 0] / mie.s11(xe, w.m, th) - 1
    assert np.abs(rel).max() < acc["small_particles_s11_max_rel_error"]["value"]
    assert math.sqrt(np.mean(rel ** 2)) < acc["s11_rms_rel_error_range"]["max"]
    assert abs(cabs) < 1e-12 * cext
    # the other elements of the matrix (Sec. 3.1: all Mueller elements in one plane are compared
    # with Mie theory): each within the paper's S11 bound relative to S11 (every element is at most
    # S11 in size), and of Mie's sign wherever Mie's element is a quarter of S11 or more.  A sign
    # slip in S34 or S44 would miss by up to 0.9 and 2 S11 here.
    Mm = mie.mueller(xe, w.m, th)
    s11 = Mm[:, 0, 0]
    for i in range(4):
        for j in range(4):
            d = np.abs(M[:, i, j] - Mm[:, i, j]) / s11
            assert d.max() < acc["small_particles_s11_max_rel_error"]["value"], (i, j, d.max())
            big = np.abs(Mm[:, i, j]) > 0.25 * s11
            assert np.all(np.sign(M[big, i, j]) == np.sign(Mm[big, i, j])), (i, j)
