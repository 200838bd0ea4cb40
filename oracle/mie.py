"""Mie theory for a homogeneous sphere — TEST INFRASTRUCTURE ONLY.

The paper compares every DDA result with "exact results of the Mie theory" (Sec. 3.1, its
ref. [22], Bohren & Huffman 1983) but prints no formula.  This is the textbook series:
scattering coefficients a_n, b_n from Riccati-Bessel functions, with the logarithmic
derivative D_n(mx) obtained by downward recurrence, and the angular functions pi_n, tau_n
by upward recurrence.

pinned by: Rayleigh limit (closed form), Qext = Qsca for real m, Qext from the series equal
to (4/x^2) Re S(0) (forward-scattering theorem), the extinction-paradox limit Qext -> 2 at
large x, and the worked example that Bohren & Huffman print for their BHMIE program
(tests/golden/); the Mueller elements by the Rayleigh closed form, the identity
S11^2 = S12^2 + S33^2 + S34^2 of a single amplitude pair, and the Stokes parameters of the
scattered field computed from their definitions.
"""
from __future__ import annotations

import math

import numpy as np


def n_terms(x):
    """Number of series terms: x + 4 x^(1/3) + 2 (Wiscombe's criterion, as used in BHMIE).

    pinned by: test_oracle_scattering.py::test_mie_bhmie_printed_example (printed values of the
        textbook's program) and test_mie_energy_and_forward_theorem.
    """
    return int(round(x + 4.0 * x ** (1.0 / 3.0) + 2.0))


def coefficients(x, m):
    """Mie coefficients a_n, b_n for n = 1..nstop (arrays of length nstop).

    pinned by: test_oracle_scattering.py::test_mie_bhmie_printed_example, test_mie_rayleigh_limit
        and test_mie_extinction_paradox.
    """
    m = complex(m)
    mx = m * x
    nstop = n_terms(x)
    nmx = int(round(max(nstop, abs(mx)))) + 16
    # logarithmic derivative D_n(mx) = psi_n'(mx)/psi_n(mx), downward recurrence from 0
    D = np.zeros(nmx + 1, dtype=np.complex128)
    for n in range(nmx, 0, -1):
        D[n - 1] = n / mx - 1.0 / (D[n] + n / mx)
    a = np.zeros(nstop, dtype=np.complex128)
    b = np.zeros(nstop, dtype=np.complex128)
    # Riccati-Bessel psi_n(x) = x j_n(x), chi_n(x) = -x y_n(x), xi_n = psi_n - i chi_n
    psi_m1, psi_0 = math.cos(x), math.sin(x)
    chi_m1, chi_0 = -math.sin(x), math.cos(x)
    xi_0 = complex(psi_0, -chi_0)
    for n in range(1, nstop + 1):
        psi = (2.0 * n - 1.0) / x * psi_0 - psi_m1
        chi = (2.0 * n - 1.0) / x * chi_0 - chi_m1
        xi = complex(psi, -chi)
        ta = D[n] / m + n / x
        tb = D[n] * m + n / x
        a[n - 1] = (ta * psi - psi_0) / (ta * xi - xi_0)
        b[n - 1] = (tb * psi - psi_0) / (tb * xi - xi_0)
        psi_m1, psi_0 = psi_0, psi
        chi_m1, chi_0 = chi_0, chi
        xi_0 = complex(psi_0, -chi_0)
    return a, b


def efficiencies(x, m):
    """(Qext, Qsca, Qabs) of a sphere with size parameter x and refractive index m.

    pinned by: test_oracle_scattering.py::test_mie_bhmie_printed_example (Qext, Qsca, Qback as
        printed), test_mie_rayleigh_limit, test_mie_energy_and_forward_theorem.
    """
    a, b = coefficients(x, m)
    n = np.arange(1, len(a) + 1)
    qsca = 2.0 / x ** 2 * float(np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2)))
    qext = 2.0 / x ** 2 * float(np.sum((2 * n + 1) * np.real(a + b)))
    return qext, qsca, qext - qsca


def amplitudes(x, m, theta):
    """Amplitude functions S1(theta), S2(theta) (Bohren & Huffman convention).

    pinned by: test_oracle_scattering.py::test_mie_bhmie_printed_example (Qback from S1(180 deg))
        and test_mie_energy_and_forward_theorem (Qext = 4 Re S(0) / x^2).
    """
    a, b = coefficients(x, m)
    mu = np.cos(np.asarray(theta, dtype=np.float64))
    S1 = np.zeros(mu.shape, dtype=np.complex128)
    S2 = np.zeros(mu.shape, dtype=np.complex128)
    pi_m1 = np.zeros_like(mu)
    pi_0 = np.ones_like(mu)          # pi_1 = 1
    for n in range(1, len(a) + 1):
        pi_n = pi_0
        tau_n = n * mu * pi_n - (n + 1) * pi_m1
        f = (2.0 * n + 1.0) / (n * (n + 1.0))
        S1 += f * (a[n - 1] * pi_n + b[n - 1] * tau_n)
        S2 += f * (a[n - 1] * tau_n + b[n - 1] * pi_n)
        # pi_{n+1} = ((2n+1) mu pi_n - (n+1) pi_{n-1}) / n
        pi_next = ((2.0 * n + 1.0) * mu * pi_n - (n + 1.0) * pi_m1) / n
        pi_m1, pi_0 = pi_n, pi_next
    return S1, S2


def s11(x, m, theta):
    """Unnormalized S11 = (|S1|^2 + |S2|^2) / 2.

    pinned by:
        test_oracle_scattering.py::test_mie_mueller_rayleigh_limit_and_single_amplitude_pair_identit
        y.
    """
    S1, S2 = amplitudes(x, m, theta)
    return 0.5 * (np.abs(S1) ** 2 + np.abs(S2) ** 2)


def mueller(x, m, theta):
    """Nonzero elements of a sphere's Mueller matrix (Bohren & Huffman eq. 4.77, unnormalized):
    S11 = (|S2|^2 + |S1|^2)/2, S12 = (|S2|^2 - |S1|^2)/2, S33 = Re(S2 S1^*), S34 = Im(S2 S1^*);
    by the sphere's symmetry S22 = S11, S21 = S12, S44 = S33, S43 = -S34 and the rest vanish.
    Returns (len(theta), 4, 4).

    pinned by:
        test_oracle_scattering.py::test_mie_mueller_rayleigh_limit_and_single_amplitude_pair_identit
        y (Rayleigh limit and S11^2 = S12^2 + S33^2 + S34^2).
    """
    S1, S2 = amplitudes(x, m, theta)
    M = np.zeros(S1.shape + (4, 4))
    M[..., 0, 0] = M[..., 1, 1] = 0.5 * (np.abs(S2) ** 2 + np.abs(S1) ** 2)
    M[..., 0, 1] = M[..., 1, 0] = 0.5 * (np.abs(S2) ** 2 - np.abs(S1) ** 2)
    M[..., 2, 2] = M[..., 3, 3] = np.real(S2 * np.conj(S1))
    M[..., 2, 3] = np.imag(S2 * np.conj(S1))
    M[..., 3, 2] = -M[..., 2, 3]
    return M


def asymmetry(x, m):
    """Asymmetry parameter <cos theta> from the series (Bohren & Huffman eq. 4.62).

    pinned by: test_oracle_scattering.py::test_mie_bhmie_printed_example (g as printed) and
        test_oracle_physics.py::test_sphere_asymmetry_near_mie.
    """
    a, b = coefficients(x, m)
    qext, qsca, _ = efficiencies(x, m)
    n = np.arange(1, len(a) + 1)
    t1 = np.sum(n[:-1] * (n[:-1] + 2.0) / (n[:-1] + 1.0)
                * np.real(a[:-1] * np.conj(a[1:]) + b[:-1] * np.conj(b[1:])))
    t2 = np.sum((2.0 * n + 1.0) / (n * (n + 1.0)) * np.real(a * np.conj(b)))
    return float(4.0 / (x * x * qsca) * (t1 + t2))
