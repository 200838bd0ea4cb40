"""Pins of the CPU oracle's building blocks against closed forms, brute force and invariants.

None of these re-type the oracle's formula: each checks it against something the
mathematics or the physics fixes independently (finite differences, textbook static
limits, loops over the grid, library FFT convolution, exact symmetries).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import dda
from paper_0704_0037_amd import inputs


# ------------------------------------------------------------------------- lattice
def test_dipoles_match_bruteforce_loops():
    rng = np.random.default_rng(1)
    mask = (rng.random((5, 4, 3)) < 0.6).astype(np.uint8)   # (nz, ny, nx)
    pos, lin = dda.dipoles(mask)
    exp_pos, exp_lin = [], []
    for z in range(5):
        for y in range(4):
            for x in range(3):
                if mask[z, y, x]:
                    exp_lin.append(x + 3 * (y + 4 * z))
                    exp_pos.append((x + 0.5 - 1.5, y + 0.5 - 2.0, z + 0.5 - 2.5))
    assert list(lin) == exp_lin
    np.testing.assert_array_equal(pos, np.array(exp_pos))


def test_sphere_counts_bruteforce():
    # count cells with centre inside the sphere by an explicit loop
    n = 16
    cnt = 0
    for z, y, x in itertools.product(range(n), repeat=3):
        r2 = (x + 0.5 - n / 2) ** 2 + (y + 0.5 - n / 2) ** 2 + (z + 0.5 - n / 2) ** 2
        cnt += r2 <= (n / 2) ** 2
    assert cnt == int(inputs.sphere_mask(n).sum()) == 2176


# ------------------------------------------------------------------ Green's tensor
def _scalar_green(r, k):
    rn = np.linalg.norm(r)
    return np.exp(1j * k * rn) / rn


def test_green_equals_k2_plus_gradgrad_of_scalar_green():
    """G = (k^2 I + grad grad) exp(ikr)/r, with the Hessian by 4th-order finite differences."""
    h = 1e-3
    for k in (0.3, 1.1):
        for r in ([1.0, 0.0, 0.0], [0.7, -1.3, 2.1], [3.0, 2.0, -1.0]):
            r = np.array(r)
            H = np.zeros((3, 3), dtype=np.complex128)
            for a in range(3):
                for b in range(3):
                    ea, eb = np.eye(3)[a] * h, np.eye(3)[b] * h
                    if a == b:
                        f = lambda s: _scalar_green(r + s * ea, k)
                        H[a, b] = (-f(2) + 16 * f(1) - 30 * f(0) + 16 * f(-1) - f(-2)) / (12 * h * h)
                    else:
                        acc = 0
                        for (sa, sb, w) in [(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]:
                            acc += w * _scalar_green(r + sa * ea + sb * eb, k)
                        H[a, b] = acc / (4 * h * h)
            expect = k * k * np.eye(3) * _scalar_green(r, k) + H
            G = dda.green(r, k)
            assert np.abs(G - expect).max() <= 2e-6 * np.abs(G).max()


def test_green_static_limit_is_dipole_field():
    # textbook static dipole field: E = (3 (p.r^) r^ - p) / r^3
    G = dda.green(np.array([0.0, 0.0, 2.0]), 0.0)
    np.testing.assert_allclose(G, np.diag([-1.0, -1.0, 2.0]) / 8.0, atol=1e-15)


def test_green_symmetric_and_even():
    rng = np.random.default_rng(2)
    r = rng.standard_normal((50, 3))
    G = dda.green(r, 0.7)
    assert np.array_equal(G, G.transpose(0, 2, 1))
    np.testing.assert_allclose(dda.green(-r, 0.7), G, rtol=0, atol=1e-15)


# ------------------------------------------------------------------- polarizability
def test_cm_closed_form_limits():
    assert dda.alpha_cm(1.0) == 0
    assert abs(dda.alpha_cm(1e8) - 3 / (4 * math.pi)) < 1e-12
    # dilute limit: alpha ~ (m^2 - 1)/(4 pi) for m -> 1
    eps = 1e-6
    assert abs(dda.alpha_cm(1 + eps) / (((1 + eps) ** 2 - 1) / (4 * math.pi)) - 1) < 1e-5


def test_ldr_reduces_to_cm_for_small_k():
    for m in (1.05, 1.5, 2.0 + 0.3j):
        a = dda.alpha_ldr(m, 1e-6, (0, 0, 1), (1, 0, 0))
        assert abs(a / dda.alpha_cm(m) - 1) < 1e-10


def test_ldr_radiative_reaction_term():
    for m in (1.05, 1.5, 2.0):
        for k in (0.1, 0.3, 0.6):
            for prop, pol in [((0, 0, 1), (1, 0, 0)), ((0.6, 0, 0.8), (0.8, 0, -0.6))]:
                a = dda.alpha_ldr(m, k, prop, pol)
                assert abs((1 / a).imag + 2 / 3 * k ** 3) < 1e-12


def test_rr_reduces_to_cm_for_small_k():
    for m in (1.05, 1.5, 2.0 + 0.3j):
        assert abs(dda.alpha_rr(m, 1e-6) / dda.alpha_cm(m) - 1) < 1e-12
        assert abs(dda.alpha_rr(m, 0.5) / dda.alpha_cm(m) - 1) > 1e-4  # it does differ at finite k


def test_rr_single_dipole_conserves_energy():
    # one dipole has no interactions, so P = alpha E_inc; for real m the radiative-reaction
    # correction makes its extinction equal its scattering (the CM value alone does not)
    pos = np.zeros((1, 3))
    prop, pol = (0.0, 0.0, 1.0), (1.0, 0.0, 0.0)
    for m in (1.2, 1.5, 2.5):
        for k in (0.2, 0.6, 1.0):
            for alpha in (dda.alpha_rr(m, k), dda.alpha_cm(m)):
                P = alpha * dda.incident_field(pos, k, prop, pol)
                cext, cabs = dda.cross_sections(pos, k, alpha, P, prop, pol)[:2]
                csca = dda.csca_exact(pos, k, P)
                if alpha == dda.alpha_rr(m, k):
                    assert abs(cabs) < 1e-12 * csca and abs(cext - csca) < 1e-12 * csca
                else:
                    assert abs(cext) < 1e-12 * csca  # CM: no extinction, yet it scatters


# ------------------------------------------------------------------ interaction matrix
def _small_particle(seed=3, shape=(5, 4, 6), fill=0.7):
    rng = np.random.default_rng(seed)
    return (rng.random(shape) < fill).astype(np.uint8)


def test_interaction_matrix_complex_symmetric():
    pos, _ = dda.dipoles(_small_particle())
    A = dda.interaction_matrix(pos, 0.9, np.sqrt(0.05 + 0.01j))
    assert np.array_equal(A, A.T)
    assert not np.allclose(A, A.conj().T)


def test_direct_sum_equals_dense():
    pos, _ = dda.dipoles(_small_particle())
    beta = np.sqrt(0.1 + 0.02j)
    x = inputs.random_vector(len(pos), 5).T.copy()
    A = dda.interaction_matrix(pos, 0.5, beta)
    y_dense = (A @ x.reshape(-1)).reshape(x.shape)
    y_direct = dda.matvec(pos, 0.5, beta, x, chunk=7)
    np.testing.assert_allclose(y_direct, y_dense, rtol=0, atol=1e-13 * np.abs(y_dense).max())
    rows = [0, 3, len(pos) - 1]
    np.testing.assert_allclose(dda.matvec_rows(pos, 0.5, beta, x, rows), y_dense[rows],
                               rtol=0, atol=1e-13 * np.abs(y_dense).max())


def _fft_convolution_matvec(mask, k, beta, x):
    """The lattice convolution done with numpy's FFT on a zero-padded circulant grid."""
    nz, ny, nx = mask.shape
    L = (2 * nx, 2 * ny, 2 * nz)
    idx = [np.arange(Lz) for Lz in L]
    disp = [np.where(i < n, i, i - Ls) for i, n, Ls in zip(idx, (nx, ny, nz), L)]
    DZ, DY, DX = np.meshgrid(disp[2], disp[1], disp[0], indexing="ij")
    r = np.stack([DX, DY, DZ], axis=-1).astype(float)
    zero = (DX == 0) & (DY == 0) & (DZ == 0)
    r[zero] = 1.0
    G = dda.green(r, k)
    G[zero] = 0.0
    grid = np.zeros((3, L[2], L[1], L[0]), dtype=np.complex128)
    sel = mask.astype(bool)
    for c in range(3):
        g = np.zeros((nz, ny, nx), dtype=np.complex128)
        g[sel] = beta * x[:, c]
        grid[c, :nz, :ny, :nx] = g
    X = np.fft.fftn(grid, axes=(1, 2, 3))
    Gh = np.fft.fftn(G, axes=(0, 1, 2))
    Y = np.einsum("zyxab,bzyx->azyx", Gh, X)
    conv = np.fft.ifftn(Y, axes=(1, 2, 3))[:, :nz, :ny, :nx]
    return x - beta * np.stack([conv[c][sel] for c in range(3)], axis=1)


def test_direct_sum_equals_library_fft_convolution():
    mask = _small_particle(seed=4, shape=(6, 5, 7))
    pos, _ = dda.dipoles(mask)
    beta = np.sqrt(dda.alpha_ldr(1.4 + 0.05j, 0.6, (0, 0, 1), (1, 0, 0)))
    x = inputs.random_vector(len(pos), 6).T.copy()
    y = dda.matvec(pos, 0.6, beta, x)
    y_fft = _fft_convolution_matvec(mask, 0.6, beta, x)
    assert np.linalg.norm(y - y_fft) / np.linalg.norm(y) < 1e-13


def test_ghat_parity_of_components():
    """Fourier transform of each G component is even/odd along each axis (octant storage)."""
    n = 4
    L = 2 * n
    d = np.where(np.arange(L) < n, np.arange(L), np.arange(L) - L)
    DZ, DY, DX = np.meshgrid(d, d, d, indexing="ij")
    r = np.stack([DX, DY, DZ], axis=-1).astype(float)
    r[L // 2, :, :] = 7.0  # never-used middle planes: any value, 0 used below
    zero = (DX == 0) & (DY == 0) & (DZ == 0)
    r[zero] = 1.0
    G = dda.green(r, 0.8)
    G[zero] = 0
    G[n, :, :] = G[:, n, :] = G[:, :, n] = 0
    Gh = np.fft.fftn(G, axes=(0, 1, 2))
    flip = lambda a, ax: np.roll(np.flip(a, axis=ax), 1, axis=ax)
    for a in range(3):
        for b in range(3):
            for axis, comp in ((2, 0), (1, 1), (0, 2)):
                odd = (a == comp) != (b == comp)
                sgn = -1.0 if odd else 1.0
                np.testing.assert_allclose(flip(Gh[..., a, b], axis), sgn * Gh[..., a, b], atol=1e-10)


# ------------------------------------------------------------------ asymmetry parameter
def test_asymmetry_quadrature_reproduces_the_exact_scattering_cross_section():
    mask = _small_particle(seed=5, shape=(4, 5, 3))
    pos, _ = dda.dipoles(mask)
    k = 0.8
    prop, pol = (0.6, 0.0, 0.8), (0.8, 0.0, -0.6)
    alpha = dda.alpha_ldr(1.4 + 0.05j, k, prop, pol)
    P = alpha * dda.incident_field(pos, k, prop, pol)  # any polarization field will do
    csca, g = dda.asymmetry(pos, k, P, prop, 24, 48)
    ref = dda.csca_exact(pos, k, P)
    assert abs(csca - ref) < 1e-10 * ref
    assert -1 < g < 1


def test_single_dipole_scatters_symmetrically():
    pos = np.zeros((1, 3))
    P = np.array([[0.3 + 0.1j, 0.0, 0.0]])
    csca, g = dda.asymmetry(pos, 0.7, P, (0, 0, 1), 16, 32)
    assert abs(g) < 1e-14
    assert abs(csca - 8 * math.pi / 3 * 0.7 ** 4 * np.sum(np.abs(P) ** 2)) < 1e-12 * csca


def test_sphere_asymmetry_near_mie():
    from oracle import mie
    n, m, kd = 10, 1.3 + 0j, 0.35
    mask = inputs.sphere_mask(n)
    pos, _ = dda.dipoles(mask)
    alpha = dda.alpha_ldr(m, kd, (0, 0, 1), (1, 0, 0))
    beta = dda.beta_of_alpha(alpha)
    A = dda.interaction_matrix(pos, kd, beta)
    b = dda.rhs(pos, kd, beta, (0, 0, 1), (1, 0, 0))
    x = np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)
    csca, g = dda.asymmetry(pos, kd, beta * x, (0, 0, 1), 32, 64)
    xeq = dda.size_parameter(kd, len(pos))
    g_mie = mie.asymmetry(xeq, m)
    assert abs(g - g_mie) < 0.03 * abs(g_mie)


# ------------------------------------------------------------------ orientation averaging
def test_romberg_is_exact_on_polynomials():
    for n in (1, 2, 3, 4):
        x = np.linspace(-1.0, 1.0, 2 ** n + 1)
        for deg in range(0, 2 * n + 2):
            v, _ = dda.romberg(x ** deg, -1.0, 1.0)
            exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
            assert abs(v - exact) < 1e-12, (n, deg)
    v, _ = dda.romberg(np.cos(np.linspace(0, 1, 17)), 0.0, 1.0)
    assert abs(v - math.sin(1.0)) < 1e-12


def test_orientation_average_of_an_isotropic_dipole():
    mask = np.ones((1, 1, 1), np.uint8)
    avg, err = dda.orientation_average(mask, 1.5, 0.6, 2, 2, polarizability="cm")
    pos = np.zeros((1, 3))
    alpha = dda.alpha_cm(1.5)
    P = alpha * dda.incident_field(pos, 0.6, (0, 0, 1), (1, 0, 0))
    cext = dda.cross_sections(pos, 0.6, alpha, P, (0, 0, 1), (1, 0, 0))[0]
    assert abs(avg["Cext"] - cext) < 1e-12 * abs(cext) + 1e-15


def test_orientation_average_invariant_under_a_lattice_rotation():
    # the average over all orientations does not depend on how the particle was placed: the same
    # particle turned by 90 degrees about x (an exact lattice rotation) gives the same average
    mask = np.zeros((3, 2, 2), np.uint8)
    mask[:, 0, 0] = 1
    mask[0, 1, 0] = 1
    mask[2, 0, 1] = 1
    turned = np.ascontiguousarray(np.rot90(mask, 1, axes=(0, 1)))
    a1, e1 = dda.orientation_average(mask, 1.5, 0.5, 4, 4)
    a2, e2 = dda.orientation_average(turned, 1.5, 0.5, 4, 4)
    assert abs(a1["Cext"] - a2["Cext"]) < 1e-4 * a1["Cext"]
    assert e1 < 1e-3 * a1["Cext"]


def test_adaptive_romberg_closed_form_and_one_evaluation_per_point():
    seen = []

    def f(x):
        seen.extend(x.tolist())
        return np.exp(x)

    v, e, n = dda.romberg_adaptive(f, -1.0, 1.0, 1e-12)
    assert abs(v[0] - (math.e - 1.0 / math.e)) < 1e-13
    assert len(seen) == 2 ** n + 1 == len(set(seen))  # every abscissa evaluated once
    assert e[0] <= 1e-12 * v[0]


def test_adaptive_romberg_stops_where_polynomials_become_exact():
    # R(n,n) is exact up to degree 2n + 1 and R(n,n-1) up to degree 2n - 1: a cubic stops at the
    # first level (n = 2), a quintic needs one doubling
    v, e, n = dda.romberg_adaptive(lambda x: x ** 3 + x ** 2 + 1.0, -1.0, 1.0, 1e-12, 2, 8)
    assert n == 2 and abs(v[0] - 8.0 / 3.0) < 1e-14
    v, e, n = dda.romberg_adaptive(lambda x: x ** 5 + x ** 4 + 1.0, -1.0, 1.0, 1e-12, 2, 8)
    assert n == 3 and abs(v[0] - 2.4) < 1e-14
    # a kink converges slowly: the level cap ends it, with the cap's error estimate
    v, e, n = dda.romberg_adaptive(lambda x: np.abs(x - 0.3), -1.0, 1.0, 1e-14, 2, 5)
    assert n == 5 and e[0] > 1e-14 * v[0] and abs(v[0] - 1.09) < 1e-2


def test_adaptive_orientation_average_equals_the_fixed_rule_at_its_level():
    mask = np.zeros((3, 2, 2), np.uint8)
    mask[:, 0, 0] = 1
    mask[0, 1, 0] = 1
    mask[2, 0, 1] = 1
    avg, err, n = dda.orientation_average_adaptive(mask, 1.5 + 0.02j, 0.5, 1e-5, 2, 6, 2)
    assert n == 4  # level 3 misses 1e-5 (3.7e-5 of <Cext>), level 4 meets it
    fixed, ferr = dda.orientation_average(mask, 1.5 + 0.02j, 0.5, n, 2)
    for q in ("Cext", "Cabs", "Csca"):
        assert abs(avg[q] - fixed[q]) < 1e-14 * fixed["Cext"]
    assert abs(err["Cext"] - ferr) < 1e-14 * fixed["Cext"] and err["Cabs"] <= 1e-5 * avg["Cext"]


def test_orientation_averaged_mueller_of_a_single_dipole_is_rayleigh():
    # an isotropic (CM) dipole: S1 = -i k^3 alpha, S2 = -i k^3 alpha cos(theta), S3 = S4 = 0 in
    # every orientation and plane
    mask = np.ones((1, 1, 1), np.uint8)
    k, m = 0.6, 1.5 + 0.1j
    th = np.linspace(0.0, math.pi, 7)
    M, err = dda.orientation_average_mueller(mask, m, k, 2, 1, 4, th, polarizability="cm")
    a2 = k ** 6 * abs(dda.alpha_cm(m)) ** 2
    c = np.cos(th)
    ref = np.zeros((len(th), 4, 4))
    ref[:, 0, 0] = ref[:, 1, 1] = a2 * (1 + c ** 2) / 2
    ref[:, 0, 1] = ref[:, 1, 0] = a2 * (c ** 2 - 1) / 2
    ref[:, 2, 2] = ref[:, 3, 3] = a2 * c
    assert np.max(np.abs(M - ref)) < 1e-12 * a2 and np.max(err) < 1e-12 * a2


def _l_particle():
    mask = np.zeros((1, 2, 2), np.uint8)
    mask[0, 0, 0] = mask[0, 0, 1] = mask[0, 1, 0] = 1
    return mask


def test_orientation_averaged_mueller_integrates_to_csca_and_has_mirror_structure():
    mask = _l_particle()  # planar: its plane is a mirror plane
    k = 0.5
    x, w = np.polynomial.legendre.leggauss(24)
    M, err = dda.orientation_average_mueller(mask, 1.5 + 0.02j, k, 4, 3, 8, np.arccos(x))
    avg, _ = dda.orientation_average(mask, 1.5 + 0.02j, k, 4, 3)
    csca = 2 * math.pi * np.sum(w * M[:, 0, 0]) / k ** 2  # the averaged matrix does not depend on phi
    assert abs(csca - avg["Csca"]) < 1e-6 * avg["Csca"]
    s11 = M[:, 0, 0]
    for i, j in ((0, 2), (0, 3), (1, 2), (1, 3), (2, 0), (2, 1), (3, 0), (3, 1)):
        assert np.max(np.abs(M[:, i, j]) / s11) < 1e-12
    assert np.max(np.abs(M[:, 1, 0] - M[:, 0, 1]) / s11) < 1e-3
    assert np.max(np.abs(M[:, 3, 2] + M[:, 2, 3]) / s11) < 1e-4


def test_orientation_averaged_mueller_does_not_depend_on_the_particle_placement():
    # the same particle turned by 90 degrees (an exact lattice rotation) has the same average;
    # without the average over the scattering planes (alpha) it differs by several per cent
    mask = _l_particle()
    turned = np.ascontiguousarray(np.rot90(mask, 1, axes=(0, 1)))
    th = np.linspace(0.0, math.pi, 9)
    M1, _ = dda.orientation_average_mueller(mask, 1.5 + 0.02j, 0.5, 4, 4, 8, th)
    M2, _ = dda.orientation_average_mueller(turned, 1.5 + 0.02j, 0.5, 4, 4, 8, th)
    scale = np.max(M1[:, 0, 0])
    assert np.max(np.abs(M1 - M2)) < 1e-3 * scale
    N2, _ = dda.orientation_average_mueller(turned, 1.5 + 0.02j, 0.5, 4, 4, 1, th)
    assert np.max(np.abs(M1 - N2)) > 1e-2 * scale


# ------------------------------------------------------------------ focused (Gaussian) beam
_CIRC = np.array([1.0, 1.0j, 0.0]) / math.sqrt(2.0)
_AZ = np.array([0.0, 0.0, 1.0])


@pytest.mark.parametrize("kw0", [2.0, 5.0, 50.0])
def test_gaussian_beam_focal_value_closed_form(kw0):
    # at the focus the phi integral of (e - (e.k^)k^) is pi (2 - sin^2) e, which leaves
    # E(c) = e [(1 - exp(-A)) - (2 / (k w0)^2) (1 - exp(-A)(1 + A))], A = (k w0)^2 / 4
    k = 0.7
    w0 = kw0 / k
    A = kw0 ** 2 / 4.0
    ref = (1 - math.exp(-A)) - (2.0 / kw0 ** 2) * (1 - math.exp(-A) * (1 + A))
    E = dda.gaussian_beam_field(np.array([[0.4, -0.1, 0.2]]), k, _AZ, _CIRC, w0, (0.4, -0.1, 0.2))[0]
    assert np.max(np.abs(E - ref * _CIRC)) < 1e-14


def test_gaussian_beam_is_transverse_and_solves_helmholtz():
    k, w0, c = 1.0, 2.0, (0.3, -0.2, 0.5)
    rng = np.random.default_rng(0)
    pts = rng.uniform(-3.0, 3.0, (5, 3))
    far = np.array([[10.0, 0.0, 0.0]])  # fixes the quadrature (it is sized by the farthest point)

    def F(r):
        return dda.gaussian_beam_field(np.vstack([r, far]), k, _AZ, _CIRC, w0, c)[:-1]

    h = 1e-3
    E0 = F(pts)
    div = np.zeros(len(pts), complex)
    lap = np.zeros_like(E0)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        Ep, Em = F(pts + e), F(pts - e)
        div += (Ep[:, d] - Em[:, d]) / (2 * h)
        lap += (Ep - 2 * E0 + Em) / h ** 2
    scale = np.max(np.abs(E0))
    assert np.max(np.abs(div)) < 1e-7 * scale
    assert np.max(np.abs(lap + k * k * E0)) < 1e-6 * scale


def test_gaussian_beam_plane_wave_and_paraxial_limits():
    k = 1.0
    rng = np.random.default_rng(1)
    pts = rng.uniform(-5.0, 5.0, (6, 3))
    E = dda.gaussian_beam_field(pts, k, _AZ, _CIRC, 1e4, (0.0, 0.0, 0.0))
    assert np.max(np.abs(E - np.exp(1j * k * pts @ _AZ)[:, None] * _CIRC)) < 1e-6
    # k w0 = 20: the paraxial Gaussian up to O(1 / (k w0)^2)
    w0 = 20.0
    pts = rng.uniform(-15.0, 15.0, (8, 3))
    pts[:, 2] *= 3
    E = dda.gaussian_beam_field(pts, k, _AZ, _CIRC, w0, (0.0, 0.0, 0.0))
    q = 1 + 2j * pts[:, 2] / (k * w0 ** 2)
    psi = np.exp(-(pts[:, 0] ** 2 + pts[:, 1] ** 2) / (w0 ** 2 * q)) / q * np.exp(1j * k * pts[:, 2])
    err = np.max(np.abs(E[:, :2] - psi[:, None] * _CIRC[:2]))
    assert err < 2.0 / (k * w0) ** 2 and np.max(np.abs(E[:, 2])) < 5.0 / (k * w0)


def test_gaussian_beam_quadrature_is_converged():
    k, w0 = 0.9, 3.0
    rng = np.random.default_rng(2)
    pts = rng.uniform(-6.0, 6.0, (20, 3))
    E = dda.gaussian_beam_field(pts, k, (0.6, 0.0, 0.8), (0.8, 0.0, -0.6), w0, (0.5, 0.5, 0.0))
    # the same field with twice the nodes: the rule sized by the farthest point is converged
    big = np.vstack([pts, [[0.5 + 40.0, 0.5, 0.0]]])
    E2 = dda.gaussian_beam_field(big, k, (0.6, 0.0, 0.8), (0.8, 0.0, -0.6), w0, (0.5, 0.5, 0.0))[:-1]
    assert np.max(np.abs(E - E2)) < 1e-12


# ------------------------------------------------------------------ inhomogeneous particles
def _two_material_mask():
    mask = np.zeros((3, 3, 4), np.uint8)
    mask[:, :, :2] = 1
    mask[:, :, 2:] = 2
    mask[0, 0, 3] = 0
    return mask


def test_inhomogeneous_symmetrized_system_equals_equation_1():
    # eq. 1 with a different alpha per dipole, solved directly for P, against the symmetrized
    # eqs. 2-3 (A = I - beta G beta, b = beta E, P = beta x)
    mask = _two_material_mask()
    pos, _ = dda.dipoles(mask)
    k, prop, pol = 0.7, np.array([0.0, 0.6, 0.8]), np.array([1.0, 0.0, 0.0])
    alpha = dda.material_alphas(mask, [1.5 + 0.1j, 1.2 + 0.3j], k, prop, pol)
    N = len(pos)
    M = np.zeros((N, 3, N, 3), complex)
    for i in range(N):
        for j in range(N):
            if i == j:
                M[i, :, i, :] = np.eye(3) / alpha[i]
            else:
                M[i, :, j, :] = -dda.green(pos[i] - pos[j], k)
    E = dda.incident_field(pos, k, prop, pol)
    P1 = np.linalg.solve(M.reshape(3 * N, 3 * N), E.reshape(-1)).reshape(N, 3)
    bt = np.sqrt(alpha)
    A = dda.interaction_matrix(pos, k, bt)
    assert np.max(np.abs(A - A.T)) == 0.0
    x = np.linalg.solve(A, dda.rhs(pos, k, bt, prop, pol).reshape(-1)).reshape(N, 3)
    assert np.max(np.abs(bt[:, None] * x - P1)) < 1e-12 * np.max(np.abs(P1))


def test_inhomogeneous_reduces_to_homogeneous_and_to_void():
    mask = _two_material_mask()
    pos, lin = dda.dipoles(mask)
    k, prop, pol = 0.7, np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0])
    a2 = dda.material_alphas(mask, [1.4 + 0.05j, 1.4 + 0.05j], k, prop, pol)
    assert np.all(a2 == dda.alpha_ldr(1.4 + 0.05j, k, prop, pol))
    # CM with m = 1 for material 2: those dipoles have alpha = 0 and the particle is material 1 alone
    a = dda.material_alphas(mask, [1.5 + 0.1j, 1.0], k, prop, pol, polarizability="cm")
    bt = np.sqrt(a)
    x = np.linalg.solve(dda.interaction_matrix(pos, k, bt), dda.rhs(pos, k, bt, prop, pol).reshape(-1))
    cext, cabs = dda.cross_sections(pos, k, np.where(a == 0, 1.0, a), bt[:, None] * x.reshape(-1, 3), prop, pol)
    only = np.where(mask == 1, 1, 0).astype(np.uint8)
    p1, _ = dda.dipoles(only)
    a1 = dda.alpha_cm(1.5 + 0.1j)
    b1 = np.sqrt(a1)
    x1 = np.linalg.solve(dda.interaction_matrix(p1, k, b1), dda.rhs(p1, k, b1, prop, pol).reshape(-1))
    c1, d1 = dda.cross_sections(p1, k, a1, b1 * x1.reshape(-1, 3), prop, pol)
    assert abs(cext - c1) < 1e-12 * abs(c1) and abs(cabs - d1) < 1e-12 * abs(c1)


def test_cldr_limits_and_relation_to_ldr():
    m = 1.5 + 0.02j
    # k -> 0: CM
    assert np.max(np.abs(dda.alpha_cldr(m, 1e-6, (0.0, 0.6, 0.8)) - dda.alpha_cm(m))) < 1e-10
    # a along z, e along x: the element along e is LDR's (a_x = 0 and S = 0); the z element differs
    a = dda.alpha_cldr(m, 0.7, (0.0, 0.0, 1.0))
    assert abs(a[0] - dda.alpha_ldr(m, 0.7, (0, 0, 1), (1, 0, 0))) < 1e-15 and a[0] == a[1] and abs(a[2] - a[0]) > 1e-3
    # radiative reaction for real m
    ar = dda.alpha_cldr(1.5, 0.7, (0.6, 0.0, 0.8))
    assert np.max(np.abs(np.imag(1.0 / ar) + (2.0 / 3.0) * 0.7 ** 3)) < 1e-12


def test_tensor_polarizability_symmetrized_system_equals_equation_1():
    mask = _two_material_mask()
    pos, _ = dda.dipoles(mask)
    k, prop, pol = 0.7, np.array([0.0, 0.6, 0.8]), np.array([1.0, 0.0, 0.0])
    alpha = dda.material_alphas(mask, [1.5 + 0.1j, 1.2 + 0.3j], k, prop, pol, polarizability="cldr")
    assert alpha.shape == (len(pos), 3)
    N = len(pos)
    M = np.zeros((N, 3, N, 3), complex)
    for i in range(N):
        for j in range(N):
            M[i, :, j, :] = np.diag(1.0 / alpha[i]) if i == j else -dda.green(pos[i] - pos[j], k)
    E = dda.incident_field(pos, k, prop, pol)
    P1 = np.linalg.solve(M.reshape(3 * N, 3 * N), E.reshape(-1)).reshape(N, 3)
    bt = np.sqrt(alpha)
    A = dda.interaction_matrix(pos, k, bt)
    assert np.max(np.abs(A - A.T)) < 1e-15 * np.max(np.abs(A))  # complex symmetric up to rounding
    x = np.linalg.solve(A, dda.rhs(pos, k, bt, prop, pol).reshape(-1)).reshape(N, 3)
    assert np.max(np.abs(bt * x - P1)) < 1e-12 * np.max(np.abs(P1))
    # Cabs with a weight per component equals the sum over components of the scalar formula
    cext, cabs = dda.cross_sections(pos, k, alpha, P1, prop, pol)
    w = -np.imag(1.0 / alpha) - (2.0 / 3.0) * k ** 3
    assert abs(cabs - 4 * math.pi * k * np.sum(w * np.abs(P1) ** 2)) < 1e-12 * abs(cext)


def test_orientation_average_of_two_equal_materials_is_the_homogeneous_one():
    mask = _two_material_mask()
    one = (mask > 0).astype(np.uint8)
    a1, e1 = dda.orientation_average(one, 1.5 + 0.02j, 0.5, 2, 1)
    a2, e2 = dda.orientation_average(mask, [1.5 + 0.02j, 1.5 + 0.02j], 0.5, 2, 1)
    for q in ("Cext", "Cabs", "Csca"):
        assert abs(a1[q] - a2[q]) < 1e-12 * a1["Cext"]
