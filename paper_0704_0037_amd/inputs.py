"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle's tests.

This module holds only geometry and random numbers: particle masks on the cubic
dipole grid, random complex vectors, random orientations and the workload
definitions (grid sizes, refractive indices, kd).  It contains none of the DDA
arithmetic (no polarizability, Green's tensor, solver or scattering formula), so
that the oracle and the HIP path stay independent of each other.

Grid convention: a mask has shape (nz, ny, nx) with x the fastest axis, and the
cell (i, j, l) has its centre at (i + 1/2 - nx/2, j + 1/2 - ny/2, l + 1/2 - nz/2)
in units of the dipole size d (a lattice centred on the origin).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def cell_centers(grid):
    """Centres of all cells of an (nx, ny, nz) grid, as three 1-D coordinate arrays."""
    nx, ny, nz = grid
    cx = np.arange(nx, dtype=np.float64) + 0.5 - nx / 2.0
    cy = np.arange(ny, dtype=np.float64) + 0.5 - ny / 2.0
    cz = np.arange(nz, dtype=np.float64) + 0.5 - nz / 2.0
    return cx, cy, cz


def sphere_mask(n):
    """Cells whose centre lies inside the sphere of diameter n (|r|^2 <= (n/2)^2)."""
    cx, cy, cz = cell_centers((n, n, n))
    r2 = cz[:, None, None] ** 2 + cy[None, :, None] ** 2 + cx[None, None, :] ** 2
    return (r2 <= (n / 2.0) ** 2).astype(np.uint8)


def ellipsoid_mask(grid, semi_axes):
    """Cells whose centre lies inside the axis-aligned ellipsoid with the given semi-axes (d units)."""
    cx, cy, cz = cell_centers(grid)
    ax, ay, az = semi_axes
    q = (cz[:, None, None] / az) ** 2 + (cy[None, :, None] / ay) ** 2 + (cx[None, None, :] / ax) ** 2
    return (q <= 1.0).astype(np.uint8)


def rotated_ellipsoid_mask(grid, semi_axes, rot):
    """Ellipsoid with semi-axes along the columns of the 3x3 rotation `rot`."""
    cx, cy, cz = cell_centers(grid)
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    r = np.stack([X, Y, Z], axis=-1)            # (nz, ny, nx, 3)
    body = r @ np.asarray(rot, dtype=np.float64)  # coordinates in the body frame
    q = sum((body[..., a] / semi_axes[a]) ** 2 for a in range(3))
    return (q <= 1.0).astype(np.uint8)


def cluster_mask(grid, centers, radii):
    """Union of spheres (centres and radii in d units, lattice-centred coordinates)."""
    cx, cy, cz = cell_centers(grid)
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    m = np.zeros(Z.shape, dtype=bool)
    for c, r in zip(centers, radii):
        m |= (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2 <= r * r
    return m.astype(np.uint8)


def random_vector(n_dipoles, seed, n_rhs=None, dtype=np.complex128):
    """Seeded complex normal vector in the [3][N] component-major layout (or [n_rhs][3][N])."""
    rng = np.random.default_rng(seed)
    shape = (3, n_dipoles) if n_rhs is None else (n_rhs, 3, n_dipoles)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return v.astype(dtype)


def random_rotation_zyz(rng):
    """Uniformly distributed rotation on SO(3) as ZYZ Euler angles (alpha, beta, gamma)."""
    alpha = rng.uniform(0.0, 2.0 * math.pi)
    beta = math.acos(rng.uniform(-1.0, 1.0))
    gamma = rng.uniform(0.0, 2.0 * math.pi)
    return alpha, beta, gamma


def zyz_matrix(alpha, beta, gamma):
    """Rotation matrix Rz(alpha) Ry(beta) Rz(gamma)."""
    def rz(a):
        c, s = math.cos(a), math.sin(a)
        return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])

    def ry(a):
        c, s = math.cos(a), math.sin(a)
        return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])

    return rz(alpha) @ ry(beta) @ rz(gamma)


@dataclass
class Beam:
    """Incident beam in the particle frame: unit propagation vector and complex unit polarization;
    w0 > 0 makes it a focused beam of waist radius w0 (units of d) focused at center."""
    prop: tuple = (0.0, 0.0, 1.0)
    pol: tuple = (1.0 + 0j, 0j, 0j)
    w0: float = 0.0
    center: tuple = (0.0, 0.0, 0.0)

    def second(self):
        """The orthogonal polarization prop x pol (used for the second incident polarization)."""
        a = np.asarray(self.prop, dtype=np.float64)
        e = np.asarray(self.pol, dtype=np.complex128)
        return Beam(tuple(a), tuple(np.cross(a, e)), self.w0, self.center)


X_POL = Beam((0.0, 0.0, 1.0), (1.0 + 0j, 0j, 0j))
Y_POL = Beam((0.0, 0.0, 1.0), (0j, 1.0 + 0j, 0j))


def beams_for_orientations(count, seed):
    """`count` random particle orientations x 2 polarizations, as beams in the particle frame.

    The lab beam travels along +z with x and y polarizations; rotating the particle by R is
    the same as rotating the beam by R^T into the particle frame.  Returns 2*count beams,
    ordered (orientation 0: x-pol, y-pol), (orientation 1: ...), ...
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        R = zyz_matrix(*random_rotation_zyz(rng))
        a = R.T @ np.array([0.0, 0.0, 1.0])
        ex = R.T @ np.array([1.0, 0.0, 0.0])
        ey = R.T @ np.array([0.0, 1.0, 0.0])
        out.append(Beam(tuple(a), tuple(ex.astype(np.complex128))))
        out.append(Beam(tuple(a), tuple(ey.astype(np.complex128))))
    return out


def kd_for_size_parameter(x, n_dipoles):
    """kd such that a sphere of the dipoles' total volume has size parameter x (volume-equivalent)."""
    return x * (4.0 * math.pi / (3.0 * n_dipoles)) ** (1.0 / 3.0)


@dataclass
class Workload:
    name: str
    grid: tuple
    mask: np.ndarray
    m: complex
    kd: float
    beams: list = field(default_factory=list)
    tol: float = 1e-5


def c1_sphere16():
    """16^3 sphere, m = 1.5, kd = 0.419, +z x-polarized, QMR to 1e-8."""
    return Workload("sphere16_m1.5_kd0.419", (16, 16, 16), sphere_mask(16), 1.5 + 0j, 0.419,
                    [X_POL], 1e-8)


def c2_sphere256():
    """256^3 sphere, x = 40, m = 1.05 (kd from the volume-equivalent size), both polarizations."""
    mask = sphere_mask(256)
    n = int(mask.sum())
    return Workload("sphere256_x40_m1.05", (256, 256, 256), mask, 1.05 + 0j,
                    kd_for_size_parameter(40.0, n), [X_POL, Y_POL], 1e-5)


def c3_sphere160():
    """160^3 sphere, x = 20, m = 2."""
    mask = sphere_mask(160)
    n = int(mask.sum())
    return Workload("sphere160_x20_m2", (160, 160, 160), mask, 2.0 + 0j,
                    kd_for_size_parameter(20.0, n), [X_POL], 1e-5)


def c4a_ellipsoid64(n_orient=64, seed=4001):
    """64^3 triaxial ellipsoid (semi-axes 32, 22.4, 16), m = 1.33+0.01i, kd = 0.3, orientations x 2 pols."""
    mask = ellipsoid_mask((64, 64, 64), (32.0, 22.4, 16.0))
    return Workload("ellipsoid64_m1.33+0.01i_kd0.3", (64, 64, 64), mask, 1.33 + 0.01j, 0.3,
                    beams_for_orientations(n_orient, seed), 1e-5)


def c4b_sphere_batch(count=32, seed=4002, kd=0.3):
    """`count` spheres with n ~ U{24..96} and m ~ U[1.05, 1.6], +z x-polarized."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(24, 97))
        m = float(rng.uniform(1.05, 1.6))
        out.append(Workload(f"sphere{n}_m{m:.4f}", (n, n, n), sphere_mask(n), m + 0j, kd, [X_POL], 1e-5))
    return out


def small_sphere(n, m=1.5 + 0j, kd=0.4):
    return Workload(f"sphere{n}", (n, n, n), sphere_mask(n), complex(m), kd, [X_POL], 1e-8)


def c5_particle(seed, G=48):
    """One particle of the learned-initial-guess workload, on a cubic grid of side n <= G.

    Family (uniform): a sphere, a randomly rotated ellipsoid (semi-axes n/2 times sorted uniform
    [0.4, 1] factors) or a cluster of 2-4 spheres (radii in [n/8, n/4], centres uniform inside the
    cube).  n uniform in [G/3, G]; m real, uniform in [1.05, 2]; size parameter x of the
    circumscribing sphere (radius n/2) uniform in [1, min(8, 0.8 n / (2 m))], so |m| kd <= 0.8;
    incidence direction and polarization of a random orientation.
    """
    rng = np.random.default_rng(seed)
    fam = int(rng.integers(3))
    n = int(rng.integers(G // 3, G + 1))
    grid = (n, n, n)
    if fam == 1:
        axes = (n / 2.0) * np.sort(rng.uniform(0.4, 1.0, 3))[::-1]
        mask = rotated_ellipsoid_mask(grid, axes, zyz_matrix(*random_rotation_zyz(rng)))
    elif fam == 2:
        k = int(rng.integers(2, 5))
        radii = rng.uniform(n / 8.0, n / 4.0, k)
        centers = [rng.uniform(-(n / 2.0 - r), n / 2.0 - r, 3) for r in radii]
        mask = cluster_mask(grid, centers, radii)
    else:
        mask = sphere_mask(n)
    if not mask.any():
        mask = sphere_mask(n)
    m = float(rng.uniform(1.05, 2.0))
    x = float(rng.uniform(1.0, min(8.0, 0.8 * n / (2.0 * m))))
    kd = x / (n / 2.0)
    beam = beams_for_orientations(1, seed=int(rng.integers(1 << 31)))[int(rng.integers(2))]
    return mask, complex(m), kd, beam
