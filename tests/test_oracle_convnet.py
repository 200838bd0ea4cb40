"""Pins of the network oracle (oracle/convnet.py) against things other than itself."""
import numpy as np
import pytest
from scipy import signal

from oracle import convnet as cn
from oracle import dda as odda
from paper_0704_0037_amd import inputs


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv_matches_scipy_correlate():
    x = _rand((6, 5, 7, 3), 1)
    W = _rand((27, 4, 3), 2)
    y = cn.conv3d(x, W)
    for co in range(4):
        ref = np.zeros(x.shape[:3])
        for ci in range(3):
            k = W[:, co, ci].reshape(3, 3, 3)  # [dz][dy][dx]
            ref += signal.correlate(x[..., ci], k, mode="same", method="direct")
        assert np.abs(y[..., co] - ref).max() < 1e-12


def test_conv_brute_force_and_single_tap_shift():
    x = _rand((4, 4, 4, 2), 3)
    W = _rand((27, 2, 2), 4)
    y = cn.conv3d(x, W)
    ref = np.zeros_like(y)
    for z in range(4):
        for yy in range(4):
            for xx in range(4):
                for t, (dz, dy, dx) in enumerate(cn.TAPS):
                    zz, y2, x2 = z + dz, yy + dy, xx + dx
                    if 0 <= zz < 4 and 0 <= y2 < 4 and 0 <= x2 < 4:
                        ref[z, yy, xx] += W[t] @ x[zz, y2, x2]
    assert np.abs(y - ref).max() < 1e-12
    # one tap (dz, dy, dx) = (0, 0, +1) with identity channels reads the +x neighbour
    Ws = np.zeros((27, 2, 2))
    Ws[cn.TAPS.index((0, 0, 1))] = np.eye(2)
    s = cn.conv3d(x, Ws)
    assert np.array_equal(s[:, :, :-1], x[:, :, 1:]) and not s[:, :, -1].any()


def test_pool_up_adjoint_and_conv_adjoints():
    a = _rand((4, 6, 8, 3), 5)
    b = _rand((2, 3, 4, 3), 6)
    assert abs(np.sum(cn.pool(a) * b) - np.sum(a * cn.up(b)) / 8) < 1e-12
    assert abs(np.sum(cn.up(b) * a) - np.sum(b * cn.up_adjoint(a))) < 1e-12
    x = _rand((5, 4, 6, 3), 7)
    W = _rand((27, 2, 3), 8)
    g = _rand((5, 4, 6, 2), 9)
    # <g, conv(x, W)> = <conv_input_grad(g, W), x> = <conv_weight_grad(x, g), W>
    lhs = np.sum(g * cn.conv3d(x, W))
    assert abs(lhs - np.sum(cn.conv3d_input_grad(g, W) * x)) < 1e-10 * abs(lhs)
    assert abs(lhs - np.sum(cn.conv3d_weight_grad(x, g) * W)) < 1e-10 * abs(lhs)


def _small_batch(G=8, B=2, seed=0):
    rng = np.random.default_rng(seed)
    feats = rng.standard_normal((B, G, G, G, cn.N_IN)) * 0.5
    targets = rng.standard_normal((B, G, G, G, cn.N_OUT)) * 0.3
    masks = (rng.random((B, G, G, G)) < 0.6).astype(np.float64)
    return feats, targets, masks


def test_gradient_matches_finite_differences():
    """Central differences of the float64 loss along random directions and single coordinates."""
    feats, targets, masks = _small_batch()
    p = cn.init_params(3).astype(np.float64)
    # non-zero biases so that every layer's bias gradient is exercised
    rng = np.random.default_rng(4)
    layers = cn.unflatten(p)
    p = cn.flatten([(W, rng.standard_normal(b.shape) * 0.05) for W, b in layers])
    L, g = cn.loss_and_grad(p, feats, targets, masks)
    assert np.isfinite(L) and L > 0
    h = 1e-6
    for s in range(3):
        d = rng.standard_normal(p.size)
        d /= np.linalg.norm(d)  # a unit step, so that h stays far below the distance to a relu kink
        fd = (cn.loss_and_grad(p + h * d, feats, targets, masks)[0]
              - cn.loss_and_grad(p - h * d, feats, targets, masks)[0]) / (2 * h)
        assert abs(fd - g @ d) < 1e-6 * max(1.0, abs(fd))
    # one weight and the bias of every layer
    off = 0
    for ci, co, *_ in cn.LAYERS:
        for idx in (off + 27 * co * ci // 3, off + 27 * co * ci + co // 2):
            e = np.zeros(p.size)
            e[idx] = 1.0
            fd = (cn.loss_and_grad(p + h * e, feats, targets, masks)[0]
                  - cn.loss_and_grad(p - h * e, feats, targets, masks)[0]) / (2 * h)
            assert abs(fd - g[idx]) < 1e-6 * max(1e-3, abs(fd)), (ci, co, idx)
        off += 27 * co * ci + co


def test_bf16_rounding_and_rounded_gradient_close_to_exact():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -3.140625, 1e-30, 65504.0])
    r = cn.bf16(x)
    # ties to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> 1; 1 + 3*2^-8 -> 1 + 2^-6
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6 and r[3] == -3.140625
    assert abs(r[4] / 1e-30 - 1) < 2 ** -8 and r[5] == 65536.0
    feats, targets, masks = _small_batch(seed=2)
    p = cn.init_params(5)
    L, g = cn.loss_and_grad(p, feats, targets, masks)
    Lr, gr = cn.loss_and_grad(p, feats, targets, masks, bf16_round=True)
    assert abs(Lr - L) < 2e-2 * L
    assert np.linalg.norm(gr - g) < 5e-2 * np.linalg.norm(g)


def test_features_target_guess_against_dda_oracle():
    mask = inputs.ellipsoid_mask((10, 8, 6), (5, 3.5, 2.5))
    G = 16
    beam = inputs.beams_for_orientations(1, seed=2)[1]
    m, kd = 1.5 + 0.02j, 0.4
    f = cn.features(mask, m, kd, beam.prop, beam.pol, G)
    pos, _ = odda.dipoles(mask)
    idx = cn.dipole_cells(mask, G)
    ff = f.reshape(-1, cn.N_IN)
    assert ff[:, 0].sum() == len(pos) and np.all(ff[idx, 0] == 1)
    E = odda.incident_field(pos, kd, beam.prop, beam.pol)
    assert np.abs(ff[idx, 4:10:2] + 1j * ff[idx, 5:10:2] - E).max() < 1e-14
    assert np.abs(ff[idx, 10::2] + 1j * ff[idx, 11::2] - (m * m - 1) * E).max() < 1e-14
    assert not ff[ff[:, 0] == 0, 10:].any()
    assert np.allclose(ff[idx, 1], 0.5) and np.allclose(ff[idx, 2], 0.02) and np.all(ff[:, 3] == kd)
    # the box cells next to a dipole are one lattice step away
    pb = cn.box_positions((10, 8, 6), G).reshape(-1, 3)
    assert np.abs(pb[idx] - pos).max() < 1e-14
    alpha = odda.alpha_ldr(m, kd, beam.prop, beam.pol)
    beta = odda.beta_of_alpha(alpha)
    x = _rand((len(pos), 3), 3) + 1j * _rand((len(pos), 3), 4)
    t = cn.target(mask, kd, beta, beam.prop, beam.pol, x, G)
    assert np.abs(cn.guess(mask, kd, beta, beam.prop, beam.pol, t, G) - x).max() < 1e-12
    # a zero network output gives x0 = b (the right-hand side of eq. 3)
    x0 = cn.guess(mask, kd, beta, beam.prop, beam.pol, np.zeros((G, G, G, 6)), G)
    assert np.abs(x0 - odda.rhs(pos, kd, beta, beam.prop, beam.pol)).max() < 1e-14
