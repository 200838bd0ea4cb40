"""GPU parity of the learned-initial-guess network with the oracle (oracle/convnet.py).

Bars (bfloat16 storage, fp32 accumulation on both sides of the rounding points the oracle
emulates): features within one bfloat16 step of the rounded oracle features; target and guess
maps within float32 / float64 rounding; network output within 1e-2 (relative norm) of the
rounded oracle; every layer's weight and bias gradient within 3e-2 (relative norm), the whole
gradient's cosine with the oracle's above 0.999.
"""
import numpy as np
import pytest
import torch

from oracle import convnet as cn
from oracle import dda as odda
from paper_0704_0037_amd import inputs

pytestmark = pytest.mark.gpu


def _dda():
    from paper_0704_0037_amd import dda
    return dda


def _particles(G):
    return [
        (inputs.ellipsoid_mask((12, 9, 7), (6, 4.5, 3.5)), 1.5 + 0.02j, 0.4, inputs.beams_for_orientations(1, seed=2)[1]),
        (inputs.sphere_mask(G - 2), 1.8, 0.3, inputs.beams_for_orientations(1, seed=5)[0]),
    ]


def _params(seed):
    p = cn.init_params(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    return cn.flatten([(W, rng.standard_normal(b.shape) * 0.05) for W, b in cn.unflatten(p)]).astype(np.float32)


def _bf16_to_np(t):
    return t.float().cpu().numpy().astype(np.float64)


def test_features_target_guess_maps():
    dda = _dda()
    G = 16
    p = _params(1)
    for mask, m, kd, beam in _particles(G):
        with dda.Context(mask, m, kd) as ctx, dda.Net(G, p, max_batch=1) as net:
            f = _bf16_to_np(net.features(ctx, beam)).reshape(G, G, G, 16)
            fo = cn.bf16(cn.features(mask, m, kd, beam.prop, beam.pol, G))
            step = np.maximum(np.abs(fo), 1e-6) * 2.0 ** -7
            assert np.all(np.abs(f - fo) <= step)
            alpha = odda.alpha_ldr(m, kd, beam.prop, beam.pol)
            beta = odda.beta_of_alpha(alpha)
            x = inputs.random_vector(ctx.n, seed=4)
            t = net.target(ctx, beam, torch.from_numpy(x).cuda()).cpu().numpy().reshape(G, G, G, 6)
            to = cn.target(mask, kd, beta, beam.prop, beam.pol, x.T, G)
            assert np.abs(t - to).max() < 1e-6 * np.abs(to).max()
            feat = net.features(ctx, beam).reshape(1, G ** 3, 16)
            out = net.forward(feat)
            x0 = net.guess(ctx, [beam], feat)[0].cpu().numpy().T
            x0o = cn.guess(mask, kd, beta, beam.prop, beam.pol, out[0].cpu().numpy().astype(np.float64), G)
            assert np.abs(x0 - x0o).max() < 1e-12 * np.abs(x0o).max()


def _batch(net, G, solved=False):
    """Features and targets of the two particles; targets from random vectors or from solutions."""
    dda = _dda()
    feats, tgts, masks = [], [], []
    for i, (mask, m, kd, beam) in enumerate(_particles(G)):
        with dda.Context(mask, m, kd) as ctx:
            feats.append(net.features(ctx, beam))
            if solved:
                x = ctx.solve([beam], tol=1e-6)[0][0].contiguous()
            else:
                x = torch.from_numpy(inputs.random_vector(ctx.n, seed=10 + i) * 0.3).cuda()
            tgts.append(net.target(ctx, beam, x))
    feat = torch.stack(feats)
    tgt = torch.stack(tgts)
    f_np = _bf16_to_np(feat).reshape(-1, G, G, G, 16)
    t_np = tgt.cpu().numpy().astype(np.float64).reshape(-1, G, G, G, 6)
    return feat, tgt, f_np, t_np, f_np[..., 0]


def test_forward_matches_oracle():
    dda = _dda()
    G = 16
    p = _params(2)
    with dda.Net(G, p, max_batch=2) as net:
        feat, tgt, f_np, t_np, m_np = _batch(net, G)
        out = net.forward(feat).cpu().numpy().astype(np.float64).reshape(-1, G, G, G, 6)
    for s in range(out.shape[0]):
        ref = cn.forward(p, f_np[s], bf16_round=True)["out"]
        assert np.linalg.norm(out[s] - ref) < 1e-2 * np.linalg.norm(ref)


def test_gradient_matches_oracle():
    dda = _dda()
    G = 16
    p = _params(3)
    with dda.Net(G, p, max_batch=2) as net:
        feat, tgt, f_np, t_np, m_np = _batch(net, G)
        loss, g = net.grad(feat, tgt)
    lo, go = cn.loss_and_grad(p, f_np, t_np, m_np, bf16_round=True)
    assert abs(loss - lo) < 1e-2 * lo
    g = g.astype(np.float64)
    assert g @ go / (np.linalg.norm(g) * np.linalg.norm(go)) > 0.999
    off = 0
    for li, (ci, co, *_) in enumerate(cn.LAYERS):
        for n in (27 * ci * co, co):
            a, b = g[off:off + n], go[off:off + n]
            assert np.linalg.norm(a - b) <= 3e-2 * np.linalg.norm(b) + 1e-12, (li, n)
            off += n


def test_training_lowers_the_loss():
    dda = _dda()
    G = 16
    with dda.Net(G, cn.init_params(4), max_batch=2) as net:
        feat, tgt, *_ = _batch(net, G, solved=True)
        l0 = net.train_step(feat, tgt, 2e-3)
        for _ in range(60):
            l = net.train_step(feat, tgt, 2e-3)
        assert l < 0.3 * l0
        p = net.params()
        assert np.all(np.isfinite(p))


def test_initial_guess_check_falls_back_to_zero():
    dda = _dda()
    mask = inputs.sphere_mask(8)
    with dda.Context(mask, 1.5, 0.5) as ctx:
        xz, iz, _ = ctx.solve([inputs.X_POL], tol=1e-8)
        bad = 10 * ctx.rhs(inputs.X_POL).reshape(1, 3, ctx.n)
        xb, ib, st = ctx.solve([inputs.X_POL], tol=1e-8, x0=bad, x0_check=True)
        assert st == 0 and ib[0]["iters"] == iz[0]["iters"]
        assert torch.equal(xb, xz)
        # a good guess is kept
        xg, ig, st = ctx.solve([inputs.X_POL], tol=1e-8, x0=xz, x0_check=True)
        assert st == 0 and ig[0]["iters"] == 0


def test_trained_guess_lowers_the_initial_residual_but_not_the_iterations():
    """What the trained network gains, measured: trained on solver output for small random particles,
    its guess starts held-out solves from a residual at least a quarter below the untrained network's
    (x0 = b), yet QMR from it needs within 10 % of the iterations from a zero guess.  This is the
    negative result of the full-size runs (2,000 training and 200 held-out particles: initial residual
    0.63 against 1.02, iterations x 0.99), asserted so that a change in either direction is seen; plain
    QMR stays the fallback and the judge of convergence (every solve converges)."""
    from paper_0704_0037_amd import learned_guess as lg
    ev, _ = lg.run(grid=48, n_train=600, n_eval=16, epochs=30, batch=8, lr=1e-3, seed=5000, quiet=True)
    assert all(r["status"] == [0, 0, 0] for r in ev["rows"])
    assert ev["mean_res0_guess"] < 0.75 * ev["mean_res0_b"], ev
    assert 0.9 < ev["iteration_ratio"] < 1.1, ev
