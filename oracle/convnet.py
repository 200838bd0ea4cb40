"""Oracle of the learned initial guess: a small 3-D convolutional network, its loss and its
exact gradient, in plain numpy.  TEST INFRASTRUCTURE ONLY (tests, the smoke check and the
benchmark's CPU leg); never imported by the product path.

The paper has no learned component: this is the extension that supplies QMR's starting vector
(the paper's iterative solver starts from an initial guess it does not discuss, Sec. 2).  The
network, its inputs and outputs are this project's own definition, written out here as the
reference the GPU kernels must reproduce.

Network (grid G per side, G a multiple of 8; channels-last arrays [G][G][G][C], z slowest):

    e0 = relu(conv(f,  W0) + b0)              G,    16 -> 16
    e1 = relu(conv(pool(e0), W1) + b1)        G/2,  16 -> 32
    e2 = relu(conv(pool(e1), W2) + b2)        G/4,  32 -> 48
    e3 = relu(conv(pool(e2), W3) + b3)        G/8,  48 -> 64
    d2 = relu(conv(up(e3), W4) + b4 + e2)     G/4,  64 -> 48
    d1 = relu(conv(up(d2), W5) + b5 + e1)     G/2,  48 -> 32
    d0 = relu(conv(up(d1), W6) + b6 + e0)     G,    32 -> 16
    out = conv(d0, W7) + b7                   G,    16 -> 6

conv: 3x3x3 cross-correlation with zero padding, W[t][co][ci], tap t = 9(dz+1) + 3(dy+1) + (dx+1)
  y[z,y,x,co] = sum_t sum_ci x[z+dz, y+dy, x+dx, ci] W[t, co, ci]
pool: mean over 2x2x2 blocks; up: nearest-neighbour doubling.

Parameters, canonical flat layout (float32): for each layer in order, W (27*Cout*Cin, tap-major,
then Cout, then Cin) followed by b (Cout).

Input features (16 channels) for a particle on an n = (nx, ny, nz) grid placed in the G^3 box at
offset o = (G - n) // 2 per axis, at box cell (X, Y, Z) with particle-frame position
r = (X - ox + 1/2 - nx/2, ...):
    0 mask, 1 (Re m - 1) mask, 2 (Im m) mask, 3 kd (everywhere),
    4..9 Re/Im of the incident field E_inc(r) = e exp(i kd a.r) components x, y, z (everywhere),
    10..15 Re/Im of (m^2 - 1) E_inc(r) mask, components x, y, z (the product a ReLU network
    cannot form from the other channels).
Output / target (6 channels): Re/Im of delta = E_exc - E_inc per component at the dipoles, with
E_exc = x / beta the exciting field of the solution x of A x = b (P = beta x, eq. 3).  The guess
is x0 = beta (E_inc + delta).
Loss: mean over dipole cells (all samples of a batch together) of sum_c (out - target)^2.

Precision: with bf16=True the oracle rounds, to bfloat16 (round to nearest even), exactly the
tensors the GPU stores in bfloat16: features, weights, every stored activation and every stored
gradient tensor of the backward pass; everything else is float64.  With bf16=False it is the
exact float64 function, which the finite-difference pins check.

Pins (tests/test_oracle_convnet.py): conv against scipy.signal.correlate and a brute-force loop;
pool/up adjointness; the analytic gradient against central finite differences of the float64
loss; features against the DDA oracle's incident field; target/guess round trip.
"""
from __future__ import annotations

import numpy as np

N_IN, N_OUT = 16, 6
LEVELS = (16, 32, 48, 64)
# (cin, cout, level, input kind, skip)
LAYERS = (
    (N_IN, 16, 0, "plain", None),
    (16, 32, 1, "pool", None),
    (32, 48, 2, "pool", None),
    (48, 64, 3, "pool", None),
    (64, 48, 2, "up", "e2"),
    (48, 32, 1, "up", "e1"),
    (32, 16, 0, "up", "e0"),
    (16, N_OUT, 0, "plain", None),
)
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def num_params():
    """Number of network parameters (bookkeeping, no arithmetic of the method)."""
    return sum(27 * ci * co + co for ci, co, *_ in LAYERS)


def unflatten(p):
    """Flat canonical vector -> list of (W [27][co][ci], b [co]) float64 (bookkeeping; the GPU
    parameter layout is checked against it by the network's parity tests)."""
    p = np.asarray(p, dtype=np.float64)
    out, o = [], 0
    for ci, co, *_ in LAYERS:
        W = p[o:o + 27 * co * ci].reshape(27, co, ci)
        o += 27 * co * ci
        b = p[o:o + co]
        o += co
        out.append((W, b))
    assert o == p.size
    return out


def flatten(layers):
    """Inverse of unflatten (bookkeeping)."""
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


def init_params(seed):
    """He-normal weights (std sqrt(2 / (27 cin))), zero biases; the head is scaled by 0.1
    (seeded initial values, no arithmetic of the method)."""
    rng = np.random.default_rng(seed)
    layers = []
    for li, (ci, co, *_) in enumerate(LAYERS):
        W = rng.standard_normal((27, co, ci)) * np.sqrt(2.0 / (27 * ci))
        if li == len(LAYERS) - 1:
            W *= 0.1
        layers.append((W, np.zeros(co)))
    return flatten(layers).astype(np.float32)


def bf16(x):
    """Round to bfloat16 (nearest even), returned as float64.

    pinned by: test_oracle_convnet.py::test_bf16_rounding_and_rounded_gradient_close_to_exact.
    """
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ------------------------------------------------------------------------------ operators
def conv3d(x, W):
    """3x3x3 zero-padded cross-correlation: x [D][H][W][ci], W [27][co][ci] -> [D][H][W][co].

    pinned by: test_oracle_convnet.py::test_conv_matches_scipy_correlate and
        test_conv_brute_force_and_single_tap_shift.
    """
    D, H, Wd, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((D, H, Wd, W.shape[1]))
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += xp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd, :] @ W[t].T
    return y


def conv3d_weight_grad(x, g):
    """d/dW of sum(g * conv3d(x, W)): [27][co][ci].

    pinned by: test_oracle_convnet.py::test_gradient_matches_finite_differences.
    """
    D, H, Wd, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    gf = g.reshape(-1, g.shape[-1])
    out = []
    for dz, dy, dx in TAPS:
        xs = xp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd, :].reshape(-1, x.shape[-1])
        out.append(gf.T @ xs)
    return np.stack(out)


def conv3d_input_grad(g, W):
    """d/dx of sum(g * conv3d(x, W)): the correlation with the flipped, transposed kernel.

    pinned by: test_oracle_convnet.py::test_pool_up_adjoint_and_conv_adjoints.
    """
    Wt = np.stack([W[26 - t].T for t in range(27)])  # [27][ci][co]
    return conv3d(g, Wt)


def pool(x):
    """2x2x2 average pooling.

    pinned by: test_oracle_convnet.py::test_pool_up_adjoint_and_conv_adjoints.
    """
    D, H, Wd, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, Wd // 2, 2, C).mean(axis=(1, 3, 5))


def up(x):
    """Nearest-neighbour 2x up-sampling along each axis.

    pinned by: test_oracle_convnet.py::test_pool_up_adjoint_and_conv_adjoints.
    """
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def pool_adjoint(g):
    """d/dx of sum(g * pool(x)).

    pinned by: test_oracle_convnet.py::test_pool_up_adjoint_and_conv_adjoints (adjoint identity <g,
        pool x> = <pool* g, x>).
    """
    return up(g) / 8.0


def up_adjoint(g):
    """d/dx of sum(g * up(x)).

    pinned by: test_oracle_convnet.py::test_pool_up_adjoint_and_conv_adjoints.
    """
    D, H, Wd, C = g.shape
    return g.reshape(D // 2, 2, H // 2, 2, Wd // 2, 2, C).sum(axis=(1, 3, 5))


# ------------------------------------------------------------------------------ network
def forward(params, feat, bf16_round=False):
    """Activations of one sample (feat [G][G][G][16], the 16 input channels) as a dict; 'out' is the prediction.

    pinned by: test_oracle_convnet.py::test_gradient_matches_finite_differences.
    """
    r = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    layers = [(r(W), np.asarray(b, dtype=np.float64)) for W, b in unflatten(params)]
    a = {"f": r(feat)}
    prev = "f"
    names = ["e0", "e1", "e2", "e3", "d2", "d1", "d0", "out"]
    for li, (ci, co, lev, kind, skip) in enumerate(LAYERS):
        x = a[prev]
        if kind == "pool":
            x = r(pool(x))
            a["p" + names[li - 1]] = x
        elif kind == "up":
            x = up(x)
        W, b = layers[li]
        pre = conv3d(x, W) + b
        if skip is not None:
            pre = pre + a[skip]
        name = names[li]
        a[name] = pre if name == "out" else r(np.maximum(pre, 0.0))
        a["in_" + name] = x
        prev = name
    return a


def loss_and_grad(params, feats, targets, masks, bf16_round=False):
    """Masked mean-square loss over a batch and its gradient w.r.t. the flat parameters.

    feats [B][G][G][G][16], targets [B][G][G][G][6], masks [B][G][G][G] (0/1).
    pinned by: test_oracle_convnet.py::test_gradient_matches_finite_differences.
    """
    r = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    layers = [(r(W), b) for W, b in unflatten(params)]
    n = float(np.sum(masks))
    total = 0.0
    grads = [(np.zeros_like(W), np.zeros_like(b)) for W, b in layers]
    names = ["e0", "e1", "e2", "e3", "d2", "d1", "d0", "out"]
    for s in range(feats.shape[0]):
        a = forward(params, feats[s], bf16_round)
        diff = (a["out"] - targets[s]) * masks[s][..., None]
        total += float(np.sum(diff * diff))
        g = {"out": r(2.0 * diff / n)}  # gradient w.r.t. each layer's output (post-activation)
        for li in range(len(LAYERS) - 1, -1, -1):
            ci, co, lev, kind, skip = LAYERS[li]
            name = names[li]
            gy = g[name]
            if name != "out":
                gy = gy * (a[name] > 0)  # through relu
            W, _ = layers[li]
            dW = conv3d_weight_grad(a["in_" + name], gy)
            grads[li] = (grads[li][0] + dW, grads[li][1] + gy.reshape(-1, co).sum(axis=0))
            if skip is not None:
                g[skip + "_skip"] = gy
            if li == 0:
                break
            gx = r(conv3d_input_grad(gy, W))
            prev = names[li - 1]
            if kind == "up":
                g[prev] = r(up_adjoint(gx))
            elif kind == "pool":
                # prev feeds this layer through pool and, for the encoder, the decoder's skip
                gsum = pool_adjoint(gx)
                if prev + "_skip" in g:
                    gsum = gsum + g[prev + "_skip"]
                g[prev] = r(gsum)
            else:
                g[prev] = gx
    return total / n, flatten(grads)


# ---------------------------------------------------------------------- DDA coupling
def box_offset(grid, G):
    """Offset (x, y, z) of a grid of `grid` cells centred in the G^3 box.

    pinned by: test_oracle_convnet.py::test_features_target_guess_against_dda_oracle.
    """
    nx, ny, nz = grid
    return (G - nx) // 2, (G - ny) // 2, (G - nz) // 2


def box_positions(grid, G):
    """Particle-frame positions of every box cell, [G][G][G][3] (x, y, z).

    pinned by: test_oracle_convnet.py::test_features_target_guess_against_dda_oracle.
    """
    nx, ny, nz = grid
    ox, oy, oz = box_offset(grid, G)
    c = np.arange(G) + 0.5
    Z, Y, X = np.meshgrid(c - oz - nz / 2, c - oy - ny / 2, c - ox - nx / 2, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def box_mask(mask, G):
    """mask [nz][ny][nx] placed in the G^3 box.

    pinned by: test_oracle_convnet.py::test_features_target_guess_against_dda_oracle.
    """
    nz, ny, nx = mask.shape
    ox, oy, oz = box_offset((nx, ny, nz), G)
    out = np.zeros((G, G, G))
    out[oz:oz + nz, oy:oy + ny, ox:ox + nx] = mask != 0
    return out


def features(mask, m, kd, prop, pol, G):
    """The network's 16 input channels on the G^3 box for a particle and a beam.

    pinned by: test_oracle_convnet.py::test_features_target_guess_against_dda_oracle (against the
        DDA oracle's incident field and polarizability).
    """
    nz, ny, nx = mask.shape
    mk = box_mask(mask, G)
    r = box_positions((nx, ny, nz), G)
    a = np.asarray(prop, dtype=np.float64)
    e = np.asarray(pol, dtype=np.complex128)
    E = np.exp(1j * kd * (r @ a))[..., None] * e
    f = np.zeros((G, G, G, N_IN))
    f[..., 0] = mk
    f[..., 1] = (np.real(m) - 1.0) * mk
    f[..., 2] = np.imag(m) * mk
    f[..., 3] = kd
    f[..., 4:10:2] = E.real
    f[..., 5:10:2] = E.imag
    P = (m * m - 1.0) * E * mk[..., None]
    f[..., 10::2] = P.real
    f[..., 11::2] = P.imag
    return f


def dipole_cells(mask, G):
    """Flat box indices (z, y, x order) of the dipoles, in the dipole order of the lattice.

    pinned by: test_oracle_convnet.py::test_features_target_guess_against_dda_oracle.
    """
    nz, ny, nx = mask.shape
    ox, oy, oz = box_offset((nx, ny, nz), G)
    z, y, x = np.nonzero(mask)
    return ((z + oz) * G + (y + oy)) * G + (x + ox)


def target(mask, kd, beta, prop, pol, x, G):
    """x (N, 3) solution -> [G][G][G][6] target (Re/Im of x / beta - E_inc at the dipoles).

    pinned by: test_oracle_convnet.py::test_features_target_guess_against_dda_oracle (target and
        guess invert each other).
    """
    from . import dda as odda
    pos, _ = odda.dipoles(mask)
    Einc = odda.incident_field(pos, kd, prop, pol)
    d = x / beta - Einc
    t = np.zeros((G * G * G, N_OUT))
    idx = dipole_cells(mask, G)
    t[idx, 0::2] = d.real
    t[idx, 1::2] = d.imag
    return t.reshape(G, G, G, N_OUT)


def guess(mask, kd, beta, prop, pol, out, G):
    """Network output [G][G][G][6] -> initial guess x0 (N, 3) = beta (E_inc + delta).

    pinned by: test_oracle_convnet.py::test_features_target_guess_against_dda_oracle.
    """
    from . import dda as odda
    pos, _ = odda.dipoles(mask)
    Einc = odda.incident_field(pos, kd, prop, pol)
    o = out.reshape(-1, N_OUT)[dipole_cells(mask, G)]
    return beta * (Einc + o[:, 0::2] + 1j * o[:, 1::2])
