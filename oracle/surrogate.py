"""FP64 reference of the learned three-body pair surrogate.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): used by the tests,
the smoke check and the benchmark's CPU baseline, never by the product path,
and sharing no code with the GPU kernels.

The paper has no learned part; the model is defined here, and the GPU
kernels implement the same definition:

* neighbours: unordered pairs with minimum-image r^2 < rc^2 (strict, FP64,
  the same decision as the exact path's pair rule, Sec. 2);
* radial channels a = 0..15: g_a(r) = exp(-((r - mu_a)/w)^2) fc(r),
  mu_a = R0 + a w, w = (rc - R0)/15, R0 = 0.8, fc(r) = (1 + cos(pi r/rc))/2;
* descriptors of molecule i over its neighbours j, u_ij = (r_j - r_i)/r_ij:
  S_a = sum g_a, V_a = sum g_a u, Q_a = sum g_a (u u^T - I/3);
  D_raw = [S_a, |V_a|^2, Q_a:Q_a, V_a^T Q_a V_a] (64 invariants), normalised
  D = (D_raw - mean) * inv_sd with statistics fixed at model set-up;
* pair input x_ij = [D_i + D_j, g(r_ij)] (80), symmetric in i and j;
* MLP 80 -> 128 -> 128 -> 128 -> 2 with ReLU; outputs s_ij and t_ij;
* three-body force F_i = sum_j s_ij (r_i - r_j)/r_ij (Newton 3 exact);
* error estimate e_i = sum_j softplus(t_ij);
* loss L = mean_i |F_i - T_i|^2 + lam * mean_i (e_i - |F_i - T_i|)^2 with the
  second target held constant;
* Adam (Kingma and Ba) with bias correction.

``bf16=True`` rounds, to bfloat16 with round-to-nearest-even, exactly the
operands the GPU feeds its BF16 matrix instructions (the descriptors, their
pair sum and W1; g; the biases b1, b2, b3; the layer inputs h1, h2 and W2,
W3; in the backward pass h3 and dL/d(s,t) for the W4 gradient, the layer
deltas and W2, W3, and dL/dA), so that the comparison with the kernels
measures only accumulation order.  With ``bf16=False`` everything is FP64.
"""
from __future__ import annotations

import numpy as np

NR = 16
NDESC = 4 * NR
NIN = NDESC + NR
WIDTH = 128
NOUT = 2
R0 = 0.8


# --------------------------------------------------------------------------
# bfloat16 rounding (round to nearest, ties to even), values kept as float64
# --------------------------------------------------------------------------
def bf16(x):
    """Round to the nearest bfloat16 (ties to even); returns float64."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(a)
    if nan.any():
        out[nan] = np.nan
    return out.reshape(np.shape(x))


def _q(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
def min_image(d, box):
    """d -= L * rint(d / L) per component (rint: half to even)."""
    return d - box * np.rint(d / box)


def neighbour_pairs(pos, box, rc):
    """Unordered pairs (i < j) with minimum-image r^2 < rc^2, sorted by (i, j),
    and their displacement r_i - r_j.  Candidates come from a periodic k-d tree
    query (a library primitive); the decision is the FP64 expression
    dx*dx + dy*dy + dz*dz < rc*rc evaluated left to right."""
    from scipy.spatial import cKDTree
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    wrapped = pos - box * np.floor(pos / box)
    wrapped = np.where(wrapped >= box, 0.0, wrapped)
    tree = cKDTree(wrapped, boxsize=box)
    cand = tree.query_pairs(rc * (1 + 1e-9), output_type="ndarray")
    if len(cand) == 0:
        return np.zeros((0, 2), np.int64), np.zeros((0, 3))
    i = np.minimum(cand[:, 0], cand[:, 1])
    j = np.maximum(cand[:, 0], cand[:, 1])
    d = min_image(pos[i] - pos[j], box)
    r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    keep = r2 < rc * rc
    i, j, d = i[keep], j[keep], d[keep]
    order = np.lexsort((j, i))
    return np.stack([i[order], j[order]], axis=1), d[order]


def radial(r, rc):
    """g_a(r) for a = 0..15, shape (len(r), 16)."""
    w = (rc - R0) / (NR - 1)
    mu = R0 + w * np.arange(NR)
    fc = 0.5 * (1.0 + np.cos(np.pi * r / rc))
    return np.exp(-(((r[:, None] - mu[None, :]) / w) ** 2)) * fc[:, None]


def raw_descriptors(n, pairs, disp, rc):
    """D_raw (n, 64) from the neighbour pairs (each pair feeds both ends)."""
    r = np.sqrt(np.sum(disp * disp, axis=1))
    g = radial(r, rc)
    S = np.zeros((n, NR))
    V = np.zeros((n, NR, 3))
    Q = np.zeros((n, NR, 3, 3))
    eye3 = np.eye(3) / 3.0
    for side, sign in ((0, -1.0), (1, 1.0)):
        # for molecule i = pairs[:, 0] the neighbour direction is r_j - r_i = -disp
        m = pairs[:, side]
        u = sign * disp / r[:, None]
        uu = u[:, :, None] * u[:, None, :] - eye3
        np.add.at(S, m, g)
        np.add.at(V, m, g[:, :, None] * u[:, None, :])
        np.add.at(Q, m, g[:, :, None, None] * uu[:, None, :, :])
    vv = np.sum(V * V, axis=2)
    qq = np.sum(Q * Q, axis=(2, 3))
    vqv = np.einsum("nai,naij,naj->na", V, Q, V)
    return np.concatenate([S, vv, qq, vqv], axis=1)


def descriptor_stats(draw):
    """Normalisation fixed at set-up: per-feature mean and 1/max(sd, 1e-6)."""
    m = draw.mean(axis=0)
    sd = draw.std(axis=0)
    return m, 1.0 / np.maximum(sd, 1e-6)


# --------------------------------------------------------------------------
# model
# --------------------------------------------------------------------------
def init_params(seed=0):
    """He-style initial weights (seeded).  W1 rows: 64 descriptor inputs then
    16 radial inputs."""
    rng = np.random.default_rng(seed)
    p = {
        "W1": rng.normal(0, np.sqrt(2.0 / NIN), (NIN, WIDTH)),
        "b1": np.zeros(WIDTH),
        "W2": rng.normal(0, np.sqrt(2.0 / WIDTH), (WIDTH, WIDTH)),
        "b2": np.zeros(WIDTH),
        "W3": rng.normal(0, np.sqrt(2.0 / WIDTH), (WIDTH, WIDTH)),
        "b3": np.zeros(WIDTH),
        "W4": rng.normal(0, np.sqrt(1.0 / WIDTH), (WIDTH, NOUT)) * 0.1,
        "b4": np.array([0.0, -3.0]),
    }
    return p


PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")


def softplus(x):
    return np.logaddexp(0.0, x)


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def forward(params, D, pairs, disp, rc, bf16_ops=False):
    """Per-pair outputs and per-molecule force / error estimate.

    Returns a dict with s, t (per pair), F (n, 3), e (n,) and the cached
    activations the backward pass needs."""
    q = bf16_ops
    n = D.shape[0]
    r = np.sqrt(np.sum(disp * disp, axis=1))
    u = disp / r[:, None]                       # (r_i - r_j)/r
    g = radial(r, rc)
    W1a, W1b = params["W1"][:NDESC], params["W1"][NDESC:]
    i, j = pairs[:, 0], pairs[:, 1]
    # x = [D_i + D_j, g(r_ij)]; in BF16 mode the descriptor sum is formed from
    # the BF16 descriptors (exact in FP32) and rounded once more, the biases
    # of the hidden layers enter the products as BF16 values, and the output
    # layer takes BF16 h3 and W4 (b4 stays exact)
    dsum = _q(_q(D[i], q) + _q(D[j], q), q)
    z1 = dsum @ _q(W1a, q) + _q(g, q) @ _q(W1b, q) + _q(params["b1"], q)
    h1 = np.maximum(z1, 0.0)
    z2 = _q(h1, q) @ _q(params["W2"], q) + _q(params["b2"], q)
    h2 = np.maximum(z2, 0.0)
    z3 = _q(h2, q) @ _q(params["W3"], q) + _q(params["b3"], q)
    h3 = np.maximum(z3, 0.0)
    out = _q(h3, q) @ _q(params["W4"], q) + params["b4"]
    s, t = out[:, 0], out[:, 1]
    F = np.zeros((n, 3))
    np.add.at(F, i, s[:, None] * u)
    np.add.at(F, j, -s[:, None] * u)
    sp = softplus(t)
    e = np.zeros(n)
    np.add.at(e, i, sp)
    np.add.at(e, j, sp)
    return {"s": s, "t": t, "F": F, "e": e, "u": u, "g": g, "z1": z1, "h1": h1, "z2": z2, "h2": h2,
            "z3": z3, "h3": h3, "D": D}


def loss(F, e, T, lam=1.0):
    n = F.shape[0]
    dF = F - T
    nrm = np.sqrt(np.sum(dF * dF, axis=1))
    return float(np.sum(dF * dF) / n + lam * np.sum((e - nrm) ** 2) / n)


def backward(params, cache, pairs, T, lam=1.0, bf16_ops=False):
    """Gradients of `loss` with respect to every parameter (same keys)."""
    q = bf16_ops
    F, e, u = cache["F"], cache["e"], cache["u"]
    n = F.shape[0]
    i, j = pairs[:, 0], pairs[:, 1]
    dF = F - T
    nrm = np.sqrt(np.sum(dF * dF, axis=1))
    gF = 2.0 * dF / n                           # dL/dF_i
    ge = 2.0 * lam * (e - nrm) / n              # dL/de_i (target held constant)
    ds = np.sum((gF[i] - gF[j]) * u, axis=1)    # dL/ds_ij
    dt = (ge[i] + ge[j]) * sigmoid(cache["t"])  # dL/dt_ij
    dout = np.stack([ds, dt], axis=1)
    grads = {}
    grads["W4"] = _q(cache["h3"], q).T @ _q(dout, q)
    grads["b4"] = dout.sum(axis=0)
    dz3 = (dout @ params["W4"].T) * (cache["z3"] > 0)
    grads["W3"] = _q(cache["h2"], q).T @ _q(dz3, q)
    grads["b3"] = dz3.sum(axis=0)
    dz2 = (_q(dz3, q) @ _q(params["W3"], q).T) * (cache["z2"] > 0)
    grads["W2"] = _q(cache["h1"], q).T @ _q(dz2, q)
    grads["b2"] = dz2.sum(axis=0)
    dz1 = (_q(dz2, q) @ _q(params["W2"], q).T) * (cache["z1"] > 0)
    grads["b1"] = dz1.sum(axis=0)
    dW1b = _q(cache["g"], q).T @ _q(dz1, q)
    dA = np.zeros((n, WIDTH))
    np.add.at(dA, i, dz1)
    np.add.at(dA, j, dz1)
    dW1a = _q(cache["D"], q).T @ _q(dA, q)
    grads["W1"] = np.concatenate([dW1a, dW1b], axis=0)
    return grads


def adam_step(params, grads, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; `state` holds m, v and the step count."""
    state["step"] = state.get("step", 0) + 1
    k = state["step"]
    for name in PARAM_ORDER:
        g = grads[name]
        m = state.setdefault("m_" + name, np.zeros_like(g))
        v = state.setdefault("v_" + name, np.zeros_like(g))
        m[...] = beta1 * m + (1 - beta1) * g
        v[...] = beta2 * v + (1 - beta2) * g * g
        mh = m / (1 - beta1 ** k)
        vh = v / (1 - beta2 ** k)
        params[name] = params[name] - lr * mh / (np.sqrt(vh) + eps)
    return params


def predict(params, stats, pos, box, rc=2.5, bf16_ops=False):
    """Three-body force, error estimate and pair outputs of a configuration."""
    pairs, disp = neighbour_pairs(pos, box, rc)
    draw = raw_descriptors(len(pos), pairs, disp, rc)
    D = (draw - stats[0]) * stats[1]
    c = forward(params, D, pairs, disp, rc, bf16_ops=bf16_ops)
    c["pairs"] = pairs
    c["disp"] = disp
    return c
