"""FP64 reference of the Riemann-guess network (test infrastructure only).

Only tests, the smoke check and the CPU leg of the benchmark import this
module; the HIP library never does.

The network is an addition to the paper: it supplies the starting value of the
Newton iteration of the exact Riemann solver the paper uses for its fluxes
(sec. 2.3.3, Toro's solver), which then converges to the same root whatever
the start.  What is fixed here, in plain numpy and FP64:

* the six face features of a Riemann problem (face frame, after
  reconstruction): ln(rho_L/rho_R), ln(P_L/P_R), slog(du / c_avg) -- which
  with gamma fix p* -- and the exact solver's starting value p0 (Toro's
  adaptive choice, ``oracle.riemann_guess``) as ln(p0 / P_avg) with two
  indicators of its estimate; the target y = ln(p* / p0), the error of p0,
  with p* from the oracle's exact solver;
* the perceptron 6 -> 64 -> 64 -> 64 -> 1 with SiLU hidden activations: a
  layer computes a_out[n] = silu(b[n] + sum_k a_in[k] W[k][n]); the output is
  b4 + sum_k a3[k] w4[k];
* inputs standardised with norm[0:6] (means) and norm[6:12] (standard
  deviations), the output mapped back as norm[12] + norm[13] * net;
* the loss (mean squared error in standardised target units) and its gradient
  by back-propagation, and one Adam step.

The parameter vector is flat FP32-compatible, ordered W1 [16][64] (rows 6..15
are padding), b1, W2 [64][64], b2, W3 [64][64], b3, w4 [64], b4.

Pins (tests/test_oracle_mlp.py): the gradient against central finite
differences; a hand-evaluated single-path network (one non-zero weight per
layer) that catches transposed or shifted weights; the features' mirror
symmetry (with the starting value's) and the target of Sod's problem from
Toro's tables.
"""
from __future__ import annotations

import numpy as np

NIN, K1, HID = 6, 16, 64
SHAPES = [("W1", (K1, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("w4", (HID,)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(params) -> dict:
    """Views of the flat parameter vector by name (FP64 copies)."""
    p = np.asarray(params, dtype=np.float64)
    assert p.size == NPARAM
    out, off = {}, 0
    for name, shp in SHAPES:
        size = int(np.prod(shp))
        out[name] = p[off:off + size].reshape(shp)
        off += size
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed: int) -> np.ndarray:
    """He-style random initialisation (padding rows of W1 zero)."""
    rng = np.random.default_rng(seed)
    d = {}
    d["W1"] = np.zeros((K1, HID))
    d["W1"][:NIN] = rng.normal(0, np.sqrt(2.0 / NIN), (NIN, HID))
    d["b1"] = np.zeros(HID)
    d["W2"] = rng.normal(0, np.sqrt(2.0 / HID), (HID, HID))
    d["b2"] = np.zeros(HID)
    d["W3"] = rng.normal(0, np.sqrt(2.0 / HID), (HID, HID))
    d["b3"] = np.zeros(HID)
    d["w4"] = rng.normal(0, np.sqrt(1.0 / HID), HID)
    d["b4"] = np.zeros(1)
    return pack(d)


def bf16(a) -> np.ndarray:
    """Round FP32 values to the nearest BF16 value (ties to even), as FP64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def slog(v):
    return np.sign(v) * np.log1p(np.abs(v))


def features(rL, pL, rR, pR, du, cL, cR, p0, branch) -> np.ndarray:
    """The six features of a face's Riemann problem (arrays broadcast; last
    axis = feature): ln(rho_L/rho_R), ln(P_L/P_R), slog(du / c_avg), and the
    plain starting value p0 as ln(p0 / P_avg) with two indicators of the
    estimate it came from (two-rarefaction, two-shock)."""
    b = np.asarray(branch)
    return np.stack(np.broadcast_arrays(
        np.log(rL / rR), np.log(pL / pR), slog(du / (0.5 * (cL + cR))),
        np.log(p0 / (0.5 * (pL + pR))), (b == 1).astype(np.float64),
        (b == 2).astype(np.float64)), axis=-1)


def standardise(X, norm, round_bf16=False):
    Xs = (np.asarray(X, dtype=np.float64) - norm[:NIN]) / norm[NIN:2 * NIN]
    return bf16(Xs) if round_bf16 else Xs


def forward(params, norm, X, round_bf16=False, keep=False):
    """Predicted y for the rows of X (n x 6).  round_bf16 rounds the weight
    matrices and the standardised inputs to BF16 first (the tensors the matrix
    cores see); everything else is FP64."""
    P = unpack(params)
    W = [P["W1"][:NIN], P["W2"], P["W3"]]
    if round_bf16:
        W = [bf16(w) for w in W]
    b = [P["b1"], P["b2"], P["b3"]]
    a = standardise(X, norm, round_bf16)
    acts, zs = [a], []
    for layer in range(3):
        z = a @ W[layer] + b[layer]
        a = silu(z)
        zs.append(z)
        acts.append(a)
    y = a @ P["w4"] + P["b4"][0]
    out = norm[2 * NIN] + norm[2 * NIN + 1] * y
    if keep:
        return out, (y, acts, zs, W)
    return out


def loss_grad(params, norm, X, t, round_bf16=False):
    """Mean squared error in standardised target units and its gradient with
    respect to the flat parameter vector."""
    n = X.shape[0]
    _, (y, acts, zs, W) = forward(params, norm, X, round_bf16, keep=True)
    ts = (np.asarray(t, dtype=np.float64) - norm[2 * NIN]) / norm[2 * NIN + 1]
    err = y - ts
    loss = float(np.mean(err * err))
    P = unpack(params)
    g = {k: np.zeros_like(v) for k, v in P.items()}
    dy = 2.0 * err / n
    g["w4"] = acts[3].T @ dy
    g["b4"] = np.array([dy.sum()])
    dz = np.outer(dy, P["w4"]) * dsilu(zs[2])
    for layer, (wn, bn) in zip((2, 1, 0), (("W3", "b3"), ("W2", "b2"), ("W1", "b1"))):
        gw = acts[layer].T @ dz
        if wn == "W1":
            g["W1"][:NIN] = gw
        else:
            g[wn] = gw
        g[bn] = dz.sum(axis=0)
        if layer > 0:
            dz = (dz @ W[layer].T) * dsilu(zs[layer - 1])
    return loss, pack(g)


def adam(params, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def norm_from(X, t) -> np.ndarray:
    """Normalisation vector (16 entries) from training features and targets."""
    norm = np.zeros(16)
    norm[:NIN] = X.mean(axis=0)
    norm[NIN:2 * NIN] = np.maximum(X.std(axis=0), 1e-6)
    norm[2 * NIN] = t.mean()
    norm[2 * NIN + 1] = max(t.std(), 1e-6)
    return norm
