"""Training data and training loop of the learned Riemann starting guess.

The network (six face features -> ln(p*/p0), the error of Toro's adaptive
starting value p0) only serves the faces that
pass its gate (``mfm.guess_gate``): pressure ratio above 2 or a normal
velocity jump above half the mean sound speed, where Toro's adaptive guess
leaves the primitive-variable value and Newton needs the most steps.  Its
training records are the ones the flux loop itself dumps (``mfm_face_dump``,
8 floats per face: the features, the converged ln(p*/p0) and the Newton
count), from plain runs of the library's own solver.

``collect`` keeps every gated face of each dumped step and a uniform random
sample of the others, so that a set of a few steps of a large run stays
within a stated size while none of the faces the network is asked about is
dropped.  ``train`` fits the network with the library's BF16-MFMA training
step (MSE on the target), drawing every batch from the gated records.
Everything here is argument marshalling and bookkeeping on torch tensors:
the solves, the forward and backward passes and the Adam update are the
library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import mfm


def init_params(seed: int) -> np.ndarray:
    """He-initialised weights, zero biases; the padded input rows of W1
    (features 6..15) are zero and stay zero under training."""
    rng = np.random.default_rng(seed)
    p = np.zeros(mfm.mfm_mlp_param_count(), dtype=np.float32)
    for name, (off, shp) in mfm.mlp_param_layout().items():
        if name.startswith("W") or name == "w4":
            fan = mfm.MLP_NIN if name == "W1" else mfm.MLP_HID
            w = rng.normal(0.0, np.sqrt((1.0 if name == "w4" else 2.0) / fan), shp)
            if name == "W1":
                w[mfm.MLP_NIN:] = 0.0
            p[off:off + w.size] = w.ravel()
    return p


def norm_of(rows: torch.Tensor) -> np.ndarray:
    """Standardisation vector of a record set: feature means (0..5) and
    standard deviations (6..11), target mean (12) and deviation (13)."""
    r = rows[:, :7].double()
    mean, std = r.mean(0).cpu().numpy(), r.std(0).cpu().numpy()
    norm = np.zeros(mfm.MLP_NNORM, dtype=np.float32)
    norm[:6], norm[6:12] = mean[:6], np.maximum(std[:6], 1e-6)
    norm[12], norm[13] = mean[6], max(std[6], 1e-6)
    return norm


def usable(rows: torch.Tensor) -> torch.Tensor:
    """Records the network is trained and scored on: those passing the gate
    whose target is finite and below 10 in magnitude (a larger one means the
    plain starting value sat on its pressure floor)."""
    t = rows[:, 6]
    return mfm.guess_gate(rows) & torch.isfinite(t) & (t.abs() < 10.0)


class Collector:
    """Face records of the steps run on one context, with the dump armed.

    rate: probability with which a face outside the gate is kept (None: keep
    every face).  gated_budget: at most about this many gated faces are kept
    per step (a uniform sample of them when there are more; None: all).
    cap: records the dump buffer holds per step (faces beyond it are counted,
    not stored, and the step is reported as truncated)."""

    def __init__(self, ctx: mfm.Context, cap: int, rate: float | None, seed: int,
                 gated_budget: int | None = None):
        self.ctx = ctx
        self.gated_budget = gated_budget
        self.buf = torch.empty((int(cap), mfm.DUMP_STRIDE), dtype=torch.float32,
                               device=ctx.dt_dev.device)
        self.rate = rate
        self.gen = torch.Generator(device=ctx.dt_dev.device).manual_seed(seed)
        self.parts = []
        self.faces = 0
        self.gated = 0
        self.truncated = 0

    def step(self, ps: mfm.ParticleSet, dt_max: float = 1.0) -> float:
        mfm.mfm_face_dump(self.ctx, self.buf)
        dt = mfm.mfm_step(self.ctx, ps, dt_max)
        cnt = mfm.mfm_face_dump_count(self.ctx)
        mfm.mfm_face_dump(self.ctx, None)
        m = min(cnt, self.buf.shape[0])
        self.truncated += cnt - m
        rows = self.buf[:m]
        gate = mfm.guess_gate(rows)
        if self.rate is None:
            keep = torch.ones_like(gate)
        else:
            u = torch.rand(m, device=rows.device, generator=self.gen)
            ng = int(gate.sum())
            kg = gate
            if self.gated_budget is not None and ng > self.gated_budget:
                kg = gate & (u < self.gated_budget / ng)
            keep = kg | (~gate & (u < self.rate)) if self.rate > 0.0 else kg
        self.parts.append(rows[keep].clone())
        self.faces += cnt
        self.gated += int(gate.sum())
        return dt

    def rows(self) -> torch.Tensor:
        return torch.cat(self.parts) if self.parts else self.buf[:0].clone()


def split(rows: torch.Tensor, frac: float, seed: int):
    """Seeded random split into (first frac, rest)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(rows.shape[0], generator=g).to(rows.device)
    k = int(round(frac * rows.shape[0]))
    return rows[perm[:k]], rows[perm[k:]]


def train(rows: torch.Tensor, steps: int, batch: int = 16384, lr: float = 3e-3,
          seed: int = 0, stream=None):
    """Fit the network to the usable gated records of ``rows`` (device tensor
    [n, 8]); returns (MLPState, losses at the first and last step).  The
    learning rate drops to a third for the last 30% of the steps."""
    gated = rows[usable(rows)].contiguous()
    if gated.shape[0] == 0:
        raise ValueError("no usable record passes the guess gate")
    st = mfm.MLPState(init_params(seed), norm_of(gated), stream=stream,
                      device=rows.device)
    g = torch.Generator(device=rows.device).manual_seed(seed)
    n = gated.shape[0]
    losses = []
    for it in range(steps):
        idx = torch.randint(0, n, (batch,), device=rows.device, generator=g)
        want = it in (0, steps - 1)
        loss = mfm.mfm_mlp_train_step(st, gated[idx], lr if it < 0.7 * steps else lr / 3.0,
                                      want_loss=want)
        if want:
            losses.append(loss)
    return st, losses


def rms_error(st: mfm.MLPState, rows: torch.Tensor) -> float:
    """Root-mean-square error of the predicted ln(p*/p0) on the usable
    gated records of ``rows`` (nan if none)."""
    gated = rows[usable(rows)].contiguous()
    if gated.shape[0] == 0:
        return float("nan")
    y = mfm.mfm_mlp_predict(st, gated)
    return float(torch.sqrt(torch.mean((y.double() - gated[:, 6].double()) ** 2)))


def iteration_stats(rows: torch.Tensor) -> dict:
    """Newton steps per face (mean and 99th percentile) over all records
    and over the gated ones; the records of a step dumped with every face
    kept (rate None)."""
    it = rows[:, 7].round().long().clamp(min=0)
    gate = mfm.guess_gate(rows)
    out = {"faces": int(rows.shape[0]), "gated": int(gate.sum())}
    for name, v in (("all", it), ("gated", it[gate])):
        if v.numel():
            # iteration counts are small integers: the percentile from their histogram
            h = torch.cumsum(torch.bincount(v), 0)
            out[name + "_mean"] = float(v.double().mean())
            out[name + "_p99"] = int(torch.searchsorted(h, 0.99 * v.numel()))
            out[name + "_max"] = int(h.numel() - 1)
            out[name + "_over_8"] = float((v > 8).double().mean())
        else:
            out[name + "_mean"] = out[name + "_p99"] = float("nan")
    return out
