"""Learned warm start of consecutive solution intervals.

The paper starts each new solution interval's C-ADMM iteration from the previous interval's
solution (Section 3).  Here a small network corrects that start per (subband, direction, station)
from features of the new data at the previous solution; a per-subband cost comparison keeps the
plain start wherever the correction is worse, and the LM/ADMM iteration then runs as usual, so it
both refines the prediction and judges it.

Every computation runs in the HIP library: features, targets, the fallback and the network's
forward, backward and Adam steps (calib.Calib.warmstart_* and calib.MLP).  This module only
orders the calls, keeps the training rows and shuffles them between epochs.

Episode protocol: interval 0 of an episode is solved from identity Jones matrices (with the
first-iteration gauge alignment); interval j >= 1 continues from interval j-1's whole C-ADMM state
(J, Y, Z, B_f Z), without a new alignment, so every interval keeps the gauge of the first.  Each
solve of an interval j >= 1 yields one training row per (subband, direction, station): the
features at J_{j-1} (with J_{j-2} and the previous B_f Z) and the gauge-aligned change
J_j U - J_{j-1}.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np

from . import calib, synth

DIMS = [calib.WS_FEATURES, 256, 256, 256, calib.WS_OUTPUTS]


@dataclasses.dataclass
class Interval:
    """One solved interval of an episode."""
    data: dict
    J: object            # device complex128 [P, K, N, 2, 2], converged solution
    Y: object            # device complex128 [P, K, N, 2, 2]
    Z: object            # device complex128 [K, Q, N, 2, 2]
    BZ: object           # device complex128 [P, K, N, 2, 2]
    trace: np.ndarray    # [iters, 4]
    features: Optional[object] = None   # device float32 [P*K*N, 32] at the previous solution
    target: Optional[object] = None     # device float32 [P*K*N, 8]


def solve_episode(cfg: synth.SynthConfig, episode: int, n_intervals: int, precision: int,
                  admm_iters: int, lm_iters: Optional[int] = None, rel_cost_tol: float = 0.0,
                  count: Optional[int] = None, lm_tol: float = 0.0, **ctx_kw) -> List[Interval]:
    """Solve the first ``count`` (default all) of the n_intervals intervals of one episode in
    order, each from the previous one's state, and collect features and targets of every interval
    after the first.  ctx_kw: further calib.Calib settings (solver, cg_tol, tile shapes)."""
    import torch
    out: List[Interval] = []
    for j in range(n_intervals if count is None else count):
        data = synth.episode_interval(cfg, episode, j, n_intervals)
        vis, coh, flags = calib.device_inputs(data, precision)
        prev = out[-1] if out else None
        ctx = calib.Calib(data, vis, coh, flags, precision=precision, lm_iters=lm_iters,
                          options=calib.OPT_GPA_FIRST_ITER if prev is None else 0, lm_tol=lm_tol,
                          **ctx_kw)
        feats = tgt = None
        if prev is not None:
            ctx.set_state(prev.J, prev.Y, prev.Z, prev.BZ)
            feats = ctx.warmstart_features(out[-2].J if len(out) > 1 else None, prev.BZ)
        tr = ctx.solve(admm_iters, rel_cost_tol)
        J, Y, Z, BZ = (ctx.get(f) for f in (calib.FIELD_J, calib.FIELD_Y, calib.FIELD_Z,
                                            calib.FIELD_BZ))
        if prev is not None:
            tgt = ctx.warmstart_target(prev.J)
        torch.cuda.current_stream().synchronize()
        ctx.close()
        out.append(Interval(data=data, J=J, Y=Y, Z=Z, BZ=BZ, trace=tr, features=feats, target=tgt))
    return out


class WarmStartNet:
    """The network of the learned warm start, trained with the library's own kernels."""

    def __init__(self, max_rows: int, seed: int = synth.SEED_BASE, dims=None):
        self.dims = list(DIMS if dims is None else dims)
        self.mlp = calib.MLP(self.dims, synth.mlp_init_params(self.dims, seed), max_rows)
        self.max_rows = max_rows
        self.history: List[float] = []

    def train(self, X_host: np.ndarray, Y_host: np.ndarray, epochs: int, batch: int, lr: float,
              seed: int = 0, lr_final: Optional[float] = None, log=None):
        """Minibatch Adam on mean square error over host rows X_host [n, 32] -> Y_host [n, 8];
        rows are reshuffled on the host every epoch.  The learning rate decays geometrically
        from lr to lr_final over the run.  log (optional) receives a line every ten epochs.
        Returns the wall time in seconds."""
        import torch
        n = X_host.shape[0]
        batch = min(batch, n, self.max_rows)
        rng = np.random.default_rng(seed)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        steps = epochs * (n // batch)
        decay = 1.0 if lr_final is None or steps < 2 else (lr_final / lr) ** (1.0 / (steps - 1))
        cur = lr
        t0 = time.perf_counter()
        for _ in range(epochs):
            perm = rng.permutation(n)
            Xd = torch.from_numpy(X_host[perm]).cuda()
            Yd = torch.from_numpy(Y_host[perm]).cuda()
            ep = 0.0
            nb = n // batch
            for b in range(nb):
                self.mlp.train_step(Xd[b * batch:(b + 1) * batch], Yd[b * batch:(b + 1) * batch],
                                    cur, loss)
                ep += float(loss.item()) if b == nb - 1 else 0.0
                cur *= decay
            self.history.append(ep)
            if log and len(self.history) % 10 == 0:
                log(f"epoch {len(self.history)}: loss {ep:.3e}")
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def predict(self, X):
        return self.mlp.forward(X)

    def loss(self, X, Y) -> float:
        import torch
        out = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.mlp.train_step(X, Y, 0.0, out)
        return float(out.item())

    def close(self):
        self.mlp.close()


def stack_rows(intervals: List[Interval]):
    """Host copies of the features and targets of every interval that has them, without the
    rows of directions a subband does not carry (all-zero features)."""
    X = np.concatenate([iv.features.cpu().numpy() for iv in intervals if iv.features is not None])
    Y = np.concatenate([iv.target.cpu().numpy() for iv in intervals if iv.target is not None])
    live = np.any(X != 0, axis=1)
    return np.ascontiguousarray(X[live]), np.ascontiguousarray(Y[live])


def iters_to_target(trace: np.ndarray, target_cost: float, rel: float = 1e-6,
                    primal_target: Optional[float] = None,
                    primal_rel: float = 1e-3) -> Optional[int]:
    """First ADMM iteration (1-based) whose data cost is within rel of target_cost and, when
    primal_target is given, whose primal residual is at most (1 + primal_rel) primal_target (the
    cost alone can pass through the target band while the subbands still disagree)."""
    g = trace[:, 0]
    ok = np.abs(g - target_cost) <= rel * abs(target_cost)
    if primal_target is not None:
        ok &= trace[:, 2] <= (1.0 + primal_rel) * primal_target
    hit = np.nonzero(ok)[0]
    return int(hit[0]) + 1 if len(hit) else None
