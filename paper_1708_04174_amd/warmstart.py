"""Learned warm start for a parametric SOS family (orchestration only).

The network and the solver run in libsos.so: this module moves arrays between them.

1. Training data: the solver's own batched cold solves of the training instances;
   sos_batch_export_solutions writes each converged (xi / tau, y / tau) in the
   library's layout; instances the solver reports SOLVED are kept, minus those whose
   solution norm is far above the median (training_mask).
2. Training: the device MLP (sos_mlp_*) on standardised targets, mini-batch Adam.
   The standardisation (per-output mean and spread of the training targets) and the
   choice of training rows are data preparation done once on the host (numpy); the
   mini-batches are gathered by index in the library, and the network's output layer
   undoes the standardisation on the device.
3. Use: predict (xi, y) for new instances, sos_batch_warm_start makes the prediction
   consistent with the cones (u = (P_K(xi), y, 1), v = (P_K*(c - A^T y), 0, 0)), the
   batch is solved, and every problem that the warm start does not bring to a
   SOLVED status or a certificate is solved from the cold start (the fallback): in the
   same launch when the settings carry a warm_budget, else by a second batched solve.
"""
from __future__ import annotations

import time
from typing import List, Optional, Sequence

import numpy as np

from . import binding as B


def training_mask(T_host: np.ndarray, factor: float = 3.0) -> np.ndarray:
    """Rows of the exported solutions (host array) that train the model: those whose norm is
    at most `factor` times the median norm.  Instances close to infeasibility end with a tiny
    tau, so their normalised solutions are huge (norms up to hundreds of times the median);
    left in, they dominate the target statistics and the network predicts neither them nor
    the rest."""
    nrm = np.linalg.norm(np.asarray(T_host, dtype=np.float64), axis=1)
    return nrm <= factor * np.median(nrm)


def export_solutions(batch: "B.Batch", layout: int):
    import torch
    out = torch.zeros((len(batch.works), layout), dtype=torch.float32, device="cuda")
    B.sos_batch_export_solutions(batch, out, layout)
    return out


def cold_solve_batch(works: Sequence["B.Work"], schedule: Optional[str] = None):
    """Cold-start batched solve; returns (infos, device tensor of normalised solutions, batch)."""
    batch = B.sos_batch_setup(list(works), schedule)
    B.sos_batch_reset(batch)
    infos = B.sos_batch_solve(batch)
    layout = B.sos_layout_size(works[0])
    return infos, export_solutions(batch, layout), batch


class WarmStartModel:
    """MLP (n_in -> hidden -> hidden -> n_out, GELU) trained on the device."""

    def __init__(self, n_in: int, n_out: int, hidden: int = 512, max_batch: int = 4096, seed: int = 0):
        self.n_in, self.n_out, self.hidden = n_in, n_out, hidden
        self.net = B.MLP(n_in, hidden, n_out, max_batch)
        rng = np.random.default_rng(seed)
        parts = []
        for fan_in, fan_out in ((n_in, hidden), (hidden, hidden), (hidden, n_out)):
            parts.append(rng.standard_normal(fan_in * fan_out) * np.sqrt(2.0 / fan_in))   # He initialisation
            parts.append(np.zeros(fan_out))
        self.net.set_params(np.concatenate(parts).astype(np.float32))
        self.mu = np.zeros(n_out, dtype=np.float32)
        self.sd = np.ones(n_out, dtype=np.float32)

    def fit(self, X_host: np.ndarray, T_host: np.ndarray, rows: Optional[np.ndarray] = None, epochs: int = 60,
            batch: int = 256, lr: float = 1e-3, seed: int = 0, log=None) -> List[float]:
        """X_host: (S, n_in), T_host: (S, n_out) host arrays (raw targets); rows: the rows to
        train on (default all).  The standardisation is computed on the host over those rows,
        the data go to the device once, and each mini-batch is a slice of a shuffled index list
        that the library gathers (sos_mlp_train_step_rows)."""
        import torch
        rows = np.arange(len(X_host)) if rows is None else np.asarray(rows)
        Tsel = np.asarray(T_host, dtype=np.float64)[rows]
        self.mu = Tsel.mean(axis=0).astype(np.float32)
        sd = Tsel.std(axis=0)
        self.sd = np.where(sd > 1e-8, sd, 1.0).astype(np.float32)
        Tn_host = ((np.asarray(T_host, dtype=np.float64) - self.mu) / self.sd).astype(np.float32)
        X = torch.from_numpy(np.ascontiguousarray(X_host, dtype=np.float32)).cuda()
        Tn = torch.from_numpy(np.ascontiguousarray(Tn_host)).cuda()
        rng = np.random.default_rng(seed)
        S = len(rows)
        losses = []
        for ep in range(epochs):
            perm = torch.from_numpy(rows[rng.permutation(S)].astype(np.int32)).cuda()
            tot, cnt = 0.0, 0
            for i in range(0, S - batch + 1, batch):
                want = (i + batch > S - batch)
                L = self.net.train_step_rows(X, Tn, perm[i:i + batch], lr, want_loss=want)
                if want:
                    tot, cnt = tot + L, cnt + 1
            losses.append(tot / max(cnt, 1))
            if log and (ep % 10 == 0 or ep == epochs - 1):
                log(f"[warm] epoch {ep}: loss {losses[-1]:.4f}")
        self.net.set_output_affine(self.sd, self.mu)
        return losses

    def predict(self, X, out=None):
        import torch
        if out is None:
            out = torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device="cuda")
        self.net.forward(X, out, apply_output_affine=True)
        return out


LAST_FIRST_PASS: List[dict] = []   # infos of the warm-started pass of the last warm_solve call
LAST_FALLBACK: dict = {}           # the last call's cold fallback: infos and launch times


def warm_solve(batch: "B.Batch", model: WarmStartModel, X, fallback_works: Optional[Sequence["B.Work"]] = None,
               layout: Optional[int] = None, schedule: Optional[str] = None):
    """Predict, warm start, solve (with the batch's own iteration budget); re-solve cold,
    with the fallback handles' budget, every problem the warm start left unsolved.

    Returns (infos, n_fallback, ms) with ms the device time of inference + warm start +
    solve + fallback solves."""
    import torch
    layout = layout or model.n_out
    LAST_FALLBACK.clear()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    pred = model.predict(X)
    torch.cuda.synchronize()
    B.sos_batch_warm_start(batch, pred, layout)
    infos = B.sos_batch_solve(batch)
    LAST_FIRST_PASS[:] = [dict(i) for i in infos]
    # cold re-solve of what the warm start left unsolved, unless the solve already restarted
    # it from the cold start in the same launch (warm_budget > 0; warm_iters > 0)
    bad = [i for i, inf in enumerate(infos) if inf["status"] not in (B.SOS_SOLVED, B.SOS_PRIMAL_INFEASIBLE,
                                                                     B.SOS_DUAL_INFEASIBLE) and inf["warm_iters"] == 0]
    if bad and fallback_works is not None:
        sub = [fallback_works[i] for i in bad]
        fb = B.sos_batch_setup(sub, schedule)
        B.sos_batch_reset(fb)
        finfos = B.sos_batch_solve(fb)
        LAST_FALLBACK.clear()
        LAST_FALLBACK.update(infos=[dict(f) for f in finfos], idx=list(bad),
                             phase_ms=(B.sos_batch_phase_ms(fb, 0), B.sos_batch_phase_ms(fb, 1)))
        for i, inf in zip(bad, finfos):
            inf["fallback"] = True
            infos[i] = inf
        fb.free()
    t1.record()
    torch.cuda.synchronize()
    return infos, len(bad), t0.elapsed_time(t1)
