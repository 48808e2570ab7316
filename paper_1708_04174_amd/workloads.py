"""Synthetic workloads (seeded) for the benchmark and the autotuner.

* pop_batch   - quartic POPs, n ~ U{6..16}, one Gram block of 28..153, in scaled variables.
* lyapunov    - Lyapunov programs for cubic vector fields with quadratic perturbations,
                n = 6, quartic V (203 free variables, Gram blocks 28 and 84, m = 1134);
                seeds 0..3583 train the warm-start model, 3584..4095 are held out.
Problems are generated in parallel worker processes (pure CPU data preparation).
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor
from typing import List

LYAP_TRAIN = range(0, 3584)
LYAP_TEST = range(3584, 4096)


def _pop(seed):
    from sosgen import families as F
    return F.pop_batch_member(seed)


def _lyap(seed):
    from sosgen import families as F
    return F.lyapunov(seed)


def _workers() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def generate(kind: str, seeds) -> List:
    fn = {"pop_batch": _pop, "lyapunov": _lyap}[kind]
    seeds = list(seeds)
    if len(seeds) < 32:
        return [fn(s) for s in seeds]
    with ProcessPoolExecutor(max_workers=_workers()) as ex:
        return list(ex.map(fn, seeds, chunksize=16))


def lyapunov_features(seeds):
    import numpy as np

    from sosgen import families as F
    return np.stack([F.lyapunov_features(s) for s in seeds]).astype(np.float32)
