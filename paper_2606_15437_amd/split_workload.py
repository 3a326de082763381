"""The split workload: formula pairs that agree on every model with at most 4 worlds,
searched for a separating model on the 6-, 7- and 8-world frame families
(Definition 2, Proposition 5).

Pair selection (every evaluation runs in the library's kernels):
  1. a seeded pool of random 2-variable formulas;
  2. buckets of equal signature (truth bits at 4,096 pointed models with <= 3 worlds,
     which include every model with <= 2 worlds);
  3. candidate pairs: consecutive members of each bucket, in pool order;
  4. exact check: the biconditional has no countermodel on any frame with n <= 4
     (census with early exit);
  5. a seeded sample of the survivors, plus the designed late-separating pairs.
"""
from __future__ import annotations

import numpy as np

from . import inputs as I
from . import kripke as K
from .proposal import Verifier, signatures


def bucket_pairs(sig_host: np.ndarray) -> np.ndarray:
    """(i, j) with i < j consecutive members of one signature bucket, in pool order."""
    rows = np.ascontiguousarray(sig_host).view(np.dtype((np.void, sig_host.shape[1] * 8)))
    _, inv = np.unique(rows.ravel(), return_inverse=True)
    order = np.lexsort((np.arange(len(inv)), inv))
    same = inv[order[1:]] == inv[order[:-1]]
    return np.stack([order[:-1][same], order[1:][same]], axis=1).astype(np.int64)


def config4_pairs(count: int = 20_000, pool: int = 200_000, log=None):
    """count pairs (random survivors first, designed pairs last) and selection stats."""
    import torch
    fs = I.config4_pool(pool)
    sig = signatures(fs)
    cand = bucket_pairs(K.as_u64(sig))
    del sig
    torch.cuda.empty_cache()
    if log:
        log(f"C4 pairs: {len(cand)} same-signature candidates from {pool} formulas")
    ver = Verifier(fs, panel={}, log=log)
    agree = ver.agree_through(cand[:, 0], cand[:, 1])
    surv = cand[agree]
    designed = I.config4_designed_pairs()
    want = max(0, count - len(designed))
    rng = I.SplitMix64(I.SEED_C4, 7)
    pick = []
    if len(surv) <= want:
        pick = list(range(len(surv)))
    else:
        chosen = set()
        while len(pick) < want:
            x = rng.below(len(surv))
            if x not in chosen:
                chosen.add(x)
                pick.append(x)
        pick.sort()
    pairs = [(fs[surv[x, 0]], fs[surv[x, 1]]) for x in pick] + designed
    stats = {"pool": pool, "candidates": int(len(cand)), "agree4": int(agree.sum()),
             "sampled": len(pick), "designed": len(designed), "evals": ver.evals}
    if log:
        log(f"C4 pairs: {stats}")
    return pairs, stats
