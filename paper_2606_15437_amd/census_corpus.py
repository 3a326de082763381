"""The five-world census of Section 6 on the library's kernels.

Corpus: every constant-free formula of at most seven nodes over two variables
(44,678 trees), one representative per class of equal truth at every pointed model
with at most three worlds (the first member in enumeration order), plus the named
axioms K, T and McKinsey.  Census: for each formula and class K, T, S4, S5, every frame with
n = 1..5 worlds and every valuation, recording the failure count per n, the least
countermodel at each n and the minimal countermodel size (Section 6, Proposition 4,
Corollary 1).  Every evaluation runs in the library's kernels; n = 5 is one fused
all-class launch.
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs as I
from . import kripke as K

CLASSES = ("K", "T", "S4", "S5")
# frames per class at n = 1..5 (S4: preorders, S5: equivalence relations)
CLASS_FRAMES = {
    "K": [2, 16, 512, 65536, 33554432],
    "T": [1, 4, 64, 4096, 1048576],
    "S4": [1, 4, 29, 355, 6942],
    "S5": [1, 2, 5, 15, 52],
}


def corpus_classes(formulas, chunk=4096):
    """(representatives, class id per formula): classes of equal truth at every
    pointed model with at most three worlds; a class's representative is its first
    member in the given order."""
    import torch
    samples = I.all_pointed_models(3, 2)
    words = len(samples) // 64
    sig = np.empty((len(formulas), words), dtype=np.uint64)
    for s in range(0, len(formulas), chunk):
        sub = formulas[s:s + chunk]
        d = torch.zeros((len(sub), words), dtype=torch.int64, device="cuda")
        K.kripke_signatures(*I.pack(sub), 2, samples, d)
        sig[s:s + len(sub)] = K.as_u64(d)
        del d
    rows = np.ascontiguousarray(sig).view(np.dtype((np.void, words * 8))).ravel()
    _, first, inv = np.unique(rows, return_index=True, return_inverse=True)
    # renumber classes by their first member
    order = np.argsort(first, kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(len(order))
    return np.sort(first), rank[inv]


def build_corpus(log=None):
    t0 = time.time()
    raw = I.enumerate_formulas(7)
    reps, _ = corpus_classes(raw)
    corpus = [raw[i] for i in reps] + I.named_axioms()
    if log:
        log(f"corpus: {len(raw)} trees -> {len(reps)} classes on <= 3 worlds + "
            f"{len(I.named_axioms())} named axioms ({time.time() - t0:.1f} s)")
    return raw, reps, corpus


def census(formulas, log=None, tune_cache=None):
    """Per formula and class: fail counts and least keys at n = 1..5, minimal
    countermodel size (0: none through five worlds), timings and evaluation count.
    tune_cache: autotuner cache for the five-world plan (None: default tiles)."""
    import torch
    code, offs = I.pack(formulas)
    B = len(formulas)
    keys = np.full((4, 5, B), K.NO_KEY, dtype=np.uint64)
    counts = np.zeros((4, 5, B), dtype=np.uint64)
    torch.cuda.synchronize()
    t0 = time.time()
    for n in range(1, 5):
        for c in range(4):
            out = torch.empty((B, 2), dtype=torch.int64, device="cuda")
            K.kripke_census(code, offs, n, c, 2, out)
            r = K.as_u64(out)
            keys[c, n - 1], counts[c, n - 1] = r[:, 0], r[:, 1]
    torch.cuda.synchronize()
    t_small = time.time() - t0
    plan = K.kripke_plan_create(code, offs, 5, 0xF, 2, tune_cache=tune_cache)
    out = torch.empty((4, B, 2), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t1 = time.time()
    K.kripke_plan_launch(plan, out)
    torch.cuda.synchronize()
    t_five = time.time() - t1
    K.kripke_plan_destroy(plan)
    r = K.as_u64(out)
    keys[:, 4], counts[:, 4] = r[:, :, 0], r[:, :, 1]
    refuted = counts > 0
    minimal = np.where(refuted.any(axis=1), refuted.argmax(axis=1) + 1, 0)  # [4][B]
    evals = float(sum(B * CLASS_FRAMES["K"][n] * 4 ** (n + 1) for n in range(5)))
    if log:
        log(f"census of {B} formulas x 4 classes x n <= 5: {t_small + t_five:.2f} s "
            f"(n = 5 fused launch {t_five:.2f} s)")
    return {"keys": keys, "counts": counts, "minimal": minimal, "seconds": t_small + t_five,
            "five_world_seconds": t_five, "k_frame_evals": evals}


def summary(res):
    """The paper's Section 6 statistics from a census result."""
    m = res["minimal"]
    surv = m == 0
    hist = {c: {str(s): int((m[i] == s).sum()) for s in range(1, 6)} for i, c in enumerate(CLASSES)}
    for i, c in enumerate(CLASSES):
        hist[c]["none"] = int(surv[i].sum())
    sep = {"K->T": int((~surv[0] & surv[1]).sum()), "T->S4": int((~surv[1] & surv[2]).sum()),
           "S4->S5": int((~surv[2] & surv[3]).sum())}
    # one certificate (the least countermodel at the minimal size) per refuted
    # (formula, class) pair
    certificates = int((~surv).sum())
    # weakest class in which each formula survives (4 = none)
    strata = np.where(surv.any(axis=0), surv.argmax(axis=0), 4)
    names = list(CLASSES) + ["none"]
    return {"minimal_size_histogram": hist, "survivors": {c: int(surv[i].sum())
                                                          for i, c in enumerate(CLASSES)},
            "separations": sep, "certificates": certificates,
            "strata": {names[k]: int((strata == k).sum()) for k in range(5)},
            "max_refuted_minimal_size": {c: int(m[i].max()) for i, c in enumerate(CLASSES)}}


def run(log=print, tune_cache=None):
    raw, reps, corpus = build_corpus(log)
    res = census(corpus, log, tune_cache)
    out = summary(res)
    out.update({"raw_trees": len(raw), "classes": int(len(reps)), "formulas": len(corpus),
                "census_seconds": res["seconds"], "five_world_seconds": res["five_world_seconds"],
                "k_frame_evals": res["k_frame_evals"]})
    return out, res, corpus
