"""The autotuner's search path (Section 4's fused scan, tiles chosen per device and
batch): a fresh cache runs every tile candidate, checks that all of them give
identical results, and stores the winner; every stored candidate then reproduces
the single-class censuses exactly, and so does the per-formula form of the fused
kernel (one launch per formula, its own tuned tiles)."""
import json
import os

import numpy as np
import pytest

from paper_2606_15437_amd import inputs as I

pytestmark = pytest.mark.gpu

CLASSES = (0, 1, 2, 3)


@pytest.fixture(scope="module")
def kr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_15437_amd import kripke
    kripke.lib()
    return kripke


def _batch():
    deep = ["(((<>p & []q) | (<>~q & []~p)) <-> ((<>(p & q) & [](p | ~q)) | (<>[]p & []<>q)))"]
    return I.config3_formulas()[:56] + [I.parse(t) for t in deep]


def _launch(kr, plan, B):
    import torch
    out = torch.full((4, B, 2), -1, dtype=torch.int64, device="cuda")
    kr.kripke_plan_launch(plan, out)
    torch.cuda.synchronize()
    return kr.as_u64(out).copy()


def _reference(kr, fs):
    return {c: kr.census(fs, 5, c, 2) for c in CLASSES}


def _matches(r, ref):
    return all((r[c, :, 0] == ref[c][0]).all() and (r[c, :, 1] == ref[c][1]).all()
               for c in CLASSES)


@pytest.mark.parametrize("per_formula", [False, True])
def test_tuner_search_and_every_candidate(kr, tmp_path, monkeypatch, per_formula):
    monkeypatch.delenv("KRIPKE_SETS_LOG2", raising=False)
    fs = _batch()
    code, offs = I.pack(fs)
    ref = _reference(kr, fs)
    cache = str(tmp_path / "tune.json")
    mask = 0xF | (kr.KRIPKE_PLAN_PLAIN if per_formula else 0)
    plan = kr.kripke_plan_create(code, offs, 5, mask, 2, tune_cache=cache)
    try:
        assert _matches(_launch(kr, plan, len(fs)), ref)
    finally:
        kr.kripke_plan_destroy(plan)
    entries = json.load(open(cache))
    assert len(entries) == 1
    key, entry = next(iter(entries.items()))
    assert key.endswith("/per-formula") == per_formula
    assert entry["ls"] in (0, 1, 2, 3) and entry["ipw"] in (4, 16, 64) and entry["slice_ms"] > 0
    # every candidate, forced through the cache, reproduces the single-class results
    for ls in (0, 1, 2, 3):
        for ipw in (4, 16, 64):
            json.dump({key: {"ls": ls, "ipw": ipw, "slice_ms": 1.0}}, open(cache, "w"))
            plan = kr.kripke_plan_create(code, offs, 5, mask, 2, tune_cache=cache)
            try:
                assert _matches(_launch(kr, plan, len(fs)), ref), (ls, ipw)
            finally:
                kr.kripke_plan_destroy(plan)


def test_plain_baseline_matches(kr):
    """The untuned per-class, per-formula baseline gives the batched plan's results."""
    fs = _batch()[:24]
    code, offs = I.pack(fs)
    ref = _reference(kr, fs)
    plan = kr.kripke_plan_create(code, offs, 5, 0xF | kr.KRIPKE_PLAN_PLAIN, 2)
    try:
        assert _matches(_launch(kr, plan, len(fs)), ref)
    finally:
        kr.kripke_plan_destroy(plan)


def test_per_formula_tuner_on_a_subset_of_a_large_batch(kr, tmp_path, monkeypatch):
    """A per-formula plan over more than 256 formulas is tuned on the batch's first 256;
    the candidates' tiers (which formulas a variant's stack holds) differ, yet every
    candidate times the same formulas and must agree, and the tuned plan reproduces the
    single-class censuses on the whole batch."""
    monkeypatch.delenv("KRIPKE_SETS_LOG2", raising=False)
    deep = [I.parse("(((<>p & []q) | (<>~q & []~p)) <-> ((<>(p & q) & [](p | ~q)) | "
                    "(<>[]p & []<>q)))")] * 4
    fs = I.config3_formulas()[:300] + deep
    code, offs = I.pack(fs)
    slots = kr.kripke_program_stats(code, offs, 2)[:, 4]
    assert slots.max() >= 2  # the deep programs need a second stack slot: tiers differ
    ref = _reference(kr, fs)
    cache = str(tmp_path / "tune.json")
    plan = kr.kripke_plan_create(code, offs, 5, 0xF | kr.KRIPKE_PLAN_PLAIN, 2, tune_cache=cache)
    try:
        assert _matches(_launch(kr, plan, len(fs)), ref)
    finally:
        kr.kripke_plan_destroy(plan)
    key = next(iter(json.load(open(cache))))
    assert key.endswith("/per-formula") and "/B304/" in key
