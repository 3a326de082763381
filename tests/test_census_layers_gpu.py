"""GPU parity over whole layers and on every reachable kernel family.

- T-class least countermodels compared with the oracle's least key over the whole
  reflexive layer (Section 2 classes, Algorithm 1's FIRST under the lexicographic
  reading), at n = 4 with three variables and on the benchmarked n = 5 plan;
- every formula the n = 5 census reports valid in K (and that does not fold to a
  constant) re-checked by the oracle on every frame with at most four worlds
  (a formula valid on all 5-world frames is valid on all smaller ones: an isolated
  extra world preserves every countermodel);
- exact counts and keys on ragged frame slices for the n = 5 / three-variable and
  n = 6 / two-variable kernel families, classes K and T, through both tiers.

Expected values come from the oracle or from facts of the paper, never from the
HIP path.
"""
import os

import numpy as np
import pytest

from paper_2606_15437_amd import inputs as I

pytestmark = pytest.mark.gpu

NONE = (1 << 64) - 1
K, T = 0, 1


@pytest.fixture(scope="module")
def kr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_15437_amd import kripke
    kripke.lib()
    return kripke


def _par(fn, items, workers=4):
    """Map over host threads; each oracle call already spreads its frames over the cores."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))


@pytest.fixture(scope="module")
def bench_plan_results(kr):
    """The benchmarked configuration: the 4,096-formula n = 5 batch in one fused plan with
    the committed tile choices; returns uint64 [4][B][2]."""
    import torch
    fs = I.config3_formulas()
    code, offs = I.pack(fs)
    cache = os.path.join(os.path.dirname(kr.__file__), "tune_cache.json")
    plan = kr.kripke_plan_create(code, offs, 5, 0xF, 2, tune_cache=cache)
    out = torch.zeros((4, len(fs), 2), dtype=torch.int64, device="cuda")
    try:
        kr.kripke_plan_launch(plan, out)
        torch.cuda.synchronize()
        r = kr.as_u64(out).copy()
    finally:
        kr.kripke_plan_destroy(plan)
    return fs, r


def test_t_keys_whole_layer_n4_three_vars(kr, orc):
    """All 64 parity formulas of the n = 4 / three-variable configuration in class T: the
    GPU key equals the oracle's least key over the whole reflexive layer (the oracle
    scans every frame index in order, skipping non-reflexive frames, and stops at its
    first countermodel or scans the whole layer)."""
    fs = I.config2_formulas()[:64]
    keys, _ = kr.census(fs, 4, T, 3)
    exp = _par(lambda f: orc.census(f, 4, T, 3, stop_at_first=True, threads=0)[0], fs)
    bad = [(I.to_text(f), int(k), e) for f, k, e in zip(fs, keys, exp) if int(k) != e]
    assert not bad, bad
    assert sum(e != NONE for e in exp) >= 32 and sum(e == NONE for e in exp) >= 1


def test_t_keys_whole_layer_n5_bench_plan(kr, orc, bench_plan_results):
    """The fused plan's T row at n = 5: 48 seeded formulas refuted in T have exactly the
    oracle's least key over the whole reflexive layer (the first reflexive frame is index
    17,043,521, so no prefix scan can stand in for this); two live formulas the plan
    reports T-valid are scanned by the oracle over the whole layer."""
    fs, r = bench_plan_results
    st = kr.kripke_program_stats(*I.pack(fs), 2)
    refuted = [i for i in range(len(fs)) if int(r[1, i, 0]) != NONE]
    rng = I.SplitMix64(0x7E5, 0)
    idx = sorted(set(refuted[rng.below(len(refuted))] for _ in range(60)))[:48]
    assert len(idx) >= 40
    exp = _par(lambda i: orc.census(fs[i], 5, T, 2, stop_at_first=True, threads=0)[0], idx)
    bad = [(i, int(r[1, i, 0]), e) for i, e in zip(idx, exp) if int(r[1, i, 0]) != e]
    assert not bad, bad
    live_valid = [i for i in range(len(fs)) if int(r[1, i, 0]) == NONE and st[i, 5] == -1]
    assert live_valid
    for i in live_valid[:2]:
        key, cnt, _ = orc.census(fs[i], 5, T, 2, threads=0)
        assert key == NONE and cnt == 0, I.to_text(fs[i])


def test_k_valid_verdicts_through_four_worlds(kr, orc, bench_plan_results):
    """Every formula the n = 5 census reports valid in K and that does not fold to a
    constant has no countermodel on any frame with at most four worlds (oracle, every
    frame and valuation of each layer)."""
    fs, r = bench_plan_results
    st = kr.kripke_program_stats(*I.pack(fs), 2)
    live_valid = [i for i in range(len(fs)) if int(r[0, i, 0]) == NONE and st[i, 5] == -1]
    assert len(live_valid) >= 100

    def check(i):
        return [orc.census(fs[i], n, K, 2, stop_at_first=True, threads=0)[0] for n in (1, 2, 3, 4)]

    res = _par(check, live_valid)
    bad = [(I.to_text(fs[i]), ks) for i, ks in zip(live_valid, res) if any(k != NONE for k in ks)]
    assert not bad, bad


def _deep_formulas(leaves):
    """Balanced trees of modal literals needing three stack slots (second tier)."""
    p, q = leaves
    u = [f"<>{p}", f"[]{q}", f"<>~{q}", f"[]~{p}", f"<>({p} & {q})", f"[]({p} | ~{q})",
         f"<>[]{p}", f"[]<>{q}"]
    pairs = [f"({u[i]} & {u[i + 1]})" for i in range(0, 8, 2)]
    quads = [f"({pairs[0]} | {pairs[1]})", f"({pairs[2]} | {pairs[3]})"]
    return [I.parse(f"{quads[0]} <-> {quads[1]}"), I.parse(f"~({quads[1]} -> {quads[0]})")]


def _refl_mask(n):
    return sum(1 << (w * n + w) for w in range(n))


@pytest.mark.parametrize("n,nvars,cls", [(5, 3, K), (5, 3, T), (6, 2, K), (6, 2, T)])
def test_range_variant_families(kr, orc, n, nvars, cls):
    """census_range over ragged slices on the kernel families that no full-layer test
    reaches: n = 5 with three variables (four valuation-chunk bits per lane) and n = 6
    with two variables (36-bit relations).  T slices start at a reflexive frame, so
    they hold reflexive frames among non-reflexive ones.  Exact keys and counts."""
    if nvars == 3:
        fs = I.config2_formulas()[100:124] + _deep_formulas(("r", "q"))
    else:
        fs = I.config3_formulas()[300:324] + _deep_formulas(("p", "q"))
    st = kr.kripke_program_stats(*I.pack(fs), nvars)
    assert st[:, 4].max() >= 3  # the batch needs a second tier
    rng = I.SplitMix64(0x5A1CE, 16 * n + 4 * nvars + cls)
    span = 193 if (n, nvars) == (5, 3) else 449
    for rep in range(2):
        if cls == K:
            f0 = rng.below((1 << (n * n)) - span)
        else:
            f0 = _refl_mask(n) | (rng.below(1 << (n * n - 2 * n)) << (2 * n))
            f0 |= _refl_mask(n)
        f0 = min(f0, (1 << (n * n)) - span - 40)
        f1 = f0 + span + rep * 37
        keys, cnts = kr.census(fs, n, cls, nvars, frame_begin=f0, frame_end=f1)
        exp = _par(lambda f: orc.census(f, n, cls, nvars, f0, f1, threads=0)[:2], fs)
        ek = np.array([e[0] for e in exp], dtype=np.uint64)
        ec = np.array([e[1] for e in exp], dtype=np.uint64)
        assert (keys == ek).all() and (cnts == ec).all(), (f0, f1)
        if cls == T:
            assert any(orc.in_class(I.frame_succ(f, n), T) for f in range(f0, f1))
