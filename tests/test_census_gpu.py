"""GPU parity: the HIP census and split paths against the CPU oracle, bit-exact.

Every comparison is on the same seeded inputs; expected values come from the
oracle (or from facts of the paper), never from the HIP path.
"""
import os

import numpy as np
import pytest

from paper_2606_15437_amd import inputs as I

pytestmark = pytest.mark.gpu

NONE = (1 << 64) - 1
CLASSES = (0, 1, 2, 3)


@pytest.fixture(scope="module")
def kr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_15437_amd import kripke
    kripke.lib()
    return kripke


def _oracle_all(orc, formulas, n, cls, nvars, f0=None, f1=None, threads=0):
    keys, cnts = [], []
    for code in formulas:
        k, c, _ = orc.census(code, n, cls, nvars, f0 or 0, f1, threads=threads)
        keys.append(k)
        cnts.append(c)
    return np.array(keys, dtype=np.uint64), np.array(cnts, dtype=np.uint64)


# ------------------------------------------------------------- config 1
@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("cls", CLASSES)
def test_config1_full_parity(kr, orc, n, cls):
    fs = I.config1_formulas()
    keys, cnts = kr.census(fs, n, cls, 2)
    ek, ec = _oracle_all(orc, fs, n, cls, 2, threads=4)
    assert (keys == ek).all() and (cnts == ec).all()


# ------------------------------------------------------------- config 2
@pytest.mark.parametrize("cls", [2, 3])
def test_config2_small_classes_full(kr, orc, cls):
    fs = I.config2_formulas()[:64]
    keys, cnts = kr.census(fs, 4, cls, 3)
    ek, ec = _oracle_all(orc, fs, 4, cls, 3)
    assert (keys == ek).all() and (cnts == ec).all()


def _check_first_keys(orc, fs, keys, n, cls, nvars, prefix):
    """The oracle scans frames [0, prefix) in key order and stops at its first countermodel.
    If it finds one the GPU key must equal it; otherwise the GPU key must lie beyond the
    prefix and decode to a certificate the oracle's pointwise checker accepts."""
    for code, k in zip(fs, keys):
        k = int(k)
        ek, _, _ = orc.census(code, n, cls, nvars, 0, prefix, stop_at_first=True, threads=0)
        if ek != NONE:
            assert k == ek, I.to_text(code)
        elif k != NONE:
            f, val, w = orc.decode_key(k, n, nvars)
            assert f >= prefix
            assert orc.check_certificate(code, I.frame_succ(f, n), nvars, val, w, cls)


@pytest.mark.parametrize("cls", [0, 1])
def test_config2_first_keys(kr, orc, cls):
    """First countermodel keys of the 64-formula subset over the whole n=4 layer."""
    fs = I.config2_formulas()[:64]
    keys, _ = kr.census(fs, 4, cls, 3)
    _check_first_keys(orc, fs, keys, 4, cls, 3, 1 << 12)
    # two formulas the GPU reports valid are re-scanned over the whole layer
    valid = [f for f, k in zip(fs, keys) if int(k) == NONE][:2]
    for code in valid:
        assert orc.census(code, 4, cls, 3, stop_at_first=True, threads=0)[0] == NONE


@pytest.mark.parametrize("cls", [0, 1])
def test_config2_count_slices(kr, orc, cls):
    """Exact counts on seeded frame slices (ragged sizes, several tiles)."""
    fs = I.config2_formulas()[:64]
    rng = I.SplitMix64(0x5EED, cls)
    for _ in range(3):
        f0 = rng.below(65536 - 700)
        f1 = f0 + 129 + rng.below(500)
        keys, cnts = kr.census(fs, 4, cls, 3, frame_begin=f0, frame_end=f1)
        ek, ec = _oracle_all(orc, fs, 4, cls, 3, f0, f1)
        assert (keys == ek).all() and (cnts == ec).all(), (f0, f1)


# ------------------------------------------------------------- config 3
def test_config3_sampled(kr, orc):
    """n = 5, 2 vars, the full 4,096-formula batch in one launch.  For 64 sampled formulas:
    the oracle scans frames [0, 2^15) in key order and stops at its first countermodel; if it
    finds one, the GPU key must equal it, otherwise the GPU key must lie beyond that prefix
    and be a certificate the oracle's pointwise checker accepts.  Counts are exact on a
    seeded frame slice, for class K and T."""
    fs = I.config3_formulas()
    keys, _ = kr.census(fs, 5, 0, 2)
    rng = I.SplitMix64(0xC3, 0)
    idx = sorted(set(rng.below(len(fs)) for _ in range(64)))
    _check_first_keys(orc, [fs[i] for i in idx], keys[idx], 5, 0, 2, 1 << 15)
    sub = [fs[i] for i in idx]
    for cls, f0 in ((0, 1 << 20), (1, (1 << 24) | (1 << 18) | (1 << 12) | 777)):
        k2, c2 = kr.census(sub, 5, cls, 2, frame_begin=f0, frame_end=f0 + 300)
        ek, ec = _oracle_all(orc, sub, 5, cls, 2, f0, f0 + 300)
        assert (k2 == ek).all() and (c2 == ec).all(), cls


def test_config3_valid_verdicts_checked_small(kr, orc):
    """Formulas the GPU reports valid on every 5-world frame are valid at n <= 3 too."""
    fs = I.config3_formulas()[:512]
    keys, _ = kr.census(fs, 5, 0, 2)
    valid = [f for f, k in zip(fs, keys) if int(k) == NONE]
    for code in valid[:40]:
        for n in (1, 2, 3):
            assert orc.census(code, n, 0, 2, threads=4)[0] == NONE


@pytest.mark.parametrize("cls", [2, 3])
def test_config3_small_classes(kr, orc, cls):
    fs = I.config3_formulas()[:32]
    keys, cnts = kr.census(fs, 5, cls, 2)
    ek, ec = _oracle_all(orc, fs, 5, cls, 2, threads=0)
    assert (keys == ek).all() and (cnts == ec).all()


# ---------------------------------------------------------- paper facts
def test_named_axioms_n5(kr):
    ax = [I.parse(t) for t in ("[](p -> q) -> ([]p -> []q)", I.TABLE1_FORMULA, "[]p -> p",
                               "[]p -> [][]p", "<>p -> []<>p")]
    res = {c: kr.census(ax, 5, c, 2) for c in CLASSES}
    for c in CLASSES:
        assert int(res[c][0][0]) == NONE and int(res[c][0][1]) == NONE  # K axiom, Table 1
    assert int(res[0][0][2]) != NONE and all(int(res[c][0][2]) == NONE for c in (1, 2, 3))
    assert int(res[0][0][3]) != NONE and int(res[1][0][3]) != NONE
    assert int(res[2][0][3]) == NONE and int(res[3][0][3]) == NONE
    assert int(res[2][0][4]) != NONE and int(res[3][0][4]) == NONE


def test_prop6_alpha_agree_through_5(kr):
    chi = I.iff(I.alpha(2), I.alpha(3))
    for n in range(1, 6):
        keys, cnts = kr.census([chi], n, 0, 0)
        assert int(keys[0]) == NONE and int(cnts[0]) == 0
    f = I.frame_index(I.path_frame(6))
    keys, _ = kr.census([chi], 6, 0, 0, frame_begin=f, frame_end=f + 1)
    assert int(keys[0]) == (f << 4) | 0


# ------------------------------------------------------------ edge cases
def test_constants_and_empty_ranges(kr):
    fs = [[I.TOP], [I.BOT], I.parse("p | ~p"), I.parse("p & ~p"), I.parse("<>T"), I.parse("[]F")]
    keys, cnts = kr.census(fs, 3, 0, 2)
    assert int(keys[0]) == NONE and int(cnts[0]) == 0
    assert int(keys[1]) == 0 and int(cnts[1]) == 512 * 64
    assert int(keys[2]) == NONE and int(keys[3]) == 0 and int(cnts[3]) == 512 * 64
    # <>T fails exactly on frames with a dead end; []F fails on frames with a successor
    assert int(keys[4]) == 0 and int(keys[5]) == (1 << (6 + 4)) | 0
    keys, cnts = kr.census(fs, 3, 0, 2, frame_begin=100, frame_end=100)
    assert (keys == NONE).all() and (cnts == 0).all()


def test_single_frame_ranges(kr, orc):
    fs = I.config1_formulas()[:16]
    for f in (0, 1, 255, 511):
        keys, cnts = kr.census(fs, 3, 0, 2, frame_begin=f, frame_end=f + 1)
        ek, ec = _oracle_all(orc, fs, 3, 0, 2, f, f + 1)
        assert (keys == ek).all() and (cnts == ec).all()


def test_decide_mode_keys(kr, orc):
    fs = I.config2_formulas()[64:96]
    keys, _ = kr.census(fs, 4, 0, 3, decide=True)
    for code, k in zip(fs, keys):
        assert int(k) == orc.census(code, 4, 0, 3, stop_at_first=True)[0]


def test_error_codes(kr):
    import torch
    out = torch.empty((1, 2), dtype=torch.int64, device="cuda")
    bad = [([99], -2), ([I.AND], -2), ([I.var(2)], -2), ([I.TOP, I.TOP], -2)]
    for code, status in bad:
        c, o = I.pack([code])
        with pytest.raises(kr.KripkeError) as e:
            kr.kripke_census(c, o, 3, 0, 2, out)
        assert e.value.status == status
    c, o = I.pack([[I.TOP]])
    for n, cls, nv in ((0, 0, 2), (7, 0, 2), (3, 9, 2), (3, 0, 5)):
        with pytest.raises(kr.KripkeError):
            kr.kripke_census(c, o, n, cls, nv, out)
    with pytest.raises(kr.KripkeError):
        kr.kripke_census(c, o, 6, 0, 2, out)  # n = 6 needs the range entry point
    with pytest.raises(kr.KripkeError):
        kr.kripke_census(c, o, 3, 0, 2, None)


def test_key_and_frame_codecs(kr):
    key = (541098242 << 4) | 0
    assert kr.kripke_key_decode(key, 6, 0) == (541098242, 0, 0)
    assert kr.kripke_frame_decode(541098242, 6) == I.path_frame(6)
    k = (12345 << (10 + 4)) | (777 << 4) | 3
    assert kr.kripke_key_decode(k, 5, 2) == (12345, 777, 3)


# ------------------------------------------------------------- plans
def test_plan_graph_replay_matches_census(kr):
    import torch
    fs = I.config1_formulas()
    code, offs = I.pack(fs)
    out = torch.zeros((4, len(fs), 2), dtype=torch.int64, device="cuda")
    plan = kr.kripke_plan_create(code, offs, 3, 0xF, 2)
    try:
        ref = {c: kr.census(fs, 3, c, 2) for c in CLASSES}
        for rep in range(4):
            out.fill_(7)
            kr.kripke_plan_launch(plan, out)
            torch.cuda.synchronize()
            r = kr.as_u64(out)
            junk = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work
            assert junk == 1000.0
            for c in CLASSES:
                assert (r[c, :, 0] == ref[c][0]).all() and (r[c, :, 1] == ref[c][1]).all(), rep
    finally:
        kr.kripke_plan_destroy(plan)


@pytest.mark.parametrize("n,nvars,getter,count", [(4, 3, "config2_formulas", 64),
                                                  (5, 2, "config3_formulas", 48)])
def test_fused_plan_matches_single_class(kr, n, nvars, getter, count):
    """The one-launch all-class plan (every K frame reduced into each class containing it)
    equals four single-class censuses, over several graph replays."""
    import torch
    fs = getattr(I, getter)()[:count]
    code, offs = I.pack(fs)
    out = torch.zeros((4, len(fs), 2), dtype=torch.int64, device="cuda")
    plan = kr.kripke_plan_create(code, offs, n, 0xF, nvars)
    try:
        ref = {c: kr.census(fs, n, c, nvars) for c in CLASSES}
        for rep in range(3):
            out.fill_(-1)
            kr.kripke_plan_launch(plan, out)
            torch.cuda.synchronize()
            r = kr.as_u64(out)
            for c in CLASSES:
                assert (r[c, :, 0] == ref[c][0]).all() and (r[c, :, 1] == ref[c][1]).all(), (rep, c)
    finally:
        kr.kripke_plan_destroy(plan)


def test_bench_plan_full_batch_sampled(kr, orc):
    """The measured configuration itself: the whole 4,096-formula n = 5 batch in one fused
    plan with the committed tile choices (as the benchmark runs it).  Sampled formulas are
    checked against the oracle in every class: first K keys on a key-order prefix, T keys
    as reflexive countermodels, exact keys and counts over the whole S4 and S5 layers;
    every sixteenth K key is a certificate;
    and K/T counts equal the single-class kernels' for the whole batch."""
    import os
    import torch
    fs = I.config3_formulas()
    code, offs = I.pack(fs)
    cache = os.path.join(os.path.dirname(kr.__file__), "tune_cache.json")
    plan = kr.kripke_plan_create(code, offs, 5, 0xF, 2, tune_cache=cache)
    out = torch.zeros((4, len(fs), 2), dtype=torch.int64, device="cuda")
    try:
        kr.kripke_plan_launch(plan, out)
        torch.cuda.synchronize()
        r = kr.as_u64(out)
    finally:
        kr.kripke_plan_destroy(plan)
    rng = I.SplitMix64(0xBE4C, 0)
    idx = sorted(set(rng.below(len(fs)) for _ in range(40)))
    sub = [fs[i] for i in idx]
    _check_first_keys(orc, sub, r[0, idx, 0], 5, 0, 2, 1 << 14)
    for code, k in zip(sub, r[1, idx, 0]):  # T keys are reflexive countermodels
        if int(k) != NONE:
            f, val, w = orc.decode_key(int(k), 5, 2)
            assert orc.check_certificate(code, I.frame_succ(f, 5), 2, val, w, 1)
    for c in (2, 3):
        ek, ec = _oracle_all(orc, sub, 5, c, 2, threads=0)
        assert (r[c, idx, 0] == ek).all() and (r[c, idx, 1] == ec).all(), c
    for c in (0, 1):
        k, n = kr.census(fs, 5, c, 2)
        assert (r[c, :, 0] == k).all() and (r[c, :, 1] == n).all(), c
    for i, code in enumerate(fs):
        k = int(r[0, i, 0])
        if k != NONE and i % 16 == 0:
            f, val, w = orc.decode_key(k, 5, 2)
            assert orc.check_certificate(code, I.frame_succ(f, 5), 2, val, w, 0)


def test_fused_plan_small_classes_vs_oracle(kr, orc):
    """Fused-plan S4 and S5 rows at n = 5 against the oracle directly."""
    import torch
    fs = I.config3_formulas()[100:116]
    code, offs = I.pack(fs)
    out = torch.zeros((4, len(fs), 2), dtype=torch.int64, device="cuda")
    plan = kr.kripke_plan_create(code, offs, 5, 0xF, 2)
    try:
        kr.kripke_plan_launch(plan, out)
        torch.cuda.synchronize()
        r = kr.as_u64(out)
    finally:
        kr.kripke_plan_destroy(plan)
    for c in (2, 3):
        ek, ec = _oracle_all(orc, fs, 5, c, 2)
        assert (r[c, :, 0] == ek).all() and (r[c, :, 1] == ec).all(), c


def _deep_formulas():
    """Programs whose compiled form needs 3 stack slots (balanced trees of modal literals),
    so a batch holding them runs as two tiers of kernel variants."""
    u = ["<>p", "[]q", "<>~q", "[]~p", "<>(p & q)", "[](p | ~q)", "<>[]p", "[]<>q"]
    pairs = [f"({u[i]} & {u[i + 1]})" for i in range(0, 8, 2)]
    quads = [f"({pairs[0]} | {pairs[1]})", f"({pairs[2]} | {pairs[3]})"]
    return [I.parse(f"{quads[0]} <-> {quads[1]}"), I.parse(f"{quads[0]} & {quads[1]}"),
            I.parse(f"~({quads[1]} -> {quads[0]})")]


def test_tiered_batch_against_oracle(kr, orc):
    from paper_2606_15437_amd.inputs import pack
    fs = I.config3_formulas()[:40] + _deep_formulas()
    st = kr.kripke_program_stats(*pack(fs), 2)
    assert st[:, 4].max() >= 3  # the batch really needs a second tier
    f0 = (1 << 22) + 12345
    keys, cnts = kr.census(fs, 5, 0, 2, frame_begin=f0, frame_end=f0 + 200)
    ek, ec = _oracle_all(orc, fs, 5, 0, 2, f0, f0 + 200)
    assert (keys == ek).all() and (cnts == ec).all()
    f0 = (1 << 24) | (1 << 18) | (1 << 12) | 64
    keys, cnts = kr.census(fs, 5, 1, 2, frame_begin=f0, frame_end=f0 + 300)
    ek, ec = _oracle_all(orc, fs, 5, 1, 2, f0, f0 + 300)
    assert (keys == ek).all() and (cnts == ec).all()


def test_tiered_fused_plan(kr):
    import torch
    fs = I.config3_formulas()[200:260] + _deep_formulas()
    code, offs = I.pack(fs)
    out = torch.zeros((4, len(fs), 2), dtype=torch.int64, device="cuda")
    plan = kr.kripke_plan_create(code, offs, 5, 0xF, 2)
    try:
        kr.kripke_plan_launch(plan, out)
        torch.cuda.synchronize()
        r = kr.as_u64(out)
    finally:
        kr.kripke_plan_destroy(plan)
    for c in CLASSES:
        k, n = kr.census(fs, 5, c, 2)
        assert (r[c, :, 0] == k).all() and (r[c, :, 1] == n).all(), c


# ------------------------------------------------------------- split
def _split_pairs(n, count=64):
    """Random pairs (mostly split at once), designed late-splitting pairs, pairs that are
    equivalent on every model (full scans, never split) and deep pairs (second tier)."""
    fs = I.formula_batch(0x5B117, count, (3, 12), (0, 4), I.LEAVES_2, stream=n)
    pairs = list(zip(fs[0::2], fs[1::2]))
    pairs += [(I.alpha(1), I.alpha(2)), (I.alpha(2), I.alpha(3)), (I.alpha(3), I.alpha(4)),
              (I.dia_k_top(4), I.dia_k_top(5)), (I.box_k_bot(5), I.box_k_bot(6))]
    pairs += [(f, I.equivalent_variant(f, k)) for k, f in enumerate(fs[:12])]
    deep = _deep_formulas()
    pairs += [(deep[0], deep[1]), (deep[2], I.equivalent_variant(deep[2], 1)),
              (deep[1], I.equivalent_variant(deep[1], 3))]
    return pairs


def _par(fn, items):
    """Map over host threads (the oracle's C calls release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(fn, items))


@pytest.mark.parametrize("n", [6, 7, 8])
def test_split_parity_families(kr, orc, n):
    frames = I.frame_family(n, {6: 600, 7: 600, 8: 120}[n])
    pairs = _split_pairs(n)
    keys = kr.split(pairs, frames, n, 2)
    exp = _par(lambda ab: orc.split(ab[0], ab[1], frames, 2), pairs)
    for (a, b), k, e in zip(pairs, keys, exp):
        assert int(k) == e, (I.to_text(a), I.to_text(b))


@pytest.mark.parametrize("n", [6, 7, 8])
def test_split_list_kernel_matches_generic(kr, n, monkeypatch):
    """The wave-uniform list kernel (default for two variables at n >= 6) and the
    per-lane-frame kernel give identical keys on a larger panel, ragged in length."""
    frames = I.frame_family(n, 3001, start=500)
    pairs = _split_pairs(n, 160)
    fast = kr.split(pairs, frames, n, 2)
    monkeypatch.setenv("KRIPKE_SPLIT_GENERIC", "1")
    slow = kr.split(pairs, frames, n, 2)
    assert (fast == slow).all()
    assert (fast == NONE).sum() >= 15 and (fast != NONE).sum() >= 60


def test_split_designed_pins(kr):
    """alpha_2/alpha_3 split first on the canonical path at its root (Proposition 6, Lemma 2);
    alpha_3/alpha_4 have separation size 8 (Table 4), so no 6- or 7-world frame splits them,
    while the 8-world path does at its root."""
    for n in (6, 7):
        frames = I.frame_family(n, 256)
        keys = kr.split([(I.alpha(2), I.alpha(3))], frames, n, 0)
        # position 0 is the canonical path; by Lemma 2 the two differ where r = 5 edges
        # remain, i.e. at world n - 6
        assert int(keys[0]) == n - 6
        keys = kr.split([(I.alpha(3), I.alpha(4))], frames, n, 0)
        assert int(keys[0]) == NONE
    keys = kr.split([(I.alpha(3), I.alpha(4))], [I.path_frame(8)], 8, 0)
    assert int(keys[0]) == 0


def test_split_symmetric_and_empty(kr):
    frames = I.frame_family(6, 100)
    fs = I.config1_formulas()[:20]
    pairs = list(zip(fs[:10], fs[10:]))
    a = kr.split(pairs, frames, 6, 2)
    b = kr.split([(y, x) for x, y in pairs], frames, 6, 2)
    assert (a == b).all()
    same = kr.split([(fs[0], fs[0])], frames, 6, 2)
    assert int(same[0]) == NONE


# ------------------------------------------------------ literal pairs
def _literal_pair_formulas():
    """Every AND / OR of two literals over p, q (either one negated), alone, under BOX
    and DIA, and as the operand of a further connective."""
    lits = [[I.VAR0], [I.var(1)], [I.VAR0, I.NOT], [I.var(1), I.NOT]]
    out = []
    for a in lits:
        for b in lits:
            for op in (I.AND, I.OR):
                f = a + b + [op]
                out += [f, f + [I.BOX], f + [I.DIA], [I.var(1), I.DIA] + f + [I.AND]]
    return out


@pytest.mark.parametrize("n,cls", [(3, 0), (4, 0), (4, 1), (4, 2)])
def test_literal_pairs(kr, orc, n, cls):
    fs = _literal_pair_formulas()
    keys, cnts = kr.census(fs, n, cls, 2)
    ek, ec = _oracle_all(orc, fs, n, cls, 2, threads=4)
    bad = [I.to_text(f) for f, k, c, a, b in zip(fs, keys, cnts, ek, ec) if k != a or c != b]
    assert not bad, bad


def test_literal_pairs_split(kr, orc):
    fs = _literal_pair_formulas()
    pairs = list(zip(fs[0::2], fs[1::2])) + list(zip(fs[1::2], fs[2::2]))
    frames = I.frame_family(6, 300)
    keys = kr.split(pairs, frames, 6, 2)
    exp = _par(lambda ab: orc.split(ab[0], ab[1], frames, 2), pairs)
    bad = [(I.to_text(a), I.to_text(b)) for (a, b), k, e in zip(pairs, keys, exp) if int(k) != e]
    assert not bad, bad
