"""Frame-correspondence recovery (Section 10): the frame-validity maps against the
oracle, the paper's correspondence table (Table 9) recovered from them, and the
recovered conditions re-confirmed on five-world frames."""
import numpy as np
import pytest

from paper_2606_15437_amd import inputs as I

pytestmark = pytest.mark.gpu

NONE = (1 << 64) - 1


@pytest.fixture(scope="module")
def cc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_15437_amd import correspondence, kripke
    kripke.lib()
    return correspondence


def _maps(n, formulas):
    import torch
    from paper_2606_15437_amd import kripke as K
    code, offs = I.pack(formulas)
    words = ((1 << (n * n)) + 31) // 32
    d = torch.zeros((len(formulas), words), dtype=torch.int32, device="cuda")
    K.kripke_frame_validity(code, offs, n, 2, d)
    return d.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("n", [4, 5])
def test_validity_maps_match_oracle(cc, orc, n):
    """Sampled frames of every formula (plus the first frame with a countermodel, from
    the oracle's scan) agree with the oracle's census of that single frame."""
    fs = I.formula_batch(0xF3A1, 40, (2, 14), (0, 3), I.LEAVES_2, stream=n)
    fs += [a for _, a in cc.table9()] + [[I.TOP], [I.BOT], I.parse("p | ~p")]
    maps = _maps(n, fs)
    rng = np.random.default_rng(n)
    frames = rng.integers(0, 1 << (n * n), size=48, dtype=np.uint64)
    for i, f in enumerate(fs):
        # the first countermodel within the first 4,096 frames
        first, _, _ = orc.census(f, n, 0, 2, 0, 1 << 12, stop_at_first=True)
        probe = list(frames)
        if first != NONE:
            fr = first >> (2 * n + 4)
            probe += [fr, max(0, fr - 1)]
            # no frame before the first countermodel's frame is invalid
            if n == 4:
                assert all((maps[i, g >> 5] >> (g & 31)) & 1 for g in range(fr)), i
        for fr in probe:
            fr = int(fr)
            _, cnt, _ = orc.census(f, n, 0, 2, fr, fr + 1)
            assert ((maps[i, fr >> 5] >> (fr & 31)) & 1) == (cnt == 0), (i, fr)


def test_table9_correspondents(cc):
    """Every Sahlqvist axiom of Table 9 recovers its textbook condition over all frames
    with at most four worlds; McKinsey has no match in the library."""
    want = {"T": "reflexive", "D": "serial", "4": "transitive", "5": "euclidean",
            "B": "symmetric", "CD": "partially functional", "C4": "dense", "G": "directed"}
    rows = cc.table9()
    got = cc.recover([f for _, f in rows], max_n=4)
    for (name, _), rec in zip(rows, got):
        if name == "M":
            assert rec == []
        else:
            assert want[name] in rec, (name, rec)


def test_textbook_axioms_recover_their_conditions(cc):
    """The one-variable definitions of the three conditions added to Table 9's: p -> []p
    (coreflexive), []([]p -> p) (shift reflexive) and <>p <-> []p (functional), over all
    frames with at most four worlds."""
    rows = [("coreflexive", "p -> []p"), ("shift reflexive", "[]([]p -> p)"),
            ("functional", "(<>p -> []p) & ([]p -> <>p)")]
    got = cc.recover([I.parse(t) for _, t in rows], max_n=4, lib=cc.textbook_library())
    for (name, _), rec in zip(rows, got):
        assert rec == [name], (name, rec)


def test_recovered_conditions_hold_on_five_worlds(cc):
    """Re-confirmation on five-world frames (Section 10): Val_5 of each Sahlqvist axiom
    of Table 9 equals its condition's extension on every one of the 33,554,432 frames;
    McKinsey's map equals none of them."""
    rows = cc.table9()
    conds = list(cc.TABLE9_CONDITIONS)
    maps = cc.condition_maps(conds, 5)
    assert all(cc.reconfirm([f for name, f in rows if name != "M"], conds, 5, maps=maps))
    mck = [f for name, f in rows if name == "M"]
    assert not any(cc.reconfirm(mck * len(conds), conds, 5, maps=maps))


def test_corpus_summary(cc):
    """The census corpus splits into recovered, trivial and unmatched formulas; the
    trivial ones (valid on every frame or on none with at most four worlds) are the
    paper's 2,798 constant extensions."""
    raw = I.enumerate_formulas(7)
    from paper_2606_15437_amd import census_corpus
    _, reps, corpus = census_corpus.build_corpus()
    got = {}
    for name, lib in (("136", cc.library()), ("table9", cc.table9_library()),
                      ("textbook", cc.textbook_library())):
        out = cc.recover(corpus, max_n=4, lib=lib)
        trivial = sum(1 for o in out if o == "trivial")
        recovered = sum(1 for o in out if isinstance(o, list) and o)
        assert len(out) == 5624 and recovered > 0 and len(raw) == 44678
        assert trivial == 2798
        got[name] = out
    # a larger library recovers a superset: every Table-9 match keeps its condition
    for a, b in zip(got["table9"], got["textbook"]):
        if isinstance(a, list) and a:
            assert set(a) <= set(b)
