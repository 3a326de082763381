"""Split search with two list frames per block (six-world lists, two variables: each
half-wave holds one frame, four valuation sets per lane): keys against the oracle and
against the one-frame-per-block kernels, on odd and tiny frame counts (a ragged last
block), with deep programs that fall back to one-frame blocks (Definition 2,
Proposition 5)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2606_15437_amd import inputs as I

pytestmark = pytest.mark.gpu

DEEP = "(((<>p & []q) | (<>~q & []~p)) <-> ((<>(p & q) & [](p | ~q)) | (<>[]p & []<>q)))"


@pytest.fixture(scope="module")
def kr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_15437_amd import kripke
    kripke.lib()
    return kripke


def _pairs():
    pool = I.config4_pool(400)
    pairs = [(pool[i], pool[i + 1]) for i in range(0, 400, 2)]
    deep = I.parse(DEEP)
    # deep programs: their biconditionals need three stack slots, more than the
    # two-frame variant holds, so they run in the one-frame tier of the same launch
    pairs += [(deep, deep), (deep, I.parse("[]p -> <>q")), (I.alpha(2), deep)]
    pairs += I.config4_designed_pairs()[:6] + [(I.alpha(2), I.alpha(3))]
    return pairs


def test_deep_pairs_need_the_fallback_tier(kr):
    deep = I.parse(DEEP)
    st = kr.kripke_program_stats(*I.pack([I.iff(deep, deep)]), 2)
    assert st[0, 4] >= 3


@pytest.mark.parametrize("nframes", [1, 2, 3, 999, 4096])
def test_two_frame_blocks_match_one_frame_blocks(kr, monkeypatch, nframes):
    pairs = _pairs()
    frames = I.frame_family(6, nframes)
    two = kr.split(pairs, frames, 6)
    monkeypatch.setenv("KRIPKE_SPLIT_ONE_FRAME", "1")
    one = kr.split(pairs, frames, 6)
    assert np.array_equal(two, one), nframes


@pytest.mark.parametrize("nframes", [1, 999])
def test_two_frame_blocks_match_the_oracle(kr, nframes):
    from oracle import oracle as orc
    pairs = _pairs()
    frames = I.frame_family(6, nframes)
    got = kr.split(pairs, frames, 6)
    # the oracle's full scans cost about a second per unseparated pair on 999 frames:
    # every separated pair, then a sample of the rest
    sep = [i for i in range(len(pairs)) if got[i] != kr.NO_KEY]
    rest = [i for i in range(len(pairs)) if got[i] == kr.NO_KEY][:24]
    check = sep + rest + list(range(len(pairs) - 10, len(pairs)))
    with ThreadPoolExecutor(max_workers=16) as ex:
        want = list(ex.map(lambda i: orc.split(pairs[i][0], pairs[i][1], frames, 2), check))
    for i, w in zip(check, want):
        assert int(got[i]) == w, (i, I.to_text(pairs[i][0]), I.to_text(pairs[i][1]))
    assert len(sep) >= 5  # the sample holds separated pairs, not only agreeing ones


@pytest.mark.parametrize("nframes", [3, 999, 4096])
def test_formula_groups_match_single_formulas(kr, monkeypatch, nframes):
    """A work item of the two-frame kernel scans a group of formulas on each decoded
    block; every group size gives the keys of one formula per item, with groups cut
    short at the end of the batch and constant programs (TOP never fails, BOT fails
    at the first model) inside groups."""
    p = I.parse("p")
    pairs = _pairs() + [([I.TOP], [I.BOT]), (p, p), ([I.BOT], [I.BOT]), (p, [I.TOP]),
                        ([I.TOP], [I.TOP])]
    frames = I.frame_family(6, nframes)
    monkeypatch.setenv("KRIPKE_LIST_GROUP", "1")
    single = kr.split(pairs, frames, 6)
    assert single[len(pairs) - 5] == 0  # TOP <-> BOT fails at the first model
    assert single[len(pairs) - 1] == kr.NO_KEY
    for g in ("2", "3", "4"):
        monkeypatch.setenv("KRIPKE_LIST_GROUP", g)
        assert np.array_equal(kr.split(pairs, frames, 6), single), (g, nframes)


@pytest.mark.parametrize("n,nframes", [(7, 777), (8, 777), (7, 1), (8, 2)])
def test_one_frame_list_groups_match_single_formulas(kr, monkeypatch, n, nframes):
    """The one-frame list kernels (seven and eight worlds) also scan groups of pairs per
    work item, each pair running its valuation chunks in order on the decoded frame: every
    group size gives the keys of one pair per item, with deep pairs in the second tier,
    constant biconditionals inside groups and a batch that ends inside a group."""
    p = I.parse("p")
    pairs = _pairs()[:150] + [([I.TOP], [I.BOT]), (p, p), ([I.BOT], [I.BOT])]
    pairs += _pairs()[-10:]
    frames = I.frame_family(n, nframes)
    monkeypatch.setenv("KRIPKE_LIST_GROUP", "1")
    single = kr.split(pairs, frames, n)
    assert single[150] == 0 and single[151] == kr.NO_KEY
    for g in ("2", "3", "4"):
        monkeypatch.setenv("KRIPKE_LIST_GROUP", g)
        assert np.array_equal(kr.split(pairs, frames, n), single), (g, n)
