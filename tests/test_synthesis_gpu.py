"""Active synthesis (32 context-iteration pairs): separation sizes against the paper's
facts, the 128 CPU/GPU parity checks through four worlds, and every witness checked
by the oracle."""
import numpy as np
import pytest

from paper_2606_15437_amd import inputs as I

pytestmark = pytest.mark.gpu

NONE = (1 << 64) - 1


@pytest.fixture(scope="module")
def syn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_15437_amd import kripke, synthesis
    kripke.lib()
    return synthesis


@pytest.fixture(scope="module")
def recs(syn):
    return {(r["context"], r["base"], r["m"]): r for r in syn.run()}


def test_alpha_family_matches_table4_and_prop6(recs):
    """alpha_m vs alpha_(m+1): separation sizes 4, 6, 8 (Table 4) and 10 = 2m + 2 (Lemma 2);
    alpha_2 / alpha_3 agree through five worlds and split on the six-world path at its
    root (Proposition 6)."""
    sizes = [recs[("BOX DIA", "TOP", m)]["separation"] for m in (1, 2, 3, 4)]
    assert sizes == [4, 6, 8, 10]
    r = recs[("BOX DIA", "TOP", 2)]
    assert r["agree_through"] == 5 and r["witness"]["template"] == "path"
    assert r["witness"]["succ"] == [2, 4, 8, 16, 32, 0] and r["witness"]["world"] == 0
    # the dual family separates at the same sizes
    assert [recs[("DIA BOX", "BOT", m)]["separation"] for m in (1, 2, 3, 4)] == [4, 6, 8, 10]


def test_path_depth_families_pigeonhole(recs):
    """DIA^(2m) TOP vs DIA^(2m+2) TOP and BOX^(2m) BOT vs BOX^(2m+2) BOT first differ on
    2m + 1 worlds (a walk of length 2m needs 2m + 1 distinct worlds or a cycle)."""
    for key in (("DIA DIA", "TOP"), ("BOX BOX", "BOT")):
        for m in (1, 2, 3, 4):
            r = recs[key + (m,)]
            assert r["separation"] == 2 * m + 1, r
            assert r["agree_through"] == min(2 * m, 5)


def test_equivalent_families_never_separate(recs):
    """BOX^k TOP is TOP and DIA^k BOT is BOT on every frame."""
    for key in (("BOX BOX", "TOP"), ("DIA DIA", "BOT")):
        for m in (1, 2, 3, 4):
            r = recs[key + (m,)]
            assert r["separation"] is None and r["agree_through"] == 5


def test_ranking_prefers_exact_late_hits(syn, recs):
    ranked = syn.run()
    top = ranked[0]
    assert top["agree_through"] == 5 and top["separation"] == 6
    scores = [r["R"] for r in ranked]
    assert scores == sorted(scores, reverse=True)


def test_parity_through_four_worlds_and_witnesses(syn, recs, orc):
    """128 parity checks: the first countermodel of every candidate biconditional at
    n = 1..4, GPU against oracle; then every reported witness is a separating model."""
    import torch
    from paper_2606_15437_amd import kripke as K
    cands = syn.candidates()
    chis = [I.iff(a, b) for _, a, b in cands]
    code, offs = I.pack(chis)
    checks = 0
    for n in (1, 2, 3, 4):
        out = torch.empty((len(chis), 2), dtype=torch.int64, device="cuda")
        K.kripke_census(code, offs, n, K.KRIPKE_K, 0, out)
        got = K.as_u64(out)
        for i, chi in enumerate(chis):
            k, c, _ = orc.census(chi, n, 0, 0)
            assert int(got[i, 0]) == k and int(got[i, 1]) == c, (i, n)
            checks += 1
    assert checks == 128
    for (label, a, b) in cands:
        r = recs[label]
        w = r["witness"]
        if w is None:
            continue
        n = w["n"]
        succ = w["succ"] if w["kind"] == "template" else I.frame_succ(w["frame"], n)
        assert orc.sat_at(a, succ, 0, 0, w["world"]) != orc.sat_at(b, succ, 0, 0, w["world"])
        if w["kind"] == "template":
            frames = np.array([syn.templates(n)[t] for t in syn.templates(n)], dtype=np.uint32)
            assert orc.split(a, b, frames, 0) != NONE
