"""Split search on large frames (world-mask kernel) and the mining / adversarial frame
synthesis protocol: parity with the other split kernels and the oracle, every
reported separation checked by the oracle."""
import numpy as np
import pytest

from paper_2606_15437_amd import inputs as I

pytestmark = pytest.mark.gpu

NONE = (1 << 64) - 1


@pytest.fixture(scope="module")
def kr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_15437_amd import kripke
    kripke.lib()
    return kripke


def _pairs(nvars, count=40, stream=0):
    leaves = I.LEAVES_2 if nvars == 2 else ((I.TOP, I.BOT, I.var(0)) if nvars == 1 else
                                            (I.TOP, I.BOT))
    fs = I.formula_batch(0xADE5, count, (2, 12), (0, 5), leaves, stream=stream)
    pairs = list(zip(fs[0::2], fs[1::2]))
    pairs += [(f, I.equivalent_variant(f, k)) for k, f in enumerate(fs[:8])]
    pairs += [(I.alpha(2), I.alpha(3)), (I.alpha(3), I.alpha(4)), (I.dia_k_top(5), I.dia_k_top(6)),
              (I.box_k_bot(6), I.box_k_bot(7))]
    return pairs


@pytest.mark.parametrize("n,nvars", [(6, 2), (7, 1), (8, 2), (8, 0)])
def test_worldmask_matches_bitsliced_kernels(kr, monkeypatch, n, nvars):
    frames = I.frame_family(n, 700, start=3)
    pairs = _pairs(nvars, stream=n)
    ref = kr.split(pairs, frames, n, nvars)
    monkeypatch.setenv("KRIPKE_SPLIT_WORLDMASK", "1")
    got = kr.split(pairs, frames, n, nvars)
    assert (got == ref).all()
    assert (ref == NONE).sum() >= 8 and (ref != NONE).sum() >= 10


@pytest.mark.parametrize("n,nvars", [(11, 1), (12, 1), (13, 0), (16, 0)])
def test_large_frames_match_oracle(kr, orc, n, nvars):
    frames = np.concatenate([I.adversarial_frames(g, n, 24) for g in I.ADVERSARIAL])
    pairs = _pairs(nvars, count=24, stream=n)
    got = kr.split(pairs, frames, n, nvars)
    for (a, b), k in zip(pairs, got):
        assert int(k) == orc.split(a, b, frames, nvars), (I.to_text(a), I.to_text(b))


def test_mining_and_adversarial_protocol(kr, orc):
    from paper_2606_15437_amd import adversarial as A
    rec, det = A.run(frames_per=192, log=None)
    assert rec["candidates"] == len(A.mining_candidates()) == 478
    assert 0 < rec["exact_prefix_survivors"] < rec["candidates"]
    cands = det["cands"]
    # the exact prefix: every survivor's biconditional has no countermodel through
    # three worlds (oracle), and alpha_2 / alpha_3 is among the survivors
    for _, a, b, nv in cands[:60]:
        for n in (1, 2, 3):
            assert orc.census(I.iff(a, b), n, 0, nv)[0] == NONE
    labels = [c[0] for c in cands]
    assert ("[]<>", "T", 2) in labels
    j = labels.index(("[]<>", "T", 2))
    assert det["template_sep"][j] == 6 and det["template_witness"][j]["template"] == "path"
    # every template and adversarial witness separates the pair (oracle)
    for j, w in enumerate(det["template_witness"]):
        if w is None:
            continue
        _, a, b, nv = cands[j]
        assert orc.sat_at(a, w["succ"], nv, w["valuation"], w["world"]) != \
            orc.sat_at(b, w["succ"], nv, w["valuation"], w["world"])
    assert det["hits"]
    for j, ws in det["hits"].items():
        _, a, b, nv = cands[j]
        for w in ws:
            assert orc.sat_at(a, w["succ"], nv, w["valuation"], w["world"]) != \
                orc.sat_at(b, w["succ"], nv, w["valuation"], w["world"])
