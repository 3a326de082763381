"""The five-world census of Section 6 reproduced on the GPU, pinned to the paper's
printed figures and checked against the oracle.

Paper figures used as pins (Section 6 and its macros): 44,678 enumerated trees,
5,621 classes on frames of at most three worlds, 5,624 formulas with the named
axioms; in K 5,086 formulas refuted on one world, 536 on two, two survivors (the
propositional tautology and axiom K) and no refutable formula needing three worlds
(Proposition 4); 428 formulas refuted in K but surviving T, 48 refuted in T but
surviving S4 and 118 refuted in S4 but surviving S5 (the separation counts of
Section 6); 20,990 certificates, one per refuted (formula, class) pair, every one
accepted by the independent checker (Section 6, Proposition 3).  The named axioms
are K, T and McKinsey; with D in place of McKinsey the K-to-T count would be 429
and the certificates 20,987.
"""
import os
from concurrent.futures import ThreadPoolExecutor

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
    from paper_2606_15437_amd import census_corpus, kripke
    kripke.lib()
    return census_corpus


@pytest.fixture(scope="module")
def corpus(cc):
    raw, reps, corpus = cc.build_corpus()
    return raw, reps, corpus


@pytest.fixture(scope="module")
def result(cc, corpus):
    return cc.census(corpus[2])


def _workers():
    return min(16, os.cpu_count() or 1)


def test_classes_match_paper_and_oracle(cc, corpus, orc):
    raw, reps, full = corpus
    assert len(raw) == 44678 and len(reps) == 5621 and len(full) == 5624
    # the oracle's own truth tables over every pointed model with <= 3 worlds give
    # the same partition, with the same first members
    samples = I.all_pointed_models(3, 2)
    chunks = [raw[i:i + 2048] for i in range(0, len(raw), 2048)]
    with ThreadPoolExecutor(max_workers=_workers()) as ex:
        sig = np.concatenate(list(ex.map(lambda ch: orc.signatures(ch, samples, 2), chunks)))
    rows = np.ascontiguousarray(sig).view(np.dtype((np.void, sig.shape[1] * 8))).ravel()
    _, first = np.unique(rows, return_index=True)
    assert (np.sort(first) == reps).all()


def test_k_frontier_matches_paper(cc, result, corpus):
    s = cc.summary(result)
    hist = s["minimal_size_histogram"]["K"]
    assert (hist["1"], hist["2"], hist["none"]) == (5086, 536, 2)
    assert s["max_refuted_minimal_size"]["K"] == 2  # Proposition 4
    # the two K survivors: the propositional tautology and axiom K (Proposition 4)
    full = corpus[2]
    surv = np.nonzero(result["minimal"][0] == 0)[0]
    texts = sorted(I.to_text(full[i]) for i in surv)
    assert I.to_text(I.named_axioms()[0]) in texts
    other = [full[i] for i in surv if full[i] != I.named_axioms()[0]][0]
    assert all(t not in other for t in (I.BOX, I.DIA))  # a propositional formula


def test_separation_counts_match_paper(cc, result):
    s = cc.summary(result)
    sep = s["separations"]
    assert sep["K->T"] == 428 and sep["T->S4"] == 48 and sep["S4->S5"] == 118
    assert s["certificates"] == 20990
    assert s["survivors"] == {"K": 2, "T": 430, "S4": 478, "S5": 596}


def test_every_certificate_verifies(cc, result, corpus, orc):
    """All 20,990 certificates (least countermodel at the minimal size, per refuted
    formula and class) are accepted by the oracle's pointwise checker."""
    full = corpus[2]
    m = result["minimal"]
    checks = [(int(i), c, int(m[c, i]), int(result["keys"][c, m[c, i] - 1, i]))
              for c in range(4) for i in np.nonzero(m[c] > 0)[0]]
    assert len(checks) == 20990

    def cert(ch):
        i, c, n, key = ch
        frame, val, world = orc.decode_key(key, n, 2)
        return orc.check_certificate(full[i], I.frame_succ(frame, n), 2, val, world, c)

    with ThreadPoolExecutor(max_workers=_workers()) as ex:
        assert all(ex.map(cert, checks, chunksize=256))


def test_census_parity_small_layers(result, corpus, orc):
    """Bit-exact first keys and fail counts for every formula and class at n <= 3."""
    full = corpus[2]

    def one(i):
        out = []
        for c in range(4):
            for n in (1, 2, 3):
                k, cnt, _ = orc.census(full[i], n, c, 2)
                out.append((c, n, k, cnt))
        return i, out

    with ThreadPoolExecutor(max_workers=_workers()) as ex:
        for i, out in ex.map(one, range(len(full))):
            for c, n, k, cnt in out:
                assert int(result["keys"][c, n - 1, i]) == k, (i, c, n)
                assert int(result["counts"][c, n - 1, i]) == cnt, (i, c, n)


def test_certificates_and_larger_layers_sampled(result, corpus, orc):
    """Every n = 4 and n = 5 first key of a refuted formula is a certificate; sampled
    n = 5 keys equal the oracle's early-exit scan; sampled T and S4 survivors have no
    countermodel on four worlds."""
    full = corpus[2]
    keys = result["keys"]
    checks = []
    for c in range(4):
        for n in (4, 5):
            for i in np.nonzero(keys[c, n - 1] != NONE)[0]:
                checks.append((int(i), c, n, int(keys[c, n - 1, i])))

    def cert(ch):
        i, c, n, key = ch
        frame, val, world = orc.decode_key(key, n, 2)
        succ = I.frame_succ(frame, n)
        return orc.check_certificate(full[i], succ, 2, val, world, c)

    with ThreadPoolExecutor(max_workers=_workers()) as ex:
        assert all(ex.map(cert, checks))
    rng = np.random.default_rng(7)
    refuted5 = np.nonzero(keys[0, 4] != NONE)[0]
    for i in rng.choice(refuted5, 40, replace=False):
        k, _, _ = orc.census(full[i], 5, 0, 2, stop_at_first=True)
        assert int(keys[0, 4, i]) == k, i
    for c in (1, 2):
        surv = np.nonzero(result["minimal"][c] == 0)[0]
        for i in rng.choice(surv, 6, replace=False):
            k, cnt, _ = orc.census(full[i], 4, c, 2, stop_at_first=True)
            assert k == NONE, (i, c)
