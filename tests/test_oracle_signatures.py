"""Pins for the oracle's signature function (truth at sampled pointed models).

A signature bit is M,w |= phi at one pointed model (Section 2, satisfaction at a
pointed model).  The oracle decodes each sample's packed fields
(n << 60 | frame << 24 | valuation << 4 | world) and evaluates the recursive
definition; these tests check it against closed forms that follow from the
satisfaction clauses alone, with the fields decoded here by plain integer
arithmetic, and against the paper's count of semantic classes in the census
corpus (Section 6: 44,678 trees fall into 5,621 classes of equal truth on every
frame with at most three worlds).
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2606_15437_amd import inputs as I


def _fields(sample):
    s = int(sample)
    n = s >> 60
    return n, (s >> 24) & ((1 << 36) - 1), (s >> 4) & ((1 << 20) - 1), s & 15


def _row(f, n, w):
    """Successor set of world w in frame f as a bitmask."""
    return (f >> (w * n)) & ((1 << n) - 1)


def _var_set(val, n, i):
    """Worlds where p_i holds."""
    return (val >> (i * n)) & ((1 << n) - 1)


# Closed forms of small formulas at a pointed model (n, f, val, w), from the
# satisfaction clauses: DIA phi holds iff some successor satisfies phi, BOX phi iff
# every successor does (so BOX holds and DIA fails at a dead end).
def _cf_p(n, f, val, w):
    return (_var_set(val, n, 0) >> w) & 1 == 1


def _cf_q(n, f, val, w):
    return (_var_set(val, n, 1) >> w) & 1 == 1


def _cf_dia_top(n, f, val, w):
    return _row(f, n, w) != 0


def _cf_box_bot(n, f, val, w):
    return _row(f, n, w) == 0


def _cf_dia_p(n, f, val, w):
    return (_row(f, n, w) & _var_set(val, n, 0)) != 0


def _cf_box_q(n, f, val, w):
    return (_row(f, n, w) & ~_var_set(val, n, 1)) == 0


def _cf_dia_dia_top(n, f, val, w):
    succ = _row(f, n, w)
    return any((succ >> v) & 1 and _row(f, n, v) != 0 for v in range(n))


def _cf_p_imp_box_q(n, f, val, w):
    return (not _cf_p(n, f, val, w)) or _cf_box_q(n, f, val, w)


CLOSED_FORMS = [("p", _cf_p), ("q", _cf_q), ("<>T", _cf_dia_top), ("[]F", _cf_box_bot),
                ("<>p", _cf_dia_p), ("[]q", _cf_box_q), ("<><>T", _cf_dia_dia_top),
                ("p -> []q", _cf_p_imp_box_q)]


def _expected_bits(fn, samples):
    words = (len(samples) + 63) // 64
    out = np.zeros(words, dtype=np.uint64)
    for s, smp in enumerate(samples):
        if fn(*_fields(smp)):
            out[s // 64] |= np.uint64(1) << np.uint64(s % 64)
    return out


@pytest.mark.parametrize("which", ["all_pointed_models", "signature_samples"])
def test_signature_closed_forms(orc, which):
    """Every pointed model with at most three worlds (and the 4,096-sample list of
    the learned proposal): the oracle's bits equal the closed forms bit for bit."""
    samples = I.all_pointed_models(3, 2) if which == "all_pointed_models" else \
        I.signature_samples()
    formulas = [I.parse(text) for text, _ in CLOSED_FORMS]
    sig = orc.signatures(formulas, samples, 2)
    for (text, fn), row in zip(CLOSED_FORMS, sig):
        exp = _expected_bits(fn, samples)
        assert (row == exp).all(), text


def test_signature_fields_are_independent(orc):
    """Samples that differ in one field only: frame, valuation, world and n each move
    the result exactly as the closed forms say (a field read from the wrong bits, or
    n taken from the wrong nibble, breaks at least one of these)."""
    pack = lambda n, f, v, w: (n << 60) | (f << 24) | (v << 4) | w
    cases = []
    for n in (1, 2, 3):
        for f in (0, (1 << (n * n)) - 1, 1 << (n * n - 1), 1 << (n - 1)):
            for v in (0, (1 << (2 * n)) - 1, 1 << n, 1):
                for w in range(n):
                    cases.append(pack(n, f, v, w))
    cases += [cases[-1]] * ((-len(cases)) % 64)
    samples = np.array(cases, dtype=np.uint64)
    formulas = [I.parse(text) for text, _ in CLOSED_FORMS]
    sig = orc.signatures(formulas, samples, 2)
    for (text, fn), row in zip(CLOSED_FORMS, sig):
        assert (row == _expected_bits(fn, samples)).all(), text


def _oracle_signatures_parallel(orc, formulas, samples, chunk=512):
    parts = [formulas[i:i + chunk] for i in range(0, len(formulas), chunk)]
    with ThreadPoolExecutor(max_workers=8) as ex:  # the C call releases the interpreter lock
        sigs = list(ex.map(lambda p: orc.signatures(p, samples, 2), parts))
    return np.concatenate(sigs, axis=0)


@pytest.mark.slow
def test_census_corpus_classes_from_oracle(orc):
    """Section 6: the 44,678 constant-free trees of at most seven nodes over p, q fall
    into 5,621 classes of equal truth at every pointed model with at most three
    worlds, computed here from the oracle's signatures alone."""
    raw = I.enumerate_formulas(7)
    assert len(raw) == 44678
    samples = I.all_pointed_models(3, 2)
    sig = _oracle_signatures_parallel(orc, raw, samples)
    rows = np.ascontiguousarray(sig).view(np.dtype((np.void, sig.shape[1] * 8))).ravel()
    assert len(np.unique(rows)) == 5621
