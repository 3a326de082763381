"""Checkpoint and resume of a census: a layer cut into ragged frame slices, each run by
kripke_census_range and merged with min(first_key) and sum(fail_count), equals the
one-shot census bit for bit (Theorem 2's layer scan is a disjoint union over frames;
the merge rule is stated in include/kripke.h).  Also: DECIDE slices give the same least
keys as COUNT slices, and an empty slice leaves the no-countermodel result."""
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


def _range(kr, fs, n, cls, nvars, f0, f1, flags=0):
    import torch
    code, offs = I.pack(fs)
    out = torch.full((len(fs), 2), 7, dtype=torch.int64, device="cuda")
    kr.kripke_census_range(code, offs, n, cls, nvars, f0, f1, flags, out)
    torch.cuda.synchronize()
    return kr.as_u64(out).copy()


def _cuts(total, parts, seed):
    rng = np.random.default_rng(seed)
    inner = np.sort(rng.choice(np.arange(1, total), size=parts - 1, replace=False))
    return [0, *inner.tolist(), total]


@pytest.mark.parametrize("n,nvars,cls,fs", [
    (5, 2, 0, "c3"), (5, 2, 1, "c3"), (5, 2, 2, "c3"), (5, 2, 3, "c3"),
    (4, 3, 0, "c2"), (4, 3, 1, "c2"), (4, 3, 2, "c2"),
])
def test_merged_slices_equal_one_shot(kr, n, nvars, cls, fs):
    formulas = (I.config3_formulas()[:256] if fs == "c3" else I.config2_formulas()[:256])
    total = 1 << (n * n)
    whole = _range(kr, formulas, n, cls, nvars, 0, total)
    keys = np.full(len(formulas), NONE, dtype=np.uint64)
    cnts = np.zeros(len(formulas), dtype=np.uint64)
    cuts = _cuts(total, 7, 1000 * n + 10 * nvars + cls)
    for a, b in zip(cuts[:-1], cuts[1:]):
        part = _range(kr, formulas, n, cls, nvars, a, b)
        keys = np.minimum(keys, part[:, 0])
        cnts = cnts + part[:, 1]
        dec = _range(kr, formulas, n, cls, nvars, a, b, flags=1)
        assert np.array_equal(dec[:, 0], part[:, 0]), (a, b)  # DECIDE: same least keys
    assert np.array_equal(keys, whole[:, 0])
    assert np.array_equal(cnts, whole[:, 1])
    # the one-shot range is the layer census itself
    if n <= 5:
        k, c = kr.census(formulas, n, cls, nvars)
        assert np.array_equal(k, whole[:, 0]) and np.array_equal(c, whole[:, 1])


def test_empty_slice_is_the_identity_of_the_merge(kr):
    fs = I.config3_formulas()[:32]
    r = _range(kr, fs, 5, 0, 2, 12345, 12345)
    assert (r[:, 0] == NONE).all() and (r[:, 1] == 0).all()
