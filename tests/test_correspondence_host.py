"""Host side of frame-correspondence recovery (Section 10): the first-order condition
library's extensions, as packed bitmaps over every frame index, against closed-form
frame counts (reflexive 2^(n^2-n); serial (2^n - 1)^n; symmetric 2^(n(n+1)/2);
partially functional (n+1)^n; functional n^n; coreflexive 2^n; transitive: the labelled
transitive relations, OEIS A006905) and against the per-frame boolean extensions."""
import numpy as np

from paper_2606_15437_amd import correspondence as R

TRANSITIVE = {1: 2, 2: 13, 3: 171, 4: 3994}


def _count(m):
    return int(np.unpackbits(m.view(np.uint8)).sum())


def test_condition_maps_closed_forms():
    for n in (2, 3, 4):
        m = R.condition_maps(["reflexive", "serial", "symmetric", "partially functional",
                              "transitive", "reflexive & transitive", "functional",
                              "coreflexive"], n)
        assert _count(m["reflexive"]) == 2 ** (n * n - n)
        assert _count(m["serial"]) == (2 ** n - 1) ** n
        assert _count(m["symmetric"]) == 2 ** (n * (n + 1) // 2)
        assert _count(m["partially functional"]) == (n + 1) ** n
        assert _count(m["transitive"]) == TRANSITIVE[n]
        assert _count(m["functional"]) == n ** n
        assert _count(m["coreflexive"]) == 2 ** n
        # preorders (OEIS A000798): 4, 29, 355
        assert _count(m["reflexive & transitive"]) == {2: 4, 3: 29, 4: 355}[n]


def test_condition_maps_match_extensions():
    names = list(R.textbook_library())
    ext = R.extensions(names, max_n=4, lib=R.textbook_library())
    maps = R.condition_maps(names, 4)
    offset = sum(1 << (k * k) for k in (1, 2, 3))  # extensions concatenate n = 1..4
    for name in names:
        bits = np.unpackbits(maps[name].view(np.uint8), bitorder="little").astype(bool)
        assert (bits[:1 << 16] == ext[name][offset:]).all(), name


def test_textbook_library_holds_table9_and_coreflexive():
    lib = R.textbook_library()
    assert list(lib)[:8] == list(R.TABLE9_CONDITIONS)
    ext = R.extensions(["coreflexive"], max_n=3, lib=lib)["coreflexive"]
    # coreflexive = symmetric and antisymmetric: R contained in the identity
    both = R.extensions(["symmetric & antisymmetric"], max_n=3)["symmetric & antisymmetric"]
    assert (ext == both).all() and int(ext.sum()) == 2 + 4 + 8
