"""Seeded input generators: determinism, exact size/depth bounds, text round trip."""
import numpy as np

from paper_2606_15437_amd import inputs as I


def test_splitmix64_reference_values():
    # SplitMix64 from state 0: the published first outputs of the generator
    r = I.SplitMix64(0)
    assert [r.next() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                            0x06C45D188009454F]
    z = np.arange(1, 4, dtype=np.uint64) * np.uint64(I.GAMMA)
    assert [int(x) for x in I.mix64_np(z)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                0x06C45D188009454F]


def test_below_np_matches_exact():
    rng = I.SplitMix64(5)
    xs = np.array([rng.next() for _ in range(1000)], dtype=np.uint64)
    for r in (1, 2, 3, 5, 7, 64, 1000):
        assert [int(v) for v in I.below_np(xs, r)] == [(int(x) * r) >> 64 for x in xs]


def test_config_generators_bounds():
    for fs, lo, hi, dmax, vmax in ((I.config1_formulas(), 1, 12, 3, 2),
                                   (I.config2_formulas(), 3, 24, 4, 3),
                                   (I.config3_formulas(), 3, 40, 6, 2)):
        for f in fs:
            assert lo <= len(f) <= hi
            assert I.modal_depth(f) <= dmax
            assert all(not I.is_var(op) or op - I.VAR0 < vmax for op in f)
    assert len(I.config3_formulas()) == 4096
    assert I.config3_formulas() == I.config3_formulas()


def test_text_roundtrip():
    for f in I.config2_formulas()[:200] + I.config1_formulas():
        assert I.parse(I.to_text(f)) == f
    assert I.parse("[](p -> q) -> (<>p -> <>q)") == [2, 3, 9, 10, 2, 11, 3, 11, 9, 9]


def test_pack_unpack():
    fs = I.config1_formulas()
    code, offs = I.pack(fs)
    assert I.unpack(code, offs) == fs
    assert int(offs[-1]) == sum(len(f) for f in fs)


def test_frame_family_structure():
    for n in (6, 7, 8):
        fr = I.frame_family(n, 4096)
        assert fr.shape == (4096, n)
        assert list(fr[0]) == I.path_frame(n)
        assert list(fr[1]) == [(1 << ((w + 1) % n)) for w in range(n)]
        kinds = I.family_kind(np.arange(4096))
        edges = np.array([[bin(int(x)).count("1") for x in row] for row in fr]).sum(1)
        assert (edges[kinds == I.FAMILY_PATH] == n - 1).all()
        assert (edges[kinds == I.FAMILY_CYCLE] == n).all()
        assert (edges[kinds == I.FAMILY_TREE] == n - 1).all()
        er = edges[kinds == I.FAMILY_ER]
        assert abs(er.mean() / (n * n) - 0.2) < 0.02
        # frames are addressable: a window equals the same rows of a longer run
        assert (I.frame_family(n, 100, start=1000) == fr[1000:1100]).all()


def test_retrieval_corpus():
    c = I.retrieval_corpus(I.SEED_C5_TEST, 3000, n_words=500)
    assert len(c) == 3000 and len(set(map(tuple, c))) == 3000
    assert all(len(f) <= 21 for f in c)
    assert I.alpha(2) in c and I.alpha(3) in c


def test_equivalent_variant_is_equivalent(orc):
    """Each rewrite keeps the truth set: the biconditional has no countermodel on any
    frame with at most 3 worlds, and every rewrite kind really fires."""
    fs = I.formula_batch(0xE0F1, 120, (2, 10), (0, 3), I.LEAVES_2)
    changed = set()
    for k, f in enumerate(fs):
        g = I.equivalent_variant(f, k)
        assert g != f
        if len(g) == len(f):
            changed.add("swap")
        elif g[-1] == I.NOT and len(g) == len(f) + 2 and g[-2] in (I.BOX, I.DIA):
            changed.add("dual")
        chi = I.iff(f, g)
        for n in (1, 2, 3):
            key, cnt, _ = orc.census(chi, n, 0, 2)
            assert key == orc.NONE and cnt == 0, (I.to_text(f), I.to_text(g))
    assert changed == {"swap", "dual"}


def test_census_enumeration_count():
    """Every tree with at most seven nodes over p, q, NOT, BOX, DIA, AND, OR, IMP:
    44,678 of them (the paper's raw census enumeration, Section 6), all distinct,
    constant-free and in size order."""
    fs = I.enumerate_formulas(7)
    assert len(fs) == 44678 and len(set(map(tuple, fs))) == 44678
    sizes = [len(f) for f in fs]
    assert sizes == sorted(sizes) and max(sizes) == 7
    assert all(op not in (I.TOP, I.BOT) for f in fs for op in f)
    # counts per size follow T(1) = 2, T(s) = 3 T(s-1) + 3 sum_a T(a) T(s-1-a)
    t = {1: 2}
    for s in range(2, 8):
        t[s] = 3 * t[s - 1] + 3 * sum(t[a] * t[s - 1 - a] for a in range(1, s - 1))
    assert [sizes.count(s) for s in range(1, 8)] == [t[s] for s in range(1, 8)]
    assert len(I.all_pointed_models(3, 2)) == 64 + 512 + 98304


def test_adversarial_generators_deterministic_and_in_range():
    for g in I.ADVERSARIAL:
        for n in (6, 11, 16):
            a = I.adversarial_frames(g, n, 300)
            b = I.adversarial_frames(g, n, 100, start=200)
            assert a.shape == (300, n) and (a < (1 << n)).all()
            assert (a[200:] == b).all()
    # bottleneck frames have no dead ends; the dead-end generator always has one
    assert (I.adversarial_frames("scc-bottleneck", 12, 200) != 0).all()
    assert ((I.adversarial_frames("dead-end", 12, 200) == 0).any(axis=1)).all()
