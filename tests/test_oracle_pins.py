"""Pins for the CPU oracle: facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (golden fixtures with citations), closed forms, textbook
reductions, invariants, and an independent brute-force evaluator built here
from the first-order standard translation of modal formulas.
"""
import itertools
import os

import pytest

from paper_2606_15437_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NONE = (1 << 64) - 1
K, T, S4, S5, K4 = 0, 1, 2, 3, 4


def _golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.strip() for ln in fh if ln.strip() and not ln.startswith("#")]


# ------------------------------------------------------------------------
# Independent brute-force evaluator: the standard translation of a modal
# formula into a first-order formula over explicit worlds, compiled to Python.
def _tree(code):
    st = []
    for op in code:
        if op in (I.NOT, I.BOX, I.DIA):
            st.append((op, st.pop()))
        elif op in (I.AND, I.OR, I.IMP, I.IFF):
            b = st.pop()
            a = st.pop()
            st.append((op, a, b))
        else:
            st.append((op,))
    assert len(st) == 1
    return st[0]


def standard_translation(code):
    """Python callable sat(R, V, n, x): R[x][y] adjacency, V[i][x] valuation."""
    counter = itertools.count()

    def st(t, x):
        op = t[0]
        if op == I.TOP:
            return "True"
        if op == I.BOT:
            return "False"
        if I.is_var(op):
            return f"bool(V[{op - I.VAR0}][{x}])"
        if op == I.NOT:
            return f"(not {st(t[1], x)})"
        if op == I.BOX:
            y = f"y{next(counter)}"
            return f"all((not R[{x}][{y}]) or {st(t[1], y)} for {y} in range(n))"
        if op == I.DIA:
            y = f"y{next(counter)}"
            return f"any(R[{x}][{y}] and {st(t[1], y)} for {y} in range(n))"
        a, b = st(t[1], x), st(t[2], x)
        if op == I.AND:
            return f"({a} and {b})"
        if op == I.OR:
            return f"({a} or {b})"
        if op == I.IMP:
            return f"((not {a}) or {b})"
        if op == I.IFF:
            return f"({a} == {b})"
        raise ValueError(op)

    return eval(f"lambda R, V, n, x0: {st(_tree(code), 'x0')}")


def brute_census(code, n, nvars, frames=None, cls_pred=None):
    """(first_key, fail_count) by enumerating frames, valuations and worlds."""
    sat = standard_translation(code)
    key, cnt = NONE, 0
    frames = range(1 << (n * n)) if frames is None else frames
    for f in frames:
        R = [[(f >> (w * n + v)) & 1 for v in range(n)] for w in range(n)]
        if cls_pred is not None and not cls_pred(R, n):
            continue
        for val in range(1 << (nvars * n)):
            V = [[(val >> (i * n + w)) & 1 for w in range(n)] for i in range(nvars)]
            bad = [w for w in range(n) if not sat(R, V, n, w)]
            if bad:
                cnt += 1
                if key == NONE:
                    key = (f << (nvars * n + 4)) | (val << 4) | bad[0]
    return key, cnt


# First-order frame conditions, written directly on the relation.
def reflexive(R, n):
    return all(R[w][w] for w in range(n))


def serial(R, n):
    return all(any(R[w]) for w in range(n))


def transitive(R, n):
    return all(not (R[u][v] and R[v][w]) or R[u][w]
               for u in range(n) for v in range(n) for w in range(n))


def euclidean(R, n):
    return all(not (R[u][v] and R[u][w]) or R[v][w]
               for u in range(n) for v in range(n) for w in range(n))


def symmetric(R, n):
    return all(R[u][v] == R[v][u] for u in range(n) for v in range(n))


def partially_functional(R, n):
    return all(not (R[u][v] and R[u][w]) or v == w
               for u in range(n) for v in range(n) for w in range(n))


def dense(R, n):
    return all(not R[u][w] or any(R[u][v] and R[v][w] for v in range(n))
               for u in range(n) for w in range(n))


def confluent(R, n):
    return all(not (R[u][v] and R[u][w]) or any(R[v][x] and R[w][x] for x in range(n))
               for u in range(n) for v in range(n) for w in range(n))


CONDITIONS = {"reflexive": reflexive, "serial": serial, "transitive": transitive,
              "euclidean": euclidean, "symmetric": symmetric,
              "partially_functional": partially_functional, "dense": dense,
              "confluent": confluent}


def s4_pred(R, n):
    return reflexive(R, n) and transitive(R, n)


def s5_pred(R, n):
    return s4_pred(R, n) and symmetric(R, n)


CLASS_PRED = {K: None, T: reflexive, S4: s4_pred, S5: s5_pred, K4: transitive}


def frame_valid(orc, code, f, n, nvars=1):
    key, _, _ = orc.census(code, n, K, nvars, f, f + 1)
    return key == NONE


# ------------------------------------------------------------------ P10
@pytest.mark.parametrize("n", [1, 2])
def test_bruteforce_agrees_on_config1(orc, n):
    """Every config-1 formula: oracle (key, count) equals the standard-translation brute force."""
    for code in I.config1_formulas():
        assert orc.census(code, n, K, 2)[:2] == brute_census(code, n, 2), I.to_text(code)


def test_bruteforce_agrees_n3_and_classes(orc):
    formulas = I.config1_formulas()[:6] + [I.parse("[]p -> [][]p"), I.parse("<>p -> []<>p"),
                                           I.parse("[](p -> <>q) | <>[]~q")]
    for code in formulas:
        for cls in (K, T, S4, S5, K4):
            got = orc.census(code, 3, cls, 2, threads=4)[:2]
            assert got == brute_census(code, 3, 2, cls_pred=CLASS_PRED[cls]), (I.to_text(code), cls)


def test_bruteforce_agrees_three_vars(orc):
    for code in I.config2_formulas()[:4]:
        assert orc.census(code, 2, K, 3)[:2] == brute_census(code, 2, 3)


# ------------------------------------------------------------------ P7
def test_class_sizes(orc):
    rows = {ln.split()[0]: [int(x) for x in ln.split()[1:]] for ln in _golden_lines("class_sizes.txt")}
    for name, cls in (("K", K), ("T", T), ("S4", S4), ("S5", S5), ("K4", K4)):
        for n in range(1, 5):
            assert orc.class_size(n, cls) == rows[name][n - 1], (name, n)
    for n in range(1, 6):
        assert rows["K"][n - 1] == 2 ** (n * n) and rows["T"][n - 1] == 2 ** (n * n - n)


@pytest.mark.slow
def test_class_sizes_n5(orc):
    rows = {ln.split()[0]: [int(x) for x in ln.split()[1:]] for ln in _golden_lines("class_sizes.txt")}
    for name, cls in (("S4", S4), ("S5", S5)):
        assert orc.class_size(5, cls) == rows[name][4]


# ------------------------------------------------------------------ P1
def test_named_axioms(orc):
    kax = I.parse("[](p -> q) -> ([]p -> []q)")
    table1 = I.parse(I.TABLE1_FORMULA)
    tax = I.parse("[]p -> p")
    ax4 = I.parse("[]p -> [][]p")
    ax5 = I.parse("<>p -> []<>p")
    for n in (1, 2, 3, 4):
        for cls in (K, T, S4, S5):
            # the normality axiom K and the Table-1 formula are valid on every frame
            assert orc.census(kax, n, cls, 2, threads=8)[0] == NONE
            assert orc.census(table1, n, cls, 2, threads=8)[0] == NONE
        # T is valid on reflexive frames, 4 on transitive ones, 5 on S5
        assert orc.census(tax, n, T, 1, threads=8)[0] == NONE
        assert orc.census(ax4, n, K4, 1, threads=8)[0] == NONE
        assert orc.census(ax4, n, S4, 1, threads=8)[0] == NONE
        assert orc.census(ax5, n, S5, 1, threads=8)[0] == NONE
    # T is refuted in K by the one-world model with no edge and p false: key 0
    key, cnt, _ = orc.census(tax, 1, K, 1)
    assert key == 0 and cnt == 1
    # 4 and 5 are refuted in K (and 5 in S4) on small frames
    assert orc.census(ax4, 2, K, 1)[0] != NONE
    assert orc.census(ax5, 3, S4, 1, threads=8)[0] != NONE


# ------------------------------------------------------------------ P6
def test_table9_correspondences(orc):
    """Each Sahlqvist axiom is valid on exactly the frames satisfying its condition (n <= 3);
    McKinsey matches none of the conditions."""
    rows = [[c.strip() for c in ln.split("|")] for ln in _golden_lines("table9_correspondence.txt")]
    for name, text, cond in rows:
        code = I.parse(text)
        ext = []
        for n in (1, 2, 3):
            for f in range(1 << (n * n)):
                R = [[(f >> (w * n + v)) & 1 for v in range(n)] for w in range(n)]
                ext.append((frame_valid(orc, code, f, n), {c: p(R, n) for c, p in CONDITIONS.items()}))
        if cond == "none":
            for c in CONDITIONS:
                assert any(v != conds[c] for v, conds in ext), (name, c)
        else:
            assert all(v == conds[cond] for v, conds in ext), name


def test_textbook_correspondences(orc):
    """Three standard correspondences beyond Table 9, on every frame with n <= 3:
    p -> []p holds exactly where R is contained in the identity, []([]p -> p) exactly where
    every world with a predecessor sees itself, <>p <-> []p exactly where every world has
    one successor."""
    def coreflexive(R, n):
        return all(not R[w][v] for w in range(n) for v in range(n) if w != v)

    def shift_reflexive(R, n):
        return all(R[v][v] for w in range(n) for v in range(n) if R[w][v])

    def functional(R, n):
        return all(sum(R[w]) == 1 for w in range(n))

    for text, cond in (("p -> []p", coreflexive), ("[]([]p -> p)", shift_reflexive),
                       ("(<>p -> []p) & ([]p -> <>p)", functional)):
        code = I.parse(text)
        for n in (1, 2, 3):
            for f in range(1 << (n * n)):
                R = [[(f >> (w * n + v)) & 1 for v in range(n)] for w in range(n)]
                assert frame_valid(orc, code, f, n) == cond(R, n), (text, n, f)


# ------------------------------------------------------------------ P2
def test_prop6_certificate(orc):
    g = dict(ln.split(":", 1) for ln in _golden_lines("prop6_certificate.txt"))
    phi, psi = I.alpha(2), I.alpha(3)
    assert I.to_text(phi) == "[]<>[]<>T"
    succ = [int(x) for x in g["succ"].split()]
    w = int(g["world"])
    assert succ == I.path_frame(6)
    assert orc.sat_at(phi, succ, 0, 0, w) == bool(int(g["phi_at_world"]))
    assert orc.sat_at(psi, succ, 0, 0, w) == bool(int(g["psi_at_world"]))
    assert orc.check_certificate(I.iff(phi, psi), succ, 0, 0, w, K)
    # the split search over a list holding only this frame finds world 0
    assert orc.split(phi, psi, [succ], 0) == w


def test_prop6_agreement_prefix(orc):
    """alpha_2 <-> alpha_3 has no countermodel on any frame with at most five worlds."""
    chi = I.iff(I.alpha(2), I.alpha(3))
    for n in range(1, 6):
        assert orc.census(chi, n, K, 0, threads=8)[0] == NONE, n
    # ... and has one at six worlds (the path)
    f = I.frame_index(I.path_frame(6))
    assert orc.census(chi, 6, K, 0, f, f + 1)[0] != NONE


# ------------------------------------------------------------------ P3
@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_lemma2_path_family(orc, m):
    """On a directed path, alpha_m is false exactly where the number r of remaining
    edges is odd and at most 2m-1."""
    for n in range(1, 14):
        truth = orc.truth_set(I.alpha(m), I.path_frame(n), 0, 0)
        for w in range(n):
            r = n - 1 - w
            assert truth[w] == (0 if (r % 2 == 1 and r <= 2 * m - 1) else 1), (m, n, w)


# ------------------------------------------------------------------ P4
def test_table4_separation_sizes(orc):
    for ln in _golden_lines("table4_separation.txt"):
        m, unsat_through, first_sat = (int(x) for x in ln.split())
        chi = I.iff(I.alpha(m), I.alpha(m + 1))
        for n in range(1, min(unsat_through, 5) + 1):
            assert orc.census(chi, n, K, 0, threads=8)[0] == NONE, (m, n)
        if first_sat <= 5:
            assert orc.census(chi, first_sat, K, 0, threads=8)[0] != NONE
        # Lemma 2's witness: the (2m+2)-world path separates at its root
        assert first_sat == 2 * m + 2
        assert orc.split(I.alpha(m), I.alpha(m + 1), [I.path_frame(first_sat)], 0) == 0


# ------------------------------------------------------------------ P5
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_dia_k_pigeonhole(orc, k):
    """DIA^k T and DIA^(k+1) T agree on every frame with at most k worlds (a walk of
    length k in <= k worlds revisits a world); on the m-world path the first
    disagreement is at world m-1-k.  Dually for BOX^k F."""
    for pair in ((I.dia_k_top(k), I.dia_k_top(k + 1)), (I.box_k_bot(k), I.box_k_bot(k + 1))):
        chi = I.iff(*pair)
        for n in range(1, k + 1):
            assert orc.census(chi, n, K, 0, threads=8)[0] == NONE
        for m in range(k + 1, 12):
            assert orc.split(pair[0], pair[1], [I.path_frame(m)], 0) == m - 1 - k


# ------------------------------------------------------------------ P9
def _prop_eval(code, assignment):
    st = []
    for op in code:
        if op == I.TOP:
            st.append(True)
        elif op == I.BOT:
            st.append(False)
        elif I.is_var(op):
            st.append(assignment[op - I.VAR0])
        elif op == I.NOT:
            st.append(not st.pop())
        else:
            b, a = st.pop(), st.pop()
            st.append({I.AND: a and b, I.OR: a or b, I.IMP: (not a) or b, I.IFF: a == b}[op])
    return st[0]


def test_propositional_reduction(orc):
    """A modal-free formula is world-local: its first countermodel is frame 0 at the least
    valuation whose per-world assignment falsifies the truth table, and its failure count is
    |frames| * (2^(kn) - (2^k - z)^n) with z falsifying assignments out of 2^k."""
    rng = I.SplitMix64(0xABCDEF, 7)
    for _ in range(40):
        k = 1 + rng.below(3)
        leaves = (I.TOP, I.BOT) + tuple(I.var(i) for i in range(k))
        code = I.gen_formula(rng, rng.uniform(1, 15), 0, leaves)
        code = [op for op in code]  # depth 0 -> no modal operators
        assert not any(op in (I.BOX, I.DIA) for op in code)
        falsifying = [a for a in itertools.product([False, True], repeat=k)
                      if not _prop_eval(code, list(a))]
        z = len(falsifying)
        for n in (1, 2, 3):
            key, cnt, _ = orc.census(code, n, K, k, threads=4)
            assert cnt == (2 ** (n * n)) * (2 ** (k * n) - (2 ** k - z) ** n)
            exp_key = NONE
            for val in range(1 << (k * n)):
                worlds = [w for w in range(n)
                          if not _prop_eval(code, [bool((val >> (i * n + w)) & 1) for i in range(k)])]
                if worlds:
                    exp_key = (val << 4) | worlds[0]
                    break
            assert key == exp_key


# ------------------------------------------------------------------ P11
def test_monotone_validity_over_classes(orc):
    """S5 within S4 within T within K: validity can only grow, refutation counts shrink."""
    for code in I.config1_formulas():
        for n in (1, 2, 3):
            res = [orc.census(code, n, c, 2, threads=4) for c in (K, T, S4, S5)]
            for a, b in zip(res, res[1:]):
                assert a[1] >= b[1]
                if a[0] == NONE:
                    assert b[0] == NONE


def test_isolated_world_extension(orc):
    """Adding an isolated world (reflexive in T/S4/S5) keeps every countermodel."""
    for code in I.config1_formulas()[:24]:
        for cls in (K, T, S4, S5):
            key, _, _ = orc.census(code, 2, cls, 2)
            if key == NONE:
                continue
            f, val, w = orc.decode_key(key, 2, 2)
            succ = I.frame_succ(f, 2) + [4 if cls != K else 0]
            # valuation bits are laid out per variable in blocks of n: re-spread for n = 3
            val3 = sum(((val >> (i * 2 + x)) & 1) << (i * 3 + x) for i in range(2) for x in range(2))
            assert orc.check_certificate(code, succ, 2, val3, w, cls)
            assert orc.census(code, 3, cls, 2, threads=4)[0] != NONE


def test_split_symmetric(orc):
    frames = I.frame_family(6, 64)
    fs = I.config1_formulas()
    for a, b in zip(fs[:16], fs[16:32]):
        assert orc.split(a, b, frames) == orc.split(b, a, frames)


def test_certificates_of_census_keys(orc):
    """Every first key the census reports decodes to a certificate the pointwise checker
    accepts (Proposition 3), and no earlier model of the same frame refutes the formula."""
    for code in I.config1_formulas():
        for cls in (K, T, S4, S5):
            key, _, _ = orc.census(code, 3, cls, 2, threads=4)
            if key == NONE:
                continue
            f, val, w = orc.decode_key(key, 3, 2)
            succ = I.frame_succ(f, 3)
            assert orc.check_certificate(code, succ, 2, val, w, cls)
            for v2 in range(val):
                assert all(orc.truth_set(code, succ, 2, v2))


def test_rejects_malformed(orc):
    with pytest.raises(ValueError):
        orc.census([I.AND], 2, K, 2)
    with pytest.raises(ValueError):
        orc.census([I.var(3)], 2, K, 2)
    with pytest.raises(ValueError):
        orc.census([I.TOP, I.TOP], 2, K, 2)
    with pytest.raises(ValueError):
        orc.census([99], 2, K, 2)
