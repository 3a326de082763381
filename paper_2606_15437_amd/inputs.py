"""Seeded synthetic inputs: formulas, frame families and corpora.

This module only *constructs* inputs.  It contains none of the semantics
(no satisfaction, no truth sets, no class tests): the census kernels and the
CPU oracle both receive what it produces as plain data (postfix bytecode and
successor-mask arrays), so neither side's arithmetic can leak into the other.

Formula language (Section 2 of the paper): TOP, BOT, variables p_i, NOT, AND,
OR, IMP, BOX, DIA.  IFF is not part of the object language; it is used only to
build the biconditional chi = phi <-> psi of Proposition 5.

Bytecode: postfix, one byte per node (so the byte length is the node count
|phi| of Section 2):

    0 TOP   1 BOT   2+i VAR p_i (i < 4)   6 NOT   7 AND   8 OR   9 IMP
    10 BOX  11 DIA  12 IFF

Randomness is SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based
generator: output j of a stream whose state starts at s is
mix(s + (j + 1) * GAMMA).
"""
from __future__ import annotations

import numpy as np

TOP, BOT, VAR0, NOT, AND, OR, IMP, BOX, DIA, IFF = 0, 1, 2, 6, 7, 8, 9, 10, 11, 12
MAX_VARS = 4
OP_NAMES = {TOP: "T", BOT: "F", NOT: "~", AND: "&", OR: "|", IMP: "->", BOX: "[]", DIA: "<>",
            IFF: "<->"}
UNARY = (NOT, BOX, DIA)
BINARY = (AND, OR, IMP, IFF)
VAR_NAMES = "pqrs"

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15

# Master seeds of the five workload configurations.
SEED_C1 = 0x4B52495000000001
SEED_C2 = 0x4B52495000000002
SEED_C3 = 0x4B52495000000003
SEED_C4 = 0x4B52495000000004
SEED_C5_TEST = 0x4B52495000000005
SEED_C5_TRAIN = 0x4B52495000000006


# ---------------------------------------------------------------- SplitMix64
def mix64(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


class SplitMix64:
    """Sequential SplitMix64 stream; stream s of master seed S starts at S ^ (s << 32)."""

    def __init__(self, seed: int, stream: int = 0):
        self.state = (seed ^ (stream << 32)) & MASK64

    def next(self) -> int:
        self.state = (self.state + GAMMA) & MASK64
        return mix64(self.state)

    def below(self, r: int) -> int:
        """Uniform integer in [0, r) by the multiply-high map (x * r) >> 64."""
        return (self.next() * r) >> 64

    def uniform(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + self.below(hi - lo + 1)


def mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def below_np(x: np.ndarray, r: int) -> np.ndarray:
    """(x * r) >> 64 for uint64 x and 0 < r < 2**31, without 128-bit integers."""
    x = x.astype(np.uint64)
    hi = x >> np.uint64(32)
    lo = x & np.uint64(0xFFFFFFFF)
    r64 = np.uint64(r)
    with np.errstate(over="ignore"):
        return ((hi * r64) + ((lo * r64) >> np.uint64(32))) >> np.uint64(32)


# ---------------------------------------------------------- formula tooling
def var(i: int) -> int:
    return VAR0 + i


def is_var(op: int) -> bool:
    return VAR0 <= op < VAR0 + MAX_VARS


def gen_formula(rng: SplitMix64, length: int, depth: int, leaves) -> list[int]:
    """Random formula with exactly `length` nodes and modal depth <= `depth`.

    length 1: a uniform leaf.  length 2: a unary operator (NOT, or BOX/DIA when
    depth >= 1) over a leaf.  Otherwise, with probability 1/2 a unary operator
    over a (length-1)-node child (modal operators consume one unit of depth),
    else a uniform binary connective among AND/OR/IMP with a left part of
    uniform size in [1, length-2].
    """
    leaves = list(leaves)
    out: list[int] = []

    def rec(L: int, D: int) -> None:
        if L == 1:
            out.append(leaves[rng.below(len(leaves))])
            return
        if L == 2 or rng.below(2) == 0:
            ops = [NOT] + ([BOX, DIA] if D >= 1 else [])
            op = ops[rng.below(len(ops))]
            rec(L - 1, D - (1 if op in (BOX, DIA) else 0))
            out.append(op)
            return
        op = (AND, OR, IMP)[rng.below(3)]
        left = 1 + rng.below(L - 2)
        rec(left, D)
        rec(L - 1 - left, D)
        out.append(op)

    rec(length, depth)
    return out


def formula_batch(seed: int, count: int, len_range, depth_range, leaves, stream: int = 0):
    """`count` formulas; per formula L ~ U[len_range], depth cap D ~ U[depth_range]."""
    rng = SplitMix64(seed, stream)
    out = []
    for _ in range(count):
        L = rng.uniform(*len_range)
        D = rng.uniform(*depth_range)
        out.append(gen_formula(rng, L, D, leaves))
    return out


def pack(formulas) -> tuple[np.ndarray, np.ndarray]:
    """CSR packing: (code uint8[sum len], offsets uint32[B+1])."""
    offs = np.zeros(len(formulas) + 1, dtype=np.uint32)
    for i, f in enumerate(formulas):
        offs[i + 1] = offs[i] + len(f)
    code = np.zeros(int(offs[-1]), dtype=np.uint8)
    for i, f in enumerate(formulas):
        code[offs[i]:offs[i + 1]] = np.asarray(f, dtype=np.uint8)
    return code, offs


def unpack(code, offsets) -> list[list[int]]:
    return [list(map(int, code[offsets[i]:offsets[i + 1]])) for i in range(len(offsets) - 1)]


def modal_depth(f) -> int:
    st = []
    for op in f:
        if op in (TOP, BOT) or is_var(op):
            st.append(0)
        elif op == NOT:
            st.append(st.pop())
        elif op in (BOX, DIA):
            st.append(st.pop() + 1)
        else:
            b, a = st.pop(), st.pop()
            st.append(max(a, b))
    assert len(st) == 1
    return st[0]


def formula_stats(f, n: int) -> dict:
    """Syntactic counts; `bitops` is the per-evaluation work of Proposition 2 in
    bit operations: n per Boolean connective, n*n per modal operator."""
    n_bool = sum(1 for op in f if op in (NOT, AND, OR, IMP, IFF))
    n_modal = sum(1 for op in f if op in (BOX, DIA))
    return {"length": len(f), "depth": modal_depth(f), "bool": n_bool, "modal": n_modal,
            "bitops": n * n_bool + n * n * n_modal}


def to_text(f) -> str:
    st: list[str] = []
    for op in f:
        if op == TOP:
            st.append("T")
        elif op == BOT:
            st.append("F")
        elif is_var(op):
            st.append(VAR_NAMES[op - VAR0])
        elif op == NOT:
            st.append("~" + st.pop())
        elif op == BOX:
            st.append("[]" + st.pop())
        elif op == DIA:
            st.append("<>" + st.pop())
        else:
            b, a = st.pop(), st.pop()
            st.append("(" + a + " " + OP_NAMES[op] + " " + b + ")")
    assert len(st) == 1, "malformed bytecode"
    return st[0]


def parse(text: str) -> list[int]:
    """Text to postfix bytecode.  Grammar, loosest first: <-> , -> (right
    associative), |, &, then prefix ~ [] <> and atoms T F p q r s ( )."""
    toks = []
    i = 0
    while i < len(text):
        c = text[i]
        if c.isspace():
            i += 1
        elif text.startswith("<->", i):
            toks.append("<->"); i += 3
        elif text.startswith("->", i):
            toks.append("->"); i += 2
        elif text.startswith("[]", i):
            toks.append("[]"); i += 2
        elif text.startswith("<>", i):
            toks.append("<>"); i += 2
        elif c in "~&|()TFpqrs":
            toks.append(c); i += 1
        else:
            raise ValueError(f"bad character {c!r} in {text!r}")
    pos = 0
    out: list[int] = []

    def peek():
        return toks[pos] if pos < len(toks) else None

    def take(t=None):
        nonlocal pos
        tok = toks[pos]
        if t is not None and tok != t:
            raise ValueError(f"expected {t} got {tok}")
        pos += 1
        return tok

    def p_iff():
        p_imp()
        while peek() == "<->":
            take(); p_imp(); out.append(IFF)

    def p_imp():
        p_or()
        if peek() == "->":
            take(); p_imp(); out.append(IMP)

    def p_or():
        p_and()
        while peek() == "|":
            take(); p_and(); out.append(OR)

    def p_and():
        p_un()
        while peek() == "&":
            take(); p_un(); out.append(AND)

    def p_un():
        t = peek()
        if t == "~":
            take(); p_un(); out.append(NOT)
        elif t == "[]":
            take(); p_un(); out.append(BOX)
        elif t == "<>":
            take(); p_un(); out.append(DIA)
        elif t == "(":
            take(); p_iff(); take(")")
        elif t == "T":
            take(); out.append(TOP)
        elif t == "F":
            take(); out.append(BOT)
        elif t is not None and t in VAR_NAMES:
            take(); out.append(VAR0 + VAR_NAMES.index(t))
        else:
            raise ValueError(f"unexpected token {t!r} in {text!r}")

    p_iff()
    if pos != len(toks):
        raise ValueError(f"trailing tokens in {text!r}")
    return out


def iff(phi, psi) -> list[int]:
    """Postfix bytecode of the biconditional phi <-> psi (Proposition 5)."""
    return list(phi) + list(psi) + [IFF]


def _root_children(f):
    """Postfix spans of the root's operands: [] for a leaf, [a] or [a, b]."""
    op = f[-1]
    if op in (NOT, BOX, DIA):
        return [list(f[:-1])]
    if op in (AND, OR, IMP, IFF):
        right = _span_start(f, len(f) - 2)
        return [list(f[:right]), list(f[right:-1])]
    return []


def _span_start(f, end):
    """Start index of the subformula whose last token is f[end]."""
    need = 1
    k = end
    while True:
        op = f[k]
        if op in (AND, OR, IMP, IFF):
            need += 1
        elif op in (NOT, BOX, DIA):
            pass
        else:
            need -= 1
        if need == 0:
            return k
        k -= 1


def equivalent_variant(f, k: int) -> list[int]:
    """A formula with the same truth set as f on every model, by one syntactic rewrite
    chosen by k mod 4: double negation; swapped operands of a commutative root (else
    double negation); modal duality at a modal root (BOX a as NOT DIA NOT a, DIA a as
    NOT BOX NOT a; else double negation); conjunction with TOP."""
    f = list(f)
    r = k % 4
    if r == 1 and f[-1] in (AND, OR, IFF):
        a, b = _root_children(f)
        return b + a + [f[-1]]
    if r == 2 and f[-1] in (BOX, DIA):
        (a,) = _root_children(f)
        return a + [NOT, DIA if f[-1] == BOX else BOX, NOT]
    if r == 3:
        return f + [TOP, AND]
    return f + [NOT, NOT]


def alpha(m: int) -> list[int]:
    """alpha_m = (BOX DIA)^m TOP (Proposition 6, Lemma 2)."""
    return [TOP] + [DIA, BOX] * m


def alpha_dual(m: int) -> list[int]:
    """(DIA BOX)^m BOT, the dual family."""
    return [BOT] + [BOX, DIA] * m


def dia_k_top(k: int) -> list[int]:
    return [TOP] + [DIA] * k


def box_k_bot(k: int) -> list[int]:
    return [BOT] + [BOX] * k


# ------------------------------------------------------------ configurations
LEAVES_2 = (TOP, BOT, var(0), var(1))
LEAVES_3 = (TOP, BOT, var(0), var(1), var(2))


def config1_formulas():
    """64 formulas over {p,q,T,F}, L ~ U[1,12], depth cap ~ U[0,3] (n = 1..3, K, 2 vars)."""
    return formula_batch(SEED_C1, 64, (1, 12), (0, 3), LEAVES_2)


def config2_formulas():
    """1,024 formulas over {p,q,r,T,F}, L ~ U[3,24], depth cap ~ U[0,4] (n = 4, 3 vars)."""
    return formula_batch(SEED_C2, 1024, (3, 24), (0, 4), LEAVES_3)


def config3_formulas(count: int = 4096):
    """4,096 formulas over {p,q,T,F}, L ~ U[3,40], depth cap ~ U[0,6] (n = 5, 2 vars)."""
    return formula_batch(SEED_C3, count, (3, 40), (0, 6), LEAVES_2)


# The matched single-formula workload of the paper's Table 1.
TABLE1_FORMULA = "[](p -> q) -> (<>p -> <>q)"
TABLE1_FRAMES = 262144


# ------------------------------------------------------------ frame families
FAMILY_PATH, FAMILY_CYCLE, FAMILY_TREE, FAMILY_ER = 0, 1, 2, 3


def family_kind(k: np.ndarray) -> np.ndarray:
    """Kind of frame k in a family: 0 canonical path, 1 canonical cycle, then by
    k mod 8: 0 relabelled path, 1 relabelled cycle, 2-3 random recursive
    out-tree, 4-7 Erdos-Renyi with edge probability 0.2 over all n*n ordered
    pairs (loops included)."""
    k = np.asarray(k, dtype=np.int64)
    r = k % 8
    kind = np.where(r == 0, FAMILY_PATH, np.where(r == 1, FAMILY_CYCLE,
                    np.where(r < 4, FAMILY_TREE, FAMILY_ER)))
    kind = np.where(k == 0, FAMILY_PATH, kind)
    kind = np.where(k == 1, FAMILY_CYCLE, kind)
    return kind


def frame_family(n: int, count: int, start: int = 0, seed: int = SEED_C4) -> np.ndarray:
    """Frames start .. start+count-1 of the seeded family on n worlds, as
    uint32[count][n] successor masks.  Frame k draws from its own SplitMix64
    stream (state base + 64*k*GAMMA), so any frame is addressable directly."""
    assert 1 <= n <= 16
    k = np.arange(start, start + count, dtype=np.int64)
    base = mix64(seed ^ (n << 48))
    with np.errstate(over="ignore"):
        st0 = np.uint64(base) + k.astype(np.uint64) * np.uint64((64 * GAMMA) & MASK64)

    def draw(j: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            return mix64_np(st0 + np.uint64(((j + 1) * GAMMA) & MASK64))

    kind = family_kind(k)
    succ = np.zeros((count, n), dtype=np.uint32)
    rows = np.arange(count)
    # random relabelling (Fisher-Yates over draws 0..n-2), identity for k < 2
    perm = np.tile(np.arange(n, dtype=np.int64), (count, 1))
    for i in range(n - 1, 0, -1):
        j = below_np(draw(n - 1 - i), i + 1).astype(np.int64)
        j = np.where(k < 2, i, j)
        a = perm[rows, i].copy()
        perm[rows, i] = perm[rows, j]
        perm[rows, j] = a
    one = np.uint32(1)
    is_path = kind == FAMILY_PATH
    is_cycle = kind == FAMILY_CYCLE
    for i in range(n - 1):
        m = is_path | is_cycle
        src, dst = perm[m, i], perm[m, i + 1]
        succ[np.nonzero(m)[0], src] |= (one << dst.astype(np.uint32))
    if n >= 1:
        idx = np.nonzero(is_cycle)[0]
        src, dst = perm[idx, n - 1], perm[idx, 0]
        succ[idx, src] |= (one << dst.astype(np.uint32))
    is_tree = kind == FAMILY_TREE
    idx = np.nonzero(is_tree)[0]
    for i in range(1, n):
        parent = below_np(draw(n + i - 1), i).astype(np.int64)[idx]
        src, dst = perm[idx, parent], perm[idx, i]
        succ[idx, src] |= (one << dst.astype(np.uint32))
    is_er = kind == FAMILY_ER
    idx = np.nonzero(is_er)[0]
    for u in range(n):
        for v in range(n):
            hit = below_np(draw(u * n + v), 5)[idx] == 0
            succ[idx[hit], u] |= np.uint32(1 << v)
    return succ


# ------------------------------------------------- adversarial frame generators
SEED_ADV = 0x4B52495000000007
ADVERSARIAL = ("erdos-renyi", "edge-flip", "scc-bottleneck", "dead-end", "back-edge",
               "permuted-bottleneck")


def adversarial_frames(generator: str, n: int, count: int, start: int = 0,
                       seed: int = SEED_ADV) -> np.ndarray:
    """Frames start .. start+count-1 of one adversarial generator on n worlds (the
    generator families of Section 7's adversarial frame synthesis), as uint32[count][n]
    successor masks, each frame from its own counter-based SplitMix64 stream:
      erdos-renyi          each ordered pair (loops included) with probability
                           (1 + k mod 8) / 20, stratified over k;
      edge-flip            a canonical seed (k mod 4: path, cycle, reverse path, star from
                           world 0) with 1 + k mod 3 uniformly chosen pairs flipped;
      scc-bottleneck       worlds cut into 2 + k mod 3 consecutive blocks, each a cycle
                           with one random chord, block i linked to block i+1 by one edge;
      dead-end             a random out-tree plus random back edges, then 1 + k mod 3
                           worlds emptied;
      back-edge            the path 0 -> ... -> n-1 plus 1 + k mod 4 edges (i, j), j < i;
      permuted-bottleneck  scc-bottleneck with the world labels permuted."""
    assert 1 <= n <= 16 and generator in ADVERSARIAL
    g = ADVERSARIAL.index(generator)
    k = np.arange(start, start + count, dtype=np.int64)
    base = mix64(seed ^ (n << 48) ^ (g << 40))
    with np.errstate(over="ignore"):
        st0 = np.uint64(base) + k.astype(np.uint64) * np.uint64((512 * GAMMA) & MASK64)

    def draw(j: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            return mix64_np(st0 + np.uint64(((j + 1) * GAMMA) & MASK64))

    rows = np.arange(count)
    succ = np.zeros((count, n), dtype=np.uint32)
    one = np.uint32(1)

    def add(mask, src, dst):
        idx = np.nonzero(mask)[0]
        np.bitwise_or.at(succ, (idx, src[idx]), (one << dst[idx].astype(np.uint32)))

    def flip(mask, src, dst):
        idx = np.nonzero(mask)[0]
        np.bitwise_xor.at(succ, (idx, src[idx]), (one << dst[idx].astype(np.uint32)))

    def bottleneck():
        nb = 2 + (k % 3)
        for b in range(2, 5):
            m = nb == b
            size = n // b
            for blk in range(b):
                lo = blk * size
                hi = n if blk == b - 1 else lo + size
                ln = hi - lo
                for i in range(lo, hi):  # a cycle through the block
                    add(m, np.full(count, i), np.full(count, lo + (i - lo + 1) % ln))
                c1 = lo + below_np(draw(8 * blk), ln).astype(np.int64)
                c2 = lo + below_np(draw(8 * blk + 1), ln).astype(np.int64)
                add(m, c1, c2)
                if blk + 1 < b:
                    nlo = hi
                    nhi = n if blk + 1 == b - 1 else nlo + size
                    s_ = lo + below_np(draw(8 * blk + 2), ln).astype(np.int64)
                    d_ = nlo + below_np(draw(8 * blk + 3), nhi - nlo).astype(np.int64)
                    add(m, s_, d_)

    if generator == "erdos-renyi":
        thr = (1 + (k % 8)).astype(np.uint64)
        for u in range(n):
            for v in range(n):
                hit = below_np(draw(u * n + v), 20) < thr
                add(hit, np.full(count, u), np.full(count, v))
    elif generator == "edge-flip":
        kind = k % 4
        for i in range(n - 1):
            add(kind == 0, np.full(count, i), np.full(count, i + 1))
            add(kind == 2, np.full(count, i + 1), np.full(count, i))
        for i in range(n):
            add(kind == 1, np.full(count, i), np.full(count, (i + 1) % n))
            if i > 0:
                add(kind == 3, np.full(count, 0), np.full(count, i))
        nflip = 1 + (k % 3)
        for t in range(3):
            u = below_np(draw(2 * t), n).astype(np.int64)
            v = below_np(draw(2 * t + 1), n).astype(np.int64)
            flip(nflip > t, u, v)
    elif generator in ("scc-bottleneck", "permuted-bottleneck"):
        bottleneck()
    elif generator == "dead-end":
        for i in range(1, n):
            parent = below_np(draw(i), i).astype(np.int64)
            add(np.ones(count, bool), parent, np.full(count, i))
        for t in range(3):
            u = below_np(draw(100 + 2 * t), n).astype(np.int64)
            v = below_np(draw(101 + 2 * t), n).astype(np.int64)
            add(v <= u, u, v)
        ndead = 1 + (k % 3)
        for t in range(3):
            w = below_np(draw(200 + t), n).astype(np.int64)
            idx = np.nonzero(ndead > t)[0]
            succ[idx, w[idx]] = 0
    else:  # back-edge
        for i in range(n - 1):
            add(np.ones(count, bool), np.full(count, i), np.full(count, i + 1))
        nback = 1 + (k % 4)
        for t in range(4):
            i = 1 + below_np(draw(2 * t), max(n - 1, 1)).astype(np.int64)
            j = below_np(draw(2 * t + 1), n).astype(np.int64) % np.maximum(i, 1)
            add((nback > t) & (i < n), np.minimum(i, n - 1), j)
    if generator == "permuted-bottleneck":
        perm = np.tile(np.arange(n, dtype=np.int64), (count, 1))
        for i in range(n - 1, 0, -1):
            j = below_np(draw(300 + i), i + 1).astype(np.int64)
            a = perm[rows, i].copy()
            perm[rows, i] = perm[rows, j]
            perm[rows, j] = a
        out = np.zeros_like(succ)
        for u in range(n):
            for v in range(n):
                bit = (succ[:, u] >> np.uint32(v)) & one
                np.bitwise_or.at(out, (rows, perm[:, u]), bit << perm[:, v].astype(np.uint32))
        succ = out
    return succ


def path_frame(n: int) -> list[int]:
    """Directed path 0 -> 1 -> ... -> n-1 as successor masks."""
    return [(1 << (w + 1)) if w + 1 < n else 0 for w in range(n)]


def frame_index(succ) -> int:
    """Row-major labelled frame index: bit (w*n + v) set iff R(w, v)."""
    n = len(succ)
    f = 0
    for w in range(n):
        f |= (int(succ[w]) & ((1 << n) - 1)) << (w * n)
    return f


def frame_succ(f: int, n: int) -> list[int]:
    return [(f >> (w * n)) & ((1 << n) - 1) for w in range(n)]


# --------------------------------------------------- five-world census corpus
def enumerate_formulas(max_nodes: int = 7, leaves=(VAR0, VAR0 + 1)) -> list[list[int]]:
    """Every formula tree with at most max_nodes nodes over the given leaves, the unary
    connectives NOT, BOX, DIA and the binary AND, OR, IMP (constant-free by default),
    in size order; within one size: unary roots (NOT, BOX, DIA, each over the smaller
    trees in order), then binary roots (AND, OR, IMP; left operand size ascending,
    then left tree, then right tree).  For seven nodes over two variables this is the
    paper's raw census enumeration (Section 6)."""
    by_size = {1: [[x] for x in leaves]}
    for size in range(2, max_nodes + 1):
        out = []
        for op in (NOT, BOX, DIA):
            out += [t + [op] for t in by_size[size - 1]]
        for op in (AND, OR, IMP):
            for a in range(1, size - 1):
                for left in by_size[a]:
                    for right in by_size[size - 1 - a]:
                        out.append(left + right + [op])
        by_size[size] = out
    return [f for size in range(1, max_nodes + 1) for f in by_size[size]]


def named_axioms() -> list[list[int]]:
    """The named axioms added to the census corpus: K (normality), T and McKinsey
    (the named control of Section 10's correspondence table)."""
    return [parse("[](p -> q) -> ([]p -> []q)"), parse("[]p -> p"), parse("[]<>p -> <>[]p")]


def all_pointed_models(max_n: int = 3, nvars: int = 2) -> np.ndarray:
    """Every pointed model with at most max_n worlds, packed as for signatures
    (n << 60 | frame << 24 | valuation << 4 | world), in aligned groups of 64 with one
    n; a group that the models of one n do not fill repeats that n's models."""
    out = []
    for n in range(1, max_n + 1):
        ms = [(n << 60) | (f << 24) | (v << 4) | w for f in range(1 << (n * n))
              for v in range(1 << (nvars * n)) for w in range(n)]
        pad = (-len(ms)) % 64
        out += ms + [ms[i % len(ms)] for i in range(pad)]
    return np.array(out, dtype=np.uint64)


# ---------------------------------------------------------------- C4 pairs
def config4_pool(count: int = 200_000) -> list[list[int]]:
    """The split workload's formula pool: random 2-variable formulas, L ~ U[3,15],
    D ~ U[0,6]."""
    return formula_batch(SEED_C4, count, (3, 15), (0, 6), LEAVES_2, stream=1)


def config4_designed_pairs() -> list[tuple[list[int], list[int]]]:
    """Pairs with known late separations (Proposition 6, Lemma 2, Table 4 and the
    pigeonhole facts): (alpha_j, alpha_k) for 2 <= j < k <= 6 and their duals, then
    DIA^k TOP / DIA^(k+1) TOP and BOX^k BOT / BOX^(k+1) BOT for k = 4..7."""
    out = []
    for j in range(2, 7):
        for k in range(j + 1, 7):
            out.append((alpha(j), alpha(k)))
    for j in range(2, 7):
        for k in range(j + 1, 7):
            out.append((alpha_dual(j), alpha_dual(k)))
    for k in range(4, 8):
        out.append((dia_k_top(k), dia_k_top(k + 1)))
    for k in range(4, 8):
        out.append((box_k_bot(k), box_k_bot(k + 1)))
    return out


# --------------------------------------------------------------- C5 corpus
def modal_word_corpus(seed: int, count: int) -> list[list[int]]:
    """Modal words over {BOX, DIA, NOT} of length 0..10 on bases {p, q, T, F},
    starting with the designed families (BOX DIA)^k T, (DIA BOX)^k F,
    DIA^k T, BOX^k F for k <= 10; syntactic duplicates are dropped."""
    out: list[list[int]] = []
    seen = set()

    def add(f):
        t = tuple(f)
        if t not in seen:
            seen.add(t)
            out.append(list(f))

    for kk in range(0, 6):
        add(alpha(kk))
        add(alpha_dual(kk))
    for kk in range(0, 11):
        add(dia_k_top(kk))
        add(box_k_bot(kk))
    rng = SplitMix64(seed, 1)
    bases = (var(0), var(1), TOP, BOT)
    while len(out) < count:
        L = rng.below(11)
        f = [bases[rng.below(4)]]
        for _ in range(L):
            f.append((BOX, DIA, NOT)[rng.below(3)])
        add(f)
    return out[:count]


def retrieval_corpus(seed: int, count: int = 10000, n_words: int = 2000, max_len: int = 21):
    """The learned-proposal corpus: modal words, then Boolean compositions
    (AND/OR/IMP) of two earlier formulas with total size <= max_len."""
    out = modal_word_corpus(seed, n_words)
    seen = set(tuple(f) for f in out)
    rng = SplitMix64(seed, 2)
    while len(out) < count:
        i = rng.below(len(out))
        j = rng.below(len(out))
        if len(out[i]) + len(out[j]) + 1 > max_len:
            continue
        op = (AND, OR, IMP)[rng.below(3)]
        f = out[i] + out[j] + [op]
        t = tuple(f)
        if t in seen:
            continue
        seen.add(t)
        out.append(f)
    return out


# ------------------------------------------------------- signature samples
def signature_samples(seed: int = SEED_C5_TEST, n3: int = 3520) -> np.ndarray:
    """4,096 pointed models (n, frame, valuation, world) over 2 variables, packed
    n << 60 | frame << 24 | val << 4 | world, in aligned groups of 64 with one n:
    n3 distinct three-world models drawn without replacement (seeded), all 512
    two-world models, and the 8 one-world models each repeated 8 times."""
    assert n3 % 64 == 0 and n3 + 512 + 64 == 4096
    rng = SplitMix64(seed, 3)
    universe = 512 * 64 * 3  # three-world (frame, valuation, world) triples
    chosen: set[int] = set()
    order: list[int] = []
    while len(order) < n3:
        x = rng.below(universe)
        if x not in chosen:
            chosen.add(x)
            order.append(x)

    def pack1(n, f, v, w):
        return (n << 60) | (f << 24) | (v << 4) | w

    out = [pack1(3, x // 192, (x // 3) % 64, x % 3) for x in order]
    out += [pack1(2, f, v, w) for f in range(16) for v in range(16) for w in range(2)]
    one = [pack1(1, f, v, 0) for f in range(2) for v in range(4)]
    out += [one[i % 8] for i in range(64)]
    return np.array(out, dtype=np.uint64)
