"""Frame-correspondence recovery (Section 10): for each formula, the set of frames with
at most N worlds on which it is valid, Val_N(phi), is compared with the extensions
Ext_N(X) of the first-order frame conditions X of a fixed library; X is recovered
for phi when the two sets are equal.

Val for n <= 3 comes from exact truth tables over every pointed model with at most
three worlds (the signature kernel), for n = 4 and 5 from the census kernel's
frame-validity maps.  The library is evaluated on the host over frame indices (bit
w*n + v of a frame index is R(w, v)).
"""
from __future__ import annotations

import itertools

import numpy as np

from . import inputs as I
from . import kripke as K


# ------------------------------------------------------------ the library
def _bits(frames: np.ndarray, n: int):
    """R(w, v) as boolean arrays over the given frame indices (each computed once)."""
    cache = {}

    def b(w, v):
        if (w, v) not in cache:
            cache[(w, v)] = ((frames >> np.uint64(w * n + v)) & np.uint64(1)).astype(bool)
        return cache[(w, v)]
    return b


def _all(terms, shape):
    out = np.ones(shape, dtype=bool)
    for t in terms:
        out &= t
    return out


def _any(terms, shape):
    out = np.zeros(shape, dtype=bool)
    for t in terms:
        out |= t
    return out


def base_conditions():
    """name -> predicate(b, n, shape) over frames, each a first-order condition on R."""
    W = range
    return {
        "reflexive": lambda b, n, s: _all((b(w, w) for w in W(n)), s),
        "irreflexive": lambda b, n, s: _all((~b(w, w) for w in W(n)), s),
        "serial": lambda b, n, s: _all((_any((b(w, v) for v in W(n)), s) for w in W(n)), s),
        "transitive": lambda b, n, s: _all((~b(w, v) | ~b(v, u) | b(w, u)
                                            for w in W(n) for v in W(n) for u in W(n)), s),
        "symmetric": lambda b, n, s: _all((~b(w, v) | b(v, w) for w in W(n) for v in W(n)), s),
        "euclidean": lambda b, n, s: _all((~b(w, v) | ~b(w, u) | b(v, u)
                                           for w in W(n) for v in W(n) for u in W(n)), s),
        "partially functional": lambda b, n, s: _all((~b(w, v) | ~b(w, u) for w in W(n)
                                                      for v in W(n) for u in W(n) if v < u), s),
        "functional": lambda b, n, s: (
            _all((_any((b(w, v) for v in W(n)), s) for w in W(n)), s)
            & _all((~b(w, v) | ~b(w, u) for w in W(n) for v in W(n) for u in W(n) if v < u), s)),
        "dense": lambda b, n, s: _all((~b(w, v) | _any((b(w, u) & b(u, v) for u in W(n)), s)
                                       for w in W(n) for v in W(n)), s),
        "directed": lambda b, n, s: _all((~b(w, v) | ~b(w, u) |
                                          _any((b(v, x) & b(u, x) for x in W(n)), s)
                                          for w in W(n) for v in W(n) for u in W(n) if v <= u), s),
        "antisymmetric": lambda b, n, s: _all((~b(w, v) | ~b(v, w) for w in W(n) for v in W(n)
                                               if w < v), s),
        "asymmetric": lambda b, n, s: _all((~b(w, v) | ~b(v, w) for w in W(n) for v in W(n)), s),
        "shift reflexive": lambda b, n, s: _all((~b(w, v) | b(v, v) for w in W(n) for v in W(n)), s),
        "connected": lambda b, n, s: _all((~b(w, v) | ~b(w, u) | b(v, u) | b(u, v)
                                           for w in W(n) for v in W(n) for u in W(n) if v < u), s),
        "empty": lambda b, n, s: _all((~b(w, v) for w in W(n) for v in W(n)), s),
        "universal": lambda b, n, s: _all((b(w, v) for w in W(n) for v in W(n)), s),
        "coreflexive": lambda b, n, s: _all((~b(w, v) for w in W(n) for v in W(n) if w != v), s),
    }


# The 16 base conditions of our own library (coreflexive frames are the conjunction
# symmetric & antisymmetric there).
LIBRARY_BASE = ("reflexive", "irreflexive", "serial", "transitive", "symmetric", "euclidean",
                "partially functional", "functional", "dense", "directed", "antisymmetric",
                "asymmetric", "shift reflexive", "connected", "empty", "universal")


def library():
    """The base conditions and every conjunction of two of them."""
    all_base = base_conditions()
    base = {name: all_base[name] for name in LIBRARY_BASE}
    lib = dict(base)
    for (a, fa), (c, fc) in itertools.combinations(base.items(), 2):
        lib[f"{a} & {c}"] = (lambda fa, fc: lambda b, n, s: fa(b, n, s) & fc(b, n, s))(fa, fc)
    return lib


# The conditions of the paper's correspondence table (Section 10, Table 9), in its order.
TABLE9_CONDITIONS = ("reflexive", "serial", "transitive", "euclidean", "symmetric",
                     "partially functional", "dense", "directed")


def table9_library():
    """Only the eight first-order conditions Table 9 names."""
    base = base_conditions()
    return {name: base[name] for name in TABLE9_CONDITIONS}


# Conditions beyond Table 9 whose one-variable modal definitions are standard: coreflexive
# (p -> []p), shift reflexive ([]([]p -> p)) and functional (<>p <-> []p).
TEXTBOOK_EXTRA = ("coreflexive", "shift reflexive", "functional")


def textbook_library():
    """Table 9's eight conditions and the three of TEXTBOOK_EXTRA."""
    base = base_conditions()
    return {name: base[name] for name in TABLE9_CONDITIONS + TEXTBOOK_EXTRA}


def extensions(names, max_n=4, chunk=1 << 20, lib=None):
    """name -> boolean array over all frames with n = 1..max_n worlds (concatenated in
    order of n, then frame index)."""
    lib = library() if lib is None else lib
    out = {name: [] for name in names}
    for n in range(1, max_n + 1):
        total = 1 << (n * n)
        for start in range(0, total, chunk):
            frames = np.arange(start, min(total, start + chunk), dtype=np.uint64)
            b = _bits(frames, n)
            for name in names:
                out[name].append(lib[name](b, n, frames.shape))
    return {name: np.concatenate(v) for name, v in out.items()}


# ------------------------------------------------------------ validity maps
def validity(formulas, max_n=4, chunk=512):
    """bool[len(formulas)][frames with n = 1..max_n]: formula valid on the frame."""
    import torch
    samples = I.all_pointed_models(3, 2)
    offsets = {1: 0, 2: 64, 3: 64 + 512}  # sample index of the first model of each n
    parts = []
    for s0 in range(0, len(formulas), chunk):
        sub = formulas[s0:s0 + chunk]
        code, offs = I.pack(sub)
        d = torch.zeros((len(sub), len(samples) // 64), dtype=torch.int64, device="cuda")
        K.kripke_signatures(code, offs, 2, samples, d)
        bits = np.unpackbits(K.as_u64(d).view(np.uint8), axis=1, bitorder="little").astype(bool)
        cols = []
        for n in range(1, min(3, max_n) + 1):
            per = (1 << (2 * n)) * n  # (valuation, world) models per frame
            blk = bits[:, offsets[n]:offsets[n] + (1 << (n * n)) * per]
            cols.append(blk.reshape(len(sub), 1 << (n * n), per).all(axis=2))
        for n in range(4, max_n + 1):
            words = ((1 << (n * n)) + 31) // 32
            dv = torch.zeros((len(sub), words), dtype=torch.int32, device="cuda")
            K.kripke_frame_validity(code, offs, n, 2, dv)
            v = np.unpackbits(dv.cpu().numpy().view(np.uint8), axis=1, bitorder="little")
            cols.append(v[:, :1 << (n * n)].astype(bool))
        parts.append(np.concatenate(cols, axis=1))
    return np.concatenate(parts, axis=0)


def recover(formulas, max_n=4, log=None, lib=None):
    """Per formula: 'trivial' (valid on all or no frames), the recovered condition
    names, or [] (no match in the library; `lib` defaults to library())."""
    lib = library() if lib is None else lib
    val = validity(formulas, max_n)
    names = list(lib)
    ext = extensions(names, max_n, lib=lib)
    table = {}
    for name in names:
        table.setdefault(np.packbits(ext[name]).tobytes(), []).append(name)
    out = []
    for row in val:
        if row.all() or not row.any():
            out.append("trivial")
        else:
            out.append(table.get(np.packbits(row).tobytes(), []))
    if log:
        rec = sum(1 for o in out if isinstance(o, list) and o)
        triv = sum(1 for o in out if o == "trivial")
        log(f"correspondence over n <= {max_n}: {rec} recovered, {triv} trivial, "
            f"{len(out) - rec - triv} unmatched")
    return out


def table9():
    """The axioms of the paper's correspondence table (Section 10)."""
    rows = [("T", "[]p -> p"), ("D", "[]p -> <>p"), ("4", "[]p -> [][]p"),
            ("5", "<>p -> []<>p"), ("B", "p -> []<>p"), ("CD", "<>p -> []p"),
            ("C4", "[][]p -> []p"), ("G", "<>[]p -> []<>p"), ("M", "[]<>p -> <>[]p")]
    return [(name, I.parse(text)) for name, text in rows]


def condition_maps(names, n=5, chunk=1 << 20):
    """name -> Ext_n(X) over every frame index on n worlds as a packed bitmap (bit f % 32
    of word f / 32, the layout of the validity maps); a conjunction "a & b" is the AND of
    its parts' maps, each base condition is evaluated once."""
    base = base_conditions()
    parts = {name: name.split(" & ") for name in names}
    need = sorted({p for ps in parts.values() for p in ps})
    total = 1 << (n * n)
    words = (total + 31) // 32
    out = {b: np.zeros(words, dtype=np.uint32) for b in need}
    for start in range(0, total, chunk):
        frames = np.arange(start, min(total, start + chunk), dtype=np.uint64)
        bits = _bits(frames, n)
        for b in need:
            v = base[b](bits, n, frames.shape)
            packed = np.packbits(v, bitorder="little")
            packed = np.pad(packed, (0, (-len(packed)) % 4))
            out[b][start // 32:start // 32 + len(packed) // 4] = packed.view(np.uint32)
    res = {}
    for name, ps in parts.items():
        m = out[ps[0]].copy()
        for p in ps[1:]:
            m &= out[p]
        res[name] = m
    return res


def reconfirm(formulas, conditions, n=5, batch=256, maps=None):
    """For each (formula, condition name): Val_n(phi) == Ext_n(X) over every frame on n
    worlds (33,554,432 at n = 5), comparing the formula's validity map from the census
    kernel with the condition's extension bitmap.  `maps` may hold precomputed
    condition_maps."""
    import torch
    ext = condition_maps(set(conditions), n) if maps is None else maps
    words = ((1 << (n * n)) + 31) // 32
    ok = []
    for s in range(0, len(formulas), batch):
        sub = formulas[s:s + batch]
        code, offs = I.pack(sub)
        dv = torch.zeros((len(sub), words), dtype=torch.int32, device="cuda")
        K.kripke_frame_validity(code, offs, n, 2, dv)
        val = dv.cpu().numpy().view(np.uint32)
        del dv
        for i, cond in enumerate(conditions[s:s + batch]):
            ok.append(bool(np.array_equal(val[i], ext[cond])))
    return ok
