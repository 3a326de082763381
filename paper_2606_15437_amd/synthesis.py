"""Active synthesis of late-separating pairs (Section 7, active synthesis protocol).

Candidates iterate a modal context C in {BOX DIA, DIA BOX, BOX BOX, DIA DIA} on a base
b in {TOP, BOT}: (C^m b, C^(m+1) b) for m = 1..4, 32 pairs.  Each biconditional is
censused exhaustively on every K frame with n = 1..5 worlds (constant formulas need
one valuation), which fixes a, the largest size through which the pair agrees.  Pairs
that agree through five worlds are challenged on template frames of six to ten worlds
(paths, reverse paths, looped paths, forked paths).  The score is
R = a + 2 [separated at a + 1] - 0.02 (|phi| + |psi|).  Every evaluation runs in the
library's kernels.
"""
from __future__ import annotations

import numpy as np

from . import inputs as I
from . import kripke as K

CONTEXTS = {"BOX DIA": (I.DIA, I.BOX), "DIA BOX": (I.BOX, I.DIA), "BOX BOX": (I.BOX, I.BOX),
            "DIA DIA": (I.DIA, I.DIA)}
BASES = {"TOP": I.TOP, "BOT": I.BOT}


def iterate(ctx: str, base: str, m: int) -> list[int]:
    """C^m b in postfix: the context's inner operator is applied first."""
    inner, outer = CONTEXTS[ctx]
    return [BASES[base]] + [inner, outer] * m


def candidates():
    """The 32 candidate pairs with their labels (context, base, m)."""
    out = []
    for ctx in CONTEXTS:
        for base in BASES:
            for m in range(1, 5):
                out.append(((ctx, base, m), iterate(ctx, base, m), iterate(ctx, base, m + 1)))
    return out


def templates(n: int) -> dict[str, list[int]]:
    """Template frames on n worlds as successor masks: the path 0 -> 1 -> ... -> n-1, its
    reverse, the path with a loop on its last world, and the path whose last edge forks
    (world n-3 has the two leaves n-2 and n-1)."""
    path = [(1 << (w + 1)) if w + 1 < n else 0 for w in range(n)]
    reverse = [(1 << (w - 1)) if w > 0 else 0 for w in range(n)]
    looped = list(path)
    looped[n - 1] |= 1 << (n - 1)
    fork = [(1 << (w + 1)) if w + 2 < n - 1 else 0 for w in range(n)]
    fork[n - 3] = (1 << (n - 2)) | (1 << (n - 1))
    return {"path": path, "reverse path": reverse, "looped path": looped, "forked path": fork}


def run(max_exact: int = 5, template_sizes=range(6, 11)):
    """Rank the candidates.  Returns one record per pair, best first."""
    import torch
    cands = candidates()
    chis = [I.iff(a, b) for _, a, b in cands]
    code, offs = I.pack(chis)
    B = len(cands)
    agree = np.full(B, max_exact, dtype=np.int64)   # a
    sep = np.zeros(B, dtype=np.int64)                # separation size found (0: none)
    witness = [None] * B
    alive = np.ones(B, dtype=bool)
    for n in range(1, max_exact + 1):
        out = torch.empty((B, 2), dtype=torch.int64, device="cuda")
        K.kripke_census(code, offs, n, K.KRIPKE_K, 0, out)
        keys = K.as_u64(out)[:, 0]
        for i in np.nonzero(alive & (keys != K.NO_KEY))[0]:
            agree[i] = n - 1
            sep[i] = n
            frame, _, world = K.kripke_key_decode(int(keys[i]), n, 0)
            witness[i] = {"n": n, "frame": int(frame), "world": int(world), "kind": "exhaustive"}
            alive[i] = False
    pair_code, pair_offs = I.pack([p for _, a, b in cands for p in (a, b)])
    for n in template_sizes:
        if not alive.any():
            break
        names = list(templates(n))
        frames = np.array([templates(n)[t] for t in names], dtype=np.uint32)
        d_fr = torch.as_tensor(frames.view(np.int32), device="cuda")
        out = torch.empty(B, dtype=torch.int64, device="cuda")
        K.kripke_split_batch(pair_code, pair_offs, d_fr, n, 0, out)
        keys = K.as_u64(out)
        for i in np.nonzero(alive & (keys != K.NO_KEY))[0]:
            pos, _, world = K.kripke_key_decode(int(keys[i]), n, 0)
            sep[i] = n
            witness[i] = {"n": n, "template": names[pos], "succ": [int(x) for x in frames[pos]],
                          "world": int(world), "kind": "template"}
            alive[i] = False
    recs = []
    for i, (label, a, b) in enumerate(cands):
        hit = sep[i] == agree[i] + 1
        score = agree[i] + 2 * int(hit) - 0.02 * (len(a) + len(b))
        recs.append({"context": label[0], "base": label[1], "m": label[2],
                     "phi": I.to_text(a), "psi": I.to_text(b), "agree_through": int(agree[i]),
                     "separation": int(sep[i]) or None, "witness": witness[i],
                     "R": round(float(score), 4)})
    recs.sort(key=lambda r: -r["R"])
    return recs
