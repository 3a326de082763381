"""Mining and adversarial frame synthesis for late-separating pairs (Section 7).

Mining: candidate pairs (C^m b, C^(m+1) b) for every primitive context word C over
{BOX, DIA} of length at most three, bases TOP, BOT, p, p -> p, p & ~p, ~p | p, and every
m >= 1 with C^(m+1) b of at most 21 nodes.  Each biconditional is censused on every K
frame through five worlds; the pairs that agree there are stressed on template frames
(paths, reverse paths, looped and forked paths, cycles, stars) of six to sixteen
worlds.

Adversarial synthesis: the exact-prefix survivors are then split on frames from six
generators (Erdos-Renyi, edge-flip mutation of canonical seeds, SCC bottlenecks,
dead-end insertion, back-edge injection, permuted bottlenecks) at n = 6, 8, ..., 16;
one-variable pairs only through twelve worlds, constant pairs at every size.  The same
generators also run on survivors of the pair-separation workload (two-variable pairs
that agree through four worlds and that no family frame separated), at 6 and 8 worlds.
Every evaluation runs in the library's kernels.
"""
from __future__ import annotations

import itertools
import time

import numpy as np

from . import inputs as I
from . import kripke as K

BASES = {"T": [I.TOP], "F": [I.BOT], "p": [I.VAR0], "p -> p": [I.VAR0, I.VAR0, I.IMP],
         "p & ~p": [I.VAR0, I.VAR0, I.NOT, I.AND], "~p | p": [I.VAR0, I.NOT, I.VAR0, I.OR]}
SIZES = (6, 8, 10, 12, 14, 16)


def _primitive(word):
    return not any(len(word) % L == 0 and word == word[:L] * (len(word) // L)
                   for L in range(1, len(word)))


def iterate(word, base, m):
    """C^m b in postfix for a context word C (outermost operator first)."""
    f = list(base)
    for _ in range(m):
        f += list(reversed(word))
    return f


def mining_candidates(max_nodes=21):
    """[(label, phi, psi, nvars)] in a fixed order."""
    out = []
    for L in (1, 2, 3):
        for word in itertools.product((I.BOX, I.DIA), repeat=L):
            if not _primitive(word):
                continue
            name = "".join("[]" if o == I.BOX else "<>" for o in word)
            for bname, base in BASES.items():
                nv = 0 if bname in ("T", "F") else 1
                m = 1
                while len(iterate(word, base, m + 1)) <= max_nodes:
                    out.append(((name, bname, m), iterate(word, base, m),
                                iterate(word, base, m + 1), nv))
                    m += 1
    return out


def templates(n):
    """Template frames on n worlds (successor masks), by name."""
    path = [(1 << (w + 1)) if w + 1 < n else 0 for w in range(n)]
    t = {"path": path,
         "reverse path": [(1 << (w - 1)) if w > 0 else 0 for w in range(n)],
         "looped path": path[:-1] + [1 << (n - 1)],
         "forked path": [(1 << (w + 1)) if w + 2 < n - 1 else 0 for w in range(n)],
         "cycle": [1 << ((w + 1) % n) for w in range(n)],
         "star": [((1 << n) - 2) if w == 0 else 0 for w in range(n)]}
    t["forked path"][n - 3] = (1 << (n - 2)) | (1 << (n - 1))
    return t


def _split(pairs, frames, n, nvars):
    import torch
    code, offs = I.pack([p for ab in pairs for p in ab])
    d_fr = torch.as_tensor(np.ascontiguousarray(frames, dtype=np.uint32).view(np.int32),
                           device="cuda")
    out = torch.empty(len(pairs), dtype=torch.int64, device="cuda")
    K.kripke_split_batch(code, offs, d_fr, n, nvars, out)
    return K.as_u64(out)


def exact_prefix(cands, max_n=5):
    """Agreement layer a per candidate: the largest n <= max_n with no countermodel of the
    biconditional on any K frame of at most n worlds."""
    import torch
    agree = np.full(len(cands), max_n, dtype=np.int64)
    for nv in (0, 1):
        idx = [i for i, c in enumerate(cands) if c[3] == nv]
        if not idx:
            continue
        code, offs = I.pack([I.iff(cands[i][1], cands[i][2]) for i in idx])
        alive = np.ones(len(idx), dtype=bool)
        for n in range(1, max_n + 1):
            out = torch.empty((len(idx), 2), dtype=torch.int64, device="cuda")
            K.kripke_census(code, offs, n, K.KRIPKE_K, nv, out)
            hit = alive & (K.as_u64(out)[:, 0] != K.NO_KEY)
            agree[np.array(idx)[hit]] = n - 1
            alive &= ~hit
    return agree


def template_stress(cands, sizes=range(6, 17)):
    """First template size separating each candidate (0: none) and the witness."""
    sep = np.zeros(len(cands), dtype=np.int64)
    wit = [None] * len(cands)
    for n in sizes:
        names = list(templates(n))
        frames = np.array([templates(n)[t] for t in names], dtype=np.uint32)
        for nv in (0, 1):
            idx = [i for i, c in enumerate(cands) if c[3] == nv and sep[i] == 0]
            if not idx:
                continue
            keys = _split([(cands[i][1], cands[i][2]) for i in idx], frames, n, nv)
            for j, key in zip(idx, keys):
                if key != K.NO_KEY:
                    pos, val, world = K.kripke_key_decode(int(key), n, nv)
                    sep[j] = n
                    wit[j] = {"n": n, "template": names[pos], "succ": [int(x) for x in frames[pos]],
                              "valuation": int(val), "world": int(world)}
    return sep, wit


def adversarial(cands, frames_per=4096, sizes=SIZES, one_var_max=12, two_var_max=8, log=None):
    """Split every candidate on every generator's frames; per generator: relations,
    pair-frame tests, valuation-frame evaluations, verified separations and seconds.
    One-variable pairs run through one_var_max worlds and two-variable pairs through
    two_var_max (4^n valuations per frame), constant pairs at every size."""
    import torch
    stats = {}
    hits = {}
    for g in I.ADVERSARIAL:
        rel = tests = evals = 0
        t_gpu = 0.0
        found = set()
        for n in sizes:
            frames = I.adversarial_frames(g, n, frames_per)
            for nv in sorted({c[3] for c in cands}):
                if (nv == 1 and n > one_var_max) or (nv >= 2 and n > two_var_max):
                    continue
                idx = [i for i, c in enumerate(cands) if c[3] == nv]
                if not idx:
                    continue
                torch.cuda.synchronize()
                t0 = time.time()
                keys = _split([(cands[i][1], cands[i][2]) for i in idx], frames, n, nv)
                t_gpu += time.time() - t0
                tests += len(idx) * len(frames)
                for j, key in zip(idx, keys):
                    scanned = len(frames)
                    if key != K.NO_KEY:
                        pos, val, world = K.kripke_key_decode(int(key), n, nv)
                        scanned = pos + 1
                        if j not in found:
                            found.add(j)
                            hits.setdefault(j, []).append(
                                {"generator": g, "n": n, "succ": [int(x) for x in frames[pos]],
                                 "valuation": int(val), "world": int(world)})
                    evals += scanned * (1 << (nv * n))
            rel += len(frames)
        stats[g] = {"relations": rel, "pair_frame_tests": tests, "valuation_frame_evals": evals,
                    "separated": len(found), "seconds": t_gpu}
        if log:
            log(f"adversarial {g}: {rel} relations, {len(found)} pairs separated, {t_gpu:.2f} s")
    return stats, hits


def c4_survivors(pairs, separated, sample=1024, seed=I.SEED_ADV):
    """The adversarial input of the pair-separation workload: a seeded sample of its pairs
    (two variables, agreeing on every model with at most four worlds) that no frame of the
    6-, 7- and 8-world families separated; as [(label, phi, psi, 2)]."""
    idx = [i for i in range(len(pairs)) if not separated[i]]
    rng = I.SplitMix64(seed, 11)
    pick = sorted(set(idx[rng.below(len(idx))] for _ in range(4 * sample)))[:sample] \
        if len(idx) > sample else idx
    return [(("c4", i), pairs[i][0], pairs[i][1], 2) for i in pick]


def run_c4(pairs, separated, sample=1024, frames_per=1024, log=print):
    """Adversarial frames (six generators, n = 6 and 8) on C4 survivors."""
    t0 = time.time()
    cands = c4_survivors(pairs, separated, sample)
    stats, hits = adversarial(cands, frames_per, sizes=(6, 8), log=log)
    return {"survivors_total": int(sum(1 for x in separated if not x)),
            "sampled": len(cands), "frames_per_generator_and_n": frames_per, "sizes": [6, 8],
            "adversarial": stats, "adversarial_separated": len(hits),
            "seconds": time.time() - t0}, hits


def run(frames_per=4096, log=print):
    t0 = time.time()
    cands = mining_candidates()
    agree = exact_prefix(cands)
    surv = [i for i in range(len(cands)) if agree[i] == 5]
    sub = [cands[i] for i in surv]
    sep, wit = template_stress(sub)
    if log:
        log(f"mining: {len(cands)} candidates, {len(surv)} agree through five worlds, "
            f"{int((sep > 0).sum())} separated on templates of 6-16 worlds")
    stats, hits = adversarial(sub, frames_per, log=log)
    resistant = [j for j in range(len(sub)) if sep[j] == 0]
    rec = {"candidates": len(cands), "exact_prefix_survivors": len(surv),
           "template_separated": int((sep > 0).sum()), "template_resistant": len(resistant),
           "adversarial": stats,
           "adversarial_separated": len(hits),
           "template_resistant_separated": sum(1 for j in resistant if j in hits),
           "seconds": time.time() - t0}
    return rec, {"cands": sub, "template_sep": sep, "template_witness": wit, "hits": hits}
