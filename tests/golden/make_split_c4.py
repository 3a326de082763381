"""Write tests/golden/split_c4_first1000.txt: expected split keys of the pair-separation
workload on the first 1,000 frames of the 6-, 7- and 8-world families, computed by the
CPU oracle alone (Definition 2, Proposition 5: the least (position, valuation, world)
where the two formulas differ, by full early-exit scans).

Pairs (from the seeded inputs, selected with the oracle only):
  - "agree4": consecutive members of buckets of equal truth at the 4,096 sampled
    pointed models (every model with at most two worlds, 3,520 three-world ones), in
    pool order, whose biconditional has no countermodel on any frame with at most four
    worlds (oracle census of each layer n = 1..4);
  - "random": consecutive pool members (2k, 2k + 1) for seeded k, unfiltered (these
    usually separate on the first frames, at varied valuations and worlds);
  - "designed": the designed late-separating pairs.
Each line of the output names the pair by pool indices (or designed index) so the
test rebuilds the formulas from the seeded generators.

Usage: python tests/golden/make_split_c4.py [--agree4 140] [--random 40] [--frames 1000]
"""
import argparse
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2606_15437_amd import inputs as I  # noqa: E402

OUT = os.path.join(HERE, "split_c4_first1000.txt")
POOL = 30_000


def candidates(sig):
    """(i, j), i < j, consecutive members of each bucket of equal signature, pool order."""
    rows = np.ascontiguousarray(sig).view(np.dtype((np.void, sig.shape[1] * 8))).ravel()
    last = {}
    out = []
    for i, r in enumerate(rows):
        key = r.tobytes()
        if key in last:
            out.append((last[key], i))
        last[key] = i
    out.sort()
    return out


def first_refuted_layer(chi, max_n=4):
    """Least n <= max_n at which the biconditional has a countermodel, else 0."""
    for n in range(1, max_n + 1):
        if orc.census(chi, n, orc.CLASS_K, 2, stop_at_first=True, threads=0)[0] != orc.NONE:
            return n
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--agree4", type=int, default=140)
    ap.add_argument("--random", type=int, default=40)
    ap.add_argument("--frames", type=int, default=1000)
    args = ap.parse_args()
    t0 = time.time()
    pool = I.config4_pool(POOL)
    samples = I.signature_samples()
    chunks = [pool[i:i + 1000] for i in range(0, len(pool), 1000)]
    with ThreadPoolExecutor(max_workers=8) as ex:
        sig = np.concatenate(list(ex.map(lambda c: orc.signatures(c, samples, 2), chunks)))
    cand = candidates(sig)
    print(f"{len(cand)} candidate pairs ({time.time() - t0:.0f} s)", flush=True)
    agree4 = []
    for i, j in cand:
        if len(agree4) >= args.agree4:
            break
        if first_refuted_layer(I.iff(pool[i], pool[j])) == 0:
            agree4.append((i, j))
    rng = I.SplitMix64(0x5B1175EED, 0)
    rand = []
    while len(rand) < args.random:
        k = rng.below(POOL // 2)
        if (2 * k, 2 * k + 1) not in rand:
            rand.append((2 * k, 2 * k + 1))
    print(f"{len(agree4)} agree through 4 worlds ({time.time() - t0:.0f} s)", flush=True)
    designed = I.config4_designed_pairs()
    named = ([("agree4", i, j) for i, j in agree4] + [("random", i, j) for i, j in rand] +
             [("designed", d, -1) for d in range(len(designed))])
    pairs = [(pool[i], pool[j]) for _, i, j in named[:len(agree4) + len(rand)]] + designed
    keys = {}
    for n in (6, 7, 8):
        frames = I.frame_family(n, args.frames)
        with ThreadPoolExecutor(max_workers=8) as ex:
            keys[n] = list(ex.map(lambda ab: orc.split(ab[0], ab[1], frames, 2), pairs))
        print(f"n={n}: {sum(k != orc.NONE for k in keys[n])} of {len(pairs)} separated "
              f"({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as fh:
        fh.write("# Split keys of the pair-separation workload on the first %d frames of the\n"
                 "# 6-, 7- and 8-world families (Definition 2, Proposition 5), from the CPU\n"
                 "# oracle's full early-exit scans; written by tests/golden/make_split_c4.py.\n"
                 "# pair <index> <kind> <i> <j>: kind agree4/random = config4_pool(%d)\n"
                 "#   members i, j; kind designed = config4_designed_pairs()[i].\n"
                 "# key <n> <pair index> <key> (18446744073709551615 = no separating model).\n"
                 % (args.frames, POOL))
        fh.write(f"frames {args.frames}\n")
        for p, (kind, i, j) in enumerate(named):
            fh.write(f"pair {p} {kind} {i} {j}\n")
        for n in (6, 7, 8):
            for p, k in enumerate(keys[n]):
                fh.write(f"key {n} {p} {k}\n")
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
