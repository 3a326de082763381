"""Benchmark: n = 5 exhaustive Kripke census throughput on one MI355X.

One step = one replay of the captured hipGraph that censuses the 4,096-formula
batch (2 variables, uneven lengths 3..40, modal depth 0..6) over every labelled
frame on 5 worlds for the classes K, T, S4 and S5, with every valuation.
`value` is evaluated (formula, frame-in-class, valuation) triples per second.

Also measured (reported inside the JSON line):
  - plain: the same kernel launched once per formula (4,096 launches) against the
    batched single launch, both over the same frame slice;
  - roofline of the dominant kernel (the K-class census), INT32 VALU bound;
  - cpu_baseline: the CPU oracle on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT32 = 256 * 64 * 2.4e9  # INT32 lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def class_frames(n):
    from paper_2606_15437_amd import inputs as I  # noqa: F401
    return {0: 1 << (n * n), 1: 1 << (n * n - n), 2: {1: 1, 2: 4, 3: 29, 4: 355, 5: 6942}[n],
            3: {1: 1, 2: 2, 3: 5, 4: 15, 5: 52}[n]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--formulas", type=int, default=4096)
    ap.add_argument("--slice-log2", type=int, default=18,
                    help="frame slice [0, 2^s) for the plain-vs-batched comparison")
    ap.add_argument("--cpu-frames-log2", type=int, default=12)
    ap.add_argument("--cpu-formulas", type=int, default=64)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design is frame-range sharding with a min/sum reduction, not run here.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_15437_amd import inputs as I
    from paper_2606_15437_amd import kripke as K

    n, nvars = 5, 2
    nval = 1 << (n * nvars)
    fs = I.config3_formulas(args.formulas)
    B = len(fs)
    code, offs = I.pack(fs)
    stats = [I.formula_stats(f, n) for f in fs]
    bitops_sum = float(sum(s["bitops"] for s in stats))
    cf = class_frames(n)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    # ---------------------------------------------------------- batched step
    log(f"plan: {B} formulas, n={n}, classes K/T/S4/S5")
    plan = K.kripke_plan_create(code, offs, n, 0xF, nvars)
    out = torch.empty((4, B, 2), dtype=torch.int64, device=dev)
    for i in range(args.warmup):
        t0 = time.time()
        K.kripke_plan_launch(plan, out, stream)
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.time() - t0:.2f} s")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for i in range(args.steps):
        K.kripke_plan_launch(plan, out, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    evals_step = float(B * nval * sum(cf.values()))
    value = evals_step / (ms / 1e3)
    res = K.as_u64(out)
    log(f"batched all-class step: {ms:.1f} ms, {value / 1e9:.1f} G evals/s")
    valid = {c: int((res[c, :, 0] == K.NO_KEY).sum()) for c in range(4)}
    K.kripke_plan_destroy(plan)

    # ------------------------------------------- dominant kernel: K census
    planK = K.kripke_plan_create(code, offs, n, 0x1, nvars)
    outK = torch.empty((4, B, 2), dtype=torch.int64, device=dev)
    K.kripke_plan_launch(planK, outK, stream)
    torch.cuda.synchronize()
    ev0.record(stream)
    K.kripke_plan_launch(planK, outK, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    msK = ev0.elapsed_time(ev1)
    K.kripke_plan_destroy(planK)
    evalsK = float(B) * cf[0] * nval
    int_ops = bitops_sum * cf[0] * nval / 32.0  # algorithmic INT32 ops (Proposition 2 in bits)
    achieved = int_ops / (msK / 1e3)
    log(f"K census: {msK:.1f} ms, {evalsK / msK / 1e6:.1f} G evals/s, "
        f"{achieved / 1e12:.2f} T INT32 ops/s ({100 * achieved / PEAK_INT32:.1f}% of peak)")

    # ------------------------------------------- plain vs batched on a slice
    plain = None
    if not args.no_plain:
        S = 1 << args.slice_log2
        o1 = torch.empty((B, 2), dtype=torch.int64, device=dev)
        K.kripke_census_range(code, offs, n, 0, nvars, 0, S, 0, o1, stream)
        torch.cuda.synchronize()
        ev0.record(stream)
        K.kripke_census_range(code, offs, n, 0, nvars, 0, S, 0, o1, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_b = ev0.elapsed_time(ev1)
        o2 = torch.empty((B, 2), dtype=torch.int64, device=dev)
        single = [(np.asarray(f, dtype=np.uint8), np.array([0, len(f)], dtype=np.uint32))
                  for f in fs]
        t0 = time.time()
        ev0.record(stream)
        for b, (c1, of1) in enumerate(single):
            K.kripke_census_range(c1, of1, n, 0, nvars, 0, S, 0, o2[b:b + 1], stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_p = ev0.elapsed_time(ev1)
        agree = bool((K.as_u64(o1) == K.as_u64(o2)).all())
        ev_slice = float(B) * S * nval
        plain = {"frames": S, "batched_G_evals_per_s": ev_slice / ms_b / 1e6,
                 "plain_G_evals_per_s": ev_slice / ms_p / 1e6, "batched_ms": ms_b,
                 "plain_ms": ms_p, "speedup": ms_p / ms_b, "launches": B,
                 "results_identical": agree, "host_s": time.time() - t0}
        log(f"plain vs batched on {S} frames: {ms_p:.1f} ms vs {ms_b:.1f} ms "
            f"({ms_p / ms_b:.2f}x), identical={agree}")

    # ---------------------------------------------------------- CPU oracle
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as orc
        sub = fs[:args.cpu_formulas]
        F = 1 << args.cpu_frames_log2
        t0 = time.time()
        threads = 0
        for f in sub:
            _, _, threads = orc.census(f, n, 0, nvars, 0, F, threads=0)
        dt = time.time() - t0
        cpu_evals = float(len(sub)) * F * nval
        cpu = {"value": cpu_evals / dt / 1e9, "unit": "G evals/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first {len(sub)} formulas of the 4,096-formula batch x frames "
                         f"[0, 2^{args.cpu_frames_log2}) x {nval} valuations, class K "
                         f"({cpu_evals:.3g} evaluations in {dt:.1f} s)"}
        log(f"cpu oracle: {cpu['value']:.4f} G evals/s on {threads} threads")

    rec = {
        "metric": "formula*frame*valuation G evals/s, n=5 census (batched hipGraph vs plain)",
        "value": value / 1e9,
        "unit": "G evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "n=5 census, 4,096 seeded formulas (len 3..40, depth 0..6), "
                               "2 vars (1,024 valuations), classes K+T+S4+S5, one graph replay",
                   "formulas": B, "n": n, "nvars": nvars, "evals_per_step": evals_step,
                   "valid_per_class": valid},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_INT32 / 1e12,
                     "unit": "T INT32 ops/s", "frac": achieved / PEAK_INT32, "traffic": None,
                     "kernel": "census K class, n=5", "kernel_ms": msK,
                     "mean_bitops_per_eval": bitops_sum / B},
        "cpu_baseline": cpu,
        "plain_vs_batched": plain,
        "k_census_G_evals_per_s": evalsK / msK / 1e6,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
