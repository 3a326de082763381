"""Benchmark: n = 5 exhaustive Kripke census throughput on one MI355X.

One step = one replay of the captured hipGraph holding the single persistent
launch that censuses the 4,096-formula batch (2 variables, uneven lengths
3..40, modal depth caps 0..6) over every labelled frame on 5 worlds and every
valuation, reducing each K frame into every class (K, T, S4, S5) containing
it.  `value` is evaluated (formula, frame, valuation) triples per second, over
the formulas that do not fold to a constant (those are decided without
evaluation); the T/S4/S5 results are reductions of the same evaluations and are
not counted again.

Also reported in the JSON line:
  - plain_vs_batched: the same census launched once per formula: "plain" with the
    per-class kernels and default tiles (16,384 launches), "per_formula_autotuned" with
    the fused all-class kernel and tiles tuned for that form (4,096 launches), no graph;
  - roofline: the census kernel against the INT32 VALU peak, counting the
    bit operations of Proposition 2 on the programs actually executed (after
    exact constant folding); the figure on the source formulas is given too;
  - cpu_baseline: the CPU oracle on bounded samples of the n = 5 workload, the
    Table-1 matched workload and the n = 4 three-variable subset, median of 5, on one
    thread and on every host core;
  - table1: the paper's matched single-formula workload;
  - split: the split search (Definition 2, Proposition 5) of formula pairs that agree on
    every model with at most 4 worlds, over the 6-, 7- and 8-world frame families;
  - mlp_scoring: the pair MLP's forward throughput on 2^20 pairs against the BF16
    matrix-core peak;
  - learned: the learned pair proposal at full scale (10,000-formula corpus, ~5.5M-pair
    universe, 10^6 budget), every proposal verified exactly, against plain enumeration;
  - census_reproduction: the paper's five-world census (Section 6): 44,678 enumerated
    formulas -> 5,621 classes -> 5,624 formulas x K/T/S4/S5 x every frame n <= 5;
  - active_synthesis: the 32 context-iteration pairs of Section 7, exact through five
    worlds, template frames of six to ten worlds beyond;
  - correspondence: frame-correspondence recovery of Section 10 over the census corpus
    (validity maps of every formula on every frame with at most four worlds);
  - adversarial: mining of context-iteration pairs, exact prefix through five worlds,
    template frames of 6-16 worlds and six adversarial frame generators (Section 7).

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

# INT32 bitwise VALU peak: the published 157.3 TFLOP/s FP32 vector rate counts an FMA as
# two flops, i.e. 256 CUs x 128 lanes/clk x 2.4 GHz = 78.6 T lane-operations/s.
PEAK_INT32 = 256 * 128 * 2.4e9
CLASS_FRAMES_N5 = (33554432, 1048576, 6942, 52)


def recorded_traffic(name="census_fast_n5_traffic.json"):
    """HBM bytes per launch of a kernel from its committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE record, or None if the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def provenance():
    """What produced this record: a hash of the library sources and this script (the GPU
    copy of the tree has no git metadata), the git revision when there is one, and the
    master seeds of the seeded inputs."""
    import glob
    import hashlib
    import subprocess
    from paper_2606_15437_amd import inputs as I
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2606_15437_amd", "csrc", "*")) +
                   [os.path.join(ROOT, "include", "kripke.h"), os.path.abspath(__file__)])
    h = hashlib.sha256()
    for f in files:
        h.update(open(f, "rb").read())
    try:
        rev = subprocess.run(["git", "rev-parse", "HEAD"], cwd=ROOT, capture_output=True,
                             text=True, timeout=10).stdout.strip() or None
    except (OSError, subprocess.SubprocessError):
        rev = None
    seeds = {name: hex(getattr(I, name)) for name in ("SEED_C1", "SEED_C2", "SEED_C3", "SEED_C4",
                                                       "SEED_C5_TEST", "SEED_C5_TRAIN",
                                                       "SEED_ADV")}
    return {"sources_sha256": h.hexdigest(), "git_rev": rev, "seeds": seeds}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed(fn, stream, reps=1):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_split(args, stream):
    """Split search over the frame families: pairs agreeing through 4 worlds (mostly never
    separated, so nearly every frame is scanned), first separating model per pair."""
    import torch
    from paper_2606_15437_amd import inputs as I
    from paper_2606_15437_amd import kripke as K
    from paper_2606_15437_amd.split_workload import config4_pairs
    t0 = time.time()
    log(f"split: selecting {args.split_pairs} pairs from a pool of {args.split_pool} formulas")
    pairs, stats = config4_pairs(args.split_pairs, pool=args.split_pool, log=log)
    sel_s = time.time() - t0
    code, offs = I.pack([p for ab in pairs for p in ab])
    st = K.kripke_program_stats(*I.pack([I.iff(a, b) for a, b in pairs]), 2)
    per = {}
    tot_ms = tot_evals = tot_ops = 0.0
    separated = np.zeros(len(pairs), dtype=bool)
    for n in (6, 7, 8):
        frames = I.frame_family(n, args.split_frames)
        d_fr = torch.as_tensor(np.ascontiguousarray(frames).view(np.int32), device="cuda")
        out = torch.empty(len(pairs), dtype=torch.int64, device="cuda")
        run = lambda: K.kripke_split_batch(code, offs, d_fr, n, 2, out, stream)
        # warm-up on the first frames only (loads the kernels; the full scan is long)
        K.kripke_split_batch(code, offs, d_fr[:4096], n, 2, out, stream)
        log(f"split n={n}: scanning {len(pairs)} pairs x {len(frames)} frames")
        ms = timed(run, stream)
        keys = K.as_u64(out)
        nval = 1 << (2 * n)
        found = keys != K.NO_KEY
        separated |= found
        # frames actually scanned: up to the separating one, else all of them
        scanned = np.where(found, (keys >> np.uint64(2 * n + 4)).astype(np.float64) + 1,
                           float(len(frames)))
        evals = float((scanned * nval).sum())
        ops = float(((n * st[:, 1] + n * n * st[:, 0]) * scanned).sum()) * nval / 32.0
        per[str(n)] = {"ms": ms, "G_evals_per_s": evals / ms / 1e6, "split": int(found.sum()),
                       "T_int32_ops_per_s": ops / ms / 1e9}
        tot_ms += ms
        tot_evals += evals
        tot_ops += ops
        log(f"split n={n}: {ms:.0f} ms, {evals / ms / 1e6:.0f} G evals/s, "
            f"{int(found.sum())} of {len(pairs)} pairs separated")
    return {"workload": f"{len(pairs)} pairs agreeing through 4 worlds ({stats['designed']} "
                        f"designed) from a pool of {args.split_pool} formulas x first "
                        f"{args.split_frames} frames of the n = 6, 7, 8 families x all "
                        f"2^(2n) valuations",
            "G_evals_per_s": tot_evals / tot_ms / 1e6, "ms": tot_ms, "per_n": per,
            # the dominant kernel is the n = 8 list kernel
            "roofline": {"bound": "alu", "achieved": per["8"]["T_int32_ops_per_s"],
                         "peak": PEAK_INT32 / 1e12, "unit": "T INT32 ops/s",
                         "frac": per["8"]["T_int32_ops_per_s"] / (PEAK_INT32 / 1e12),
                         # the counters were taken on a smaller workload than this one:
                         # reported beside, not as this launch's traffic
                         "traffic": None,
                         "traffic_profiled": {
                             "bytes_per_launch": recorded_traffic("split_list_n8_traffic.json"),
                             "workload": "2,048 pairs x 262,144 frames at n = 8 "
                                         "(profiles/split_list_n8.md)"},
                         "kernel": "census_fast<8,2,*,LIST>",
                         "all_n_achieved": tot_ops / tot_ms / 1e9},
            "selection": dict(stats, seconds=sel_s),
            "note": "timed per call including host compile and upload of the pair programs",
            "_survivors": (pairs, separated)}


def bench_cpu(fs, reps=5):
    """The CPU oracle (recursive satisfaction over explicit sets) timed on the host cores,
    on bounded samples of three workloads, median of `reps` runs, on one thread and on
    every core (the oracle splits a frame range over threads and merges min/sum)."""
    import statistics
    from oracle import oracle as orc
    from paper_2606_15437_amd import inputs as I
    nproc = os.cpu_count()
    # (name, formulas, n, nvars, (formulas, frames) on one thread, ... on all cores)
    work = [
        ("table1_matched", [I.parse(I.TABLE1_FORMULA)], 5, 2, (1, 1 << 12), (1, 1 << 16)),
        ("c2_subset_n4_K", I.config2_formulas()[:64], 4, 3, (4, 1 << 8), (64, 1 << 8)),
        ("c3_slice_n5_K", fs[:64], 5, 2, (8, 1 << 10), (64, 1 << 11)),
    ]
    out = {}
    for name, formulas, n, nvars, one, every in work:
        rec = {}
        for label, (nf, frames), threads in (("single_thread", one, 1), ("all_cores", every, 0)):
            times, used = [], 1
            for _ in range(reps):
                t0 = time.perf_counter()
                for f in formulas[:nf]:
                    _, _, used = orc.census(f, n, 0, nvars, 0, frames, threads=threads)
                times.append(time.perf_counter() - t0)
            evals = float(nf) * frames * (1 << (n * nvars))
            med = statistics.median(times)
            rec[label] = {"G_evals_per_s": evals / med / 1e9, "threads": used,
                          "median_s": med, "runs_s": times,
                          "sample": f"{nf} formula(s) x frames [0, {frames}) x "
                                    f"{1 << (n * nvars)} valuations, n = {n}, class K"}
        out[name] = rec
        log(f"cpu oracle {name}: {rec['single_thread']['G_evals_per_s']:.4f} G evals/s on one "
            f"thread, {rec['all_cores']['G_evals_per_s']:.4f} on {rec['all_cores']['threads']}")
    head = out["c3_slice_n5_K"]
    return {"value": head["all_cores"]["G_evals_per_s"], "unit": "G evals/s",
            "cores": head["all_cores"]["threads"], "kind": "oracle",
            "sample": "n = 5 census workload slice: " + head["all_cores"]["sample"] +
                      f", median of {reps} runs",
            "single_thread_value": head["single_thread"]["G_evals_per_s"],
            "nproc": nproc, "workloads": out,
            "paper_context": {"cpu_scalar_1_thread": 0.0471, "cpu_bitmask_openmp_26": 0.814,
                              "cpu_avx512_openmp_26": 5.43, "gpu_h100_table1": 38.33,
                              "hardware": "Xeon Platinum 8480+ and H100 PCIe"}}


PEAK_BF16 = 2.5e15  # dense BF16 matrix-core peak of one MI355X (FLOP/s)


def bench_mlp(stream, npairs=1 << 20, reps=3):
    """Scoring throughput of the pair MLP (8192 -> 512 -> 256 -> 1, BF16 operands, FP32
    accumulation) on seeded random signatures, in the scoring path's chunks."""
    import statistics
    import torch
    from paper_2606_15437_amd import kripke as K
    from paper_2606_15437_amd.proposal import SCORE_CHUNK
    rng = np.random.default_rng(0x5C0)
    sig = rng.integers(0, 2 ** 63, size=(10000, 64), dtype=np.uint64)
    ij = rng.integers(0, 10000, size=(npairs, 2)).astype(np.uint64)
    pairs = (ij[:, 0] << np.uint64(32)) | ij[:, 1]
    d_sig = torch.as_tensor(sig.view(np.int64), device="cuda")
    d_pairs = torch.as_tensor(pairs.view(np.int64), device="cuda")
    d_z = torch.empty(npairs, dtype=torch.float32, device="cuda")
    h = K.kripke_mlp_create(1, SCORE_CHUNK)
    try:
        K.kripke_mlp_forward(h, d_sig, d_pairs, d_z, stream)
        ms = statistics.median(timed(lambda: K.kripke_mlp_forward(h, d_sig, d_pairs, d_z, stream),
                                     stream) for _ in range(reps))
    finally:
        K.kripke_mlp_destroy(h)
    flop = 2.0 * npairs * (8192 * 512 + 512 * 256 + 256)
    log(f"mlp forward: {npairs} pairs in {ms:.1f} ms, {flop / ms / 1e9:.1f} TFLOP/s")
    return {"pairs": npairs, "chunk": SCORE_CHUNK, "ms": ms, "TFLOP_per_s": flop / ms / 1e9,
            "roofline": {"bound": "mfma", "achieved": flop / ms / 1e9, "peak": PEAK_BF16 / 1e12,
                         "unit": "TFLOP/s", "frac": flop / ms / 1e-3 / PEAK_BF16},
            "flop_per_pair": flop / npairs}


def bench_learned():
    """The learned proposal protocol at full scale (every heavy step in the library)."""
    from paper_2606_15437_amd import proposal as P
    rec = P.run(log=log)
    rec["train"]["loss"] = rec["train"]["loss"][-1]
    return rec


def bench_reproduction():
    """The five-world census of Section 6 (paper: 1.63e14 evaluations in 45 minutes)."""
    from paper_2606_15437_amd import census_corpus as C
    out, _, _ = C.run(log=log, tune_cache=os.path.join(ROOT, "paper_2606_15437_amd",
                                                       "tune_cache.json"))
    out["G_evals_per_s_five_world"] = out["k_frame_evals"] / out["census_seconds"] / 1e9
    out["paper"] = {"raw_trees": 44678, "classes": 5621, "formulas": 5624,
                    "K_refuted_on_1": 5086, "K_refuted_on_2": 536, "K_survivors": 2,
                    "K->T": 428, "T->S4": 48, "S4->S5": 118, "certificates": 20990,
                    "minutes": 45, "evals": 1.63e14}
    out["named_axioms"] = "K, T, McKinsey"
    return out


def bench_synthesis():
    from paper_2606_15437_amd import synthesis as S
    t0 = time.time()
    recs = S.run()
    return {"seconds": time.time() - t0, "pairs": len(recs),
            "late_hits": sum(1 for r in recs if r["agree_through"] == 5 and r["separation"]),
            "top": [{k: r[k] for k in ("phi", "psi", "agree_through", "separation", "R")}
                    for r in recs[:3]]}


def bench_correspondence():
    """Frame-correspondence recovery (Section 10) over the census corpus with three condition
    libraries: the eight conditions Table 9 names; those and coreflexive, shift reflexive and
    functional frames; and our 136-condition library (16 base conditions and every
    conjunction of two).  Every recovered (formula, condition) is
    re-confirmed over all 33,554,432 five-world frames."""
    import collections
    from paper_2606_15437_amd import census_corpus as C
    from paper_2606_15437_amd import correspondence as R
    _, _, corpus = C.build_corpus()
    out = {"formulas": len(corpus),
           "paper": {"recovered": 220, "trivial": 2798, "unmatched": 2606,
                     "reconfirmed_on": "all 33,554,432 five-world frames"}}
    maps = None
    for name, lib in (("table9_conditions", R.table9_library()),
                      ("table9_and_textbook", R.textbook_library()),
                      ("library_136", R.library())):
        t0 = time.time()
        res = R.recover(corpus, max_n=4, log=log, lib=lib)
        rec_idx = [i for i, o in enumerate(res) if isinstance(o, list) and o]
        dt = time.time() - t0
        # re-confirm every recovered formula with its first matching condition
        t1 = time.time()
        conds = [res[i][0] for i in rec_idx]
        need = set(conds)
        if maps is None or not need <= set(maps):
            maps = R.condition_maps(sorted(need | set(maps or {})), 5)
        ok = R.reconfirm([corpus[i] for i in rec_idx], conds, 5, maps=maps)
        counts = collections.Counter(conds)
        out[name] = {"library_size": len(lib), "recovered": len(rec_idx),
                     "trivial": sum(1 for o in res if o == "trivial"),
                     "unmatched": sum(1 for o in res if o == []), "seconds": dt,
                     "reconfirmed_five_worlds": int(sum(ok)),
                     "reconfirm_frames": 1 << 25, "reconfirm_s": time.time() - t1,
                     "most_recovered": counts.most_common(8)}
        log(f"correspondence ({name}): {len(rec_idx)} recovered, {int(sum(ok))} re-confirmed on "
            f"every five-world frame ({time.time() - t1:.1f} s)")
    rows = R.table9()
    out["table9"] = {n: r for (n, _), r in zip(rows, R.recover([f for _, f in rows], 4))}
    return out


def bench_adversarial(split_survivors=None):
    from paper_2606_15437_amd import adversarial as A
    c4 = None
    if split_survivors is not None:
        c4, _ = A.run_c4(*split_survivors, log=log)
    rec, _ = A.run(frames_per=16384, log=log)
    rec["input"] = ("the context-iteration mining candidates of Section 7 (the paper's "
                    "adversarial input came from its mining report); c4_survivors: the same "
                    "generators on pairs of the pair-separation workload no family frame split")
    rec["c4_survivors"] = c4
    rec["relations"] = sum(g["relations"] for g in rec["adversarial"].values())
    rec["valuation_frame_evals"] = sum(g["valuation_frame_evals"]
                                       for g in rec["adversarial"].values())
    rec["paper"] = {"candidates": 476, "relations": 8995007, "valuation_frame_evals": 94.68e9,
                    "hits_by_generator": {"erdos-renyi": 55, "edge-flip": 35, "scc-bottleneck": 0,
                                          "dead-end": 0, "back-edge": 0, "permuted-bottleneck": 0}}
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--formulas", type=int, default=4096)
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2606_15437_amd",
                                                         "tune_cache.json"))
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (reference for "
                         "HBM byte counters)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--split-pairs", type=int, default=20_000)
    ap.add_argument("--split-pool", type=int, default=200_000)
    ap.add_argument("--split-frames", type=int, default=1_000_000)
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-reproduction", action="store_true")
    ap.add_argument("--only", choices=("mlp", "split", "correspondence"),
                    help="run one secondary leg alone and print its record (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design (frame-range shards, one min/sum reduction) is not run here.",
              file=sys.stderr)
        sys.exit(2)

    # the library's autotuner reports each candidate it times (stderr)
    os.environ.setdefault("KRIPKE_TUNE_LOG", "1")
    import torch
    from paper_2606_15437_amd import inputs as I
    from paper_2606_15437_amd import kripke as K

    if args.copy_mib:  # reference dispatch for the HBM byte counters
        torch.cuda.set_device(0)
        src = torch.ones(args.copy_mib << 18, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.only:
        torch.cuda.set_device(0)
        stream = torch.cuda.current_stream()
        if args.only == "mlp":
            leg = bench_mlp(stream)
        elif args.only == "split":
            leg = bench_split(args, stream)
        else:
            leg = bench_correspondence()
        leg.pop("_survivors", None)
        print(json.dumps({"only": args.only, args.only: leg}))
        return

    n, nvars = 5, 2
    nval = 1 << (n * nvars)
    fs = I.config3_formulas(args.formulas)
    B = len(fs)
    code, offs = I.pack(fs)
    src_bitops = float(sum(I.formula_stats(f, n)["bitops"] for f in fs))
    st = K.kripke_program_stats(code, offs, nvars)
    exe_bitops = float((n * st[:, 1] + n * n * st[:, 0]).sum())
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    calib = K.kripke_calibrate_int32(stream)
    log(f"INT32 VALU calibration: {calib / 1e12:.2f} T lane-ops/s "
        f"(nominal {PEAK_INT32 / 1e12:.2f})")

    # ---------------------------------------------------------- batched step
    t0 = time.time()
    plan = K.kripke_plan_create(code, offs, n, 0xF, nvars, tune_cache=args.tune_cache)
    log(f"plan (compile, class tables, autotune): {time.time() - t0:.1f} s")
    out = torch.empty((4, B, 2), dtype=torch.int64, device=dev)
    for i in range(args.warmup):
        ms_w = timed(lambda: K.kripke_plan_launch(plan, out, stream), stream)
        log(f"warmup {i}: {ms_w:.0f} ms")
    ms = timed(lambda: K.kripke_plan_launch(plan, out, stream), stream, args.steps)
    # formulas that fold to TOP or BOT are decided without evaluation (TOP is skipped,
    # BOT fails at world 0 of every model): only the others' triples are counted
    live = int((st[:, 5] == -1).sum())
    evals_step = float(live) * CLASS_FRAMES_N5[0] * nval
    evals_step_all = float(B) * CLASS_FRAMES_N5[0] * nval
    value = evals_step / (ms / 1e3)
    res = K.as_u64(out).copy()
    log(f"batched all-class step: {ms:.1f} ms, {value / 1e9:.0f} G evals/s")
    K.kripke_plan_destroy(plan)

    # the step is one init kernel (microseconds) plus the census kernel
    int_ops_exe = exe_bitops * CLASS_FRAMES_N5[0] * nval / 32.0
    int_ops_src = src_bitops * CLASS_FRAMES_N5[0] * nval / 32.0
    achieved = int_ops_exe / (ms / 1e3)
    log(f"roofline: {achieved / 1e12:.2f} T INT32 ops/s executed "
        f"({100 * achieved / PEAK_INT32:.1f}% of peak)")

    # ------------------------------------------------- unbatched baselines
    plain = None
    if not args.no_plain:
        plain = {"batched_ms": ms, "launches_batched": 1}
        for name, mask, cache in (("plain", 0xF | K.KRIPKE_PLAN_PLAIN, None),
                                  ("per_formula_autotuned", 0xF | K.KRIPKE_PLAN_PLAIN,
                                   args.tune_cache)):
            log(f"{name}: creating the per-formula plan"
                + (" (autotuned unless cached)" if cache else ""))
            t0 = time.time()
            pplan = K.kripke_plan_create(code, offs, n, mask, nvars, tune_cache=cache)
            create_s = time.time() - t0
            out2 = torch.empty((4, B, 2), dtype=torch.int64, device=dev)
            t0 = time.time()
            ms_p = timed(lambda: K.kripke_plan_launch(pplan, out2, stream), stream)
            host_s = time.time() - t0
            K.kripke_plan_destroy(pplan)
            same = bool((K.as_u64(out2) == res).all())
            plain[name] = {"ms": ms_p, "G_evals_per_s": evals_step / ms_p / 1e6,
                           "launches": (4 if cache is None else 1) * B,
                           "speedup_batched": ms_p / ms, "results_identical": same,
                           "host_s": host_s, "create_s": create_s}
            log(f"{name}: {ms_p:.0f} ms ({ms_p / ms:.2f}x the batched step), identical={same}")
        # the figures of the untuned form stay at the top level for continuity
        plain.update({k: plain["plain"][k] for k in ("ms", "G_evals_per_s", "launches",
                                                     "speedup_batched", "results_identical")})

    # ------------------------------------------- Table 1 matched workload
    t1 = I.parse(I.TABLE1_FORMULA)
    c1, o1 = I.pack([t1])
    r1 = torch.empty((1, 2), dtype=torch.int64, device=dev)
    run1 = lambda: K.kripke_census_range(c1, o1, n, 0, nvars, 0, I.TABLE1_FRAMES, 0, r1, stream)
    run1()
    ms1 = timed(run1, stream, 5)
    table1 = {"formula": I.TABLE1_FORMULA, "frames": I.TABLE1_FRAMES, "valuations": nval,
              "ms": ms1, "G_evals_per_s": I.TABLE1_FRAMES * nval / ms1 / 1e6,
              "fail_count": int(K.as_u64(r1)[0, 1]),
              "note": "includes host-side compile/upload of the one formula per call"}
    log(f"table-1 matched workload: {table1['G_evals_per_s']:.1f} G evals/s")

    # ---------------------------------------------------------- CPU oracle
    cpu = None if args.no_cpu else bench_cpu(fs)

    split = None if args.no_split else bench_split(args, stream)
    mlp = bench_mlp(stream)
    learned = None if args.no_learned else bench_learned()
    reproduction = None if args.no_reproduction else bench_reproduction()
    synthesis = bench_synthesis()
    correspondence = None if args.no_reproduction else bench_correspondence()
    survivors = split.pop("_survivors") if split else None
    adversarial = None if args.no_reproduction else bench_adversarial(survivors)

    valid = {name: int((res[c, :, 0] == K.NO_KEY).sum()) for c, name in enumerate("K T S4 S5".split())}
    rec = {
        "metric": "formula*frame*valuation G evals/s, n=5 census (batched hipGraph vs plain)",
        "value": value / 1e9,
        "value_counting_folded_formulas": evals_step_all / (ms / 1e3) / 1e9,
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
        "config": {"workload": "n=5 exhaustive census: 4,096 seeded formulas (length 3..40, "
                               "depth cap 0..6) x 33,554,432 frames x 1,024 valuations (2 vars), "
                               "classes K+T+S4+S5 fused in one graph-replayed launch",
                   "formulas": B, "n": n, "nvars": nvars, "evals_per_step": evals_step,
                   "evaluated_formulas": live,
                   "folded_formulas": {"TOP": int((st[:, 5] == 1).sum()),
                                       "BOT": int((st[:, 5] == 0).sum())},
                   "no_countermodel_per_class": valid},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_INT32 / 1e12,
                     "unit": "T INT32 ops/s", "frac": achieved / PEAK_INT32,
                     "traffic": recorded_traffic(),
                     "kernel": "census_fast<5,2,*,K,fused>",
                     "measured_int32_ceiling": calib / 1e12,
                     "frac_of_measured_ceiling": achieved / calib,
                     "executed_bitops_per_eval": exe_bitops / B,
                     "source_bitops_per_eval": src_bitops / B,
                     "source_formula_frac": int_ops_src / (ms / 1e3) / PEAK_INT32},
        "cpu_baseline": cpu,
        "plain_vs_batched": plain,
        "table1": table1,
        "split": split,
        "mlp_scoring": mlp,
        "learned": learned,
        "census_reproduction": reproduction,
        "active_synthesis": synthesis,
        "correspondence": correspondence,
        "adversarial": adversarial,
        "provenance": provenance(),
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
