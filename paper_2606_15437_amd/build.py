"""Build libkripke.so in-tree with hipcc for gfx950 (cross-compiles without a GPU)."""
import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libkripke.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["census_kernels.hip", "fast_kernels.hip", "calibrate.hip", "pair_kernels.hip",
           "mlp_kernels.hip", "worldmask_kernels.hip", "kripke_api.hip",
           "kripke_compile.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed-FP32 instructions are disabled for all device code.
# The interpreters dispatch on wave-uniform opcodes; letting the structurizer
# skip uniform regions keeps their switch from being rewritten into flow
# blocks full of register copies.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-structurizecfg-skip-uniform-regions=true"]


def _stale(src: str, obj: str) -> bool:
    """An object is stale if it is older than its source or any header in csrc or include."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    inc = os.path.join(os.path.dirname(HERE), "include")
    deps = [os.path.join(CSRC, src)] + [os.path.join(d, h) for d in (CSRC, inc)
                                        for h in os.listdir(d) if h.endswith(".h")]
    return any(os.path.getmtime(d) > t for d in deps)


def _compile(src: str, verbose: bool, force: bool = True) -> str:
    obj = os.path.join(OBJDIR, src + ".o")
    if not force and not _stale(src, obj):
        return obj
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "c++"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile every source (force=False: only stale objects) and link the library."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, force), srcs))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


def resources(out_path: str, sources=None) -> str:
    """Per-kernel register, scratch and occupancy figures as the compiler reports them
    (device-only compile of each source with kernel resource-usage remarks), written as
    a markdown table to out_path."""
    import re
    srcs = [s for s in (sources or SOURCES) if s.endswith(".hip")]
    fields = ("TotalSGPRs", "VGPRs", "AGPRs", "ScratchSize [bytes/lane]", "LDS Size [bytes/block]",
              "Occupancy [waves/SIMD]")

    def one(src):
        cmd = [HIPCC, *FLAGS, "--cuda-device-only", "-Rpass-analysis=kernel-resource-usage",
               "-c", os.path.join(CSRC, src), "-o", os.devnull]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        rows, cur = [], None
        for line in r.stderr.splitlines():
            m = re.search(r"remark: Function Name: (\S+)", line)
            if m:
                cur = {"src": src, "name": m.group(1)}
                rows.append(cur)
                continue
            m = re.search(r"remark:\s+([^:]+): (\S+) \[-Rpass-analysis", line)
            if m and cur is not None and m.group(1).strip() in fields:
                cur[m.group(1).strip()] = m.group(2)
        return rows

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        rows = [r for part in ex.map(one, srcs) for r in part]
    names = subprocess.run(["c++filt"], input="\n".join(r["name"] for r in rows),
                           capture_output=True, text=True).stdout.splitlines()
    lines = ["| source | kernel | VGPRs | AGPRs | SGPRs | scratch B/lane | LDS B/block | "
             "waves/SIMD |", "|---|---|---|---|---|---|---|---|"]
    # library (rocPRIM/hipCUB) instantiations: one summary row per source, not one per
    # template instance
    lib = {}
    for r, nm in zip(rows, names):
        if "rocprim::" in nm or "hipcub::" in nm:
            d = lib.setdefault(r["src"], {"count": 0, "vgpr": 0, "sgpr": 0, "scratch": 0})
            d["count"] += 1
            for key, field in (("vgpr", "VGPRs"), ("sgpr", "TotalSGPRs"),
                               ("scratch", "ScratchSize [bytes/lane]")):
                try:
                    d[key] = max(d[key], int(r.get(field, 0)))
                except ValueError:
                    pass
    for r, nm in zip(rows, names):
        if "rocprim::" in nm or "hipcub::" in nm:
            continue
        nm = nm.replace("kripke::", "").replace("(anonymous namespace)::", "")
        nm = nm.replace("|", "\\|")
        lines.append(f"| {r['src']} | `{nm}` | {r.get('VGPRs', '?')} | {r.get('AGPRs', '?')} | "
                     f"{r.get('TotalSGPRs', '?')} | {r.get('ScratchSize [bytes/lane]', '?')} | "
                     f"{r.get('LDS Size [bytes/block]', '?')} | "
                     f"{r.get('Occupancy [waves/SIMD]', '?')} |")
    for src, d in sorted(lib.items()):
        lines.append(f"| {src} | {d['count']} rocPRIM/hipCUB sort and scan instantiations "
                     f"(maxima over them) | {d['vgpr']} | — | {d['sgpr']} | {d['scratch']} | "
                     f"— | — |")
    with open(out_path, "w") as fh:
        fh.write("# Kernel resources (compiler resource-usage remarks, gfx950)\n\n"
                 "Command: `python paper_2606_15437_amd/build.py --resources "
                 "profiles/kernel_resources.md` (device-only compile of every HIP source with "
                 "`-Rpass-analysis=kernel-resource-usage` and the library's flags).\n\n")
        fh.write("\n".join(lines) + "\n")
    return out_path


if __name__ == "__main__":
    import sys
    if "--resources" in sys.argv:
        print(resources(sys.argv[sys.argv.index("--resources") + 1]))
    else:
        print(build(verbose=True, force="--changed" not in sys.argv))
