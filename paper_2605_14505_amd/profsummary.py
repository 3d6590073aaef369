"""Summarise rocprofv3 CSV output of a bench.py run into the short text files kept in profiles/.

    python -m paper_2605_14505_amd.profsummary --key KEY --cmd "..." \
        --trace DIR [--fetch DIR --write DIR --copy-bytes N --n N --bytes-per-node B]

--trace: a `rocprofv3 --kernel-trace --stats --output-format csv` output folder;
writes profiles/KEY_kernel_stats.txt (per-kernel calls and durations).
--fetch / --write: `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` folders of the
same command; writes profiles/KEY_counters.txt with the HBM bytes per launch of
the step kernels.  Each counter is scaled by what it reads for the streaming
copy kernel, which moves a known number of bytes (--copy-bytes read and as many
written per launch), and the summary records the hash of the kernel sources it
was taken on so that bench.py can tell when it no longer applies.
"""
import argparse
import csv
import glob
import hashlib
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


# the sources the step kernels are compiled from (the profiled kernels)
STEP_SOURCES = ("stencil.hpp", "lbm_device.hpp", "mlp_device.hpp", "lbm_kernels.hpp", "lbm_launch.hpp",
                "lbm_instances.hpp", "lbm_fp32.hip", "lbm_fp16.hip", "lbm_bf16.hip", "learned_step.hip")


def code_only(src):
    """C++ source without its comments and with every whitespace run made one space, so that
    a hash of it follows the code the kernels are compiled from, not the comments.  (None of
    the hashed sources has a comment marker inside a string literal.)"""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_source_hash():
    csrc = os.path.join(ROOT, "paper_2605_14505_amd", "csrc")
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        h.update(f.encode())
        h.update(code_only(open(os.path.join(csrc, f), encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def _one(pattern):
    hits = glob.glob(pattern)
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def kernel_stats(trace_dir):
    rows = list(csv.DictReader(open(_one(os.path.join(trace_dir, "*kernel_stats.csv")))))
    out = []
    for r in rows:
        out.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                    float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return out


def counter_table(pmc_dir):
    """{kernel: {counter: mean value per dispatch}} of one rocprofv3 --pmc run."""
    rows = list(csv.DictReader(open(_one(os.path.join(pmc_dir, "*counter_collection.csv")))))
    agg = {}
    for r in rows:
        agg.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in agg.items()}


def counter_means(pmc_dir):
    """{kernel: mean value per dispatch} of a run that collected one counter."""
    return {k: next(iter(cs.values())) for k, cs in counter_table(pmc_dir).items()}


def is_step_kernel(name):
    return "lbm_step_kernel" in name or "lbm_step_ring_kernel" in name


def is_plain_step(name):
    """A time step without diagnostic outputs: FLAGS == 1 (the last template argument, in
    the demangled or the mangled name), or the row-aligned odd step, which has no flags."""
    if "lbm_step_ring_kernel" in name:
        return True
    m = re.search(r"lbm_step_kernel<[^>]*, (\d+)>\(", name) or re.search(r"lbm_step_kernelI.*ELi(\d+)EEEv", name)
    return bool(m) and m.group(1) == "1"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--key", required=True)
    ap.add_argument("--cmd", required=True, help="the command that produced the folders")
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-bytes", type=int)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--bytes-per-node", type=int, default=368)
    ap.add_argument("--note", default="")
    ap.add_argument("--pmc", action="append", default=[],
                    help="further --pmc folders of the same command: their counters per kernel "
                         "go to profiles/KEY_pmc.txt")
    ap.add_argument("--match", default="", help="only kernels whose name contains this in KEY_pmc.txt")
    a = ap.parse_args()
    os.makedirs(PROFILES, exist_ok=True)
    if a.trace:
        path = os.path.join(PROFILES, f"{a.key}_kernel_stats.txt")
        with open(path, "w") as fh:
            fh.write(f"# rocprofv3 --kernel-trace --stats summary\n# command: {a.cmd}\n")
            fh.write(f"# kernel sources: {kernel_source_hash()}\n")
            if a.note:
                fh.write(f"# {a.note}\n")
            fh.write(f"{'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}  kernel\n")
            for name, calls, avg, mn, mx, pct in kernel_stats(a.trace):
                fh.write(f"{calls:6d} {avg:10.2f} {mn:10.2f} {mx:10.2f} {pct:6.2f}  {name[:150]}\n")
        print("wrote", path)
    if a.fetch and a.write:
        fetch, write = counter_means(a.fetch), counter_means(a.write)
        copy = [k for k in fetch if "bw_copy_kernel" in k][0]
        kib = a.copy_bytes / 1024.0
        f_scale, w_scale = kib / fetch[copy], kib / write[copy]
        steps = [k for k in fetch if is_step_kernel(k) and k in write]
        n3 = a.n ** 3
        path = os.path.join(PROFILES, f"{a.key}_counters.txt")
        with open(path, "w") as fh:
            fh.write("# rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE (two runs), KiB per dispatch\n")
            fh.write(f"# command: {a.cmd}\n")
            fh.write(f"# copy kernel {copy[:60]}: FETCH {fetch[copy]:.1f} KiB, WRITE {write[copy]:.1f} KiB "
                     f"for {kib:.1f} KiB moved each way -> scale fetch x{f_scale:.4f}, write x{w_scale:.4f}\n")
            if a.note:
                fh.write(f"# {a.note}\n")
            algo = a.bytes_per_node * n3
            plain = []
            for k in steps:
                fb, wb = fetch[k] * f_scale * 1024, write[k] * w_scale * 1024
                fh.write(f"# {k[:110]}\n#   fetch {fb / 1e9:.4f} GB  write {wb / 1e9:.4f} GB  "
                         f"total/algorithmic {(fb + wb) / algo:.4f}\n")
                if is_plain_step(k):
                    plain.append(fb + wb)
            per_launch = sum(plain) / len(plain) if plain else float("nan")
            fh.write(f"source_hash = {kernel_source_hash()}\n")
            fh.write(f"algorithmic_bytes_per_launch = {algo}\n")
            fh.write(f"hbm_bytes_per_launch = {per_launch:.0f}\n")
            fh.write(f"fetch_scale = {f_scale:.5f}\nwrite_scale = {w_scale:.5f}\n")
        print("wrote", path)
    if a.pmc:
        table = {}
        for d in a.pmc:
            for k, cs in counter_table(d).items():
                table.setdefault(k, {}).update(cs)
        path = os.path.join(PROFILES, f"{a.key}_pmc.txt")
        with open(path, "w") as fh:
            fh.write("# rocprofv3 --pmc counters, mean per dispatch (one run per counter set)\n")
            fh.write(f"# command: {a.cmd}\n# kernel sources: {kernel_source_hash()}\n")
            if a.note:
                fh.write(f"# {a.note}\n")
            for k in sorted(table):
                if a.match and a.match not in k:
                    continue
                fh.write(f"{k[:150]}\n")
                for c in sorted(table[k]):
                    fh.write(f"  {c} = {table[k][c]:.6g}\n")
        print("wrote", path)


if __name__ == "__main__":
    main()
