"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2604_27058_amd.profiling stats DIR           kernel-trace --stats CSVs -> text table
    python -m paper_2604_27058_amd.profiling traffic FETCH_DIR WRITE_DIR COPY_BYTES WORKLOAD PREC OUT.json
        HBM bytes per launch of the sampling kernel from two --pmc runs
        (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), each scaled by the
        counter's reading for the plain copy kernel of COPY_BYTES bytes
        (bench.py --calibrate-copy), stamped with the kernel source hash.
"""
import csv
import glob
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAMPLING_KERNELS = ("k_sample", "k_frames", "k_batch", "clifft_frames_spec")


def code_tokens(text):
    """Source text without comments and with whitespace collapsed, so that
    documentation edits do not void counters taken on unchanged code."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


# Sources that decide what a kernel family executes: the device code and the
# host compiler that produces the instruction stream it runs.
FAMILY_SOURCES = {
    "interpreter": ("shot.h", "kernels.hip", "frames.hip", "batch.hip", "batch_kernel.h", "sample_f32.hip", "sample_f64.hip",
                    "kernels.h", "program.h", "philox.h", "compiler.cpp", "compiler.h"),
    "specialized": ("specialize.cpp", "spec_prelude.h", "spec_args.h", "program.h", "philox.h", "compiler.cpp",
                    "compiler.h"),
}


def kernel_family(kernel_name):
    return "specialized" if "clifft_frames_spec" in kernel_name else "interpreter"


def kernel_source_hash(family="interpreter", read=None):
    """Hash of the sources of one kernel family (comments and whitespace
    ignored)."""
    h = hashlib.sha256()
    for f in FAMILY_SOURCES[family]:
        text = read(f) if read else open(os.path.join(ROOT, "paper_2604_27058_amd", "csrc", f)).read()
        h.update(code_tokens(text).encode())
    return h.hexdigest()[:16]


def _csv(d, suffix):
    files = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not files:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    return list(csv.DictReader(open(files[0])))


def stats(d):
    rows = _csv(d, "kernel_stats.csv")
    out = ["%-72s %8s %14s %14s %7s" % ("kernel", "calls", "total_ns", "average_ns", "pct")]
    for r in rows:
        out.append("%-72s %8s %14s %14s %7.2f" % (r["Name"][:72], r["Calls"], r["TotalDurationNs"],
                                                   r["AverageNs"], float(r["Percentage"])))
    return "\n".join(out)


def _pmc(d, counter):
    rows = _csv(d, "counter_collection.csv")
    per = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        per.setdefault((r["Kernel_Name"], r["Dispatch_Id"]), 0.0)
        per[(r["Kernel_Name"], r["Dispatch_Id"])] += float(r["Counter_Value"])
    return per


def traffic(fetch_dir, write_dir, copy_bytes, workload, prec):
    batched = workload == "batched64"
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        per = _pmc(d, counter)
        # the calibration copy (the rate probes that bench also runs are not it)
        copy = [v for (k, _), v in per.items()
                if ("copy" in k.lower() or "elementwise" in k.lower()) and "probe" not in k.lower()]
        # the timed launch is the last sampling dispatch (earlier ones are the
        # launch-shape trials of the autotuner, if it ran); a batched step is
        # the last dispatch of each of its queue kernels
        samp = sorted(((int(d), k, v) for (k, d), v in per.items() if any(n in k for n in SAMPLING_KERNELS)))
        if batched:
            samp = [x for x in samp if "k_batch" in x[1]]
        if not copy or not samp:
            raise RuntimeError("missing copy or sampling dispatches for " + counter)
        kib_copy = max(copy)
        factor = kib_copy * 1024.0 / copy_bytes
        if batched:
            last = {}
            for _, k, v in samp:
                last[k] = v
            name, kib = " + ".join(sorted(last)), sum(last.values())
        else:
            _, name, kib = samp[-1]
        res[counter] = dict(kernel=name, kib_per_dispatch=kib, copy_kib=kib_copy, factor=factor,
                            bytes_per_launch=kib * 1024.0 / factor)
    family = kernel_family(res["FETCH_SIZE"]["kernel"])
    return dict(workload=workload, precision=prec, kernel_family=family, kernel_source_hash=kernel_source_hash(family),
                bytes_per_launch=res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"],
                fetch=res["FETCH_SIZE"], write=res["WRITE_SIZE"], copy_bytes=copy_bytes)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2]))
    elif sys.argv[1] == "traffic":
        d = traffic(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5], sys.argv[6])
        json.dump(d, open(sys.argv[7], "w"), indent=1)
        print(json.dumps(d))
