"""Build libclifft.so (HIP kernels for gfx950 + host compiler + C-ABI runtime) in-tree."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libclifft.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", "-Wall", "-Wno-unused-result",
          "-I" + os.path.join(os.path.dirname(HERE), "include"), "-I" + os.path.join(HERE, "_build")]
# Packed FP32 VALU ops stay disabled in device code on this target.
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# The interpreter's instantiations are spread over several translation units
# so that they compile in parallel; the slowest ones are listed first.
SOURCES = [("sample_f32.hip", True), ("sample_f64.hip", True), ("trace_f32.hip", True), ("trace_f64.hip", True),
           ("sample_ext_f32.hip", True), ("sample_ext_f64.hip", True), ("batch_ext.hip", True),
           ("vsample_f32.hip", True), ("vsample_f64.hip", True),
           ("batch.hip", True), ("frames.hip", True), ("kernels.hip", True), ("probe.hip", True),
           ("runtime.cpp", True), ("specialize.cpp", True), ("compiler.cpp", False)]
# device text compiled at run time by the specialized-kernel generator
PRELUDE = ["philox.h", "spec_args.h", "spec_prelude.h"]


def _write_prelude():
    """Concatenates the run-time device headers into a C++ string literal."""
    parts = []
    for name in PRELUDE:
        for line in open(os.path.join(CSRC, name)):
            if line.startswith("#pragma once") or line.startswith("#include"):
                continue
            parts.append(line)
    text = "".join(parts)
    assert ")CLIFFT_PRELUDE\"" not in text
    out = os.path.join(HERE, "_build", "spec_prelude.inc")
    with open(out + ".tmp", "w") as f:
        f.write('R"CLIFFT_PRELUDE(' + text + ')CLIFFT_PRELUDE"\n')
    os.replace(out + ".tmp", out)


def _obj(name):
    return os.path.join(HERE, "_build", name + ".o")


def _compile(item):
    name, hip = item
    src = os.path.join(CSRC, name)
    cmd = [HIPCC] + COMMON + (DEVICE + ["-x", "hip"] if name.endswith(".hip") else []) + ["-c", src, "-o", _obj(name)]
    if not hip:
        cmd = ["g++"] + COMMON + ["-c", src, "-o", _obj(name)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return r.stderr


def build(verbose=False):
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    _write_prelude()
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        logs = list(ex.map(_compile, SOURCES))
    if verbose:
        for l in logs:
            if l.strip():
                print(l, file=sys.stderr)
    cmd = ([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", LIB + ".tmp"] + [_obj(n) for n, _ in SOURCES]
           + ["-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"])
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
