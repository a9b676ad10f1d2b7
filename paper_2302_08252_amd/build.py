"""Build libadept.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled with -ffp-contract=off (no FMA contraction,
so binary64/binary32 results follow source order) and with packed-FP32
instructions disabled.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libadept.so")
ARCH = os.environ.get("ADEPT_OFFLOAD_ARCH", "gfx950")

SOURCES = ["capi.hip", "inst_dense_f64.hip", "inst_dense_mixed.hip", "inst_sparse_f64.hip", "inst_sparse_mixed.hip",
           "inst_typed.hip"]
HEADERS = ["kernels.hpp", "layout.hpp", "model.hpp", os.path.join("..", "..", "include", "adept.h")]
# -amdgpu-sched-strategy=max-ilp: the backend's instruction scheduler set to maximise
# instruction-level parallelism within a wavefront (measured: the step kernel 0.6 % faster on
# 10^5 e- x 10 GeV, 0.9 % on the 512-event workload; the default and max-memory-clause tie)
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mllvm", "-amdgpu-sched-strategy=max-ilp",
    "-Wall", "-Wno-unused-function",
]


def _newest(paths):
    return max(os.path.getmtime(p) for p in paths)


def build(force=True, jobs=None, verbose=False, defines=(), lib_path=LIB, build_dir=BUILD):
    """Compile every HIP translation unit and link libadept.so.  With force=False
    an up-to-date library is kept.  defines: extra -D tuning or diagnostic macros
    (ADEPT_WAVES_PER_EU, ADEPT_NT, ADEPT_PHASE_CLOCKS), with lib_path / build_dir
    for a separate build."""
    LIB_OUT, BDIR = lib_path, build_dir
    os.makedirs(BDIR, exist_ok=True)
    hdr = _newest([os.path.join(CSRC, h) for h in HEADERS])
    if not force and os.path.exists(LIB_OUT):
        if os.path.getmtime(LIB_OUT) >= max(hdr, _newest([os.path.join(CSRC, s) for s in SOURCES])):
            return LIB_OUT

    def compile_one(src):
        obj = os.path.join(BDIR, src.replace(".hip", ".o"))
        cmd = ["hipcc", *FLAGS, *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True, cwd=BDIR)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        if verbose:
            sys.stderr.write(r.stderr)
        return obj

    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB_OUT + ".tmp"
    r = subprocess.run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True, cwd=BDIR)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB_OUT)
    return LIB_OUT


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description="build libadept.so for gfx950")
    ap.add_argument("--if-stale", action="store_true", help="keep an up-to-date library")
    ap.add_argument("-v", action="store_true", help="show compiler output")
    ap.add_argument("--define", action="append", default=[], metavar="NAME=VALUE",
                    help="tuning / diagnostic macro, e.g. ADEPT_PHASE_CLOCKS=1 (with --out)")
    ap.add_argument("--out", default=None, help="library path of a separate build (its objects go next to it)")
    a = ap.parse_args()
    if a.define and not a.out:
        ap.error("--define needs --out: the in-tree library stays the plain build")
    out = os.path.abspath(a.out) if a.out else LIB
    bdir = os.path.join(os.path.dirname(out), "_build") if a.out else BUILD
    os.makedirs(os.path.dirname(out), exist_ok=True)
    print(build(force=not a.if_stale, verbose=a.v, defines=a.define, lib_path=out, build_dir=bdir))
