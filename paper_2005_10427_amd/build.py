"""Compile libqsd.so for gfx950 with hipcc (cross-compiles without a GPU).

Each source is compiled to an object in parallel (the digit-pass kernels are split by
coordinate/value type into separate translation units), then linked into one shared
library in-tree.
"""
import concurrent.futures
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqsd.so")

SOURCES = ["api.cpp", "plan.cpp", "select.cpp", "kernels.hip", "select_kernels.hip", "digit_u32_u64.hip",
           "digit_u32_u32.hip", "digit_u64_u64.hip", "digit_u64_u32.hip", "noalloc.hip", "csf_kernels.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CFLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # keep the compiler from emitting packed fp32 instructions (host pass ignores it)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def _compile(src, obj, extra=()):
    cmd = [HIPCC] + CFLAGS + list(extra) + ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n" + res.stdout + res.stderr)
    return obj


def build(verbose=False, jobs=None, extra_flags=(), out=LIB):
    """Compile every source and link `out` (the in-tree library by default); `extra_flags` are
    added to every compile (e.g. -D overrides of tuning constants)."""
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1))
    with tempfile.TemporaryDirectory(prefix="qsd_build_") as tmp:
        objs = [os.path.join(tmp, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
            futs = [ex.submit(_compile, s, o, extra_flags) for s, o in zip(SOURCES, objs)]
            for f in futs:
                f.result()
        out_tmp = out + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", out_tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(out_tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
