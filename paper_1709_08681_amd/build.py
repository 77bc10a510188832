"""Build libpsc.so (HIP, gfx950) in-tree with hipcc: each source compiled to
an object in parallel, then linked."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpsc.so")
SOURCES = ["psc_api.hip", "psc_kernels.hip", "psc_window.hip", "psc_grid.hip", "psc_aperture.hip", "psc_scale.hip"]
ARCH = os.environ.get("PSC_OFFLOAD_ARCH", "gfx950")
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", "-Wall",
         # no packed FP32 instructions in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc_command(out=LIB, extra=()):
    """One hipcc line that compiles and links every source (for reference)."""
    return ["hipcc", *FLAGS, "-shared", *extra, "-o", out] + [os.path.join(CSRC, s) for s in SOURCES]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass warns about the device-only target feature; that is harmless
    errs = [ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln]
    return res.returncode, errs


def build(verbose=False, extra=()):
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    with tempfile.TemporaryDirectory(prefix="psc_build_") as d:
        objs = [os.path.join(d, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [["hipcc", *FLAGS, *extra, "-c", "-o", o, os.path.join(CSRC, s)] for s, o in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(jobs) as pool:
            results = list(pool.map(_run, cmds))
        failed = [(s, errs) for s, (rc, errs) in zip(SOURCES, results) if rc != 0]
        if failed:
            for s, errs in failed:
                sys.stderr.write(f"{s}:\n" + "\n".join(errs) + "\n")
            raise RuntimeError("hipcc failed building libpsc.so")
        if verbose:
            for s, (_, errs) in zip(SOURCES, results):
                if errs:
                    sys.stderr.write(f"{s}:\n" + "\n".join(errs) + "\n")
        tmp = LIB + ".tmp%d" % os.getpid()
        rc, errs = _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, "-o", tmp, *objs])
        if rc != 0:
            sys.stderr.write("\n".join(errs) + "\n")
            raise RuntimeError("hipcc failed linking libpsc.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=tuple(sys.argv[1:]))
