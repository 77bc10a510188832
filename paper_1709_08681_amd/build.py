"""Build libpsc.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpsc.so")
SOURCES = ["psc_api.hip", "psc_kernels.hip", "psc_window.hip", "psc_grid.hip", "psc_aperture.hip", "psc_scale.hip"]
ARCH = os.environ.get("PSC_OFFLOAD_ARCH", "gfx950")


def hipcc_command(out=LIB, extra=()):
    return ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-fvisibility=hidden", "-Wall",
            # no packed FP32 instructions in device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            *extra, "-o", out] + [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose=False, extra=()):
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = hipcc_command(tmp, extra)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass warns about the device-only target feature; that is harmless
    errs = [ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln]
    if res.returncode != 0:
        sys.stderr.write("\n".join(errs) + "\n")
        raise RuntimeError("hipcc failed building libpsc.so")
    if verbose and errs:
        sys.stderr.write("\n".join(errs) + "\n")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=tuple(sys.argv[1:]))
