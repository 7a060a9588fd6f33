"""Build the HIP library ``libsfhk.so`` (gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsfhk.so")
ARCH = os.environ.get("SFHK_OFFLOAD_ARCH", "gfx950")

# -ffp-contract=off: the trajectory arithmetic is an explicit sequence of IEEE operations and
# fused multiply-adds; the compiler must not fuse anything else. Packed FP32 instructions are
# disabled for every kernel.
HIPCC_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
               "-ffp-contract=off", "-fno-fast-math", "-munsafe-fp-atomics",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument",
               # roctx ranges around the host API calls
               "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    src = os.path.join(CSRC, "sfhk.hip")
    tmp = out + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, *[f"-D{d}" for d in defines], "-o", tmp, src]
    r = subprocess.run(cmd, capture_output=True, text=True)
    log = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{log}")
    if verbose and log.strip():
        print(log, file=sys.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
