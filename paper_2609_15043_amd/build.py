"""Build libphasorpic.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["api.hip", "particles.hip", "fields.hip", "direct.hip", "circuit.hip", "mlp.hip"]
LIB = os.path.join(HERE, "libphasorpic.so")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.exists(c) or c == "hipcc"):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False, arch="gfx950"):
    csrc = os.path.join(HERE, "csrc")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-shared",
           # no packed FP32 (v_pk_*_f32) instructions in the generated code
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           # every atomic in these kernels is already issued by one lane per
           # wave after an explicit wave reduction; the compiler's own
           # atomic scan would only add instructions
           "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
           "-o", tmp] + [os.path.join(csrc, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
