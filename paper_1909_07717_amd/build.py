"""Build libdpps.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdpps.so")
ARCH = os.environ.get("DPPS_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no automatic contraction: explicit fmaf only, so results do not depend
    # on how a function was inlined
    "-ffp-contract=off",
    # packed FP32 instructions stay off on the test machines
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{os.path.join(ROOT, 'include')}",
]
# Device code of the kernels carries no NaN through any compared or selected
# value (inputs are validated on the host); without NaN semantics min/max
# need no quieting of their operands.  Host code keeps full IEEE semantics.
SOURCES = {
    "dpps_api.hip": [],
    "dpps_kernels.hip": ["-Xarch_device", "-fno-honor-nans", "-Xarch_device", "-mno-amdgpu-ieee"],
    "dpps_noalloc.hip": [],
    "mlp_api.hip": [],
    "mlp_kernels.hip": [],
}


def kernel_rev() -> str:
    """Short hash of the search kernels' sources, compiled into the library so
    that cached launch shapes tuned on other kernels are not reused."""
    h = hashlib.sha256()
    for f in ("dpps_kernels.hip", "dpps_internal.h"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def hipcc() -> str:
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError(f"hipcc failed: {' '.join(cmd)}")
    return out


def build(verbose: bool = False, extra: list[str] | None = None, out: str | None = None,
          link_extra: list[str] | None = None) -> str:
    """Compile every source and link libdpps.so, or `out` (always recompiles)."""
    lib_path = out or LIB
    rev = [f'-DDPPS_KERNEL_REV="{kernel_rev()}"']
    with tempfile.TemporaryDirectory() as td:
        objs = []
        for src, flags in SOURCES.items():
            obj = os.path.join(td, src + ".o")
            _run([hipcc()] + COMMON + flags + rev + (extra or []) +
                 ["-c", os.path.join(CSRC, src), "-o", obj], verbose)
            objs.append(obj)
        tmp = lib_path + ".tmp"
        _run([hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs +
             (link_extra or []), verbose)
        os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    print(build(verbose=True))
