"""Build libswf.so (gfx950) in-tree with hipcc.

Every HIP source is compiled with ``-Xclang -target-feature -Xclang
-packed-fp32-ops`` so the compiler never emits packed FP32 instructions.
The per-size kernel instantiations are compiled in parallel.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libswf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
N_GROUPS = 9

FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(HERE, "..", "include"), "-I", CSRC]


def source_hash() -> str:
    """sha256 over the HIP/C++ sources (sorted by name): identifies the kernels
    a stored profile was taken from."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".h", ".hip", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def _jobs():
    units = [("swf_api.cpp", [], "swf_api.o"), ("swf_table.cpp", [], "swf_table.o"),
             ("swf_reduce.hip", [], "swf_reduce.o"), ("swf_pair.hip", [], "swf_pair.o")]
    for real, tag in (("float", "f32"), ("double", "f64")):
        for g in range(N_GROUPS):
            units.append(("swf_sizes.hip", [f"-DSWF_REAL={real}", f"-DSWF_TAG={tag}", f"-DSWF_GROUP={g}"],
                          f"swf_sizes_{tag}_{g}.o"))
    return units


def _compile(unit):
    import time
    src, defs, obj = unit
    cmd = [HIPCC] + FLAGS + defs + ["-c", os.path.join(CSRC, src), "-o", os.path.join(OUT, obj)]
    t0 = time.time()
    p = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (p.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    if os.environ.get("SWF_BUILD_TIMES"):
        print(f"{obj}: {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    return obj, p.returncode, err


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every source and link libswf.so; returns the library path."""
    os.makedirs(OUT, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    units = _jobs()
    # the slow instantiation units first
    units.sort(key=lambda u: 0 if "sizes" in u[2] else 1)
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, units))
    bad = [(o, e) for o, rc, e in results if rc != 0]
    if bad:
        msg = "\n".join(f"--- {o}\n{e}" for o, e in bad)
        raise RuntimeError(f"hipcc failed:\n{msg}")
    if verbose:
        for o, _, e in results:
            if e.strip():
                print(f"--- {o}\n{e}", file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
        [os.path.join(OUT, u[2]) for u in units]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
