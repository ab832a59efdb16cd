"""Build the HIP library ``libet.so`` for gfx950 with hipcc.

Every HIP translation unit under ``csrc/`` is compiled to an object in a
build folder next to this file and linked into ``libet.so`` in the package
directory, where the Python binding loads it.

The random-access ceiling probe (``probe/ceiling.hip``) is a standalone
measurement program that does not use the library; the library build does
not touch it. ``python paper_2103_15217_amd/build.py probe`` (or
:func:`build_probe`) builds it next to its source.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libet.so")
PROBE_SRC = os.path.join(HERE, "probe", "ceiling.hip")
PROBE = os.path.join(HERE, "probe", "ceiling")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
ARCH = os.environ.get("ET_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-I", INCLUDE,
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r


def build(verbose=False):
    """Compile every .hip unit and link libet.so; raises on failure."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    errors = []
    for src, _, r in results:
        noise = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if r.returncode != 0:
            errors.append(f"{os.path.basename(src)}:\n{r.stderr}")
        elif verbose and noise:
            print("\n".join(noise), file=sys.stderr)
    if errors:
        raise RuntimeError("hipcc failed\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
           *[obj for _, obj, _ in results]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def build_probe():
    """Build the random-access ceiling probe (measurement only)."""
    tmp = PROBE + ".tmp"
    r = subprocess.run([HIPCC, *FLAGS, PROBE_SRC, "-o", tmp], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("probe build failed\n" + r.stderr)
    os.replace(tmp, PROBE)
    return PROBE


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "probe":
        print(build_probe())
    else:
        print(build(verbose=True))
