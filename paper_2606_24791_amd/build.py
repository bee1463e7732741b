"""Build liblamg.so (the HIP library behind include/lamg.h) for gfx950 with hipcc.

Setup sources are compiled with -ffp-contract=off (canonical, reproducible setup
arithmetic); the cycle kernels use the compiler's default contraction. Packed FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
INCLUDE = ROOT / "include"
LIB = PKG / "liblamg.so"
BUILD = ROOT / "_build"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", f"-I{INCLUDE}", f"-I{CSRC}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]
SOURCES = {
    "setup_kernels.hip": ["-ffp-contract=off"],
    "setup.cpp": ["-ffp-contract=off", "-x", "hip"],
    "cycle_kernels.hip": [],
    "tail_kernel.hip": [],
    "solve.cpp": ["-x", "hip"],
    "api.cpp": ["-x", "hip"],
    "noalloc.cpp": ["-x", "hip"],
}


def _deps(path: Path, seen: set) -> set:
    """The file and the local headers it includes, transitively."""
    if path in seen or not path.exists():
        return seen
    seen.add(path)
    for line in path.read_text().splitlines():
        line = line.strip()
        if line.startswith("#include \""):
            name = line.split('"')[1]
            for d in (CSRC, INCLUDE):
                _deps(d / name, seen)
    return seen


def _stale(src: str, obj: Path) -> bool:
    """Whether obj is older than its source or a local header it includes."""
    if not obj.exists():
        return True
    t = obj.stat().st_mtime
    return any(d.stat().st_mtime > t for d in _deps(CSRC / src, set()))


def _compile(src: str, flags: list[str], changed_only: bool = False) -> Path:
    obj = BUILD / (src + ".o")
    if changed_only and not _stale(src, obj):
        return obj
    cmd = [HIPCC, *COMMON, *flags, "-c", str(CSRC / src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, changed_only: bool = False) -> Path:
    """Compile every source (with changed_only: those whose object is older than the source
    or a header) and link liblamg.so in the package directory."""
    BUILD.mkdir(exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda kv: _compile(*kv, changed_only), SOURCES.items()))
    tmp = LIB.with_suffix(f".so.tmp{os.getpid()}")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True, changed_only="--changed" in sys.argv)
