"""Builds libddks.so (gfx950) in-tree with hipcc.

Every HIP/C++ source under csrc/ is compiled for gfx950 only, with packed
FP32 instructions disabled, then linked into one shared library next to
this file.  Objects go to csrc/_build/ and are rebuilt when their source or
any header changed.
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libddks.so")
BUILD = os.path.join(CSRC, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _headers():
    return glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(ROOT, "include", "*.h"))


def _compile(src, force, verbose):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    newest = max([os.path.getmtime(src)] + [os.path.getmtime(h) for h in _headers()])
    if not force and os.path.exists(obj) and os.path.getmtime(obj) >= newest:
        return obj
    lang = ["-x", "hip"]
    cmd = [HIPCC] + FLAGS + lang + ["-c", src, "-o", obj + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    if verbose and msg.strip():
        print(msg, flush=True)
    os.replace(obj + ".tmp", obj)
    return obj


PROBES = os.path.join(HERE, "probes")


def build_probes(verbose: bool = False) -> list:
    """Compiles each probes/*.hip (a standalone measurement program, not part
    of the library) into an executable beside it."""
    out = []
    for src in sorted(glob.glob(os.path.join(PROBES, "*.hip"))):
        exe = src[:-len(".hip")]
        cmd = [HIPCC, "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-Wall",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", src, "-o", exe + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}{r.stderr}")
        os.replace(exe + ".tmp", exe)
        out.append(exe)
    return out


def build(force: bool = True, verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force, verbose), srcs))
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", OUT + ".tmp"] + objs + [
        "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(OUT + ".tmp", OUT)
    build_probes(verbose)
    return OUT


if __name__ == "__main__":
    build(force="--incremental" not in sys.argv, verbose=True)
