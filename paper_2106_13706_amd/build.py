"""Builds libddks.so (gfx950) in-tree with hipcc.

Every HIP/C++ source under csrc/ is compiled for gfx950 only, with packed
FP32 instructions disabled, then linked into one shared library next to
this file.  Objects go to csrc/_build/ and are rebuilt when their source or
any header changed.  The same sources are also compiled with
AddressSanitizer and UndefinedBehaviorSanitizer on their host code (the
device code as usual) into csrc/_build_hostsan/ and linked with the serving
stress driver tests/native/serve_stress.cpp into tests/native/serve_stress,
which a GPU test runs.
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


# host-side sanitizers only: each -fsanitize= goes to the host compilation
HOST_SANITIZE = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer".split()
BUILD_SAN = os.path.join(CSRC, "_build_hostsan")
STRESS_SRC = os.path.join(ROOT, "tests", "native", "serve_stress.cpp")
STRESS_EXE = os.path.join(ROOT, "tests", "native", "serve_stress")


def _compile(src, force, verbose, flags=None, outdir=None):
    flags = FLAGS if flags is None else flags
    outdir = BUILD if outdir is None else outdir
    obj = os.path.join(outdir, os.path.basename(src) + ".o")
    newest = max([os.path.getmtime(src)] + [os.path.getmtime(h) for h in _headers()])
    if not force and os.path.exists(obj) and os.path.getmtime(obj) >= newest:
        return obj
    lang = ["-x", "hip"]
    cmd = [HIPCC] + flags + lang + ["-c", src, "-o", obj + ".tmp"]
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


def build_stress(force: bool = True, verbose: bool = False, jobs: int = 8) -> str:
    """tests/native/serve_stress: the serving stress driver linked with the
    library's sources built with host-side AddressSanitizer and
    UndefinedBehaviorSanitizer (objects only on the link line: hipcc's
    "-x hip" would otherwise apply to them)."""
    os.makedirs(BUILD_SAN, exist_ok=True)
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-gline-tables-only"] + HOST_SANITIZE
    srcs = _sources() + [STRESS_SRC]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force, verbose, flags, BUILD_SAN), srcs))
    cmd = [HIPCC, f"--offload-arch={ARCH}"] + HOST_SANITIZE + ["-o", STRESS_EXE + ".tmp"] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link of the stress driver failed:\n" + r.stdout + r.stderr)
    os.replace(STRESS_EXE + ".tmp", STRESS_EXE)
    return STRESS_EXE


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
    build_stress(force, verbose, jobs)
    return OUT


if __name__ == "__main__":
    build(force="--incremental" not in sys.argv, verbose=True)
