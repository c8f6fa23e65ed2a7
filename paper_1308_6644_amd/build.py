"""Build libnuasm.so (the gfx950 kernels and the C ABI) in-tree with hipcc.

Usage: python -m paper_1308_6644_amd.build [--jobs N] [--verbose] [--sanitized]

--sanitized builds, in addition, a copy of the library whose host code is
instrumented with AddressSanitizer and UndefinedBehaviorSanitizer (the kernels
are not: every sanitizer flag is passed through -Xarch_host) together with the
C-ABI driver of tests/abi_driver.cpp, both under sanitized/ in the package.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libnuasm.so")
SAN_DIR = os.path.join(PKG, "sanitized")
SAN_LIB = os.path.join(SAN_DIR, "libnuasm.so")
SAN_DRIVER = os.path.join(SAN_DIR, "abi_driver")
DRIVER_SRC = os.path.join(ROOT, "tests", "abi_driver.cpp")

SOURCES = ["nuasm.hip", "k_fft.hip", "k_points.hip", "k_rs.hip", "k_grid.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
        # no packed-FP32 instructions in any kernel
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # matrix-core accumulators in ordinary VGPRs, updated in place (the
        # accumulation-register form copies them around the spreading loop)
        "-mllvm", "-amdgpu-mfma-vgpr-form",
        "-I", INCLUDE, "-I", CSRC,
    ]


def sanitizer_flags() -> list[str]:
    """Host-side ASan + UBSan; device code is compiled as usual."""
    flags = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer",
              "-fno-sanitize-recover=undefined", "-g"):
        flags += ["-Xarch_host", f]
    return flags


def _compile(src: str, verbose: bool, sanitized: bool = False) -> str:
    out_dir = os.path.join(BUILD_DIR, "sanitized") if sanitized else BUILD_DIR
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    flags = compile_flags()
    if sanitized:  # -O1 keeps sanitizer reports readable and halves the build time
        flags = ["-O1" if f == "-O3" else f for f in flags] + sanitizer_flags()
    cmd = [hipcc(), *flags, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def build(jobs: int = 4, verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link libnuasm.so in-tree."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def _run(cmd: list[str], verbose: bool, what: str) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{what} failed:\n{r.stdout}\n{r.stderr}")


def sanitized_sources() -> list[str]:
    """Every file the sanitized build depends on."""
    hdrs = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".h")]
    return ([os.path.join(CSRC, s) for s in SOURCES] + hdrs
            + [os.path.join(INCLUDE, "nuasm.h"), DRIVER_SRC, os.path.abspath(__file__)])


SAN_STAMP = os.path.join(SAN_DIR, "sources.sha256")


def sanitized_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in sanitized_sources():
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def sanitized_stale() -> bool:
    """True unless the sanitized build exists and was made from the current
    sources (compared by content, so copies of the tree keep it valid)."""
    if not all(os.path.exists(f) for f in (SAN_LIB, SAN_DRIVER, SAN_STAMP)):
        return True
    with open(SAN_STAMP) as fh:
        return fh.read().strip() != sanitized_sources_hash()


def build_sanitized(jobs: int = 5, verbose: bool = False) -> str:
    """The host-sanitized library and the C-ABI driver linked against it.

    The driver finds the library through its run path ($ORIGIN), so it runs
    from wherever the package is, with the ASan runtime loaded first (the
    driver itself is linked with -fsanitize=address)."""
    os.makedirs(os.path.join(BUILD_DIR, "sanitized"), exist_ok=True)
    os.makedirs(SAN_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, sanitized=True), SOURCES))
    san_link = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    tmp = SAN_LIB + ".tmp"
    stamp = sanitized_sources_hash()
    _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *san_link, "-o", tmp, *objs],
         verbose, "sanitized link")
    os.replace(tmp, SAN_LIB)
    tmp = SAN_DRIVER + ".tmp"
    _run([hipcc(), "-O1", "-std=c++17", *sanitizer_flags(), "-I", INCLUDE, DRIVER_SRC,
          "-o", tmp, "-L", SAN_DIR, "-lnuasm", "-Wl,-rpath,$ORIGIN"], verbose, "driver build")
    os.replace(tmp, SAN_DRIVER)
    with open(SAN_STAMP, "w") as fh:
        fh.write(stamp + "\n")
    return SAN_DRIVER


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--sanitized", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.verbose))
    if a.sanitized:
        print(build_sanitized(max(a.jobs, 5), a.verbose))


if __name__ == "__main__":
    main()
