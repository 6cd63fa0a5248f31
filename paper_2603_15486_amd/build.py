"""Build libcf.so (HIP, gfx950) in-tree with hipcc.

Each source compiles to its own object in parallel (the kernel
instantiations are split by fingerprint width across several translation
units for that reason), then one link step makes the shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libcf.so")
SOURCES = ["cf_api.hip", "cf_inst_f8.hip", "cf_inst_f16.hip", "cf_inst_f32.hip",
           "cf_insi_f8.hip", "cf_insi_f16.hip", "cf_insi_f32.hip",
           "cf_set.hip", "cf_set_inst_f8.hip", "cf_set_inst_f16.hip", "cf_set_inst_f32.hip",
           "cf_set_insi_f8.hip", "cf_set_insi_f16.hip", "cf_set_insi_f32.hip",
           "cf_set_persist_insi_f8.hip", "cf_set_persist_insi_f16.hip",
           "cf_set_persist_insi_f32.hip",
           "cf_server.hip", "cf_tune.hip", "cf_keygen.hip"]
# The insert kernels (the cf_*insi_* units) are built at -O1.  Built at -O2
# or -O3 they lost fingerprints under heavy contention (one-launch fills of
# a 2^20-slot table, buckets of two or four 64-bit words); bisecting the
# optimisation passes pins the loss on the backend's Early Machine LICM run
# over the insert kernel, and -O3 without Machine LICM passes too.  -O1 is
# the configuration validated over the most runs and inserts as fast.
# Everything else is built at -O3.
OPT_LEVEL = {s: "-O1" for s in SOURCES if "insi_" in s}
ARCH = os.environ.get("CF_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"),
                 shutil.which("hipcc") or ""):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the HIP toolchain is required to build libcf.so")


def compile_flags(src: str = "") -> list[str]:
    return [
        f"--offload-arch={ARCH}", OPT_LEVEL.get(src, "-O3"), "-std=c++17", "-fPIC",
        "-Wall", "-Wno-unused-function", "-pthread",
        # no packed fp32 instructions anywhere in this library
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE, "-I", CSRC,
    ]


def object_of(src: str) -> str:
    return os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")


def compile_command(src: str) -> list[str]:
    return [hipcc()] + compile_flags(src) + ["-c", os.path.join(CSRC, src), "-o", object_of(src)]


def link_command(out: str) -> list[str]:
    return [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", out] + \
        [object_of(s) for s in SOURCES]


def _jobs() -> int:
    env = os.environ.get("MAX_JOBS")
    n = int(env) if env and env.isdigit() else (os.cpu_count() or 4)
    return max(1, min(n, 16, len(SOURCES)))


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)

    def one(src):
        cmd = compile_command(src)
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        return src, res

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(one, SOURCES))
    failed = [(src, res) for src, res in results if res.returncode != 0]
    for src, res in results:
        # the host pass does not know the packed-fp32 target feature; keep
        # every other diagnostic visible
        lines = [ln for ln in (res.stdout + res.stderr).splitlines()
                 if "packed-fp32-ops" not in ln and ln.strip()]
        if lines and (verbose or res.returncode != 0):
            print(f"--- {src}\n" + "\n".join(lines), flush=True)
    if failed:
        raise subprocess.CalledProcessError(failed[0][1].returncode,
                                            compile_command(failed[0][0]))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = link_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
