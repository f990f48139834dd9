"""Build the HIP shared library in-tree: paper_2606_13825_amd/libcosmo_unroll.so.

Every translation unit is compiled for gfx950 only.  Packed FP32 arithmetic
is disabled for the device code (the host pass warns that it does not know
the feature; that is harmless).
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcosmo_unroll.so")
SOURCES = ["plan.hip", "k_vec.hip", "k_pcg.hip", "k_soc.hip", "k_psd.hip", "k_ns.hip", "k_dense.hip", "k_policy.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result"]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer for the plan,
# validation and launch code; device code is built as usual.
HOST_SANITIZE = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer".split()


def _compile(src: str, verbose: bool, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, src.replace(".hip", ".o"))
    cmd = [hipcc()] + common_flags() + list(extra) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)
    return obj


def build(verbose: bool = False) -> str:
    return _build(LIB, BUILD, (), verbose)


def build_host_sanitized(verbose: bool = False) -> str:
    """The same library with ASan and UBSan on its host code, under _build/
    (never the shipped library).  A process that loads it must preload the
    ASan runtime (sanitizer_runtime())."""
    out_dir = os.path.join(BUILD, "host_sanitized")
    return _build(os.path.join(out_dir, "libcosmo_unroll.so"), out_dir, HOST_SANITIZE, verbose)


def sanitizer_runtime() -> str:
    r = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


def _build(lib: str, build_dir: str, extra, verbose: bool) -> str:
    os.makedirs(build_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, build_dir, extra), SOURCES))
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + list(extra) + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
