"""Build libdicod.so (HIP kernels for gfx950 + host runtime + C ABI) in-tree."""
import concurrent.futures
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdicod.so")
SOURCES = ["kernels.hip", "lgcd_wave.hip", "lgcd_async.hip", "lambda_bound.hip", "noalloc.hip", "dicod_api.cpp", "dicod_serve.cpp"]
ARCH = os.environ.get("DICOD_ARCH", "gfx950")


FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-mcode-object-version=5",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def compile_command(src, obj):
    """One translation unit to an object (device code for ARCH plus host code)."""
    return ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]


def link_command(objs, out=LIB):
    return ["hipcc", f"--offload-arch={ARCH}", "-fPIC", "-shared", "-o", out, *objs,
            "-Wl,-rpath,/opt/rocm/lib", "-lpthread"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 feature; drop that warning
    noise = [ln for ln in (res.stdout + res.stderr).splitlines()
             if ln.strip() and "packed-fp32-ops" not in ln]
    return res.returncode, noise


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel, objects in a temporary folder), link
    libdicod.so.tmp and move it into place."""
    jobs = jobs or max(1, min(len(SOURCES), os.cpu_count() or 1))
    with tempfile.TemporaryDirectory(prefix="dicod_build_") as tmpdir:
        objs = [os.path.join(tmpdir, s + ".o") for s in SOURCES]
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(lambda so: _run(compile_command(*so), verbose),
                                  zip(SOURCES, objs)))
        for src, (rc, noise) in zip(SOURCES, results):
            if rc != 0 or (verbose and noise):
                sys.stderr.write(f"{src}:\n" + "\n".join(noise) + "\n")
            if rc != 0:
                raise RuntimeError(f"hipcc failed to compile {src}")
        tmp = LIB + ".tmp"
        rc, noise = _run(link_command(objs, tmp), verbose)
        if rc != 0:
            sys.stderr.write("\n".join(noise) + "\n")
            raise RuntimeError("hipcc failed to link libdicod.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
