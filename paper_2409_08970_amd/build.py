"""Build libdctplus.so (all HIP sources under csrc/) for gfx950 with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libdctplus.so")
ARCH = os.environ.get("DCTPLUS_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay disabled: some of their forms have given wrong results on this part
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", f"-I{INCLUDE}",
]
LIBS = []


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libdctplus.so")


def build(verbose: bool = False) -> str:
    """Compile every HIP source (one hipcc per source, in parallel) and link them
    into one shared library.  Always recompiles."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    compile_flags = [f for f in FLAGS if f != "-shared"]
    jobs = max(1, min(len(sources()), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with tempfile.TemporaryDirectory(prefix="dctplus_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in sources()]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            for f in [ex.submit(_run, ["hipcc", *compile_flags, "-c", src, "-o", obj], verbose)
                      for src, obj in zip(sources(), objs)]:
                f.result()
        tmp = LIB + ".tmp"
        _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, *LIBS], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
