"""Build step for libcbct.so (HIP, gfx950), compiled in-tree with hipcc."""
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libcbct.so")

# Packed FP32 instructions stay disabled for every HIP translation unit.
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    csrc = os.path.join(HERE, "csrc")
    return sorted(glob.glob(os.path.join(csrc, "*.cpp")) + glob.glob(os.path.join(csrc, "*.hip")))


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + msgs)
    return msgs


def build_library(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source under csrc/ into paper_2512_21180_amd/libcbct.so:
    one object per source, compiled in parallel (`jobs` processes, default
    the CPU count up to 8), then one link."""
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    cflags = [f for f in HIP_FLAGS if f != "-shared"]

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        return obj, _run([hipcc] + cflags + inc + ["-c", "-o", obj, src])

    def stamps():
        files = sources() + glob.glob(os.path.join(HERE, "csrc", "*.h")) + \
            glob.glob(os.path.join(ROOT, "include", "*.h"))
        return {f: os.stat(f).st_mtime_ns for f in files}

    before = stamps()
    n = jobs or min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=n) as ex:
        results = list(ex.map(compile_one, sources()))
    # hipcc reads a source once for the device pass and again for the host
    # pass: an edit during the build can pair one version's kernels with the
    # other's launchers, so such a build is refused
    changed = sorted(f for f, t in stamps().items() if before.get(f) != t)
    if changed:
        raise RuntimeError("sources changed during the build, rebuild: " + ", ".join(changed))
    tmp = LIB + ".tmp"
    msgs = [m for _, m in results] + [
        _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] +
             [o for o, _ in results])]
    if verbose:
        text = "\n".join(m for m in msgs if m.strip())
        if text:
            print(text)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
