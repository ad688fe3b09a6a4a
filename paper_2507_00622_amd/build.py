"""Build libchx.so (the HIP library behind include/chx.h) for gfx950.

Every .hip file under csrc/ is compiled with hipcc in parallel into
_build/ and linked into paper_2507_00622_amd/libchx.so.
"""
import concurrent.futures as cf
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libchx.so")
ARCH = "gfx950"

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Wno-cuda-compat",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


# Host code checked by AddressSanitizer + UndefinedBehaviorSanitizer (device
# code unchanged); load such a library with the compiler's ASan runtime
# preloaded.  Each -fsanitize= follows its -Xarch_host.
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def _up_to_date(obj, dep):
    """True when obj is newer than every file its dependency list names."""
    if not (os.path.exists(obj) and os.path.exists(dep)):
        return False
    text = open(dep).read().replace("\\\n", " ")
    files = [f for f in text.split(":", 1)[1].split() if f]
    t = os.path.getmtime(obj)
    return all(os.path.exists(f) and os.path.getmtime(f) <= t for f in files)


def _compile(src, incremental=False, build_dir=BUILD, extra=()):
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    dep = obj + ".d"
    if incremental and _up_to_date(obj, dep):
        return obj
    cmd = ["hipcc", *FLAGS, *extra, "-MD", "-MF", dep, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    return obj


def build(jobs=None, incremental=False, sanitize_host=False, out=None):
    """Compile every csrc/*.hip and link libchx.so; returns the library path.
    With incremental, an object newer than its source and every header is
    kept (a developer's shortcut; the default rebuilds everything).  With
    sanitize_host, the host code is built with ASan + UBSan into its own
    object directory and linked to out (default: libchx.san.so)."""
    build_dir = BUILD + ("_san" if sanitize_host else "")
    extra = SANITIZE_HOST if sanitize_host else []
    lib = out or (os.path.join(HERE, "libchx.san.so") if sanitize_host else LIB)
    os.makedirs(build_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = jobs or min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, incremental, build_dir, extra), srcs))
    tmp = lib + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, *objs, "-o", tmp,
           "-lhiprtc"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    import sys
    print(build(incremental="--incremental" in sys.argv,
                sanitize_host="--sanitize-host" in sys.argv))
