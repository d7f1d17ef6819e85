"""Build libhs.so (HIP for gfx950) in-tree with hipcc.

    python paper_1805_12258_amd/build.py [--force] [--jobs N]

Run it by path: it needs only the standard library, while importing the
package requires the built library.

Every HIP translation unit is compiled for gfx950 only, with -ffp-contract=off
(sums must round exactly as the sequential fp32 recursion) and with packed
fp32 instructions disabled.  Objects go to csrc/_build/, the library to the
package directory.
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libhs.so")
BUILD = os.path.join(CSRC, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DEVICE_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]
HOST_FLAGS = ["--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall"]
INCLUDES = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def _compile(src, obj, flags):
    cmd = [HIPCC] + flags + INCLUDES + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(force=True, jobs=None, verbose=True):
    """Compile every source and link libhs.so.  Returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    hip, cpp = sources()
    def dep_time(path, seen=None):
        """Latest modification time of a source and the local headers it
        includes (transitively)."""
        seen = set() if seen is None else seen
        if path in seen or not os.path.exists(path):
            return 0.0
        seen.add(path)
        t = os.path.getmtime(path)
        for line in open(path):
            line = line.strip()
            if line.startswith("#include \""):
                name = line.split('"')[1]
                for d in (CSRC, os.path.join(ROOT, "include")):
                    if os.path.exists(os.path.join(d, name)):
                        t = max(t, dep_time(os.path.join(d, name), seen))
                        break
        return t
    tasks = []
    for f in hip:
        tasks.append((f, os.path.join(BUILD, f + ".o"), DEVICE_FLAGS))
    for f in cpp:
        tasks.append((f, os.path.join(BUILD, f + ".o"), HOST_FLAGS))
    todo = []
    for src, obj, flags in tasks:
        stale = (not os.path.exists(obj) or
                 os.path.getmtime(obj) < dep_time(os.path.join(CSRC, src)))
        if force or stale:
            todo.append((src, obj, flags))
    # the largest translation units first (more planes unroll to more code)
    def cost(t):
        name = t[0]
        g = int(name.rsplit("_g", 1)[1][0]) if "_fused_" in name else -1
        return (-g, "f32" not in name)
    todo.sort(key=cost)
    jobs = jobs or min(8, max(1, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_compile, *t) for t in todo]
        for fu in futs:
            fu.result()
    objs = [t[1] for t in tasks]
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("--jobs", type=int, default=None)
    a = ap.parse_args()
    build(force=a.force, jobs=a.jobs)
    sys.exit(0)
