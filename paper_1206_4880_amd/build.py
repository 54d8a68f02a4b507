"""Build the HIP library libfic.so in-tree for gfx950 (hipcc, no JIT cache).

Each csrc/*.hip is compiled to an object in parallel, then linked into
paper_1206_4880_amd/libfic.so next to this file.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfic.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    # no packed fp32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# The search screen never sees a NaN (padding columns carry a finite u and
# are masked), so its |x| maxima need no NaN canonicalisation. Without the
# atomic optimizer, a work-queue claim made by lane 0 stays one atomic whose
# reply is read only when the next item starts (the optimizer would rewrite
# it into a wave-wide atomic that waits for its reply at once).
PER_FILE = {"encode.hip": ["-fno-honor-nans", "-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]}


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def kernel_hash():
    """First 16 hex digits of SHA-256 over the build flags and the library's
    sources (every csrc/*.hip and *.h, then include/fic.h): the tag of
    autotuning caches."""
    import hashlib
    h = hashlib.sha256()
    h.update(repr((FLAGS, sorted(PER_FILE.items()))).encode())   # the build flags too
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".h")))
    for f in files + ["../../include/fic.h"]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def build(verbose=False, jobs=8):
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    srcs = sources()
    per_file = dict(PER_FILE)
    per_file["api.hip"] = per_file.get("api.hip", []) + ['-DFIC_KERNEL_HASH="%s"' % kernel_hash()]
    objs = [os.path.join(BUILD, os.path.basename(s)[:-4] + ".o") for s in srcs]

    def one(pair):
        s, o = pair
        cmd = [hipcc] + FLAGS + per_file.get(os.path.basename(s), []) + ["-c", s, "-o", o]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (s, r.stderr))
        return r.stderr

    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        for err in ex.map(one, zip(srcs, objs)):
            if verbose and err:
                sys.stderr.write(err)
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
