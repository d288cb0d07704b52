"""Build liblgf.so (HIP, gfx950) in-tree.

    python -m paper_2010_13213_amd.build

Every translation unit is compiled by hipcc for gfx950 only, with packed
FP32 instructions disabled, then linked into paper_2010_13213_amd/liblgf.so.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblgf.so")
SOURCES = ["lgf_table.hip", "lgf_fft.hip", "lgf_smac.hip", "lgf_lattice.hip", "lgf_composite.hip", "lgf_refine.hip", "lgf_refresh.hip", "lgf_flgf.hip", "lgf_runtime.cpp", "lgf_schedule.cpp",
           "lgf_tuning.cpp", "lgf_capi.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
         "-Werror=infinite-recursion",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def source_digest():
    """SHA-256 over the library's sources (csrc/, include/) and the compiler
    flags, in a fixed order; the build bakes it into lgf_build_id()."""
    import hashlib
    h = hashlib.sha256()
    h.update(" ".join(FLAGS[:-2]).encode())
    files = []
    for d in (CSRC, os.path.join(ROOT, "include")):
        for name in sorted(os.listdir(d)):
            if os.path.splitext(name)[1] in (".hip", ".cpp", ".hpp", ".h"):
                files.append(os.path.join(d, name))
    for path in files:
        h.update(os.path.relpath(path, ROOT).encode() + b"\0")
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _compile(src, digest):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ['-DLGF_SOURCE_SHA256="%s"' % digest, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


def build(jobs=8):
    os.makedirs(BUILD, exist_ok=True)
    digest = source_digest()
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, digest), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
    sys.exit(0)
