"""Build steps of the package: the gfx950 HIP library and the input generator.

``build_all()`` always compiles (it is the "does it build" check); the loaders
call ``build_hip(force=False)`` only when no library is present.
"""
from __future__ import annotations

import glob
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcsaw.so")
ARCH = os.environ.get("CSAW_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # keep the compiler from forming packed fp32 ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + glob.glob(os.path.join(CSRC, "*.h")) + [
        os.path.join(os.path.dirname(HERE), "include", "csaw.h")]
    return any(os.path.getmtime(p) > t for p in deps if os.path.exists(p))


def build_hip(force: bool = True, verbose: bool = False) -> str:
    """Compile csrc/*.hip for gfx950 and link libcsaw.so in-tree."""
    if not force and not _stale():
        return LIB
    hipcc = _hipcc()
    tmpdir = tempfile.mkdtemp(prefix="csaw_build_")
    objs, procs = [], []
    for src in sources():
        obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [hipcc] + HIPCC_FLAGS + ["-c", src, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                            text=True)))
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("hipcc failed: %s\n%s" % (" ".join(cmd), out))
        if verbose and out.strip():
            print(out)
    tmp_lib = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp_lib] + objs
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), res.stdout))
    os.replace(tmp_lib, LIB)
    for o in objs:
        os.remove(o)
    os.rmdir(tmpdir)
    return LIB


def build_all(verbose: bool = False) -> None:
    from . import inputs
    inputs.build(force=True)
    build_hip(force=True, verbose=verbose)
