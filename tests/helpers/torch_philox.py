"""Build and call the PyTorch-header Philox reference (tests only)."""
import functools
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


@functools.lru_cache(maxsize=1)
def binary() -> str:
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    out = os.path.join(tempfile.gettempdir(), "csaw_philox_torch_ref_%d" % os.getuid())
    src = os.path.join(HERE, "philox_torch_ref.cpp")
    if not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        subprocess.run(["g++", "-O2", "-std=c++17", "-I", inc, "-o", out + ".tmp", src], check=True)
        os.replace(out + ".tmp", out)
    return out


def blocks(keys, ctrs) -> np.ndarray:
    """keys [N,2], ctrs [N,4] (uint32) -> [N,4] uint32 output words."""
    keys = np.asarray(keys, dtype=np.uint64)
    ctrs = np.asarray(ctrs, dtype=np.uint64)
    lines = "\n".join("%d %d %d %d %d %d" % (k[0], k[1], c[0], c[1], c[2], c[3])
                      for k, c in zip(keys, ctrs))
    res = subprocess.run([binary()], input=lines + "\n", capture_output=True, text=True, check=True)
    return np.array([[int(x) for x in ln.split()] for ln in res.stdout.strip().splitlines()],
                    dtype=np.uint64).astype(np.uint32)


def draw(rng_seed: int, ctr, W: int) -> int:
    """The contract's draw computed from the reference block with Python ints:
    key = (seed lo, seed hi), u = x0 + 2^32 x1, r = floor(u*W / 2^64)."""
    x = blocks([[rng_seed & 0xFFFFFFFF, rng_seed >> 32]], [ctr])[0]
    u = int(x[0]) | (int(x[1]) << 32)
    return (u * W) >> 64
