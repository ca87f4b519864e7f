"""Thin Python binding of libcsaw (C-ABI in include/csaw.h).

Argument marshalling only: every step of sampling and walking runs in the
library's HIP kernels. torch provides device memory (tensors) and streams.
There is no CPU fallback: if the library is missing or fails to load, import
fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime that libcsaw then shares

from . import _build

UNIFORM, EDGE_WEIGHT, NEIGHBOR_DEGREE, NODE2VEC, METROPOLIS_HASTINGS = 0, 1, 2, 3, 4
DIRECT_ONLY = -1  # csaw_sample_args.rounds: no repeated-sampling rounds
FANOUT_ALL = -1
MAX_FANOUT = 64
MAX_LAYERS = 16
NOALLOC_SCRATCH_BYTES = 128 << 20  # CSAW_NOALLOC_SCRATCH_BYTES
ROUNDS = 8

_BIAS_NAMES = {"uniform": UNIFORM, "edge_weight": EDGE_WEIGHT, "neighbor_degree": NEIGHBOR_DEGREE,
               "node2vec": NODE2VEC, "metropolis_hastings": METROPOLIS_HASTINGS}
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "DEVICE", 4: "BUSY", 5: "NOT_READY",
          6: "UNSUPPORTED", 7: "CANCELLED"}


class CsawError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class SampleArgs(ctypes.Structure):
    _fields_ = [("num_instances", ctypes.c_int32), ("seed_offsets", ctypes.c_void_p),
                ("seeds", ctypes.c_void_p), ("instance_base", ctypes.c_uint64),
                ("num_layers", ctypes.c_int32), ("fanouts", ctypes.c_void_p),
                ("fanout_stride", ctypes.c_int32), ("bias_kind", ctypes.c_int32),
                ("bias_kinds", ctypes.c_void_p), ("rng_seed", ctypes.c_uint64),
                ("instance_ids", ctypes.c_void_p), ("rng_seeds", ctypes.c_void_p), ("rounds", ctypes.c_int32),
                ("burn_threshold", ctypes.c_uint32)]


class SampleOut(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("edge_capacity", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("num_edges", ctypes.c_int64)]


class WalkArgs(ctypes.Structure):
    _fields_ = [("bias_kind", ctypes.c_int32), ("w_return", ctypes.c_uint32),
                ("w_common", ctypes.c_uint32), ("w_outward", ctypes.c_uint32),
                ("num_walkers", ctypes.c_int64), ("starts", ctypes.c_void_p),
                ("walker_base", ctypes.c_uint64), ("length", ctypes.c_int32),
                ("rng_seed", ctypes.c_uint64), ("walker_ids", ctypes.c_void_p),
                ("restart_threshold", ctypes.c_uint32), ("jump_threshold", ctypes.c_uint32)]


class MdrwArgs(ctypes.Structure):
    _fields_ = [("num_instances", ctypes.c_int32), ("pool_offsets", ctypes.c_void_p), ("pool", ctypes.c_void_p),
                ("instance_base", ctypes.c_uint64), ("budget", ctypes.c_int64), ("rng_seed", ctypes.c_uint64)]


class LayerArgs(ctypes.Structure):
    _fields_ = [("num_instances", ctypes.c_int32), ("seed_offsets", ctypes.c_void_p), ("seeds", ctypes.c_void_p),
                ("instance_base", ctypes.c_uint64), ("num_layers", ctypes.c_int32), ("fanouts", ctypes.c_void_p),
                ("bias_kind", ctypes.c_int32), ("rng_seed", ctypes.c_uint64), ("rounds", ctypes.c_int32)]


AllocFn = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FreeFn = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class StreamStats(ctypes.Structure):
    _fields_ = [("partition_loads", ctypes.c_int64), ("bytes_loaded", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("bound16", ctypes.c_int32), ("bound32", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("memory_budget_bytes", ctypes.c_int64), ("max_batch", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("num_streams", ctypes.c_int32),
                ("max_batch_walkers", ctypes.c_int64), ("result_pool_bytes", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("id", ctypes.c_uint64), ("rng_seed", ctypes.c_uint64),
                ("bias_kind", ctypes.c_int32), ("seeds", ctypes.c_void_p), ("num_seeds", ctypes.c_int64),
                ("fanouts", ctypes.c_void_p), ("num_layers", ctypes.c_int32),
                ("starts", ctypes.c_void_p), ("num_walkers", ctypes.c_int64), ("length", ctypes.c_int32),
                ("w_return", ctypes.c_uint32), ("w_common", ctypes.c_uint32), ("w_outward", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("kind", ctypes.c_int32), ("num_edges", ctypes.c_int64),
                ("src", ctypes.POINTER(ctypes.c_int32)), ("dst", ctypes.POINTER(ctypes.c_int32)),
                ("num_layers", ctypes.c_int32), ("layer_offsets", ctypes.POINTER(ctypes.c_int64)),
                ("paths", ctypes.POINTER(ctypes.c_int32)), ("num_walkers", ctypes.c_int64),
                ("length", ctypes.c_int32), ("steps", ctypes.c_int64), ("queued_us", ctypes.c_double),
                ("total_us", ctypes.c_double), ("batch_requests", ctypes.c_int32)]


EXPORTS = ["csaw_graph_create", "csaw_graph_destroy", "csaw_graph_info", "csaw_sample", "csaw_sample_noalloc",
           "csaw_sample_bound", "csaw_set_tuning", "csaw_get_tuning", "csaw_set_walk_guides", "csaw_get_walk_guides", "csaw_autotune_sample", "csaw_walk",
           "csaw_mdrw", "csaw_layer_sample", "csaw_set_allocator", "csaw_profile_enable", "csaw_profile_reset", "csaw_profile_read", "csaw_last_error", "csaw_version", "csaw_server_create",
           "csaw_server_submit", "csaw_server_poll", "csaw_server_wait", "csaw_server_cancel",
           "csaw_server_memory", "csaw_result_free", "csaw_server_destroy", "csaw_pgraph_create",
           "csaw_pgraph_destroy", "csaw_sample_streamed"]


def _load():
    if not os.path.exists(_build.LIB):
        _build.build_hip(force=False)
    L = ctypes.CDLL(_build.LIB)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    L.csaw_graph_create.argtypes = [i64, i64, vp, vp, vp, u32, vp, ctypes.POINTER(vp)]
    L.csaw_graph_destroy.argtypes = [vp]
    L.csaw_graph_info.argtypes = [vp, vp, vp, vp, vp]
    L.csaw_sample.argtypes = [vp, ctypes.POINTER(SampleArgs), ctypes.POINTER(SampleOut), vp]
    L.csaw_sample_noalloc.argtypes = [vp, ctypes.POINTER(SampleArgs), ctypes.POINTER(SampleOut), vp]
    L.csaw_sample_bound.argtypes = [vp, ctypes.POINTER(SampleArgs), ctypes.POINTER(ctypes.c_int64)]
    L.csaw_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.csaw_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.csaw_set_walk_guides.argtypes = [vp, i32]
    L.csaw_get_walk_guides.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.csaw_autotune_sample.argtypes = [vp, ctypes.POINTER(SampleArgs), ctypes.POINTER(SampleOut), i32, vp,
                                       ctypes.POINTER(Tuning)]
    L.csaw_walk.argtypes = [vp, ctypes.POINTER(WalkArgs), vp, ctypes.POINTER(ctypes.c_int64), vp]
    L.csaw_layer_sample.argtypes = [vp, ctypes.POINTER(LayerArgs), vp, vp, vp, vp]
    L.csaw_set_allocator.argtypes = [AllocFn, FreeFn, vp]
    L.csaw_mdrw.argtypes = [vp, ctypes.POINTER(MdrwArgs), vp, vp, vp, ctypes.POINTER(ctypes.c_int64), vp]
    L.csaw_profile_enable.argtypes = [i32]
    L.csaw_profile_reset.argtypes = []
    L.csaw_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64)]
    L.csaw_server_create.argtypes = [vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    L.csaw_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.csaw_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.POINTER(Result))]
    L.csaw_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(ctypes.POINTER(Result))]
    L.csaw_pgraph_create.argtypes = [i64, i64, vp, vp, vp, i32, i32, vp, ctypes.POINTER(vp)]
    L.csaw_pgraph_destroy.argtypes = [vp]
    L.csaw_sample_streamed.argtypes = [vp, ctypes.POINTER(SampleArgs), ctypes.POINTER(SampleOut), vp,
                                       ctypes.POINTER(StreamStats)]
    L.csaw_server_cancel.argtypes = [vp, ctypes.c_uint64]
    L.csaw_server_memory.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.csaw_result_free.argtypes = [ctypes.POINTER(Result)]
    L.csaw_server_destroy.argtypes = [vp]
    for f in EXPORTS:
        if f not in ("csaw_last_error", "csaw_version", "csaw_result_free"):
            getattr(L, f).restype = ctypes.c_int
    L.csaw_result_free.restype = None
    L.csaw_last_error.restype = ctypes.c_char_p
    L.csaw_version.restype = ctypes.c_char_p
    return L


lib = _load()


def _check(status: int):
    if status != 0:
        raise CsawError(status, lib.csaw_last_error().decode())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _bias_code(b) -> int:
    if isinstance(b, str):
        return _BIAS_NAMES[b]
    return int(b)


def _dev_i32(x, device) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=torch.int32)
    else:
        t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).to(device)
    return t.contiguous()


_allocator_refs = []  # callbacks must outlive every buffer they handed out


def set_allocator(alloc=None, free=None):
    """Workspace device memory from alloc(nbytes) -> int pointer and
    free(pointer) (csaw_set_allocator); both None restores hipMalloc."""
    if alloc is None and free is None:
        _check(lib.csaw_set_allocator(AllocFn(), FreeFn(), None))
        return
    a = AllocFn(lambda n, user: alloc(int(n)) or None)
    f = FreeFn(lambda p, user: free(int(p)))
    _allocator_refs.append((a, f))
    _check(lib.csaw_set_allocator(a, f, None))


def version() -> str:
    return lib.csaw_version().decode()


class SampleResult:
    """Edges in (layer, instance, source, slot) order; ``offsets[l*ni + i]`` is
    the first edge of (layer l, instance i)."""

    def __init__(self, src, dst, offsets, num_layers, num_instances):
        self.src, self.dst, self.offsets = src, dst, offsets
        self.num_layers, self.num_instances = num_layers, num_instances

    @property
    def num_edges(self) -> int:
        return int(self.src.shape[0])


class Graph:
    """A CSR graph resident in HBM on the current device."""

    def __init__(self, rowptr, col, edge_weight=None, stream=None):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        ew = None if edge_weight is None else np.ascontiguousarray(edge_weight, dtype=np.uint32)
        n = len(rowptr) - 1
        h = ctypes.c_void_p()
        _check(lib.csaw_graph_create(n, len(col), rowptr.ctypes.data, col.ctypes.data,
                                     None if ew is None else ew.ctypes.data, 0, _stream(stream),
                                     ctypes.byref(h)))
        self._h = h
        self.n, self.m = n, len(col)
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "_h", None):
            lib.csaw_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        n, m, md = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        srt = ctypes.c_int32()
        _check(lib.csaw_graph_info(self._h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(md),
                                   ctypes.byref(srt)))
        return dict(n=n.value, m=m.value, max_degree=md.value, sorted=bool(srt.value))

    # -------------------------------------------------------------- sampling
    def _sample_args(self, seed_offsets, seeds_dev, fanouts, bias, rng_seed, instance_base,
                     instance_ids=None, rng_seeds=None, rounds=0, burn=0):
        so = np.ascontiguousarray(seed_offsets, dtype=np.int64)
        fo = np.ascontiguousarray(fanouts, dtype=np.int32)
        ni = len(so) - 1
        if fo.ndim == 1:
            L, stride = fo.shape[0], 0
        else:
            L, stride = fo.shape[1], fo.shape[1]
        a = SampleArgs()
        a.num_instances = ni
        a.seed_offsets = so.ctypes.data
        a.seeds = seeds_dev.data_ptr() if seeds_dev is not None and seeds_dev.numel() else None
        a.instance_base = int(instance_base)
        a.num_layers = L
        a.fanouts = fo.ctypes.data
        a.fanout_stride = stride
        keep = [so, fo]
        if isinstance(bias, (list, tuple, np.ndarray)):
            bk = np.ascontiguousarray([_bias_code(b) for b in bias], dtype=np.int32)
            a.bias_kinds = bk.ctypes.data
            a.bias_kind = 0
            keep.append(bk)
        else:
            a.bias_kinds = None
            a.bias_kind = _bias_code(bias)
        a.rng_seed = int(rng_seed)
        a.rounds = int(rounds)
        a.burn_threshold = int(burn)
        a.instance_ids = None
        a.rng_seeds = None
        if instance_ids is not None:
            ids = np.ascontiguousarray(instance_ids, dtype=np.uint64)
            assert len(ids) == ni
            a.instance_ids = ids.ctypes.data
            keep.append(ids)
        if rng_seeds is not None:
            rs = np.ascontiguousarray(rng_seeds, dtype=np.uint64)
            assert len(rs) == ni
            a.rng_seeds = rs.ctypes.data
            keep.append(rs)
        return a, keep, ni, L

    def sample_bound(self, seed_offsets, fanouts, bias=UNIFORM) -> int:
        a, keep, _, _ = self._sample_args(seed_offsets, None, fanouts, bias, 0, 0)
        mx = ctypes.c_int64()
        _check(lib.csaw_sample_bound(self._h, ctypes.byref(a), ctypes.byref(mx)))
        return mx.value

    def sample(self, seed_offsets, seeds, fanouts, bias=UNIFORM, rng_seed=1, instance_base=0,
               capacity=None, stream=None, out=None, instance_ids=None, rng_seeds=None, rounds=0,
               burn=0) -> SampleResult:
        """Neighbor sampling (csaw_sample). ``seeds`` may be a device tensor
        (used in place) or host data (copied). ``out`` may pass preallocated
        (src, dst, offsets) device tensors. ``rounds``: 0 (default, 8), 1..8,
        or DIRECT_ONLY. ``burn``: forest fire threshold over [0, 2^32)."""
        return self._run_sample(lambda a, o: lib.csaw_sample(self._h, a, o, _stream(stream)), seed_offsets, seeds,
                                fanouts, bias, rng_seed, instance_base, capacity, out, instance_ids, rng_seeds,
                                rounds, burn)

    def sample_noalloc(self, seed_offsets, seeds, fanouts, out, bias=UNIFORM, rng_seed=1, instance_base=0,
                       stream=None, instance_ids=None, rng_seeds=None, rounds=0, burn=0) -> SampleResult:
        """csaw_sample_noalloc: as ``sample``, with the library's fixed device
        scratch and no device allocation anywhere on the path. ``seeds`` must
        be a contiguous int32 tensor on the graph's device and ``out`` the
        (src, dst, offsets) device tensors; the results are views of them."""
        if not (isinstance(seeds, torch.Tensor) and seeds.dtype == torch.int32 and seeds.is_contiguous()
                and seeds.device == self.device):
            raise ValueError("seeds must be a contiguous int32 tensor on %s" % self.device)
        if out is None or any(t is not None and t.device != self.device for t in out):
            raise ValueError("out must be (src, dst, offsets) tensors on %s" % self.device)
        return self._run_sample(lambda a, o: lib.csaw_sample_noalloc(self._h, a, o, _stream(stream)), seed_offsets,
                                seeds, fanouts, bias, rng_seed, instance_base, None, out, instance_ids, rng_seeds,
                                rounds, burn)

    def autotune_sample(self, seed_offsets, seeds, fanouts, bias=UNIFORM, rng_seed=1, instance_base=0,
                        capacity=None, stream=None, out=None, instance_ids=None, rng_seeds=None, reps=3, rounds=0,
                        burn=0):
        """Autotuner (csaw_autotune_sample): times the call under each
        sub-wave bucket setting, keeps the fastest on the graph. Returns
        (SampleResult, (bound16, bound32))."""
        t = Tuning()
        res = self._run_sample(lambda a, o: lib.csaw_autotune_sample(self._h, a, o, int(reps), _stream(stream),
                                                                     ctypes.byref(t)),
                               seed_offsets, seeds, fanouts, bias, rng_seed, instance_base, capacity, out,
                               instance_ids, rng_seeds, rounds, burn)
        return res, (t.bound16, t.bound32)

    def set_tuning(self, bound16: int, bound32: int):
        """Sub-wave bucket bounds of the sampling kernel (csaw_set_tuning)."""
        t = Tuning(int(bound16), int(bound32))
        _check(lib.csaw_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self):
        t = Tuning()
        _check(lib.csaw_get_tuning(self._h, ctypes.byref(t)))
        return t.bound16, t.bound32

    def set_walk_guides(self, enable: bool):
        """Weighted walks through the walk guide (True, the default) or the
        chunk tables (csaw_set_walk_guides)."""
        _check(lib.csaw_set_walk_guides(self._h, 1 if enable else 0))

    def get_walk_guides(self) -> bool:
        e = ctypes.c_int32()
        _check(lib.csaw_get_walk_guides(self._h, ctypes.byref(e)))
        return bool(e.value)

    def _run_sample(self, call, seed_offsets, seeds, fanouts, bias, rng_seed, instance_base, capacity, out,
                    instance_ids, rng_seeds, rounds=0, burn=0) -> SampleResult:
        seeds_dev = _dev_i32(seeds, self.device)
        a, keep, ni, L = self._sample_args(seed_offsets, seeds_dev, fanouts, bias, rng_seed,
                                           instance_base, instance_ids, rng_seeds, rounds, burn)
        if out is None:
            if capacity is None:
                mx = ctypes.c_int64()
                _check(lib.csaw_sample_bound(self._h, ctypes.byref(a), ctypes.byref(mx)))
                capacity = mx.value
            src = torch.empty(max(capacity, 1), dtype=torch.int32, device=self.device)
            dst = torch.empty(max(capacity, 1), dtype=torch.int32, device=self.device)
            offsets = torch.empty(L * ni + 1, dtype=torch.int64, device=self.device)
        else:
            src, dst, offsets = out
            capacity = src.numel()
        o = SampleOut()
        o.src, o.dst, o.edge_capacity = src.data_ptr(), dst.data_ptr(), int(capacity)
        o.offsets = offsets.data_ptr() if offsets is not None else None
        _check(call(ctypes.byref(a), ctypes.byref(o)))
        ne = o.num_edges
        return SampleResult(src[:ne], dst[:ne], offsets, L, ni)

    # ----------------------------------------------------------------- walks
    def walk(self, starts, length, bias=UNIFORM, rng_seed=1, walker_base=0, node2vec=(1, 1, 1),
             stream=None, paths=None, walker_ids=None, restart=0, jump=0):
        """Random walks (csaw_walk); restart / jump are the per-step move
        thresholds over [0, 2^32). Returns (paths [nw, length+1] int32 device
        tensor, total steps)."""
        st = _dev_i32(starts, self.device)
        nw = st.numel()
        if paths is None:
            paths = torch.empty((nw, length + 1), dtype=torch.int32, device=self.device)
        a = WalkArgs()
        a.bias_kind = _bias_code(bias)
        a.w_return, a.w_common, a.w_outward = (int(x) for x in node2vec)
        a.num_walkers = nw
        a.starts = st.data_ptr() if nw else None
        a.walker_base = int(walker_base)
        a.length = int(length)
        a.rng_seed = int(rng_seed)
        ids_dev = None
        if walker_ids is not None:
            ids_dev = torch.from_numpy(np.ascontiguousarray(walker_ids, dtype=np.uint64).view(np.int64)).to(
                self.device)
            assert ids_dev.numel() == nw
        a.walker_ids = ids_dev.data_ptr() if ids_dev is not None and nw else None
        a.restart_threshold = int(restart)
        a.jump_threshold = int(jump)
        steps = ctypes.c_int64()
        _check(lib.csaw_walk(self._h, ctypes.byref(a), paths.data_ptr() if nw else None,
                             ctypes.byref(steps), _stream(stream)))
        return paths, steps.value

    def layer_sample(self, seed_offsets, seeds, fanouts, bias=UNIFORM, rng_seed=1, instance_base=0, rounds=0,
                     stream=None):
        """Layer sampling (csaw_layer_sample). Each instance's seeds must be
        sorted and distinct. Returns (src [ni, L, K], dst [ni, L, K], counts
        [ni, L]) int32 device tensors, K = max(fanouts), -1 padded."""
        so = np.ascontiguousarray(seed_offsets, dtype=np.int64)
        fo = np.ascontiguousarray(fanouts, dtype=np.int32)
        ni, L = len(so) - 1, len(fo)
        K = int(fo.max()) if L else 0
        sd = _dev_i32(seeds, self.device)
        src = torch.empty((ni, L, max(K, 1)), dtype=torch.int32, device=self.device)
        dst = torch.empty_like(src)
        counts = torch.empty((ni, max(L, 1)), dtype=torch.int32, device=self.device)
        a = LayerArgs()
        a.num_instances, a.seed_offsets = ni, so.ctypes.data
        a.seeds = sd.data_ptr() if sd.numel() else None
        a.instance_base, a.num_layers, a.fanouts = int(instance_base), L, fo.ctypes.data
        a.bias_kind, a.rng_seed, a.rounds = _bias_code(bias), int(rng_seed), int(rounds)
        _check(lib.csaw_layer_sample(self._h, ctypes.byref(a), src.data_ptr(), dst.data_ptr(), counts.data_ptr(),
                                     _stream(stream)))
        return src[:, :, :K], dst[:, :, :K], counts[:, :L]

    def mdrw(self, pool_offsets, pool, budget, rng_seed=1, instance_base=0, stream=None, out=None):
        """Multi-dimensional random walks (csaw_mdrw): one frontier pool per
        instance, ``budget`` steps each. Returns (src [ni, budget], dst
        [ni, budget], steps [ni] int64, all device tensors, total edges)."""
        po = np.ascontiguousarray(pool_offsets, dtype=np.int64)
        ni = len(po) - 1
        pl = _dev_i32(pool, self.device)
        if out is None:
            src = torch.empty((ni, budget), dtype=torch.int32, device=self.device)
            dst = torch.empty((ni, budget), dtype=torch.int32, device=self.device)
            steps = torch.empty(max(ni, 1), dtype=torch.int64, device=self.device)
        else:
            src, dst, steps = out
        a = MdrwArgs()
        a.num_instances = ni
        a.pool_offsets = po.ctypes.data
        a.pool = pl.data_ptr() if pl.numel() else None
        a.instance_base = int(instance_base)
        a.budget = int(budget)
        a.rng_seed = int(rng_seed)
        total = ctypes.c_int64()
        big = ni * budget > 0
        _check(lib.csaw_mdrw(self._h, ctypes.byref(a), src.data_ptr() if big else None,
                             dst.data_ptr() if big else None, steps.data_ptr(), ctypes.byref(total),
                             _stream(stream)))
        return src, dst, steps[:ni], total.value


class PartitionedGraph(Graph):
    """A graph kept in pinned host memory and streamed to the device in
    vertex-range partitions (csaw_pgraph_*): only the sampling calls apply."""

    def __init__(self, rowptr, col, edge_weight=None, num_partitions=4, max_resident=2, stream=None):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        ew = None if edge_weight is None else np.ascontiguousarray(edge_weight, dtype=np.uint32)
        n = len(rowptr) - 1
        h = ctypes.c_void_p()
        _check(lib.csaw_pgraph_create(n, len(col), rowptr.ctypes.data, col.ctypes.data,
                                      None if ew is None else ew.ctypes.data, int(num_partitions),
                                      int(max_resident), _stream(stream), ctypes.byref(h)))
        self._ph = h
        self._h = None
        self.n, self.m = n, len(col)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.last_stats = None

    def close(self):
        if getattr(self, "_ph", None):
            lib.csaw_pgraph_destroy(self._ph)
            self._ph = None

    def sample_bound(self, seed_offsets, fanouts, bias=UNIFORM) -> int:
        raise NotImplementedError("size the outputs with a resident Graph's sample_bound or pass capacity")

    def sample(self, seed_offsets, seeds, fanouts, bias=UNIFORM, rng_seed=1, instance_base=0,
               capacity=None, stream=None, out=None, instance_ids=None, rng_seeds=None, rounds=0,
               burn=0) -> SampleResult:
        """csaw_sample_streamed; ``capacity`` (or ``out``) is required. The
        call's partition loads are in ``last_stats`` afterwards."""
        if capacity is None and out is None:
            raise ValueError("a partitioned graph needs capacity= or out=")
        st = StreamStats()
        res = self._run_sample(lambda a, o: lib.csaw_sample_streamed(self._ph, a, o, _stream(stream),
                                                                     ctypes.byref(st)),
                               seed_offsets, seeds, fanouts, bias, rng_seed, instance_base, capacity, out,
                               instance_ids, rng_seeds, rounds, burn)
        self.last_stats = (st.partition_loads, st.bytes_loaded)
        return res


def profile_enable(on: bool = True):
    _check(lib.csaw_profile_enable(1 if on else 0))


def profile_reset():
    _check(lib.csaw_profile_reset())


def profile_read(prefix: str):
    """(total ms, launches) of kernels whose name starts with ``prefix``."""
    t, c = ctypes.c_double(), ctypes.c_int64()
    _check(lib.csaw_profile_read(prefix.encode(), ctypes.byref(t), ctypes.byref(c)))
    return t.value, c.value


class _ResultMemory:
    """Owns a server result (csaw_result); frees it once no array views it."""

    def __init__(self, rp):
        self.rp = rp

    def __del__(self):
        try:
            lib.csaw_result_free(self.rp)
        except Exception:
            pass


def _result_view(owner: _ResultMemory, cptr, n: int) -> np.ndarray:
    """int32 array over n elements of a result's host memory, without a copy:
    the array keeps the result alive."""
    buf = (ctypes.c_int32 * max(n, 1)).from_address(ctypes.cast(cptr, ctypes.c_void_p).value)
    buf._owner = owner
    return np.frombuffer(buf, dtype=np.int32)[:n]


class ServedResult:
    """A finished server request. Its edge and path arrays are views of the
    library's result memory (no copy), freed when the last of them goes."""

    def __init__(self, rp):
        r = rp.contents
        owner = _ResultMemory(rp)
        self.status = r.status
        self.kind = r.kind
        self.queued_us, self.total_us = r.queued_us, r.total_us
        self.batch_requests = r.batch_requests  # requests served by the same call
        if r.kind == 0 and r.status == 0:
            ne = r.num_edges
            self.src = _result_view(owner, r.src, ne)
            self.dst = _result_view(owner, r.dst, ne)
            self.layer_offsets = np.ctypeslib.as_array(r.layer_offsets, shape=(r.num_layers + 1,)).copy()
            self.num_edges = ne
        elif r.kind == 1 and r.status == 0:
            n = r.num_walkers * (r.length + 1)
            self.paths = _result_view(owner, r.paths, n).reshape(r.num_walkers, r.length + 1)
            self.steps = r.steps
            self.num_edges = r.steps


class Server:
    """Request server over a resident graph (csaw_server_*)."""

    def __init__(self, graph: Graph, memory_budget_bytes=0, max_batch=0, queue_capacity=0, num_streams=0,
                 max_batch_walkers=0, result_pool_bytes=0):
        cfg = ServerConfig(int(memory_budget_bytes), int(max_batch), int(queue_capacity), int(num_streams),
                           int(max_batch_walkers), int(result_pool_bytes))
        h = ctypes.c_void_p()
        _check(lib.csaw_server_create(graph._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.graph = graph

    def submit_sample(self, seeds, fanouts, bias=UNIFORM, rng_seed=1, request_id=0) -> int:
        sd = np.ascontiguousarray(seeds, dtype=np.int32)
        fo = np.ascontiguousarray(fanouts, dtype=np.int32)
        q = Request()
        q.kind, q.id, q.rng_seed, q.bias_kind = 0, int(request_id), int(rng_seed), _bias_code(bias)
        q.seeds, q.num_seeds = sd.ctypes.data, len(sd)
        q.fanouts, q.num_layers = fo.ctypes.data, len(fo)
        t = ctypes.c_uint64()
        _check(lib.csaw_server_submit(self._h, ctypes.byref(q), ctypes.byref(t)))
        return t.value

    def submit_walk(self, starts, length, bias=UNIFORM, rng_seed=1, request_id=0, node2vec=(1, 1, 1)) -> int:
        st = np.ascontiguousarray(starts, dtype=np.int32)
        q = Request()
        q.kind, q.id, q.rng_seed, q.bias_kind = 1, int(request_id), int(rng_seed), _bias_code(bias)
        q.starts, q.num_walkers, q.length = st.ctypes.data, len(st), int(length)
        q.w_return, q.w_common, q.w_outward = (int(x) for x in node2vec)
        t = ctypes.c_uint64()
        _check(lib.csaw_server_submit(self._h, ctypes.byref(q), ctypes.byref(t)))
        return t.value

    def _take(self, rp):
        return ServedResult(rp)

    def poll(self, ticket: int):
        rp = ctypes.POINTER(Result)()
        st = lib.csaw_server_poll(self._h, ticket, ctypes.byref(rp))
        if st == 5:
            return None
        _check(st)
        return self._take(rp)

    def wait(self, ticket: int, timeout_us: int = -1):
        rp = ctypes.POINTER(Result)()
        st = lib.csaw_server_wait(self._h, ticket, int(timeout_us), ctypes.byref(rp))
        if st == 5:
            return None
        _check(st)
        return self._take(rp)

    def cancel(self, ticket: int) -> bool:
        """Withdraws a request that has not started (csaw_server_cancel); its
        result then has status CANCELLED. False if it already runs or ran."""
        st = lib.csaw_server_cancel(self._h, ticket)
        if st == 4:
            return False
        _check(st)
        return True

    def memory(self):
        """(device bytes, pinned host bytes) the server holds."""
        d, h = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.csaw_server_memory(self._h, ctypes.byref(d), ctypes.byref(h)))
        return d.value, h.value

    def close(self):
        if getattr(self, "_h", None):
            lib.csaw_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
