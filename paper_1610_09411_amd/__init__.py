"""Exact induced 4- and 5-vertex subgraph counts on an MI355X (gfx950).

Thin ctypes binding over ``libescape.so`` (C ABI in ``include/escape.h``); the
functions keep the ABI's names.  Every step of the computation runs in the
library's HIP kernels; this module only marshals arguments.  PyTorch is used
for device memory and streams when the caller passes device tensors.

    import paper_1610_09411_amd as esc
    ctx = esc.esc_create(0)
    counts = esc.esc_count_subgraphs(ctx, n, row_ptr, col, k=5)   # 45 Python ints
    esc.esc_destroy(ctx)

The library must have been built (``python -m paper_1610_09411_amd.build``);
without it every call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libescape.so")

ESC_OK, ESC_EINVAL, ESC_ENOTSIMPLE, ESC_ERANGE, ESC_ENOMEM, ESC_EDEVICE, ESC_EOVERFLOW, ESC_EBUSY = range(8)
ESC_F_VALIDATE = 1
ESC_F_CANONICALIZE = 2
ESC_F_INPUT_ON_DEVICE = 4
ESC_F_RANDOM_ORDER = 8
ESC_F_COMPACT_LISTS = 16

ABI_FUNCTIONS = [
    "esc_create", "esc_destroy", "esc_count_subgraphs", "esc_count_subgraphs_noalloc", "esc_count_fragments",
    "esc_count_batched",
    "esc_server_start", "esc_submit", "esc_poll", "esc_wait", "esc_server_stats", "esc_server_stop",
    "esc_tune", "esc_tune_batched", "esc_set_params", "esc_last_params",
    "esc_last_work", "esc_last_profile", "esc_last_products", "esc_last_noninduced", "esc_last_three", "esc_inverse_matrix", "esc_strerror",
]

PATTERN_NAMES = [
    "3-star", "3-path", "tailed-triangle", "4-cycle", "diamond", "4-clique",
    "4-ind-set", "4-only-edge", "4-matching", "4-only-wedge", "4-only-triangle",
] + ["P%d" % i for i in range(1, 22)] + [
    "5-ind-set", "5-only-edge", "5-matching", "5-only-wedge", "5-only-triangle",
    "5-only-3-star", "5-only-3-path", "5-only-tailed-triangle", "5-only-4-cycle",
    "5-only-diamond", "5-only-4-clique", "5-wedge+edge", "5-triangle+edge",
]


class EscapeError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s: %s (status %d)" % (where, esc_strerror(status), status))


class _U128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]


class _Params(ctypes.Structure):
    _fields_ = [("task_chunk", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32), ("k5_work_log2", ctypes.c_int32),
                ("five_order", ctypes.c_int32), ("k5_light", ctypes.c_int32), ("k5_wave_words", ctypes.c_int32),
                ("k5_dense_pct", ctypes.c_int32), ("wheel_split_deg", ctypes.c_int32),
                ("four_range_deg", ctypes.c_int32), ("pairs_hub_ranks", ctypes.c_int32),
                ("pairs_hub_q", ctypes.c_int32), ("wheel_dense_deg", ctypes.c_int32),
                ("wheel_dense_ratio", ctypes.c_int32), ("k4_dense_dplus", ctypes.c_int32)]


# defaults of the fields a set_params dict may leave out
PARAM_DEFAULTS = {"five_order": 0, "k5_light": 64, "k5_wave_words": 8, "k5_dense_pct": 50,
                  "wheel_split_deg": 1024, "four_range_deg": 256, "pairs_hub_ranks": -1,
                  "pairs_hub_q": 256, "wheel_dense_deg": 1024, "wheel_dense_ratio": 1024,
                  "k4_dense_dplus": 128}


def _params_dict(p):
    return {name: int(getattr(p, name)) for name, _ in _Params._fields_}


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libescape.so is not built; run `python -m paper_1610_09411_amd.build`")
        # One HIP runtime per process: PyTorch ships its own libamdhip64 with the
        # same soname, so load it first and let the library bind to that copy.
        try:
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover
            pass
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
        lib.esc_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_size_t]
        lib.esc_create.restype = ctypes.c_int
        lib.esc_destroy.argtypes = [vp]
        lib.esc_destroy.restype = None
        lib.esc_count_subgraphs.argtypes = [vp, i32, vp, vp, ctypes.c_int, u32, vp, vp]
        lib.esc_count_subgraphs.restype = ctypes.c_int
        lib.esc_count_subgraphs_noalloc.argtypes = [vp, i32, vp, vp, ctypes.c_int, u32, vp, vp]
        lib.esc_count_subgraphs_noalloc.restype = ctypes.c_int
        lib.esc_count_fragments.argtypes = [vp, i32, vp, vp, ctypes.c_int, u32, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.esc_count_fragments.restype = ctypes.c_int
        lib.esc_count_batched.argtypes = [vp, i32, vp, vp, vp, vp, ctypes.c_int, u32, vp, vp, vp]
        lib.esc_count_batched.restype = ctypes.c_int
        lib.esc_server_start.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp)]
        lib.esc_server_start.restype = ctypes.c_int
        lib.esc_submit.argtypes = [vp, i32, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
        lib.esc_submit.restype = ctypes.c_int
        lib.esc_poll.argtypes = [vp, ctypes.c_uint64, vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        lib.esc_poll.restype = ctypes.c_int
        lib.esc_wait.argtypes = [vp, ctypes.c_uint64, vp, ctypes.POINTER(ctypes.c_double)]
        lib.esc_wait.restype = ctypes.c_int
        lib.esc_server_stats.argtypes = [vp, vp]
        lib.esc_server_stats.restype = ctypes.c_int
        lib.esc_server_stop.argtypes = [vp]
        lib.esc_server_stop.restype = ctypes.c_int
        lib.esc_tune.argtypes = [vp, i32, vp, vp, ctypes.c_int, u32, vp, vp, vp]
        lib.esc_tune.restype = ctypes.c_int
        lib.esc_tune_batched.argtypes = [vp, i32, vp, vp, vp, vp, ctypes.c_int, u32, vp, vp, vp]
        lib.esc_tune_batched.restype = ctypes.c_int
        lib.esc_set_params.argtypes = [vp, vp]
        lib.esc_set_params.restype = ctypes.c_int
        lib.esc_last_params.argtypes = [vp, vp]
        lib.esc_last_params.restype = ctypes.c_int
        lib.esc_last_work.argtypes = [vp, vp]
        lib.esc_last_work.restype = ctypes.c_int
        lib.esc_last_profile.argtypes = [vp, vp, vp]
        lib.esc_last_profile.restype = ctypes.c_int
        lib.esc_last_products.argtypes = [vp, vp, vp, vp]
        lib.esc_last_products.restype = ctypes.c_int
        lib.esc_last_noninduced.argtypes = [vp, vp]
        lib.esc_last_noninduced.restype = ctypes.c_int
        lib.esc_last_three.argtypes = [vp, vp]
        lib.esc_last_three.restype = ctypes.c_int
        lib.esc_inverse_matrix.argtypes = [ctypes.c_int, vp]
        lib.esc_inverse_matrix.restype = ctypes.c_int
        lib.esc_strerror.argtypes = [ctypes.c_int]
        lib.esc_strerror.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def esc_strerror(status: int) -> str:
    return _load().esc_strerror(status).decode()


def _check(status, where):
    if status != ESC_OK:
        raise EscapeError(status, where)


class Context:
    """Owns an ``esc_ctx``; usable as a context manager."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.ptr = esc_create(device, hbm_budget_bytes)

    def close(self):
        if self.ptr:
            esc_destroy(self.ptr)
            self.ptr = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def count(self, graph, k=5, flags=0, stream=None):
        return esc_count_subgraphs(self.ptr, graph.n, graph.row_ptr, graph.col, k, flags, stream)

    def fragments(self, graph, k=5, flags=0, stream=None):
        return esc_count_fragments(self.ptr, graph.n, graph.row_ptr, graph.col, k, flags, stream)

    def count_batched(self, graphs, k=5, flags=0, stream=None):
        """Counts of every graph in `graphs` (objects with n, row_ptr, col) in
        one call: a G x (11|45) uint64 array and the per-graph overflow flags."""
        return esc_count_batched(self.ptr, *pack_batch(graphs), k=k, flags=flags, stream=stream)

    def tune(self, graph, k=5, flags=0, stream=None):
        """Time the candidate launch parameters on this graph; the fastest are
        kept for graphs with the same degree statistics.  Returns (params, ms)."""
        rp, ci, flags, keep = _csr_args(graph.row_ptr, graph.col, flags)
        best = _Params()
        ms = ctypes.c_float()
        _check(_load().esc_tune(self.ptr, int(graph.n), rp, ci, int(k), flags, ctypes.byref(best), ctypes.byref(ms),
                                _stream_ptr(stream)), "esc_tune")
        del keep
        return _params_dict(best), float(ms.value)

    def tune_batched(self, graphs, k=5, flags=0, stream=None):
        vo, ao, rp, ci = pack_batch(graphs)
        rpp, cip, flags, keep = _csr_args(rp, ci, flags)
        best = _Params()
        ms = ctypes.c_float()
        _check(_load().esc_tune_batched(self.ptr, len(graphs), vo.ctypes.data_as(ctypes.c_void_p),
                                        ao.ctypes.data_as(ctypes.c_void_p), rpp, cip, int(k), flags,
                                        ctypes.byref(best), ctypes.byref(ms), _stream_ptr(stream)), "esc_tune_batched")
        del keep
        return _params_dict(best), float(ms.value)

    def set_params(self, params):
        """Force launch parameters (dict with task_chunk, wg_per_cu,
        k5_work_log2 and optionally the fields of PARAM_DEFAULTS) on later
        calls; None returns to the tuned/default ones."""
        if params is None:
            _check(_load().esc_set_params(self.ptr, None), "esc_set_params")
            return
        full = dict(PARAM_DEFAULTS)
        full.update(params)
        p = _Params(*[int(full[name]) for name, _ in _Params._fields_])
        _check(_load().esc_set_params(self.ptr, ctypes.byref(p)), "esc_set_params")

    def last_params(self):
        p = _Params()
        _check(_load().esc_last_params(self.ptr, ctypes.byref(p)), "esc_last_params")
        return _params_dict(p)

    def last_work(self):
        return esc_last_work(self.ptr)

    def last_profile(self):
        return esc_last_profile(self.ptr)

    def last_products(self):
        return esc_last_products(self.ptr)

    def last_noninduced(self, k=5):
        return esc_last_noninduced(self.ptr, k)

    def last_three(self):
        return esc_last_three(self.ptr)


def esc_create(device: int = 0, hbm_budget_bytes: int = 0):
    ptr = ctypes.c_void_p()
    _check(_load().esc_create(ctypes.byref(ptr), device, hbm_budget_bytes), "esc_create")
    return ptr


def esc_destroy(ctx):
    _load().esc_destroy(ctx)


def _csr_args(row_ptr, col, flags):
    """Pointers for host numpy arrays or device torch tensors."""
    try:
        import torch
        is_dev = isinstance(row_ptr, torch.Tensor) and row_ptr.is_cuda
    except ImportError:  # pragma: no cover
        is_dev = False
    if is_dev:
        if row_ptr.dtype != torch.int32 or col.dtype != torch.int32:
            raise TypeError("device CSR must be int32")
        return (ctypes.c_void_p(row_ptr.data_ptr()), ctypes.c_void_p(col.data_ptr()),
                flags | ESC_F_INPUT_ON_DEVICE, (row_ptr, col))
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    return rp.ctypes.data_as(ctypes.c_void_p), ci.ctypes.data_as(ctypes.c_void_p), flags, (rp, ci)


def _stream_ptr(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ints(buf, cnt):
    return [buf[i].lo | (buf[i].hi << 64) for i in range(cnt)]


def esc_count_subgraphs(ctx, n, row_ptr, col, k=5, flags=0, stream=None):
    """Induced counts of all k-vertex patterns (11 for k=4, 45 for k=5)."""
    rp, ci, flags, keep = _csr_args(row_ptr, col, flags)
    out = (_U128 * 45)()
    st = _load().esc_count_subgraphs(ctx, int(n), rp, ci, int(k), flags, out, _stream_ptr(stream))
    _check(st, "esc_count_subgraphs")
    del keep
    return _ints(out, 11 if k == 4 else 45)


def esc_count_subgraphs_noalloc(ctx, n, row_ptr, col, k=5, flags=0, stream=None):
    """esc_count_subgraphs with every device buffer taken from the library's
    fixed per-GPU region (no device allocation by the call)."""
    rp, ci, flags, keep = _csr_args(row_ptr, col, flags)
    out = (_U128 * 45)()
    st = _load().esc_count_subgraphs_noalloc(ctx, int(n), rp, ci, int(k), flags, out, _stream_ptr(stream))
    _check(st, "esc_count_subgraphs_noalloc")
    del keep
    return _ints(out, 11 if k == 4 else 45)


def esc_count_fragments(ctx, n, row_ptr, col, k=5, flags=0, stream=None):
    """Counts plus per-vertex / per-arc fragment arrays (numpy uint64):
    returns (counts, {"tri_v","c4_v","k4_v","tri_e","c4_e","k4_e"})."""
    rp, ci, flags, keep = _csr_args(row_ptr, col, flags)
    m2 = int(keep[0][-1]) if not (flags & ESC_F_INPUT_ON_DEVICE) else int(keep[0][-1].item())
    arrs = {name: np.zeros(int(n) if name.endswith("_v") else m2, dtype=np.uint64)
            for name in ("tri_v", "c4_v", "k4_v", "tri_e", "c4_e", "k4_e")}
    ptrs = [arrs[x].ctypes.data_as(ctypes.c_void_p) for x in ("tri_v", "c4_v", "k4_v", "tri_e", "c4_e", "k4_e")]
    out = (_U128 * 45)()
    st = _load().esc_count_fragments(ctx, int(n), rp, ci, int(k), flags, out, *ptrs, _stream_ptr(stream))
    _check(st, "esc_count_fragments")
    del keep
    return _ints(out, 11 if k == 4 else 45), arrs


def pack_batch(graphs):
    """Concatenate graphs into the batched layout: (vtx_off, arc_off, row_ptr,
    col) with vtx_off/arc_off int64 of G+1 entries, every graph's n+1 local row
    offsets back to back and its local column ids back to back."""
    G = len(graphs)
    vtx_off = np.zeros(G + 1, dtype=np.int64)
    arc_off = np.zeros(G + 1, dtype=np.int64)
    for g, x in enumerate(graphs):
        vtx_off[g + 1] = vtx_off[g] + int(x.n)
        arc_off[g + 1] = arc_off[g] + int(len(x.col))
    rps = [np.asarray(x.row_ptr, dtype=np.int32) for x in graphs]
    cols = [np.asarray(x.col, dtype=np.int32) for x in graphs]
    row_ptr = np.concatenate(rps) if G else np.zeros(0, np.int32)
    col = np.concatenate(cols) if G else np.zeros(0, np.int32)
    return vtx_off, arc_off, row_ptr, col


def esc_count_batched(ctx, vtx_off, arc_off, row_ptr, col, k=5, flags=0, stream=None):
    """Per-graph induced counts of a batch (layout of pack_batch): returns a
    (G, 11|45) uint64 array and a (G,) uint8 array of overflow flags."""
    vo = np.ascontiguousarray(vtx_off, dtype=np.int64)
    ao = np.ascontiguousarray(arc_off, dtype=np.int64)
    G = len(vo) - 1
    if G < 0 or len(ao) != len(vo):
        raise ValueError("vtx_off and arc_off need G+1 entries each")
    rp, ci, flags, keep = _csr_args(row_ptr, col, flags)
    cnt = 11 if k == 4 else 45
    out = np.zeros((max(G, 0), cnt), dtype=np.uint64)
    ovf = np.zeros(max(G, 0), dtype=np.uint8)
    st = _load().esc_count_batched(ctx, int(G), vo.ctypes.data_as(ctypes.c_void_p),
                                   ao.ctypes.data_as(ctypes.c_void_p), rp, ci, int(k), flags,
                                   out.ctypes.data_as(ctypes.c_void_p), ovf.ctypes.data_as(ctypes.c_void_p),
                                   _stream_ptr(stream))
    _check(st, "esc_count_batched")
    del keep
    return out, ovf


class Server:
    """Request loop (esc_server_*): submit graphs, collect exact counts.

    ``submit`` copies the CSR and returns a ticket at once; ``poll`` returns
    None while the request is pending, else ``(counts, seconds)``; ``wait``
    blocks.  A failed request raises EscapeError from poll / wait."""

    def __init__(self, ctx, max_inflight=4):
        self._keep_ctx = ctx
        ptr = ctypes.c_void_p()
        _check(_load().esc_server_start(ctx.ptr if isinstance(ctx, Context) else ctx, int(max_inflight),
                                        ctypes.byref(ptr)), "esc_server_start")
        self.ptr = ptr

    def submit(self, graph, k=5):
        rp = np.ascontiguousarray(graph.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(graph.col, dtype=np.int32)
        t = ctypes.c_uint64()
        _check(_load().esc_submit(self.ptr, int(graph.n), rp.ctypes.data_as(ctypes.c_void_p),
                                  ci.ctypes.data_as(ctypes.c_void_p), int(k), ctypes.byref(t)), "esc_submit")
        return (int(t.value), int(k))

    def poll(self, ticket):
        t, k = ticket
        out = (_U128 * 45)()
        done = ctypes.c_int()
        sec = ctypes.c_double()
        _check(_load().esc_poll(self.ptr, t, out, ctypes.byref(done), ctypes.byref(sec)), "esc_poll")
        if not done.value:
            return None
        return _ints(out, 11 if k == 4 else 45), float(sec.value)

    def wait(self, ticket):
        t, k = ticket
        out = (_U128 * 45)()
        sec = ctypes.c_double()
        _check(_load().esc_wait(self.ptr, t, out, ctypes.byref(sec)), "esc_wait")
        return _ints(out, 11 if k == 4 else 45), float(sec.value)

    def stats(self):
        out = (ctypes.c_uint64 * 8)()
        _check(_load().esc_server_stats(self.ptr, out), "esc_server_stats")
        keys = ["completed", "launches", "batched_requests", "peak_inflight", "peak_reserved_bytes",
                "budget_bytes", "queued", "workers"]
        return dict(zip(keys, [int(x) for x in out]))

    def stop(self):
        if self.ptr:
            _check(_load().esc_server_stop(self.ptr), "esc_server_stop")
            self.ptr = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()


def esc_last_work(ctx):
    out = (ctypes.c_uint64 * 10)()
    _check(_load().esc_last_work(ctx, out), "esc_last_work")
    keys = ["W++", "W+-", "W", "T", "D", "max_dplus", "n", "m", "DP", "DBP"]
    return dict(zip(keys, [int(x) for x in out]))


def esc_last_noninduced(ctx, k=5):
    """Non-induced counts of the last call (same order as its induced output)."""
    out = (_U128 * 45)()
    _check(_load().esc_last_noninduced(ctx, out), "esc_last_noninduced")
    return _ints(out, 11 if k == 4 else 45)


def esc_last_three(ctx):
    """Induced 3-vertex counts of the last call: [no edge, one edge, path, triangle]."""
    out = (_U128 * 4)()
    _check(_load().esc_last_three(ctx, out), "esc_last_three")
    return _ints(out, 4)


STAGES = ["orient", "triangles", "four_cycles", "k4_triangles", "five_cliques", "reduce", "pairs_13_17",
          "wheels", "five_cycles", "combine"]


def esc_last_profile(ctx):
    """{stage: (device ms, elements visited)} of the last call."""
    ms = (ctypes.c_float * len(STAGES))()
    vis = (ctypes.c_uint64 * len(STAGES))()
    _check(_load().esc_last_profile(ctx, ms, vis), "esc_last_profile")
    return {k: (float(ms[i]), int(vis[i])) for i, k in enumerate(STAGES)}


def esc_last_products(ctx):
    """{stage: (walk ms, product ms, product multiply-adds)} of the last call."""
    w = (ctypes.c_float * len(STAGES))()
    p = (ctypes.c_float * len(STAGES))()
    mac = (ctypes.c_uint64 * len(STAGES))()
    _check(_load().esc_last_products(ctx, w, p, mac), "esc_last_products")
    return {k: (float(w[i]), float(p[i]), int(mac[i])) for i, k in enumerate(STAGES)}


def esc_inverse_matrix(k):
    """The library's signed inverse of the induced-to-non-induced matrix
    (11x11 for k=4, 34x34 for k=5), host-only."""
    cnt = 11 if k == 4 else 34
    out = (ctypes.c_int32 * (cnt * cnt))()
    _check(_load().esc_inverse_matrix(int(k), out), "esc_inverse_matrix")
    return [[int(out[i * cnt + j]) for j in range(cnt)] for i in range(cnt)]
