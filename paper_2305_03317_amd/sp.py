"""Python binding of ``libsp.so`` (C ABI in ``include/sp.h``).

Argument marshalling only: every step of the BC computation runs in the HIP
library.  torch supplies device memory (CUDA tensors) and the current stream;
functions take and return torch tensors.  The library must be built
(``python -m paper_2305_03317_amd._build``); importing this module without it
raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsp.so")

SP_OK = 0
SP_WARN_SIGMA_LARGE = 1
SP_ERR_INVALID_ARGUMENT = -1
SP_ERR_OUT_OF_MEMORY = -2
SP_ERR_DEVICE = -3
SP_ERR_NOT_SUPPORTED = -4
SP_ERR_REJECTED = -5
SP_ERR_TIMEOUT = -6
SP_ERR_CANCELLED = -7
SP_PTR_DEVICE = 1
SP_VALIDATE = 2
SP_SSSP_AUTO = 0
SP_SSSP_PUSH = 1
SP_SSSP_PULL = 2
SP_ENGINE_AUTO = 0
SP_ENGINE_BITMAP = 1
SP_ENGINE_BLOCKS = 2


class sp_batch_config(ctypes.Structure):
    _fields_ = [("batch_width", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("chunk_levels", ctypes.c_int32), ("engine", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class sp_stats(ctypes.Structure):
    _fields_ = [("n_sources", ctypes.c_int32), ("n_passes", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("sigma_flagged", ctypes.c_int32),
                ("levels_total", ctypes.c_int64), ("topdown_levels", ctypes.c_int64),
                ("bottomup_levels", ctypes.c_int64), ("reached_total", ctypes.c_int64),
                ("sigma_max", ctypes.c_double), ("device_ms", ctypes.c_double),
                ("batch_width", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("chunk_levels", ctypes.c_int32), ("graph_launches", ctypes.c_int32),
                ("group_ms", ctypes.c_double), ("engine", ctypes.c_int32)]


SP_TUNE_MAX_CANDIDATES = 16


class sp_tune_candidate(ctypes.Structure):
    _fields_ = [("cfg", sp_batch_config), ("ms_per_source", ctypes.c_double),
                ("accepted", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class sp_tune_report(ctypes.Structure):
    _fields_ = [("fingerprint", ctypes.c_uint64), ("from_cache", ctypes.c_int32),
                ("sample_sources", ctypes.c_int32), ("repetitions", ctypes.c_int32),
                ("n_candidates", ctypes.c_int32), ("tuning_ms", ctypes.c_double),
                ("group_ms", ctypes.c_double), ("chosen", sp_batch_config),
                ("cand", sp_tune_candidate * SP_TUNE_MAX_CANDIDATES)]


class sp_sssp_config(ctypes.Structure):
    _fields_ = [("direction", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("chunk_rounds", ctypes.c_int32),
                ("max_blocks", ctypes.c_int32), ("local_hops", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 1)]


class sp_sssp_stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("push_rounds", ctypes.c_int32),
                ("pull_rounds", ctypes.c_int32), ("reached", ctypes.c_int32),
                ("device_ms", ctypes.c_double), ("graph_launches", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("direction", ctypes.c_int32), ("chunk_rounds", ctypes.c_int32),
                ("local_hops", ctypes.c_int32)]


class sp_pagerank_config(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_int32), ("chunk_iters", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


class sp_pagerank_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("graph_launches", ctypes.c_int32),
                ("diff", ctypes.c_double), ("device_ms", ctypes.c_double)]


class sp_tc_stats(ctypes.Structure):
    _fields_ = [("triangles", ctypes.c_int64), ("oriented_edges", ctypes.c_int64),
                ("build_ms", ctypes.c_double), ("count_ms", ctypes.c_double)]


class sp_server_config(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_size_t), ("max_batch", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


class sp_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("passes", ctypes.c_int64),
                ("slots_used", ctypes.c_int64), ("edges_traversed", ctypes.c_int64),
                ("admitted_bytes", ctypes.c_size_t), ("peak_admitted_bytes", ctypes.c_size_t),
                ("queue_depth", ctypes.c_int32), ("in_flight", ctypes.c_int32),
                ("workspaces_created", ctypes.c_int64), ("workspaces_evicted", ctypes.c_int64)]


class sp_kernel_profile(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("items", ctypes.c_int64),
                ("edges", ctypes.c_int64), ("pairs", ctypes.c_int64),
                ("item_slots", ctypes.c_int64)]


def _struct_dict(s):
    return {k: (list(getattr(s, k)) if k == "reserved" else getattr(s, k)) for k, _ in s._fields_}


_I32P = ctypes.POINTER(ctypes.c_int32)
_VP = ctypes.c_void_p
_ST = ctypes.c_int32

# (name, restype, argtypes) of every exported entry point.
SIGNATURES = [
    ("sp_status_string", ctypes.c_char_p, [_ST]),
    ("sp_last_error", ctypes.c_char_p, []),
    ("sp_version", ctypes.c_int32, []),
    ("sp_header_hash", ctypes.c_uint64, []),
    ("sp_graph_upload", _ST, [ctypes.c_int32, ctypes.c_int64, _VP, _VP, ctypes.c_uint32, _VP,
                              ctypes.POINTER(_VP)]),
    ("sp_graph_upload_directed", _ST, [ctypes.c_int32, ctypes.c_int64, _VP, _VP, ctypes.c_uint32, _VP,
                                       ctypes.POINTER(_VP)]),
    ("sp_graph_release", _ST, [_VP]),
    ("sp_graph_info", _ST, [_VP, _I32P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_size_t)]),
    ("sp_bc", _ST, [_VP, _I32P, ctypes.c_int32, _VP, _VP]),
    ("sp_bc_batch", _ST, [_VP, _I32P, ctypes.c_int32, _VP, ctypes.POINTER(sp_batch_config), _VP]),
    ("sp_bc_noalloc", _ST, [_VP, _I32P, ctypes.c_int32, _VP, _VP]),
    ("sp_get_last_stats", _ST, [ctypes.POINTER(sp_stats)]),
    ("sp_bfs_levels", _ST, [_VP, ctypes.c_int32, _VP, _VP, _VP, _VP]),
    ("sp_batch_levels", _ST, [_VP, _I32P, ctypes.c_int32, _VP, _VP, _VP,
                              ctypes.POINTER(sp_batch_config), _VP]),
    ("sp_bc_workspace_bytes", _ST, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    ("sp_autotune", _ST, [_VP, _I32P, ctypes.c_int32, ctypes.POINTER(sp_batch_config), _VP]),
    ("sp_autotune_get_last_report", _ST, [ctypes.POINTER(sp_tune_report)]),
    ("sp_graph_fingerprint", _ST, [_VP, ctypes.POINTER(ctypes.c_uint64)]),
    ("sp_graph_set_tuned", _ST, [_VP, ctypes.POINTER(sp_batch_config)]),
    ("sp_tune_cache_clear", _ST, []),
    ("sp_graph_set_weights", _ST, [_VP, _VP, ctypes.c_uint32, _VP]),
    ("sp_sssp", _ST, [_VP, ctypes.c_int32, _VP, ctypes.POINTER(sp_sssp_config), _VP]),
    ("sp_sssp_get_last_stats", _ST, [ctypes.POINTER(sp_sssp_stats)]),
    ("sp_pagerank", _ST, [_VP, ctypes.c_double, ctypes.c_double, ctypes.c_int32, _VP,
                          ctypes.POINTER(sp_pagerank_config), _VP]),
    ("sp_pagerank_get_last_stats", _ST, [ctypes.POINTER(sp_pagerank_stats)]),
    ("sp_triangle_count", _ST, [_VP, ctypes.POINTER(ctypes.c_int64), _VP, _VP]),
    ("sp_tc_get_last_stats", _ST, [ctypes.POINTER(sp_tc_stats)]),
    ("sp_profile_enable", _ST, [ctypes.c_int32]),
    ("sp_profile_read", _ST, [ctypes.POINTER(sp_kernel_profile), ctypes.c_int32, _I32P]),
    ("sp_server_create", _ST, [ctypes.POINTER(sp_server_config), ctypes.POINTER(_VP)]),
    ("sp_server_add_graph", _ST, [_VP, _VP, _I32P]),
    ("sp_stream_submit", _ST, [_VP, ctypes.c_int32, _I32P, ctypes.c_int32, _VP, ctypes.POINTER(_VP)]),
    ("sp_request_wait", _ST, [_VP, ctypes.c_int64, _I32P]),
    ("sp_request_poll", _ST, [_VP, _I32P, _I32P]),
    ("sp_request_cancel", _ST, [_VP]),
    ("sp_request_latency_us", _ST, [_VP, ctypes.POINTER(ctypes.c_double)]),
    ("sp_request_release", _ST, [_VP]),
    ("sp_server_get_stats", _ST, [_VP, ctypes.POINTER(sp_server_stats)]),
    ("sp_server_destroy", _ST, [_VP]),
]

_lib = None


def lib():
    """The loaded libsp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsp.so is not built (run python -m paper_2305_03317_amd._build); "
                               "there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        from . import _build
        if L.sp_header_hash() != _build.header_hash():
            raise RuntimeError("libsp.so was built from another version of include/sp.h "
                               "(rebuild with python -m paper_2305_03317_amd._build)")
        _lib = L
    return _lib


class SpError(RuntimeError):
    def __init__(self, status, where):
        L = lib()
        self.status = status
        detail = L.sp_last_error().decode()
        super().__init__("%s: %s (%d)%s" % (where, L.sp_status_string(status).decode(), status,
                                            (": " + detail) if detail else ""))


def _check(status, where):
    if status < 0:
        raise SpError(status, where)
    return status


def sp_status_string(status: int) -> str:
    return lib().sp_status_string(status).decode()


def sp_last_error() -> str:
    return lib().sp_last_error().decode()


def sp_version() -> int:
    return lib().sp_version()


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _host_i32(a):
    a = np.ascontiguousarray(np.asarray(a), dtype=np.int32)
    return a, a.ctypes.data_as(_I32P)


class Graph:
    """An uploaded graph (library-owned device CSR)."""

    def __init__(self, handle, n, nnz):
        self.handle = handle
        self.n = n
        self.nnz = nnz

    def release(self):
        if self.handle:
            _check(lib().sp_graph_release(self.handle), "sp_graph_release")
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def sp_graph_upload(row_ptr, col_idx, validate: bool = False, stream=None, directed: bool = False) -> Graph:
    """Upload CSR arrays (numpy / host or CUDA torch tensors) to the device;
    directed=True treats row u as u's out-edges (sp_graph_upload_directed)."""
    torch = _torch()
    flags = SP_VALIDATE if validate else 0
    keep = []
    if isinstance(row_ptr, torch.Tensor) and row_ptr.is_cuda:
        rp = row_ptr.to(torch.int32).contiguous()
        ci = col_idx.to(torch.int32).contiguous()
        keep += [rp, ci]
        rp_ptr, ci_ptr = rp.data_ptr(), ci.data_ptr()
        n, nnz = rp.numel() - 1, ci.numel()
        flags |= SP_PTR_DEVICE
    else:
        rp = np.ascontiguousarray(np.asarray(row_ptr), dtype=np.int32)
        ci = np.ascontiguousarray(np.asarray(col_idx), dtype=np.int32)
        if ci.size == 0:
            ci = np.zeros(1, np.int32)
            nnz = 0
        else:
            nnz = ci.size
        keep += [rp, ci]
        rp_ptr, ci_ptr = rp.ctypes.data, ci.ctypes.data
        n = rp.size - 1
    h = ctypes.c_void_p()
    up = lib().sp_graph_upload_directed if directed else lib().sp_graph_upload
    _check(up(n, nnz, rp_ptr, ci_ptr, flags, _stream(stream), ctypes.byref(h)), "sp_graph_upload")
    return Graph(h, n, nnz)


def sp_graph_release(g: Graph):
    g.release()


def sp_graph_info(g: Graph):
    n = ctypes.c_int32()
    nnz = ctypes.c_int64()
    b = ctypes.c_size_t()
    _check(lib().sp_graph_info(g.handle, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(b)),
           "sp_graph_info")
    return dict(n_vertices=n.value, nnz=nnz.value, device_bytes=b.value)


def _out_f64(g, out):
    torch = _torch()
    if out is None:
        out = torch.empty(max(g.n, 1), dtype=torch.float64, device="cuda")
    assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() >= g.n
    return out


def _config(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, sp_batch_config):
        return ctypes.byref(cfg)
    c = sp_batch_config()
    for k, v in cfg.items():
        setattr(c, k, v)
    return ctypes.byref(c)


def sp_bc(g: Graph, sources, out_bc=None, stream=None):
    """Per-source path. Returns (out_bc[:V] tensor, status)."""
    out_bc = _out_f64(g, out_bc)
    src, p = _host_i32(sources)
    st = _check(lib().sp_bc(g.handle, p, len(src), out_bc.data_ptr(), _stream(stream)), "sp_bc")
    return out_bc[:g.n], st


def sp_bc_batch(g: Graph, sources, out_bc=None, config=None, stream=None):
    """Batched (multi-source bitmap) path. Returns (out_bc[:V] tensor, status)."""
    out_bc = _out_f64(g, out_bc)
    src, p = _host_i32(sources)
    st = _check(lib().sp_bc_batch(g.handle, p, len(src), out_bc.data_ptr(), _config(config),
                                  _stream(stream)), "sp_bc_batch")
    return out_bc[:g.n], st


def sp_bc_noalloc(g: Graph, sources, out_bc=None, stream=None):
    """sp_bc on the library's fixed device workspace (no allocation inside the
    call; graphs up to about 1.6M vertices). Returns (out_bc[:V], status)."""
    out_bc = _out_f64(g, out_bc)
    src, p = _host_i32(sources)
    st = _check(lib().sp_bc_noalloc(g.handle, p, len(src), out_bc.data_ptr(), _stream(stream)),
                "sp_bc_noalloc")
    return out_bc[:g.n], st


def sp_get_last_stats() -> dict:
    s = sp_stats()
    _check(lib().sp_get_last_stats(ctypes.byref(s)), "sp_get_last_stats")
    return _struct_dict(s)


def sp_bfs_levels(g: Graph, source: int, with_sigma=True, with_delta=False, stream=None):
    """(dist int32, sigma f64 or None, delta f64 or None, status) of one source."""
    torch = _torch()
    n = max(g.n, 1)
    dist = torch.empty(n, dtype=torch.int32, device="cuda")
    sigma = torch.empty(n, dtype=torch.float64, device="cuda") if with_sigma else None
    delta = torch.empty(n, dtype=torch.float64, device="cuda") if with_delta else None
    st = _check(lib().sp_bfs_levels(g.handle, int(source), dist.data_ptr(),
                                    sigma.data_ptr() if sigma is not None else None,
                                    delta.data_ptr() if delta is not None else None,
                                    _stream(stream)), "sp_bfs_levels")
    cut = lambda t: None if t is None else t[:g.n]
    return dist[:g.n], cut(sigma), cut(delta), st


def sp_batch_levels(g: Graph, sources, with_sigma=True, with_delta=True, config=None, stream=None):
    """Per-source (dist, sigma, delta) of one multi-source pass, shape [len(sources), V]."""
    torch = _torch()
    src, p = _host_i32(sources)
    k = len(src)
    shape = (k, max(g.n, 1))
    dist = torch.empty(shape, dtype=torch.int32, device="cuda")
    sigma = torch.empty(shape, dtype=torch.float64, device="cuda") if with_sigma else None
    delta = torch.empty(shape, dtype=torch.float64, device="cuda") if with_delta else None
    st = _check(lib().sp_batch_levels(g.handle, p, k, dist.data_ptr(),
                                      sigma.data_ptr() if sigma is not None else None,
                                      delta.data_ptr() if delta is not None else None,
                                      _config(config), _stream(stream)), "sp_batch_levels")
    cut = lambda t: None if t is None else t[:, :g.n]
    return dist[:, :g.n], cut(sigma), cut(delta), st


def sp_graph_set_weights(g: Graph, weights, validate: bool = False, stream=None):
    """Attach int32 edge weights (one per CSR entry; numpy / host or CUDA tensor)."""
    torch = _torch()
    flags = SP_VALIDATE if validate else 0
    if isinstance(weights, torch.Tensor) and weights.is_cuda:
        w = weights.to(torch.int32).contiguous()
        ptr = w.data_ptr()
        flags |= SP_PTR_DEVICE
    else:
        w = np.ascontiguousarray(np.asarray(weights), dtype=np.int32)
        if w.size == 0:
            w = np.zeros(1, np.int32)
        ptr = w.ctypes.data
    if (w.numel() if hasattr(w, "numel") else w.size) < g.nnz:
        raise ValueError("need one weight per CSR entry (%d)" % g.nnz)
    _check(lib().sp_graph_set_weights(g.handle, ptr, flags, _stream(stream)), "sp_graph_set_weights")


def _sssp_config(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, sp_sssp_config):
        return ctypes.byref(cfg)
    c = sp_sssp_config()
    for k, v in cfg.items():
        setattr(c, k, v)
    return ctypes.byref(c)


def sp_sssp(g: Graph, source: int, out_dist=None, config=None, stream=None):
    """int32 distances from `source` (INT32_MAX where unreached), a CUDA tensor [V]."""
    torch = _torch()
    if out_dist is None:
        out_dist = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")
    assert out_dist.is_cuda and out_dist.dtype == torch.int32 and out_dist.is_contiguous()
    assert out_dist.numel() >= g.n
    _check(lib().sp_sssp(g.handle, int(source), out_dist.data_ptr(), _sssp_config(config),
                         _stream(stream)), "sp_sssp")
    return out_dist[:g.n]


def sp_sssp_get_last_stats() -> dict:
    s = sp_sssp_stats()
    _check(lib().sp_sssp_get_last_stats(ctypes.byref(s)), "sp_sssp_get_last_stats")
    return _struct_dict(s)


def sp_pagerank(g: Graph, beta: float = 1e-6, delta: float = 0.85, max_iter: int = 100, out_pr=None,
                config=None, stream=None):
    """float64 PageRank of every vertex, a CUDA tensor [V]."""
    out_pr = _out_f64(g, out_pr)
    cfg = None
    if config is not None:
        c = config if isinstance(config, sp_pagerank_config) else sp_pagerank_config(**config)
        cfg = ctypes.byref(c)
    _check(lib().sp_pagerank(g.handle, float(beta), float(delta), int(max_iter), out_pr.data_ptr(), cfg,
                             _stream(stream)), "sp_pagerank")
    return out_pr[:g.n]


def sp_pagerank_get_last_stats() -> dict:
    s = sp_pagerank_stats()
    _check(lib().sp_pagerank_get_last_stats(ctypes.byref(s)), "sp_pagerank_get_last_stats")
    return _struct_dict(s)


def sp_triangle_count(g: Graph, per_vertex: bool = False, stream=None):
    """(triangle count, per-vertex uint64 CUDA tensor [V] or None)."""
    torch = _torch()
    per = torch.empty(max(g.n, 1), dtype=torch.uint64, device="cuda") if per_vertex else None
    out = ctypes.c_int64()
    _check(lib().sp_triangle_count(g.handle, ctypes.byref(out), per.data_ptr() if per is not None else None,
                                   _stream(stream)), "sp_triangle_count")
    return out.value, (per[:g.n] if per is not None else None)


def sp_tc_get_last_stats() -> dict:
    s = sp_tc_stats()
    _check(lib().sp_tc_get_last_stats(ctypes.byref(s)), "sp_tc_get_last_stats")
    return _struct_dict(s)


def sp_bc_workspace_bytes(g: Graph, batch_width: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().sp_bc_workspace_bytes(g.handle, batch_width, ctypes.byref(b)), "sp_bc_workspace_bytes")
    return b.value


SP_PROFILE_TIMES = 1
SP_PROFILE_COUNTS = 2


def sp_profile_enable(on=True):
    """True: times and counters; False: off; or an int of SP_PROFILE_* bits."""
    what = (SP_PROFILE_TIMES | SP_PROFILE_COUNTS) if on is True else (0 if on is False else int(on))
    _check(lib().sp_profile_enable(what), "sp_profile_enable")


def sp_profile_read() -> dict:
    """{family: dict(launches, total_ms, items, edges, pairs, item_slots)}; resets."""
    buf = (sp_kernel_profile * 32)()
    n = ctypes.c_int32()
    _check(lib().sp_profile_read(buf, 32, ctypes.byref(n)), "sp_profile_read")
    out = {}
    for i in range(n.value):
        d = _struct_dict(buf[i])
        out[d.pop("name").decode()] = d
    return out


def sp_autotune(g: Graph, sources, stream=None) -> dict:
    src, p = _host_i32(sources)
    c = sp_batch_config()
    _check(lib().sp_autotune(g.handle, p, len(src), ctypes.byref(c), _stream(stream)), "sp_autotune")
    return _struct_dict(c)


def sp_autotune_get_last_report() -> dict:
    r = sp_tune_report()
    _check(lib().sp_autotune_get_last_report(ctypes.byref(r)), "sp_autotune_get_last_report")
    out = {k: getattr(r, k) for k, _ in r._fields_ if k not in ("chosen", "cand")}
    out["chosen"] = _struct_dict(r.chosen)
    out["candidates"] = [dict(cfg=_struct_dict(r.cand[i].cfg), ms_per_source=r.cand[i].ms_per_source,
                              accepted=bool(r.cand[i].accepted)) for i in range(r.n_candidates)]
    return out


def sp_graph_fingerprint(g: Graph) -> int:
    v = ctypes.c_uint64()
    _check(lib().sp_graph_fingerprint(g.handle, ctypes.byref(v)), "sp_graph_fingerprint")
    return v.value


def sp_graph_set_tuned(g: Graph, config) -> None:
    """Make `config` (dict or sp_batch_config) the graph's tuned configuration; None clears it."""
    _check(lib().sp_graph_set_tuned(g.handle, _config(config)), "sp_graph_set_tuned")


def sp_tune_cache_clear() -> None:
    _check(lib().sp_tune_cache_clear(), "sp_tune_cache_clear")


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------

class Request:
    """A submitted BC request; `out_bc` is filled when it completes."""

    def __init__(self, handle, out_bc):
        self.handle = handle
        self.out_bc = out_bc

    def wait(self, timeout_us: int = -1) -> int:
        st = ctypes.c_int32()
        rc = lib().sp_request_wait(self.handle, timeout_us, ctypes.byref(st))
        if rc == SP_ERR_TIMEOUT:
            raise TimeoutError("request still running")
        _check(rc, "sp_request_wait")
        return st.value

    def poll(self):
        done = ctypes.c_int32()
        st = ctypes.c_int32()
        _check(lib().sp_request_poll(self.handle, ctypes.byref(done), ctypes.byref(st)), "sp_request_poll")
        return bool(done.value), st.value

    def cancel(self) -> int:
        return lib().sp_request_cancel(self.handle)

    def latency_us(self) -> float:
        v = ctypes.c_double()
        _check(lib().sp_request_latency_us(self.handle, ctypes.byref(v)), "sp_request_latency_us")
        return v.value

    def release(self):
        if self.handle:
            _check(lib().sp_request_release(self.handle), "sp_request_release")
            self.handle = None


class Server:
    """Continuous-batching BC server over resident graphs (sp_server_*)."""

    def __init__(self, memory_budget: int = 0, max_batch: int = 0, n_streams: int = 0):
        c = sp_server_config()
        c.memory_budget = memory_budget
        c.max_batch = max_batch
        c.n_streams = n_streams
        h = ctypes.c_void_p()
        _check(lib().sp_server_create(ctypes.byref(c), ctypes.byref(h)), "sp_server_create")
        self.handle = h
        self.graphs = {}

    def add_graph(self, g: Graph) -> int:
        gid = ctypes.c_int32()
        _check(lib().sp_server_add_graph(self.handle, g.handle, ctypes.byref(gid)), "sp_server_add_graph")
        self.graphs[gid.value] = g
        return gid.value

    def submit(self, graph_id: int, sources, out_bc=None) -> Request:
        torch = _torch()
        g = self.graphs.get(graph_id)
        if out_bc is None:
            n = g.n if g is not None else 1
            out_bc = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
        src, p = _host_i32(sources)
        h = ctypes.c_void_p()
        _check(lib().sp_stream_submit(self.handle, graph_id, p, len(src), out_bc.data_ptr(),
                                      ctypes.byref(h)), "sp_stream_submit")
        return Request(h, out_bc)

    def stats(self) -> dict:
        s = sp_server_stats()
        _check(lib().sp_server_get_stats(self.handle, ctypes.byref(s)), "sp_server_get_stats")
        return _struct_dict(s)

    def destroy(self):
        if self.handle:
            _check(lib().sp_server_destroy(self.handle), "sp_server_destroy")
            self.handle = None


def sp_server_create(memory_budget: int = 0, max_batch: int = 0, n_streams: int = 0) -> Server:
    return Server(memory_budget, max_batch, n_streams)


def sp_stream_submit(server: Server, graph_id: int, sources, out_bc=None) -> Request:
    return server.submit(graph_id, sources, out_bc)
