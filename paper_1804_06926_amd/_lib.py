"""ctypes binding of libtc_mi355x.so. Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(HERE, "libtc_mi355x.so")

SELECT_HEURISTIC, SELECT_LEARNED, FORCE_MERGE, FORCE_BSEARCH, FORCE_BITMAP = 0, 1, 2, 3, 4
F_STAGE_TIMING = 0x1

_STATUS = {0: "ok", 1: "invalid argument", 2: "vertex id out of range", 3: "workspace too small",
           4: "HIP runtime error", 5: "unsupported size"}

_lib = None
_lock = threading.Lock()
_ctxs = {}          # (device, stream handle) -> tc_ctx*
_workspaces = {}    # device -> uint8 tensor


class TCError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        msg = _STATUS.get(status, f"status {status}")
        super().__init__(f"{msg}: {detail}" if detail else msg)


class Options(ctypes.Structure):
    _fields_ = [("select", ctypes.c_int32), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32 * 6)]


def library_path() -> str:
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        raise RuntimeError(f"HIP library not built ({_SO}); run __graft_entry__.build()")
    lib = ctypes.CDLL(_SO)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sz = ctypes.c_size_t
    lib.tc_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp]
    lib.tc_destroy.argtypes = [vp]
    lib.tc_workspace_size.argtypes = [i64, i32, ctypes.POINTER(Options), ctypes.POINTER(sz)]
    lib.tc_count_triangles.argtypes = [vp, vp, i64, i32, vp, sz, ctypes.POINTER(Options),
                                       ctypes.POINTER(ctypes.c_uint64), vp]
    lib.tc_count_triangles_async.argtypes = [vp, vp, i64, i32, vp, sz, ctypes.POINTER(Options), vp, vp]
    lib.tc_formulation_workspace_size.argtypes = [i64, i32, ctypes.POINTER(Options), i32, ctypes.POINTER(sz)]
    lib.tc_count_triangles_formulation.argtypes = [vp, vp, i64, i32, vp, sz, ctypes.POINTER(Options), i32, vp, vp]
    lib.tc_list_workspace_size.argtypes = [i64, i32, ctypes.POINTER(Options), ctypes.POINTER(sz)]
    lib.tc_list_triangles.argtypes = [vp, vp, i64, i32, vp, sz, ctypes.POINTER(Options), vp, i64,
                                      ctypes.POINTER(ctypes.c_uint64)]
    lib.tc_edge_support.argtypes = [vp, vp, i64, i32, vp, sz, ctypes.POINTER(Options), vp, vp,
                                    ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_uint64)]
    lib.tc_clustering.argtypes = [vp, vp, i64, i32, vp, sz, ctypes.POINTER(Options), vp, vp,
                                  ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                  ctypes.POINTER(ctypes.c_double)]
    lib.tc_edge_counts.argtypes = [vp, vp, i64, i32, vp, sz, ctypes.POINTER(Options), vp, vp,
                                   ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_uint64)]
    lib.tc_build_csr.argtypes = [vp, vp, i64, i32, vp, sz, ctypes.POINTER(Options), vp, vp, vp,
                                 ctypes.POINTER(i64)]
    lib.tc_radix_sort_workspace_size.argtypes = [i64]
    lib.tc_radix_sort_workspace_size.restype = sz
    lib.tc_radix_sort_u64.argtypes = [vp, vp, vp, i64, i32, i32, vp, sz]
    lib.tc_radix_partition_u64.argtypes = [vp, vp, vp, i64, i32, i32, vp, sz]
    lib.tc_sort_runs_u64.argtypes = [vp, vp, vp, i64, i32]
    lib.tc_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32]
    lib.tc_stage_times.restype = i32
    lib.tc_stage_name.argtypes = [i32]
    lib.tc_stage_name.restype = ctypes.c_char_p
    lib.tc_last_error.argtypes = [vp]
    lib.tc_last_error.restype = ctypes.c_char_p
    for f in ("tc_create", "tc_destroy", "tc_workspace_size", "tc_count_triangles", "tc_count_triangles_async",
              "tc_clustering", "tc_edge_support", "tc_list_workspace_size", "tc_list_triangles",
              "tc_edge_counts",
              "tc_build_csr", "tc_radix_sort_u64", "tc_radix_partition_u64", "tc_sort_runs_u64"):
        getattr(lib, f).restype = ctypes.c_int
    _ = u32
    _lib = lib
    return lib


def _torch():
    import torch
    return torch


def _ctx(device):
    torch = _torch()
    dev = torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    stream = torch.cuda.current_stream(idx).cuda_stream
    key = (idx, stream)
    with _lock:
        h = _ctxs.get(key)
        if h is None:
            lib = _load()
            p = ctypes.c_void_p()
            st = lib.tc_create(ctypes.byref(p), idx, ctypes.c_void_p(stream))
            if st != 0:
                raise TCError(st, "tc_create")
            h = p
            _ctxs[key] = h
    return h, idx


def _check(st: int, ctx) -> None:
    if st != 0:
        detail = _load().tc_last_error(ctx).decode() if ctx else ""
        raise TCError(st, detail)


def _options(select: int, timing: bool) -> Options:
    o = Options()
    o.select = select
    o.flags = F_STAGE_TIMING if timing else 0
    return o


def workspace_size(num_edges: int, num_vertices: int, select: int = SELECT_HEURISTIC) -> int:
    out = ctypes.c_size_t()
    o = _options(select, False)
    st = _load().tc_workspace_size(num_edges, num_vertices, ctypes.byref(o), ctypes.byref(out))
    _check(st, None)
    return int(out.value)


def _workspace(idx: int, nbytes: int, workspace=None):
    torch = _torch()
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise TCError(3, "given workspace too small")
        return workspace
    ws = _workspaces.get(idx)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=f"cuda:{idx}")
        _workspaces[idx] = ws
    return ws


def _edges_arg(edges):
    torch = _torch()
    if not (isinstance(edges, torch.Tensor) and edges.is_cuda):
        raise TypeError("edges must be a CUDA (HIP) torch tensor")
    if edges.dtype != torch.int32 or edges.dim() != 2 or edges.shape[1] != 2 or not edges.is_contiguous():
        raise TypeError("edges must be a contiguous int32 tensor of shape [E, 2]")
    return edges


def _timings(ctx):
    lib = _load()
    buf = (ctypes.c_float * 32)()
    k = lib.tc_stage_times(ctx, buf, 32)
    return {lib.tc_stage_name(i).decode(): float(buf[i]) for i in range(k)}


def stage_names():
    lib = _load()
    out, i = [], 0
    while True:
        s = lib.tc_stage_name(i).decode()
        if not s:
            return out
        out.append(s)
        i += 1


def count_triangles(edges, num_vertices: int, per_vertex: bool = False, select: int = SELECT_HEURISTIC,
                    workspace=None, timing: bool = False):
    """Exact triangle count of the graph denoted by ``edges`` (int32 [E, 2] on the GPU).

    Returns T (int), or (T, t) with per_vertex, t a uint64 tensor [num_vertices]
    on the same device (int64 holding the uint64 t[v] = triangles containing v). With timing, a dict of
    per-stage device milliseconds is appended to the result.
    """
    torch = _torch()
    e = _edges_arg(edges)
    ctx, idx = _ctx(e.device)
    E = e.shape[0]
    o = _options(select, timing)
    nbytes = workspace_size(E, num_vertices, select)
    ws = _workspace(idx, nbytes, workspace)
    # t[v] < 2^63, so the uint64 results are held in an int64 tensor
    pv = torch.empty(num_vertices, dtype=torch.int64, device=e.device) if per_vertex else None
    count = ctypes.c_uint64()
    st = _load().tc_count_triangles(ctx, e.data_ptr() if E else None, E, num_vertices, ws.data_ptr(),
                                    ws.numel(), ctypes.byref(o), ctypes.byref(count),
                                    pv.data_ptr() if pv is not None and num_vertices else None)
    _check(st, ctx)
    res = [int(count.value)]
    if per_vertex:
        res.append(pv)
    if timing:
        res.append(_timings(ctx))
    return res[0] if len(res) == 1 else tuple(res)


FORMULATIONS = {"filtered": 0, "full": 1, "matrix": 2, "matrix_upper": 3}


def count_triangles_formulation(edges, num_vertices: int, formulation: str = "full",
                                select: int = SELECT_HEURISTIC, workspace=None, timing: bool = False):
    """T by one of the paper's formulations, with the sum of hits it divides.

    formulation: "filtered" (N+(u) against N+(v), sum T), "full" (whole
    neighbour lists over the half-filtered edges, sum 3T), "matrix"
    (Algorithm 3, C = A o (L U), sum of C = 2T) or "matrix_upper" (the
    matrix form with the mask cut to the upper triangle, sum T).
    Returns (T, sum), plus a dict of per-stage milliseconds with timing.
    """
    if formulation not in FORMULATIONS:
        raise ValueError(f"unknown formulation {formulation!r}")
    f = FORMULATIONS[formulation]
    e = _edges_arg(edges)
    ctx, idx = _ctx(e.device)
    E = e.shape[0]
    o = _options(select, timing)
    lib = _load()
    nb = ctypes.c_size_t()
    _check(lib.tc_formulation_workspace_size(E, num_vertices, ctypes.byref(o), f, ctypes.byref(nb)), None)
    ws = _workspace(idx, nb.value, workspace)
    count, total = ctypes.c_uint64(), ctypes.c_uint64()
    st = lib.tc_count_triangles_formulation(ctx, e.data_ptr() if E else None, E, num_vertices, ws.data_ptr(),
                                            ws.numel(), ctypes.byref(o), f, ctypes.byref(count), ctypes.byref(total))
    _check(st, ctx)
    if timing:
        return int(count.value), int(total.value), _timings(ctx)
    return int(count.value), int(total.value)


def count_triangles_async(edges, num_vertices: int, result=None, per_vertex=None, select: int = SELECT_HEURISTIC,
                          workspace=None):
    """Queue a count on torch's current stream without waiting for it.

    Returns ``result``, an int64 tensor [2] on the device (allocated when not
    given): after the stream reaches the call, result[0] = T and result[1] = 0,
    or the status code of an out-of-range vertex id. ``per_vertex`` (optional,
    int64 [num_vertices] on the device) receives t[v]. The workspace must not
    be reused by other streams until the call has finished.
    """
    torch = _torch()
    e = _edges_arg(edges)
    ctx, idx = _ctx(e.device)
    E = e.shape[0]
    o = _options(select, False)
    ws = _workspace(idx, workspace_size(E, num_vertices, select), workspace)
    if result is None:
        result = torch.empty(2, dtype=torch.int64, device=e.device)
    if per_vertex is not None and (per_vertex.dtype != torch.int64 or per_vertex.numel() < num_vertices):
        raise TypeError("per_vertex must be an int64 tensor with num_vertices entries")
    st = _load().tc_count_triangles_async(ctx, e.data_ptr() if E else None, E, num_vertices, ws.data_ptr(),
                                          ws.numel(), ctypes.byref(o), result.data_ptr(),
                                          per_vertex.data_ptr() if per_vertex is not None and num_vertices
                                          else None)
    _check(st, ctx)
    return result


NOALLOC_SCRATCH_BYTES = 64 << 20   # TC_NOALLOC_SCRATCH_BYTES


def count_triangles_noalloc(edges, num_vertices: int, result, per_vertex=None, select: int = SELECT_HEURISTIC):
    """count_triangles_async on the library's fixed per-GPU scratch: neither this call
    nor the library allocates device memory (the context must exist already: create it
    with any earlier call on this stream). ``result`` (int64 [2] on the device) is the
    caller's; graphs whose workspace exceeds NOALLOC_SCRATCH_BYTES raise TCError
    (status 3) before anything is queued."""
    torch = _torch()
    e = _edges_arg(edges)
    ctx, _ = _ctx(e.device)
    E = e.shape[0]
    o = _options(select, False)
    if result is None or result.dtype != torch.int64 or result.numel() < 2 or not result.is_cuda:
        raise TypeError("result must be an int64 device tensor with 2 entries")
    if per_vertex is not None and (per_vertex.dtype != torch.int64 or per_vertex.numel() < num_vertices):
        raise TypeError("per_vertex must be an int64 tensor with num_vertices entries")
    lib = _load()
    vp = ctypes.c_void_p
    lib.tc_count_triangles_noalloc.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(Options), vp,
                                               vp]
    lib.tc_count_triangles_noalloc.restype = ctypes.c_int
    st = lib.tc_count_triangles_noalloc(ctx, e.data_ptr() if E else None, E, num_vertices, ctypes.byref(o),
                                        result.data_ptr(),
                                        per_vertex.data_ptr() if per_vertex is not None and num_vertices else None)
    _check(st, ctx)
    return result


def clustering(edges, num_vertices: int, per_vertex: bool = False, select: int = SELECT_HEURISTIC, workspace=None):
    """Local clustering coefficients and transitivity.

    Returns (coeff float64 [num_vertices] on the device, T, wedges, transitivity),
    with t (int64 [num_vertices], the uint64 per-vertex counts) appended when
    per_vertex is set.
    """
    torch = _torch()
    e = _edges_arg(edges)
    ctx, idx = _ctx(e.device)
    E = e.shape[0]
    o = _options(select, False)
    ws = _workspace(idx, workspace_size(E, num_vertices, select), workspace)
    coeff = torch.empty(max(num_vertices, 1), dtype=torch.float64, device=e.device)[:num_vertices]
    pv = torch.empty(num_vertices, dtype=torch.int64, device=e.device) if per_vertex else None
    T, W, tr = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_double()
    st = _load().tc_clustering(ctx, e.data_ptr() if E else None, E, num_vertices, ws.data_ptr(), ws.numel(),
                               ctypes.byref(o), coeff.data_ptr() if num_vertices else None,
                               pv.data_ptr() if pv is not None and num_vertices else None, ctypes.byref(T),
                               ctypes.byref(W), ctypes.byref(tr))
    _check(st, ctx)
    res = (coeff, int(T.value), int(W.value), float(tr.value))
    return res + (pv,) if per_vertex else res


def list_triangles(edges, num_vertices: int, select: int = SELECT_HEURISTIC, workspace=None):
    """All triangles as an int32 tensor [T, 3] of original ids (u, v, w), u before v before w in
    (degree, id) order; grouped by the edge (u, v) in CSR order, unordered inside a group."""
    torch = _torch()
    e = _edges_arg(edges)
    ctx, idx = _ctx(e.device)
    E = e.shape[0]
    o = _options(select, False)
    nbytes = ctypes.c_size_t()
    _check(_load().tc_list_workspace_size(E, num_vertices, ctypes.byref(o), ctypes.byref(nbytes)), None)
    ws = _workspace(idx, int(nbytes.value), workspace)
    T = ctypes.c_uint64()
    cap = 0
    out = None
    for _ in range(2):   # the first call reports T when the capacity is short
        out = torch.empty((max(cap, 1), 3), dtype=torch.int32, device=e.device)
        st = _load().tc_list_triangles(ctx, e.data_ptr() if E else None, E, num_vertices, ws.data_ptr(), ws.numel(),
                                       ctypes.byref(o), out.data_ptr(), cap, ctypes.byref(T))
        if st == 3 and T.value > cap:
            cap = int(T.value)
            continue
        _check(st, ctx)
        break
    return out[: int(T.value)]


def edge_support(edges, num_vertices: int, select: int = SELECT_HEURISTIC, workspace=None):
    """Triangles containing each kept edge: (pairs int32 [m, 2] original ids, support uint32 [m] held
    in int32, T)."""
    torch = _torch()
    e = _edges_arg(edges)
    ctx, idx = _ctx(e.device)
    E = e.shape[0]
    o = _options(select, False)
    ws = _workspace(idx, workspace_size(E, num_vertices, select), workspace)
    pairs = torch.empty((max(E, 1), 2), dtype=torch.int32, device=e.device)
    sup = torch.empty(max(E, 1), dtype=torch.int32, device=e.device)
    m = ctypes.c_int64()
    T = ctypes.c_uint64()
    st = _load().tc_edge_support(ctx, e.data_ptr() if E else None, E, num_vertices, ws.data_ptr(), ws.numel(),
                                 ctypes.byref(o), pairs.data_ptr(), sup.data_ptr(), ctypes.byref(m),
                                 ctypes.byref(T))
    _check(st, ctx)
    k = int(m.value)
    return pairs[:k], sup[:k], int(T.value)


def edge_counts(edges, num_vertices: int, select: int = SELECT_HEURISTIC, workspace=None):
    """Per-edge intersection sizes: (pairs int32 [m, 2] original ids (u before v), counts uint32 [m], T)."""
    torch = _torch()
    e = _edges_arg(edges)
    ctx, idx = _ctx(e.device)
    E = e.shape[0]
    o = _options(select, False)
    ws = _workspace(idx, workspace_size(E, num_vertices, select), workspace)
    pairs = torch.empty((max(E, 1), 2), dtype=torch.int32, device=e.device)
    counts = torch.empty(max(E, 1), dtype=torch.int32, device=e.device)   # uint32 counts < 2^31
    m = ctypes.c_int64()
    T = ctypes.c_uint64()
    st = _load().tc_edge_counts(ctx, e.data_ptr() if E else None, E, num_vertices, ws.data_ptr(), ws.numel(),
                                ctypes.byref(o), pairs.data_ptr(), counts.data_ptr(), ctypes.byref(m),
                                ctypes.byref(T))
    _check(st, ctx)
    k = int(m.value)
    return pairs[:k], counts[:k], int(T.value)


def build_csr(edges, num_vertices: int, workspace=None):
    """The degree-ordered CSR: (rank int32 [n], offsets int64 [n+1], col int32 [m])."""
    torch = _torch()
    e = _edges_arg(edges)
    ctx, idx = _ctx(e.device)
    E = e.shape[0]
    o = _options(SELECT_HEURISTIC, False)
    ws = _workspace(idx, workspace_size(E, num_vertices), workspace)
    rank = torch.empty(max(num_vertices, 1), dtype=torch.int32, device=e.device)
    off = torch.empty(num_vertices + 1, dtype=torch.int64, device=e.device)
    col = torch.empty(max(E, 1), dtype=torch.int32, device=e.device)
    m = ctypes.c_int64()
    st = _load().tc_build_csr(ctx, e.data_ptr() if E else None, E, num_vertices, ws.data_ptr(), ws.numel(),
                              ctypes.byref(o), rank.data_ptr(), off.data_ptr(), col.data_ptr(), ctypes.byref(m))
    _check(st, ctx)
    return rank[:num_vertices], off, col[:int(m.value)]


def radix_sort_u64(keys, bit_lo: int = 0, bit_hi: int = 64):
    """Sort a uint64 (or int64 bit-pattern) CUDA tensor in place on bits [bit_lo, bit_hi)."""
    torch = _torch()
    if not (isinstance(keys, torch.Tensor) and keys.is_cuda and keys.element_size() == 8 and keys.is_contiguous()):
        raise TypeError("keys must be a contiguous 64-bit CUDA tensor")
    ctx, idx = _ctx(keys.device)
    n = keys.numel()
    lib = _load()
    nbytes = int(lib.tc_radix_sort_workspace_size(n))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=keys.device)
    alt = torch.empty_like(keys)
    st = lib.tc_radix_sort_u64(ctx, keys.data_ptr(), alt.data_ptr(), n, bit_lo, bit_hi, ws.data_ptr(), nbytes)
    _check(st, ctx)
    return keys


def radix_partition_u64(keys, shift: int, bits: int):
    """One partitioning radix pass of a 64-bit CUDA tensor: a new tensor holding the keys grouped
    by digit (key >> shift) & (2**bits - 1), digits ascending, order inside a digit arbitrary."""
    torch = _torch()
    if not (isinstance(keys, torch.Tensor) and keys.is_cuda and keys.element_size() == 8 and keys.is_contiguous()):
        raise TypeError("keys must be a contiguous 64-bit CUDA tensor")
    ctx, idx = _ctx(keys.device)
    n = keys.numel()
    lib = _load()
    nbytes = int(lib.tc_radix_sort_workspace_size(n))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=keys.device)
    out = torch.empty_like(keys)
    st = lib.tc_radix_partition_u64(ctx, keys.data_ptr(), out.data_ptr(), n, shift, bits, ws.data_ptr(), nbytes)
    _check(st, ctx)
    return out


def sort_runs_u64(keys, shift: int):
    """Sort, in place, each run of equal keys >> shift of a 64-bit CUDA tensor by the whole key
    (the keys grouped by their high bits beforehand give a sorted tensor)."""
    torch = _torch()
    if not (isinstance(keys, torch.Tensor) and keys.is_cuda and keys.element_size() == 8 and keys.is_contiguous()):
        raise TypeError("keys must be a contiguous 64-bit CUDA tensor")
    ctx, idx = _ctx(keys.device)
    tmp = torch.empty_like(keys)
    st = _load().tc_sort_runs_u64(ctx, keys.data_ptr(), tmp.data_ptr(), keys.numel(), shift)
    _check(st, ctx)
    return keys


class Stats(ctypes.Structure):
    _fields_ = [("num_edges_kept", ctypes.c_uint64), ("num_pairs_valid", ctypes.c_uint64),
                ("num_tiles", ctypes.c_uint32), ("tile_begin", ctypes.c_uint32 * 4),
                ("bucket_vertices", ctypes.c_uint32 * 256), ("bucket_in_edges", ctypes.c_uint64 * 256),
                ("bucket_out_edges", ctypes.c_uint64 * 256), ("bucket_work", ctypes.c_uint64 * 256),
                ("bucket_kernel", ctypes.c_uint8 * 256), ("bucket_chunk", ctypes.c_uint16 * 256),
                ("bucket_group", ctypes.c_uint8 * 256)]


def last_stats(device="cuda:0") -> dict:
    """Work statistics of the last counting call on the current stream's context."""
    import numpy as np
    ctx, _ = _ctx(device)
    s = Stats()
    lib = _load()
    lib.tc_last_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(Stats)]
    lib.tc_last_stats.restype = ctypes.c_int
    _check(lib.tc_last_stats(ctx, ctypes.byref(s)), ctx)
    out = {"m": int(s.num_edges_kept), "m_valid": int(s.num_pairs_valid), "num_tiles": int(s.num_tiles),
           "tile_begin": list(s.tile_begin)}
    for f in ("bucket_vertices", "bucket_in_edges", "bucket_out_edges", "bucket_work", "bucket_kernel",
              "bucket_chunk", "bucket_group"):
        out[f] = np.ctypeslib.as_array(getattr(s, f)).copy()
    return out


# ---------------------------------------------------------------- selector network
SELECTOR_NUM_PARAMS = 1379
SELECTOR_NUM_FEATURES = 6


def _sel_lib():
    lib = _load()
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    fp = ctypes.POINTER(ctypes.c_float)
    lib.tc_bucket_features.argtypes = [vp, fp]
    lib.tc_profile_buckets.argtypes = [vp, vp, i64, i32, vp, ctypes.c_size_t, i32, fp, fp]
    lib.tc_selector_set_params.argtypes = [vp, fp]
    lib.tc_selector_get_params.argtypes = [vp, fp]
    lib.tc_selector_forward.argtypes = [vp, vp, i32, vp]
    lib.tc_selector_gradient.argtypes = [vp, vp, vp, vp, i32, vp, fp]
    lib.tc_selector_train_step.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, fp]
    lib.tc_selector_set_tile_params.argtypes = [vp, fp]
    lib.tc_selector_get_tile_params.argtypes = [vp, fp]
    lib.tc_selector_load.argtypes = [vp, ctypes.c_char_p]
    lib.tc_selector_save.argtypes = [vp, ctypes.c_char_p]
    for f in ("tc_bucket_features", "tc_profile_buckets", "tc_selector_set_params", "tc_selector_get_params",
              "tc_selector_forward", "tc_selector_gradient", "tc_selector_train_step",
              "tc_selector_set_tile_params", "tc_selector_get_tile_params", "tc_selector_load",
              "tc_selector_save"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def selector_set_params(params, device="cuda:0") -> None:
    """Load float32 master parameters of the selector network on the device's context."""
    import numpy as np
    p = np.ascontiguousarray(params, dtype=np.float32).ravel()
    if p.size != SELECTOR_NUM_PARAMS:
        raise ValueError(f"expected {SELECTOR_NUM_PARAMS} parameters")
    ctx, _ = _ctx(device)
    _check(_sel_lib().tc_selector_set_params(ctx, _fptr(p)), ctx)


def selector_load(path, device="cuda:0") -> None:
    """Install both networks from a selector parameter file (the library's own JSON reader)."""
    ctx, _ = _ctx(device)
    _check(_sel_lib().tc_selector_load(ctx, os.fsencode(path)), ctx)


def selector_save(path, device="cuda:0") -> None:
    """Write the context's selector parameters to a file in the same format."""
    ctx, _ = _ctx(device)
    _check(_sel_lib().tc_selector_save(ctx, os.fsencode(path)), ctx)


def selector_get_params(device="cuda:0"):
    import numpy as np
    p = np.empty(SELECTOR_NUM_PARAMS, dtype=np.float32)
    ctx, _ = _ctx(device)
    _check(_sel_lib().tc_selector_get_params(ctx, _fptr(p)), ctx)
    return p


def selector_set_tile_params(params, device="cuda:0") -> None:
    """Load the tile network's float32 parameters (None removes the network)."""
    import numpy as np
    ctx, _ = _ctx(device)
    if params is None:
        _check(_sel_lib().tc_selector_set_tile_params(ctx, None), ctx)
        return
    p = np.ascontiguousarray(params, dtype=np.float32).ravel()
    if p.size != SELECTOR_NUM_PARAMS:
        raise ValueError(f"expected {SELECTOR_NUM_PARAMS} parameters")
    _check(_sel_lib().tc_selector_set_tile_params(ctx, _fptr(p)), ctx)


def selector_get_tile_params(device="cuda:0"):
    import numpy as np
    p = np.empty(SELECTOR_NUM_PARAMS, dtype=np.float32)
    ctx, _ = _ctx(device)
    _check(_sel_lib().tc_selector_get_tile_params(ctx, _fptr(p)), ctx)
    return p


def _dev_f32(x, cols):
    torch = _torch()
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
            and x.dim() == 2 and x.shape[1] == cols):
        raise TypeError(f"expected a contiguous float32 CUDA tensor [B, {cols}]")
    return x


def selector_forward(x):
    """Logits [B, 3] (float32 CUDA) of features x [B, 6] (float32 CUDA)."""
    torch = _torch()
    x = _dev_f32(x, SELECTOR_NUM_FEATURES)
    ctx, _ = _ctx(x.device)
    out = torch.empty((x.shape[0], 3), dtype=torch.float32, device=x.device)
    _check(_sel_lib().tc_selector_forward(ctx, x.data_ptr(), x.shape[0], out.data_ptr()), ctx)
    return out


def _labels_weights(x, y, w):
    torch = _torch()
    if not (isinstance(y, torch.Tensor) and y.is_cuda and y.dtype == torch.int32 and y.numel() == x.shape[0]):
        raise TypeError("labels must be an int32 CUDA tensor [B]")
    if w is not None and not (isinstance(w, torch.Tensor) and w.is_cuda and w.dtype == torch.float32
                              and w.numel() == x.shape[0]):
        raise TypeError("weights must be a float32 CUDA tensor [B]")
    return y.contiguous(), (w.contiguous() if w is not None else None)


def selector_gradient(x, y, w=None):
    """(gradient float32 [1379] CUDA, loss) of the weighted cross-entropy."""
    torch = _torch()
    x = _dev_f32(x, SELECTOR_NUM_FEATURES)
    y, w = _labels_weights(x, y, w)
    ctx, _ = _ctx(x.device)
    g = torch.empty(SELECTOR_NUM_PARAMS, dtype=torch.float32, device=x.device)
    loss = ctypes.c_float()
    _check(_sel_lib().tc_selector_gradient(ctx, x.data_ptr(), y.data_ptr(), w.data_ptr() if w is not None else None,
                                           x.shape[0], g.data_ptr(), ctypes.byref(loss)), ctx)
    return g, float(loss.value)


def selector_train_step(x, y, w=None, lr=1e-3) -> float:
    x = _dev_f32(x, SELECTOR_NUM_FEATURES)
    y, w = _labels_weights(x, y, w)
    ctx, _ = _ctx(x.device)
    loss = ctypes.c_float()
    _check(_sel_lib().tc_selector_train_step(ctx, x.data_ptr(), y.data_ptr(),
                                             w.data_ptr() if w is not None else None, x.shape[0], lr,
                                             ctypes.byref(loss)), ctx)
    return float(loss.value)


def bucket_features(device="cuda:0"):
    """Features [256, 6] of the buckets of the last counting call."""
    import numpy as np
    out = np.zeros((256, SELECTOR_NUM_FEATURES), dtype=np.float32)
    ctx, _ = _ctx(device)
    _check(_sel_lib().tc_bucket_features(ctx, _fptr(out)), ctx)
    return out


def profile_buckets(edges, num_vertices: int, repeats: int = 5, workspace=None):
    """Per-(strategy, bucket) median milliseconds [3, 256] (-1 = empty) and features [256, 6]."""
    import numpy as np
    e = _edges_arg(edges)
    ctx, idx = _ctx(e.device)
    E = e.shape[0]
    ws = _workspace(idx, workspace_size(E, num_vertices), workspace)
    ms = np.zeros((3, 256), dtype=np.float32)
    feat = np.zeros((256, SELECTOR_NUM_FEATURES), dtype=np.float32)
    _check(_sel_lib().tc_profile_buckets(ctx, e.data_ptr() if E else None, E, num_vertices, ws.data_ptr(),
                                         ws.numel(), repeats, _fptr(ms), _fptr(feat)), ctx)
    return ms, feat


def profile_choices(edges, num_vertices: int, choice, chunk=None, repeats: int = 5, workspace=None):
    """The intersection stage as a counting call launches it, with the given strategy per
    bucket (choice uint8 [256]: 0 merge, 1 binary search, 2 bitmap, other = the fixed
    thresholds' choice) and optional in-edges per tile (chunk uint16 [256], 0 = default).
    Returns (median ms of the stage, median ms per kernel [3], T)."""
    import numpy as np
    e = _edges_arg(edges)
    ctx, idx = _ctx(e.device)
    E = e.shape[0]
    ws = _workspace(idx, workspace_size(E, num_vertices), workspace)
    ch = np.ascontiguousarray(choice, dtype=np.uint8)
    if ch.shape != (256,):
        raise ValueError("choice must have 256 entries")
    ck = None if chunk is None else np.ascontiguousarray(chunk, dtype=np.uint16)
    if ck is not None and ck.shape != (256,):
        raise ValueError("chunk must have 256 entries")
    ms = np.zeros(4, dtype=np.float32)
    T = ctypes.c_uint64(0)
    lib = _load()
    vp = ctypes.c_void_p
    lib.tc_profile_choices.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, vp, ctypes.c_size_t, vp, vp,
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_uint64)]
    lib.tc_profile_choices.restype = ctypes.c_int
    _check(lib.tc_profile_choices(ctx, e.data_ptr() if E else None, E, num_vertices, ws.data_ptr(), ws.numel(),
                                  ch.ctypes.data, ck.ctypes.data if ck is not None else None, repeats, _fptr(ms),
                                  ctypes.byref(T)), ctx)
    return float(ms[0]), ms[1:].astype(float), int(T.value)


# ---------------------------------------------------------------- batched counting, tile shapes
F_NO_GRAPH = 0x2


def _batch_lib():
    lib = _load()
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.tc_batch_workspace_size.argtypes = [i64, i64, i32, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)]
    lib.tc_count_triangles_batch.argtypes = [vp, vp, vp, vp, i32, vp, ctypes.c_size_t, ctypes.POINTER(Options), vp]
    lib.tc_set_tile_shapes.argtypes = [vp, vp, vp]
    lib.tc_profile_selected.argtypes = [vp, vp, i64, i32, vp, ctypes.c_size_t, ctypes.POINTER(Options), i32,
                                        ctypes.POINTER(ctypes.c_float)]
    for f in ("tc_batch_workspace_size", "tc_count_triangles_batch", "tc_set_tile_shapes", "tc_profile_selected"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


_batch_ws = {}


def count_triangles_batch(edges, edge_offsets, num_vertices, select: int = SELECT_HEURISTIC, graph: bool = True,
                          workspace=None):
    """Exact triangle count of each graph of a batch (one pass over their disjoint union).

    edges: int32 CUDA tensor [E, 2], graph g's pairs in rows
    edge_offsets[g] .. edge_offsets[g+1] with ids local to the graph.
    edge_offsets: int64 [G+1] host array; num_vertices: int32 [G] host array.
    With graph=True the device work is captured once and replayed.
    Returns a uint64 numpy array [G].
    """
    import numpy as np
    torch = _torch()
    e = _edges_arg(edges)
    ctx, idx = _ctx(e.device)
    eo = np.ascontiguousarray(edge_offsets, dtype=np.int64)
    nv = np.ascontiguousarray(num_vertices, dtype=np.int32)
    G = nv.size
    if eo.size != G + 1:
        raise ValueError("edge_offsets must have num_graphs + 1 entries")
    lib = _batch_lib()
    o = _options(select, False)
    o.flags = 0 if graph else F_NO_GRAPH
    nbytes = ctypes.c_size_t()
    _check(lib.tc_batch_workspace_size(int(eo[-1]), int(nv.astype(np.int64).sum()), G, ctypes.byref(o),
                                       ctypes.byref(nbytes)), None)
    if workspace is None:
        ws = _batch_ws.get(idx)
        if ws is None or ws.numel() < nbytes.value:
            ws = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=e.device)
            _batch_ws[idx] = ws
    else:
        ws = workspace
    counts = np.zeros(G, dtype=np.uint64)
    _check(lib.tc_count_triangles_batch(ctx, e.data_ptr() if e.shape[0] else None, eo.ctypes.data, nv.ctypes.data, G,
                                        ws.data_ptr(), ws.numel(), ctypes.byref(o), counts.ctypes.data), ctx)
    return counts


def set_tile_shapes(chunk=None, group=None, device="cuda:0") -> None:
    """Per-bucket tile shapes: chunk[256] in-edges per tile, group[256] lanes per in-edge (0 = default)."""
    import numpy as np
    ctx, _ = _ctx(device)
    c = None if chunk is None else np.ascontiguousarray(chunk, dtype=np.uint16)
    g = None if group is None else np.ascontiguousarray(group, dtype=np.uint8)
    _check(_batch_lib().tc_set_tile_shapes(ctx, c.ctypes.data if c is not None else None,
                                           g.ctypes.data if g is not None else None), ctx)


def profile_selected(edges, num_vertices: int, select: int = SELECT_HEURISTIC, repeats: int = 3, workspace=None):
    """Per-bucket median milliseconds [256] with the strategy the mode selects (-1 = empty)."""
    import numpy as np
    e = _edges_arg(edges)
    ctx, idx = _ctx(e.device)
    E = e.shape[0]
    ws = _workspace(idx, workspace_size(E, num_vertices), workspace)
    ms = np.zeros(256, dtype=np.float32)
    o = _options(select, False)
    _check(_batch_lib().tc_profile_selected(ctx, e.data_ptr() if E else None, E, num_vertices, ws.data_ptr(),
                                            ws.numel(), ctypes.byref(o), repeats, _fptr(ms)), ctx)
    return ms
