"""Python binding of libmcm.so: argument marshalling only.

Every step of the matching runs in the library's gfx950 kernels; torch is
used for device memory and streams.  Names follow include/mcm.h.  If the
library is missing this module raises on import of the library (no CPU
fallback exists).
"""
from __future__ import annotations

import atexit
import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcm.so")

MCM_OK = 0
MCM_EINVAL = -1
MCM_ENOMEM = -2
MCM_EHIP = -3
MCM_EBADINIT = -4
MCM_EINTERNAL = -5
MCM_ENOTMAX = -6


class McmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mcm error {code}: {msg}")
        self.code = code


class mcm_graph(ctypes.Structure):
    _fields_ = [("ncols", ctypes.c_int32), ("nrows", ctypes.c_int32), ("colptr_off", ctypes.c_int64),
                ("rowind_off", ctypes.c_int64), ("col_off", ctypes.c_int64), ("row_off", ctypes.c_int64)]


class mcm_request_info(ctypes.Structure):
    _fields_ = [("card", ctypes.c_int64), ("submit_ms", ctypes.c_double), ("admit_ms", ctypes.c_double),
                ("start_ms", ctypes.c_double), ("done_ms", ctypes.c_double), ("path", ctypes.c_int32),
                ("batch_size", ctypes.c_int32)]


class mcm_server_stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("submitted", "completed", "rejected", "queued", "in_flight",
                                              "bytes_in_use", "peak_bytes", "budget_bytes", "launches_batched",
                                              "launches_grid", "max_batch_seen")]


class mcm_stats(ctypes.Structure):
    _fields_ = [("phases", ctypes.c_int64), ("levels", ctypes.c_int64), ("edges_scanned", ctypes.c_int64),
                ("cols_expanded", ctypes.c_int64), ("cols_claimed", ctypes.c_int64), ("rows_found", ctypes.c_int64),
                ("alt_steps", ctypes.c_int64), ("fix_resets", ctypes.c_int64), ("roots", ctypes.c_int64),
                ("t_expand_ms", ctypes.c_double), ("t_flush_ms", ctypes.c_double), ("t_barrier_ms", ctypes.c_double),
                ("t_small_ms", ctypes.c_double), ("t_augment_ms", ctypes.c_double), ("init_card", ctypes.c_int64),
                ("card", ctypes.c_int64), ("kernel_ms", ctypes.c_double), ("loop", ctypes.c_int32),
                ("mapping", ctypes.c_int32), ("claims_tried", ctypes.c_int64), ("claim", ctypes.c_int32),
                ("flush", ctypes.c_int32), ("wr_check", ctypes.c_int32), ("alternate", ctypes.c_int32),
                ("pass_bytes", ctypes.c_int64), ("schedule", ctypes.c_int32),
                ("local_levels", ctypes.c_int32)]


EXPORTS = ["mcm_match", "mcm_match_noalloc", "mcm_match_batched", "mcm_konig_cover", "mcm_bfs_levels", "mcm_cheap_init_host",
           "mcm_cheap_init", "mcm_batch_plan_create", "mcm_batch_plan_run", "mcm_batch_plan_info",
           "mcm_batch_plan_destroy", "mcm_server_create", "mcm_server_submit", "mcm_server_poll",
           "mcm_server_stats_get", "mcm_server_destroy", "mcm_set_option", "mcm_get_option", "mcm_last_stats",
           "mcm_last_phases", "mcm_strerror", "mcm_version", "mcm_shutdown", "mcm_bfs_forest"]

_lib = None


def lib():
    """Load libmcm.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.mcm_match.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp]
    L.mcm_match.restype = i64
    L.mcm_match_noalloc.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp]
    L.mcm_match_noalloc.restype = i64
    L.mcm_match_batched.argtypes = [i32, ctypes.POINTER(mcm_graph), vp, vp, vp, vp, vp, vp, vp, vp]
    L.mcm_match_batched.restype = i64
    L.mcm_konig_cover.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp]
    L.mcm_konig_cover.restype = i64
    L.mcm_bfs_levels.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp]
    L.mcm_bfs_levels.restype = i64
    L.mcm_bfs_forest.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.mcm_bfs_forest.restype = i64
    L.mcm_cheap_init_host.argtypes = [i32, i32, vp, vp, vp, vp]
    L.mcm_cheap_init_host.restype = i64
    L.mcm_cheap_init.argtypes = [i32, i32, vp, vp, vp, vp, vp]
    L.mcm_cheap_init.restype = i64
    L.mcm_batch_plan_create.argtypes = [i32, ctypes.POINTER(mcm_graph), vp, vp, vp, vp, vp, vp,
                                        ctypes.POINTER(ctypes.c_void_p)]
    L.mcm_batch_plan_create.restype = i64
    L.mcm_batch_plan_run.argtypes = [vp, vp, vp]
    L.mcm_batch_plan_run.restype = i64
    L.mcm_batch_plan_info.argtypes = [vp, ctypes.c_char_p, i32]
    L.mcm_batch_plan_info.restype = ctypes.c_int
    L.mcm_batch_plan_destroy.argtypes = [vp]
    L.mcm_batch_plan_destroy.restype = ctypes.c_int
    L.mcm_server_create.argtypes = [i64, i32, ctypes.POINTER(ctypes.c_void_p)]
    L.mcm_server_create.restype = i64
    L.mcm_server_submit.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    L.mcm_server_submit.restype = i64
    L.mcm_server_poll.argtypes = [vp, i64, ctypes.POINTER(mcm_request_info), ctypes.c_double]
    L.mcm_server_poll.restype = i64
    L.mcm_server_stats_get.argtypes = [vp, ctypes.POINTER(mcm_server_stats)]
    L.mcm_server_stats_get.restype = ctypes.c_int
    L.mcm_server_destroy.argtypes = [vp]
    L.mcm_server_destroy.restype = ctypes.c_int
    L.mcm_set_option.argtypes = [ctypes.c_char_p, ctypes.c_char_p]
    L.mcm_set_option.restype = ctypes.c_int
    L.mcm_get_option.argtypes = [ctypes.c_char_p, ctypes.c_char_p, i32]
    L.mcm_get_option.restype = ctypes.c_int
    L.mcm_last_stats.argtypes = [ctypes.POINTER(mcm_stats)]
    L.mcm_last_stats.restype = ctypes.c_int
    L.mcm_last_phases.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    L.mcm_last_phases.restype = ctypes.c_int64
    L.mcm_strerror.argtypes = [i64]
    L.mcm_strerror.restype = ctypes.c_char_p
    L.mcm_version.argtypes = []
    L.mcm_version.restype = ctypes.c_char_p
    L.mcm_shutdown.argtypes = []
    L.mcm_shutdown.restype = ctypes.c_int
    _lib = L
    # release the library's device memory, pinned buffers, events, live
    # plans and servers while the HIP runtime is still up (before the
    # interpreter and the runtime tear down)
    atexit.register(L.mcm_shutdown)
    return L


def _check(rc: int) -> int:
    if rc < 0:
        raise McmError(int(rc), lib().mcm_strerror(rc).decode())
    return int(rc)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr() if t.numel() > 0 else None


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dev_i32(t, n: int, name: str):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous int32 CUDA tensor")
    if t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, needs {n}")


# ---------------------------------------------------------------- options / stats
def set_option(key: str, value) -> None:
    _check(lib().mcm_set_option(key.encode(), str(value).encode()))


def get_option(key: str) -> str:
    buf = ctypes.create_string_buffer(256)
    _check(lib().mcm_get_option(key.encode(), buf, 256))
    return buf.value.decode()


def last_stats() -> dict:
    s = mcm_stats()
    _check(lib().mcm_last_stats(ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in mcm_stats._fields_}


def last_phases():
    """(levels, ends) per phase of the last mcm_match run with stats=1 on the
    device- or host-loop path: BFS levels expanded and unmatched rows reached."""
    n = _check(lib().mcm_last_phases(None, None, 0))
    lv = np.zeros(max(n, 1), np.int32)
    en = np.zeros(max(n, 1), np.int32)
    _check(lib().mcm_last_phases(lv.ctypes.data, en.ctypes.data, n))
    return lv[:n], en[:n]


def version() -> str:
    return lib().mcm_version().decode()


# ---------------------------------------------------------------- host helper
def cheap_init_host(colptr: np.ndarray, rowind: np.ndarray, nrows: int):
    """Greedy initial matching on host arrays; returns (card, cmatch, rmatch)."""
    cp = np.ascontiguousarray(colptr, dtype=np.int32)
    ri = np.ascontiguousarray(rowind, dtype=np.int32)
    nc = len(cp) - 1
    cm = np.empty(max(nc, 1), np.int32)
    rm = np.empty(max(nrows, 1), np.int32)
    ri_p = ri.ctypes.data if ri.size else None
    card = _check(lib().mcm_cheap_init_host(nc, nrows, cp.ctypes.data, ri_p, cm.ctypes.data, rm.ctypes.data))
    return card, cm[:nc].copy(), rm[:nrows].copy()


# ---------------------------------------------------------------- device graph
@dataclass
class DeviceGraph:
    nc: int
    nr: int
    colptr: "object"   # torch int32 [nc+1]
    rowind: "object"   # torch int32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowind.numel())


def to_device(g, device="cuda:0") -> DeviceGraph:
    """Copy a host graph (graphgen.Graph or any object with nc, nr, colptr, rowind) to the GPU."""
    import torch
    cp = torch.from_numpy(np.ascontiguousarray(g.colptr, dtype=np.int32)).to(device)
    ri = torch.from_numpy(np.ascontiguousarray(g.rowind, dtype=np.int32)).to(device)
    return DeviceGraph(int(g.nc), int(g.nr), cp, ri)


# ---------------------------------------------------------------- entry points
def match(dg: DeviceGraph, init_cmatch=None, init_rmatch=None, out_cmatch=None, out_rmatch=None, stream=None):
    """mcm_match; returns (|M|, cmatch, rmatch) as CUDA tensors."""
    import torch
    dev = dg.colptr.device
    if out_cmatch is None:
        out_cmatch = torch.empty(max(dg.nc, 0), dtype=torch.int32, device=dev)
    if out_rmatch is None:
        out_rmatch = torch.empty(max(dg.nr, 0), dtype=torch.int32, device=dev)
    _dev_i32(dg.colptr, dg.nc + 1, "colptr")
    _dev_i32(out_cmatch, dg.nc, "out_cmatch")
    _dev_i32(out_rmatch, dg.nr, "out_rmatch")
    if init_cmatch is not None:
        _dev_i32(init_cmatch, dg.nc, "init_cmatch")
        _dev_i32(init_rmatch, dg.nr, "init_rmatch")
    card = _check(lib().mcm_match(dg.nc, dg.nr, _ptr(dg.colptr), _ptr(dg.rowind), _ptr(init_cmatch),
                                  _ptr(init_rmatch), _ptr(out_cmatch), _ptr(out_rmatch), _stream(stream)))
    return card, out_cmatch, out_rmatch


def match_noalloc(dg: DeviceGraph, init_cmatch, init_rmatch, out_cmatch, out_rmatch, stream=None):
    """mcm_match_noalloc: the caller passes every array (nothing is
    allocated here or in the library); returns |M|."""
    _dev_i32(dg.colptr, dg.nc + 1, "colptr")
    _dev_i32(out_cmatch, dg.nc, "out_cmatch")
    _dev_i32(out_rmatch, dg.nr, "out_rmatch")
    if init_cmatch is not None:
        _dev_i32(init_cmatch, dg.nc, "init_cmatch")
        _dev_i32(init_rmatch, dg.nr, "init_rmatch")
    return _check(lib().mcm_match_noalloc(dg.nc, dg.nr, _ptr(dg.colptr), _ptr(dg.rowind), _ptr(init_cmatch),
                                          _ptr(init_rmatch), _ptr(out_cmatch), _ptr(out_rmatch), _stream(stream)))


def konig_cover(dg: DeviceGraph, cmatch, rmatch, stream=None):
    """mcm_konig_cover; returns (|K|, col_in_cover, row_in_cover) as CUDA uint8 tensors."""
    import torch
    dev = dg.colptr.device
    cc = torch.empty(dg.nc, dtype=torch.uint8, device=dev)
    rc = torch.empty(dg.nr, dtype=torch.uint8, device=dev)
    k = _check(lib().mcm_konig_cover(dg.nc, dg.nr, _ptr(dg.colptr), _ptr(dg.rowind), _ptr(cmatch), _ptr(rmatch),
                                     _ptr(cc), _ptr(rc), _stream(stream)))
    return k, cc, rc


def bfs_levels(dg: DeviceGraph, cmatch, rmatch, stream=None):
    """mcm_bfs_levels; returns (free rows reached, col_level, row_pred)."""
    import torch
    dev = dg.colptr.device
    cl = torch.empty(dg.nc, dtype=torch.int32, device=dev)
    rp = torch.empty(dg.nr, dtype=torch.int32, device=dev)
    f = _check(lib().mcm_bfs_levels(dg.nc, dg.nr, _ptr(dg.colptr), _ptr(dg.rowind), _ptr(cmatch), _ptr(rmatch),
                                    _ptr(cl), _ptr(rp), _stream(stream)))
    return f, cl, rp


def bfs_forest(dg: DeviceGraph, cmatch, rmatch, stream=None):
    """mcm_bfs_forest; returns (ends, col_level, col_root, row_pred), ends
    being the unmatched rows reached that Alternate would start from."""
    import torch
    dev = dg.colptr.device
    cl = torch.empty(dg.nc, dtype=torch.int32, device=dev)
    cr = torch.empty(dg.nc, dtype=torch.int32, device=dev)
    rp = torch.empty(dg.nr, dtype=torch.int32, device=dev)
    en = torch.empty(max(dg.nr, 1), dtype=torch.int32, device=dev)
    n = _check(lib().mcm_bfs_forest(dg.nc, dg.nr, _ptr(dg.colptr), _ptr(dg.rowind), _ptr(cmatch), _ptr(rmatch),
                                    _ptr(cl), _ptr(cr), _ptr(rp), _ptr(en), _stream(stream)))
    return en[:n], cl, cr, rp


@dataclass
class DeviceBatch:
    """Packed graphs: per-graph local CSC concatenated, descriptors on host."""
    descs: "ctypes.Array"
    colptr: "object"
    rowind: "object"
    ncol_total: int
    nrow_total: int

    @property
    def ngraphs(self) -> int:
        return len(self.descs)


def pack_batch(graphs: Sequence, device="cuda:0") -> DeviceBatch:
    """Pack host graphs into one DeviceBatch (colptr blocks of nc+1, rows local)."""
    import torch
    n = len(graphs)
    descs = (mcm_graph * max(n, 1))()
    cps, ris = [], []
    cpo = rio = co = ro = 0
    for i, g in enumerate(graphs):
        descs[i] = mcm_graph(int(g.nc), int(g.nr), cpo, rio, co, ro)
        cps.append(np.asarray(g.colptr, np.int32))
        ris.append(np.asarray(g.rowind, np.int32))
        cpo += g.nc + 1
        rio += len(g.rowind)
        co += g.nc
        ro += g.nr
    cp = np.concatenate(cps) if cps else np.zeros(1, np.int32)
    ri = np.concatenate(ris) if ris else np.zeros(1, np.int32)
    if ri.size == 0:
        ri = np.zeros(1, np.int32)
    b = DeviceBatch(descs, torch.from_numpy(cp).to(device), torch.from_numpy(ri).to(device), co, ro)
    b.descs = descs if n else (mcm_graph * 0)()
    return b


def match_batched(b: DeviceBatch, init_cmatch=None, init_rmatch=None, out_cmatch=None, out_rmatch=None,
                  stream=None):
    """mcm_match_batched; returns (sum |M_g|, per-graph |M_g| numpy, cmatch, rmatch)."""
    import torch
    dev = b.colptr.device
    if out_cmatch is None:
        out_cmatch = torch.empty(max(b.ncol_total, 1), dtype=torch.int32, device=dev)
    if out_rmatch is None:
        out_rmatch = torch.empty(max(b.nrow_total, 1), dtype=torch.int32, device=dev)
    card = np.zeros(max(b.ngraphs, 1), np.int64)
    total = _check(lib().mcm_match_batched(b.ngraphs, b.descs, _ptr(b.colptr), _ptr(b.rowind), _ptr(init_cmatch),
                                           _ptr(init_rmatch), _ptr(out_cmatch), _ptr(out_rmatch),
                                           card.ctypes.data, _stream(stream)))
    return total, card[: b.ngraphs], out_cmatch, out_rmatch


def cheap_init(dg: DeviceGraph, stream=None):
    """mcm_cheap_init (device parallel greedy); returns (|M0|, cmatch, rmatch)."""
    import torch
    dev = dg.colptr.device
    cm = torch.empty(dg.nc, dtype=torch.int32, device=dev)
    rm = torch.empty(dg.nr, dtype=torch.int32, device=dev)
    card = _check(lib().mcm_cheap_init(dg.nc, dg.nr, _ptr(dg.colptr), _ptr(dg.rowind), _ptr(cm), _ptr(rm),
                                       _stream(stream)))
    return card, cm, rm


class BatchPlan:
    """mcm_batch_plan_*: a captured, replayable batched match over fixed arrays."""

    def __init__(self, b: DeviceBatch, init_cmatch=None, init_rmatch=None, out_cmatch=None, out_rmatch=None):
        import torch
        dev = b.colptr.device
        self.batch = b
        self.init_cmatch, self.init_rmatch = init_cmatch, init_rmatch
        self.out_cmatch = out_cmatch if out_cmatch is not None else torch.empty(max(b.ncol_total, 1),
                                                                                dtype=torch.int32, device=dev)
        self.out_rmatch = out_rmatch if out_rmatch is not None else torch.empty(max(b.nrow_total, 1),
                                                                                dtype=torch.int32, device=dev)
        h = ctypes.c_void_p()
        _check(lib().mcm_batch_plan_create(b.ngraphs, b.descs, _ptr(b.colptr), _ptr(b.rowind), _ptr(init_cmatch),
                                           _ptr(init_rmatch), _ptr(self.out_cmatch), _ptr(self.out_rmatch),
                                           ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        card = np.zeros(max(self.batch.ngraphs, 1), np.int64)
        total = _check(lib().mcm_batch_plan_run(self._h, card.ctypes.data, _stream(stream)))
        return total, card[: self.batch.ngraphs]

    def info(self) -> dict:
        import json
        buf = ctypes.create_string_buffer(1024)
        _check(lib().mcm_batch_plan_info(self._h, buf, 1024))
        return json.loads(buf.value.decode())

    def close(self):
        if self._h:
            lib().mcm_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """mcm_server_*: continuous-batching matching server on the current device.

    submit() copies a host graph into pinned buffers the server reads from
    (kept alive here until the request is polled done) and returns a ticket;
    poll() returns None while the request is in flight, else (card, info,
    cmatch, rmatch) with the outputs as numpy arrays."""

    def __init__(self, budget_bytes: int, max_batch: int = 1024):
        h = ctypes.c_void_p()
        _check(lib().mcm_server_create(int(budget_bytes), int(max_batch), ctypes.byref(h)))
        self._h = h
        self._bufs = {}

    def submit(self, g) -> int:
        import torch
        cp = torch.from_numpy(np.ascontiguousarray(g.colptr, dtype=np.int32)).pin_memory()
        ri = torch.from_numpy(np.ascontiguousarray(g.rowind, dtype=np.int32)).pin_memory()
        cm = torch.empty(int(g.nc), dtype=torch.int32).pin_memory()
        rm = torch.empty(int(g.nr), dtype=torch.int32).pin_memory()
        return self.submit_pinned(int(g.nc), int(g.nr), cp, ri, cm, rm)

    def submit_pinned(self, nc, nr, cp, ri, cm, rm) -> int:
        """Submit already pinned host tensors (kept referenced until done)."""
        t = _check(lib().mcm_server_submit(self._h, nc, nr, _ptr(cp), _ptr(ri), _ptr(cm), _ptr(rm)))
        self._bufs[t] = (cp, ri, cm, rm)
        return t

    def poll(self, ticket: int, wait_ms: float = 0.0):
        info = mcm_request_info()
        rc = _check(lib().mcm_server_poll(self._h, int(ticket), ctypes.byref(info), float(wait_ms)))
        if rc == 0:
            return None
        cp, ri, cm, rm = self._bufs.pop(ticket)
        d = {f: getattr(info, f) for f, _ in mcm_request_info._fields_}
        return d["card"], d, cm.numpy(), rm.numpy()

    def stats(self) -> dict:
        s = mcm_server_stats()
        _check(lib().mcm_server_stats_get(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in mcm_server_stats._fields_}

    def close(self):
        if self._h:
            lib().mcm_server_destroy(self._h)
            self._h = None
            self._bufs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

