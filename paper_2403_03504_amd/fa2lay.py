"""Thin Python binding of libfa2lay.so (the C ABI in include/fa2lay.h).

Argument marshalling only: every step of the layout runs in the library's HIP
kernels.  PyTorch supplies device memory and the current HIP stream.  There is
no CPU fallback: importing this module raises if the library is not built, and
every call raises ``FlError`` on a non-zero status.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfa2lay.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2403_03504_amd.build` "
                      "(hipcc --offload-arch=gfx950); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)

FL_OK, FL_EINVAL, FL_ENOMEM, FL_EHIP, FL_ENONFINITE, FL_EBUSY, FL_ECANCELED, FL_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
GRAV_STRONG_MASS, GRAV_FA2_CONST, GRAV_STRONG_UNIT = 0, 1, 2
SWING_PAPER, SWING_FA2 = 0, 1
REP_EXACT, REP_FMM, REP_AUTO = 0, 1, 2
KK_MAJORIZATION, KK_NEWTON = 0, 1
KK_REDUCE_LEAVES, KK_REDUCE_CHAINS = 1, 2
TUNE_MAX_BUCKETS = 16
PHASES = ("tree", "lists", "upward", "m2l", "eval", "attract", "update", "exact", "bh", "far")

EXPORTED = ("fl_create", "fl_destroy", "fl_last_error", "fl_set_stream", "fl_synchronize", "fl_workspace_bytes",
            "fl_version", "fl_build_csr", "fl_components", "fl_morton", "fl_sort_keys", "fl_tree",
            "fl_fa2_default_params", "fl_fa2_forces", "fl_fa2_step", "fl_fa2_step_noalloc", "fl_fa2_run",
            "fl_fmm_stats",
            "fl_set_timing", "fl_set_graphs", "fl_get_timing", "fl_kk_default_params", "fl_hop_distances",
            "fl_kk_steps", "fl_kk_layout", "fl_layout", "fl_server_create", "fl_server_create_fake",
            "fl_server_submit", "fl_server_poll", "fl_server_wait", "fl_server_result", "fl_server_release",
            "fl_server_cancel", "fl_server_stats_get", "fl_server_last_error", "fl_server_destroy",
            "fl_default_tuning", "fl_set_tuning", "fl_get_tuning", "fl_autotune", "fl_server_set_tuning",
            "fl_assemble_default_params", "fl_assemble", "fl_bh_repulsion")
JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED, JOB_CANCELED = 0, 1, 2, 3, 4


class FlError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class FA2Params(ctypes.Structure):
    _fields_ = [("kr", ctypes.c_double), ("kg", ctypes.c_double), ("ka", ctypes.c_double),
                ("gravity_mode", ctypes.c_int32), ("swing_mode", ctypes.c_int32),
                ("tau", ctypes.c_double), ("ks", ctypes.c_double), ("ksmax", ctypes.c_double),
                ("max_rise", ctypes.c_double), ("repulsion", ctypes.c_int32), ("p", ctypes.c_int32),
                ("leaf_size", ctypes.c_int32), ("morton_bits", ctypes.c_int32), ("list_lanes", ctypes.c_int32)]


class _State(ctypes.Structure):
    _fields_ = [("fx_prev", ctypes.c_void_p), ("fy_prev", ctypes.c_void_p), ("scalars", ctypes.c_void_p),
                ("iter", ctypes.c_int64), ("n_comp", ctypes.c_int32), ("comp_offsets", ctypes.c_void_p)]


class KKParams(ctypes.Structure):
    _fields_ = [("l", ctypes.c_double), ("steps", ctypes.c_int32), ("minimiser", ctypes.c_int32),
                ("eps", ctypes.c_double), ("reduce", ctypes.c_int32)]


class AssembleParams(ctypes.Structure):
    _fields_ = [("density", ctypes.c_double), ("gap", ctypes.c_double), ("max_group", ctypes.c_int32),
                ("sweeps", ctypes.c_int32)]


class AssembleStats(ctypes.Structure):
    _fields_ = [("n_comp", ctypes.c_int32), ("levels", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class LayoutStats(ctypes.Structure):
    _fields_ = [("n_comp", ctypes.c_int32), ("n_single", ctypes.c_int32), ("n_kk", ctypes.c_int32),
                ("n_fa2", ctypes.c_int32), ("kk_nodes", ctypes.c_int64), ("fa2_nodes", ctypes.c_int64),
                ("ms_setup", ctypes.c_double), ("ms_kk", ctypes.c_double), ("ms_fa2", ctypes.c_double)]


class _Job(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("x0", ctypes.c_void_p), ("y0", ctypes.c_void_p), ("iters", ctypes.c_int32),
                ("params", FA2Params)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "admitted", "completed", "failed", "canceled", "queued",
                                               "running", "bytes_in_use", "peak_bytes", "node_updates",
                                               "held_bytes", "peak_held_bytes", "trims", "over_estimate")]


class Tuning(ctypes.Structure):
    _fields_ = [("fmm_min_nodes", ctypes.c_int32), ("n_buckets", ctypes.c_int32),
                ("bucket_max", ctypes.c_int32 * TUNE_MAX_BUCKETS), ("p", ctypes.c_int32 * TUNE_MAX_BUCKETS),
                ("leaf_size", ctypes.c_int32 * TUNE_MAX_BUCKETS), ("list_lanes", ctypes.c_int32 * TUNE_MAX_BUCKETS),
                ("max_rel_err", ctypes.c_double)]

    def to_dict(self) -> dict:
        nb = self.n_buckets
        return {"fmm_min_nodes": self.fmm_min_nodes, "bucket_max": list(self.bucket_max[:nb]),
                "p": list(self.p[:nb]), "leaf_size": list(self.leaf_size[:nb]),
                "list_lanes": list(self.list_lanes[:nb]), "max_rel_err": self.max_rel_err}

    @staticmethod
    def from_dict(d: dict) -> "Tuning":
        t = Tuning()
        nb = len(d["p"])
        if not (len(d["bucket_max"]) == len(d["leaf_size"]) == nb):
            raise ValueError("tuning: bucket_max, p and leaf_size differ in length")
        t.fmm_min_nodes, t.n_buckets, t.max_rel_err = int(d["fmm_min_nodes"]), nb, float(d.get("max_rel_err", 0.0))
        lanes = d.get("list_lanes", [0] * nb)
        if len(lanes) != nb:
            raise ValueError("tuning: list_lanes differs in length")
        for i in range(nb):
            t.bucket_max[i], t.p[i], t.leaf_size[i] = int(d["bucket_max"][i]), int(d["p"][i]), int(d["leaf_size"][i])
            t.list_lanes[i] = int(lanes[i])
        return t


class TuneSample(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int32), ("p", ctypes.c_int32), ("leaf_size", ctypes.c_int32),
                ("list_lanes", ctypes.c_int32), ("feasible", ctypes.c_int32), ("ms", ctypes.c_double),
                ("rel_err", ctypes.c_double)]


class StepStats(ctypes.Structure):
    _fields_ = [("swg", ctypes.c_double), ("tra", ctypes.c_double), ("speed", ctypes.c_double)]


P = ctypes.c_void_p
_i32, _i64 = ctypes.c_int32, ctypes.c_int64
_sig = {
    "fl_create": ([ctypes.POINTER(P), ctypes.c_int, P, ctypes.c_size_t], _i32),
    "fl_destroy": ([P], None),
    "fl_last_error": ([P], ctypes.c_char_p),
    "fl_set_stream": ([P, P], _i32),
    "fl_synchronize": ([P], _i32),
    "fl_workspace_bytes": ([P], ctypes.c_size_t),
    "fl_version": ([], ctypes.c_char_p),
    "fl_build_csr": ([P, _i32, _i64, P, P, P, P, P, ctypes.POINTER(_i64)], _i32),
    "fl_components": ([P, _i32, P, P, P, ctypes.POINTER(_i32)], _i32),
    "fl_morton": ([P, _i32, P, P, _i32, P, P], _i32),
    "fl_sort_keys": ([P, _i32, P, _i32, P, P], _i32),
    "fl_tree": ([P, _i32, P, P, _i32, _i32, P, _i32, ctypes.POINTER(_i32)], _i32),
    "fl_fa2_default_params": ([ctypes.POINTER(FA2Params)], None),
    "fl_fa2_forces": ([P, _i32, P, P, P, P, P, ctypes.POINTER(FA2Params), P, P, P, P, P, P], _i32),
    "fl_fa2_step": ([P, _i32, P, P, P, P, P, ctypes.POINTER(_State), ctypes.POINTER(FA2Params),
                     ctypes.POINTER(StepStats)], _i32),
    "fl_fa2_step_noalloc": ([P, _i32, P, P, P, P, P, ctypes.POINTER(_State), ctypes.POINTER(FA2Params),
                             ctypes.POINTER(StepStats)], _i32),
    "fl_fa2_run": ([P, _i32, P, P, P, P, P, ctypes.POINTER(_State), ctypes.POINTER(FA2Params), _i32,
                    ctypes.POINTER(StepStats)], _i32),
    "fl_fmm_stats": ([P, ctypes.POINTER(_i64), ctypes.c_int], _i32),
    "fl_set_timing": ([P, ctypes.c_int], _i32),
    "fl_set_graphs": ([P, ctypes.c_int], _i32),
    "fl_kk_default_params": ([ctypes.POINTER(KKParams)], None),
    "fl_hop_distances": ([P, _i32, P, P, P, P, P], _i32),
    "fl_kk_steps": ([P, _i32, P, P, P, P, ctypes.POINTER(KKParams)], _i32),
    "fl_kk_layout": ([P, _i32, P, P, P, P, P, ctypes.POINTER(KKParams)], _i32),
    "fl_layout": ([P, _i32, P, P, P, P, P, ctypes.POINTER(FA2Params), _i32, ctypes.POINTER(KKParams), _i32, _i32,
                   ctypes.POINTER(LayoutStats)], _i32),
    "fl_get_timing": ([P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)], _i32),
    "fl_assemble_default_params": ([ctypes.POINTER(AssembleParams)], None),
    "fl_bh_repulsion": ([P, _i32, P, P, P, ctypes.c_double, ctypes.c_double, _i32, _i32, P, P], _i32),
    "fl_assemble": ([P, _i32, P, _i32, P, P, P, ctypes.POINTER(AssembleParams), P, P,
                     ctypes.POINTER(AssembleStats)], _i32),
    "fl_default_tuning": ([ctypes.POINTER(Tuning)], None),
    "fl_set_tuning": ([P, ctypes.POINTER(Tuning)], _i32),
    "fl_get_tuning": ([P, ctypes.POINTER(Tuning)], _i32),
    "fl_autotune": ([P, _i32, P, P, P, _i32, P, ctypes.c_double, _i32, ctypes.POINTER(Tuning),
                     ctypes.POINTER(TuneSample), _i32, ctypes.POINTER(_i32)], _i32),
}
_U64 = ctypes.c_uint64
_sig.update({
    "fl_server_create": ([ctypes.POINTER(P), ctypes.c_int, ctypes.c_size_t, _i32], _i32),
    "fl_server_create_fake": ([ctypes.POINTER(P), ctypes.c_size_t, _i32, ctypes.c_double], _i32),
    "fl_server_submit": ([P, ctypes.POINTER(_Job), ctypes.POINTER(_U64)], _i32),
    "fl_server_poll": ([P, _U64, ctypes.POINTER(_i32)], _i32),
    "fl_server_wait": ([P, _U64, ctypes.c_double, ctypes.POINTER(_i32)], _i32),
    "fl_server_result": ([P, _U64, P, P, P], _i32),
    "fl_server_release": ([P, _U64], _i32),
    "fl_server_cancel": ([P, _U64], _i32),
    "fl_server_stats_get": ([P, ctypes.POINTER(ServerStats)], _i32),
    "fl_server_last_error": ([P], ctypes.c_char_p),
    "fl_server_destroy": ([P], None),
    "fl_server_set_tuning": ([P, ctypes.POINTER(Tuning)], _i32),
})
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def version() -> str:
    return _lib.fl_version().decode()


def default_params(**kw) -> FA2Params:
    p = FA2Params()
    _lib.fl_fa2_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def default_tuning() -> dict:
    t = Tuning()
    _lib.fl_default_tuning(ctypes.byref(t))
    return t.to_dict()


def kk_params(**kw) -> KKParams:
    p = KKParams()
    _lib.fl_kk_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def assemble_params(**kw) -> AssembleParams:
    p = AssembleParams()
    _lib.fl_assemble_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _host_i32(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _ptr(t: torch.Tensor | None, dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


@dataclasses.dataclass
class FA2State:
    """Caller-owned iteration state (previous forces, device scalars, count);
    with comp_offsets (host int32, n_comp + 1 entries) the nodes form
    independent systems, each with its own four scalars."""
    fx_prev: torch.Tensor
    fy_prev: torch.Tensor
    scalars: torch.Tensor  # float64 [4 * systems]: s_G, SWG, TRA per system
    iter: int = 0
    comp_offsets: object = None

    @staticmethod
    def zeros(n: int, device, comp_offsets=None) -> "FA2State":
        import numpy as np
        off = None if comp_offsets is None else np.ascontiguousarray(comp_offsets, dtype=np.int32)
        k = 1 if off is None else max(off.shape[0] - 1, 1)
        return FA2State(torch.zeros(n, dtype=torch.float32, device=device),
                        torch.zeros(n, dtype=torch.float32, device=device),
                        torch.zeros(4 * k, dtype=torch.float64, device=device), 0, off)

    def _c(self) -> _State:
        off = self.comp_offsets
        if off is None:
            return _State(self.fx_prev.data_ptr(), self.fy_prev.data_ptr(), self.scalars.data_ptr(), self.iter, 0,
                          None)
        return _State(self.fx_prev.data_ptr(), self.fy_prev.data_ptr(), self.scalars.data_ptr(), self.iter,
                      off.shape[0] - 1, off.ctypes.data_as(ctypes.c_void_p))


class Graph:
    """A CSR graph on the device (int32 row_ptr, col_idx, deg)."""

    def __init__(self, n: int, row_ptr: torch.Tensor, col: torch.Tensor, deg: torch.Tensor):
        self.n, self.row_ptr, self.col, self.deg = n, row_ptr, col, deg


class Context:
    """An fl_ctx bound to a device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None, budget_bytes: int = 0):
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._h = P()
        self._check(_lib.fl_create(ctypes.byref(self._h), device, P(stream.cuda_stream), budget_bytes),
                    "fl_create")

    def close(self):
        if getattr(self, "_h", None):
            _lib.fl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str):
        if st != FL_OK:
            msg = _lib.fl_last_error(self._h).decode() if self._h else what
            raise FlError(st, f"{what}: {msg}")

    def set_stream(self, stream):
        self._check(_lib.fl_set_stream(self._h, P(stream.cuda_stream)), "fl_set_stream")

    def synchronize(self):
        self._check(_lib.fl_synchronize(self._h), "fl_synchronize")

    def workspace_bytes(self) -> int:
        return int(_lib.fl_workspace_bytes(self._h))

    # graph preparation ----------------------------------------------------
    def build_csr(self, n: int, src: torch.Tensor, dst: torch.Tensor) -> Graph:
        m = int(src.numel())
        row_ptr = torch.empty(n + 1, dtype=torch.int32, device=self.device)
        col = torch.empty(max(2 * m, 1), dtype=torch.int32, device=self.device)
        deg = torch.empty(n, dtype=torch.int32, device=self.device)
        nnz = _i64()
        self._check(_lib.fl_build_csr(self._h, n, m, _ptr(src, torch.int32), _ptr(dst, torch.int32), _ptr(row_ptr),
                                      _ptr(col), _ptr(deg), ctypes.byref(nnz)), "fl_build_csr")
        return Graph(n, row_ptr, col[:max(nnz.value, 1)].contiguous() if nnz.value else col, deg)

    def components(self, g: Graph):
        label = torch.empty(g.n, dtype=torch.int32, device=self.device)
        k = _i32()
        self._check(_lib.fl_components(self._h, g.n, _ptr(g.row_ptr, torch.int32), _ptr(g.col, torch.int32),
                                       _ptr(label), ctypes.byref(k)), "fl_components")
        return label, int(k.value)

    # quadtree hooks ----------------------------------------------------------
    def morton(self, x: torch.Tensor, y: torch.Tensor, bits: int = 16):
        n = x.numel()
        key = torch.empty(n, dtype=torch.int32, device=self.device)  # uint32 bit patterns
        root = torch.empty(4, dtype=torch.float64, device=self.device)
        self._check(_lib.fl_morton(self._h, n, _ptr(x, torch.float32), _ptr(y, torch.float32), bits, _ptr(key),
                                   _ptr(root)), "fl_morton")
        return key, root

    def sort_keys(self, key: torch.Tensor, bits: int = 16):
        n = key.numel()
        out = torch.empty_like(key)
        perm = torch.empty(n, dtype=torch.int32, device=self.device)
        self._check(_lib.fl_sort_keys(self._h, n, _ptr(key, torch.int32), bits, _ptr(out), _ptr(perm)),
                    "fl_sort_keys")
        return out, perm

    def tree(self, x: torch.Tensor, y: torch.Tensor, bits: int = 16, leaf_size: int = 64, cap: int | None = None):
        n = x.numel()
        cap = cap if cap is not None else 4 * n + 16
        cells = torch.empty(cap * 10, dtype=torch.int32, device=self.device)
        nc = _i32()
        self._check(_lib.fl_tree(self._h, n, _ptr(x, torch.float32), _ptr(y, torch.float32), bits, leaf_size,
                                 _ptr(cells), cap, ctypes.byref(nc)), "fl_tree")
        return cells[:10 * nc.value].view(nc.value, 10)

    # ForceAtlas2 -------------------------------------------------------------
    def fa2_forces(self, g: Graph, x: torch.Tensor, y: torch.Tensor, params: FA2Params, components=True):
        n = g.n
        out = {k: torch.empty(n, dtype=torch.float32, device=self.device) for k in ("frx", "fry")}
        if components:
            for k in ("fax", "fay", "fgx", "fgy"):
                out[k] = torch.empty(n, dtype=torch.float32, device=self.device)
        self._check(_lib.fl_fa2_forces(self._h, n, _ptr(g.row_ptr, torch.int32), _ptr(g.col, torch.int32),
                                       _ptr(g.deg, torch.int32), _ptr(x, torch.float32), _ptr(y, torch.float32),
                                       ctypes.byref(params), _ptr(out["frx"]), _ptr(out["fry"]),
                                       _ptr(out.get("fax")), _ptr(out.get("fay")), _ptr(out.get("fgx")),
                                       _ptr(out.get("fgy"))), "fl_fa2_forces")
        return out

    def fa2_step(self, g: Graph, x: torch.Tensor, y: torch.Tensor, state: FA2State, params: FA2Params,
                 stats: bool = True):
        cs = state._c()
        st = StepStats()
        self._check(_lib.fl_fa2_step(self._h, g.n, _ptr(g.row_ptr, torch.int32), _ptr(g.col, torch.int32),
                                     _ptr(g.deg, torch.int32), _ptr(x, torch.float32), _ptr(y, torch.float32),
                                     ctypes.byref(cs), ctypes.byref(params), ctypes.byref(st) if stats else None),
                    "fl_fa2_step")
        state.iter = int(cs.iter)
        return (st.swg, st.tra, st.speed) if stats else None

    def fa2_step_noalloc(self, g: Graph, x: torch.Tensor, y: torch.Tensor, state: FA2State, params: FA2Params,
                         stats: bool = True):
        """fl_fa2_step_noalloc: fl_fa2_step with its workspace in the library's
        fixed per-GPU scratch array (allocates nothing)."""
        cs = state._c()
        st = StepStats()
        self._check(_lib.fl_fa2_step_noalloc(self._h, g.n, _ptr(g.row_ptr, torch.int32), _ptr(g.col, torch.int32),
                                             _ptr(g.deg, torch.int32), _ptr(x, torch.float32),
                                             _ptr(y, torch.float32), ctypes.byref(cs), ctypes.byref(params),
                                             ctypes.byref(st) if stats else None), "fl_fa2_step_noalloc")
        state.iter = int(cs.iter)
        return (st.swg, st.tra, st.speed) if stats else None

    def fa2_run(self, g: Graph, x: torch.Tensor, y: torch.Tensor, state: FA2State, params: FA2Params, iters: int,
                stats: bool = False):
        cs = state._c()
        arr = (StepStats * max(iters, 1))() if stats else None
        self._check(_lib.fl_fa2_run(self._h, g.n, _ptr(g.row_ptr, torch.int32), _ptr(g.col, torch.int32),
                                    _ptr(g.deg, torch.int32), _ptr(x, torch.float32), _ptr(y, torch.float32),
                                    ctypes.byref(cs), ctypes.byref(params), iters, arr), "fl_fa2_run")
        state.iter = int(cs.iter)
        if stats:
            return [(a.swg, a.tra, a.speed) for a in arr[:iters]]
        return None

    # Kamada-Kawai (components given as node ranges, host offsets) ----------
    def hop_distances(self, g: Graph, comp_offsets):
        import numpy as np
        off, offp = _host_i32(comp_offsets)
        sizes = np.diff(off.astype(np.int64))
        dist = torch.empty(int(np.sum(sizes * sizes)), dtype=torch.int32, device=self.device)
        doff = np.zeros(off.shape[0], dtype=np.int64)
        self._check(_lib.fl_hop_distances(self._h, off.shape[0] - 1, offp, _ptr(g.row_ptr, torch.int32),
                                          _ptr(g.col, torch.int32), _ptr(dist),
                                          doff.ctypes.data_as(ctypes.c_void_p)), "fl_hop_distances")
        return dist, doff

    def kk_steps(self, comp_offsets, dist: torch.Tensor, x: torch.Tensor, y: torch.Tensor, params: KKParams):
        off, offp = _host_i32(comp_offsets)
        self._check(_lib.fl_kk_steps(self._h, off.shape[0] - 1, offp, _ptr(dist, torch.int32),
                                     _ptr(x, torch.float32), _ptr(y, torch.float32), ctypes.byref(params)),
                    "fl_kk_steps")

    def kk_layout(self, g: Graph, comp_offsets, x: torch.Tensor, y: torch.Tensor, params: KKParams):
        off, offp = _host_i32(comp_offsets)
        self._check(_lib.fl_kk_layout(self._h, off.shape[0] - 1, offp, _ptr(g.row_ptr, torch.int32),
                                      _ptr(g.col, torch.int32), _ptr(x, torch.float32), _ptr(y, torch.float32),
                                      ctypes.byref(params)), "fl_kk_layout")

    def layout(self, g: Graph, x: torch.Tensor, y: torch.Tensor, fa2: FA2Params, fa2_iters: int,
               kk: KKParams, kk_max_nodes: int = 256, fmm_min_nodes: int = 4096) -> dict:
        st = LayoutStats()
        self._check(_lib.fl_layout(self._h, g.n, _ptr(g.row_ptr, torch.int32), _ptr(g.col, torch.int32),
                                   _ptr(g.deg, torch.int32), _ptr(x, torch.float32), _ptr(y, torch.float32),
                                   ctypes.byref(fa2), fa2_iters, ctypes.byref(kk), kk_max_nodes, fmm_min_nodes,
                                   ctypes.byref(st)), "fl_layout")
        return {k: getattr(st, k) for k, _ in LayoutStats._fields_}

    def bh_repulsion(self, x: torch.Tensor, y: torch.Tensor, deg: torch.Tensor, kr: float = 1.0,
                     theta: float = 0.5, leaf_size: int = 64, morton_bits: int = 16):
        """fl_bh_repulsion: Barnes-Hut F_r as (frx, fry) device tensors."""
        n = x.shape[0]
        frx = torch.empty(n, dtype=torch.float32, device=x.device)
        fry = torch.empty_like(frx)
        self._check(_lib.fl_bh_repulsion(self._h, n, _ptr(x, torch.float32), _ptr(y, torch.float32),
                                         _ptr(deg, torch.int32), kr, theta, leaf_size, morton_bits, _ptr(frx),
                                         _ptr(fry)), "fl_bh_repulsion")
        return frx, fry

    def assemble(self, label: torch.Tensor, n_comp: int, order, x: torch.Tensor, y: torch.Tensor,
                 params: AssembleParams, frame: torch.Tensor | None = None,
                 parent: torch.Tensor | None = None) -> dict:
        """fl_assemble: in place on x, y; order is a host permutation of
        0..n_comp-1; frame (float64, n_comp*6) and parent (int32, n_comp) are
        optional device outputs."""
        o, op = _host_i32(order)
        if o.shape != (n_comp,):
            raise ValueError("order must hold n_comp entries")
        st = AssembleStats()
        self._check(_lib.fl_assemble(self._h, x.shape[0], _ptr(label, torch.int32), n_comp, op,
                                     _ptr(x, torch.float32), _ptr(y, torch.float32), ctypes.byref(params),
                                     _ptr(frame, torch.float64), _ptr(parent, torch.int32), ctypes.byref(st)),
                    "fl_assemble")
        return {k: getattr(st, k) for k, _ in AssembleStats._fields_}

    def fmm_stats(self, reset: bool = False) -> dict:
        out = (_i64 * 12)()
        self._check(_lib.fl_fmm_stats(self._h, out, 1 if reset else 0), "fl_fmm_stats")
        keys = ("cells", "leaves", "near_pairs", "v_entries", "w_entries", "x_entries", "max_level", "u_entries",
                "total_near_pairs", "total_v_entries", "evaluations", "total_particles")
        return dict(zip(keys, (int(v) for v in out)))

    def set_timing(self, enable: bool):
        self._check(_lib.fl_set_timing(self._h, 1 if enable else 0), "fl_set_timing")

    def set_graphs(self, enable: bool):
        self._check(_lib.fl_set_graphs(self._h, 1 if enable else 0), "fl_set_graphs")

    def set_tuning(self, tuning: dict | None):
        t = Tuning.from_dict(tuning) if tuning is not None else None
        self._check(_lib.fl_set_tuning(self._h, ctypes.byref(t) if t is not None else None), "fl_set_tuning")

    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(_lib.fl_get_tuning(self._h, ctypes.byref(t)), "fl_get_tuning")
        return t.to_dict()

    def autotune(self, x: torch.Tensor, y: torch.Tensor, deg: torch.Tensor, sizes, max_rel_err: float = 1e-3,
                 reps: int = 3):
        """fl_autotune: returns (tuning dict, list of measurement dicts); the
        table is also installed in this context."""
        sz, szp = _host_i32(sizes)
        cap = len(sz) * 128
        arr = (TuneSample * cap)()
        ns = _i32()
        t = Tuning()
        self._check(_lib.fl_autotune(self._h, x.shape[0], _ptr(x, torch.float32), _ptr(y, torch.float32),
                                     _ptr(deg, torch.int32), len(sz), szp, max_rel_err, reps, ctypes.byref(t), arr,
                                     cap, ctypes.byref(ns)), "fl_autotune")
        samples = [{k: getattr(arr[i], k) for k, _ in TuneSample._fields_} for i in range(min(ns.value, cap))]
        return t.to_dict(), samples

    def get_timing(self):
        ms = (ctypes.c_double * len(PHASES))()
        cnt = (_i64 * len(PHASES))()
        self._check(_lib.fl_get_timing(self._h, ms, cnt), "fl_get_timing")
        return {p: (ms[i], int(cnt[i])) for i, p in enumerate(PHASES)}


class Server:
    """Continuous-batching layout server (fl_server_*).  Jobs are host arrays;
    results come back as host numpy arrays with arrival/start/done times."""

    def __init__(self, device: int = 0, budget_bytes: int = 32 << 30, slots: int = 4,
                 fake_ns_per_update: float = 0.0):
        self._h = P()
        if fake_ns_per_update > 0:
            st = _lib.fl_server_create_fake(ctypes.byref(self._h), budget_bytes, slots, fake_ns_per_update)
        else:
            st = _lib.fl_server_create(ctypes.byref(self._h), device, budget_bytes, slots)
        if st != FL_OK:
            raise FlError(st, "fl_server_create failed")
        self._keep = {}

    def _check(self, st: int, what: str):
        if st != FL_OK:
            raise FlError(st, f"{what}: {_lib.fl_server_last_error(self._h).decode()}")

    def submit(self, n: int, src, dst, x0, y0, iters: int, params: FA2Params) -> int:
        import numpy as np
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        x0 = np.ascontiguousarray(x0, dtype=np.float32)
        y0 = np.ascontiguousarray(y0, dtype=np.float32)
        j = _Job(n, src.shape[0], src.ctypes.data, dst.ctypes.data, x0.ctypes.data, y0.ctypes.data, iters, params)
        jid = _U64()
        self._check(_lib.fl_server_submit(self._h, ctypes.byref(j), ctypes.byref(jid)), "fl_server_submit")
        self._keep[jid.value] = n
        return int(jid.value)

    def poll(self, jid: int) -> int:
        s = _i32()
        self._check(_lib.fl_server_poll(self._h, jid, ctypes.byref(s)), "fl_server_poll")
        return int(s.value)

    def wait(self, jid: int, timeout: float = -1.0) -> int:
        s = _i32()
        st = _lib.fl_server_wait(self._h, jid, timeout, ctypes.byref(s))
        if st not in (FL_OK, FL_EBUSY):
            self._check(st, "fl_server_wait")
        return int(s.value)

    def result(self, jid: int, release: bool = True):
        import numpy as np
        n = self._keep[jid]
        x = np.empty(n, np.float32)
        y = np.empty(n, np.float32)
        t = np.zeros(3)
        st = _lib.fl_server_result(self._h, jid, x.ctypes.data, y.ctypes.data, t.ctypes.data)
        self._check(st, "fl_server_result")
        if release:
            _lib.fl_server_release(self._h, jid)
            self._keep.pop(jid, None)
        return x, y, tuple(t)

    def cancel(self, jid: int):
        self._check(_lib.fl_server_cancel(self._h, jid), "fl_server_cancel")

    def set_tuning(self, tuning: dict | None):
        t = Tuning.from_dict(tuning) if tuning is not None else None
        self._check(_lib.fl_server_set_tuning(self._h, ctypes.byref(t) if t is not None else None),
                    "fl_server_set_tuning")

    def stats(self) -> dict:
        s = ServerStats()
        self._check(_lib.fl_server_stats_get(self._h, ctypes.byref(s)), "fl_server_stats_get")
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _lib.fl_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
