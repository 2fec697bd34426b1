"""Python binding of libmulment (multilevel maxent-stress layout on MI355X).

Argument marshalling only: every step runs in the HIP kernels of
libmulment.so, called through its C-ABI (include/mulment.h).  PyTorch is used
for device memory (tensors are passed by data_ptr) and for the stream the
context is bound to.  There is no CPU fallback: if the library is missing or
no GPU is visible, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmulment.so")

MM_HOST, MM_DEVICE = 0, 1
MAX_LEVELS = 64
_STATUS = {0: "MM_OK", 1: "MM_EINVAL", 2: "MM_ENOMEM", 3: "MM_EDEVICE", 4: "MM_EUNSUPPORTED",
           5: "MM_EINTERNAL"}


class MulmentError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class MMGraph(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("node_w", C.c_void_p), ("edge_w", C.c_void_p),
                ("mem", C.c_int32)]


class MMParams(C.Structure):
    _fields_ = [("k", C.c_int32), ("q", C.c_double), ("theta", C.c_double),
                ("alpha0", C.c_double), ("alpha_decay", C.c_double), ("alpha_min", C.c_double),
                ("iters_per_round", C.c_int32), ("eps_round", C.c_double),
                ("eps_final", C.c_double), ("max_final_iters", C.c_int32),
                ("max_levels", C.c_int32), ("coarsest_n", C.c_int32), ("b", C.c_double),
                ("f", C.c_double), ("lp_rounds", C.c_int32), ("coarse_dist_scale", C.c_double),
                ("seed", C.c_uint64), ("validate", C.c_int32), ("mlp_weights", C.c_void_p),
                ("use_graphs", C.c_int32), ("autotune", C.c_int32), ("exact_below", C.c_int32),
                ("approx_h", C.c_int32), ("khop_direct", C.c_int32)]


class MMStats(C.Structure):
    _fields_ = [("levels", C.c_int32), ("level_n", C.c_int32 * MAX_LEVELS),
                ("level_nnz", C.c_int64 * MAX_LEVELS), ("level_khop", C.c_int64 * MAX_LEVELS),
                ("level_iters", C.c_int32 * MAX_LEVELS),
                ("level_final_iters", C.c_int32 * MAX_LEVELS),
                ("level_cap_hit", C.c_int32 * MAX_LEVELS),
                ("level_delta", C.c_double * MAX_LEVELS),
                ("level_sweep_ms", C.c_double * MAX_LEVELS),
                ("level_far_ms", C.c_double * MAX_LEVELS),
                ("level_khop_ms", C.c_double * MAX_LEVELS), ("t_total_ms", C.c_double),
                ("t_coarsen_ms", C.c_double), ("t_khop_ms", C.c_double),
                ("t_farfield_ms", C.c_double), ("t_sweep_ms", C.c_double),
                ("t_other_ms", C.c_double), ("vertex_updates", C.c_int64),
                ("finest_updates", C.c_int64), ("level_tile_bits", C.c_int32 * MAX_LEVELS),
                ("level_group", C.c_int32 * MAX_LEVELS), ("t_tune_ms", C.c_double),
                ("level_blocks", C.c_int32 * MAX_LEVELS), ("t_iterate_ms", C.c_double),
                ("level_wall_ms", C.c_double * MAX_LEVELS)]

    def to_dict(self) -> dict:
        L = self.levels
        return {
            "levels": L,
            "per_level": [
                {"level": i, "n": self.level_n[i], "nnz": self.level_nnz[i],
                 "khop_entries": self.level_khop[i], "iters": self.level_iters[i],
                 "final_iters": self.level_final_iters[i], "cap_hit": self.level_cap_hit[i],
                 "delta": self.level_delta[i], "sweep_ms": self.level_sweep_ms[i],
                 "far_ms": self.level_far_ms[i], "khop_ms": self.level_khop_ms[i],
                 "tile_bits": self.level_tile_bits[i], "group": self.level_group[i],
                 "blocks": self.level_blocks[i], "wall_ms": self.level_wall_ms[i]}
                for i in range(L)],
            "t_total_ms": self.t_total_ms, "t_coarsen_ms": self.t_coarsen_ms,
            "t_khop_ms": self.t_khop_ms, "t_farfield_ms": self.t_farfield_ms,
            "t_sweep_ms": self.t_sweep_ms, "t_other_ms": self.t_other_ms,
            "vertex_updates": self.vertex_updates, "finest_updates": self.finest_updates,
            "t_tune_ms": self.t_tune_ms, "t_iterate_ms": self.t_iterate_ms,
        }


EXPORTS = ["mm_params_default", "mm_context_create", "mm_context_destroy", "mm_sync",
           "mm_last_error", "mm_layout", "mm_khop_build", "mm_khop_free", "mm_khop_info",
           "mm_khop_arrays", "mm_khop_export", "mm_repulsion", "mm_sweep", "mm_sweep_ex",
           "mm_coarsen",
           "mm_coarse_graph", "mm_coarse_export", "mm_coarse_free", "mm_init_layout",
           "mm_prolong", "mm_objective", "mm_full_stress", "mm_repulsion_learned",
           "mm_far_samples", "mm_mlp_forward", "mm_mlp_grad", "mm_mlp_train", "mm_layout_batch",
           "mm_tune_clear", "mm_tune_export", "mm_tune_import", "mm_sweep_cfg",
           "mm_repulsion_cluster", "mm_full_stress_ex", "mm_khop_validate", "mm_khop_import",
           "mm_sweep_noalloc", "mm_mlp_init"]

TUNE_FIELDS = 7  # coarse?, n, sum |S|, k, tile bits, lanes, blocks per step
MLP_PARAMS = 4866  # W1 64x8, b1 64, W2 64x64, b2 64, W3 2x64, b3 2 (FP32, packed)
SWEEP_NOALLOC_MAX_N = 1 << 20  # vertex limit of mm_sweep_noalloc's fixed scratch

_lib = None


def lib():
    """Load libmulment.so (built by paper_1506_04383_amd/build.py); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python paper_1506_04383_amd/build.py` (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    P = C.POINTER
    sig = {
        "mm_params_default": [P(MMParams)],
        "mm_context_create": [P(vp), i32, vp],
        "mm_sync": [vp],
        "mm_layout": [vp, P(MMGraph), P(MMParams), vp, vp, P(MMStats)],
        "mm_khop_build": [vp, P(MMGraph), i32, P(vp)],
        "mm_khop_info": [vp, P(i32), P(i32), P(i64)],
        "mm_khop_arrays": [vp, P(vp), P(vp), P(vp)],
        "mm_khop_export": [vp, vp, vp, vp, vp, i32],
        "mm_khop_validate": [i32, i32, vp, vp, vp],
        "mm_khop_import": [vp, i32, i32, vp, vp, vp, i32, P(vp)],
        "mm_repulsion": [vp, i32, vp, f64, f64, vp, vp, vp, vp, vp],
        "mm_sweep": [vp, vp, i32, vp, f64, vp, vp, f64, f64, vp, vp],
        "mm_sweep_ex": [vp, vp, i32, vp, f64, vp, vp, f64, f64, vp, vp, i32],
        "mm_sweep_noalloc": [vp, vp, i32, vp, f64, vp, vp, f64, f64, vp, vp],
        "mm_sweep_cfg": [vp, vp, i32, vp, f64, vp, vp, f64, f64, vp, vp, i32, i32, i32],
        "mm_coarsen": [vp, P(MMGraph), f64, i32, u64, i32, vp, P(vp), vp, vp],
        "mm_coarse_graph": [vp, P(MMGraph)],
        "mm_coarse_export": [vp, vp, vp, vp, vp, vp, i32],
        "mm_init_layout": [vp, i32, u64, i32, vp],
        "mm_prolong": [vp, i32, vp, vp, vp, u64, i32, vp],
        "mm_objective": [vp, vp, i32, vp, f64, vp, f64, f64, vp],
        "mm_mlp_init": [vp, u64, f64, vp],
        "mm_full_stress": [vp, P(MMGraph), vp, vp],
        "mm_full_stress_ex": [vp, P(MMGraph), vp, i32, vp],
        "mm_repulsion_learned": [vp, i32, vp, f64, vp, vp],
        "mm_layout_batch": [vp, i32, vp, P(MMGraph), P(MMParams), vp, vp, vp, P(MMStats)],
        "mm_tune_clear": [vp],
        "mm_repulsion_cluster": [vp, i32, vp, vp, vp, i32, vp, i32, f64, vp],
        "mm_tune_export": [vp, P(i64), i32, P(i32)],
        "mm_tune_import": [vp, P(i64), i32],
        "mm_far_samples": [vp, i32, vp, f64, i64, vp, vp, vp, vp, vp, P(i64)],
        "mm_mlp_forward": [vp, i64, vp, vp, vp],
        "mm_mlp_grad": [vp, i64, vp, vp, vp, vp, vp],
        "mm_mlp_train": [vp, i64, vp, vp, vp, vp, i32, i32, f64, u64, i32, vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.mm_last_error.restype = C.c_char_p
    L.mm_last_error.argtypes = []
    L.mm_context_destroy.argtypes = [vp]
    L.mm_context_destroy.restype = None
    L.mm_khop_free.argtypes = [vp]
    L.mm_khop_free.restype = None
    L.mm_coarse_free.argtypes = [vp]
    L.mm_coarse_free.restype = None
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise MulmentError(status, lib().mm_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ params

@dataclass
class Params:
    """Mirror of mm_params; defaults are the paper's configuration."""

    k: int = 1
    q: float = 0.0
    theta: float = 0.5
    alpha0: float = 1.0
    alpha_decay: float = 0.3
    alpha_min: float = 0.008
    iters_per_round: int = 2
    eps_round: float = 1e-4
    eps_final: float = 1e-4
    max_final_iters: int = 200
    max_levels: int = 62
    coarsest_n: int = 2
    b: float = 2.0
    f: float = 20.0
    lp_rounds: int = 10
    coarse_dist_scale: float = 1.0
    seed: int = 1
    validate: int = 1
    mlp_weights: object = None  # float32 device tensor of MLP_PARAMS (learned far field)
    use_graphs: int = 1  # replay small levels' iterations from HIP graphs
    autotune: int = 0  # time each level's sweep configurations once per level shape
    exact_below: int = 0  # levels with <= this many vertices use the exact far field
    approx_h: int = 0  # MulMent_h: cluster far field of Eq. 3, h levels beneath
    khop_direct: int = 1  # tile-major sets of bitmap rows straight from the 2-hop search

    def to_c(self) -> MMParams:
        p = MMParams()
        _check(lib().mm_params_default(C.byref(p)))
        for fd in fields(self):
            v = getattr(self, fd.name)
            if fd.name == "mlp_weights":
                v = None if v is None else C.c_void_p(v.data_ptr())
            setattr(p, fd.name, v)
        return p


def default_params() -> Params:
    p = MMParams()
    _check(lib().mm_params_default(C.byref(p)))
    return Params(**{fd.name: getattr(p, fd.name) for fd in fields(Params)
                     if fd.name != "mlp_weights"})


# ------------------------------------------------------------------ context

class Context:
    """One device + the torch stream current at creation."""

    def __init__(self, device: int = 0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: libmulment runs on MI355X only")
        self.device = device
        self.torch = torch
        with torch.cuda.device(device):
            self.stream = torch.cuda.current_stream(device)
        h = C.c_void_p()
        _check(lib().mm_context_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().mm_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        _check(lib().mm_sync(self.h))

    def tune_export(self):
        """The autotuner's choices: int64 array (records, 7) of
        (coarse?, n, sum |S|, k, tile bits (0 = row kernel), lanes, blocks)."""
        cnt = C.c_int32(0)
        _check(lib().mm_tune_export(self.h, None, 0, C.byref(cnt)))
        recs = np.zeros((max(cnt.value, 1), TUNE_FIELDS), np.int64)
        _check(lib().mm_tune_export(self.h, recs.ctypes.data_as(C.POINTER(C.c_int64)), cnt.value,
                                    C.byref(cnt)))
        return recs[: cnt.value]

    def tune_import(self, recs):
        recs = np.ascontiguousarray(recs, dtype=np.int64).reshape(-1, TUNE_FIELDS)
        _check(lib().mm_tune_import(self.h, recs.ctypes.data_as(C.POINTER(C.c_int64)),
                                    recs.shape[0]))

    def tune_clear(self):
        _check(lib().mm_tune_clear(self.h))

    # -- helpers
    def _dev(self, a, dtype):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=f"cuda:{self.device}", dtype=dtype).contiguous()
        return t.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=f"cuda:{self.device}")

    def graph(self, row_ptr, col, node_w=None, edge_w=None):
        """Device graph (tensors kept alive on the returned object)."""
        return DeviceGraph(self, row_ptr, col, node_w, edge_w)


class DeviceGraph:
    def __init__(self, ctx: Context, row_ptr, col, node_w=None, edge_w=None):
        t = ctx.torch
        self.row_ptr = ctx._dev(row_ptr, t.int32)
        self.col = ctx._dev(col, t.int32)
        self.node_w = None if node_w is None else ctx._dev(node_w, t.int32)
        self.edge_w = None if edge_w is None else ctx._dev(edge_w, t.int32)
        self.n = int(self.row_ptr.numel() - 1)
        self.nnz = int(self.col.numel())

    def c(self) -> MMGraph:
        g = MMGraph()
        g.n = self.n
        g.nnz = self.nnz
        g.row_ptr = self.row_ptr.data_ptr()
        g.col = self.col.data_ptr()
        g.node_w = None if self.node_w is None else self.node_w.data_ptr()
        g.edge_w = None if self.edge_w is None else self.edge_w.data_ptr()
        g.mem = MM_DEVICE
        return g


# ------------------------------------------------------------------ entry points

def layout(ctx: Context, g: DeviceGraph, params: Params | None = None, init_xy=None):
    """Full multilevel layout; returns (xy float32 [n,2] on the device, stats dict)."""
    t = ctx.torch
    p = (params or Params()).to_c()
    out = t.empty((g.n, 2), dtype=t.float32, device=f"cuda:{ctx.device}")
    init = None if init_xy is None else ctx._dev(init_xy, t.float32)
    st = MMStats()
    gc = g.c()
    _check(lib().mm_layout(ctx.h, C.byref(gc), C.byref(p), _ptr(init), _ptr(out), C.byref(st)))
    return out, st.to_dict()


def layout_batch(ctx: Context, row_ptr, col, graph_off, params: Params | None = None,
                 init_xy=None):
    """Lay out a batch of independent graphs given as their block-diagonal
    union (row_ptr, col) with vertex offsets graph_off (G+1).  Returns
    (xy float32 [n,2] device tensor, per-graph level counts, stats dict)."""
    t = ctx.torch
    offs = np.ascontiguousarray(graph_off, dtype=np.int64)
    G = offs.size - 1
    dg = row_ptr if isinstance(row_ptr, DeviceGraph) else DeviceGraph(ctx, row_ptr, col)
    # row_ptr may be a DeviceGraph already on the device (col is then ignored)
    p = (params or Params()).to_c()
    out = t.empty((dg.n, 2), dtype=t.float32, device=f"cuda:{ctx.device}")
    init = None if init_xy is None else ctx._dev(init_xy, t.float32)
    lev = np.zeros(G, dtype=np.int32)
    st = MMStats()
    gc = dg.c()
    _check(lib().mm_layout_batch(ctx.h, G, offs.ctypes.data_as(C.c_void_p), C.byref(gc),
                                 C.byref(p), _ptr(init), _ptr(out),
                                 lev.ctypes.data_as(C.c_void_p), C.byref(st)))
    return out, lev, st.to_dict()


class KHop:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h
        n, k, tot = C.c_int32(), C.c_int32(), C.c_int64()
        _check(lib().mm_khop_info(h, C.byref(n), C.byref(k), C.byref(tot)))
        self.n, self.k, self.total = n.value, k.value, tot.value

    def export(self):
        """Host copies (numpy): off int64[n+1], hend int32[n*k], nbr int32[total]."""
        off = np.zeros(self.n + 1, np.int64)
        hend = np.zeros(self.n * self.k, np.int32)
        nbr = np.zeros(max(self.total, 1), np.int32)
        _check(lib().mm_khop_export(self.ctx.h, self.h, off.ctypes.data_as(C.c_void_p),
                                    hend.ctypes.data_as(C.c_void_p),
                                    nbr.ctypes.data_as(C.c_void_p), MM_HOST))
        return off, hend, nbr[:self.total]

    def free(self):
        if self.h:
            lib().mm_khop_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def khop_build(ctx: Context, g: DeviceGraph, k: int) -> KHop:
    h = C.c_void_p()
    gc = g.c()
    _check(lib().mm_khop_build(ctx.h, C.byref(gc), k, C.byref(h)))
    return KHop(ctx, h)


def _set_arrays(off, hend, nbr):
    off = np.ascontiguousarray(off, dtype=np.int64)
    hend = np.ascontiguousarray(hend, dtype=np.int32)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    return off, hend, nbr


def khop_validate(n: int, k: int, off, hend, nbr) -> None:
    """Host check of a general stress set S (raises MMError naming the first
    violation); no device work."""
    off, hend, nbr = _set_arrays(off, hend, nbr)
    if off.size != n + 1 or hend.size != n * k or nbr.size < (off[-1] if off.size else 0):
        raise ValueError("array sizes do not match n, k and off[n]")
    _check(lib().mm_khop_validate(n, k, off.ctypes.data_as(C.c_void_p),
                                  hend.ctypes.data_as(C.c_void_p),
                                  nbr.ctypes.data_as(C.c_void_p)))


def khop_import(ctx: Context, n: int, k: int, off, hend, nbr) -> KHop:
    """A general stress set S ⊇ E with integer target distances 1..k, in the
    layout of the k-hop sets (host numpy arrays or CUDA tensors); usable by
    every sweep configuration and the objective."""
    t = ctx.torch
    h = C.c_void_p()
    dev = [isinstance(a, t.Tensor) and a.is_cuda for a in (off, hend, nbr)]
    if all(dev):
        if off.dtype != t.int64 or hend.dtype != t.int32 or nbr.dtype != t.int32:
            raise TypeError("device arrays must be int64 off, int32 hend and nbr")
        if off.numel() != n + 1 or hend.numel() != n * k:
            raise ValueError("array sizes do not match n and k")
        off, hend, nbr = off.contiguous(), hend.contiguous(), nbr.contiguous()
        if nbr.numel() < int(off[-1].item()):
            raise ValueError("nbr shorter than off[n]")
        _check(lib().mm_khop_import(ctx.h, n, k, _ptr(off), _ptr(hend), _ptr(nbr), MM_DEVICE,
                                    C.byref(h)))
    elif any(dev):
        raise TypeError("off, hend and nbr must all live on the host or all on the device")
    else:
        off, hend, nbr = _set_arrays(off, hend, nbr)
        if off.size != n + 1 or hend.size != n * k or nbr.size < (off[-1] if off.size else 0):
            raise ValueError("array sizes do not match n, k and off[n]")
        _check(lib().mm_khop_import(ctx.h, n, k, off.ctypes.data_as(C.c_void_p),
                                    hend.ctypes.data_as(C.c_void_p),
                                    nbr.ctypes.data_as(C.c_void_p), MM_HOST, C.byref(h)))
    return KHop(ctx, h)


def repulsion(ctx: Context, xy, q: float = 0.0, theta: float = 0.5, export: bool = False,
              counters: bool = False) -> dict:
    """Far field F (float32 [n,2]); with export=True also Morton codes (id order),
    the sorted order and the pre-order node table (Barnes-Hut only)."""
    t = ctx.torch
    xy = ctx._dev(xy, t.float32)
    n = xy.shape[0]
    F = t.empty((n, 2), dtype=t.float32, device=xy.device)
    codes = order = nodes = None
    if export and theta >= 0:
        codes = t.empty(n, dtype=t.int64, device=xy.device)
        order = t.empty(n, dtype=t.int32, device=xy.device)
        nodes = t.zeros((2 * n, 5), dtype=t.int64, device=xy.device)
    cnt = np.zeros(4, np.int64)
    _check(lib().mm_repulsion(ctx.h, n, _ptr(xy), q, theta, _ptr(F), _ptr(codes), _ptr(order),
                              _ptr(nodes), cnt.ctypes.data_as(C.c_void_p) if (counters or export)
                              else None))
    out = {"F": F}
    if export and theta >= 0:
        nn = int(cnt[3])
        out.update(codes=codes.cpu().numpy().view(np.uint64), order=order, nodes=nodes[:nn])
    if counters or export:
        out.update(accepted=int(cnt[0]), leaf_pairs=int(cnt[1]), n_nodes=int(cnt[3]))
    return out


def repulsion_cluster(ctx: Context, xy, cluster1, n1: int, cluster_h, nh: int, node_w=None,
                      q: float = 0.0):
    """Cluster far field of Eq. 3 (mm_repulsion_cluster): float32 [n,2]."""
    t = ctx.torch
    xy = ctx._dev(xy, t.float32)
    n = xy.shape[0]
    c1 = ctx._dev(cluster1, t.int32)
    ch = ctx._dev(cluster_h, t.int32)
    nw = None if node_w is None else ctx._dev(node_w, t.int32)
    F = t.empty((n, 2), dtype=t.float32, device=xy.device)
    _check(lib().mm_repulsion_cluster(ctx.h, n, _ptr(xy), _ptr(nw), _ptr(c1), int(n1), _ptr(ch),
                                      int(nh), q, _ptr(F)))
    return F


def mlp_init(ctx: Context, seed: int, out_scale: float = 0.1):
    """Initial network weights (float32 device tensor of MLP_PARAMS) from
    mm_mlp_init: He-normal hidden layers, output layer scaled by out_scale,
    zero biases."""
    t = ctx.torch
    w = t.empty(MLP_PARAMS, dtype=t.float32, device=f"cuda:{ctx.device}")
    _check(lib().mm_mlp_init(ctx.h, int(seed), float(out_scale), _ptr(w)))
    return w


def repulsion_learned(ctx: Context, xy, theta: float, weights):
    """Barnes-Hut far field (q = 0) with the learned cell correction."""
    t = ctx.torch
    xy = ctx._dev(xy, t.float32)
    w = ctx._dev(weights, t.float32)
    F = t.empty((xy.shape[0], 2), dtype=t.float32, device=xy.device)
    _check(lib().mm_repulsion_learned(ctx.h, xy.shape[0], _ptr(xy), theta, _ptr(w), _ptr(F)))
    return F


def far_samples(ctx: Context, xy, theta: float) -> dict:
    """Accepted (target, cell) pairs with features, exact residual targets and
    kappa e (device tensors), in Morton rank of the target and visit order."""
    t = ctx.torch
    xy = ctx._dev(xy, t.float32)
    n = xy.shape[0]
    cnt = C.c_int64(0)
    _check(lib().mm_far_samples(ctx.h, n, _ptr(xy), theta, 0, None, None, None, None, None,
                                C.byref(cnt)))
    m = cnt.value
    dev = xy.device
    u = t.empty(m, dtype=t.int32, device=dev)
    node = t.empty(m, dtype=t.int32, device=dev)
    feat = t.empty((m, 8), dtype=t.float32, device=dev)
    tgt = t.empty((m, 2), dtype=t.float32, device=dev)
    coef = t.empty((m, 2), dtype=t.float32, device=dev)
    _check(lib().mm_far_samples(ctx.h, n, _ptr(xy), theta, m, _ptr(u), _ptr(node), _ptr(feat),
                                _ptr(tgt), _ptr(coef), C.byref(cnt)))
    return {"u": u, "node": node, "feat": feat, "target": tgt, "coef": coef}


def mlp_forward(ctx: Context, feat, weights):
    t = ctx.torch
    feat = ctx._dev(feat, t.float32)
    w = ctx._dev(weights, t.float32)
    out = t.empty((feat.shape[0], 2), dtype=t.float32, device=feat.device)
    _check(lib().mm_mlp_forward(ctx.h, feat.shape[0], _ptr(feat), _ptr(w), _ptr(out)))
    return out


def mlp_grad(ctx: Context, feat, target, weights):
    """(loss, gradient) of L = 1/(2B) sum |h - y|^2."""
    t = ctx.torch
    feat = ctx._dev(feat, t.float32)
    target = ctx._dev(target, t.float32)
    w = ctx._dev(weights, t.float32)
    g = t.empty(MLP_PARAMS, dtype=t.float32, device=feat.device)
    loss = t.empty(1, dtype=t.float32, device=feat.device)
    _check(lib().mm_mlp_grad(ctx.h, feat.shape[0], _ptr(feat), _ptr(target), _ptr(w), _ptr(g),
                             _ptr(loss)))
    return float(loss.item()), g


def mlp_train(ctx: Context, feat, target, weights, adam, steps: int, batch: int, lr: float,
              seed: int, step0: int = 0):
    """Adam steps in place on `weights` (and the 2*MLP_PARAMS `adam` state);
    returns the per-step minibatch losses (device tensor)."""
    t = ctx.torch
    losses = t.empty(max(steps, 1), dtype=t.float32, device=weights.device)
    _check(lib().mm_mlp_train(ctx.h, feat.shape[0], _ptr(feat), _ptr(target), _ptr(weights),
                              _ptr(adam), steps, batch, lr, seed, step0, _ptr(losses)))
    return losses[:steps]


SWEEP_AUTO, SWEEP_ROWS, SWEEP_TILED = 0, 1, 2


def sweep(ctx: Context, kh: KHop, xy, F, alpha: float, q: float = 0.0, level: int = 0,
          node_w=None, scale: float = 1.0, mode: int = SWEEP_ROWS, config=None):
    """One Jacobi iteration of Eq. 2; returns (xy_out, (|x'-x|^2, |x|^2)).
    mode: SWEEP_ROWS (row-gather kernel), SWEEP_TILED (LDS-tiled), SWEEP_AUTO.
    config = (tile_bits, lanes[, blocks]) forces a configuration instead (mm_sweep_cfg)."""
    t = ctx.torch
    xy = ctx._dev(xy, t.float32)
    F = ctx._dev(F, t.float32)
    nw = None if node_w is None else ctx._dev(node_w, t.int32)
    out = t.empty_like(xy)
    d = np.zeros(2)
    if config is None:
        _check(lib().mm_sweep_ex(ctx.h, kh.h, level, _ptr(nw), scale, _ptr(xy), _ptr(F), alpha, q,
                                 _ptr(out), d.ctypes.data_as(C.c_void_p), mode))
    else:
        blocks = int(config[2]) if len(config) > 2 else 0
        _check(lib().mm_sweep_cfg(ctx.h, kh.h, level, _ptr(nw), scale, _ptr(xy), _ptr(F), alpha,
                                  q, _ptr(out), d.ctypes.data_as(C.c_void_p), int(config[0]),
                                  int(config[1]), blocks))
    return out, (float(d[0]), float(d[1]))


def sweep_noalloc(ctx: Context, kh: KHop, xy, F, alpha: float, q: float = 0.0, level: int = 0,
                  node_w=None, scale: float = 1.0, out=None):
    """mm_sweep_noalloc: the row-kernel Jacobi iteration with the library's
    fixed scratch (no device allocation by the library); out (optional) is
    the caller's output tensor.  Returns (xy_out, (|x'-x|^2, |x|^2))."""
    t = ctx.torch
    xy = ctx._dev(xy, t.float32)
    F = ctx._dev(F, t.float32)
    nw = None if node_w is None else ctx._dev(node_w, t.int32)
    if out is None:
        out = t.empty_like(xy)
    d = np.zeros(2)
    _check(lib().mm_sweep_noalloc(ctx.h, kh.h, level, _ptr(nw), scale, _ptr(xy), _ptr(F), alpha,
                                  q, _ptr(out), d.ctypes.data_as(C.c_void_p)))
    return out, (float(d[0]), float(d[1]))


def coarsen(ctx: Context, g: DeviceGraph, U: float, lp_rounds: int, seed: int, level_h: int):
    """One label-propagation + contraction step.  Returns (cluster[n] device,
    coarse graph as host numpy arrays (row_ptr, col, node_w, edge_w), rounds, moves)."""
    t = ctx.torch
    cluster = t.empty(g.n, dtype=t.int32, device=f"cuda:{ctx.device}")
    h = C.c_void_p()
    rr = C.c_int32()
    moves = np.zeros(max(lp_rounds, 1), np.int64)
    gc = g.c()
    _check(lib().mm_coarsen(ctx.h, C.byref(gc), U, lp_rounds, seed, level_h, _ptr(cluster),
                            C.byref(h), C.byref(rr), moves.ctypes.data_as(C.c_void_p)))
    try:
        view = MMGraph()
        _check(lib().mm_coarse_graph(h, C.byref(view)))
        nc, nnz = view.n, view.nnz
        rp = np.zeros(nc + 1, np.int32)
        col = np.zeros(max(nnz, 1), np.int32)
        cw = np.zeros(nc, np.int32)
        ew = np.zeros(max(nnz, 1), np.int32)
        vp = lambda a: a.ctypes.data_as(C.c_void_p)
        _check(lib().mm_coarse_export(ctx.h, h, vp(rp), vp(col), vp(cw), vp(ew), MM_HOST))
    finally:
        lib().mm_coarse_free(h)
    return cluster, (rp, col[:nnz], cw, ew[:nnz]), rr.value, moves[:rr.value]


def init_layout(ctx: Context, n: int, seed: int, level: int):
    t = ctx.torch
    xy = t.empty((n, 2), dtype=t.float32, device=f"cuda:{ctx.device}")
    _check(lib().mm_init_layout(ctx.h, n, seed, level, _ptr(xy)))
    return xy


def prolong(ctx: Context, cluster, coarse_w, coarse_xy, seed: int, level: int):
    t = ctx.torch
    cl = ctx._dev(cluster, t.int32)
    cw = None if coarse_w is None else ctx._dev(coarse_w, t.int32)
    cxy = ctx._dev(coarse_xy, t.float32)
    out = t.empty((cl.numel(), 2), dtype=t.float32, device=cl.device)
    _check(lib().mm_prolong(ctx.h, cl.numel(), _ptr(cl), _ptr(cw), _ptr(cxy), seed, level,
                            _ptr(out)))
    return out


def objective(ctx: Context, kh: KHop, xy, alpha: float, q: float = 0.0, level: int = 0,
              node_w=None, scale: float = 1.0) -> dict:
    t = ctx.torch
    xy = ctx._dev(xy, t.float32)
    nw = None if node_w is None else ctx._dev(node_w, t.int32)
    out = np.zeros(4)
    _check(lib().mm_objective(ctx.h, kh.h, level, _ptr(nw), scale, _ptr(xy), alpha, q,
                              out.ctypes.data_as(C.c_void_p)))
    return {"M": out[0], "stress": out[1], "ent": out[2], "coincident": int(out[3])}


def full_stress(ctx: Context, g: DeviceGraph, xy, method: int = 0) -> dict:
    """Full stress at the optimal scale; method 0 auto, 1 multi-source BFS,
    2 one BFS per source, 3 banded multi-source search (mm_full_stress_ex)."""
    t = ctx.torch
    xy = ctx._dev(xy, t.float32)
    out = np.zeros(3)
    gc = g.c()
    _check(lib().mm_full_stress_ex(ctx.h, C.byref(gc), _ptr(xy), int(method),
                                   out.ctypes.data_as(C.c_void_p)))
    return {"F_unscaled": out[0], "s_opt": out[1], "F": out[2]}
