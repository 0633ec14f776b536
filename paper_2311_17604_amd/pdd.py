"""Thin ctypes binding of libpdd (the C ABI in include/pdd.h).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch provides device memory and the stream.  The library must have been
built (``paper_2311_17604_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdd.so")

PDD_OK, PDD_EINVAL, PDD_ERANGE, PDD_ENOMEM, PDD_EHIP, PDD_EINTERNAL = range(6)
PDD_F_CHECK = 1
PDD_F_TIMING = 2
PDD_F_PROGRESS = 4
PDD_F_EAGER = 8
PHASES = ("grid", "knn", "reverse", "rounds", "final")

STATS = ("rounds", "researches", "danger_checks", "reverse_rebuilds", "scratch_bytes", "voxel_log2",
         "list_width", "touched", "knn_tested", "pred_hits", "pred_misses", "knn_fallbacks",
         "research_tested", "danger_enumerated", "graph_rounds")
PRED_NPARAM = 8385

_lib = None


class PddError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("b", ctypes.c_int32), ("voxel_log2", ctypes.c_int32),
                ("round_frac", ctypes.c_float), ("point_stride", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("round_blocks", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


QMAX_R, QNFRAC = 32, 7
QFRACTILES = (0.01, 0.1, 0.25, 0.5, 0.75, 0.9, 0.99)


class Quality(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int32), ("fractile_capped", ctypes.c_int32), ("m", ctypes.c_int64),
                ("area_m2", ctypes.c_double * QMAX_R), ("mean", ctypes.c_double * QMAX_R),
                ("fractile", (ctypes.c_uint32 * QNFRAC) * QMAX_R), ("sum", ctypes.c_uint64 * QMAX_R),
                ("sum_sq", ctypes.c_uint64 * QMAX_R), ("slope", ctypes.c_double), ("intercept", ctypes.c_double),
                ("r_squared", ctypes.c_double), ("rmse", ctypes.c_double), ("nn2_min", ctypes.c_int64)]


def load():
    """Load libpdd.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libpdd.so is not built (run paper_2311_17604_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.pdd_ctx_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P]
    lib.pdd_ctx_create.restype = ctypes.c_int
    lib.pdd_ctx_destroy.argtypes = [P]
    lib.pdd_ctx_destroy.restype = None
    lib.pdd_build_grid.argtypes = [P, P, i64, i32, i32, ctypes.POINTER(P)]
    lib.pdd_build_grid.restype = ctypes.c_int
    lib.pdd_grid_free.argtypes = [P, P]
    lib.pdd_grid_free.restype = None
    lib.pdd_grid_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    lib.pdd_grid_info.restype = ctypes.c_int
    lib.pdd_knn_cost.argtypes = [P, P, i32, i32, P, P, P]
    lib.pdd_knn_cost.restype = ctypes.c_int
    lib.pdd_decimate.argtypes = [P, P, i64, i64, ctypes.POINTER(Opts), P, P, P]
    lib.pdd_decimate.restype = ctypes.c_int
    lib.pdd_decimate_batch.argtypes = [P, P, P, i32, P, ctypes.POINTER(Opts), P, P, P]
    lib.pdd_decimate_batch.restype = ctypes.c_int
    lib.pdd_autotune.argtypes = [P, P, i64, i64, ctypes.POINTER(Opts), i64, ctypes.POINTER(Opts),
                                 ctypes.POINTER(ctypes.c_float)]
    lib.pdd_autotune.restype = ctypes.c_int
    lib.pdd_autotune_batch.argtypes = [P, P, P, i32, P, ctypes.POINTER(Opts), i64, ctypes.POINTER(Opts),
                                       ctypes.POINTER(ctypes.c_float)]
    lib.pdd_autotune_batch.restype = ctypes.c_int
    lib.pdd_quality_measure.argtypes = [P, P, i64, i32, P, i32, P, P, ctypes.POINTER(Quality)]
    lib.pdd_quality_measure.restype = ctypes.c_int
    lib.pdd_last_stats.argtypes = [P, ctypes.POINTER(i64), ctypes.c_int]
    lib.pdd_last_stats.restype = ctypes.c_int
    lib.pdd_last_timing.argtypes = [P, ctypes.POINTER(ctypes.c_float), ctypes.c_int]
    lib.pdd_last_timing.restype = ctypes.c_int
    f32 = ctypes.c_float
    lib.pdd_pred_set_weights.argtypes = [P, P, i64]
    lib.pdd_pred_get_weights.argtypes = [P, P, i64]
    lib.pdd_pred_enable.argtypes = [P, i32, f32]
    lib.pdd_pred_samples.argtypes = [P, P, i32, i32, P, P, i64, ctypes.POINTER(i64)]
    lib.pdd_pred_forward.argtypes = [P, P, i64, P]
    lib.pdd_pred_grad.argtypes = [P, P, P, i64, f32, P, P]
    lib.pdd_pred_train.argtypes = [P, P, P, i64, i32, i32, f32, f32, ctypes.c_uint64, P]
    for f in ("pdd_pred_set_weights", "pdd_pred_get_weights", "pdd_pred_enable", "pdd_pred_samples",
              "pdd_pred_forward", "pdd_pred_grad", "pdd_pred_train"):
        getattr(lib, f).restype = ctypes.c_int
    lib.pdd_strerror.argtypes = [ctypes.c_int]
    lib.pdd_strerror.restype = ctypes.c_char_p
    lib.pdd_last_error.argtypes = [P]
    lib.pdd_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """A libpdd context bound to one device and stream (torch's current
    stream of that device by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.pdd_ctx_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if rc != PDD_OK:
            raise PddError(rc, "pdd_ctx_create: " + self.lib.pdd_strerror(rc).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.pdd_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != PDD_OK:
            detail = self.lib.pdd_last_error(self.h).decode()
            raise PddError(rc, "%s: %s %s" % (what, self.lib.pdd_strerror(rc).decode(), detail))

    def timing(self) -> dict:
        """Phase durations (ms, HIP events) of the last timed decimation."""
        arr = (ctypes.c_float * 8)()
        n = self.lib.pdd_last_timing(self.h, arr, 8)
        return {PHASES[i]: float(arr[i]) for i in range(n)}

    def stats(self) -> dict:
        arr = (ctypes.c_int64 * len(STATS))()
        n = self.lib.pdd_last_stats(self.h, arr, len(STATS))
        return {STATS[i]: int(arr[i]) for i in range(n) if not STATS[i].startswith("unused")}


def _points(xyz):
    import torch
    if not (isinstance(xyz, torch.Tensor) and xyz.is_cuda and xyz.dtype == torch.int32 and xyz.dim() == 2
            and xyz.shape[1] in (3, 4) and xyz.is_contiguous()):
        raise ValueError("points must be a contiguous int32 CUDA tensor of shape [n, 3] or [n, 4]")
    return xyz, 4 * xyz.shape[1]


def knn_cost(ctx: Context, xyz, k: int, b: int = 0, voxel_log2: int = 0):
    """(nbr [n, k+b] int32, r2k [n] int64, cost [n] int64 holding uint64 bits)."""
    import torch
    pts, stride = _points(xyz)
    n = pts.shape[0]
    g = ctypes.c_void_p()
    ctx._check(ctx.lib.pdd_build_grid(ctx.h, _ptr(pts), n, stride, voxel_log2, ctypes.byref(g)), "pdd_build_grid")
    try:
        nbr = torch.empty((n, k + b), dtype=torch.int32, device=pts.device)
        r2k = torch.empty(n, dtype=torch.int64, device=pts.device)
        cost = torch.empty(n, dtype=torch.int64, device=pts.device)
        ctx._check(ctx.lib.pdd_knn_cost(ctx.h, g, k, b, _ptr(nbr), _ptr(r2k), _ptr(cost)), "pdd_knn_cost")
        ctx.stream.synchronize()
    finally:
        ctx.lib.pdd_grid_free(ctx.h, g)
    return nbr, r2k, cost


def grid_info(ctx: Context, xyz, voxel_log2: int = 0):
    pts, stride = _points(xyz)
    g = ctypes.c_void_p()
    ctx._check(ctx.lib.pdd_build_grid(ctx.h, _ptr(pts), pts.shape[0], stride, voxel_log2, ctypes.byref(g)),
               "pdd_build_grid")
    nc, s = ctypes.c_int64(), ctypes.c_int32()
    ctx.lib.pdd_grid_info(g, ctypes.byref(nc), ctypes.byref(s))
    ctx.lib.pdd_grid_free(ctx.h, g)
    return int(nc.value), int(s.value)


def decimate(ctx: Context, xyz, keep: int, k: int, b: int = 0, voxel_log2: int = 0, round_frac: float = 0.0,
             check: bool = False, with_order: bool = True, out=None, timing: bool = False,
             progress: bool = False, round_blocks: int = 0, eager: bool = False):
    """Greedy decimation to `keep` points.  Returns (kept [keep] int32,
    order [n-keep] int32 or None, order_cost [n-keep] int64 (uint64 bits) or
    None).  `out` may supply preallocated (kept, order, order_cost)."""
    import torch
    pts, stride = _points(xyz)
    n = pts.shape[0]
    if out is not None:
        kept, order, order_cost = out
    else:
        kept = torch.empty(keep, dtype=torch.int32, device=pts.device)
        order = torch.empty(n - keep, dtype=torch.int32, device=pts.device) if with_order else None
        order_cost = torch.empty(n - keep, dtype=torch.int64, device=pts.device) if with_order else None
    o = Opts(k=k, b=b, voxel_log2=voxel_log2, round_frac=round_frac, point_stride=stride,
             flags=(PDD_F_CHECK if check else 0) | (PDD_F_TIMING if timing else 0)
             | (PDD_F_PROGRESS if progress else 0) | (PDD_F_EAGER if eager else 0), round_blocks=round_blocks)
    ctx._check(ctx.lib.pdd_decimate(ctx.h, _ptr(pts), n, keep, ctypes.byref(o), _ptr(kept), _ptr(order),
                                    _ptr(order_cost)), "pdd_decimate")
    return kept, order, order_cost


def autotune(ctx: Context, xyz, keep: int, k: int, sample: int = 0, b: int = 0, voxel_log2: int = 0,
             round_frac: float = 0.0):
    """Chosen settings for decimating xyz: dict(b, voxel_log2, round_frac,
    best_ms) from timed trials on a strided sample (results never depend on
    them)."""
    pts, stride = _points(xyz)
    base = Opts(k=k, b=b, voxel_log2=voxel_log2, round_frac=round_frac, point_stride=stride, flags=0)
    out = Opts()
    ms = ctypes.c_float()
    ctx._check(ctx.lib.pdd_autotune(ctx.h, _ptr(pts), pts.shape[0], keep, ctypes.byref(base), sample,
                                    ctypes.byref(out), ctypes.byref(ms)), "pdd_autotune")
    return {"b": int(out.b), "voxel_log2": int(out.voxel_log2), "round_frac": float(out.round_frac),
            "best_ms": float(ms.value)}


def autotune_batch(ctx: Context, xyz, offsets, keeps, k: int, sample: int = 0, b: int = 0, voxel_log2: int = 0,
                   round_frac: float = 0.0):
    """Chosen settings for decimate_batch on this batch: dict(b, voxel_log2,
    round_frac, best_ms) from timed trials on every step-th cloud (results
    never depend on them)."""
    import numpy as np
    pts, stride = _points(xyz)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    kp = np.ascontiguousarray(keeps, dtype=np.int64)
    if off.shape != (len(kp) + 1,) or off[-1] != pts.shape[0]:
        raise ValueError("offsets must have len(keeps) + 1 entries ending at the number of points")
    base = Opts(k=k, b=b, voxel_log2=voxel_log2, round_frac=round_frac, point_stride=stride, flags=0)
    out = Opts()
    ms = ctypes.c_float()
    ctx._check(ctx.lib.pdd_autotune_batch(ctx.h, _ptr(pts), off.ctypes.data_as(ctypes.c_void_p), len(kp),
                                          kp.ctypes.data_as(ctypes.c_void_p), ctypes.byref(base), sample,
                                          ctypes.byref(out), ctypes.byref(ms)), "pdd_autotune_batch")
    return {"b": int(out.b), "voxel_log2": int(out.voxel_log2), "round_frac": float(out.round_frac),
            "best_ms": float(ms.value)}


def quality(ctx: Context, xyz, r2, with_counts: bool = True):
    """The quality measures of a cloud (pdd_quality_measure): returns
    (summary dict, counts [m, R] int32 tensor or None, nn2 [m] int64 tensor)."""
    import numpy as np
    import torch
    pts, stride = _points(xyz)
    m = pts.shape[0]
    r2a = np.ascontiguousarray(r2, dtype=np.int64)
    R = len(r2a)
    counts = torch.empty((m, R), dtype=torch.int32, device=pts.device) if with_counts else None
    nn2 = torch.empty(m, dtype=torch.int64, device=pts.device)
    q = Quality()
    ctx._check(ctx.lib.pdd_quality_measure(ctx.h, _ptr(pts), m, stride, r2a.ctypes.data_as(ctypes.c_void_p), R,
                                           _ptr(counts), _ptr(nn2), ctypes.byref(q)), "pdd_quality_measure")
    summ = {"m": int(q.m), "area_m2": list(q.area_m2[:R]), "mean": list(q.mean[:R]),
            "fractiles": [list(q.fractile[r]) for r in range(R)], "sum": list(q.sum[:R]),
            "sum_sq": list(q.sum_sq[:R]), "slope": q.slope, "intercept": q.intercept, "r_squared": q.r_squared,
            "rmse": q.rmse, "nn2_min": int(q.nn2_min), "fractile_capped": bool(q.fractile_capped)}
    return summ, counts, nn2


def decimate_batch(ctx: Context, xyz, offsets, keeps, k: int, b: int = 0, voxel_log2: int = 0,
                   round_frac: float = 0.0, check: bool = False, with_order: bool = True, timing: bool = False,
                   progress: bool = False, round_blocks: int = 0, eager: bool = False):
    """Independent clouds decimated together: cloud s is rows
    offsets[s]:offsets[s+1] of xyz and keeps keeps[s] points.  Returns
    (kept, order, order_cost), each the clouds' results one after another,
    indices relative to each cloud's first row."""
    import numpy as np
    import torch
    pts, stride = _points(xyz)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    kp = np.ascontiguousarray(keeps, dtype=np.int64)
    nscan = len(kp)
    if off.shape != (nscan + 1,) or off[-1] != pts.shape[0]:
        raise ValueError("offsets must have len(keeps) + 1 entries ending at the number of points")
    total_keep = int(kp.sum())
    m = int(pts.shape[0] - total_keep)
    kept = torch.empty(total_keep, dtype=torch.int32, device=pts.device)
    order = torch.empty(m, dtype=torch.int32, device=pts.device) if with_order else None
    order_cost = torch.empty(m, dtype=torch.int64, device=pts.device) if with_order else None
    o = Opts(k=k, b=b, voxel_log2=voxel_log2, round_frac=round_frac, point_stride=stride,
             flags=(PDD_F_CHECK if check else 0) | (PDD_F_TIMING if timing else 0)
             | (PDD_F_PROGRESS if progress else 0) | (PDD_F_EAGER if eager else 0), round_blocks=round_blocks)
    ctx._check(ctx.lib.pdd_decimate_batch(ctx.h, _ptr(pts), off.ctypes.data_as(ctypes.c_void_p), nscan,
                                          kp.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o), _ptr(kept),
                                          _ptr(order), _ptr(order_cost)), "pdd_decimate_batch")
    return kept, order, order_cost


# ---------------------------------------------------------------------------
# search-radius predictor
# ---------------------------------------------------------------------------

def pred_init(seed: int, out_bias: float = 0.0):
    """Initial predictor parameters in the library's flat layout (W1 [64 in]
    [64 out], b1, W2, b2, w3, b3): He-normal hidden weights, zero hidden
    biases, small output weights, output bias `out_bias`."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, np.sqrt(2 / 64), 64 * 64), np.zeros(64), rng.normal(0, np.sqrt(2 / 64), 64 * 64),
             np.zeros(64), rng.normal(0, 0.05, 64), np.array([out_bias])]
    p = np.concatenate(parts).astype(np.float32)
    assert p.shape == (PRED_NPARAM,)
    return p


def pred_set_weights(ctx: Context, params):
    """Set the predictor's PRED_NPARAM fp32 parameters (numpy array)."""
    import numpy as np
    a = np.ascontiguousarray(params, dtype=np.float32)
    if a.shape != (PRED_NPARAM,):
        raise ValueError("expected %d parameters" % PRED_NPARAM)
    ctx._check(ctx.lib.pdd_pred_set_weights(ctx.h, a.ctypes.data_as(ctypes.c_void_p), a.size), "pdd_pred_set_weights")


def pred_get_weights(ctx: Context):
    import numpy as np
    a = np.empty(PRED_NPARAM, dtype=np.float32)
    ctx._check(ctx.lib.pdd_pred_get_weights(ctx.h, a.ctypes.data_as(ctypes.c_void_p), a.size), "pdd_pred_get_weights")
    return a


def pred_enable(ctx: Context, on: bool, margin_log2: float = 0.25):
    ctx._check(ctx.lib.pdd_pred_enable(ctx.h, 1 if on else 0, margin_log2), "pdd_pred_enable")


def pred_samples(ctx: Context, xyz, k: int, b: int = 0, voxel_log2: int = 0):
    """Training rows of a cloud: (features [m, 64] int16 holding bf16 bits,
    targets [m] float32), one row per anchor cell."""
    import torch
    pts, stride = _points(xyz)
    n = pts.shape[0]
    g = ctypes.c_void_p()
    ctx._check(ctx.lib.pdd_build_grid(ctx.h, _ptr(pts), n, stride, voxel_log2, ctypes.byref(g)), "pdd_build_grid")
    try:
        cnt = ctypes.c_int64()
        ctx._check(ctx.lib.pdd_pred_samples(ctx.h, g, k, b, None, None, 0, ctypes.byref(cnt)), "pdd_pred_samples")
        m = int(cnt.value)
        feat = torch.empty((max(m, 1), 64), dtype=torch.int16, device=pts.device)
        tgt = torch.empty(max(m, 1), dtype=torch.float32, device=pts.device)
        ctx._check(ctx.lib.pdd_pred_samples(ctx.h, g, k, b, _ptr(feat), _ptr(tgt), m, ctypes.byref(cnt)),
                   "pdd_pred_samples")
    finally:
        ctx.lib.pdd_grid_free(ctx.h, g)
    return feat[:m], tgt[:m]


def pred_forward(ctx: Context, feat):
    import torch
    out = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
    ctx._check(ctx.lib.pdd_pred_forward(ctx.h, _ptr(feat), feat.shape[0], _ptr(out)), "pdd_pred_forward")
    return out


def pred_grad(ctx: Context, feat, target, tau: float):
    """(gradient [PRED_NPARAM] float32, loss) over all rows (at most 128)."""
    import torch
    grad = torch.empty(PRED_NPARAM, dtype=torch.float32, device=feat.device)
    loss = torch.empty(1, dtype=torch.float32, device=feat.device)
    ctx._check(ctx.lib.pdd_pred_grad(ctx.h, _ptr(feat), _ptr(target), feat.shape[0], tau, _ptr(grad), _ptr(loss)),
               "pdd_pred_grad")
    return grad, float(loss.item())


def pred_train(ctx: Context, feat, target, steps: int, batch: int = 128, lr: float = 1e-3, tau: float = 0.9,
               seed: int = 1):
    """Adam steps on the context's predictor; returns the per-step losses."""
    import torch
    loss = torch.empty(max(steps, 1), dtype=torch.float32, device=feat.device)
    ctx._check(ctx.lib.pdd_pred_train(ctx.h, _ptr(feat), _ptr(target), feat.shape[0], steps, batch, lr, tau, seed,
                                      _ptr(loss)), "pdd_pred_train")
    return loss[:steps]
