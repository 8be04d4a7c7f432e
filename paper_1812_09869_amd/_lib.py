"""ctypes binding of libtsne355.so (argument marshalling only).

Every function here takes torch CUDA tensors, checks shape/dtype/device,
passes their device pointers and the current HIP stream to the C ABI of
``include/tsne355.h`` and turns a non-zero status into ``TsneError``. No
arithmetic of the method is done in Python; if the library is missing the
call fails loudly instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsne355.so")

TSNE_OK = 0
STATUS = {
    0: "TSNE_OK",
    1: "TSNE_E_ARG",
    2: "TSNE_E_PERPLEXITY",
    3: "TSNE_E_WORKSPACE",
    4: "TSNE_E_DEVICE",
    5: "TSNE_E_NONFINITE",
    6: "TSNE_E_NOCONV",
    7: "TSNE_E_STATE",
}
DIST_MODES = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3, "fp16": 4, "fp16x3": 5}

EXPORTED = [
    "tsne_workspace_bytes",
    "tsne_affinities",
    "tsne_affinities_dissim",
    "tsne_step",
    "tsne_forces",
    "tsne_update",
    "tsne_gradient",
    "tsne_cost",
    "tsne_sync_status",
    "tsne_last_error",
    "tsne_export_rowstats",
    "tsne_export_scalars",
    "tsne_export_p_rows",
    "tsne_export_order",
    "tsne_batch_workspace_bytes",
    "tsne_batch_plan",
    "tsne_batch_step",
    "tsne_batch_cost",
    "tsne_mlp_param_count",
    "tsne_mlp_workspace_bytes",
    "tsne_mlp_forward",
    "tsne_mlp_forward_noalloc",
    "tsne_mlp_gradient",
    "tsne_mlp_adam",
    "tsne_pt_workspace_bytes",
    "tsne_pt_iterations",
    "tsne_pt_init",
    "tsne_pt_epoch",
    "tsne_pt_sync_status",
    "tsne_pt_last_error",
    "tsne_pt_partial",
    "tsne_kde_workspace_bytes",
    "tsne_kde_bandwidths",
    "tsne_kde_raster",
    "tsne_workspace_bytes_implicit",
    "tsne_step_implicit",
    "tsne_gradient_implicit",
    "tsne_cost_implicit",
]


class TsneError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class AffOpts(ctypes.Structure):
    _fields_ = [("dist_mode", ctypes.c_int32), ("max_bisect", ctypes.c_int32),
                ("tol_h", ctypes.c_double), ("reorder", ctypes.c_int32),
                ("implicit_p", ctypes.c_int32)]


class BatchProblem(ctypes.Structure):
    _fields_ = [("ws", ctypes.c_void_p), ("n", ctypes.c_int64), ("y", ctypes.c_void_p),
                ("u", ctypes.c_void_p), ("g", ctypes.c_void_p)]


class StepParams(ctypes.Structure):
    _fields_ = [("exaggeration", ctypes.c_float), ("momentum", ctypes.c_float),
                ("learning_rate", ctypes.c_float), ("min_gain", ctypes.c_float),
                ("recentre", ctypes.c_int32), ("lr_rule", ctypes.c_int32)]


class Raster(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_float), ("y0", ctypes.c_float), ("cx", ctypes.c_float),
                ("cy", ctypes.c_float), ("gx", ctypes.c_int32), ("gy", ctypes.c_int32)]


class PtOpts(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("layers", ctypes.c_int32),
                ("perplexity", ctypes.c_double), ("momentum", ctypes.c_float),
                ("iters", ctypes.c_int32), ("dist_mode", ctypes.c_int32),
                ("reorder", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with `python -m paper_1812_09869_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    sigs = {
        "tsne_workspace_bytes": (ctypes.c_size_t, [_i64, _i32, _i32]),
        "tsne_affinities": (ctypes.c_int, [_vp, _i64, _i32, ctypes.c_double,
                                           ctypes.POINTER(AffOpts), _vp, ctypes.c_size_t, _vp]),
        "tsne_affinities_dissim": (ctypes.c_int, [_vp, _i64, ctypes.c_double,
                                                  ctypes.POINTER(AffOpts), _vp, ctypes.c_size_t,
                                                  _vp]),
        "tsne_step": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, ctypes.POINTER(StepParams), _vp,
                                     _vp, _vp]),
        "tsne_forces": (ctypes.c_int, [_vp, _i64, _vp, _vp]),
        "tsne_update": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, ctypes.POINTER(StepParams), _vp,
                                       _vp, _vp]),
        "tsne_gradient": (ctypes.c_int, [_vp, _i64, _vp, ctypes.c_float, _vp, _vp, _vp]),
        "tsne_cost": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp]),
        "tsne_sync_status": (ctypes.c_int, [_vp, _vp]),
        "tsne_last_error": (ctypes.c_char_p, []),
        "tsne_export_rowstats": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
        "tsne_export_scalars": (ctypes.c_int, [_vp, _i64, _vp, _vp]),
        "tsne_export_p_rows": (ctypes.c_int, [_vp, _i64, _i64, _i64, _vp, _vp]),
        "tsne_export_order": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp]),
        "tsne_batch_workspace_bytes": (ctypes.c_size_t, [_i32]),
        "tsne_batch_plan": (ctypes.c_int, [ctypes.POINTER(BatchProblem), _i32, _vp,
                                           ctypes.c_size_t, _vp]),
        "tsne_batch_step": (ctypes.c_int, [ctypes.POINTER(BatchProblem), _i32, _vp,
                                           ctypes.POINTER(StepParams), _vp]),
        "tsne_batch_cost": (ctypes.c_int, [ctypes.POINTER(BatchProblem), _i32, _vp, _vp, _vp]),
        "tsne_mlp_param_count": (ctypes.c_int64, [_i32, _i32]),
        "tsne_mlp_workspace_bytes": (ctypes.c_size_t, [_i32, _i32, _i64, _i32]),
        "tsne_mlp_forward": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _vp, _i64, _vp, _vp,
                                            ctypes.c_size_t, _vp]),
        "tsne_mlp_forward_noalloc": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _vp, _i64, _vp,
                                                     _vp]),
        "tsne_mlp_gradient": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _i64, _vp,
                                             _vp, _vp, ctypes.c_size_t, _vp]),
        "tsne_mlp_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_float, _i32, _vp]),
        "tsne_pt_workspace_bytes": (ctypes.c_size_t, [_i64, _i32, ctypes.POINTER(PtOpts)]),
        "tsne_pt_iterations": (_i32, [_i64, ctypes.POINTER(PtOpts)]),
        "tsne_pt_init": (ctypes.c_int, [_i64, _i32, ctypes.POINTER(PtOpts), _vp, ctypes.c_size_t,
                                        _vp]),
        "tsne_pt_epoch": (ctypes.c_int, [_vp, _i64, _i32, ctypes.POINTER(PtOpts), _vp, _vp, _vp,
                                         ctypes.c_size_t, _vp, _vp]),
        "tsne_pt_sync_status": (ctypes.c_int, [_i64, _i32, ctypes.POINTER(PtOpts), _vp,
                                               ctypes.c_size_t, _vp]),
        "tsne_pt_last_error": (ctypes.c_char_p, []),
        "tsne_kde_workspace_bytes": (ctypes.c_size_t, [_i64]),
        "tsne_workspace_bytes_implicit": (ctypes.c_size_t, [_i64, _i32, _i32]),
        "tsne_step_implicit": (ctypes.c_int, [_vp, _i64, _i32, _i32, _vp, _vp, _vp,
                                              ctypes.POINTER(StepParams), _vp, _vp, _vp]),
        "tsne_gradient_implicit": (ctypes.c_int, [_vp, _i64, _i32, _i32, _vp, ctypes.c_float,
                                                  _vp, _vp, _vp]),
        "tsne_cost_implicit": (ctypes.c_int, [_vp, _i64, _i32, _i32, _vp, _vp, _vp]),
        "tsne_kde_bandwidths": (ctypes.c_int, [_vp, _i64, ctypes.c_double, _vp, _vp,
                                               ctypes.c_size_t, _vp]),
        "tsne_kde_raster": (ctypes.c_int, [_vp, _i64, _vp, ctypes.POINTER(Raster), _vp, _vp]),
        "tsne_pt_partial": (ctypes.c_int, [_i64, _i32, ctypes.POINTER(PtOpts), _vp,
                                           ctypes.c_size_t, _i32, ctypes.POINTER(_vp),
                                           ctypes.POINTER(_i64)]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != TSNE_OK:
        raise TsneError(rc, load().tsne_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=torch.float32, shape=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def workspace_bytes(n: int, d: int, dist_mode: str | int = "fp64") -> int:
    mode = DIST_MODES[dist_mode] if isinstance(dist_mode, str) else int(dist_mode)
    return int(load().tsne_workspace_bytes(n, d, mode))


def new_workspace(n: int, d: int, dist_mode: str | int = "fp64", device="cuda") -> torch.Tensor:
    nbytes = workspace_bytes(n, d, dist_mode)
    if nbytes == 0:
        raise TsneError(1, f"no workspace size for n={n}, d={d}, mode={dist_mode}")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def affinities(x: torch.Tensor, perplexity: float, ws: torch.Tensor, dist_mode="fp64",
               max_bisect: int = 200, tol_h: float = 1e-6, reorder: bool = True,
               implicit: bool = False):
    n, d = x.shape
    mode = DIST_MODES[dist_mode] if isinstance(dist_mode, str) else int(dist_mode)
    opts = AffOpts(mode, max_bisect, tol_h, 1 if reorder else 0, 1 if implicit else 0)
    _check(load().tsne_affinities(_ptr(x, name="x"), n, d, float(perplexity),
                                  ctypes.byref(opts), _ptr(ws, torch.uint8, name="ws"),
                                  ws.numel(), _stream()))


LR_RULES = {"gains": 0, "range": 1}


def _params(exaggeration, momentum, learning_rate, min_gain, recentre, lr_rule):
    rule = LR_RULES[lr_rule] if isinstance(lr_rule, str) else int(lr_rule)
    return StepParams(exaggeration, momentum, learning_rate, min_gain, 1 if recentre else 0, rule)


def affinities_dissim(dis: torch.Tensor, perplexity: float, ws: torch.Tensor,
                      max_bisect: int = 200, tol_h: float = 1e-6):
    """Affinities from an n x n dissimilarity matrix (its square enters Eq. 1)."""
    n = dis.shape[0]
    opts = AffOpts(DIST_MODES["fp64"], max_bisect, tol_h, 0, 0)
    _check(load().tsne_affinities_dissim(_ptr(dis, shape=(n, n), name="dis"), n,
                                         float(perplexity), ctypes.byref(opts),
                                         _ptr(ws, torch.uint8, name="ws"), ws.numel(), _stream()))


def step(ws, n, y, u, g, exaggeration, momentum, learning_rate, min_gain=0.01, recentre=True,
         grad_out=None, z_out=None, lr_rule="gains"):
    """One iteration. lr_rule "gains": fixed rate with adaptive gains; "range":
    the rate of Eq. 11 from the map's extent, no gains (g may be None)."""
    prm = _params(exaggeration, momentum, learning_rate, min_gain, recentre, lr_rule)
    sh = (n, 2)
    _check(load().tsne_step(_ptr(ws, torch.uint8, name="ws"), n, _ptr(y, shape=sh, name="y"),
                            _ptr(u, shape=sh, name="u"), _ptr(g, shape=sh, name="g"),
                            ctypes.byref(prm), _ptr(grad_out, shape=sh, name="grad_out"),
                            _ptr(z_out, torch.float64, name="z_out"), _stream()))


def forces(ws, n, y):
    _check(load().tsne_forces(_ptr(ws, torch.uint8, name="ws"), n, _ptr(y, shape=(n, 2), name="y"),
                              _stream()))


def update(ws, n, y, u, g, exaggeration, momentum, learning_rate, min_gain=0.01, recentre=True,
           grad_out=None, z_out=None, lr_rule="gains"):
    prm = _params(exaggeration, momentum, learning_rate, min_gain, recentre, lr_rule)
    sh = (n, 2)
    _check(load().tsne_update(_ptr(ws, torch.uint8, name="ws"), n, _ptr(y, shape=sh, name="y"),
                              _ptr(u, shape=sh, name="u"), _ptr(g, shape=sh, name="g"),
                              ctypes.byref(prm), _ptr(grad_out, shape=sh, name="grad_out"),
                              _ptr(z_out, torch.float64, name="z_out"), _stream()))


def gradient(ws, n, y, alpha, grad_out, z_out=None):
    sh = (n, 2)
    _check(load().tsne_gradient(_ptr(ws, torch.uint8, name="ws"), n, _ptr(y, shape=sh, name="y"),
                                float(alpha), _ptr(grad_out, shape=sh, name="grad_out"),
                                _ptr(z_out, torch.float64, name="z_out"), _stream()))


def cost(ws, n, y, out):
    _check(load().tsne_cost(_ptr(ws, torch.uint8, name="ws"), n, _ptr(y, shape=(n, 2), name="y"),
                            _ptr(out, torch.float64, shape=(2,), name="out"), _stream()))


def sync_status(ws) -> int:
    """Synchronise and return the device status code (0 = OK), without raising."""
    return int(load().tsne_sync_status(_ptr(ws, torch.uint8, name="ws"), _stream()))


def check_status(ws):
    _check(sync_status(ws))


def export_rowstats(ws, n):
    dev = ws.device
    beta = torch.empty(n, dtype=torch.float64, device=dev)
    m = torch.empty(n, dtype=torch.float32, device=dev)
    S = torch.empty(n, dtype=torch.float64, device=dev)
    H = torch.empty(n, dtype=torch.float64, device=dev)
    ev = torch.empty(n, dtype=torch.int32, device=dev)
    _check(load().tsne_export_rowstats(_ptr(ws, torch.uint8, name="ws"), n,
                                       _ptr(beta, torch.float64), _ptr(m), _ptr(S, torch.float64),
                                       _ptr(H, torch.float64), _ptr(ev, torch.int32), _stream()))
    return beta, m, S, H, ev


def export_scalars(ws, n):
    """(sum P, sum p ln p, Z of the last force pass, perplexity) as Python floats."""
    out = torch.empty(4, dtype=torch.float64, device=ws.device)
    _check(load().tsne_export_scalars(_ptr(ws, torch.uint8, name="ws"), n,
                                      _ptr(out, torch.float64), _stream()))
    return tuple(float(v) for v in out.cpu())


def export_p_rows(ws, n, row0, nrows):
    out = torch.empty((nrows, n), dtype=torch.float32, device=ws.device)
    _check(load().tsne_export_p_rows(_ptr(ws, torch.uint8, name="ws"), n, row0, nrows, _ptr(out),
                                     _stream()))
    return out


def export_order(ws, n):
    """(perm, tile_flags): internal position -> caller index, and one byte per upper tile."""
    nb = (n + 255) // 256
    perm = torch.empty(n, dtype=torch.int32, device=ws.device)
    flags = torch.empty(nb * (nb + 1) // 2, dtype=torch.uint8, device=ws.device)
    _check(load().tsne_export_order(_ptr(ws, torch.uint8, name="ws"), n, _ptr(perm, torch.int32),
                                    _ptr(flags, torch.uint8), _stream()))
    return perm, flags


# --------------------------------------------------------------------------
# Surrogate network
# --------------------------------------------------------------------------

def mlp_param_count(d_in: int, hidden: int) -> int:
    return int(load().tsne_mlp_param_count(d_in, hidden))


def mlp_new_workspace(d_in: int, hidden: int, batch: int, train: bool, device="cuda"):
    nbytes = int(load().tsne_mlp_workspace_bytes(d_in, hidden, batch, 1 if train else 0))
    if nbytes == 0:
        raise TsneError(1, f"no surrogate workspace for d_in={d_in}, hidden={hidden}")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def mlp_forward(params, d_in, hidden, mean, invstd, x, out, ws):
    n = x.shape[0]
    _check(load().tsne_mlp_forward(_ptr(params, name="params"), d_in, hidden, _ptr(mean),
                                   _ptr(invstd), _ptr(x, shape=(n, d_in), name="x"), n,
                                   _ptr(out, shape=(n, 2), name="out"),
                                   _ptr(ws, torch.uint8, name="ws"), ws.numel(), _stream()))


def mlp_forward_noalloc(params, d_in, hidden, mean, invstd, x, out):
    """tsne_mlp_forward without a workspace (the library's device scratch)."""
    n = x.shape[0]
    _check(load().tsne_mlp_forward_noalloc(_ptr(params, name="params"), d_in, hidden, _ptr(mean),
                                           _ptr(invstd), _ptr(x, shape=(n, d_in), name="x"), n,
                                           _ptr(out, shape=(n, 2), name="out"), _stream()))


def mlp_gradient(params, d_in, hidden, mean, invstd, x, y, idx, batch, grad, loss, ws):
    _check(load().tsne_mlp_gradient(_ptr(params, name="params"), d_in, hidden, _ptr(mean),
                                    _ptr(invstd), _ptr(x, name="x"), _ptr(y, name="y"),
                                    _ptr(idx, torch.int32, name="idx"), batch,
                                    _ptr(grad, name="grad"), _ptr(loss, torch.float64, name="loss"),
                                    _ptr(ws, torch.uint8, name="ws"), ws.numel(), _stream()))


def mlp_adam(params, grad, m, v, lr, beta1, beta2, eps, t):
    _check(load().tsne_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), lr,
                                beta1, beta2, eps, int(t), _stream()))


# --------------------------------------------------------------------------
# Batched iteration
# --------------------------------------------------------------------------

def batch_problems(entries):
    """ctypes array of (ws, n, y, u, g) tuples of torch tensors."""
    arr = (BatchProblem * len(entries))()
    for k, (ws, n, y, u, g) in enumerate(entries):
        sh = (n, 2)
        arr[k] = BatchProblem(_ptr(ws, torch.uint8, name="ws").value, n,
                              _ptr(y, shape=sh, name="y").value, _ptr(u, shape=sh, name="u").value,
                              _ptr(g, shape=sh, name="g").value)
    return arr


def batch_plan(arr, device="cuda"):
    count = len(arr)
    nbytes = int(load().tsne_batch_workspace_bytes(count))
    bws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    _check(load().tsne_batch_plan(arr, count, _ptr(bws, torch.uint8), nbytes, _stream()))
    return bws


def batch_cost(arr, bws, out):
    """{KL, C_norm} of every problem (out: float64 device tensor of 2 x count)."""
    _check(load().tsne_batch_cost(arr, len(arr), _ptr(bws, torch.uint8),
                                  _ptr(out, torch.float64, shape=(len(arr), 2), name="out"),
                                  _stream()))


def batch_step(arr, bws, exaggeration, momentum, learning_rate, min_gain=0.01, recentre=True,
               lr_rule="gains"):
    prm = _params(exaggeration, momentum, learning_rate, min_gain, recentre, lr_rule)
    _check(load().tsne_batch_step(arr, len(arr), _ptr(bws, torch.uint8), ctypes.byref(prm),
                                  _stream()))


# --------------------------------------------------------------------------
# Parallel scheme (ptSNE)
# --------------------------------------------------------------------------

def _check_pt(rc: int):
    if rc != TSNE_OK:
        raise TsneError(rc, load().tsne_pt_last_error().decode())


def pt_opts(threads, layers, perplexity, momentum=0.8, iters=0, dist_mode="fp64",
            reorder=False) -> PtOpts:
    mode = DIST_MODES[dist_mode] if isinstance(dist_mode, str) else int(dist_mode)
    return PtOpts(int(threads), int(layers), float(perplexity), float(momentum), int(iters), mode,
                  1 if reorder else 0, 0)


def pt_iterations(n: int, opts: PtOpts) -> int:
    return int(load().tsne_pt_iterations(n, ctypes.byref(opts)))


def pt_new_workspace(n: int, d: int, opts: PtOpts, device="cuda") -> torch.Tensor:
    nbytes = int(load().tsne_pt_workspace_bytes(n, d, ctypes.byref(opts)))
    if nbytes == 0:
        _check_pt(load().tsne_pt_init(n, d, ctypes.byref(opts), None, 0, None))
        raise TsneError(1, "invalid ptSNE options")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def pt_init(n: int, d: int, opts: PtOpts, ws: torch.Tensor):
    _check_pt(load().tsne_pt_init(n, d, ctypes.byref(opts), _ptr(ws, torch.uint8, name="ws"),
                                  ws.numel(), _stream()))


def pt_epoch(x, opts: PtOpts, order, maps, ws, monitors=None):
    n, d = x.shape
    _check_pt(load().tsne_pt_epoch(_ptr(x, name="x"), n, d, ctypes.byref(opts),
                                   _ptr(order, torch.int32, shape=(n,), name="order"),
                                   _ptr(maps, shape=(opts.layers, n, 2), name="maps"),
                                   _ptr(ws, torch.uint8, name="ws"), ws.numel(),
                                   _ptr(monitors, torch.float64, shape=(2,), name="monitors"),
                                   _stream()))


def pt_sync_status(n: int, d: int, opts: PtOpts, ws) -> int:
    return int(load().tsne_pt_sync_status(n, d, ctypes.byref(opts),
                                          _ptr(ws, torch.uint8, name="ws"), ws.numel(),
                                          _stream()))


def pt_partial(n: int, d: int, opts: PtOpts, ws, k: int):
    """(workspace view, n_k) of partial problem k (a uint8 tensor over its bytes)."""
    ptr, nk = _vp(), _i64()
    _check_pt(load().tsne_pt_partial(n, d, ctypes.byref(opts), _ptr(ws, torch.uint8, name="ws"),
                                     ws.numel(), k, ctypes.byref(ptr), ctypes.byref(nk)))
    off = ptr.value - ws.data_ptr()
    return ws[off:off + workspace_bytes(nk.value, d, opts.dist_mode)], nk.value


# --------------------------------------------------------------------------
# Perplexity-adaptive KDE of a map (paKDE)
# --------------------------------------------------------------------------

def kde_new_workspace(n: int, device="cuda") -> torch.Tensor:
    nbytes = int(load().tsne_kde_workspace_bytes(n))
    if nbytes == 0:
        raise TsneError(1, f"no KDE workspace size for n={n}")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def kde_bandwidths(y, perplexity: float, ws, beta):
    n = y.shape[0]
    _check(load().tsne_kde_bandwidths(_ptr(y, shape=(n, 2), name="y"), n, float(perplexity),
                                      _ptr(beta, torch.float64, shape=(n,), name="beta"),
                                      _ptr(ws, torch.uint8, name="ws"), ws.numel(), _stream()))


def kde_raster(y, beta, x0, y0, cx, cy, gx, gy, out):
    n = y.shape[0]
    g = Raster(float(x0), float(y0), float(cx), float(cy), int(gx), int(gy))
    _check(load().tsne_kde_raster(_ptr(y, shape=(n, 2), name="y"), n,
                                  _ptr(beta, torch.float64, shape=(n,), name="beta"),
                                  ctypes.byref(g), _ptr(out, shape=(gy, gx), name="out"),
                                  _stream()))


# --------------------------------------------------------------------------
# Implicit P (recomputed in every pass)
# --------------------------------------------------------------------------

def _mode(dist_mode) -> int:
    return DIST_MODES[dist_mode] if isinstance(dist_mode, str) else int(dist_mode)


def workspace_bytes_implicit(n: int, d: int, dist_mode: str | int = "fp64") -> int:
    return int(load().tsne_workspace_bytes_implicit(n, d, _mode(dist_mode)))


def new_workspace_implicit(n: int, d: int, device="cuda", dist_mode: str | int = "fp64"):
    nbytes = workspace_bytes_implicit(n, d, dist_mode)
    if nbytes == 0:
        raise TsneError(1, f"no implicit workspace size for n={n}, d={d}, mode={dist_mode}")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def step_implicit(ws, n, d, y, u, g, exaggeration, momentum, learning_rate, min_gain=0.01,
                  recentre=True, grad_out=None, z_out=None, lr_rule="gains", dist_mode="fp64"):
    prm = _params(exaggeration, momentum, learning_rate, min_gain, recentre, lr_rule)
    sh = (n, 2)
    _check(load().tsne_step_implicit(_ptr(ws, torch.uint8, name="ws"), n, d, _mode(dist_mode),
                                     _ptr(y, shape=sh, name="y"), _ptr(u, shape=sh, name="u"),
                                     _ptr(g, shape=sh, name="g"), ctypes.byref(prm),
                                     _ptr(grad_out, shape=sh, name="grad_out"),
                                     _ptr(z_out, torch.float64, name="z_out"), _stream()))


def gradient_implicit(ws, n, d, y, alpha, grad_out, z_out=None, dist_mode="fp64"):
    sh = (n, 2)
    _check(load().tsne_gradient_implicit(_ptr(ws, torch.uint8, name="ws"), n, d,
                                         _mode(dist_mode),
                                         _ptr(y, shape=sh, name="y"), float(alpha),
                                         _ptr(grad_out, shape=sh, name="grad_out"),
                                         _ptr(z_out, torch.float64, name="z_out"), _stream()))


def cost_implicit(ws, n, d, y, out, dist_mode="fp64"):
    _check(load().tsne_cost_implicit(_ptr(ws, torch.uint8, name="ws"), n, d, _mode(dist_mode),
                                     _ptr(y, shape=(n, 2), name="y"),
                                     _ptr(out, torch.float64, shape=(2,), name="out"), _stream()))
