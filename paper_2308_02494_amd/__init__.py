"""Python binding of libapmg: the MI355X hot path of the adaptively placed
multi-grid scene representation network (APMGSRN).

Every entry point of include/apmg.h has a function of the same name here
that only marshals arguments (torch tensors -> device pointers, the current
stream); all arithmetic runs in the library's HIP kernels.  The library must
have been built (paper_2308_02494_amd.build); importing this module raises if
it is missing.  `APMGFunction` and `DensityLossFunction` expose the forward
pass, its hand-written adjoint and the feature-density loss to autograd.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libapmg.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2308_02494_amd.build")
_lib = ctypes.CDLL(LIB_PATH)

# ----------------------------------------------------------------------------- ABI mirror
OK, EINVAL, EUNSUPPORTED, EWORKSPACE, EHIP = 0, -1, -2, -3, -4
F32, F16, BF16 = 0, 1, 2
ACCUMULATE, DETERMINISTIC, ADD_REC_DG, ERR_ABS = 0x1, 0x2, 0x4, 0x8
DENSITY_ABS_DET, DENSITY_NORM_TARGET = 0x10, 0x20
GRIDS_MCRRR, GRIDS_MRRRC = 0, 1
OP_FORWARD, OP_BACKWARD, OP_DENSITY, OP_BATCHED_STEP, OP_DD_FORWARD = 0, 1, 2, 3, 4
ENC_HASH, ENC_TIME = 1, 2
PROF_ADJOINT, PROF_GATHER = 0, 1
MAX_LAYERS = 8

c_i32, c_i64, c_u32, c_u64, c_f32, c_f64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                              ctypes.c_uint64, ctypes.c_float, ctypes.c_double)
c_p = ctypes.c_void_p


class ApmgModel(ctypes.Structure):
    _fields_ = [("M", c_i32), ("C", c_i32), ("R", c_i32), ("n_layers", c_i32),
                ("width", c_i32 * (MAX_LAYERS + 1)), ("grid_dtype", c_i32), ("mlp_dtype", c_i32),
                ("G", c_p), ("F", c_p), ("W", c_p * MAX_LAYERS), ("vmin", c_f32), ("vmax", c_f32),
                ("grid_layout", c_i32), ("G_rows", c_i32)]


class ApmgEncoder(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("levels", c_i32), ("table_log2", c_i32), ("level_res", c_i32 * 8),
                ("Rt", c_i32)]


class ApmgBrick(ctypes.Structure):
    _fields_ = [("ijk", c_i32 * 3), ("e0", c_i32 * 3), ("e1", c_i32 * 3), ("vmin", c_f32), ("vmax", c_f32)]


class ApmgBrickTable(ctypes.Structure):
    _fields_ = [("dims", c_i32 * 3), ("vol", c_i32 * 3), ("B", c_i32), ("ghost", c_i32)]


class ApmgTuning(ctypes.Structure):
    _fields_ = [("tile_blocks", c_i32), ("cell_unroll", c_i32), ("cell_kernel", c_i32), ("cell_group", c_i32),
                ("adjoint_kernel", c_i32), ("reserved", c_i32 * 3)]


class ApmgBatch(ctypes.Structure):
    _fields_ = [("nb", c_i32), ("shape", ApmgModel), ("G", c_p), ("F", c_p), ("W", c_p),
                ("mG", c_p), ("vG", c_p), ("mF", c_p), ("vF", c_p), ("mW", c_p), ("vW", c_p),
                ("t", c_p), ("tG", c_p), ("density_active", c_p), ("volume", c_p), ("bricks", c_p),
                ("vol", c_i32 * 3), ("n", c_i64), ("seed", c_u64), ("step", c_p),
                ("lr", c_f32), ("lr_G", c_f32), ("beta1", c_f32), ("beta2", c_f32), ("adam_eps", c_f32),
                ("eps_density", c_f64), ("p", c_i32), ("flags", c_u32), ("losses", c_p),
                ("tuning", ctypes.POINTER(ApmgTuning)), ("frozen", c_p), ("lr_scale", c_p), ("stream0", c_u32)]


class ApmgDdModels(ctypes.Structure):
    _fields_ = [("nb", c_i32), ("shape", ApmgModel), ("G", c_p), ("F", c_p), ("W", c_p), ("bricks", c_p)]


class ApmgCtlState(ctypes.Structure):
    _fields_ = [("iter", c_i32), ("density_done", c_i32), ("ma_count", c_i32), ("have_prev", c_i32),
                ("bad", c_i32), ("reductions", c_i32), ("ma_sum", c_f64), ("ma_prev", c_f64), ("best", c_f64)]


class ApmgControl(ctypes.Structure):
    _fields_ = [("nb", c_i32), ("delay", c_i32), ("total_iters", c_i32), ("ma_window", c_i32),
                ("patience", c_i32), ("max_reductions", c_i32), ("stop_frac", c_f32), ("plateau_factor", c_f32),
                ("ma_rel", c_f64), ("plateau_rel", c_f64), ("state", c_p), ("density_active", c_p),
                ("frozen", c_p), ("lr_scale", c_p)]


_sigs = {
    "apmg_forward": [ctypes.POINTER(ApmgModel), c_p, c_i64, c_i64, c_p, c_p, ctypes.c_size_t, c_p],
    "apmg_forward_noalloc": [ctypes.POINTER(ApmgModel), c_p, c_i64, c_i64, c_p, c_p],
    "apmg_forward_noalloc_scratch_bytes": [],
    "apmg_backward": [ctypes.POINTER(ApmgModel), c_p, c_i64, c_i64, c_p, c_p, c_p, c_p, c_u32, c_p,
                      ctypes.c_size_t, c_p],
    "apmg_density_loss": [ctypes.POINTER(ApmgModel), c_p, c_i64, c_i64, c_p, c_f64, c_i32, c_p, c_p, c_p,
                          c_u32, c_p, ctypes.c_size_t, c_p],
    "apmg_make_bricks": [c_i32, c_i32, c_i32, c_i32, c_i32, ctypes.POINTER(ApmgBrickTable),
                         ctypes.POINTER(ApmgBrick), c_i32],
    "apmg_assign_bricks": [ctypes.POINTER(ApmgBrickTable), c_p, c_i64, c_i64, c_p, c_p],
    "apmg_batched_step": [ctypes.POINTER(ApmgBatch), c_p, ctypes.c_size_t, c_p],
    "apmg_workspace_bytes": [ctypes.c_int, c_p, c_i64],
    "apmg_status_string": [ctypes.c_int],
    "apmg_convert_grids": [c_i32, c_i32, c_i32, c_p, c_i32, c_p, c_i32, c_i32, c_p],
    "apmg_cells": [ctypes.POINTER(ApmgModel), c_p, c_i64, c_i64, c_p, c_p, c_p],
    "apmg_uniform_points": [c_u64, c_u64, c_u32, c_i64, c_i64, c_p, c_i64, c_p],
    "apmg_gt_sample": [c_p, c_i32, c_i32, c_i32, c_p, c_i64, c_i64, c_p, c_p],
    "apmg_profile_events": [c_p, c_p],
    "apmg_profile_kernel_events": [c_i32, c_p, c_p],
    "apmg_autotune_batched_step": [ctypes.POINTER(ApmgBatch), c_p, ctypes.c_size_t, c_p,
                                   ctypes.POINTER(ApmgTuning), ctypes.POINTER(c_f32)],
    "apmg_train_control": [ctypes.POINTER(ApmgControl), c_p, c_p],
    "apmg_variant_workspace_bytes": [ctypes.c_int, ctypes.POINTER(ApmgModel), ctypes.POINTER(ApmgEncoder), c_i64],
    "apmg_variant_forward": [ctypes.POINTER(ApmgModel), ctypes.POINTER(ApmgEncoder), c_p, c_i64, c_i64, c_p, c_p,
                             ctypes.c_size_t, c_p],
    "apmg_variant_backward": [ctypes.POINTER(ApmgModel), ctypes.POINTER(ApmgEncoder), c_p, c_i64, c_i64, c_p, c_p,
                              c_p, c_p, c_u32, c_p, ctypes.c_size_t, c_p],
    "apmg_dd_forward": [ctypes.POINTER(ApmgDdModels), ctypes.POINTER(ApmgBrickTable), c_p, c_i64, c_i64, c_p, c_p,
                        ctypes.c_size_t, c_p],
}
for _name, _args in _sigs.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = ctypes.c_int
_lib.apmg_workspace_bytes.restype = ctypes.c_size_t
_lib.apmg_variant_workspace_bytes.restype = ctypes.c_size_t
_lib.apmg_forward_noalloc_scratch_bytes.restype = ctypes.c_size_t
_lib.apmg_status_string.restype = ctypes.c_char_p

EXPORTS = tuple(_sigs)


class ApmgError(RuntimeError):
    def __init__(self, name, code):
        super().__init__(f"{name}: {status_string(code)} ({code})")
        self.code = code


def status_string(code):
    return _lib.apmg_status_string(code).decode()


def _check(name, code):
    if code != OK:
        raise ApmgError(name, code)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


# ----------------------------------------------------------------------------- model
class Model:
    """Device tensors of one APMGSRN as the paper states the model (Sec. 4.1).

    G [M,3,4] or [M,4,4] float32 (the transforms of Eq. (1); row 3 of a 4x4 is
    not read), F [M,C,R,R,R] float32 or float16 (the encoder tensor, axes z, y,
    x), W = [W1 [H,M*C], W2 [H,H], W3 [1,H]] float32, vmin/vmax floats;
    mlp_dtype F32 or BF16.  layout=GRIDS_MRRRC says F is channel-last
    [M,R,R,R,C] instead (the order the kernels gather from).
    """

    def __init__(self, G, F, W, vmin=0.0, vmax=1.0, mlp_dtype=F32, layout=GRIDS_MCRRR):
        self.G, self.F, self.W = G, F, list(W)
        self.vmin, self.vmax = float(vmin), float(vmax)
        self.mlp_dtype = mlp_dtype
        self.layout = layout

    @property
    def M(self):
        return self.F.shape[0]

    @property
    def C(self):
        return self.F.shape[1] if self.layout == GRIDS_MCRRR else self.F.shape[4]

    @property
    def R(self):
        return self.F.shape[2] if self.layout == GRIDS_MCRRR else self.F.shape[1]

    def struct(self):
        m = ApmgModel()
        m.M, m.R, m.C = self.M, self.R, self.C
        m.n_layers = len(self.W)
        m.width[0] = self.W[0].shape[1]
        for k, w in enumerate(self.W):
            m.width[k + 1] = w.shape[0]
        m.grid_dtype = F16 if self.F.dtype == torch.float16 else F32
        m.mlp_dtype = self.mlp_dtype
        m.G = self.G.data_ptr()
        m.F = self.F.data_ptr()
        for k, w in enumerate(self.W):
            m.W[k] = w.data_ptr()
        m.vmin, m.vmax = self.vmin, self.vmax
        m.grid_layout = self.layout
        m.G_rows = self.G.shape[1]
        return m

    @staticmethod
    def from_host(params, device="cuda", grid_dtype=torch.float32, mlp_dtype=F32):
        """params: dict with G [M,3,4] or [M,4,4], F [M,C,R,R,R] (the paper's order), W list,
        vmin, vmax (numpy or torch), copied to the device as they are."""
        G = torch.as_tensor(params["G"], dtype=torch.float32).contiguous().to(device)
        F = torch.as_tensor(params["F"]).contiguous().to(device=device, dtype=grid_dtype)
        W = [torch.as_tensor(w, dtype=torch.float32).contiguous().to(device) for w in params["W"]]
        return Model(G, F, W, float(params.get("vmin", 0.0)), float(params.get("vmax", 1.0)), mlp_dtype)


def _soa(pts):
    """[N,3] -> contiguous SoA [3,N] float32 on the same device."""
    return pts.t().contiguous().to(torch.float32)


def _workspace(op, obj, n, device):
    nbytes = _lib.apmg_workspace_bytes(op, ctypes.byref(obj), n)
    if nbytes == 0:
        raise ApmgError("apmg_workspace_bytes", EINVAL)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


# ----------------------------------------------------------------------------- entry points
def apmg_forward(model: Model, pts_soa, n=None, ld=None, out=None, ws=None):
    """f[n] for points pts_soa [3, ld] (float32 SoA on the model's device)."""
    n = pts_soa.shape[1] if n is None else n
    ld = pts_soa.shape[1] if ld is None else ld
    dev = model.G.device
    m = model.struct()
    f = torch.empty(n, dtype=torch.float32, device=dev) if out is None else out
    ws = _workspace(OP_FORWARD, m, n, dev) if ws is None else ws
    _check("apmg_forward", _lib.apmg_forward(ctypes.byref(m), _ptr(pts_soa), ld, n, _ptr(f), _ptr(ws),
                                             ws.numel(), _stream(dev)))
    return f


def apmg_forward_noalloc(model: Model, pts_soa, n=None, ld=None, out=None):
    """apmg_forward without a workspace (the library's static per-device scratch); f[n]."""
    n = pts_soa.shape[1] if n is None else n
    ld = pts_soa.shape[1] if ld is None else ld
    dev = model.G.device
    m = model.struct()
    f = torch.empty(n, dtype=torch.float32, device=dev) if out is None else out
    _check("apmg_forward_noalloc", _lib.apmg_forward_noalloc(ctypes.byref(m), _ptr(pts_soa), ld, n, _ptr(f),
                                                             _stream(dev)))
    return f


def apmg_backward(model: Model, pts_soa, df, want_dF=True, want_dG=True, want_dW=True, flags=0,
                  n=None, ld=None, dF=None, dG=None, dW=None, ws=None):
    """Gradients of sum_n df[n] f(x_n): (dF f32 in F's shape and layout, dG f64 in G's shape,
    [dW1, dW2, dW3])."""
    n = pts_soa.shape[1] if n is None else n
    ld = pts_soa.shape[1] if ld is None else ld
    dev = model.G.device
    m = model.struct()
    if want_dF and dF is None:
        dF = torch.empty(model.F.shape, dtype=torch.float32, device=dev)
    if want_dG and dG is None:
        dG = torch.empty(tuple(model.G.shape), dtype=torch.float64, device=dev)
    if want_dW and dW is None:
        dW = [torch.empty_like(w) for w in model.W]
    dw_arr = None
    if want_dW:
        dw_arr = (ctypes.c_void_p * len(dW))(*[w.data_ptr() for w in dW])
    ws = _workspace(OP_BACKWARD, m, n, dev) if ws is None else ws
    _check("apmg_backward", _lib.apmg_backward(
        ctypes.byref(m), _ptr(pts_soa), ld, n, _ptr(df), _ptr(dF) if want_dF else None,
        _ptr(dG) if want_dG else None, ctypes.cast(dw_arr, c_p) if want_dW else None, flags, _ptr(ws),
        ws.numel(), _stream(dev)))
    return (dF if want_dF else None), (dG if want_dG else None), (dW if want_dW else None)


class VariantModel:
    """Device tensors of an APMGSRN with one of the encoder variants of Sec. 9.

    kind ENC_HASH: G [M,3,4] or [M,4,4], F = hash tables [M, L, T, C] float32 (T = 2^k),
    level_res = the L per-level cell counts.  kind ENC_TIME: F = 4-D grids [M, C, Rt, R, R, R]
    (layout GRIDS_MCRRR) or [M, Rt, R, R, R, C] (GRIDS_MRRRC), float32; the points then carry
    the time as a fourth row.  W, vmin, vmax, mlp_dtype as Model."""

    def __init__(self, kind, G, F, W, vmin=0.0, vmax=1.0, mlp_dtype=F32, level_res=None, layout=GRIDS_MCRRR):
        self.kind, self.G, self.F, self.W = kind, G, F, list(W)
        self.vmin, self.vmax, self.mlp_dtype, self.layout = float(vmin), float(vmax), mlp_dtype, layout
        self.level_res = list(level_res) if level_res is not None else []

    def structs(self):
        m = ApmgModel()
        e = ApmgEncoder()
        e.kind = self.kind
        m.M = self.F.shape[0]
        if self.kind == ENC_HASH:
            _, L, T, C = self.F.shape
            e.levels, e.table_log2 = L, int(T).bit_length() - 1
            for k, r in enumerate(self.level_res):
                e.level_res[k] = int(r)
            m.C, m.R = C, 2
        else:
            if self.layout == GRIDS_MCRRR:
                _, C, Rt, R = self.F.shape[:4]
            else:
                _, Rt, R = self.F.shape[:3]
                C = self.F.shape[5]
            e.Rt = Rt
            m.C, m.R = C, R
        m.n_layers = len(self.W)
        m.width[0] = self.W[0].shape[1]
        for k, w in enumerate(self.W):
            m.width[k + 1] = w.shape[0]
        m.grid_dtype, m.mlp_dtype = F32, self.mlp_dtype
        m.G, m.F = self.G.data_ptr(), self.F.data_ptr()
        for k, w in enumerate(self.W):
            m.W[k] = w.data_ptr()
        m.vmin, m.vmax = self.vmin, self.vmax
        m.grid_layout = self.layout
        m.G_rows = self.G.shape[1]
        return m, e


def _variant_ws(op, m, e, n, device):
    nbytes = _lib.apmg_variant_workspace_bytes(op, ctypes.byref(m), ctypes.byref(e), n)
    if nbytes == 0:
        raise ApmgError("apmg_variant_workspace_bytes", EINVAL)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def apmg_variant_forward(model: VariantModel, pts_soa, out=None, ws=None):
    """f[n] for points pts_soa [3 or 4, n] (the time row for ENC_TIME)."""
    n = pts_soa.shape[1]
    dev = model.G.device
    m, e = model.structs()
    f = torch.empty(n, dtype=torch.float32, device=dev) if out is None else out
    ws = _variant_ws(OP_FORWARD, m, e, n, dev) if ws is None else ws
    _check("apmg_variant_forward", _lib.apmg_variant_forward(ctypes.byref(m), ctypes.byref(e), _ptr(pts_soa), n, n,
                                                             _ptr(f), _ptr(ws), ws.numel(), _stream(dev)))
    return f


def apmg_variant_backward(model: VariantModel, pts_soa, df, want_dF=True, want_dG=True, want_dW=True, flags=0,
                          ws=None):
    """Gradients of sum_n df[n] f(x_n): (dF f32 in F's shape, dG f64 in G's shape, [dW1, dW2, dW3])."""
    n = pts_soa.shape[1]
    dev = model.G.device
    m, e = model.structs()
    dF = torch.empty(model.F.shape, dtype=torch.float32, device=dev) if want_dF else None
    dG = torch.empty(tuple(model.G.shape), dtype=torch.float64, device=dev) if want_dG else None
    dW = [torch.empty_like(w) for w in model.W] if want_dW else None
    dw_arr = (ctypes.c_void_p * len(dW))(*[w.data_ptr() for w in dW]) if want_dW else None
    ws = _variant_ws(OP_BACKWARD, m, e, n, dev) if ws is None else ws
    _check("apmg_variant_backward", _lib.apmg_variant_backward(
        ctypes.byref(m), ctypes.byref(e), _ptr(pts_soa), n, n, _ptr(df), _ptr(dF) if want_dF else None,
        _ptr(dG) if want_dG else None, ctypes.cast(dw_arr, c_p) if want_dW else None, flags, _ptr(ws), ws.numel(),
        _stream(dev)))
    return dF, dG, dW


def apmg_density_loss(model: Model, pts_soa, err, eps=1e-12, p=10, want_dG=True, want_rho=False, flags=0,
                      n=None, ld=None, ws=None):
    """(loss [1] f64, dG f64 in G's shape or None, rho [n] f32 or None).  flags: ACCUMULATE,
    DENSITY_ABS_DET, DENSITY_NORM_TARGET."""
    n = pts_soa.shape[1] if n is None else n
    ld = pts_soa.shape[1] if ld is None else ld
    dev = model.G.device
    m = model.struct()
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    dG = torch.zeros(tuple(model.G.shape), dtype=torch.float64, device=dev) if want_dG else None
    rho = torch.empty(max(n, 1), dtype=torch.float32, device=dev) if want_rho else None
    ws = _workspace(OP_DENSITY, m, n, dev) if ws is None else ws
    _check("apmg_density_loss", _lib.apmg_density_loss(
        ctypes.byref(m), _ptr(pts_soa), ld, n, _ptr(err), eps, p, _ptr(loss), _ptr(dG), _ptr(rho), flags,
        _ptr(ws), ws.numel(), _stream(dev)))
    return loss, dG, (rho[:n] if want_rho else None)


def apmg_cells(model: Model, pts_soa):
    """(cell [n, M, 3] int32, inside [n, M] uint8)."""
    n = pts_soa.shape[1]
    dev = model.G.device
    m = model.struct()
    cell = torch.empty((n, model.M, 3), dtype=torch.int32, device=dev)
    inside = torch.empty((n, model.M), dtype=torch.uint8, device=dev)
    _check("apmg_cells", _lib.apmg_cells(ctypes.byref(m), _ptr(pts_soa), n, n, _ptr(cell), _ptr(inside),
                                         _stream(dev)))
    return cell, inside


def apmg_uniform_points(seed, step, stream_id, start, n, device="cuda"):
    pts = torch.empty((3, max(n, 1)), dtype=torch.float32, device=device)
    _check("apmg_uniform_points", _lib.apmg_uniform_points(seed, step, stream_id, start, n, _ptr(pts),
                                                           max(n, 1), _stream(torch.device(device))))
    return pts[:, :n]


def apmg_gt_sample(volume, pts_soa):
    nz, ny, nx = volume.shape
    n = pts_soa.shape[1]
    v = torch.empty(max(n, 1), dtype=torch.float32, device=volume.device)
    _check("apmg_gt_sample", _lib.apmg_gt_sample(_ptr(volume), nx, ny, nz, _ptr(pts_soa), n, n, _ptr(v),
                                                 _stream(volume.device)))
    return v[:n]


def apmg_make_bricks(nx, ny, nz, B, ghost):
    """Host-only: (table, list of ApmgBrick)."""
    t = ApmgBrickTable()
    _check("apmg_make_bricks", _lib.apmg_make_bricks(nx, ny, nz, B, ghost, ctypes.byref(t), None, 0))
    nb = t.dims[0] * t.dims[1] * t.dims[2]
    arr = (ApmgBrick * nb)()
    _check("apmg_make_bricks", _lib.apmg_make_bricks(nx, ny, nz, B, ghost, ctypes.byref(t), arr, nb))
    return t, list(arr)


def apmg_assign_bricks(table, pts_soa):
    n = pts_soa.shape[1]
    out = torch.empty(max(n, 1), dtype=torch.int32, device=pts_soa.device)
    _check("apmg_assign_bricks", _lib.apmg_assign_bricks(ctypes.byref(table), _ptr(pts_soa), n, n, _ptr(out),
                                                         _stream(pts_soa.device)))
    return out[:n]


def apmg_convert_grids(src, to_channel_last, dst_dtype=None):
    """[M,C,R,R,R] <-> [M,R,R,R,C]; float32/float16."""
    dst_dtype = src.dtype if dst_dtype is None else dst_dtype
    if to_channel_last:
        M, C, R = src.shape[0], src.shape[1], src.shape[2]
        dst = torch.empty((M, R, R, R, C), dtype=dst_dtype, device=src.device)
    else:
        M, R, C = src.shape[0], src.shape[1], src.shape[4]
        dst = torch.empty((M, C, R, R, R), dtype=dst_dtype, device=src.device)
    code = {torch.float32: F32, torch.float16: F16}
    _check("apmg_convert_grids", _lib.apmg_convert_grids(M, C, R, _ptr(src), code[src.dtype], _ptr(dst),
                                                         code[dst_dtype], 1 if to_channel_last else 0,
                                                         _stream(src.device)))
    return dst


def brick_tensor(bricks, device):
    """Device array of apmg_brick structs from a list of ApmgBrick."""
    raw = bytes((ApmgBrick * len(bricks))(*bricks))
    return torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)


# ----------------------------------------------------------------------------- training step
class Trainer:
    """Parameters, Adam state and counters of nb brick models, stepped by
    apmg_batched_step.  Parameters are arenas: G [nb,M,3,4], F [nb,M,C,R,R,R]
    (float32 masters in the paper's order; with grid_dtype float16 the encoder
    gathers from an F16 copy the step makes), W [nb, sum of layer sizes] (W1, W2,
    W3 concatenated).  flags: ADD_REC_DG, ERR_ABS, DENSITY_ABS_DET,
    DENSITY_NORM_TARGET."""

    def __init__(self, models_host, volume, bricks, n, seed=7, mlp_dtype=F32, grid_dtype=torch.float32,
                 lr=0.01, lr_G=0.001, betas=(0.9, 0.99), adam_eps=1e-8, eps_density=1e-12, p=10, flags=0,
                 device="cuda", control=None, tuning=None, stream0=0):
        nb = len(models_host)
        assert nb == len(bricks)
        dev = torch.device(device)
        self.device = dev
        # the step's transform arena is [nb,M,3,4] (rows 0..2 of each matrix)
        G = torch.stack([torch.as_tensor(mh["G"], dtype=torch.float32)[:, :3, :] for mh in models_host])
        F = torch.stack([torch.as_tensor(mh["F"], dtype=torch.float32) for mh in models_host])
        W = torch.stack([torch.cat([torch.as_tensor(w, dtype=torch.float32).reshape(-1) for w in mh["W"]])
                         for mh in models_host])
        self.G, self.F, self.W = G.contiguous().to(dev), F.contiguous().to(dev), W.contiguous().to(dev)
        self.grid_dtype = grid_dtype
        z = torch.zeros_like
        self.mG, self.vG, self.mF, self.vF = z(self.G), z(self.G), z(self.F), z(self.F)
        self.mW, self.vW = z(self.W), z(self.W)
        self.t = torch.zeros(nb, dtype=torch.int32, device=dev)
        self.tG = torch.zeros(nb, dtype=torch.int32, device=dev)
        self.density_active = torch.zeros(nb, dtype=torch.int32, device=dev)
        self.step_ctr = torch.zeros(1, dtype=torch.int64, device=dev)
        self.losses = torch.zeros((nb, 2), dtype=torch.float64, device=dev)
        self.volume = volume
        self.bricks_dev = brick_tensor(bricks, dev)
        self.widths = [models_host[0]["W"][0].shape[1]] + [w.shape[0] for w in models_host[0]["W"]]
        M, C, R = F.shape[1], F.shape[2], F.shape[3]
        b = ApmgBatch()
        b.nb = nb
        s = b.shape
        s.M, s.C, s.R, s.n_layers = M, C, R, len(self.widths) - 1
        for k, wd in enumerate(self.widths):
            s.width[k] = wd
        s.grid_dtype = F16 if grid_dtype == torch.float16 else F32
        s.mlp_dtype = mlp_dtype
        b.G, b.F, b.W = self.G.data_ptr(), self.F.data_ptr(), self.W.data_ptr()
        b.mG, b.vG, b.mF, b.vF = self.mG.data_ptr(), self.vG.data_ptr(), self.mF.data_ptr(), self.vF.data_ptr()
        b.mW, b.vW = self.mW.data_ptr(), self.vW.data_ptr()
        b.t, b.tG = self.t.data_ptr(), self.tG.data_ptr()
        b.density_active = self.density_active.data_ptr()
        b.volume = volume.data_ptr()
        b.bricks = self.bricks_dev.data_ptr()
        nz, ny, nx = volume.shape
        b.vol[0], b.vol[1], b.vol[2] = nx, ny, nz
        b.n = n
        b.seed = seed
        b.step = self.step_ctr.data_ptr()
        b.lr, b.lr_G, b.beta1, b.beta2, b.adam_eps = lr, lr_G, betas[0], betas[1], adam_eps
        b.eps_density, b.p, b.flags = eps_density, p, flags
        b.losses = self.losses.data_ptr()
        self.frozen = torch.zeros(nb, dtype=torch.int32, device=dev)
        self.lr_scale = torch.ones(nb, dtype=torch.float32, device=dev)
        b.frozen = self.frozen.data_ptr()
        b.lr_scale = self.lr_scale.data_ptr()
        b.stream0 = stream0
        self.tuning = None
        self.batch = b
        if tuning is not None:
            self.set_tuning(tuning)
        self.ws = _workspace(OP_BATCHED_STEP, b, n, dev)
        self.control = None
        if control is not None:
            self.enable_control(**control)

    def set_tuning(self, tuning):
        """Launch shapes for the step: an ApmgTuning, a dict (tile_blocks, cell_unroll, cell_kernel,
        cell_group) or None."""
        if isinstance(tuning, dict):
            t = ApmgTuning()
            t.tile_blocks = tuning.get("tile_blocks", 0)
            t.cell_unroll = tuning.get("cell_unroll", 0)
            t.cell_kernel = tuning.get("cell_kernel", 0)
            t.cell_group = tuning.get("cell_group", 0)
            t.adjoint_kernel = tuning.get("adjoint_kernel", 0)
            tuning = t
        self.tuning = tuning
        self.batch.tuning = ctypes.pointer(tuning) if tuning is not None else None

    def autotune(self):
        """Runs apmg_autotune_batched_step (synchronising; parameters unchanged) and adopts
        the fastest launch shapes.  Returns (tuning dict, ms per step)."""
        best = ApmgTuning()
        ms = c_f32()
        _check("apmg_autotune_batched_step",
               _lib.apmg_autotune_batched_step(ctypes.byref(self.batch), _ptr(self.ws), self.ws.numel(),
                                              _stream(self.device), ctypes.byref(best), ctypes.byref(ms)))
        self.set_tuning(best)
        return {"tile_blocks": best.tile_blocks, "cell_unroll": best.cell_unroll,
                "cell_kernel": best.cell_kernel, "cell_group": best.cell_group,
                "adjoint_kernel": best.adjoint_kernel}, ms.value

    def enable_control(self, total_iters, delay=500, ma_window=1000, ma_rel=1e-4, stop_frac=0.8, patience=500,
                       plateau_rel=1e-4, plateau_factor=0.1, max_reductions=3):
        """On-device training schedule (apmg_train_control) applied after every step: delayed
        start of the transforms, their early stop, and the plateau scheduler that retires
        models.  Defaults are the paper's values."""
        nb = self.batch.nb
        self.ctl_state = torch.zeros((nb, ctypes.sizeof(ApmgCtlState)), dtype=torch.uint8, device=self.device)
        self.density_active.fill_(1 if delay == 0 else 0)
        self.frozen.zero_()
        self.lr_scale.fill_(1.0)
        c = ApmgControl()
        c.nb, c.delay, c.total_iters, c.ma_window = nb, delay, total_iters, ma_window
        c.patience, c.max_reductions, c.stop_frac, c.plateau_factor = patience, max_reductions, stop_frac, plateau_factor
        c.ma_rel, c.plateau_rel = ma_rel, plateau_rel
        c.state = self.ctl_state.data_ptr()
        c.density_active = self.density_active.data_ptr()
        c.frozen = self.frozen.data_ptr()
        c.lr_scale = self.lr_scale.data_ptr()
        self.control = c

    def control_state(self):
        """Per-model control state as a list of dicts (copies to the host)."""
        raw = self.ctl_state.cpu().numpy()
        out = []
        for row in raw:
            st = ApmgCtlState.from_buffer_copy(row.tobytes())
            out.append({k: getattr(st, k) for k, _ in ApmgCtlState._fields_})
        return out

    def step(self):
        st = _stream(self.device)
        _check("apmg_batched_step", _lib.apmg_batched_step(ctypes.byref(self.batch), _ptr(self.ws),
                                                           self.ws.numel(), st))
        if self.control is not None:
            _check("apmg_train_control", _lib.apmg_train_control(ctypes.byref(self.control),
                                                                 self.losses.data_ptr(), st))


class DDModels:
    """The brick models of a domain decomposition for global-query inference
    (apmg_dd_forward): arenas G [nb,M,3,4] or [nb,M,4,4], F [nb,M,C,R,R,R] (float32
    or float16; [nb,M,R,R,R,C] with layout=GRIDS_MRRRC), W [nb, layers concatenated],
    the brick table and the device brick records."""

    def __init__(self, G, F, W, widths, table, bricks, mlp_dtype=F32, layout=GRIDS_MCRRR):
        self.G, self.F, self.W = G.contiguous(), F.contiguous(), W.contiguous()
        self.table, self.bricks_dev = table, brick_tensor(bricks, G.device)
        d = ApmgDdModels()
        d.nb = G.shape[0]
        sh = d.shape
        C, R = (F.shape[2], F.shape[3]) if layout == GRIDS_MCRRR else (F.shape[5], F.shape[2])
        sh.M, sh.C, sh.R, sh.n_layers = G.shape[1], C, R, len(widths) - 1
        for k, wd in enumerate(widths):
            sh.width[k] = wd
        sh.grid_dtype = F16 if F.dtype == torch.float16 else F32
        sh.mlp_dtype = mlp_dtype
        sh.grid_layout = layout
        sh.G_rows = G.shape[2]
        d.G, d.F, d.W, d.bricks = self.G.data_ptr(), self.F.data_ptr(), self.W.data_ptr(), self.bricks_dev.data_ptr()
        self.struct = d

    @classmethod
    def from_trainer(cls, tr, table, bricks):
        """The trainer's models as they were trained: with F16 gathers, the grids are given to
        inference as their F16 copy (apmg_convert_grids, channel-last)."""
        if tr.grid_dtype == torch.float16:
            nb, M, C, R = tr.F.shape[0], tr.F.shape[1], tr.F.shape[2], tr.F.shape[3]
            Fh = apmg_convert_grids(tr.F.view(nb * M, C, R, R, R), True, torch.float16)
            return cls(tr.G, Fh.view(nb, M, R, R, R, C), tr.W, tr.widths, table, bricks, tr.batch.shape.mlp_dtype,
                       GRIDS_MRRRC)
        return cls(tr.G, tr.F, tr.W, tr.widths, table, bricks, tr.batch.shape.mlp_dtype)


def apmg_dd_forward(models, pts_soa, out=None, ws=None):
    """f at global points pts_soa [3, n] over all bricks of `models` (a DDModels)."""
    n = pts_soa.shape[1]
    dev = pts_soa.device
    f = out if out is not None else torch.empty(max(n, 1), dtype=torch.float32, device=dev)[:n]
    if ws is None:
        ws = _workspace(OP_DD_FORWARD, models.struct, n, dev)
    _check("apmg_dd_forward", _lib.apmg_dd_forward(ctypes.byref(models.struct), ctypes.byref(models.table),
                                                   _ptr(pts_soa), pts_soa.stride(0), n, _ptr(f), _ptr(ws),
                                                   ws.numel(), _stream(dev)))
    return f


def train_control(control, losses):
    """apmg_train_control on an ApmgControl and a [nb, 2] float64 device tensor of losses."""
    _check("apmg_train_control", _lib.apmg_train_control(ctypes.byref(control), losses.data_ptr(),
                                                         _stream(losses.device)))


# ----------------------------------------------------------------------------- autograd
class APMGFunction(torch.autograd.Function):
    """f = APMGSRN(pts) with the library's forward and hand-written adjoint.

    apply(pts [N,3], G [M,3,4] or [M,4,4], F [M,C,R,R,R], W1, W2, W3, vmin, vmax, mlp_dtype)
    Returns f [N].  Gradients for G (cast from float64, G's shape, row 3 of a 4x4 zero), F
    (the paper's order, cast to F's dtype), W1..W3; none for pts.
    """

    @staticmethod
    def forward(ctx, pts, G, F, W1, W2, W3, vmin, vmax, mlp_dtype):
        model = Model(G.contiguous(), F.contiguous(), [W1.contiguous(), W2.contiguous(), W3.contiguous()],
                      vmin, vmax, mlp_dtype)
        soa = _soa(pts)
        ctx.save_for_backward(soa, G, F, W1, W2, W3)
        ctx.meta = (vmin, vmax, mlp_dtype)
        return apmg_forward(model, soa)

    @staticmethod
    def backward(ctx, grad_f):
        soa, G, F, W1, W2, W3 = ctx.saved_tensors
        vmin, vmax, mlp_dtype = ctx.meta
        model = Model(G.contiguous(), F.contiguous(), [W1.contiguous(), W2.contiguous(), W3.contiguous()],
                      vmin, vmax, mlp_dtype)
        dF, dG, dW = apmg_backward(model, soa, grad_f.contiguous().to(torch.float32),
                                   want_dF=ctx.needs_input_grad[2], want_dG=ctx.needs_input_grad[1],
                                   want_dW=any(ctx.needs_input_grad[3:6]))
        dG = dG.to(G.dtype) if dG is not None else None
        dF = dF.to(F.dtype) if dF is not None else None
        if dW is None:
            dW = [None, None, None]
        return None, dG, dF, dW[0], dW[1], dW[2], None, None, None


class DensityLossFunction(torch.autograd.Function):
    """L_density(G) for points pts [N,3] and per-point error err [N] (Eqs. (7)-(9)),
    with the target density held constant; gradient for G only ([M,3,4] or [M,4,4]).
    flags: DENSITY_ABS_DET, DENSITY_NORM_TARGET (alternative readings)."""

    @staticmethod
    def forward(ctx, pts, G, err, eps, p, flags=0):
        M = G.shape[0]
        dummyF = torch.empty((M, 1, 2, 2, 2), dtype=torch.float32, device=G.device)
        model = Model(G.contiguous(), dummyF, [torch.empty((64, M), device=G.device),
                                                torch.empty((64, 64), device=G.device),
                                                torch.empty((1, 64), device=G.device)])
        loss, dG, _ = apmg_density_loss(model, _soa(pts), err.contiguous().to(torch.float32), eps, p,
                                        want_dG=G.requires_grad, flags=flags)
        ctx.save_for_backward(dG if dG is not None else torch.empty(0))
        return loss.to(G.dtype)[0]

    @staticmethod
    def backward(ctx, g):
        (dG,) = ctx.saved_tensors
        return None, (g * dG).to(torch.float32), None, None, None, None


def apmg_profile_events(start, stop):
    """Arm the adjoint-kernel timing hook with two hipEvent_t handles (ints), or clear it."""
    _check("apmg_profile_events", _lib.apmg_profile_events(start, stop))


def apmg_profile_kernel_events(kernel, start, stop):
    """Arm the timing hook of one kernel kind (PROF_ADJOINT or PROF_GATHER) with two
    hipEvent_t handles, or clear it."""
    _check("apmg_profile_kernel_events", _lib.apmg_profile_kernel_events(kernel, start, stop))
