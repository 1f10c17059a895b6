"""Python binding of libmf4d (include/mf4d.h): argument marshalling only.

Every step of the filter runs in the HIP library; this module checks tensor
shapes, dtypes and devices, passes raw device pointers and the current HIP
stream through ctypes, and turns non-zero status codes into exceptions.
PyTorch provides device memory and streams. There is no CPU fallback: if the
library has not been built, loading it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # imported first so that libmf4d binds to torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmf4d.so")

MF4D_OK, MF4D_EINVAL, MF4D_ENOMEM, MF4D_EHIP = 0, -1, -2, -3
MF4D_ENONFINITE, MF4D_EUNSTABLE = -4, -5
MF4D_RIDGE, MF4D_VALLEY, MF4D_BOTH = 0, 1, 2
MF4D_MAFOD, MF4D_IFOD = 0, 1
MF4D_MAX_SCALES, MF4D_MAX_RADIUS, MF4D_MAX_SUBSTEPS = 16, 64, 1024

# every symbol include/mf4d.h declares
EXPORTS = ["mf4d_status_string", "mf4d_params_default", "mf4d_fed_schedule",
           "mf4d_fed_substeps", "mf4d_fed_plan", "mf4d_workspace_bytes",
           "mf4d_scale_select", "mf4d_tensor", "mf4d_fed_cycle", "mf4d_fed_cycle_tensor",
           "mf4d_filter", "mf4d_filter_noalloc", "mf4d_noalloc_max_bytes", "mf4d_filter_l2stop",
           "mf4d_creases_workspace_bytes", "mf4d_creases", "mf4d_crease_match", "mf4d_batch_create", "mf4d_batch_workspace_bytes", "mf4d_filter_batch",
           "mf4d_batch_autotune", "mf4d_batch_get_tuning", "mf4d_batch_set_tuning", "mf4d_batch_destroy",
           "mf4d_net_param_count", "mf4d_net_workspace_bytes", "mf4d_net_forward", "mf4d_net_backward",
           "mf4d_net_step", "mf4d_learned_workspace_bytes", "mf4d_filter_learned",
           "mf4d3d_workspace_bytes", "mf4d3d_scale_select", "mf4d3d_tensor", "mf4d3d_dtensor",
           "mf4d3d_fed_cycle_tensor", "mf4d3d_filter"]


class MF4DError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class mf4d_params(ctypes.Structure):
    _fields_ = [
        ("nscales", ctypes.c_int),
        ("sigmas", ctypes.POINTER(ctypes.c_float)),
        ("mode", ctypes.c_int),
        ("lambda_", ctypes.c_float),
        ("rho", ctypes.c_float),
        ("beta", ctypes.c_float),
        ("c", ctypes.c_float),
        ("cycles", ctypes.c_int),
        ("substeps", ctypes.c_int),
        ("stop_time", ctypes.c_double),
        ("tau_max", ctypes.c_double),
        ("reselect_each_cycle", ctypes.c_int),
        ("theta", ctypes.c_float),
        ("postprocess", ctypes.c_int),
        ("check", ctypes.c_int),
        ("model", ctypes.c_int),
    ]


class Params:
    """Filter parameters (paper notation); owns the host sigma array."""

    def __init__(self, sigmas, mode=MF4D_BOTH, lam=0.005, rho=0.5, beta=0.5, c=-1.0,
                 cycles=1, substeps=10, stop_time=0.0, tau_max=0.05, reselect_each_cycle=1,
                 theta=0.0, postprocess=0, check=0, model=MF4D_MAFOD):
        self.sigmas = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float32))
        self.mode, self.lam, self.rho, self.beta, self.c = mode, lam, rho, beta, c
        self.cycles, self.substeps, self.stop_time, self.tau_max = cycles, substeps, stop_time, tau_max
        self.reselect_each_cycle, self.theta, self.postprocess = reselect_each_cycle, theta, postprocess
        self.check, self.model = check, model

    @classmethod
    def from_workload(cls, w, **kw):
        d = dict(mode=w.mode, lam=w.lam, rho=w.rho, beta=w.beta, cycles=w.cycles,
                 substeps=w.substeps, tau_max=w.tau_max)
        d.update(kw)
        return cls(w.sigmas, **d)

    def struct(self) -> mf4d_params:
        p = mf4d_params()
        p.nscales = len(self.sigmas)
        p.sigmas = self.sigmas.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        p.mode = int(self.mode)
        p.lambda_ = float(self.lam)
        p.rho = float(self.rho)
        p.beta = float(self.beta)
        p.c = float(self.c)
        p.cycles = int(self.cycles)
        p.substeps = int(self.substeps)
        p.stop_time = float(self.stop_time)
        p.tau_max = float(self.tau_max)
        p.reselect_each_cycle = int(self.reselect_each_cycle)
        p.theta = float(self.theta)
        p.postprocess = int(self.postprocess)
        p.check = int(self.check)
        p.model = int(self.model)
        return p


_lib = None


def lib():
    """Load libmf4d.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp, sz, i, d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
        L.mf4d_status_string.argtypes = [i]
        L.mf4d_status_string.restype = ctypes.c_char_p
        L.mf4d_params_default.argtypes = [P(mf4d_params), i, P(ctypes.c_float)]
        L.mf4d_params_default.restype = i
        L.mf4d_fed_schedule.argtypes = [i, d, P(d), P(i)]
        L.mf4d_fed_schedule.restype = i
        L.mf4d_fed_substeps.argtypes = [d, i, d]
        L.mf4d_fed_substeps.restype = i
        L.mf4d_fed_plan.argtypes = [P(mf4d_params), P(i), P(d)]
        L.mf4d_fed_plan.restype = i
        L.mf4d_workspace_bytes.argtypes = [i, i, P(mf4d_params)]
        L.mf4d_workspace_bytes.restype = sz
        L.mf4d_scale_select.argtypes = [vp, i, i, P(mf4d_params), vp, vp, vp, vp, sz, vp]
        L.mf4d_scale_select.restype = i
        L.mf4d_tensor.argtypes = [vp, i, i, vp, P(mf4d_params), vp, vp, vp, sz, vp]
        L.mf4d_tensor.restype = i
        L.mf4d_fed_cycle.argtypes = [vp, vp, i, i, vp, P(mf4d_params), P(d), i, vp]
        L.mf4d_fed_cycle.restype = i
        L.mf4d_fed_cycle_tensor.argtypes = [vp, vp, i, i, vp, P(d), i, i, vp]
        L.mf4d_fed_cycle_tensor.restype = i
        L.mf4d_filter.argtypes = [vp, vp, i, i, P(mf4d_params), vp, sz, vp]
        L.mf4d_filter.restype = i
        L.mf4d_filter_noalloc.argtypes = [vp, vp, i, i, P(mf4d_params), vp]
        L.mf4d_filter_noalloc.restype = i
        L.mf4d_noalloc_max_bytes.argtypes = []
        L.mf4d_noalloc_max_bytes.restype = sz
        L.mf4d_filter_l2stop.argtypes = [vp, vp, i, i, P(mf4d_params), vp, vp, vp, vp, sz, vp]
        L.mf4d_filter_l2stop.restype = i
        L.mf4d_creases_workspace_bytes.argtypes = [i, i]
        L.mf4d_creases_workspace_bytes.restype = sz
        L.mf4d_creases.argtypes = [vp, i, i, ctypes.c_float, ctypes.c_float, i, vp, vp, vp, vp, vp, sz, vp]
        L.mf4d_creases.restype = i
        L.mf4d_crease_match.argtypes = [vp, vp, i, i, vp, vp, i, ctypes.c_float, vp, vp, vp]
        L.mf4d_crease_match.restype = i
        L.mf4d_batch_create.argtypes = [i, P(ctypes.c_int64), P(i), P(i), P(mf4d_params), P(vp)]
        L.mf4d_batch_create.restype = i
        L.mf4d_batch_workspace_bytes.argtypes = [vp]
        L.mf4d_batch_workspace_bytes.restype = sz
        L.mf4d_filter_batch.argtypes = [vp, vp, vp, vp, sz, vp]
        L.mf4d_filter_batch.restype = i
        L.mf4d_batch_autotune.argtypes = [vp, vp, sz, vp]
        L.mf4d_batch_autotune.restype = i
        L.mf4d_batch_get_tuning.argtypes = [vp, P(i), P(i)]
        L.mf4d_batch_get_tuning.restype = i
        L.mf4d_batch_set_tuning.argtypes = [vp, i, i]
        L.mf4d_batch_set_tuning.restype = i
        L.mf4d_batch_destroy.argtypes = [vp]
        L.mf4d_batch_destroy.restype = i
        L.mf4d_net_param_count.argtypes = []
        L.mf4d_net_param_count.restype = sz
        L.mf4d_net_workspace_bytes.argtypes = [i, i, i, i]
        L.mf4d_net_workspace_bytes.restype = sz
        L.mf4d_net_forward.argtypes = [vp, vp, i, i, i, vp, vp, vp, vp, sz, vp]
        L.mf4d_net_forward.restype = i
        L.mf4d_net_backward.argtypes = [vp, vp, vp, i, i, i, ctypes.c_float, vp, vp, vp, sz, vp]
        L.mf4d_net_backward.restype = i
        L.mf4d_net_step.argtypes = [vp, vp, vp, vp, i, ctypes.c_float, vp]
        L.mf4d_net_step.restype = i
        L.mf4d_learned_workspace_bytes.argtypes = [i, i, P(mf4d_params)]
        L.mf4d_learned_workspace_bytes.restype = sz
        L.mf4d_filter_learned.argtypes = [vp, vp, i, i, P(mf4d_params), vp, ctypes.c_float, vp, vp, sz, vp]
        L.mf4d_filter_learned.restype = i
        L.mf4d3d_workspace_bytes.argtypes = [i, i, i, P(mf4d_params)]
        L.mf4d3d_workspace_bytes.restype = sz
        L.mf4d3d_scale_select.argtypes = [vp, i, i, i, P(mf4d_params), vp, vp, vp, vp, sz, vp]
        L.mf4d3d_scale_select.restype = i
        L.mf4d3d_tensor.argtypes = [vp, i, i, i, vp, P(mf4d_params), vp, vp, vp, sz, vp]
        L.mf4d3d_tensor.restype = i
        L.mf4d3d_dtensor.argtypes = [vp, i, i, i, P(mf4d_params), vp, vp]
        L.mf4d3d_dtensor.restype = i
        L.mf4d3d_fed_cycle_tensor.argtypes = [vp, vp, i, i, i, vp, P(d), i, vp]
        L.mf4d3d_fed_cycle_tensor.restype = i
        L.mf4d3d_filter.argtypes = [vp, vp, i, i, i, P(mf4d_params), vp, sz, vp]
        L.mf4d3d_filter.restype = i
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().mf4d_status_string(int(status)).decode()


def _check(st, where):
    if st != MF4D_OK:
        raise MF4DError(st, where)


def _dev(t, dtype, shape=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _hw(u):
    if u.dim() != 2:
        raise ValueError("image must be 2-D [H, W]")
    return int(u.shape[0]), int(u.shape[1])


# ------------------------------------------------------------------ host calls
def mf4d_fed_schedule(n: int, tau_max: float = 0.05):
    """Ordered FED steps of one cycle; returns (taus, perm, kappa)."""
    taus = np.zeros(max(int(n), 1))
    perm = np.zeros(max(int(n), 1), np.int32)
    k = lib().mf4d_fed_schedule(int(n), float(tau_max),
                                taus.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if k < 1:
        raise MF4DError(k, "mf4d_fed_schedule")
    return taus[:n], perm[:n], k


def mf4d_fed_substeps(stop_time: float, cycles: int, tau_max: float = 0.05) -> int:
    n = lib().mf4d_fed_substeps(float(stop_time), int(cycles), float(tau_max))
    if n < 1:
        raise MF4DError(n, "mf4d_fed_substeps")
    return n


def mf4d_fed_plan(params: Params):
    st = params.struct()
    n = ctypes.c_int(0)
    taus = np.zeros(MF4D_MAX_SUBSTEPS)
    _check(lib().mf4d_fed_plan(ctypes.byref(st), ctypes.byref(n),
                               taus.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "mf4d_fed_plan")
    return n.value, taus[:n.value].copy()


def mf4d_workspace_bytes(H: int, W: int, params: Params) -> int:
    st = params.struct()
    return int(lib().mf4d_workspace_bytes(int(H), int(W), ctypes.byref(st)))


def workspace(H: int, W: int, params: Params, device="cuda"):
    nb = mf4d_workspace_bytes(H, W, params)
    if nb == 0:
        raise MF4DError(MF4D_EINVAL, "mf4d_workspace_bytes")
    return torch.empty(nb, dtype=torch.uint8, device=device)


# ---------------------------------------------------------------- device calls
def mf4d_scale_select(u, params: Params, idx_out, vmax_out=None, c_out=None, ws=None, stream=None):
    H, W = _hw(_dev(u, torch.float32, name="u"))
    _dev(idx_out, torch.uint8, (H, W), "idx_out")
    _dev(vmax_out, torch.float32, (H, W), "vmax_out")
    _dev(c_out, torch.float32, (1,), "c_out")
    if ws is None:
        ws = workspace(H, W, params, u.device)
    _dev(ws, torch.uint8, name="ws")
    st = params.struct()
    _check(lib().mf4d_scale_select(_ptr(u), H, W, ctypes.byref(st), _ptr(idx_out), _ptr(vmax_out),
                                   _ptr(c_out), _ptr(ws), ws.numel(), _stream(stream)),
           "mf4d_scale_select")


def mf4d_tensor(u, idx, params: Params, hrho_out, dparams_out=None, ws=None, stream=None):
    H, W = _hw(_dev(u, torch.float32, name="u"))
    _dev(idx, torch.uint8, (H, W), "idx")
    _dev(hrho_out, torch.float32, (3, H, W), "hrho_out")
    _dev(dparams_out, torch.float32, (3, H, W), "dparams_out")
    if ws is None:
        ws = workspace(H, W, params, u.device)
    _dev(ws, torch.uint8, name="ws")
    st = params.struct()
    _check(lib().mf4d_tensor(_ptr(u), H, W, _ptr(idx), ctypes.byref(st), _ptr(hrho_out),
                             _ptr(dparams_out), _ptr(ws), ws.numel(), _stream(stream)), "mf4d_tensor")


def mf4d_fed_cycle(u, u_tmp, hrho, params: Params, taus, stream=None):
    H, W = _hw(_dev(u, torch.float32, name="u"))
    _dev(u_tmp, torch.float32, (H, W), "u_tmp")
    _dev(hrho, torch.float32, (3, H, W), "hrho")
    t = np.ascontiguousarray(np.asarray(taus, dtype=np.float64))
    st = params.struct()
    _check(lib().mf4d_fed_cycle(_ptr(u), _ptr(u_tmp), H, W, _ptr(hrho), ctypes.byref(st),
                                t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(t),
                                _stream(stream)), "mf4d_fed_cycle")


def mf4d_fed_cycle_tensor(u, u_tmp, dparams, taus, steps_per_launch=2, stream=None):
    H, W = _hw(_dev(u, torch.float32, name="u"))
    _dev(u_tmp, torch.float32, (H, W), "u_tmp")
    _dev(dparams, torch.float32, (3, H, W), "dparams")
    t = np.ascontiguousarray(np.asarray(taus, dtype=np.float64))
    _check(lib().mf4d_fed_cycle_tensor(_ptr(u), _ptr(u_tmp), H, W, _ptr(dparams),
                                       t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(t),
                                       int(steps_per_launch), _stream(stream)), "mf4d_fed_cycle_tensor")


def mf4d_filter(u_in, u_out, params: Params, ws=None, stream=None):
    H, W = _hw(_dev(u_in, torch.float32, name="u_in"))
    _dev(u_out, torch.float32, (H, W), "u_out")
    if ws is None:
        ws = workspace(H, W, params, u_in.device)
    _dev(ws, torch.uint8, name="ws")
    st = params.struct()
    _check(lib().mf4d_filter(_ptr(u_in), _ptr(u_out), H, W, ctypes.byref(st), _ptr(ws), ws.numel(),
                             _stream(stream)), "mf4d_filter")


def mf4d_filter_noalloc(u_in, u_out, params: Params, stream=None):
    """mf4d_filter with the library's fixed scratch array (no workspace)."""
    H, W = _hw(_dev(u_in, torch.float32, name="u_in"))
    _dev(u_out, torch.float32, (H, W), "u_out")
    st = params.struct()
    _check(lib().mf4d_filter_noalloc(_ptr(u_in), _ptr(u_out), H, W, ctypes.byref(st), _stream(stream)),
           "mf4d_filter_noalloc")


def mf4d_noalloc_max_bytes() -> int:
    return int(lib().mf4d_noalloc_max_bytes())


def mf4d_filter_l2stop(u_in, u_out, params: Params, ground_truth, l2_out=None, best_out=None, ws=None,
                       stream=None):
    """l2-optimal stopping (Sec. 4): u_out receives the cycle-end state closest
    to ground_truth; l2_out (float64 [cycles + 1]) and best_out (int32 [1])
    receive the distances and the chosen cycle."""
    H, W = _hw(_dev(u_in, torch.float32, name="u_in"))
    _dev(u_out, torch.float32, (H, W), "u_out")
    _dev(ground_truth, torch.float32, (H, W), "ground_truth")
    _dev(l2_out, torch.float64, (params.cycles + 1,), "l2_out")
    _dev(best_out, torch.int32, (1,), "best_out")
    if ws is None:
        ws = workspace(H, W, params, u_in.device)
    _dev(ws, torch.uint8, name="ws")
    st = params.struct()
    _check(lib().mf4d_filter_l2stop(_ptr(u_in), _ptr(u_out), H, W, ctypes.byref(st), _ptr(ground_truth),
                                    _ptr(l2_out), _ptr(best_out), _ptr(ws), ws.numel(), _stream(stream)),
           "mf4d_filter_l2stop")


# ------------------------------------------------------------ creases
def mf4d_creases(u, sigma_d=1.0, strength=0.0, mode=MF4D_BOTH, seg_out=None, type_out=None, count_out=None,
                 field_out=None, ws=None, stream=None):
    """Crease segments of an image (Sec. 3.6). Returns (seg [H-1][W-1][2][4]
    float32, type [H-1][W-1][2] int8) device tensors."""
    H, W = _hw(_dev(u, torch.float32, name="u"))
    if seg_out is None:
        seg_out = torch.empty((H - 1, W - 1, 2, 4), dtype=torch.float32, device=u.device)
    if type_out is None:
        type_out = torch.empty((H - 1, W - 1, 2), dtype=torch.int8, device=u.device)
    _dev(seg_out, torch.float32, (H - 1, W - 1, 2, 4), "seg_out")
    _dev(type_out, torch.int8, (H - 1, W - 1, 2), "type_out")
    _dev(count_out, torch.int32, (1,), "count_out")
    _dev(field_out, torch.float32, (6, H, W), "field_out")
    if ws is None:
        nb = int(lib().mf4d_creases_workspace_bytes(H, W))
        if nb == 0:
            raise MF4DError(MF4D_EINVAL, "mf4d_creases_workspace_bytes")
        ws = torch.empty(nb, dtype=torch.uint8, device=u.device)
    _check(lib().mf4d_creases(_ptr(u), H, W, float(sigma_d), float(strength), int(mode), _ptr(seg_out),
                              _ptr(type_out), _ptr(count_out), _ptr(field_out), _ptr(ws), ws.numel(),
                              _stream(stream)), "mf4d_creases")
    return seg_out, type_out


def mf4d_crease_match(seg, typ, gt, gt_type, radius=6.0, dist_out=None, match_out=None, stream=None):
    """Matches ground-truth segments gt [n][4] (types gt_type [n]) to the
    extracted segments (Sec. 4). Returns (dist [n] float32, match [n] int32)."""
    _dev(seg, torch.float32, name="seg")
    if seg.dim() != 4 or tuple(seg.shape[2:]) != (2, 4):
        raise ValueError("seg must be [H-1][W-1][2][4]")
    H, W = int(seg.shape[0]) + 1, int(seg.shape[1]) + 1
    _dev(typ, torch.int8, (H - 1, W - 1, 2), "type")
    n = int(gt.shape[0]) if gt.dim() == 2 else 0
    _dev(gt, torch.float32, (n, 4), "gt")
    _dev(gt_type, torch.int32, (n,), "gt_type")
    if dist_out is None:
        dist_out = torch.empty(n, dtype=torch.float32, device=seg.device)
    if match_out is None:
        match_out = torch.empty(n, dtype=torch.int32, device=seg.device)
    _check(lib().mf4d_crease_match(_ptr(seg), _ptr(typ), H, W, _ptr(gt), _ptr(gt_type), n, float(radius),
                                   _ptr(dist_out), _ptr(match_out), _stream(stream)), "mf4d_crease_match")
    return dist_out, match_out


# ------------------------------------------------------------------ batches
class Batch:
    """A batch plan (mf4d_batch_create) for images packed in one buffer.

    shapes: list of (H, W); params: list of Params (mode and cycles may
    differ). offsets default to the images packed back to back.
    """

    def __init__(self, shapes, params, offsets=None):
        self.shapes = [(int(h), int(w)) for h, w in shapes]
        if offsets is None:
            offsets = np.concatenate([[0], np.cumsum([h * w for h, w in self.shapes])[:-1]])
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.total = int(max(o + h * w for o, (h, w) in zip(self.offsets, self.shapes)))
        self._params = list(params)
        arr = (mf4d_params * len(params))(*[p.struct() for p in params])
        H = (ctypes.c_int * len(shapes))(*[h for h, _ in self.shapes])
        W = (ctypes.c_int * len(shapes))(*[w for _, w in self.shapes])
        h = ctypes.c_void_p()
        _check(lib().mf4d_batch_create(len(shapes), self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       H, W, arr, ctypes.byref(h)), "mf4d_batch_create")
        self.handle = h

    def workspace_bytes(self) -> int:
        return int(lib().mf4d_batch_workspace_bytes(self.handle))

    def workspace(self, device="cuda"):
        return torch.empty(self.workspace_bytes(), dtype=torch.uint8, device=device)

    def autotune(self, ws, stream=None):
        _dev(ws, torch.uint8, name="ws")
        _check(lib().mf4d_batch_autotune(self.handle, _ptr(ws), ws.numel(), _stream(stream)), "mf4d_batch_autotune")

    def tuning(self):
        a, b = ctypes.c_int(0), ctypes.c_int(0)
        _check(lib().mf4d_batch_get_tuning(self.handle, ctypes.byref(a), ctypes.byref(b)), "mf4d_batch_get_tuning")
        return a.value, b.value

    def set_tuning(self, substeps_per_launch, rows_per_wave=0):
        _check(lib().mf4d_batch_set_tuning(self.handle, int(substeps_per_launch), int(rows_per_wave)),
               "mf4d_batch_set_tuning")

    def filter(self, packed_in, packed_out, ws, stream=None):
        _dev(packed_in, torch.float32, name="packed_in")
        _dev(packed_out, torch.float32, name="packed_out")
        _dev(ws, torch.uint8, name="ws")
        if packed_in.numel() < self.total or packed_out.numel() < self.total:
            raise ValueError("packed buffers are smaller than the plan's layout")
        _check(lib().mf4d_filter_batch(self.handle, _ptr(packed_in), _ptr(packed_out), _ptr(ws), ws.numel(),
                                       _stream(stream)), "mf4d_filter_batch")

    def close(self):
        if getattr(self, "handle", None):
            lib().mf4d_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ learned net
def mf4d_net_param_count() -> int:
    return int(lib().mf4d_net_param_count())


def net_workspace(B, H, W, train, device="cuda"):
    nb = int(lib().mf4d_net_workspace_bytes(int(B), int(H), int(W), int(bool(train))))
    if nb == 0:
        raise MF4DError(MF4D_EINVAL, "mf4d_net_workspace_bytes")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def _bhw(u):
    if u.dim() == 2:
        return 1, int(u.shape[0]), int(u.shape[1])
    if u.dim() == 3:
        return int(u.shape[0]), int(u.shape[1]), int(u.shape[2])
    raise ValueError("images must be [H, W] or [B, H, W]")


def mf4d_net_forward(theta, u, logits=None, idx_out=None, conf_out=None, ws=None, stream=None):
    _dev(theta, torch.float32, (mf4d_net_param_count(),), "theta")
    B, H, W = _bhw(_dev(u, torch.float32, name="u"))
    _dev(logits, torch.float32, (B * H * W, 16), "logits")
    _dev(idx_out, torch.uint8, tuple(u.shape), "idx_out")
    _dev(conf_out, torch.float32, tuple(u.shape), "conf_out")
    if ws is None:
        ws = net_workspace(B, H, W, False, u.device)
    _check(lib().mf4d_net_forward(_ptr(theta), _ptr(u), B, H, W, _ptr(logits), _ptr(idx_out), _ptr(conf_out),
                                  _ptr(ws), ws.numel(), _stream(stream)), "mf4d_net_forward")


def mf4d_net_backward(theta, u, labels, grad, w_conf=0.1, stats_out=None, ws=None, stream=None):
    _dev(theta, torch.float32, (mf4d_net_param_count(),), "theta")
    B, H, W = _bhw(_dev(u, torch.float32, name="u"))
    _dev(labels, torch.uint8, tuple(u.shape), "labels")
    _dev(grad, torch.float32, (mf4d_net_param_count(),), "grad")
    _dev(stats_out, torch.float32, (2,), "stats_out")
    if ws is None:
        ws = net_workspace(B, H, W, True, u.device)
    _check(lib().mf4d_net_backward(_ptr(theta), _ptr(u), _ptr(labels), B, H, W, float(w_conf), _ptr(grad),
                                   _ptr(stats_out), _ptr(ws), ws.numel(), _stream(stream)), "mf4d_net_backward")


def mf4d_net_step(theta, grad, adam_m, adam_v, step, lr, stream=None):
    n = mf4d_net_param_count()
    for t, nm in ((theta, "theta"), (grad, "grad"), (adam_m, "adam_m"), (adam_v, "adam_v")):
        _dev(t, torch.float32, (n,), nm)
    _check(lib().mf4d_net_step(_ptr(theta), _ptr(grad), _ptr(adam_m), _ptr(adam_v), int(step), float(lr),
                               _stream(stream)), "mf4d_net_step")


def mf4d_filter_learned(u_in, u_out, params: Params, theta, conf_threshold=0.9, fallback_count=None, ws=None,
                        stream=None):
    H, W = _hw(_dev(u_in, torch.float32, name="u_in"))
    _dev(u_out, torch.float32, (H, W), "u_out")
    _dev(theta, torch.float32, (mf4d_net_param_count(),), "theta")
    _dev(fallback_count, torch.int32, (1,), "fallback_count")
    st = params.struct()
    if ws is None:
        nb = int(lib().mf4d_learned_workspace_bytes(H, W, ctypes.byref(st)))
        if nb == 0:
            raise MF4DError(MF4D_EINVAL, "mf4d_learned_workspace_bytes")
        ws = torch.empty(nb, dtype=torch.uint8, device=u_in.device)
    _check(lib().mf4d_filter_learned(_ptr(u_in), _ptr(u_out), H, W, ctypes.byref(st), _ptr(theta),
                                     float(conf_threshold), _ptr(fallback_count), _ptr(ws), ws.numel(),
                                     _stream(stream)), "mf4d_filter_learned")


def learned_workspace(H, W, params: Params, device="cuda"):
    st = params.struct()
    nb = int(lib().mf4d_learned_workspace_bytes(int(H), int(W), ctypes.byref(st)))
    if nb == 0:
        raise MF4DError(MF4D_EINVAL, "mf4d_learned_workspace_bytes")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def net_init(seed=0, device="cuda"):
    """He-normal initial parameters (host RNG), as a device tensor."""
    rng = np.random.default_rng(seed)
    ch = (1, 32, 32, 32, 32, 9)
    parts = []
    for l in range(5):
        fan_in = ch[l] * 9
        parts.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), size=ch[l + 1] * ch[l] * 9))
        parts.append(np.zeros(ch[l + 1]))
    return torch.from_numpy(np.concatenate(parts).astype(np.float32)).to(device)


# ------------------------------------------------------------------- volumes
def _dhw(u):
    if u.dim() != 3:
        raise ValueError("volume must be 3-D [D, H, W]")
    return int(u.shape[0]), int(u.shape[1]), int(u.shape[2])


def mf4d3d_workspace_bytes(D: int, H: int, W: int, params: Params) -> int:
    st = params.struct()
    return int(lib().mf4d3d_workspace_bytes(int(D), int(H), int(W), ctypes.byref(st)))


def workspace3(D: int, H: int, W: int, params: Params, device="cuda"):
    nb = mf4d3d_workspace_bytes(D, H, W, params)
    if nb == 0:
        raise MF4DError(MF4D_EINVAL, "mf4d3d_workspace_bytes")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def mf4d3d_scale_select(u, params: Params, idx_out, vmax_out=None, c_out=None, ws=None, stream=None):
    D, H, W = _dhw(_dev(u, torch.float32, name="u"))
    _dev(idx_out, torch.uint8, (D, H, W), "idx_out")
    _dev(vmax_out, torch.float32, (D, H, W), "vmax_out")
    _dev(c_out, torch.float32, (1,), "c_out")
    if ws is None:
        ws = workspace3(D, H, W, params, u.device)
    _dev(ws, torch.uint8, name="ws")
    st = params.struct()
    _check(lib().mf4d3d_scale_select(_ptr(u), D, H, W, ctypes.byref(st), _ptr(idx_out), _ptr(vmax_out),
                                     _ptr(c_out), _ptr(ws), ws.numel(), _stream(stream)), "mf4d3d_scale_select")


def mf4d3d_tensor(u, idx, params: Params, hrho_out, dparams_out=None, ws=None, stream=None):
    D, H, W = _dhw(_dev(u, torch.float32, name="u"))
    _dev(idx, torch.uint8, (D, H, W), "idx")
    _dev(hrho_out, torch.float32, (6, D, H, W), "hrho_out")
    _dev(dparams_out, torch.float32, (D, H, W, 6), "dparams_out")
    if ws is None:
        ws = workspace3(D, H, W, params, u.device)
    _dev(ws, torch.uint8, name="ws")
    st = params.struct()
    _check(lib().mf4d3d_tensor(_ptr(u), D, H, W, _ptr(idx), ctypes.byref(st), _ptr(hrho_out), _ptr(dparams_out),
                               _ptr(ws), ws.numel(), _stream(stream)), "mf4d3d_tensor")


def mf4d3d_dtensor(hrho, params: Params, dparams_out, stream=None):
    _dev(hrho, torch.float32, name="hrho")
    if hrho.dim() != 4 or hrho.shape[0] != 6:
        raise ValueError("hrho must be [6, D, H, W]")
    D, H, W = int(hrho.shape[1]), int(hrho.shape[2]), int(hrho.shape[3])
    _dev(dparams_out, torch.float32, (D, H, W, 6), "dparams_out")
    st = params.struct()
    _check(lib().mf4d3d_dtensor(_ptr(hrho), D, H, W, ctypes.byref(st), _ptr(dparams_out), _stream(stream)),
           "mf4d3d_dtensor")


def mf4d3d_fed_cycle_tensor(u, dparams, taus, u_tmp=None, stream=None):
    D, H, W = _dhw(_dev(u, torch.float32, name="u"))
    _dev(dparams, torch.float32, (D, H, W, 6), "dparams")
    if u_tmp is None:
        u_tmp = torch.empty_like(u)
    _dev(u_tmp, torch.float32, (D, H, W), "u_tmp")
    t = np.ascontiguousarray(np.asarray(taus, dtype=np.float64))
    _check(lib().mf4d3d_fed_cycle_tensor(_ptr(u), _ptr(u_tmp), D, H, W, _ptr(dparams),
                                         t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(t),
                                         _stream(stream)), "mf4d3d_fed_cycle_tensor")


def mf4d3d_filter(u_in, u_out, params: Params, ws=None, stream=None):
    D, H, W = _dhw(_dev(u_in, torch.float32, name="u_in"))
    _dev(u_out, torch.float32, (D, H, W), "u_out")
    if ws is None:
        ws = workspace3(D, H, W, params, u_in.device)
    _dev(ws, torch.uint8, name="ws")
    st = params.struct()
    _check(lib().mf4d3d_filter(_ptr(u_in), _ptr(u_out), D, H, W, ctypes.byref(st), _ptr(ws), ws.numel(),
                               _stream(stream)), "mf4d3d_filter")
