"""FP64 CPU oracle of the MAFOD hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, double-precision reference written from the paper
(multi-scale anisotropic fourth-order diffusion, FED integration). It is
what the GPU library is checked against and must never be on the product
path: only tests/, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it. It shares no code with
``paper_1611_06906_amd`` and does not import it.

The arithmetic lives in ``mf4d_oracle.c`` (built with gcc, -O2,
-ffp-contract=off, OpenMP over pixel rows); this module only marshals
numpy arrays through ctypes.

Parity pins: every function here is pinned by tests/test_oracle_*.py
against closed forms, invariants, brute force on tiny inputs or library
routines (numpy.linalg, numpy.convolve). No function is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mf4d_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "net_oracle.c"), os.path.join(_HERE, "crease_oracle.c"),
         os.path.join(_HERE, "mf4d3d_oracle.c")]
_LIB = os.path.join(_HERE, "libmf4d_oracle.so")

RIDGE, VALLEY, BOTH = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU involved)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, *_SRCS, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class _RefOpts(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("postprocess", ctypes.c_int), ("theta", ctypes.c_double),
                ("idx_inject", _u8p)]


def _declare(L):
    L.ref_fed_n.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double]
    L.ref_fed_n.restype = ctypes.c_int
    L.ref_fed_taus.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp]
    L.ref_kappa_order.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _ip, _dp]
    L.ref_kappa_order.restype = ctypes.c_int
    L.ref_fed_schedule.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _ip]
    L.ref_fed_schedule.restype = ctypes.c_int
    L.ref_gauss_taps.argtypes = [ctypes.c_double, _dp]
    L.ref_gauss_taps.restype = ctypes.c_int
    L.ref_gauss_radius.argtypes = [ctypes.c_double]
    L.ref_gauss_radius.restype = ctypes.c_int
    L.ref_blur.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp]
    L.ref_derivatives.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
    L.ref_scale_select.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                                   ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   _u8p, _dp, _dp, _dp, _dp]
    L.ref_scale_select.restype = ctypes.c_int
    L.ref_tensor.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _u8p, ctypes.c_int, _dp,
                             ctypes.c_double, _dp]
    L.ref_tensor.restype = ctypes.c_int
    L.ref_dtensor_px.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_int, _dp, _dp, _dp]
    L.ref_dtensor.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp]
    L.ref_apply_P.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int, _dp]
    L.ref_explicit_step.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double]
    L.ref_fed_cycle.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int]
    L.ref_filter.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, _dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                             ctypes.c_double, ctypes.c_double, ctypes.c_int,
                             _u8p, _dp, _dp, _dp, ctypes.POINTER(_RefOpts)]
    L.ref_ifod_diffusivity.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp]
    L.ref_ifod_dtensor.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _dp]
    L.ref_cross_direction.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _u8p, _dp, _dp]
    L.ref_postprocess.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _u8p, _dp, _dp, _dp,
                                  ctypes.c_double, ctypes.c_int, _u8p]
    L.ref_filter.restype = ctypes.c_int
    L.ref_crease_field.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp]
    L.ref_marching_creases.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp,
                                       ctypes.POINTER(ctypes.c_int8)]
    L.ref_marching_creases.restype = ctypes.c_long
    L.ref_segment_hausdorff.argtypes = [_dp, _dp]
    L.ref_segment_hausdorff.restype = ctypes.c_double
    L.ref_crease_match.argtypes = [_dp, ctypes.POINTER(ctypes.c_int8), ctypes.c_int, ctypes.c_int, _dp, _ip,
                                   ctypes.c_long, ctypes.c_double, _dp, ctypes.POINTER(ctypes.c_long)]
    L.net_param_count.restype = ctypes.c_int
    L.net_forward.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp]
    L.net_loss.argtypes = [_dp, _u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp]
    L.net_loss.restype = ctypes.c_double
    L.net_grad.argtypes = [_dp, _dp, _u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp]
    L.net_grad.restype = ctypes.c_double
    i_ = ctypes.c_int
    L.ref3_blur.argtypes = [_dp, i_, i_, i_, ctypes.c_double, _dp]
    L.ref3_derivatives.argtypes = [_dp, i_, i_, i_, _dp]
    L.ref3_eig.argtypes = [_dp, _dp, _dp]
    L.ref3_vesselness_px.argtypes = [_dp, ctypes.c_double, i_, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     _dp]
    L.ref3_vesselness_px.restype = ctypes.c_double
    L.ref3_scale_select.argtypes = [_dp, i_, i_, i_, i_, _dp, i_, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, _u8p, _dp, _dp]
    L.ref3_tensor.argtypes = [_dp, i_, i_, i_, _u8p, i_, _dp, ctypes.c_double, _dp]
    L.ref3_dtensor_px.argtypes = [_dp, ctypes.c_double, i_, _dp, _dp]
    L.ref3_dtensor.argtypes = [_dp, i_, i_, i_, ctypes.c_double, i_, _dp]
    L.ref3_apply_P.argtypes = [_dp, _dp, i_, i_, i_, _dp]
    L.ref3_fed_cycle.argtypes = [_dp, _dp, i_, i_, i_, _dp, i_]
    L.ref3_filter.argtypes = [_dp, _dp, i_, i_, i_, i_, _dp, i_, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_double, ctypes.c_double, i_, i_, ctypes.c_double, _u8p,
                              _dp]
    L.net_forward_bf16.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _null(t):
    return ctypes.cast(None, t)


# ---------------------------------------------------------------- schedule
def fed_n(T, M, tau_max=0.05):
    """Eq. (22)."""
    return lib().ref_fed_n(float(T), int(M), float(tau_max))


def fed_taus(n, T, M):
    """Eq. (23), natural order."""
    out = np.zeros(n)
    lib().ref_fed_taus(int(n), float(T), int(M), _d(out))
    return out


def kappa_order(tau, tau_max=0.05):
    tau = _f64(tau)
    n = len(tau)
    perm = np.zeros(n, np.int32)
    ordered = np.zeros(n)
    k = lib().ref_kappa_order(n, _d(tau), float(tau_max), perm.ctypes.data_as(_ip), _d(ordered))
    return k, perm, ordered


def fed_schedule(n, tau_max=0.05):
    """Ordered steps of one cycle for given n. Returns (ordered, perm, kappa)."""
    perm = np.zeros(n, np.int32)
    ordered = np.zeros(n)
    k = lib().ref_fed_schedule(int(n), float(tau_max), _d(ordered), perm.ctypes.data_as(_ip))
    return ordered, perm, k


# ---------------------------------------------------------------- scale space
def gauss_taps(sigma):
    r = lib().ref_gauss_radius(float(sigma))
    g = np.zeros(2 * r + 1)
    lib().ref_gauss_taps(float(sigma), _d(g))
    return g


def blur(u, sigma):
    u = _f64(u)
    H, W = u.shape
    out = np.zeros_like(u)
    lib().ref_blur(_d(u), H, W, float(sigma), _d(out))
    return out


def derivatives(v):
    """(ux, uy, uxx, uxy, uyy) of an already smoothed image."""
    v = _f64(v)
    H, W = v.shape
    outs = [np.zeros_like(v) for _ in range(5)]
    lib().ref_derivatives(_d(v), H, W, *[_d(o) for o in outs])
    return tuple(outs)


def scale_select(u, sigmas, mode, beta=0.5, c=-1.0):
    """Returns dict(idx, V, S, vmax, c)."""
    u = _f64(u)
    H, W = u.shape
    sig = _f64(np.asarray(sigmas, dtype=np.float32))  # scales as the GPU receives them
    ns = len(sig)
    idx = np.zeros((H, W), np.uint8)
    V = np.zeros((ns, H, W))
    S = np.zeros((ns, H, W))
    vmax = np.zeros((H, W))
    cc = np.zeros(1)
    lib().ref_scale_select(_d(u), H, W, ns, _d(sig), int(mode), float(beta), float(c),
                           idx.ctypes.data_as(_u8p), _d(V), _d(S), _d(vmax), _d(cc))
    return dict(idx=idx, V=V, S=S, vmax=vmax, c=float(cc[0]))


def tensor(u, idx, sigmas, rho=0.5):
    """H_rho planes (3, H, W) = (a, b, d)."""
    u = _f64(u)
    H, W = u.shape
    sig = _f64(np.asarray(sigmas, dtype=np.float32))
    idx = np.ascontiguousarray(idx, dtype=np.uint8)
    out = np.zeros((3, H, W))
    lib().ref_tensor(_d(u), H, W, idx.ctypes.data_as(_u8p), len(sig), _d(sig), float(rho), _d(out))
    return out


def dtensor_px(a, b, d, lam, mode):
    D = np.zeros(16)
    e = np.zeros(4)
    mu = np.zeros(4)
    lib().ref_dtensor_px(float(a), float(b), float(d), float(lam), int(mode), _d(D), _d(e), _d(mu))
    return D.reshape(4, 4), e, mu


def dtensor(hrho, lam, mode):
    hrho = _f64(hrho)
    _, H, W = hrho.shape
    out = np.zeros((H, W, 16))
    lib().ref_dtensor(_d(hrho), H, W, float(lam), int(mode), _d(out))
    return out


def apply_P(u, D):
    u = _f64(u)
    D = _f64(D)
    H, W = u.shape
    r = np.zeros_like(u)
    lib().ref_apply_P(_d(u), _d(D), H, W, _d(r))
    return r


def explicit_step(u, D, tau):
    u = _f64(u).copy()
    H, W = u.shape
    lib().ref_explicit_step(_d(u), _d(_f64(D)), H, W, float(tau))
    return u


def fed_cycle(u, D, ordered_tau):
    u = _f64(u).copy()
    H, W = u.shape
    t = _f64(ordered_tau)
    lib().ref_fed_cycle(_d(u), _d(_f64(D)), H, W, _d(t), len(t))
    return u


def filter(u, sigmas, mode, lam=0.005, rho=0.5, beta=0.5, c=-1.0, cycles=1, substeps=10,
           stop_time=0.0, tau_max=0.05, reselect=1, record=False, model=0, postprocess=0,
           theta=0.2, idx_inject=None):
    """The whole filter. Returns u_out, or (u_out, records) if record.

    model: 0 the anisotropic filter, 1 IFOD (Eq. (4), g on H(u_sigma) with
    sigma = sigmas[0]). postprocess, theta: scale-image postprocessing
    (Sec. 3.3). idx_inject: [cycles][H][W] uint8 scale indices used instead
    of the selection in each cycle (teacher forcing)."""
    u = _f64(u)
    H, W = u.shape
    sig = _f64(np.asarray(sigmas, dtype=np.float32))
    out = np.zeros_like(u)
    lam32 = float(np.float32(lam))
    if record:
        idx_rec = np.zeros((cycles, H, W), np.uint8)
        c_rec = np.zeros(max(cycles, 1))
        hrho_rec = np.zeros((cycles, 3, H, W))
        u_rec = np.zeros((cycles, H, W))
        args = (idx_rec.ctypes.data_as(_u8p), _d(c_rec), _d(hrho_rec), _d(u_rec))
    else:
        args = (_null(_u8p), _null(_dp), _null(_dp), _null(_dp))
    inj = None
    if idx_inject is not None:
        inj = np.ascontiguousarray(idx_inject, dtype=np.uint8)
        if inj.shape != (cycles, H, W):
            raise ValueError("idx_inject must be [cycles][H][W]")
    opts = _RefOpts(int(model), int(postprocess), float(np.float32(theta)),
                    inj.ctypes.data_as(_u8p) if inj is not None else _null(_u8p))
    n = lib().ref_filter(_d(u), _d(out), H, W, len(sig), _d(sig), int(mode), lam32,
                         float(np.float32(rho)), float(np.float32(beta)), float(np.float32(c)),
                         int(cycles), int(substeps), float(stop_time), float(tau_max), int(reselect),
                         *args, ctypes.byref(opts))
    if n < 0:
        raise ValueError("invalid schedule")
    if record:
        return out, dict(idx=idx_rec, c=c_rec[:cycles], hrho=hrho_rec, u=u_rec, n=n)
    return out


def filter_l2stop(u, gt, sigmas, mode, cycles, **kw):
    """l2-optimal stopping against a noise-free image (Sec. 4: the evolution
    is stopped where the l2 difference to the ground truth is smallest),
    taken at the ends of FED cycles. Returns (u_best, e, k_best): e[k] is
    ||u^k - gt||_2 for k = 0..cycles (u^0 the input), k_best the smallest
    k of minimal e[k], u_best = u^{k_best}."""
    u0 = _f64(u)
    g = _f64(gt)
    if cycles > 0:
        _, rec = filter(u, sigmas, mode, cycles=cycles, record=True, **kw)
        states = [u0] + [rec["u"][k] for k in range(cycles)]
    else:
        states = [u0]
    e = np.array([np.sqrt(np.sum((s - g) ** 2)) for s in states])
    k = int(np.argmin(e))          # first index of the minimum
    return states[k].copy(), e, k


def ifod_diffusivity(u, sigma, lam=0.005):
    """g = 1 / (1 + ||H(u_sigma)||_F^2 / lambda^2) (Eq. (4) with Eq. (1));
    returns (g, hess[3])."""
    u = _f64(u)
    H, W = u.shape
    g = np.zeros_like(u)
    hess = np.zeros((3, H, W))
    lib().ref_ifod_diffusivity(_d(u), H, W, float(np.float32(sigma)), float(np.float32(lam)), _d(g), _d(hess))
    return g, hess


def ifod_dtensor(g):
    """D = g Id as [H][W][16] (vec order xx, xy, yx, yy)."""
    g = _f64(g)
    H, W = g.shape
    out = np.zeros((H, W, 16))
    lib().ref_ifod_dtensor(_d(g), H, W, _d(out))
    return out


def cross_direction(u, idx, sigmas):
    """Unit vector across the crease: eigenvector of the stronger eigenvalue
    of H(u_sigma) at each pixel's selected scale. Returns (ex, ey)."""
    u = _f64(u)
    H, W = u.shape
    sig = _f64(np.asarray(sigmas, dtype=np.float32))
    idx = np.ascontiguousarray(idx, dtype=np.uint8)
    ex, ey = np.zeros_like(u), np.zeros_like(u)
    lib().ref_cross_direction(_d(u), H, W, len(sig), _d(sig), idx.ctypes.data_as(_u8p), _d(ex), _d(ey))
    return ex, ey


def postprocess(idx, vmax, ex, ey, sigmas, theta, tmax=None):
    """Scale-image postprocessing (Sec. 3.3) from given scale indices, max
    vesselness and cross directions. tmax defaults to ceil(3 sigma_max)."""
    idx = np.ascontiguousarray(idx, dtype=np.uint8)
    H, W = idx.shape
    sig = _f64(np.asarray(sigmas, dtype=np.float32))
    if tmax is None:
        tmax = int(np.ceil(3.0 * sig[-1]))
    out = np.zeros_like(idx)
    lib().ref_postprocess(H, W, len(sig), _d(sig), idx.ctypes.data_as(_u8p), _d(_f64(vmax)), _d(_f64(ex)),
                          _d(_f64(ey)), float(np.float32(theta)), int(tmax), out.ctypes.data_as(_u8p))
    return out


def scale_select_postprocessed(u, sigmas, mode, theta, beta=0.5, c=-1.0):
    """Scale selection followed by the postprocessing, as the filter does it."""
    sel = scale_select(u, sigmas, mode, beta=beta, c=c)
    ex, ey = cross_direction(u, sel["idx"], sigmas)
    sel["idx_raw"] = sel["idx"]
    sel["ex"], sel["ey"] = ex, ey
    sel["idx"] = postprocess(sel["idx_raw"], sel["vmax"], ex, ey, sigmas, theta)
    return sel


# ------------------------------------------------------------------ 3-D
ALPHA3 = 0.5   # Frangi's tube/plate parameter of the 3-D measure (with beta = 0.5)


def blur3(u, sigma):
    u = _f64(u)
    D, H, W = u.shape
    out = np.zeros_like(u)
    lib().ref3_blur(_d(u), D, H, W, float(np.float32(sigma)), _d(out))
    return out


def derivatives3(v):
    """(g_x, g_y, g_z, h_xx, h_yy, h_zz, h_xy, h_xz, h_yz) of a smoothed volume."""
    v = _f64(v)
    D, H, W = v.shape
    out = np.zeros((9, D, H, W))
    lib().ref3_derivatives(_d(v), D, H, W, _d(out))
    return out


def eig3(A):
    """Jacobi eigen-decomposition of a symmetric 3x3: (descending values, vectors as columns)."""
    A = _f64(A).reshape(3, 3)
    ev, V = np.zeros(3), np.zeros((3, 3))
    lib().ref3_eig(_d(np.ascontiguousarray(A)), _d(ev), _d(V))
    return ev, V


def vesselness3_px(h6, sigma, mode, c, beta=0.5, alpha=ALPHA3):
    S = np.zeros(1)
    v = lib().ref3_vesselness_px(_d(_f64(h6)), float(np.float32(sigma)), int(mode), float(alpha), float(beta),
                                 float(c), _d(S))
    return v, float(S[0])


def scale_select3(u, sigmas, mode, beta=0.5, c=-1.0, alpha=ALPHA3):
    u = _f64(u)
    D, H, W = u.shape
    sig = _f64(np.asarray(sigmas, np.float32))
    idx = np.zeros((D, H, W), np.uint8)
    V = np.zeros((len(sig), D, H, W))
    cc = np.zeros(1)
    lib().ref3_scale_select(_d(u), D, H, W, len(sig), _d(sig), int(mode), float(alpha), float(np.float32(beta)),
                            float(np.float32(c)), idx.ctypes.data_as(_u8p), _d(V), _d(cc))
    return dict(idx=idx, V=V, c=float(cc[0]))


def tensor3(u, idx, sigmas, rho=0.5):
    """H_rho planes (xx, yy, zz, xy, xz, yz)."""
    u = _f64(u)
    D, H, W = u.shape
    sig = _f64(np.asarray(sigmas, np.float32))
    idx = np.ascontiguousarray(idx, np.uint8)
    out = np.zeros((6, D, H, W))
    lib().ref3_tensor(_d(u), D, H, W, idx.ctypes.data_as(_u8p), len(sig), _d(sig), float(np.float32(rho)), _d(out))
    return out


def dtensor3_px(h6, lam, mode):
    Dm, mu = np.zeros(81), np.zeros(3)
    lib().ref3_dtensor_px(_d(_f64(h6)), float(lam), int(mode), _d(Dm), _d(mu))
    return Dm.reshape(9, 9), mu


def dtensor3(hrho, lam, mode):
    hrho = _f64(hrho)
    _, D, H, W = hrho.shape
    out = np.zeros((D, H, W, 81))
    lib().ref3_dtensor(_d(hrho), D, H, W, float(lam), int(mode), _d(out))
    return out


def apply_P3(u, Dall):
    u = _f64(u)
    D, H, W = u.shape
    r = np.zeros_like(u)
    lib().ref3_apply_P(_d(u), _d(_f64(Dall)), D, H, W, _d(r))
    return r


def fed_cycle3(u, Dall, taus):
    u = _f64(u).copy()
    D, H, W = u.shape
    t = _f64(taus)
    lib().ref3_fed_cycle(_d(u), _d(_f64(Dall)), D, H, W, _d(t), len(t))
    return u


def filter3(u, sigmas, mode, lam=0.005, rho=0.5, beta=0.5, c=-1.0, cycles=1, substeps=10, tau_max=1.0 / 27.0,
            alpha=ALPHA3, record=False):
    u = _f64(u)
    D, H, W = u.shape
    sig = _f64(np.asarray(sigmas, np.float32))
    out = np.zeros_like(u)
    idx_rec = np.zeros((cycles, D, H, W), np.uint8)
    c_rec = np.zeros(max(cycles, 1))
    lib().ref3_filter(_d(u), _d(out), D, H, W, len(sig), _d(sig), int(mode), float(np.float32(lam)),
                      float(np.float32(rho)), float(alpha), float(np.float32(beta)), float(np.float32(c)),
                      int(cycles), int(substeps), float(tau_max), idx_rec.ctypes.data_as(_u8p), _d(c_rec))
    return (out, dict(idx=idx_rec, c=c_rec[:cycles])) if record else out


# ------------------------------------------------------ crease extraction
def crease_field(u, sigma_d=1.0):
    """Planes (g_x, g_y, h_xx, h_xy, h_yy, d) of u_sigma_d, d = det(g | Hg)
    (Sec. 3.6)."""
    u = _f64(u)
    H, W = u.shape
    out = np.zeros((6, H, W))
    lib().ref_crease_field(_d(u), H, W, float(np.float32(sigma_d)), _d(out))
    return out


def marching_creases(planes, strength=0.0, mode=BOTH):
    """Marching squares on d with the crease test. Returns (seg, type, count):
    seg [H-1][W-1][2][4] (x0, y0, x1, y1), type [H-1][W-1][2] int8
    (+1 ridge, -1 valley, 0 empty)."""
    planes = _f64(planes)
    _, H, W = planes.shape
    seg = np.zeros((H - 1, W - 1, 2, 4))
    typ = np.zeros((H - 1, W - 1, 2), np.int8)
    n = lib().ref_marching_creases(_d(planes), H, W, float(np.float32(strength)), int(mode), _d(seg),
                                   typ.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
    return seg, typ, int(n)


def creases(u, sigma_d=1.0, strength=0.0, mode=BOTH):
    return marching_creases(crease_field(u, sigma_d), strength, mode)


def segment_hausdorff(a, b):
    return lib().ref_segment_hausdorff(_d(_f64(a)), _d(_f64(b)))


def gt_segments(lines):
    """Ground-truth centrelines [(points (K, 2) as (x, y), sign), ...] as
    segments between consecutive samples: (segs [n][4], types [n])."""
    segs, types = [], []
    for pts, sgn in lines:
        pts = np.asarray(pts, np.float64)
        if len(pts) < 2:
            continue
        segs.append(np.concatenate([pts[:-1], pts[1:]], axis=1))
        types.append(np.full(len(pts) - 1, int(sgn), np.int32))
    if not segs:
        return np.zeros((0, 4)), np.zeros(0, np.int32)
    return np.ascontiguousarray(np.concatenate(segs)), np.ascontiguousarray(np.concatenate(types))


def crease_match(seg, typ, gt, gt_type, radius=6.0):
    """Per ground-truth segment: distance of its midpoint to the matched
    reconstruction (-1 if none) and the match index (2 cell + slot)."""
    seg = _f64(seg)
    Hm, Wm = seg.shape[:2]
    typ = np.ascontiguousarray(typ, np.int8)
    gt = _f64(gt).reshape(-1, 4)
    gtt = np.ascontiguousarray(gt_type, np.int32)
    n = len(gt)
    dist = np.zeros(n)
    match = np.zeros(n, np.int64)
    lib().ref_crease_match(_d(seg), typ.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), Hm + 1, Wm + 1, _d(gt),
                           gtt.ctypes.data_as(_ip), n, float(radius), _d(dist),
                           match.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
    return dist, match


def crease_scores(dist):
    """E = mean distance over detected ground-truth segments, p = detected share (Sec. 4)."""
    dist = np.asarray(dist)
    ok = dist >= 0
    return (float(dist[ok].mean()) if ok.any() else float("nan")), float(ok.mean()) if len(dist) else float("nan")


# ------------------------------------------------------------- learned net
NET_CHANNELS = (1, 32, 32, 32, 32, 9)


def net_param_count():
    return lib().net_param_count()


def net_unpack(theta):
    """theta -> list of (W [cout][cin][3][3], b [cout]) per layer."""
    out, pos = [], 0
    for l in range(5):
        ci, co = NET_CHANNELS[l], NET_CHANNELS[l + 1]
        w = theta[pos:pos + co * ci * 9].reshape(co, ci, 3, 3)
        pos += co * ci * 9
        b = theta[pos:pos + co]
        pos += co
        out.append((w, b))
    return out


def net_pack(layers):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in layers]).astype(np.float64)


def net_forward(theta, u):
    """u: [B][H][W]; returns z [B][9][H][W]."""
    theta = _f64(theta)
    u = _f64(u)
    B, H, W = u.shape
    z = np.zeros((B, 9, H, W))
    lib().net_forward(_d(theta), _d(u), B, H, W, _null(_dp), _d(z))
    return z


def net_forward_bf16(theta, u):
    """The network with BF16 weights, inputs and activations (the library's
    definition); theta as float32 values. u: [B][H][W]; returns z [B][9][H][W]."""
    theta = _f64(np.asarray(theta, np.float32))
    u = _f64(np.asarray(u, np.float32))
    if u.ndim == 2:
        u = u[None]
    B, H, W = u.shape
    z = np.zeros((B, 9, H, W))
    lib().net_forward_bf16(_d(theta), _d(np.ascontiguousarray(u)), B, H, W, _d(z))
    return z


def net_decisions(z, ns, thr):
    """Per pixel of a single image's logits z [9][H][W]: the network's scale
    (first maximum of the first min(ns, 8) logits) and whether its
    confidence sigmoid(z_8) reaches thr."""
    k = min(ns, 8)
    scale = np.argmax(z[:k], axis=0).astype(np.uint8)
    conf = 1.0 / (1.0 + np.exp(-z[8]))
    return scale, conf >= thr, conf


def filter_learned(u, theta, sigmas, mode, thr=0.9, lam=0.005, rho=0.5, beta=0.5, c=-1.0, cycles=1,
                   substeps=10, tau_max=0.05, record=False):
    """The learned filter: in each cycle the network's scale where its
    confidence (on the cycle's image) reaches thr, the exact argmax of
    Eq. (9) elsewhere. With c <= 0 the image-wide c of the first cycle is
    kept for every later cycle (the learned filter does not sweep every
    scale over every pixel after the first cycle); c > 0 is used as given.
    Returns u_out (and per-cycle records: net scale, confident mask, exact
    selection, indices used, c)."""
    uk = _f64(u)
    sig = list(sigmas)
    recs = []
    c_held = float(np.float32(c)) if c > 0 else None
    for k in range(cycles):
        z = net_forward_bf16(theta, uk.astype(np.float32))[0]
        ns_, conf_ok, conf = net_decisions(z, len(sig), thr)
        sel = scale_select(uk, sig, mode, beta=beta, c=c_held if c_held is not None else -1.0)
        if c_held is None:
            c_held = sel["c"]
        idx = np.where(conf_ok, ns_, sel["idx"]).astype(np.uint8)
        nxt = filter(uk, sig, mode, lam=lam, rho=rho, beta=beta, c=c_held, cycles=1, substeps=substeps,
                     tau_max=tau_max, idx_inject=idx[None])
        if record:
            recs.append(dict(z=z, net=ns_, conf=conf, confident=conf_ok, sel=sel, idx=idx, c=c_held, u_in=uk))
        uk = nxt
    return (uk, recs) if record else uk


def net_loss(z, label, w_conf=0.1):
    z = _f64(z)
    B, _, H, W = z.shape
    lab = np.ascontiguousarray(label, dtype=np.uint8)
    dz = np.zeros_like(z)
    loss = lib().net_loss(_d(z), lab.ctypes.data_as(_u8p), B, H, W, float(w_conf), _d(dz))
    return loss, dz


def net_grad(theta, u, label, w_conf=0.1):
    theta = _f64(theta)
    u = _f64(u)
    B, H, W = u.shape
    lab = np.ascontiguousarray(label, dtype=np.uint8)
    g = np.zeros_like(theta)
    loss = lib().net_grad(_d(theta), _d(u), lab.ctypes.data_as(_u8p), B, H, W, float(w_conf), _d(g))
    return loss, g
