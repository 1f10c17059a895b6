"""Pins of the oracle's Gaussian scale space, derivatives, scale selection
and normalised Hessian (Sec. 3.1 Eq. (6), Sec. 3.3 Eq. (9))."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _direct_blur(u, g):
    """Brute-force 2-D correlation of the symmetric (numpy 'symmetric')
    extension with the outer product of the taps."""
    r = (len(g) - 1) // 2
    up = np.pad(u, r, mode="symmetric")
    K = np.outer(g, g)
    H, W = u.shape
    out = np.zeros_like(u)
    for y in range(H):
        for x in range(W):
            out[y, x] = (up[y:y + 2 * r + 1, x:x + 2 * r + 1] * K).sum()
    return out


def test_gauss_taps(oracle_lib):
    for s in (0.2, 0.5, 1.0, 1.4859, 3.0, 7.25, 16.0):
        g = oracle_lib.gauss_taps(s)
        r = (len(g) - 1) // 2
        assert r == max(1, math.ceil(3 * s))
        assert math.isclose(g.sum(), 1.0, rel_tol=1e-14)
        assert np.allclose(g, g[::-1], rtol=0, atol=0)
        j = np.arange(-r, r + 1)
        ref = np.exp(-j * j / (2 * s * s))
        assert np.allclose(g, ref / ref.sum(), rtol=1e-14)


def test_blur_matches_brute_force_2d(oracle_lib):
    rng = np.random.default_rng(1)
    for (H, W), s in [((9, 9), 1.0), ((9, 7), 2.5), ((6, 11), 4.0), ((5, 5), 0.5)]:
        u = rng.uniform(size=(H, W))
        g = oracle_lib.gauss_taps(s)
        assert np.allclose(oracle_lib.blur(u, s), _direct_blur(u, g), rtol=0, atol=1e-13)


def test_blur_constant_and_equivariance(oracle_lib):
    u = np.full((13, 17), 0.37)
    assert np.allclose(oracle_lib.blur(u, 3.0), 0.37, atol=1e-15)
    rng = np.random.default_rng(2)
    v = rng.uniform(size=(13, 17))
    b = oracle_lib.blur(v, 2.0)
    assert np.allclose(oracle_lib.blur(v.T, 2.0), b.T, atol=1e-14)
    assert np.allclose(oracle_lib.blur(v[:, ::-1], 2.0), b[:, ::-1], atol=1e-14)
    assert np.allclose(oracle_lib.blur(v[::-1], 2.0), b[::-1], atol=1e-14)


def test_quadratic_image_exact_derivatives(oracle_lib):
    # symmetric normalised kernels shift a quadratic by a constant, so the
    # central differences of u_sigma reproduce the exact derivatives
    H, W = 48, 40
    y, x = np.mgrid[0:H, 0:W].astype(float)
    q = [3e-4, -2e-4, 5e-4, 0.01, -0.02, 0.3]
    u = q[0] * x * x + q[1] * x * y + q[2] * y * y + q[3] * x + q[4] * y + q[5]
    for s in (1.0, 2.0, 3.3):
        r = max(1, math.ceil(3 * s))
        ux, uy, uxx, uxy, uyy = oracle_lib.derivatives(oracle_lib.blur(u, s))
        sl = (slice(r + 1, H - r - 1), slice(r + 1, W - r - 1))
        assert np.allclose(uxx[sl], 2 * q[0], atol=1e-12)
        assert np.allclose(uxy[sl], q[1], atol=1e-12)
        assert np.allclose(uyy[sl], 2 * q[2], atol=1e-12)
        assert np.allclose(ux[sl], (2 * q[0] * x + q[1] * y + q[3])[sl], atol=1e-11)
        assert np.allclose(uy[sl], (q[1] * x + 2 * q[2] * y + q[4])[sl], atol=1e-11)


def test_derivative_stencils_brute_force(oracle_lib):
    rng = np.random.default_rng(3)
    v = rng.uniform(size=(7, 8))
    ux, uy, uxx, uxy, uyy = oracle_lib.derivatives(v)
    p = np.pad(v, 1, mode="symmetric")
    c = p[1:-1, 1:-1]
    assert np.allclose(ux, (p[1:-1, 2:] - p[1:-1, :-2]) / 2, atol=1e-15)
    assert np.allclose(uy, (p[2:, 1:-1] - p[:-2, 1:-1]) / 2, atol=1e-15)
    assert np.allclose(uxx, p[1:-1, :-2] - 2 * c + p[1:-1, 2:], atol=1e-15)
    assert np.allclose(uyy, p[:-2, 1:-1] - 2 * c + p[2:, 1:-1], atol=1e-15)
    assert np.allclose(uxy, (p[:-2, :-2] + p[2:, 2:] - p[2:, :-2] - p[:-2, 2:]) / 4, atol=1e-15)


def _vesselness_numpy(u, sigmas, mode, beta=0.5, c=None):
    """Independent brute force: numpy eigvalsh per pixel, Eq. (9)."""
    sig = np.asarray(sigmas, dtype=np.float32).astype(float)
    import oracle
    Vs, Ss = [], []
    for s in sig:
        _, _, hxx, hxy, hyy = oracle.derivatives(oracle.blur(u, s))
        Hm = np.stack([np.stack([hxx, hxy], -1), np.stack([hxy, hyy], -1)], -2) * s * s
        ev = np.linalg.eigvalsh(Hm)
        order = np.argsort(np.abs(ev), axis=-1)
        ev = np.take_along_axis(ev, order, -1)
        Ss.append(np.sqrt((ev ** 2).sum(-1)))
        Vs.append(ev)
    S = np.stack(Ss)
    cc = 0.5 * S.max() if c is None else c
    V = []
    for ev, Sx in zip(Vs, Ss):
        n1, n2 = ev[..., 0], ev[..., 1]
        with np.errstate(divide="ignore", invalid="ignore"):
            v = np.exp(-(n1 / n2) ** 2 / (2 * beta ** 2)) * (1 - np.exp(-Sx ** 2 / (2 * cc ** 2)))
        if mode == 0:
            v[n2 > 0] = 0
        elif mode == 1:
            v[n2 < 0] = 0
        v[n2 == 0] = 0
        V.append(v)
    V = np.stack(V)
    return V, S, cc


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_vesselness_brute_force(oracle_lib, mode):
    rng = np.random.default_rng(10 + mode)
    u = rng.uniform(size=(14, 12))
    sig = [0.7, 1.2, 2.0]
    res = oracle_lib.scale_select(u, sig, mode)
    V, S, c = _vesselness_numpy(u, sig, mode)
    assert math.isclose(res["c"], c, rel_tol=1e-13)
    assert np.allclose(res["S"], S, atol=1e-13)
    assert np.allclose(res["V"], V, atol=1e-12)
    assert np.array_equal(res["idx"], np.argmax(res["V"], axis=0))
    assert np.allclose(res["vmax"], V.max(0), atol=1e-12)


def test_straight_ridge_reduces_to_1d_and_picks_sqrt2_w(oracle_lib):
    # image constant along y: blur along y is the identity, H = diag(u_xx, 0)
    W, H = 81, 9
    x = np.arange(W) - 40.0
    w = math.sqrt(2.0)
    prof = 0.6 * np.exp(-x * x / (2 * w * w))
    u = np.tile(prof, (H, 1))
    sig = [1.0, 1.5, 2.0, 3.0]
    res = oracle_lib.scale_select(u, sig, 0)
    # 1-D route with numpy.convolve on the symmetric extension
    S1 = []
    for s in np.asarray(sig, np.float32).astype(float):
        g = oracle_lib.gauss_taps(s)
        r = (len(g) - 1) // 2
        us = np.convolve(np.pad(prof, r, mode="symmetric"), g, mode="valid")
        e = np.pad(us, 1, mode="symmetric")
        S1.append(s * s * np.abs(e[:-2] - 2 * e[1:-1] + e[2:]))
    S1 = np.array(S1)
    assert np.allclose(res["S"][:, 4, :], S1, atol=1e-13)
    c = 0.5 * S1.max()
    V1 = 1 - np.exp(-S1[:, 40] ** 2 / (2 * c * c))  # R_B = 0 on the axis
    assert np.allclose(res["V"][:, 4, 40], V1, atol=1e-13)
    # continuum optimum sigma = sqrt(2) w = 2 -> index 2
    assert res["idx"][4, 40] == 2
    assert np.all(res["idx"][:, 40] == 2)


def test_sign_tests_and_degenerate_images(oracle_lib):
    W, H = 41, 7
    x = np.arange(W) - 20.0
    prof = 0.5 * np.exp(-x * x / 4.0)
    ridge = np.tile(0.2 + prof, (H, 1))
    valley = np.tile(0.8 - prof, (H, 1))
    sig = [1.0, 2.0]
    assert np.all(oracle_lib.scale_select(valley, sig, 0)["V"][:, :, 19:22] == 0)
    assert np.all(oracle_lib.scale_select(ridge, sig, 1)["V"][:, :, 19:22] == 0)
    assert oracle_lib.scale_select(ridge, sig, 0)["V"][:, 3, 20].min() > 0.3
    assert oracle_lib.scale_select(valley, sig, 1)["V"][:, 3, 20].min() > 0.3
    both_r = oracle_lib.scale_select(ridge, sig, 2)
    both_v = oracle_lib.scale_select(valley, sig, 2)
    assert np.allclose(both_r["V"], both_v["V"], atol=1e-13)
    const = np.full((9, 9), 0.4)
    res = oracle_lib.scale_select(const, sig, 0)
    assert res["c"] == 0.0 and np.all(res["V"] == 0) and np.all(res["idx"] == 0)
    # a given c is used as is
    res = oracle_lib.scale_select(ridge, sig, 0, c=0.25)
    assert res["c"] == 0.25


def test_normalised_hessian_quadratic_closed_form(oracle_lib):
    H, W = 40, 44
    y, x = np.mgrid[0:H, 0:W].astype(float)
    q = [2e-3, 1e-3, -1e-3, 0.05, 0.02, 0.1]
    u = q[0] * x * x + q[1] * x * y + q[2] * y * y + q[3] * x + q[4] * y + q[5]
    sig = [1.0, 2.0]
    idx = np.zeros((H, W), np.uint8)
    idx[:, W // 2:] = 1
    hr = oracle_lib.tensor(u, idx, sig, rho=0.5)
    gx = 2 * q[0] * x + q[1] * y + q[3]
    gy = q[1] * x + 2 * q[2] * y + q[4]
    f = 1.0 / np.sqrt(1.0 + np.hypot(gx, gy))
    N = np.stack([2 * q[0] * f, q[1] * f, 2 * q[2] * f])
    g = oracle_lib.gauss_taps(0.5)
    K = np.outer(g, g)
    for yy in range(10, H - 10, 7):
        for xx in range(10, W - 10, 5):
            ref = (N[:, yy - 2:yy + 3, xx - 2:xx + 3] * K).sum(axis=(1, 2))
            assert np.allclose(hr[:, yy, xx], ref, atol=1e-14)


def test_normalised_hessian_rho_zero_is_pointwise(oracle_lib):
    rng = np.random.default_rng(4)
    u = rng.uniform(size=(16, 16))
    sig = [1.0, 1.5]
    idx = (rng.uniform(size=(16, 16)) < 0.5).astype(np.uint8)
    hr = oracle_lib.tensor(u, idx, sig, rho=0.0)
    for s in range(2):
        sv = float(np.float32(sig[s]))
        ux, uy, uxx, uxy, uyy = oracle_lib.derivatives(oracle_lib.blur(u, sv))
        f = 1 / np.sqrt(1 + np.hypot(ux, uy))
        m = idx == s
        assert np.allclose(hr[0][m], (uxx * f)[m], atol=1e-15)
        assert np.allclose(hr[1][m], (uxy * f)[m], atol=1e-15)
        assert np.allclose(hr[2][m], (uyy * f)[m], atol=1e-15)
