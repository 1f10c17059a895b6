"""Pins of the oracle's fourth-order tensor (Sec. 3.2, Eqs. (7), (8)) and of
the discrete operator P = L^T D L with natural boundaries (Sec. 3.4)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _vec(A):
    return np.array([A[0, 0], A[0, 1], A[1, 0], A[1, 1]])


def test_eigenvectors_match_lapack(oracle_lib):
    rng = np.random.default_rng(0)
    cases = [tuple(rng.normal(size=3)) for _ in range(300)]
    cases += [(1.0, 0.0, 1.0), (2.0, 1e-12, 2.0), (0.0, 0.0, 0.0), (-1.0, 3.0, 2.0)]
    for a, b, d in cases:
        D, e, mu = oracle_lib.dtensor_px(a, b, d, 0.3, 2)
        A = np.array([[a, b], [b, d]])
        w, V = np.linalg.eigh(A)
        e1, e2 = e[:2], e[2:]
        assert math.isclose(e1 @ e1, 1, rel_tol=1e-14) and abs(e1 @ e2) < 1e-14
        assert np.allclose(A @ e1, w[1] * e1, atol=1e-12)
        assert np.allclose(A @ e2, w[0] * e2, atol=1e-12)


def test_tensor_eigen_structure(oracle_lib):
    rng = np.random.default_rng(1)
    for trial in range(200):
        a, b, d = rng.normal(scale=0.02, size=3)
        lam = 0.005 * (1 + trial % 3)
        mode = trial % 3
        D, e, mu = oracle_lib.dtensor_px(a, b, d, lam, mode)
        e1, e2 = e[:2], e[2:]
        E = [np.outer(e1, e1), np.outer(e2, e2),
             (np.outer(e1, e2) + np.outer(e2, e1)) / math.sqrt(2),
             (np.outer(e1, e2) - np.outer(e2, e1)) / math.sqrt(2)]
        # orthonormal under A:B = tr(B^T A)
        G = np.array([[np.trace(Ej.T @ Ei) for Ej in E] for Ei in E])
        assert np.allclose(G, np.eye(4), atol=1e-14)
        # D vec(E_i) = mu_i vec(E_i)
        for i in range(4):
            assert np.allclose(D @ _vec(E[i]), mu[i] * _vec(E[i]), atol=1e-14)
        assert np.allclose(D, D.T, atol=1e-15)
        assert np.linalg.norm(D, 2) <= 1 + 1e-14
        nu1, nu2 = np.linalg.eigvalsh(np.array([[a, b], [b, d]]))[::-1]
        pm = lambda v: 1 / (1 + v * v / lam ** 2)
        m1, m2 = pm(nu1), pm(nu2)
        if mode == 0:
            m1 = 1.0 if nu1 >= 0 else m1
            m2 = 1.0 if nu2 >= 0 else m2
        elif mode == 1:
            m1 = 1.0 if nu1 <= 0 else m1
            m2 = 1.0 if nu2 <= 0 else m2
        assert np.allclose(mu, [m1, m2, (m1 + m2) / 2, 0.0], atol=1e-12)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_tensor_compact_form(oracle_lib, mode):
    """With mu3 the mean of mu1 and mu2 and mu4 = 0 (Sec. 3.2), D[xx][yy]
    vanishes and D acts on a symmetric h through three numbers:
    T_xx = (mb + al) h_xx + be h_xy, T_xy = T_yx = mb h_xy + be (h_xx + h_yy) / 2,
    T_yy = (mb - al) h_yy + be h_xy, with mb = (D00 + D33) / 2,
    al = (D00 - D33) / 2 and be = D01 + D02, where mb = (mu1 + mu2) / 2 and
    (al, be) = (mu1 - mu2) / 2 (cos 2t, sin 2t) for the angle t of e1."""
    rng = np.random.default_rng(40 + mode)
    for _ in range(200):
        a, b, d = rng.normal(scale=0.01, size=3)
        D, e, mu = oracle_lib.dtensor_px(a, b, d, 0.005, mode)
        assert abs(D[0, 3]) <= 1e-15 and abs(D[3, 0]) <= 1e-15
        mb, al, be = (D[0, 0] + D[3, 3]) / 2, (D[0, 0] - D[3, 3]) / 2, D[0, 1] + D[0, 2]
        t = math.atan2(e[1], e[0])   # e holds e1 = (cos t, sin t) first
        assert math.isclose(mb, (mu[0] + mu[1]) / 2, abs_tol=1e-14)
        assert math.isclose(al, (mu[0] - mu[1]) / 2 * math.cos(2 * t), abs_tol=1e-14)
        assert math.isclose(be, (mu[0] - mu[1]) / 2 * math.sin(2 * t), abs_tol=1e-14)
        hxx, hxy, hyy = rng.normal(size=3)
        T = D @ np.array([hxx, hxy, hxy, hyy])
        want = [(mb + al) * hxx + be * hxy, mb * hxy + be * (hxx + hyy) / 2, mb * hxy + be * (hxx + hyy) / 2,
                (mb - al) * hyy + be * hxy]
        assert np.allclose(T, want, rtol=0, atol=1e-14)


def test_tensor_acts_by_rotation(oracle_lib):
    # independent route: rotate a symmetric H into the eigenbasis of H_rho,
    # scale (h11, h12, h22) by (mu1, mu3, mu2), rotate back
    rng = np.random.default_rng(2)
    for _ in range(200):
        a, b, d = rng.normal(scale=0.01, size=3)
        D, _, mu = oracle_lib.dtensor_px(a, b, d, 0.005, 2)
        w, V = np.linalg.eigh(np.array([[a, b], [b, d]]))
        R = V[:, ::-1]  # columns e1 (larger), e2
        h = rng.normal(size=3)
        Hm = np.array([[h[0], h[1]], [h[1], h[2]]])
        Hp = R.T @ Hm @ R
        Tp = np.array([[mu[0] * Hp[0, 0], mu[2] * Hp[0, 1]], [mu[2] * Hp[1, 0], mu[1] * Hp[1, 1]]])
        T = R @ Tp @ R.T
        assert np.allclose(D @ _vec(Hm), _vec(T), atol=1e-14)


def test_tensor_invariances_and_pm_values(oracle_lib):
    lam = 0.01
    D, _, mu = oracle_lib.dtensor_px(lam, 0.0, 0.0, lam, 2)
    assert math.isclose(mu[0], 0.5, rel_tol=1e-15) and mu[1] == 1.0   # mu(lambda) = 1/2, mu(0) = 1
    # isotropic H_rho: mu1 = mu2 = mu3 and D independent of the eigenvectors
    D1, _, _ = oracle_lib.dtensor_px(0.02, 0.0, 0.02, lam, 2)
    D2, _, _ = oracle_lib.dtensor_px(0.02, 1e-13, 0.02, lam, 2)
    assert np.allclose(D1, D2, atol=1e-9)
    # lambda = +inf: D = I - vec(E4) vec(E4)^T with vec(E4) = (0, 1, -1, 0)/sqrt2
    Dinf, _, _ = oracle_lib.dtensor_px(0.3, -0.2, 0.1, math.inf, 2)
    e4 = np.array([0, 1, -1, 0]) / math.sqrt(2)
    assert np.allclose(Dinf, np.eye(4) - np.outer(e4, e4), atol=1e-15)
    # flux s mu(s): increasing below lambda, decreasing above (Sec. 3.2 regimes)
    s = np.linspace(-5 * lam, 5 * lam, 2001)
    # a = v, b = d = 0: v is nu_1 when v >= 0 and nu_2 when v < 0
    flux = np.array([v * oracle_lib.dtensor_px(v, 0, 0, lam, 2)[2][0 if v >= 0 else 1] for v in s])
    df = np.diff(flux)
    mid = 0.5 * (s[1:] + s[:-1])
    assert np.all(df[np.abs(mid) < 0.99 * lam] > 0)
    assert np.all(df[np.abs(mid) > 1.01 * lam] < 0)


def _dense_L(H, W):
    """The paper's L_xx, L_xy, L_yx, L_yy as dense matrices with rows only at
    interior pixels (natural boundary condition)."""
    m = H * W
    rows = []
    for y in range(1, H - 1):
        for x in range(1, W - 1):
            Lxx = np.zeros(m); Lxy = np.zeros(m); Lyy = np.zeros(m)
            p = lambda yy, xx: yy * W + xx
            Lxx[p(y, x - 1)] += 1; Lxx[p(y, x)] -= 2; Lxx[p(y, x + 1)] += 1
            Lyy[p(y - 1, x)] += 1; Lyy[p(y, x)] -= 2; Lyy[p(y + 1, x)] += 1
            Lxy[p(y - 1, x - 1)] += .25; Lxy[p(y + 1, x + 1)] += .25
            Lxy[p(y + 1, x - 1)] -= .25; Lxy[p(y - 1, x + 1)] -= .25
            rows.append((y * W + x, np.stack([Lxx, Lxy, Lxy, Lyy])))
    return rows


def _dense_P(oracle_lib, D, H, W):
    m = H * W
    P = np.zeros((m, m))
    for j in range(m):
        e = np.zeros(m); e[j] = 1
        P[:, j] = oracle_lib.apply_P(e.reshape(H, W), D).ravel()
    return P


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_dense_operator_properties(oracle_lib, mode):
    rng = np.random.default_rng(5 + mode)
    for H, W in [(3, 3), (5, 7), (8, 6)]:
        hr = rng.normal(scale=0.01, size=(3, H, W))
        D = oracle_lib.dtensor(hr, 0.005, mode)
        P = _dense_P(oracle_lib, D, H, W)
        # P equals L^T D L assembled from the dense stencil matrices
        Pd = np.zeros_like(P)
        for p, L4 in _dense_L(H, W):
            Pd += L4.T @ D[p // W, p % W].reshape(4, 4) @ L4
        assert np.allclose(P, Pd, atol=1e-14)
        assert np.allclose(P, P.T, atol=1e-14)
        ev = np.linalg.eigvalsh(P)
        assert ev.min() >= -1e-13
        assert ev.max() <= 34.0 + 1e-12
        # mass: 1^T P = 0
        assert np.allclose(P.sum(axis=0), 0, atol=1e-13)


def test_affine_images_are_stationary(oracle_lib):
    rng = np.random.default_rng(6)
    H, W = 20, 23
    y, x = np.mgrid[0:H, 0:W].astype(float)
    u = 0.25 + x / 1024 + y / 2048
    D = oracle_lib.dtensor(rng.normal(scale=0.01, size=(3, H, W)), 0.005, 2)
    assert np.all(oracle_lib.apply_P(u, D) == 0.0)


def test_isotropic_operator_is_13_point_stencil(oracle_lib):
    H, W = 11, 12
    D = oracle_lib.dtensor(np.zeros((3, H, W)), math.inf, 2)
    e = np.zeros((H, W)); e[5, 6] = 1.0
    col = oracle_lib.apply_P(e, D)
    ref = np.zeros((H, W))
    ref[5, 6] = 12.5
    for dy, dx in [(0, 1), (0, -1), (1, 0), (-1, 0)]:
        ref[5 + dy, 6 + dx] = -4.0
    for dy, dx in [(0, 2), (0, -2), (2, 0), (-2, 0)]:
        ref[5 + dy, 6 + dx] = 0.75
    for dy, dx in [(2, 2), (2, -2), (-2, 2), (-2, -2)]:
        ref[5 + dy, 6 + dx] = 0.125
    assert np.allclose(col, ref, atol=1e-15)


def test_fourier_mode_scaled_by_symbol(oracle_lib):
    # lambda = inf: symbol s(w) = (2-2cos wx)^2 + (2-2cos wy)^2 + 2 sin^2 wx sin^2 wy
    H, W = 30, 34
    y, x = np.mgrid[0:H, 0:W].astype(float)
    D = oracle_lib.dtensor(np.zeros((3, H, W)), math.inf, 2)
    ordered, _, _ = oracle_lib.fed_schedule(4, 0.05)
    for wx, wy, ph in [(0.3, 1.1, 0.2), (2.0, 0.7, 1.0), (math.pi, math.pi, 0.0)]:
        u = np.cos(wx * x + wy * y + ph)
        s = (2 - 2 * math.cos(wx)) ** 2 + (2 - 2 * math.cos(wy)) ** 2 \
            + 2 * math.sin(wx) ** 2 * math.sin(wy) ** 2
        r = oracle_lib.apply_P(u, D)
        assert np.allclose(r[2:-2, 2:-2], s * u[2:-2, 2:-2], atol=1e-12)
        out = oracle_lib.fed_cycle(u, D, ordered)
        fac = np.prod(1 - ordered * s)
        k = 2 * len(ordered)
        assert np.allclose(out[k:-k, k:-k], fac * u[k:-k, k:-k], atol=1e-11)


def test_l2_stability(oracle_lib):
    rng = np.random.default_rng(7)
    H, W = 24, 24
    for mode in (0, 1, 2):
        D = oracle_lib.dtensor(rng.normal(scale=0.02, size=(3, H, W)), 0.005, mode)
        u = rng.uniform(size=(H, W))
        # explicit step at the Gershgorin limit 1/17
        v = oracle_lib.explicit_step(u, D, 1.0 / 17.0)
        assert np.linalg.norm(v) <= np.linalg.norm(u) * (1 + 1e-14)
        # a FED cycle as a whole, with steps far above 1/17
        ordered, _, _ = oracle_lib.fed_schedule(20, 0.05)
        w = oracle_lib.fed_cycle(u, D, ordered)
        assert np.linalg.norm(w) <= np.linalg.norm(u) * (1 + 1e-9)
        assert math.isclose(w.sum(), u.sum(), rel_tol=1e-12)
