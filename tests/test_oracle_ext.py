"""Pins of the oracle's extensions beyond the plain filter:

- the isotropic fourth-order model (IFOD, Sec. 3.1 Eq. (4) with the
  Perona-Malik diffusivity of Eq. (1));
- the scale-image postprocessing of Sec. 3.3 (text after Eq. (9));
- l2-optimal stopping against a noise-free image (Sec. 4);
- the per-cycle index injection hook (teacher forcing);
- the stability bound of Sec. 3.4 as a negative case (tau_max above 1/17).

Every expected value below is a closed form, a hand-computed fixture, a
library routine (numpy) or an identity between independent oracle paths.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.usefixtures("oracle_lib")


# ---------------------------------------------------------------- IFOD
def test_ifod_diffusivity_quadratic_closed_form(oracle_lib):
    """u = q1 x^2 + q2 x y + q3 y^2 + ...: away from the border (distance >
    r + 1) H(u_sigma) = [[2 q1, q2], [q2, 2 q3]] exactly, so
    g = 1 / (1 + (4 q1^2 + 2 q2^2 + 4 q3^2) / lambda^2)."""
    H, W = 40, 44
    y, x = np.mgrid[0:H, 0:W].astype(float)
    q1, q2, q3 = 1.5e-4, -2.5e-4, 0.75e-4
    u = 0.3 + q1 * x * x + q2 * x * y + q3 * y * y + 1e-3 * x - 2e-3 * y
    for sigma, lam in [(1.0, 0.005), (2.0, 0.001), (1.5, 0.02)]:
        g, hess = oracle_lib.ifod_diffusivity(u, sigma, lam)
        lam32 = float(np.float32(lam))
        r = int(math.ceil(3 * float(np.float32(sigma))))
        sl = (slice(r + 2, H - r - 2), slice(r + 2, W - r - 2))
        assert np.allclose(hess[0][sl], 2 * q1, atol=1e-12)
        assert np.allclose(hess[1][sl], q2, atol=1e-12)
        assert np.allclose(hess[2][sl], 2 * q3, atol=1e-12)
        F = 4 * q1 ** 2 + 2 * q2 ** 2 + 4 * q3 ** 2
        assert np.allclose(g[sl], 1.0 / (1.0 + F / lam32 ** 2), rtol=1e-9)


def test_ifod_diffusivity_constant_and_range(oracle_lib):
    g, hess = oracle_lib.ifod_diffusivity(np.full((9, 13), 0.4), 1.0, 0.005)
    assert np.all(g == 1.0) and np.all(hess == 0.0)
    rng = np.random.default_rng(3)
    g, _ = oracle_lib.ifod_diffusivity(rng.uniform(size=(30, 31)), 1.0, 0.005)
    assert np.all(g > 0) and np.all(g <= 1)


def test_ifod_tensor_is_scaled_identity(oracle_lib):
    rng = np.random.default_rng(4)
    g = rng.uniform(0.1, 1.0, size=(5, 6))
    D = oracle_lib.ifod_dtensor(g)
    for y in range(5):
        for x in range(6):
            h = rng.normal(size=4)
            assert np.array_equal(D[y, x].reshape(4, 4) @ h, g[y, x] * h)


def test_ifod_matches_anisotropic_tensor_at_equal_eigenvalues(oracle_lib):
    """With H_rho = a Id both eigenvalues are a, mu_1 = mu_2 = mu_3 = g(a^2)
    (Eq. (7)), and the anisotropic D acts on symmetric Hessians as g Id."""
    for a in (0.0, 0.003, -0.01, 0.2):
        lam = 0.005
        Dm, _, mu = oracle_lib.dtensor_px(a, 0.0, a, lam, 2)
        g = 1.0 / (1.0 + a * a / lam ** 2)
        Di = oracle_lib.ifod_dtensor(np.full((1, 1), g))[0, 0].reshape(4, 4)
        rng = np.random.default_rng(int(1e4 * abs(a)))
        for _ in range(5):
            hxx, hxy, hyy = rng.normal(size=3)
            h = np.array([hxx, hxy, hxy, hyy])
            assert np.allclose(Dm @ h, Di @ h, atol=1e-15)


def _dense_L(H, W):
    m = H * W
    out = []
    for y in range(1, H - 1):
        for x in range(1, W - 1):
            Lxx = np.zeros(m); Lxy = np.zeros(m); Lyy = np.zeros(m)
            p = lambda yy, xx: yy * W + xx
            Lxx[p(y, x - 1)] += 1; Lxx[p(y, x)] -= 2; Lxx[p(y, x + 1)] += 1
            Lyy[p(y - 1, x)] += 1; Lyy[p(y, x)] -= 2; Lyy[p(y + 1, x)] += 1
            Lxy[p(y - 1, x - 1)] += .25; Lxy[p(y + 1, x + 1)] += .25
            Lxy[p(y + 1, x - 1)] -= .25; Lxy[p(y - 1, x + 1)] -= .25
            out.append((y * W + x, np.stack([Lxx, Lxy, Lxy, Lyy])))
    return out


def test_ifod_dense_operator(oracle_lib):
    """P = sum_p L_p^T g_p Id L_p (Eq. (4) discretised like Sec. 3.4): the
    oracle's apply_P with the IFOD tensor equals the dense assembly, is
    symmetric PSD with max eigenvalue <= 34, and conserves mass."""
    rng = np.random.default_rng(8)
    H, W = 6, 7
    g = rng.uniform(0.05, 1.0, size=(H, W))
    D = oracle_lib.ifod_dtensor(g)
    m = H * W
    P = np.zeros((m, m))
    for j in range(m):
        e = np.zeros(m); e[j] = 1
        P[:, j] = oracle_lib.apply_P(e.reshape(H, W), D).ravel()
    Pd = np.zeros_like(P)
    for p, L4 in _dense_L(H, W):
        Pd += g.ravel()[p] * (L4.T @ L4)
    assert np.allclose(P, Pd, atol=1e-14)
    ev = np.linalg.eigvalsh((P + P.T) / 2)
    assert np.allclose(P, P.T, atol=1e-14) and ev.min() >= -1e-13 and ev.max() <= 34 + 1e-12
    assert np.allclose(P.sum(axis=0), 0, atol=1e-13)


def test_ifod_filter_linear_limit_fourier(oracle_lib):
    """lambda -> inf: g = 1 and one IFOD cycle scales a Fourier mode far from
    the border by prod(1 - tau_i s(w)) with the 13-point symbol
    s = (2-2cos wx)^2 + (2-2cos wy)^2 + 2 sin^2 wx sin^2 wy."""
    H, W = 40, 44
    y, x = np.mgrid[0:H, 0:W].astype(float)
    wx, wy = 0.9, 0.4
    u = 0.5 + 0.1 * np.cos(wx * x + wy * y + 0.3)
    n = 5
    out = oracle_lib.filter(u, [1.0], 2, lam=1e30, cycles=1, substeps=n, model=1)
    s = (2 - 2 * math.cos(wx)) ** 2 + (2 - 2 * math.cos(wy)) ** 2 + 2 * math.sin(wx) ** 2 * math.sin(wy) ** 2
    ordered, _, _ = oracle_lib.fed_schedule(n, 0.05)
    fac = np.prod(1 - ordered * s)
    k = 2 * n
    assert np.allclose(out[k:-k, k:-k], 0.5 + fac * (u[k:-k, k:-k] - 0.5), atol=1e-12)


def test_ifod_filter_invariants(oracle_lib):
    rng = np.random.default_rng(9)
    u = np.clip(0.5 + 0.2 * rng.normal(size=(26, 30)), 0, 1)
    out = oracle_lib.filter(u, [1.0], 2, cycles=3, substeps=10, model=1)
    assert math.isclose(out.sum(), u.sum(), rel_tol=1e-12)
    assert np.linalg.norm(out - out.mean()) < np.linalg.norm(u - u.mean())
    # D4: transposition and flips commute with the filter
    for f in (np.transpose, np.fliplr, np.flipud):
        o2 = oracle_lib.filter(np.ascontiguousarray(f(u)), [1.0], 2, cycles=3, substeps=10, model=1)
        assert np.allclose(o2, f(out), atol=1e-12)
    y, x = np.mgrid[0:20, 0:23].astype(float)
    aff = 0.25 + x / 1024 + y / 2048
    assert np.array_equal(oracle_lib.filter(aff, [1.0], 2, cycles=2, substeps=7, model=1), aff)


# ------------------------------------------------------ postprocessing
SIG4 = [1.0, 2.0, 3.0, 4.0]


def test_postprocess_band_fixture(oracle_lib):
    """Hand-computed: a vessel band of rows 1-3 in a 5 x 9 image, direction
    across it (0, 1); raw scales row 1 -> sigma 1, row 2 -> sigma 3,
    row 3 -> sigma 4. Every band pixel's cross-section holds the three
    rows of its column: mean (1 + 3 + 4) / 3 = 2.667, closest scale 3
    (index 2). Rows 0 and 4 are background and keep their indices."""
    H, W = 5, 9
    idx = np.zeros((H, W), np.uint8)
    idx[0] = 3
    idx[1] = 0
    idx[2] = 2
    idx[3] = 3
    idx[4] = 1
    vmax = np.zeros((H, W))
    vmax[1:4] = 0.8
    ex, ey = np.zeros((H, W)), np.ones((H, W))
    out = oracle_lib.postprocess(idx, vmax, ex, ey, SIG4, 0.5)
    exp = idx.copy()
    exp[1:4] = 2
    assert np.array_equal(out, exp)
    # a threshold above every vesselness leaves the scale image unchanged
    assert np.array_equal(oracle_lib.postprocess(idx, vmax, ex, ey, SIG4, 0.9), idx)
    # the march stops at tmax: with tmax = 1 the edge rows see two samples
    # (rows 1, 2: mean 2 -> index 1; rows 2, 3: mean 3.5 -> tie 3 | 4 -> index 2)
    # and the middle row three (mean 2.667 -> index 2)
    out1 = oracle_lib.postprocess(idx, vmax, ex, ey, SIG4, 0.5, tmax=1)
    assert np.array_equal(out1[1], np.full(W, 1)) and np.array_equal(out1[2], np.full(W, 2))
    assert np.array_equal(out1[3], np.full(W, 2))


def test_postprocess_diagonal_march_fixture(oracle_lib):
    """Direction (1, 1)/sqrt 2 from (4, 4) in a 9 x 9 all-vessel image:
    offsets round(t / sqrt 2) for t = 1..4 are 1, 1, 2, 3 (half away from
    zero), so the + side visits (5,5), (5,5), (6,6), (7,7) and the - side
    (3,3), (3,3), (2,2), (1,1): repeats are counted. With scale index 3 on
    the diagonal pixels (5,5) and (3,3) and 0 elsewhere the sum is
    1 + 4 sigma_4 (the four visits of (5,5), (3,3)) + 4 sigma_1 = 21 over 9
    samples: mean 2.333, closest 2 (index 1)."""
    H = W = 9
    idx = np.zeros((H, W), np.uint8)
    idx[5, 5] = idx[3, 3] = 3
    vmax = np.ones((H, W))
    ex = np.full((H, W), 1 / math.sqrt(2))
    ey = np.full((H, W), 1 / math.sqrt(2))
    out = oracle_lib.postprocess(idx, vmax, ex, ey, SIG4, 0.5, tmax=4)
    assert out[4, 4] == 1
    # exact half offsets: direction (1/2, sqrt 3 / 2) from (4, 4), tmax = 2:
    # + side (5, 5), (5, 6); - side offsets -1/2 -> -1 and -1 -> -1 give
    # (3, 3), (3, 2) (as (x, y)). Scale index 3 at (x, y) = (3, 3): sum
    # 4 + 4 over 5 samples = 1.6 -> closest 2 (index 1).
    idx6 = np.zeros((H, W), np.uint8)
    idx6[3, 3] = 3
    ex6 = np.full((H, W), 0.5)
    ey6 = np.full((H, W), math.sqrt(0.75))
    assert oracle_lib.postprocess(idx6, vmax, ex6, ey6, SIG4, 0.5, tmax=2)[4, 4] == 1
    # the march leaves the image: from (0, 0) only the + side runs:
    # (1,1), (1,1), (2,2), (3,3) -> sum 1 + 1 + 1 + 1 + 4 = 8 over 5: 1.6 -> index 1
    assert out[0, 0] == 1


def test_postprocess_constant_scale_and_equivariance(oracle_lib):
    rng = np.random.default_rng(12)
    H, W = 23, 31
    vmax = rng.uniform(size=(H, W))
    t = rng.uniform(0, math.pi, size=(H, W))
    ex, ey = np.cos(t), np.sin(t)
    cst = np.full((H, W), 2, np.uint8)
    assert np.array_equal(oracle_lib.postprocess(cst, vmax, ex, ey, SIG4, 0.3), cst)
    idx = rng.integers(0, 4, size=(H, W)).astype(np.uint8)
    out = oracle_lib.postprocess(idx, vmax, ex, ey, SIG4, 0.3)
    # transposition swaps the direction components
    outT = oracle_lib.postprocess(idx.T, vmax.T, ey.T, ex.T, SIG4, 0.3)
    assert np.array_equal(outT, out.T)
    # a left-right flip negates the x component
    outF = oracle_lib.postprocess(idx[:, ::-1], vmax[:, ::-1], -ex[:, ::-1], ey[:, ::-1], SIG4, 0.3)
    assert np.array_equal(outF, out[:, ::-1])
    # the sign of the direction does not matter (both sides are marched)
    assert np.array_equal(oracle_lib.postprocess(idx, vmax, -ex, -ey, SIG4, 0.3), out)


def test_postprocess_brute_force(oracle_lib):
    """The definition evaluated with Python loops and fractions (exact
    arithmetic) on random small fields."""
    from fractions import Fraction
    rng = np.random.default_rng(13)
    sig = [1.0, 1.5, 2.0, 3.0]
    sig32 = [Fraction(float(np.float32(s))) for s in sig]
    H, W = 11, 13
    for trial in range(4):
        idx = rng.integers(0, 4, size=(H, W)).astype(np.uint8)
        vmax = rng.uniform(size=(H, W))
        t = rng.uniform(0, 2 * math.pi, size=(H, W))
        ex, ey = np.cos(t), np.sin(t)
        theta = float(np.float32(0.25 + 0.1 * trial))
        out = oracle_lib.postprocess(idx, vmax, ex, ey, sig, theta, tmax=5)

        def rnd(v):
            return math.floor(v + 0.5) if v >= 0 else -math.floor(-v + 0.5)
        for y in range(H):
            for x in range(W):
                if vmax[y, x] < theta:
                    assert out[y, x] == idx[y, x]
                    continue
                samples = [idx[y, x]]
                for d in (1, -1):
                    for s in range(1, 6):
                        xx, yy = x + rnd(d * s * ex[y, x]), y + rnd(d * s * ey[y, x])
                        if not (0 <= xx < W and 0 <= yy < H) or vmax[yy, xx] < theta:
                            break
                        samples.append(idx[yy, xx])
                mean = sum(sig32[k] for k in samples) / len(samples)
                dist = [abs(mean - s) for s in sig32]
                assert out[y, x] == dist.index(min(dist))


def test_cross_direction_quadratic(oracle_lib):
    """On a quadratic image the Hessian is constant away from the border;
    the direction is the eigenvector (numpy eigh) of its stronger
    eigenvalue, up to sign. With equal eigenvalues every unit vector is an
    eigenvector; an exactly zero Hessian gives (1, 0)."""
    H, W = 30, 30
    y, x = np.mgrid[0:H, 0:W].astype(float)
    for q1, q2, q3 in [(1e-3, 4e-4, -2e-3), (-3e-3, 1e-3, 1e-3), (2e-3, 0.0, 2e-3)]:
        u = q1 * x * x + q2 * x * y + q3 * y * y
        idx = np.zeros((H, W), np.uint8)
        ex, ey = oracle_lib.cross_direction(u, idx, [1.0])
        Hm = np.array([[2 * q1, q2], [q2, 2 * q3]])
        w, V = np.linalg.eigh(Hm)
        e = np.array([ex[15, 15], ey[15, 15]])
        assert math.isclose(e @ e, 1.0, rel_tol=1e-14)
        if abs(w[0]) != abs(w[1]):
            v = V[:, int(np.argmax(np.abs(w)))]
            assert math.isclose(abs(e @ v), 1.0, rel_tol=1e-12), (q1, q2, q3, e, v)
        else:
            assert np.allclose(Hm @ e, w[0] * e, atol=1e-15)
    ex, ey = oracle_lib.cross_direction(np.full((12, 12), 0.3), np.zeros((12, 12), np.uint8), [1.0])
    assert np.all(ex == 1.0) and np.all(ey == 0.0)


def test_postprocess_straight_ridge_uniform_scale(oracle_lib):
    """A straight horizontal Gaussian ridge: every column's cross-section is
    the same, so every vessel pixel of the band gets one common scale."""
    H, W = 48, 40
    y = np.arange(H, dtype=float)[:, None]
    u = 0.2 + 0.6 * np.exp(-((y - 23.5) ** 2) / (2 * 1.5 ** 2)) * np.ones((1, W))
    sig = [1.0, 1.5, 2.0, 3.0, 4.0]
    sel = oracle_lib.scale_select_postprocessed(u, sig, 0, theta=0.3)
    band = sel["vmax"] >= 0.3
    cols = slice(14, 26)   # away from the left and right borders (support of sigma = 4)
    vals = sel["idx"][:, cols][band[:, cols]]
    assert vals.size > 0 and np.all(vals == vals[0])
    # raw selection varies across the band (boundary effects of Sec. 3.3)
    assert len(np.unique(sel["idx_raw"][:, cols][band[:, cols]])) > 1


# ------------------------------------------------------- l2 stopping
def _ridges(seed, H=32, W=36):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:H, 0:W].astype(float)
    gt = 0.2 + 0.6 * np.exp(-((x - 0.4 * y - 12) ** 2) / (2 * 1.8 ** 2))
    return np.clip(gt + rng.normal(scale=0.05, size=gt.shape), 0, 1), gt


def test_l2stop_identities(oracle_lib):
    u, gt = _ridges(0)
    sig = [1.0, 2.0]
    kw = dict(substeps=6, lam=0.005)
    ub, e, k = oracle_lib.filter_l2stop(u, gt, sig, 2, 4, **kw)
    assert len(e) == 5 and math.isclose(e[0], np.linalg.norm(u - gt), rel_tol=1e-15)
    # each e[k] is the distance of a separate k-cycle run
    for kk in range(1, 5):
        uk = oracle_lib.filter(u, sig, 2, cycles=kk, **kw)
        assert math.isclose(e[kk], np.linalg.norm(uk - gt), rel_tol=1e-12)
    assert k == int(np.argmin(e)) and np.array_equal(
        ub, u if k == 0 else oracle_lib.filter(u, sig, 2, cycles=k, **kw))
    # ground truth = input: stop at once; = the 3-cycle result: stop there
    _, e0, k0 = oracle_lib.filter_l2stop(u, u, sig, 2, 4, **kw)
    assert k0 == 0 and e0[0] == 0
    u3 = oracle_lib.filter(u, sig, 2, cycles=3, **kw)
    _, e3, k3 = oracle_lib.filter_l2stop(u, u3, sig, 2, 4, **kw)
    assert k3 == 3 and e3[3] == 0.0
    # a stationary image gives equal distances: the first index wins
    cst = np.full((12, 14), 0.5)
    _, ec, kc = oracle_lib.filter_l2stop(cst, np.zeros_like(cst), sig, 2, 3, **kw)
    assert kc == 0 and np.all(ec == ec[0])


def test_l2stop_denoises(oracle_lib):
    """On a noisy ridge the filter first moves towards the noise-free image."""
    u, gt = _ridges(1)
    _, e, k = oracle_lib.filter_l2stop(u, gt, [1.0, 1.5, 2.0], 0, 6, substeps=8)
    assert e.min() < e[0] and k >= 1


# ------------------------------------------------- injection hook
def test_injected_indices_reproduce_selection(oracle_lib):
    u, _ = _ridges(2)
    sig = [1.0, 1.5, 2.0, 3.0]
    out, rec = oracle_lib.filter(u, sig, 0, cycles=3, substeps=5, record=True)
    out2 = oracle_lib.filter(u, sig, 0, cycles=3, substeps=5, idx_inject=rec["idx"])
    assert np.array_equal(out, out2)
    # a constant injected index k is the filter with the single scale sigma_k
    for k in (0, 2):
        inj = np.full((3,) + u.shape, k, np.uint8)
        a = oracle_lib.filter(u, sig, 0, cycles=3, substeps=5, idx_inject=inj)
        b = oracle_lib.filter(u, [sig[k]], 0, cycles=3, substeps=5)
        assert np.array_equal(a, b)


def test_postprocessed_filter_records_postprocessed_indices(oracle_lib):
    u, _ = _ridges(3)
    sig = [1.0, 1.5, 2.0, 3.0]
    out, rec = oracle_lib.filter(u, sig, 0, cycles=2, substeps=5, record=True, postprocess=1, theta=0.2)
    sel = oracle_lib.scale_select_postprocessed(u, sig, 0, theta=0.2)
    assert np.array_equal(rec["idx"][0], sel["idx"])
    assert np.array_equal(oracle_lib.filter(u, sig, 0, cycles=2, substeps=5, idx_inject=rec["idx"]), out)


# ---------------------------------------------- stability, negative case
def test_tau_above_stability_bound_grows(oracle_lib):
    """Sec. 3.4 bounds the explicit step by 1/17 (||P|| <= 34). A cycle whose
    steps come from tau_max = 0.2 (2 / tau_max = 10 < 32) amplifies the
    highest-frequency mode: l2 growth, which the bound forbids."""
    H, W = 24, 24
    y, x = np.mgrid[0:H, 0:W].astype(float)
    u = 0.5 + 0.01 * np.cos(math.pi * x + math.pi * y)
    D = oracle_lib.dtensor(np.zeros((3, H, W)), math.inf, 2)
    bad, _, _ = oracle_lib.fed_schedule(5, 0.2)
    good, _, _ = oracle_lib.fed_schedule(5, 0.05)
    ub = oracle_lib.fed_cycle(u, D, bad)
    ug = oracle_lib.fed_cycle(u, D, good)
    assert np.linalg.norm(ub - 0.5) > 10 * np.linalg.norm(u - 0.5)
    assert np.linalg.norm(ug - 0.5) <= np.linalg.norm(u - 0.5)
