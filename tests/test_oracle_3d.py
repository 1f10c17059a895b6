"""Pins of the oracle's 3-D extension (the paper's 2-D definitions carried
to volumes; the paper names 3-D as future work): blur and derivatives,
the Jacobi eigen-solver, Frangi's 3-D tube measure, the literal 9 x 9
fourth-order tensor, the operator P = L^T D L and the whole filter. Expected
values come from brute force, LAPACK, closed forms and invariants."""
import itertools
import math

import numpy as np
import pytest

pytestmark = pytest.mark.usefixtures("oracle_lib")


def test_blur3_is_brute_force_correlation(oracle_lib):
    rng = np.random.default_rng(0)
    D, H, W = 5, 6, 7
    u = rng.uniform(size=(D, H, W))
    sigma = 1.3
    g = oracle_lib.gauss_taps(float(np.float32(sigma)))
    r = len(g) // 2

    def sym(i, n):
        i %= 2 * n
        return i if i < n else 2 * n - 1 - i
    ref = np.zeros_like(u)
    for z, y, x in itertools.product(range(D), range(H), range(W)):
        s = 0.0
        for a, b, c in itertools.product(range(-r, r + 1), repeat=3):
            s += g[a + r] * g[b + r] * g[c + r] * u[sym(z + a, D), sym(y + b, H), sym(x + c, W)]
        ref[z, y, x] = s
    assert np.allclose(oracle_lib.blur3(u, sigma), ref, atol=1e-13)


def test_derivatives3_quadratic_exact(oracle_lib):
    """A quadratic volume: away from the border the gradient and Hessian of
    u_sigma are those of u exactly (symmetric normalised kernel)."""
    D, H, W = 22, 23, 24
    z, y, x = np.mgrid[0:D, 0:H, 0:W].astype(float)
    q = dict(xx=1e-3, yy=-2e-3, zz=1.5e-3, xy=4e-4, xz=-3e-4, yz=5e-4)
    u = (q["xx"] * x * x + q["yy"] * y * y + q["zz"] * z * z + q["xy"] * x * y + q["xz"] * x * z +
         q["yz"] * y * z + 0.01 * x - 0.02 * y + 0.03 * z)
    der = oracle_lib.derivatives3(oracle_lib.blur3(u, 1.0))
    sl = (slice(6, -6),) * 3
    gx = 2 * q["xx"] * x + q["xy"] * y + q["xz"] * z + 0.01
    gy = 2 * q["yy"] * y + q["xy"] * x + q["yz"] * z - 0.02
    gz = 2 * q["zz"] * z + q["xz"] * x + q["yz"] * y + 0.03
    for k, ref in enumerate([gx, gy, gz]):
        assert np.allclose(der[k][sl], ref[sl], atol=1e-12)
    for k, val in enumerate([2 * q["xx"], 2 * q["yy"], 2 * q["zz"], q["xy"], q["xz"], q["yz"]]):
        assert np.allclose(der[3 + k][sl], val, atol=1e-12)


def test_eig3_against_lapack(oracle_lib):
    rng = np.random.default_rng(1)
    mats = [rng.normal(size=(3, 3)) for _ in range(200)]
    mats = [(m + m.T) / 2 for m in mats]
    mats += [np.diag([1.0, 1.0, -2.0]), np.eye(3), np.zeros((3, 3)), np.diag([3.0, 1e-12, 1e-12])]
    rot = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    mats.append(rot @ np.diag([2.0, 2.0, 5.0]) @ rot.T)
    for A in mats:
        ev, V = oracle_lib.eig3(A)
        w = np.linalg.eigvalsh(A)[::-1]
        assert np.allclose(ev, w, atol=1e-13 * max(1, np.abs(w).max()))
        assert np.allclose(V.T @ V, np.eye(3), atol=1e-13)
        assert np.allclose(A @ V, V * ev, atol=1e-12 * max(1, np.abs(w).max()))
        assert np.all(np.diff(ev) <= 0)


def _tube(D, H, W, w, sign=1.0, along="z"):
    z, y, x = np.mgrid[0:D, 0:H, 0:W].astype(float)
    if along == "z":
        d2 = (x - (W - 1) / 2) ** 2 + (y - (H - 1) / 2) ** 2
    else:
        d2 = (z - (D - 1) / 2) ** 2 + (y - (H - 1) / 2) ** 2
    return 0.3 + sign * 0.5 * np.exp(-d2 / (2 * w * w))


def test_vesselness3_tube_scale_and_modes(oracle_lib):
    """A bright straight tube with a Gaussian cross-section of width w: at
    its axis the selected scale is the one nearest sqrt(2) w (the continuum
    maximiser of sigma^2 |u_sigma''|, with the image-wide c the measure is
    monotone in S there); RIDGE on a dark tube and VALLEY on a bright one
    respond only where the symmetric extension puts the tube's tail between
    mirror images of it (the volume's corners), at 1e-11 of the tube's V."""
    w = 1.4
    u = _tube(9, 25, 25, w)
    sig = [1.0, 2.0, 3.0]
    sel = oracle_lib.scale_select3(u, sig, 0)
    assert sel["idx"][4, 12, 12] == 1            # sqrt(2) * 1.4 = 1.98 -> sigma 2
    vt = sel["V"][:, 4, 12, 12].max()
    assert vt > 0.5
    assert oracle_lib.scale_select3(u, sig, 1)["V"].max() <= 1e-9 * vt
    assert oracle_lib.scale_select3(_tube(9, 25, 25, w, -1.0), sig, 0)["V"].max() <= 1e-9 * vt
    # the valley measure of the dark tube mirrors the ridge measure of the bright one
    assert np.allclose(oracle_lib.scale_select3(_tube(9, 25, 25, w, -1.0), sig, 1)["V"], sel["V"], atol=1e-12)
    # the same tube laid along x gives the same axis response (rotation by 90 degrees)
    ux = _tube(25, 25, 9, w, along="x")
    sx = oracle_lib.scale_select3(ux, sig, 0)
    assert sx["idx"][12, 12, 4] == 1
    assert math.isclose(sx["V"][1, 12, 12, 4], sel["V"][1, 4, 12, 12], rel_tol=1e-9)


def test_vesselness3_suppresses_plates_and_blobs(oracle_lib):
    """Frangi's factors: a plate (one strong eigenvalue) has R_A = 0 and so
    V = 0; a blob (three equal eigenvalues) has R_B = 1 and is damped by
    exp(-1 / (2 beta^2)) = e^-2 against an ideal tube of the same strength."""
    c = 1.0
    plate = oracle_lib.vesselness3_px([-1.0, 0.0, 0.0, 0.0, 0.0, 0.0], 1.0, 0, c)[0]
    blob = oracle_lib.vesselness3_px([-1.0, -1.0, -1.0, 0.0, 0.0, 0.0], 1.0, 0, c)[0]
    tube = oracle_lib.vesselness3_px([-1.0, -1.0, 0.0, 0.0, 0.0, 0.0], 1.0, 0, c)[0]
    S_tube = math.sqrt(2.0)
    assert plate == 0.0
    assert math.isclose(tube, (1 - math.exp(-2.0)) * (1 - math.exp(-S_tube ** 2 / 2)), rel_tol=1e-12)
    S_blob = math.sqrt(3.0)
    assert math.isclose(blob, (1 - math.exp(-2.0)) * math.exp(-2.0) * (1 - math.exp(-S_blob ** 2 / 2)),
                        rel_tol=1e-12)
    # scale normalisation: sigma^2 multiplies the eigenvalues
    v2, S2 = oracle_lib.vesselness3_px([-0.25, -0.25, 0.0, 0.0, 0.0, 0.0], 2.0, 0, c)
    assert math.isclose(S2, S_tube, rel_tol=1e-12) and math.isclose(v2, tube, rel_tol=1e-12)


def test_vesselness3_general_closed_form(oracle_lib):
    """Three distinct eigenvalues in a rotated frame: V equals Frangi's
    formula evaluated by hand on the known eigenvalues (R_A = |n2|/|n3|,
    R_B = |n1| / sqrt|n2 n3|), in every mode."""
    rng = np.random.default_rng(11)
    Q = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    for ev, ok in [((-0.2, -0.5, -1.0), (True, False, True)), ((0.3, 0.6, -0.9), (False, False, True)),
                   ((0.1, 0.4, 0.8), (False, True, True))]:
        A = Q @ np.diag(ev) @ Q.T
        h = [A[0, 0], A[1, 1], A[2, 2], A[0, 1], A[0, 2], A[1, 2]]
        n = sorted(ev, key=abs)
        S = math.sqrt(sum(x * x for x in ev))
        c = 0.7
        ra, rb = abs(n[1]) / abs(n[2]), abs(n[0]) / math.sqrt(abs(n[1] * n[2]))
        want = (1 - math.exp(-ra * ra / 0.5)) * math.exp(-rb * rb / 0.5) * (1 - math.exp(-S * S / (2 * c * c)))
        for mode in (0, 1, 2):
            v, S_out = oracle_lib.vesselness3_px(h, 1.0, mode, c)
            assert math.isclose(S_out, S, rel_tol=1e-12)
            assert math.isclose(v, want if ok[mode] else 0.0, rel_tol=1e-10, abs_tol=1e-15), (ev, mode)


def _vec(A):
    return A.reshape(9)


def test_dtensor3_eigenstructure(oracle_lib):
    rng = np.random.default_rng(2)
    for trial in range(60):
        h = rng.normal(scale=0.02, size=6)
        lam = 0.005 * (1 + trial % 3)
        mode = trial % 3
        Dm, mu = oracle_lib.dtensor3_px(h, lam, mode)
        A = np.array([[h[0], h[3], h[4]], [h[3], h[1], h[5]], [h[4], h[5], h[2]]])
        w, V = np.linalg.eigh(A)
        w, V = w[::-1], V[:, ::-1]
        pm = 1 / (1 + w ** 2 / lam ** 2)
        if mode == 0:
            pm = np.where(w >= 0, 1.0, pm)
        elif mode == 1:
            pm = np.where(w <= 0, 1.0, pm)
        assert np.allclose(mu, pm, atol=1e-12)
        assert np.allclose(Dm, Dm.T, atol=1e-15) and np.linalg.norm(Dm, 2) <= 1 + 1e-12
        for i in range(3):
            for j in range(3):
                Eij = np.outer(V[:, i], V[:, j])
                if i == j:
                    assert np.allclose(Dm @ _vec(Eij), pm[i] * _vec(Eij), atol=1e-12)
                else:
                    S = (Eij + Eij.T) / math.sqrt(2)
                    Aa = (Eij - Eij.T) / math.sqrt(2)
                    assert np.allclose(Dm @ _vec(S), 0.5 * (pm[i] + pm[j]) * _vec(S), atol=1e-12)
                    assert np.allclose(Dm @ _vec(Aa), 0.0, atol=1e-12)
    # lambda = inf: D acts as the identity on symmetric matrices
    Dm, _ = oracle_lib.dtensor3_px(rng.normal(size=6), math.inf, 2)
    Hs = rng.normal(size=(3, 3))
    Hs = Hs + Hs.T
    assert np.allclose(Dm @ _vec(Hs), _vec(Hs), atol=1e-14)


def test_dtensor3_compact_form(oracle_lib):
    """The literal 9 x 9 D acts on every symmetric h as (P h + h P) / 2 with
    P = D(I) (the weights (mu_k + mu_l) / 2 on the symmetric pairs make
    M o G = (Lambda G + G Lambda) / 2), and P = sum_k mu_k e_k e_k^T: the six
    entries of P determine the tensor's action on symmetric matrices. Also at
    equal and zero eigenvalues and lambda = inf (P = I)."""
    rng = np.random.default_rng(11)
    cases = [rng.normal(scale=0.02, size=6) for _ in range(30)]
    cases += [np.zeros(6), np.array([0.01, 0.01, 0.01, 0, 0, 0]), np.array([0.02, 0.02, -0.01, 0, 0, 0])]
    for t, h6 in enumerate(cases):
        for mode in (0, 1, 2):
            lam = math.inf if t == 5 else 0.005 * (1 + t % 3)
            Dm, mu = oracle_lib.dtensor3_px(h6, lam, mode)
            P = (Dm @ _vec(np.eye(3))).reshape(3, 3)
            assert np.allclose(P, P.T, atol=1e-15)
            A = np.array([[h6[0], h6[3], h6[4]], [h6[3], h6[1], h6[5]], [h6[4], h6[5], h6[2]]])
            w, V = np.linalg.eigh(A)
            w, V = w[::-1], V[:, ::-1]
            if np.min(np.abs(np.diff(w))) > 1e-9:   # simple eigenvalues: mu pairs with V's columns
                assert np.allclose(P, (V * mu) @ V.T, atol=1e-12)
            assert np.allclose(np.sort(np.linalg.eigvalsh(P)), np.sort(mu), atol=1e-12)
            if lam == math.inf:
                assert np.allclose(P, np.eye(3), atol=1e-14)
            for _ in range(4):
                h = rng.normal(size=(3, 3))
                h = h + h.T
                got = 0.5 * (P @ h + h @ P)
                assert np.allclose((Dm @ _vec(h)).reshape(3, 3), got, atol=1e-12)


def _dense_P3(oracle_lib, Dall, shape):
    m = int(np.prod(shape))
    P = np.zeros((m, m))
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1.0
        P[:, j] = oracle_lib.apply_P3(e.reshape(shape), Dall).ravel()
    return P


def _dense_L3(shape):
    D, H, W = shape
    m = D * H * W
    idx = lambda z, y, x: (z * H + y) * W + x
    rows = []
    for z, y, x in itertools.product(range(1, D - 1), range(1, H - 1), range(1, W - 1)):
        L = np.zeros((9, m))
        for k, (dz, dy, dx) in enumerate([(0, 0, 1), (0, 1, 0), (1, 0, 0)]):
            row = [0, 4, 8][k]
            L[row, idx(z - dz, y - dy, x - dx)] += 1
            L[row, idx(z, y, x)] -= 2
            L[row, idx(z + dz, y + dy, x + dx)] += 1
        for rows_, (a, b) in [((1, 3), ((0, 0, 1), (0, 1, 0))), ((2, 6), ((0, 0, 1), (1, 0, 0))),
                              ((5, 7), ((0, 1, 0), (1, 0, 0)))]:
            for r in rows_:
                for sa, sb, wgt in [(-1, -1, .25), (1, 1, .25), (-1, 1, -.25), (1, -1, -.25)]:
                    off = tuple(sa * a[i] + sb * b[i] for i in range(3))
                    L[r, idx(z + off[0], y + off[1], x + off[2])] += wgt
        rows.append((idx(z, y, x), L))
    return rows


def test_operator3_dense_properties(oracle_lib):
    """P = L^T D L assembled from dense stencil matrices equals the oracle's
    scatter form; it is symmetric PSD with max eigenvalue <= 54 (the 3-D
    bound behind tau <= 1/27) and conserves mass; affine volumes are
    stationary."""
    rng = np.random.default_rng(3)
    shape = (4, 5, 5)
    for mode in (0, 2):
        hr = rng.normal(scale=0.01, size=(6,) + shape)
        Dall = oracle_lib.dtensor3(hr, 0.005, mode)
        P = _dense_P3(oracle_lib, Dall, shape)
        Pd = np.zeros_like(P)
        Dflat = Dall.reshape(-1, 9, 9)
        for p, L in _dense_L3(shape):
            Pd += L.T @ Dflat[p] @ L
        assert np.allclose(P, Pd, atol=1e-13)
        assert np.allclose(P, P.T, atol=1e-13)
        ev = np.linalg.eigvalsh(P)
        assert ev.min() >= -1e-12 and ev.max() <= 54 + 1e-9
        assert np.allclose(P.sum(axis=0), 0, atol=1e-12)
    z, y, x = np.mgrid[0:6, 0:7, 0:8].astype(float)
    aff = 0.25 + x / 1024 + y / 2048 - z / 4096
    Dall = oracle_lib.dtensor3(rng.normal(scale=0.01, size=(6, 6, 7, 8)), 0.005, 2)
    assert np.all(oracle_lib.apply_P3(aff, Dall) == 0.0)


def test_operator3_isotropic_symbol_and_stability(oracle_lib):
    """lambda = inf: far from the border P scales cos(w . x) by the symbol
    s = sum_i (2 - 2 cos w_i)^2 + 2 sum_{i<j} sin^2 w_i sin^2 w_j, whose
    maximum 48 is below the bound 54. A cycle from tau_max = 1/27 is stable
    on the highest mode; tau_max = 0.05 (the 2-D bound) makes it grow."""
    shape = (16, 17, 18)
    z, y, x = np.mgrid[0:shape[0], 0:shape[1], 0:shape[2]].astype(float)
    Dall = oracle_lib.dtensor3(np.zeros((6,) + shape), math.inf, 2)
    for w in [(0.4, 1.1, 0.7), (math.pi, math.pi, math.pi), (2.0, 0.3, 1.5)]:
        u = np.cos(w[2] * x + w[1] * y + w[0] * z + 0.2)
        s = sum((2 - 2 * math.cos(t)) ** 2 for t in w) + 2 * sum(
            math.sin(a) ** 2 * math.sin(b) ** 2 for a, b in itertools.combinations(w, 2))
        r = oracle_lib.apply_P3(u, Dall)
        assert np.allclose(r[2:-2, 2:-2, 2:-2], s * u[2:-2, 2:-2, 2:-2], atol=1e-11)
    u = 0.5 + 0.01 * np.cos(math.pi * (x + y + z))
    good, _, _ = oracle_lib.fed_schedule(6, 1.0 / 27.0)
    bad, _, _ = oracle_lib.fed_schedule(6, 0.05)
    assert np.linalg.norm(oracle_lib.fed_cycle3(u, Dall, good) - 0.5) <= np.linalg.norm(u - 0.5) * (1 + 1e-12)
    assert np.linalg.norm(oracle_lib.fed_cycle3(u, Dall, bad) - 0.5) > 2 * np.linalg.norm(u - 0.5)


def test_filter3_invariants(oracle_lib):
    rng = np.random.default_rng(4)
    u = np.clip(_tube(10, 12, 13, 1.2) + 0.05 * rng.normal(size=(10, 12, 13)), 0, 1)
    sig = [1.0, 1.5]
    out = oracle_lib.filter3(u, sig, 2, cycles=2, substeps=6)
    assert math.isclose(out.sum(), u.sum(), rel_tol=1e-12)
    # axis permutations and flips commute with the filter (the 3-D analogue of D4)
    for f in (lambda a: np.ascontiguousarray(a.transpose(0, 2, 1)),
              lambda a: np.ascontiguousarray(a.transpose(2, 1, 0)),
              lambda a: np.ascontiguousarray(a[::-1]), lambda a: np.ascontiguousarray(a[:, :, ::-1])):
        assert np.allclose(oracle_lib.filter3(f(u), sig, 2, cycles=2, substeps=6), f(out), atol=1e-12)
    cst = np.full((6, 7, 8), 0.4)
    assert np.array_equal(oracle_lib.filter3(cst, sig, 2, cycles=1, substeps=5), cst)
