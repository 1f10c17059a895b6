"""Pins of the oracle's crease extraction (Sec. 3.6: zero contour of
d = det(g | Hg) by marching squares) and of its evaluation measures
(Sec. 4: matching by Hausdorff distance within a neighbourhood, the mean
distance E and the detected share p). Expected values are closed forms and
hand-computed cases."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.usefixtures("oracle_lib")


def test_field_quadratic_closed_form(oracle_lib):
    """u = a x^2 + b x y + c y^2 + e x + f y: away from the border (> r + 1)
    g = (2 a x + b y + e, b x + 2 c y + f), H = [[2a, b], [b, 2c]] exactly,
    so d = g_x (b g_x + 2c g_y) - g_y (2a g_x + b g_y)."""
    H, W = 36, 40
    y, x = np.mgrid[0:H, 0:W].astype(float)
    a, b, c, e, f = 2e-3, -1.5e-3, 1e-3, 0.05, -0.02
    u = a * x * x + b * x * y + c * y * y + e * x + f * y
    P = oracle_lib.crease_field(u, 1.0)
    sl = (slice(6, H - 6), slice(6, W - 6))
    gx = 2 * a * x + b * y + e
    gy = b * x + 2 * c * y + f
    assert np.allclose(P[0][sl], gx[sl], atol=1e-12) and np.allclose(P[1][sl], gy[sl], atol=1e-12)
    assert np.allclose(P[2][sl], 2 * a, atol=1e-12) and np.allclose(P[3][sl], b, atol=1e-12)
    assert np.allclose(P[4][sl], 2 * c, atol=1e-12)
    d = gx * (b * gx + 2 * c * gy) - gy * (2 * a * gx + b * gy)
    assert np.allclose(P[5][sl], d[sl], atol=1e-14)


def _planes_for(d, v=(1.0, 0.0), ridge=True):
    """Field planes with the given d and, everywhere, H = -n n^T (ridge) or
    +n n^T (valley), n the unit normal of direction v: the crease runs along
    v (weak eigenvalue 0 along v, strong -1 or +1 across)."""
    H, W = d.shape
    vx, vy = v
    L = math.hypot(vx, vy)
    nx, ny = -vy / L, vx / L
    s = -1.0 if ridge else 1.0
    P = np.zeros((6, H, W))
    P[2], P[3], P[4] = s * nx * nx, s * nx * ny, s * ny * ny
    P[5] = d
    return P


@pytest.mark.parametrize("pattern", range(16))
def test_marching_cases_by_hand(oracle_lib, pattern):
    """One cell with corners (0,0), (1,0), (1,1), (0,1) at d = +-1 (inside:
    d >= 0): every crossing lies at the middle of its edge; the segments
    join the edges listed below (hand-derived), sorted by first edge."""
    sign = [1.0 if pattern >> k & 1 else -1.0 for k in range(4)]
    corners = [(0, 0), (1, 0), (1, 1), (0, 1)]
    d = np.zeros((2, 2))
    for (cx, cy), s in zip(corners, sign):
        d[cy, cx] = s
    mid = {0: (0.5, 0.0), 1: (1.0, 0.5), 2: (0.5, 1.0), 3: (0.0, 0.5)}
    expected = {0: [], 15: [], 1: [(0, 3)], 14: [(0, 3)], 2: [(0, 1)], 13: [(0, 1)], 4: [(1, 2)], 11: [(1, 2)],
                8: [(2, 3)], 7: [(2, 3)], 3: [(1, 3)], 12: [(1, 3)], 6: [(0, 2)], 9: [(0, 2)],
                # saddles: the centre mean is 0, i.e. inside; the outside corners are cut off
                5: [(0, 1), (2, 3)], 10: [(0, 3), (1, 2)]}[pattern]
    v = (1.0, 0.0)
    if expected:   # the crease runs along the (first) segment; both saddle segments are parallel
        a, b = np.array(mid[expected[0][0]]), np.array(mid[expected[0][1]])
        v = tuple(b - a)
    seg, typ, n = oracle_lib.marching_creases(_planes_for(d, v), 0.0, 0)
    assert n == len(expected)
    for k, (e0, e1) in enumerate(expected):
        assert typ[0, 0, k] == 1
        assert np.allclose(seg[0, 0, k], mid[e0] + mid[e1], atol=1e-15)
    assert np.all(typ[0, 0, len(expected):] == 0)
    # the valley field gives valley segments, and mode filters by type
    seg, typ, n = oracle_lib.marching_creases(_planes_for(d, v, ridge=False), 0.0, 2)
    assert n == len(expected) and np.all(typ[0, 0, :n] == -1)
    assert oracle_lib.marching_creases(_planes_for(d, v, ridge=False), 0.0, 0)[2] == 0
    # a crease field across the segments keeps none of them
    if expected:
        assert oracle_lib.marching_creases(_planes_for(d, (-v[1], v[0])), 0.0, 2)[2] == 0


def test_marching_interpolation_and_saddle_split(oracle_lib):
    # edge 0 from d = 3 to d = -1 crosses at t = 3/4; edge 3 from d = -2 (corner 3) to 3 at t = 2/5
    d = np.array([[3.0, -1.0], [-2.0, -1.0]])
    seg, typ, n = oracle_lib.marching_creases(_planes_for(d, (-0.75, 0.6)), 0.0, 0)
    assert n == 1 and np.allclose(seg[0, 0, 0], [0.75, 0.0, 0.0, 1 - 0.4], atol=1e-15)
    # saddle with a negative centre: the inside corners 0 and 2 are cut off
    d = np.array([[1.0, -3.0], [-3.0, 1.0]])
    seg, typ, n = oracle_lib.marching_creases(_planes_for(d, (-1.0, 1.0)), 0.0, 0)
    assert n == 2
    assert np.allclose(seg[0, 0, 0], [0.25, 0.0, 0.0, 0.25], atol=1e-15)    # edges 0 and 3
    assert np.allclose(seg[0, 0, 1], [1.0, 0.75, 0.75, 1.0], atol=1e-15)    # edges 1 and 2


def test_crease_test_cases(oracle_lib):
    """A vertical segment (d = +1 left, -1 right: it runs from (1/2, 0) to
    (1/2, 1)) is a ridge when the stronger eigenvalue of H is negative, at
    least `strength` in magnitude, and the segment runs closer to the weaker
    eigenvector; a valley with the sign reversed."""
    d = np.array([[1.0, -1.0], [1.0, -1.0]])
    cases = [
        ((-1.0, 0.0, 0.0), 0.0, 1),      # strong -1 across (x): ridge along y
        ((0.0, 0.0, -1.0), 0.0, 0),      # strong -1 along the segment: it crosses the crease
        ((1.0, 0.0, 0.0), 0.0, -1),      # valley
        ((-1.0, 0.0, 0.0), 1.5, 0),      # below the strength
        ((-1.0, 0.0, -1.0), 0.0, 0),     # equal eigenvalues: no direction
        ((-1.0, 0.0, 0.5), 0.0, 1),      # eigenvalues -1 and 1/2: the negative one is stronger
        ((-1.0, 0.0, 1.0), 0.0, 0),      # equal magnitudes of opposite sign
        ((0.0, 0.5, 0.0), 0.0, 0),       # likewise
        ((-1.0, 0.5, 0.0), 0.0, 1),      # strong eigenvector tilted, still nearer x than y
        ((-0.1, 1.0, 0.0), 0.0, 1),      # strong eigenvector near 45 degrees, on the x side
        ((0.1, 1.0, 0.0), 0.0, -1),      # positive stronger eigenvalue, eigenvector at 43.6 deg: valley along y
        ((0.0, 1.0, 0.1), 0.0, 0),       # its eigenvector at 46.4 deg, nearer y: the segment crosses it
    ]
    for (hxx, hxy, hyy), strength, expect in cases:
        P = np.zeros((6, 2, 2))
        P[2], P[3], P[4] = hxx, hxy, hyy
        P[5] = d
        seg, typ, n = oracle_lib.marching_creases(P, strength, 2)
        got = int(typ[0, 0, 0]) if n else 0
        assert got == expect, ((hxx, hxy, hyy), strength, got)


def test_hausdorff_by_hand(oracle_lib):
    h = oracle_lib.segment_hausdorff
    assert h([0, 0, 1, 0], [0, 0.5, 1, 0.5]) == 0.5                 # parallel, offset 1/2
    assert math.isclose(h([0, 0, 1, 0], [0, 0, 3, 0]), 0.0)          # contained
    assert math.isclose(h([0, 0, 3, 0], [0, 0, 1, 0]), 2.0)          # directed: the far end of A
    assert math.isclose(h([0, 1, 0, 2], [0, 0, 1, 0]), 2.0)
    assert math.isclose(h([2, 1, 2, 1], [0, 0, 1, 0]), math.sqrt(2))  # a point


def test_match_measures(oracle_lib):
    """Reconstruction equal to the ground truth: E = 0, p = 1; shifted by
    0.3 px across: E = 0.3; beyond the 6 px neighbourhood: not detected;
    another type never matches."""
    H, W = 20, 30
    seg = np.zeros((H - 1, W - 1, 2, 4))
    typ = np.zeros((H - 1, W - 1, 2), np.int8)
    gt = []
    for x in range(5, 20):          # a horizontal crease at y = 10.4, one piece per cell
        seg[10, x, 0] = [x, 10.4, x + 1, 10.4]
        typ[10, x, 0] = 1
        gt.append([x + 0.25, 10.4, x + 0.75, 10.4])
    gt = np.array(gt)
    gtt = np.ones(len(gt), np.int32)
    d, mt = oracle_lib.crease_match(seg, typ, gt, gtt, 6.0)
    E, p = oracle_lib.crease_scores(d)
    assert E == 0.0 and p == 1.0 and np.all(mt >= 0)
    d, _ = oracle_lib.crease_match(seg, typ, gt + [0, 0.3, 0, 0.3], gtt, 6.0)
    assert np.allclose(d, 0.3, atol=1e-12)
    d, _ = oracle_lib.crease_match(seg, typ, gt + [0, 6.5, 0, 6.5], gtt, 6.0)
    assert np.all(d == -1.0) and oracle_lib.crease_scores(d)[1] == 0.0
    d, _ = oracle_lib.crease_match(seg, typ, gt, -gtt, 6.0)
    assert np.all(d == -1.0)
    # among two candidates the one of least distance wins
    seg[12, 5, 1] = [5, 12.0, 6, 12.0]
    typ[12, 5, 1] = 1
    d, mt = oracle_lib.crease_match(seg, typ, np.array([[5.25, 11.9, 5.75, 11.9]]), np.ones(1, np.int32), 6.0)
    assert math.isclose(d[0], 0.1, abs_tol=1e-12) and mt[0] == 2 * (12 * (W - 1) + 5) + 1


def test_extraction_transposes(oracle_lib):
    """D4: transposing the image transposes the set of segments."""
    from paper_1611_06906_amd import synth
    u = synth.creases(40, 44, 2, seed=5)
    def segset(img):
        seg, typ, n = oracle_lib.creases(img, 1.0, 0.0, 2)
        out = set()
        for (y, x, k) in np.argwhere(typ != 0):
            a, b = tuple(np.round(seg[y, x, k, :2], 9)), tuple(np.round(seg[y, x, k, 2:], 9))
            out.add((min(a, b), max(a, b), int(typ[y, x, k])))
        return out
    s1 = segset(u)
    s2 = segset(np.ascontiguousarray(u.T))
    tr = set()
    for a, b, t in s2:
        a2, b2 = (a[1], a[0]), (b[1], b[0])
        tr.add((min(a2, b2), max(a2, b2), t))
    assert len(s1) > 10 and s1 == tr


def test_extraction_finds_a_curved_ridge(oracle_lib):
    """A bright parabola-shaped ridge whose height varies slowly along it
    (so that d changes sign across the crest). Near the vertex, where the
    ridge is level, the ridge segments lie on the generating curve; where it
    tilts, the height ridge of a profile taken along y departs from that
    curve by a fraction of a pixel. The crest is found along all of it."""
    H, W = 64, 72
    y, x = np.mgrid[0:H, 0:W].astype(float)
    yc = 20 + 0.01 * (x - 36) ** 2
    amp = 0.5 + 0.004 * x
    u = 0.2 + amp * np.exp(-((y - yc) ** 2) / (2 * 2.0 ** 2))
    seg, typ, n = oracle_lib.creases(u, 1.0, 0.0, 0)
    pts = []
    for (yy, xx, k) in np.argwhere(typ == 1):
        pts.append(0.5 * (seg[yy, xx, k, :2] + seg[yy, xx, k, 2:]))
    pts = np.array(pts)
    dev = np.abs(pts[:, 1] - (20 + 0.01 * (pts[:, 0] - 36) ** 2))
    near = (pts[:, 0] > 26) & (pts[:, 0] < 46)      # slope below 0.2
    assert near.sum() >= 18 and np.median(dev[near]) < 0.1 and dev[near].max() < 0.3
    xs = np.arange(6, W - 6)
    gt = np.stack([xs, 20 + 0.01 * (xs - 36) ** 2, xs + 1, 20 + 0.01 * (xs + 1 - 36) ** 2], axis=1).astype(float)
    d, _ = oracle_lib.crease_match(seg, typ, gt, np.ones(len(gt), np.int32), 6.0)
    E, p = oracle_lib.crease_scores(d)
    assert p > 0.95 and E < 0.35
