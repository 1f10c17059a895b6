"""Seeded synthetic inputs and workload parameter sets.

This module draws images; it contains none of the filter's arithmetic.
Both the FP64 oracle (through the tests) and the HIP path read the same
float32 arrays produced here.

The paper measured on images that are not available (concentric rings,
a simulated occluded vessel, infrared fundus ROIs; Sec. 4.1-4.3). The
generators below stand in for them with the same kind of structure:
bright or dark creases with Gaussian cross-sections at several widths,
additive Gaussian noise, intensities clipped to [0, 1].

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64), computes
in float64 and returns a C-contiguous float32 array.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage

RIDGE, VALLEY, BOTH = 0, 1, 2


# --------------------------------------------------------------------------
# crease rendering: every pixel takes the profile of its nearest crease
# --------------------------------------------------------------------------
def _render_nearest(H, W, pts, normals, amp, width, reach=5.0):
    """Profile image from densely sampled crease points.

    pts: (K, 2) float (x, y) samples along all creases, spacing <= 0.5 px.
    normals: (K, 2) unit normals of the crease at each sample.
    amp, width: (K,) signed amplitude and Gaussian width of the crease a
    sample belongs to. A pixel takes the profile of the crease sample whose
    rasterised position is nearest (Euclidean distance transform), with
    the distance refined by projecting onto that sample's normal.
    """
    out = np.zeros((H, W), np.float64)
    if len(pts) == 0:
        return out
    ix = np.rint(pts[:, 0]).astype(np.int64)
    iy = np.rint(pts[:, 1]).astype(np.int64)
    inside = (ix >= 0) & (ix < W) & (iy >= 0) & (iy < H)
    if not inside.any():
        return out
    k_in = np.nonzero(inside)[0]
    owner = np.full((H, W), -1, np.int64)
    owner[iy[k_in], ix[k_in]] = k_in          # last sample wins, deterministic
    free = owner < 0
    _, (ny, nx) = ndimage.distance_transform_edt(free, return_indices=True)
    k = owner[ny, nx]
    yy, xx = np.mgrid[0:H, 0:W]
    dx = xx - pts[k, 0]
    dy = yy - pts[k, 1]
    d = np.abs(dx * normals[k, 0] + dy * normals[k, 1])
    w = width[k]
    prof = amp[k] * np.exp(-(d * d) / (2.0 * w * w))
    prof[d > reach * w] = 0.0
    return prof


def _bezier_samples(p0, p1, p2, spacing=0.5):
    """Points and unit normals along a quadratic Bezier curve."""
    chord = np.linalg.norm(p1 - p0) + np.linalg.norm(p2 - p1)
    n = max(8, int(math.ceil(chord / spacing)) + 1)
    t = np.linspace(0.0, 1.0, n)[:, None]
    pts = (1 - t) ** 2 * p0 + 2 * (1 - t) * t * p1 + t ** 2 * p2
    tan = 2 * (1 - t) * (p1 - p0) + 2 * t * (p2 - p1)
    tn = np.linalg.norm(tan, axis=1, keepdims=True)
    tn[tn == 0] = 1.0
    tan = tan / tn
    nrm = np.stack([-tan[:, 1], tan[:, 0]], axis=1)
    return pts, nrm


def creases(H, W, n_creases, seed, *, background=0.2, amplitude=0.6,
            width_range=(1.0, 3.0), control_range=(0.1, 0.9),
            signs="bright", noise=0.05, ground_truth=False):
    """Quadratic-Bezier creases with Gaussian cross-section plus noise.

    signs: "bright" (ridges), or "mixed" (alternating bright / dark,
    so half of the creases are ridges and half valleys).
    ground_truth: also return the noise-free image (clipped to [0, 1]) and
    the centreline of every crease as an (K, 2) array of (x, y) samples less
    than 1 px apart, with its sign (+1 ridge, -1 valley), as
    (image, clean, [(polyline, sign), ...]). The noisy image is the same
    either way.
    """
    rng = np.random.default_rng(seed)
    lo, hi = control_range
    all_p, all_n, all_a, all_w, lines = [], [], [], [], []
    for c in range(n_creases):
        ctrl = rng.uniform(lo, hi, size=(3, 2)) * np.array([W - 1, H - 1])
        w = rng.uniform(*width_range)
        sgn = 1.0 if (signs == "bright" or c % 2 == 0) else -1.0
        p, nrm = _bezier_samples(ctrl[0], ctrl[1], ctrl[2])
        all_p.append(p)
        all_n.append(nrm)
        all_a.append(np.full(len(p), sgn * amplitude))
        all_w.append(np.full(len(p), w))
        lines.append((p, sgn))
    prof = _render_nearest(H, W, np.concatenate(all_p), np.concatenate(all_n),
                           np.concatenate(all_a), np.concatenate(all_w))
    clean = background + prof
    img = clean + rng.normal(0.0, noise, size=(H, W))
    img = np.ascontiguousarray(np.clip(img, 0.0, 1.0).astype(np.float32))
    if ground_truth:
        return img, np.ascontiguousarray(np.clip(clean, 0.0, 1.0).astype(np.float32)), lines
    return img


def fundus(H, W, seed, *, noise=0.03, max_walks=256, ground_truth=False):
    """Fundus-like image: bright vignetted disc with a dark vessel tree.

    The tree grows from 4 roots on the disc rim by persistent random walks
    (1 px steps, heading noise N(0, 0.1 rad), branching probability 0.01
    per step) whose radius tapers from 8 px to 1 px; each tree has a
    contrast drawn from U[0.15, 0.35] and a Gaussian cross-section of
    width radius / sqrt(2).
    ground_truth: also return the noise-free image and the centreline of
    every walk (valleys, sign -1), as for creases().
    """
    rng = np.random.default_rng(seed)
    cy, cx = (H - 1) / 2.0, (W - 1) / 2.0
    R = 0.45 * min(H, W)
    yy, xx = np.mgrid[0:H, 0:W]
    rr = np.hypot(xx - cx, yy - cy)
    disc = 1.0 / (1.0 + np.exp(-(R - rr) / 4.0))
    base = (0.1 + 0.6 * disc) * (1.0 - 0.3 * np.minimum(rr / R, 1.0) ** 2)

    pts, nrms, amps, wids = [], [], [], []
    walks = []
    lmax = 1.2 * R
    for _ in range(4):
        a = rng.uniform(0, 2 * math.pi)
        start = np.array([cx + 0.95 * R * math.cos(a), cy + 0.95 * R * math.sin(a)])
        head = a + math.pi + rng.normal(0, 0.2)
        contrast = rng.uniform(0.15, 0.35)
        walks.append((start, head, 8.0, lmax, contrast))
    done = 0
    lines = []
    while walks and done < max_walks:
        pos, head, r0, length, contrast = walks.pop(0)
        done += 1
        pos = pos.copy()
        steps = int(length)
        line = []
        for s in range(steps):
            rad = r0 + (1.0 - r0) * (s / max(steps - 1, 1))
            if rad < 1.0:
                break
            tan = np.array([math.cos(head), math.sin(head)])
            pts.append(pos.copy())
            line.append(pos.copy())
            nrms.append(np.array([-tan[1], tan[0]]))
            amps.append(-contrast)
            wids.append(rad / math.sqrt(2.0))
            if rng.uniform() < 0.01 and len(walks) + done < max_walks:
                turn = rng.uniform(0.3, 0.8) * (1 if rng.uniform() < 0.5 else -1)
                walks.append((pos.copy(), head + turn, max(1.0, 0.7 * rad),
                              length - s, contrast))
            head += rng.normal(0.0, 0.1)
            pos += tan
            if math.hypot(pos[0] - cx, pos[1] - cy) > R:
                break
        if len(line) >= 2:
            lines.append((np.array(line), -1.0))
    if pts:
        P = np.array(pts)
        Nn = np.array(nrms)
        prof = _render_nearest(H, W, P, Nn, np.array(amps), np.array(wids), reach=4.0)
    else:
        prof = 0.0
    clean = base + prof
    img = clean + rng.normal(0.0, noise, size=(H, W))
    img = np.ascontiguousarray(np.clip(img, 0.0, 1.0).astype(np.float32))
    if ground_truth:
        return img, np.ascontiguousarray(np.clip(clean, 0.0, 1.0).astype(np.float32)), lines
    return img


# --------------------------------------------------------------------------
# workloads: image recipe plus filter parameters
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    H: int
    W: int
    sigmas: list
    mode: int
    cycles: int
    substeps: int
    lam: float = 0.005
    rho: float = 0.5
    beta: float = 0.5
    tau_max: float = 0.05
    seed: int = 0
    extra: dict = field(default_factory=dict)

    def sigmas_f32(self):
        return np.asarray(self.sigmas, dtype=np.float32)

    def image(self):
        return make_image(self)

    def ground_truth(self):
        """(noisy image, noise-free image, centrelines) of this workload."""
        return make_image(self, ground_truth=True)

    @property
    def px_substeps(self):
        return self.H * self.W * self.cycles * self.substeps


def ridges128(seed=0, H=128, W=128):
    """Small plain-method case: 3 bright ridges (width U[1,3]) on 0.2."""
    return Workload("ridges128", H, W, [1.0, 1.5, 2.0, 3.0], RIDGE, 5, 10, seed=seed)


def fundus1024(seed=0, H=1024, W=1024):
    """Fundus-like vessel tree, 6 log-spaced scales 1..8, valley mode."""
    return Workload("fundus1024", H, W, [8.0 ** (k / 5.0) for k in range(6)], VALLEY,
                    20, 15, seed=seed)


def creases4096(seed=0, H=4096, W=4096, cycles=30):
    """Roofline-scale case: 64 bright and dark creases of width U[1,16],
    8 log-spaced scales 1..16, ridge+valley mode, 30 cycles of 20 substeps."""
    return Workload("creases4096", H, W, [16.0 ** (k / 7.0) for k in range(8)], BOTH,
                    cycles, 20, seed=seed)


WORKLOADS = {"ridges128": ridges128, "fundus1024": fundus1024, "creases4096": creases4096}


def make_image(w: Workload, ground_truth=False):
    gt = dict(ground_truth=ground_truth)
    if w.name == "ridges128":
        n = max(1, int(round(3 * math.sqrt(w.H * w.W / 128.0 ** 2))))
        return creases(w.H, w.W, n, w.seed, **gt)
    if w.name == "fundus1024":
        return fundus(w.H, w.W, w.seed, **gt)
    if w.name == "creases4096":
        n = max(2, int(round(64 * math.sqrt(w.H * w.W / 4096.0 ** 2))))
        return creases(w.H, w.W, n, w.seed, background=0.5, amplitude=0.4,
                       width_range=(1.0, 16.0), control_range=(0.0, 1.0), signs="mixed", **gt)
    raise KeyError(w.name)


def batch_of_images(n_images=256, seed=4, size_range=(256, 1536)):
    """Uneven batch: sizes U{256..1536}, config-1 creases with per-image seed
    1000+i (crease count scaled with sqrt(area)), ridge or valley with p=1/2
    (a valley image is 1 - a ridge image), cycles U{5..25}."""
    rng = np.random.default_rng(seed)
    Hs = rng.integers(size_range[0], size_range[1] + 1, n_images)
    Ws = rng.integers(size_range[0], size_range[1] + 1, n_images)
    modes = np.where(rng.uniform(size=n_images) < 0.5, RIDGE, VALLEY)
    cycles = rng.integers(5, 26, n_images)
    specs = []
    for i in range(n_images):
        specs.append(dict(H=int(Hs[i]), W=int(Ws[i]), mode=int(modes[i]),
                          cycles=int(cycles[i]), seed=1000 + i))
    return specs


def batch_image(spec):
    H, W = spec["H"], spec["W"]
    n = max(1, int(round(3 * math.sqrt(H * W / 128.0 ** 2))))
    img = creases(H, W, n, spec["seed"])
    if spec["mode"] == VALLEY:
        img = np.ascontiguousarray((1.0 - img.astype(np.float64)).astype(np.float32))
    return img


# --------------------------------------------------------------------------
# volumes: tubes along quadratic Bezier curves in 3-D
# --------------------------------------------------------------------------
def _bezier3_samples(p0, p1, p2, spacing=0.5):
    """Points and unit tangents along a quadratic Bezier curve in (x, y, z)."""
    chord = np.linalg.norm(p1 - p0) + np.linalg.norm(p2 - p1)
    n = max(8, int(math.ceil(chord / spacing)) + 1)
    t = np.linspace(0.0, 1.0, n)[:, None]
    pts = (1 - t) ** 2 * p0 + 2 * (1 - t) * t * p1 + t ** 2 * p2
    tan = 2 * (1 - t) * (p1 - p0) + 2 * t * (p2 - p1)
    tn = np.linalg.norm(tan, axis=1, keepdims=True)
    tn[tn == 0] = 1.0
    return pts, tan / tn


def tubes3d(D, H, W, n_tubes, seed, *, background=0.2, amplitude=0.6, width_range=(1.0, 2.5),
            control_range=(0.1, 0.9), signs="bright", noise=0.05, reach=5.0):
    """Volume [D][H][W] of tubes with Gaussian cross-section plus noise.

    Each tube follows a quadratic Bezier curve with control points uniform in
    the control_range box of the volume; every voxel takes the profile
    amp exp(-d^2 / 2 w^2) of its nearest centreline sample (3-D Euclidean
    distance transform), d its distance from that sample's tangent line (0
    beyond reach w). signs: "bright", or "mixed" (alternating bright / dark).
    """
    rng = np.random.default_rng(seed)
    lo, hi = control_range
    pts, tans, amps, wids = [], [], [], []
    for c in range(n_tubes):
        ctrl = rng.uniform(lo, hi, size=(3, 3)) * np.array([W - 1, H - 1, D - 1])
        w = rng.uniform(*width_range)
        sgn = 1.0 if (signs == "bright" or c % 2 == 0) else -1.0
        p, t = _bezier3_samples(ctrl[0], ctrl[1], ctrl[2])
        pts.append(p)
        tans.append(t)
        amps.append(np.full(len(p), sgn * amplitude))
        wids.append(np.full(len(p), w))
    prof = np.zeros((D, H, W))
    if n_tubes:
        P, T, A, Wd = (np.concatenate(a) for a in (pts, tans, amps, wids))
        ix, iy, iz = (np.rint(P[:, k]).astype(np.int64) for k in range(3))
        inside = (ix >= 0) & (ix < W) & (iy >= 0) & (iy < H) & (iz >= 0) & (iz < D)
        k_in = np.nonzero(inside)[0]
        if len(k_in):
            owner = np.full((D, H, W), -1, np.int64)
            owner[iz[k_in], iy[k_in], ix[k_in]] = k_in     # last sample wins, deterministic
            _, (nz, ny, nx) = ndimage.distance_transform_edt(owner < 0, return_indices=True)
            k = owner[nz, ny, nx]
            del nz, ny, nx
            zz, yy, xx = np.meshgrid(np.arange(D), np.arange(H), np.arange(W), indexing="ij")
            vx, vy, vz = xx - P[k, 0], yy - P[k, 1], zz - P[k, 2]
            del zz, yy, xx
            along = vx * T[k, 0] + vy * T[k, 1] + vz * T[k, 2]
            d2 = np.maximum(vx * vx + vy * vy + vz * vz - along * along, 0.0)
            w = Wd[k]
            prof = A[k] * np.exp(-d2 / (2.0 * w * w))
            prof[d2 > (reach * w) ** 2] = 0.0
    img = background + prof + rng.normal(0.0, noise, size=(D, H, W))
    return np.ascontiguousarray(np.clip(img, 0.0, 1.0).astype(np.float32))


def noise_image(H, W, seed, lo=0.0, hi=1.0):
    """Uniform white noise, for stage-level tests."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(lo, hi, size=(H, W)).astype(np.float32))
