"""GPU parity of the filter on volumes (the 3-D extension of Sec. 5) against
the FP64 oracle, stage by stage and end to end:

- scale selection: c, the tube measure's maximum and the indices (exact
  except at stated near-ties, decided from the oracle's data alone);
- the integrated Hessian H_rho at the oracle's indices;
- the tensor: its action on symmetric matrices against the oracle's literal
  9 x 9 D, from the same H_rho;
- one FED cycle from the same tensor, and the whole filter in every mode,
  including the smallest and ragged volume shapes.

Tolerances: the plain filter's bar (final max-abs <= 2e-4, relative L2 <=
1e-5 on [0, 1] intensities); the stages are held far tighter.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MAXABS, RELL2 = 2e-4, 1e-5
TAU3 = 1.0 / 27.0


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_06906_amd import mf4d, synth
    import oracle
    mf4d.lib()
    oracle.lib()
    return dict(torch=torch, m=mf4d, synth=synth, o=oracle, dev=torch.device("cuda:0"))


def _to(env, a):
    return env["torch"].from_numpy(np.ascontiguousarray(a)).to(env["dev"])


def _err(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.abs(got - ref).max()), float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def _volume(env, shape, seed, mode):
    signs = {0: "bright", 1: "bright", 2: "mixed"}[mode]
    v = env["synth"].tubes3d(*shape, n_tubes=4, seed=seed, signs=signs)
    return np.ascontiguousarray(1.0 - v) if mode == 1 else v   # VALLEY: dark tubes


def _sign_tie(n, S):
    """The oracle's sign test or magnitude order is itself near a tie: one of
    the two largest-magnitude eigenvalues is near 0, or the two smallest
    magnitudes nearly coincide (which of them is n2 then decides the sign)."""
    a = np.sort(np.abs(n))
    return a[1] <= 1e-5 * S or a[2] <= 1e-5 * S or (a[1] - a[0]) <= 1e-5 * S


def _near_ties(env, u, sigmas, gi, sel):
    """Voxels whose GPU index differs from the oracle's; the ones that are
    not near-ties (V gap > 1e-5 + 1e-4 Vmax, and no sign tie)."""
    o = env["o"]
    diff = np.argwhere(gi != sel["idx"])
    hess = {}
    bad = []
    for z, y, x in diff:
        g, r = int(gi[z, y, x]), int(sel["idx"][z, y, x])
        V = sel["V"][:, z, y, x]
        if V[g] >= V[r] - (1e-5 + 1e-4 * V[r]):
            continue
        if g not in hess:
            hess[g] = o.derivatives3(o.blur3(u, sigmas[g]))[3:]
        h = hess[g][:, z, y, x] * float(np.float32(sigmas[g])) ** 2
        A = np.array([[h[0], h[3], h[4]], [h[3], h[1], h[5]], [h[4], h[5], h[2]]])
        if _sign_tie(np.linalg.eigvalsh(A), np.linalg.norm(A)):
            continue
        bad.append((int(z), int(y), int(x), g, r))
    return len(diff), bad


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_scale_select3_parity(env, mode):
    m, o, torch = env["m"], env["o"], env["torch"]
    sig = [1.0, 1.5, 2.2, 3.0]
    u = _volume(env, (40, 44, 48), 11 + mode, mode)
    _log(f"[3d select] mode {mode} shape {u.shape}")
    p = m.Params(sig, mode=mode, tau_max=TAU3)
    idx = torch.empty(u.shape, dtype=torch.uint8, device=env["dev"])
    vmax = torch.empty(u.shape, dtype=torch.float32, device=env["dev"])
    c = torch.empty(1, dtype=torch.float32, device=env["dev"])
    m.mf4d3d_scale_select(_to(env, u), p, idx, vmax, c)
    torch.cuda.synchronize()
    sel = o.scale_select3(u, sig, mode)
    assert math.isclose(float(c.item()), sel["c"], rel_tol=1e-5)
    gi = idx.cpu().numpy()
    ndiff, bad = _near_ties(env, u, sig, gi, sel)
    _log(f"[3d select] mode {mode}: {ndiff} index differences, {len(bad)} not near-ties")
    assert not bad, bad[:5]
    assert ndiff <= 1e-3 * u.size
    vref = sel["V"].max(axis=0)
    assert np.abs(vmax.cpu().numpy() - vref).max() <= 1e-5 + 1e-4 * vref.max()
    assert vref.max() > 0.1   # the tubes respond


def test_scale_select3_fixed_c_and_zero(env):
    """c given as a parameter is used as is; a constant volume has S = 0,
    c = 0 and index 0 everywhere."""
    m, o, torch = env["m"], env["o"], env["torch"]
    sig = [1.0, 2.0]
    u = _volume(env, (20, 22, 24), 5, 2)
    p = m.Params(sig, mode=2, c=0.07, tau_max=TAU3)
    idx = torch.empty(u.shape, dtype=torch.uint8, device=env["dev"])
    c = torch.empty(1, dtype=torch.float32, device=env["dev"])
    m.mf4d3d_scale_select(_to(env, u), p, idx, None, c)
    sel = o.scale_select3(u, sig, 2, c=0.07)
    assert float(c.item()) == np.float32(0.07)
    ndiff, bad = _near_ties(env, u, sig, idx.cpu().numpy(), sel)
    assert not bad
    flat = np.full((6, 7, 8), 0.4, np.float32)
    idx = torch.ones(flat.shape, dtype=torch.uint8, device=env["dev"])
    m.mf4d3d_scale_select(_to(env, flat), m.Params(sig, tau_max=TAU3), idx, None, c)
    torch.cuda.synchronize()
    assert float(c.item()) == 0.0 and int(idx.max().item()) == 0


@pytest.mark.parametrize("rho,shape", [(0.5, (30, 33, 37)), (0.0, (30, 33, 37)), (0.3, (70, 20, 40)),
                                       (0.5, (70, 20, 40)), (1.0, (30, 33, 37))])
def test_tensor3_parity(env, rho, shape):
    """H_rho at the oracle's indices against the oracle (relative to its
    largest component): integration radii 0, 1 and 2 (one fused z-marching
    kernel; 70 planes take three z segments, the last one ragged) and 3 (the
    separable passes)."""
    m, o, torch = env["m"], env["o"], env["torch"]
    sig = [1.0, 1.5, 2.2]
    u = _volume(env, shape, 21, 2)
    sel = o.scale_select3(u, sig, 2)
    ref = o.tensor3(u, sel["idx"], sig, rho=rho)
    p = m.Params(sig, mode=2, rho=rho, tau_max=TAU3)
    hr = torch.empty((6,) + u.shape, dtype=torch.float32, device=env["dev"])
    m.mf4d3d_tensor(_to(env, u), _to(env, sel["idx"]), p, hr)
    torch.cuda.synchronize()
    err = np.abs(hr.cpu().numpy() - ref).max()
    _log(f"[3d tensor] rho {rho} {shape}: max err {err:.3e} of scale {np.abs(ref).max():.3e}")
    assert err <= 2e-6 * np.abs(ref).max() + 1e-9


@pytest.mark.parametrize("rho", [0.5, 1.0])
def test_tensor3_clamps_indices(env, rho):
    """Scale indices of nscales or more count as nscales - 1 (the fused
    integration at radius 2 and the separable passes at radius 3): the same
    H_rho as the oracle's on the clamped indices."""
    m, o, torch = env["m"], env["o"], env["torch"]
    sig = [1.0, 1.6]
    u = _volume(env, (9, 21, 70), 5, 2)
    rng = np.random.default_rng(3)
    idx = rng.integers(0, 2, size=u.shape).astype(np.uint8)
    big = rng.random(u.shape) < 0.3
    idx[big] = rng.choice(np.array([2, 7, 255], np.uint8), size=int(big.sum()))
    ref = o.tensor3(u, np.minimum(idx, len(sig) - 1), sig, rho=rho)
    p = m.Params(sig, mode=2, rho=rho, tau_max=TAU3)
    hr = torch.empty((6,) + u.shape, dtype=torch.float32, device=env["dev"])
    m.mf4d3d_tensor(_to(env, u), _to(env, idx), p, hr)
    torch.cuda.synchronize()
    err = np.abs(hr.cpu().numpy() - ref).max()
    _log(f"[3d tensor clamp] rho {rho}: max err {err:.3e} of scale {np.abs(ref).max():.3e}")
    assert err <= 2e-6 * np.abs(ref).max() + 1e-9


def _sym(p6):
    """The symmetric 3 x 3 matrix of six entries xx, yy, zz, xy, xz, yz."""
    return np.array([[p6[0], p6[3], p6[4]], [p6[3], p6[1], p6[5]], [p6[4], p6[5], p6[2]]])


@pytest.mark.parametrize("mode,lam", [(0, 0.005), (1, 0.01), (2, 0.005), (2, math.inf), (2, 1e-5)])
def test_dtensor3_action_parity(env, mode, lam):
    """The tensor planes against the oracle's literal 9 x 9 D built from the
    same H_rho: P equals D applied to the identity, and (P h + h P) / 2
    equals D h for symmetric h. In BOTH mode P is the inverse of
    I + H^2 / lambda^2 where |H|^2 / lambda^2 <= 1e6 and comes from the
    eigenpairs elsewhere (lambda = 1e-5: mostly the latter, both in a wave)."""
    m, o, torch = env["m"], env["o"], env["torch"]
    rng = np.random.default_rng(7 + mode)
    shape = (5, 6, 7)
    hr = rng.normal(scale=0.01, size=(6,) + shape).astype(np.float32)
    # a few degenerate voxels: equal eigenvalues, zero matrix
    hr[:, 0, 0, 0] = 0.0
    hr[:, 0, 0, 1] = [0.01, 0.01, 0.01, 0, 0, 0]
    hr[:, 0, 0, 2] = [0.02, 0.02, -0.01, 0, 0, 0]
    p = m.Params([1.0], mode=mode, lam=lam, tau_max=TAU3)
    dp = torch.empty(shape + (6,), dtype=torch.float32, device=env["dev"])
    m.mf4d3d_dtensor(_to(env, hr), p, dp)
    torch.cuda.synchronize()
    dp = dp.cpu().numpy().astype(np.float64)
    Dall = o.dtensor3(hr.astype(np.float64), float(np.float32(lam)), mode)
    eye = np.eye(3).reshape(9)
    worst, worst_p = 0.0, 0.0
    for z, y, x in np.ndindex(shape):
        P = _sym(dp[z, y, x])
        Dm = Dall[z, y, x].reshape(9, 9)
        worst_p = max(worst_p, np.abs(P - (Dm @ eye).reshape(3, 3)).max())
        for _ in range(3):
            h = rng.normal(size=(3, 3))
            h = h + h.T
            got = 0.5 * (P @ h + h @ P)
            ref = (Dm @ h.reshape(9)).reshape(3, 3)
            worst = max(worst, np.abs(got - ref).max() / np.abs(h).max())
    _log(f"[3d dtensor] mode {mode} lam {lam}: action err {worst:.3e}, P err {worst_p:.3e}")
    assert worst <= 2e-6 and worst_p <= 1e-6


def test_fed_cycle3_parity(env):
    """One cycle of 8 kappa-ordered substeps from the same H_rho: the GPU's
    tensor planes and substeps against the oracle's literal D and scatter
    form of L^T D L."""
    m, o, torch = env["m"], env["o"], env["torch"]
    sig = [1.0, 2.0]
    u = _volume(env, (22, 25, 70), 3, 2)
    sel = o.scale_select3(u, sig, 2)
    hr = o.tensor3(u, sel["idx"], sig).astype(np.float32)
    taus, _, _ = o.fed_schedule(8, TAU3)
    p = m.Params(sig, mode=2, tau_max=TAU3)
    dp = torch.empty(u.shape + (6,), dtype=torch.float32, device=env["dev"])
    m.mf4d3d_dtensor(_to(env, hr), p, dp)
    ug = _to(env, u)
    m.mf4d3d_fed_cycle_tensor(ug, dp, taus)
    torch.cuda.synchronize()
    ref = o.fed_cycle3(u, o.dtensor3(hr.astype(np.float64), float(np.float32(0.005)), 2), taus)
    ea, er = _err(ug.cpu().numpy(), ref)
    _log(f"[3d cycle] max-abs {ea:.3e} rel-l2 {er:.3e}")
    assert ea <= 2e-5 and er <= 1e-6
    assert math.isclose(float(ug.double().sum().item()), float(u.astype(np.float64).sum()), rel_tol=1e-6)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_filter3_parity(env, mode):
    m, o, torch = env["m"], env["o"], env["torch"]
    sig = [1.0, 1.5, 2.2]
    u = _volume(env, (24, 28, 33), 41 + mode, mode)
    _log(f"[3d filter] mode {mode} shape {u.shape}")
    p = m.Params(sig, mode=mode, cycles=2, substeps=8, tau_max=TAU3)
    ui = _to(env, u)
    uo = torch.empty_like(ui)
    m.mf4d3d_filter(ui, uo, p)
    torch.cuda.synchronize()
    ref, rec = o.filter3(u, sig, mode, cycles=2, substeps=8, record=True)
    ea, er = _err(uo.cpu().numpy(), ref)
    _log(f"[3d filter] mode {mode}: max-abs {ea:.3e} rel-l2 {er:.3e}")
    assert ea <= MAXABS and er <= RELL2
    # the first cycle's indices: exact up to near-ties
    idx = torch.empty(u.shape, dtype=torch.uint8, device=env["dev"])
    m.mf4d3d_scale_select(ui, p, idx)
    ndiff, bad = _near_ties(env, u, sig, idx.cpu().numpy(), o.scale_select3(u, sig, mode))
    assert not bad
    assert np.array_equal(ui.cpu().numpy(), u)   # the input is left alone


def test_filter3_full_size_block(env):
    """One cycle of the bench's volume filter (256^3, 24 tubes, 4 scales
    1..3.375, both modes, 10 substeps) against the oracle on a 96^3 block of
    it, given the GPU's image-wide c: the selection within 12 voxels of the
    block's faces and the output within 34 (the derivative support 11 + 1,
    the integration radius 2 and 2 per substep) depend only on the block, so
    there the oracle's values are those of the whole volume. Indices exact
    up to stated near-ties; the output within the image tolerances outside
    the reach of such picks."""
    import time
    from scipy import ndimage
    m, o, torch = env["m"], env["o"], env["torch"]
    D = H = W = 256
    v = env["synth"].tubes3d(D, H, W, 24, seed=0, signs="mixed", width_range=(1.0, 3.0))
    sig = [1.5 ** k for k in range(4)]
    p = m.Params(sig, mode=2, cycles=1, substeps=10, tau_max=TAU3)
    vi = _to(env, v)
    vo = torch.empty_like(vi)
    m.mf4d3d_filter(vi, vo, p)
    idx = torch.empty(v.shape, dtype=torch.uint8, device=env["dev"])
    c = torch.empty(1, dtype=torch.float32, device=env["dev"])
    m.mf4d3d_scale_select(vi, p, idx, None, c)
    torch.cuda.synchronize()
    gc = float(c.item())
    z0 = y0 = x0 = 96
    n = 96
    blk = np.ascontiguousarray(v[z0:z0 + n, y0:y0 + n, x0:x0 + n])
    t0 = time.time()
    sel = o.scale_select3(blk, sig, 2, c=gc)
    ref = o.filter3(blk, sig, 2, c=gc, cycles=1, substeps=10)
    _log(f"[3d block] oracle on 96^3 in {time.time() - t0:.1f}s, c {gc:.6g}")
    a, b = 12, n - 12
    gi = idx.cpu().numpy()[z0:z0 + n, y0:y0 + n, x0:x0 + n]
    sel_in = np.zeros(gi.shape, bool)
    sel_in[a:b, a:b, a:b] = True
    gi_in = np.where(sel_in, gi, sel["idx"])   # the faces' zone is the block's own, not the volume's
    ndiff, bad = _near_ties(env, blk, sig, gi_in, sel)
    assert not bad, bad[:5]
    flips = gi_in != sel["idx"]
    flips_in = flips
    got = vo.cpu().numpy()[z0:z0 + n, y0:y0 + n, x0:x0 + n].astype(np.float64)
    r = 34
    reach = 2 + 2 * 10
    near = ndimage.maximum_filter(flips.astype(np.uint8), size=2 * reach + 1) > 0
    inner = np.zeros_like(near)
    inner[r:n - r, r:n - r, r:n - r] = True
    d = np.abs(got - ref)
    e_far = float(d[inner & ~near].max())
    rel = float(np.linalg.norm((got - ref)[inner]) / np.linalg.norm(ref[inner]))
    _log(f"[3d block] {int(flips_in.sum())} index differences in the selection interior ({int(sel_in.sum())} voxels); "
         f"output interior {int(inner.sum())} voxels: max-abs {float(d[inner].max()):.3e} "
         f"({e_far:.3e} outside the reach of differing picks), rel-L2 {rel:.3e}")
    assert e_far <= MAXABS and rel <= RELL2


def test_filter3_small_lambda(env):
    """BOTH mode at lambda = 1e-5, where |H_rho|^2 / lambda^2 lies on both
    sides of the bound that chooses between the inverse of
    I + H_rho^2 / lambda^2 and the eigenpairs (about 43% of the voxels of the
    first cycle take the inverse): the whole filter against the oracle."""
    m, o, torch = env["m"], env["o"], env["torch"]
    sig = [1.0, 1.5, 2.2]
    u = _volume(env, (20, 26, 31), 77, 2)
    p = m.Params(sig, mode=2, lam=1e-5, cycles=2, substeps=8, tau_max=TAU3)
    ui = _to(env, u)
    uo = torch.empty_like(ui)
    m.mf4d3d_filter(ui, uo, p)
    torch.cuda.synchronize()
    ref = o.filter3(u, sig, 2, lam=1e-5, cycles=2, substeps=8)
    ea, er = _err(uo.cpu().numpy(), ref)
    _log(f"[3d filter] lambda 1e-5: max-abs {ea:.3e} rel-l2 {er:.3e}")
    assert ea <= MAXABS and er <= RELL2


@pytest.mark.parametrize("shape", [(3, 3, 3), (3, 5, 70), (5, 3, 4), (4, 66, 3)])
def test_filter3_edge_shapes(env, shape):
    """The smallest volumes (one interior voxel or none along an axis) and
    rows shorter or longer than a wave, against the oracle."""
    m, o, torch = env["m"], env["o"], env["torch"]
    rng = np.random.default_rng(sum(shape))
    u = rng.uniform(0.2, 0.8, size=shape).astype(np.float32)
    sig = [1.0, 1.5]
    _log(f"[3d edge] shape {shape}")
    p = m.Params(sig, mode=2, cycles=2, substeps=3, tau_max=TAU3)
    ui = _to(env, u)
    uo = torch.empty_like(ui)
    m.mf4d3d_filter(ui, uo, p)
    torch.cuda.synchronize()
    ref = o.filter3(u, sig, 2, cycles=2, substeps=3)
    ea, er = _err(uo.cpu().numpy(), ref)
    assert ea <= MAXABS and er <= RELL2, (ea, er)


def test_filter3_in_place_and_zero_cycles(env):
    m, torch = env["m"], env["torch"]
    sig = [1.0, 2.0]
    u = _volume(env, (12, 14, 16), 9, 2)
    p = m.Params(sig, mode=2, cycles=1, substeps=5, tau_max=TAU3)
    a = _to(env, u)
    b = torch.empty_like(a)
    m.mf4d3d_filter(a, b, p)
    m.mf4d3d_filter(a, a, p)   # u_out aliases u_in
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    p0 = m.Params(sig, mode=2, cycles=0, substeps=5, tau_max=TAU3)
    c = torch.full_like(a, -1.0)
    m.mf4d3d_filter(_to(env, u), c, p0)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy(), u)
