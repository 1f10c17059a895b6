"""GPU parity of crease extraction (Sec. 3.6) and of its evaluation (Sec. 4)
against the FP64 oracle.

- Field: g, H and d of u_sigma to FP32 accuracy.
- Segments, cell by cell: where the oracle's decision is stable the GPU must
  make the same one (same slots and types) and put the ends where the
  oracle does, within the error that the measured error of d at the
  cell's corners implies for the linear interpolation (first order). A
  decision is a stated near-tie when a corner's d, the mean of the corners
  (saddles), the sign of the stronger eigenvalue's trace, the strength or
  the direction test lie within the FP32 error of the oracle's value.
- Matching: the GPU matcher on the oracle's segments (rounded to float32)
  equals the oracle on the same values, up to near-ties between candidates.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


def _gpu_creases(env, u, sigma_d, strength, mode):
    torch, m = env["torch"], env["m"]
    H, W = u.shape
    field = torch.empty((6, H, W), dtype=torch.float32, device=env["dev"])
    cnt = torch.zeros(1, dtype=torch.int32, device=env["dev"])
    seg, typ = m.mf4d_creases(_to(env, u), sigma_d, strength, mode, count_out=cnt, field_out=field)
    torch.cuda.synchronize()
    return seg.cpu().numpy(), typ.cpu().numpy(), int(cnt.item()), field.cpu().numpy()


def _fragile_cells(P, Pg, strength):
    """Cells whose oracle decision a perturbation of the size of the FP32
    error could change (the oracle's own field P; Pg only sizes the error)."""
    H, W = P.shape[1:]
    err = np.abs(Pg.astype(np.float64) - P)
    d, ed = P[5], 3 * err[5] + 1e-12 * np.abs(P[5]).max()
    eh = 3 * np.maximum(np.maximum(err[2], err[3]), err[4]) + 1e-9 * np.abs(P[2:5]).max()
    frag = np.zeros((H - 1, W - 1), bool)
    for dy in (0, 1):
        for dx in (0, 1):
            sl = (slice(dy, H - 1 + dy), slice(dx, W - 1 + dx))
            frag |= np.abs(d[sl]) <= ed[sl]
            # the stronger eigenvalue's sign (trace near 0), equal magnitudes, the strength
            a, b, c = P[2][sl], P[3][sl], P[4][sl]
            m = 0.5 * (a + c)
            r = np.sqrt(0.25 * (a - c) ** 2 + b * b)
            e = eh[sl]
            frag |= np.abs(m) <= 2 * e
            frag |= r <= 2 * e
            frag |= np.abs(np.abs(m) + r - strength) <= 3 * e
    centre = 0.25 * (d[:-1, :-1] + d[:-1, 1:] + d[1:, :-1] + d[1:, 1:])
    ec = 0.25 * (ed[:-1, :-1] + ed[:-1, 1:] + ed[1:, :-1] + ed[1:, 1:])
    frag |= np.abs(centre) <= ec
    return frag


def _direction_margin(seg, P, y, x, k):
    """|q| / (|v|^2 r) of the oracle's own segment (the cosine of twice the
    angle between it and the eigenvectors): near 0 the direction test is a
    near-tie."""
    H, W = P.shape[1:]
    x0, y0, x1, y1 = seg[y, x, k]
    def interp(px, py, plane):
        # the oracle interpolates along an edge: the end lies on one, so bilinear equals linear there
        fx, fy = px - x, py - y
        p00, p10 = plane[y, x], plane[y, x + 1]
        p01, p11 = plane[y + 1, x], plane[y + 1, x + 1]
        return (1 - fx) * (1 - fy) * p00 + fx * (1 - fy) * p10 + (1 - fx) * fy * p01 + fx * fy * p11
    a = 0.5 * (interp(x0, y0, P[2]) + interp(x1, y1, P[2]))
    b = 0.5 * (interp(x0, y0, P[3]) + interp(x1, y1, P[3]))
    c = 0.5 * (interp(x0, y0, P[4]) + interp(x1, y1, P[4]))
    vx, vy = x1 - x0, y1 - y0
    r = np.sqrt(0.25 * (a - c) ** 2 + b * b)
    q = 0.5 * (a - c) * (vx * vx - vy * vy) + 2 * b * vx * vy
    return abs(q) / max((vx * vx + vy * vy) * r, 1e-300)


@pytest.mark.parametrize("case", ["noisy", "filtered"])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_crease_extraction_parity(env, case, mode):
    o, m, synth = env["o"], env["m"], env["synth"]
    u = synth.creases(120, 150, 5, seed=70 + mode, signs="mixed", width_range=(1.0, 3.0))
    if case == "filtered":
        u = o.filter(u, [1.0, 1.5, 2.0, 3.0], 2, cycles=2, substeps=10).astype(np.float32)
    sigma_d, strength = 1.0, 0.005
    seg, typ, cnt, field = _gpu_creases(env, u, sigma_d, strength, mode)
    P = o.crease_field(u, sigma_d)
    scale = np.abs(P).reshape(6, -1).max(axis=1)
    ferr = np.abs(field - P).reshape(6, -1).max(axis=1)
    assert np.all(ferr <= 2e-6 * scale[[0, 1, 2, 3, 4, 5]] + 1e-12), (ferr, scale)
    rseg, rtyp, rcnt = o.marching_creases(P, strength, mode)
    assert cnt == int((typ != 0).sum())
    frag = _fragile_cells(P, field, strength)
    differ = np.any(typ != rtyp, axis=2)
    # the direction test at the oracle's own segments
    for (y, x, k) in np.argwhere((rtyp != 0) | (typ != 0)):
        if rtyp[y, x, k] != 0 and _direction_margin(rseg, P, y, x, k) <= 1e-4:
            frag[y, x] = True
    bad_type = differ & ~frag
    # ends of segments both sides agree on: first-order bound from the corner errors of d
    same = ~differ & ~frag & np.any(rtyp != 0, axis=2)
    H, W = u.shape
    ed = np.abs(field[5].astype(np.float64) - P[5])
    worst = 0.0
    for (y, x) in np.argwhere(same):
        dc = [P[5][y, x], P[5][y, x + 1], P[5][y + 1, x + 1], P[5][y + 1, x]]
        ec = [ed[y, x], ed[y, x + 1], ed[y + 1, x + 1], ed[y + 1, x]]
        tol = 2 * sum(ec) / min(abs(dc[i] - dc[(i + 1) % 4]) or 1e-300 for i in range(4)
                                if (dc[i] >= 0) != (dc[(i + 1) % 4] >= 0)) + 1e-5
        dev = np.abs(seg[y, x] - rseg[y, x]).max()
        worst = max(worst, dev / tol)
        assert dev <= tol, (y, x, seg[y, x], rseg[y, x], tol)
    _log(f"creases {case} mode {mode}: GPU {cnt} / oracle {rcnt} segments, {int(differ.sum())} cells differ "
         f"({int(bad_type.sum())} outside near-ties, {int(frag.sum())} near-tie cells), worst end error "
         f"{worst:.2f} of its bound")
    assert rcnt > 20 and not bad_type.any()


def test_crease_extraction_full_size(env):
    """The 4096^2 creases image (the bench's extraction), mode BOTH.
    - Every cell's decision against the oracle's, outside corner near-ties as
      in the small cases. A decision that differs otherwise must be what the
      oracle's marching makes of the GPU's field (whose error is bounded
      first), and the GPU's marching must match that one up to float32-level
      perturbations of a cell's field.
    - The segment ends of 20 000 sampled cells where both sides agree, within
      the first-order bound of the corners' d errors plus the float32
      rounding of the stored coordinates (up to 4095 here)."""
    import time
    o, m, synth = env["o"], env["m"], env["synth"]
    u = synth.creases4096().image()
    sigma_d, strength, mode = 1.0, 0.005, 2
    t0 = time.time()
    seg, typ, cnt, field = _gpu_creases(env, u, sigma_d, strength, mode)
    P = o.crease_field(u, sigma_d)
    rseg, rtyp, rcnt = o.marching_creases(P, strength, mode)
    _log(f"creases 4096^2: GPU and oracle in {time.time() - t0:.1f}s")
    scale = np.abs(P).reshape(6, -1).max(axis=1)
    ferr = np.abs(field - P).reshape(6, -1).max(axis=1)
    assert np.all(ferr <= 2e-6 * scale + 1e-12), (ferr, scale)
    assert cnt == int((typ != 0).sum())
    frag = _fragile_cells(P, field, strength)
    differ = np.any(typ != rtyp, axis=2)
    # The oracle's marching of the GPU's own field (in FP64) must give the
    # GPU's decisions, except where the cell's decision flips under a
    # perturbation of its 2 x 2 field at the float32 level (the marching's
    # own rounding: crossings, interpolated Hessians, the direction test).
    own_seg, own_typ, _ = o.marching_creases(field.astype(np.float64), strength, mode)
    differ_own = np.any(typ != own_typ, axis=2)
    rng = np.random.default_rng(9)
    flipped = np.zeros_like(differ_own)
    for (y, x) in np.argwhere(differ_own):
        block = field[:, y:y + 2, x:x + 2].astype(np.float64)
        for _ in range(64):
            pert = block * (1.0 + 1e-6 * rng.uniform(-1.0, 1.0, size=block.shape))
            _, t2, _ = o.marching_creases(np.ascontiguousarray(pert), strength, mode)
            if np.array_equal(t2[0, 0], typ[y, x]):
                flipped[y, x] = True
                break
    unexplained = int((differ_own & ~flipped).sum())
    # Against the oracle's own field, a decision that differs and is not a
    # corner near-tie must follow from the GPU's field (its float32 error,
    # bounded above, is what moved it), up to those perturbations.
    frag |= differ & (~differ_own | flipped)
    bad_type = differ & ~frag
    same = np.argwhere(~differ & ~frag & np.any(rtyp != 0, axis=2))
    rng = np.random.default_rng(5)
    pick = same[rng.choice(len(same), size=min(20000, len(same)), replace=False)]
    ed = np.abs(field[5].astype(np.float64) - P[5])
    worst = 0.0
    for (y, x) in pick:
        dc = [P[5][y, x], P[5][y, x + 1], P[5][y + 1, x + 1], P[5][y + 1, x]]
        ec = [ed[y, x], ed[y, x + 1], ed[y + 1, x + 1], ed[y + 1, x]]
        tol = 2 * sum(ec) / min(abs(dc[i] - dc[(i + 1) % 4]) or 1e-300 for i in range(4)
                                if (dc[i] >= 0) != (dc[(i + 1) % 4] >= 0)) + 1e-5
        # plus the float32 rounding of each stored end coordinate (one ulp of
        # its magnitude: 6e-5 at 566, 2.4e-4 near 4096)
        lim = tol + np.spacing(np.abs(rseg[y, x]).astype(np.float32)).astype(np.float64)
        dev = np.abs(seg[y, x] - rseg[y, x])
        worst = max(worst, float((dev / lim).max()))
        assert np.all(dev <= lim), (y, x, seg[y, x], rseg[y, x], tol)
    _log(f"creases 4096^2: GPU {cnt} / oracle {rcnt} segments, {int(differ.sum())} cells differ "
         f"({int(bad_type.sum())} outside near-ties); against the oracle's marching of the GPU's field "
         f"{int(differ_own.sum())} differ ({unexplained} not flipped by 1e-6 perturbations); worst sampled end "
         f"error {worst:.2f} of its bound")
    assert rcnt > 100000 and not bad_type.any() and unexplained == 0


def test_crease_match_parity(env):
    """The GPU matcher on the oracle's own segments (as float32) against the
    oracle on the same values, with the generator's centrelines."""
    o, m, torch = env["o"], env["m"], env["torch"]
    w = env["synth"].ridges128()
    u, clean, lines = w.ground_truth()
    rseg, rtyp, _ = o.creases(u, 1.0, 0.005, 0)
    seg32 = rseg.astype(np.float32)
    gts, gtt = o.gt_segments(lines)
    gts32 = gts.astype(np.float32)
    dist_ref, match_ref = o.crease_match(seg32.astype(np.float64), rtyp, gts32.astype(np.float64), gtt, 6.0)
    dist, match = m.mf4d_crease_match(_to(env, seg32), _to(env, rtyp), _to(env, gts32),
                                      _to(env, gtt.astype(np.int32)), 6.0)
    torch.cuda.synchronize()
    dist, match = dist.cpu().numpy(), match.cpu().numpy()
    diff = np.argwhere(match != match_ref).ravel()
    # a differing pick must be a near-tie: the oracle's distance to the GPU's pick within 1e-5 of its best
    for i in diff:
        if match[i] < 0 or match_ref[i] < 0:
            # at the edge of the neighbourhood
            G = gts32[i].astype(np.float64)
            k = match[i] if match[i] >= 0 else match_ref[i]
            assert abs(o.segment_hausdorff(G, seg32.reshape(-1, 4)[k].astype(np.float64)) - 6.0) <= 1e-5
            continue
        G = gts32[i].astype(np.float64)
        hg = o.segment_hausdorff(G, seg32.reshape(-1, 4)[match[i]].astype(np.float64))
        hr = o.segment_hausdorff(G, seg32.reshape(-1, 4)[match_ref[i]].astype(np.float64))
        assert abs(hg - hr) <= 1e-5, (i, hg, hr)
    ok = (match == match_ref) & (match >= 0)
    # FP32 differences of coordinates up to max(H, W): a few ulp of that size
    atol = 8 * np.finfo(np.float32).eps * max(u.shape)
    assert np.allclose(dist[ok], dist_ref[ok], atol=atol)
    E, p = o.crease_scores(dist)
    Er, pr = o.crease_scores(dist_ref)
    _log(f"match: {len(gts)} ground-truth segments, {len(diff)} near-tie picks; E {E:.4f} / {Er:.4f}, "
         f"p {p:.4f} / {pr:.4f}")
    assert abs(E - Er) <= 1e-4 and abs(p - pr) <= 2.0 / len(gts)


def test_crease_match_full_size(env):
    """The matcher at the bench's size: the 555k centreline segments of the
    4096^2 image against the GPU's 6.3M extracted segments (as float32, the
    same values on both sides), GPU against oracle. A pick that differs must
    be a near-tie within 1e-5 px, and the distances agree to 1e-5."""
    o, m, torch = env["o"], env["m"], env["torch"]
    w = env["synth"].creases4096()
    u, clean, lines = w.ground_truth()
    seg, typ = m.mf4d_creases(_to(env, u), 1.0, 0.005, 2)
    gts, gtt = o.gt_segments(lines)
    gts32 = gts.astype(np.float32)
    dist, match = m.mf4d_crease_match(seg, typ, _to(env, gts32), _to(env, gtt.astype(np.int32)), 6.0)
    torch.cuda.synchronize()
    seg32, typ8 = seg.cpu().numpy(), typ.cpu().numpy()
    dist, match = dist.cpu().numpy(), match.cpu().numpy()
    dist_ref, match_ref = o.crease_match(seg32.astype(np.float64), typ8, gts32.astype(np.float64), gtt, 6.0)
    # distances in float32 from offsets of a few pixels (the GPU measures
    # them from the ground-truth segment's first end)
    tol = 1e-5
    flat = seg32.reshape(-1, 4).astype(np.float64)
    diff = np.argwhere(match != match_ref).ravel()
    for i in diff:
        G = gts32[i].astype(np.float64)
        if match[i] < 0 or match_ref[i] < 0:   # at the edge of the neighbourhood
            k = match[i] if match[i] >= 0 else match_ref[i]
            assert abs(o.segment_hausdorff(G, flat[k]) - 6.0) <= tol
            continue
        assert abs(o.segment_hausdorff(G, flat[match[i]]) - o.segment_hausdorff(G, flat[match_ref[i]])) <= tol
    ok = (match == match_ref) & (match >= 0)
    assert np.allclose(dist[ok], dist_ref[ok], atol=tol)
    E, p = o.crease_scores(dist)
    Er, pr = o.crease_scores(dist_ref)
    _log(f"match 4096^2: {len(gts)} ground-truth segments, {len(diff)} near-tie picks; E {E:.4f} / {Er:.4f}, "
         f"p {p:.4f} / {pr:.4f}")
    assert len(gts) > 500000 and abs(E - Er) <= 1e-4 and abs(p - pr) <= 2.0 / len(gts) + len(diff) / len(gts)


def test_crease_pipeline_on_filtered_image(env):
    """End to end on ridges128: the filter, the extraction and the matching
    all on the GPU, against the oracle's three steps; E and p agree to the
    share of segments near-tie decisions move."""
    o, m, torch = env["o"], env["m"], env["torch"]
    w = env["synth"].ridges128()
    u, clean, lines = w.ground_truth()
    p = m.Params.from_workload(w, cycles=1)
    ui = _to(env, u)
    uo = torch.empty_like(ui)
    m.mf4d_filter(ui, uo, p)
    seg, typ = m.mf4d_creases(uo, 1.0, 0.005, 0)
    gts, gtt = o.gt_segments(lines)
    dist, _ = m.mf4d_crease_match(seg, typ, _to(env, gts.astype(np.float32)), _to(env, gtt.astype(np.int32)), 6.0)
    torch.cuda.synchronize()
    E, pp = o.crease_scores(dist.cpu().numpy())
    ref = o.filter(u, w.sigmas, w.mode, lam=w.lam, cycles=1, substeps=w.substeps)
    rseg, rtyp, _ = o.creases(ref, 1.0, 0.005, 0)
    rd, _ = o.crease_match(rseg, rtyp, gts, gtt, 6.0)
    Er, pr = o.crease_scores(rd)
    _log(f"ridges128, one cycle: E {E:.4f} (oracle {Er:.4f}), p {pp:.4f} (oracle {pr:.4f})")
    assert abs(E - Er) <= 0.02 and abs(pp - pr) <= 0.02
