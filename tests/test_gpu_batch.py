"""Batched filter (one recorded hipGraph for many uneven images) against
per-image mf4d_filter calls: results must be bit-identical, for every
substep decomposition, across graph replays and for in-place buffers."""
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
    mf4d.lib()
    return dict(torch=torch, m=mf4d, synth=synth, dev=torch.device("cuda:0"))


SHAPES = [(67, 131), (128, 96), (40, 40), (200, 75), (3, 3), (96, 260), (33, 17)]
MODES = [0, 1, 2, 0, 1, 2, 1]
CYCLES = [3, 1, 4, 2, 2, 0, 3]


def _setup(env, substeps=7):
    m, synth, torch = env["m"], env["synth"], env["torch"]
    sig = [1.0, 1.5, 2.0, 3.0]
    imgs = [synth.creases(h, w, 3, seed=11 * i + h) for i, (h, w) in enumerate(SHAPES)]
    params = [m.Params(sig, mode=mo, cycles=cy, substeps=substeps) for mo, cy in zip(MODES, CYCLES)]
    packed = np.concatenate([im.ravel() for im in imgs])
    return imgs, params, torch.from_numpy(packed).to(env["dev"])


def _same(got, ref):
    """Bitwise equality; on failure names the images that differ."""
    import torch
    if torch.equal(got, ref):
        return True
    pos = 0
    for k, (h, w) in enumerate(SHAPES):
        a, b = got[pos:pos + h * w], ref[pos:pos + h * w]
        if not torch.equal(a, b):
            d = (a - b).abs()
            _log(f"  image {k} {h}x{w} mode {MODES[k]} cycles {CYCLES[k]}: max diff {float(d.nan_to_num(1e9).max())}, "
                 f"{int((a != b).sum())} px differ")
        pos += h * w
    return False


def _singles(env, imgs, params):
    m, torch = env["m"], env["torch"]
    out = []
    for im, p in zip(imgs, params):
        ui = torch.from_numpy(im).to(env["dev"])
        uo = torch.empty_like(ui)
        m.mf4d_filter(ui, uo, p)
        out.append(uo)
    torch.cuda.synchronize()
    return torch.cat([o.ravel() for o in out])


def test_batch_bitwise_equals_single_images(env):
    m, torch = env["m"], env["torch"]
    imgs, params, pin = _setup(env)
    _log("batch vs single images")
    ref = _singles(env, imgs, params)
    b = m.Batch(SHAPES, params)
    ws = b.workspace(env["dev"])
    pout = torch.full_like(pin, float("nan"))
    b.filter(pin, pout, ws)
    torch.cuda.synchronize()
    assert _same(pout, ref)
    # replays of the recorded graph, with eager work and syncs in between
    for rep in range(3):
        pout.fill_(-1.0)
        _ = _singles(env, imgs[:2], params[:2])
        b.filter(pin, pout, ws)
        torch.cuda.synchronize()
        assert _same(pout, ref), rep
    # every substep decomposition gives the same values
    for spl, rows in [(1, 0), (2, 24), (3, 0), (4, 16), (4, 96)]:
        b.set_tuning(spl, rows)
        pout.zero_()
        b.filter(pin, pout, ws)
        torch.cuda.synchronize()
        assert _same(pout, ref), (spl, rows)
    b.autotune(ws)
    _log(f"  autotuned: {b.tuning()}")
    b.filter(pin, pout, ws)
    torch.cuda.synchronize()
    assert _same(pout, ref)
    b.close()


def test_batch_in_place_and_even_substeps(env):
    m, torch = env["m"], env["torch"]
    imgs, params, pin = _setup(env, substeps=8)
    _log("batch in place")
    ref = _singles(env, imgs, params)
    b = m.Batch(SHAPES, params)
    ws = b.workspace(env["dev"])
    buf = pin.clone()
    b.filter(buf, buf, ws)
    torch.cuda.synchronize()
    assert _same(buf, ref)
    buf.copy_(pin)
    b.filter(buf, buf, ws)   # graph replay in place
    torch.cuda.synchronize()
    assert _same(buf, ref)
    b.close()


def test_batch_strided_offsets(env):
    """Images at arbitrary non-overlapping offsets in a larger buffer."""
    m, torch = env["m"], env["torch"]
    imgs, params, _ = _setup(env)
    offs, pos = [], 5
    for h, w in SHAPES:
        offs.append(pos)
        pos += h * w + 37
    big = np.zeros(pos + 11, np.float32)
    for o, im in zip(offs, imgs):
        big[o:o + im.size] = im.ravel()
    pin = torch.from_numpy(big).to(env["dev"])
    ref = _singles(env, imgs, params)
    b = m.Batch(SHAPES, params, offsets=offs)
    ws = b.workspace(env["dev"])
    pout = torch.zeros_like(pin)
    b.filter(pin, pout, ws)
    torch.cuda.synchronize()
    got = torch.cat([pout[o:o + h * w] for o, (h, w) in zip(offs, SHAPES)])
    assert _same(got, ref)
    b.close()


def test_batch_total_beyond_2e31_pixels(env):
    """Two images of 46000 x 25000 (2.3 G px packed, past element 2^31 of the
    packed buffers): the batch equals per-image calls bit for bit."""
    m, synth, torch = env["m"], env["synth"], env["torch"]
    dev = env["dev"]
    H, W = 46000, 25000
    n = H * W
    assert n < 2 ** 31 < 2 * n

    def folded(tile):   # the tile's half-sample-symmetric periodic extension, H x W
        th, tw = tile.shape
        iy = torch.arange(H, device=dev) % (2 * th)
        iy = torch.where(iy < th, iy, 2 * th - 1 - iy)
        ix = torch.arange(W, device=dev) % (2 * tw)
        ix = torch.where(ix < tw, ix, 2 * tw - 1 - ix)
        return torch.from_numpy(tile).to(dev)[iy][:, ix]

    _log(f"batch of two {H} x {W} images ({2 * n} px packed)")
    p = m.Params([1.0], mode=0, cycles=1, substeps=4)
    pin = torch.empty(2 * n, dtype=torch.float32, device=dev)
    for k in range(2):
        pin[k * n:(k + 1) * n] = folded(synth.creases(230, 250, 3, seed=70 + k)).ravel()
    b = m.Batch([(H, W)] * 2, [p, p])
    ws = b.workspace(dev)
    pout = torch.empty_like(pin)
    b.filter(pin, pout, ws)
    torch.cuda.synchronize()
    b.close()
    del ws
    torch.cuda.empty_cache()
    ws1 = m.workspace(H, W, p, dev)
    ref = torch.empty((H, W), dtype=torch.float32, device=dev)
    for k in range(2):
        m.mf4d_filter(pin[k * n:(k + 1) * n].view(H, W), ref, p, ws1)
        torch.cuda.synchronize()
        assert torch.equal(pout[k * n:(k + 1) * n].view(H, W), ref), k
        assert not torch.equal(ref, pin[k * n:(k + 1) * n].view(H, W))
    del ws1, ref, pin, pout
    torch.cuda.empty_cache()


# images of the 256-image batched workload (indices into synth.batch_of_images():
# ridge and valley, 6 to 25 cycles, one side >= 1024)
ORACLE_PICK = [210, 162, 58, 144, 12, 22]


def test_batch_against_oracle(env):
    """Batched outputs against the FP64 oracle, element by element, on
    images of the batched workload itself (sizes U[256, 1536], per-image
    mode and cycle count, scales 1, 1.5, 2, 3, n = 10)."""
    import oracle
    m, synth, torch = env["m"], env["synth"], env["torch"]
    specs = synth.batch_of_images()
    pick = [specs[i] for i in ORACLE_PICK]
    assert {s["mode"] for s in pick} == {0, 1} and max(max(s["H"], s["W"]) for s in pick) >= 1024
    assert len({s["cycles"] for s in pick}) == len(pick)
    sig = [1.0, 1.5, 2.0, 3.0]
    imgs = [synth.batch_image(s) for s in pick]
    params = [m.Params(sig, mode=s["mode"], cycles=s["cycles"], substeps=10) for s in pick]
    shapes = [(s["H"], s["W"]) for s in pick]
    packed = torch.from_numpy(np.concatenate([im.ravel() for im in imgs])).to(env["dev"])
    out = torch.empty_like(packed)
    plan = m.Batch(shapes, params)
    ws = plan.workspace(env["dev"])
    plan.autotune(ws)
    plan.filter(packed, out, ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    plan.close()
    pos = 0
    for s, im in zip(pick, imgs):
        h, w = s["H"], s["W"]
        g = got[pos:pos + h * w].reshape(h, w).astype(np.float64)
        pos += h * w
        ref = oracle.filter(im, sig, s["mode"], cycles=s["cycles"], substeps=10)
        e = float(np.abs(g - ref).max())
        r = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
        _log(f"batch vs oracle {h}x{w} mode {s['mode']} cycles {s['cycles']}: max-abs {e:.3e} rel-L2 {r:.3e}")
        assert e <= 2e-4 and r <= 1e-5
