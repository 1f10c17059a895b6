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
