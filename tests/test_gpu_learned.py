"""Learned scale surrogate: MFMA forward and backward against the FP64
oracle, training on labels from the exact sweep, and the learned filter's
equivalences with the exact filter."""
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


def _bf16(a):
    import torch
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _theta(env, seed):
    """Seeded parameters made on the host: He-normal weights plus a small
    perturbation of every entry, so that the biases are non-zero and every
    parameter has a gradient path. The oracle reads this host array; the
    device gets a copy of it."""
    rng = np.random.default_rng(seed)
    ch = env["o"].NET_CHANNELS
    parts = []
    for ci, co in zip(ch[:-1], ch[1:]):
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=co * ci * 9))
        parts.append(np.zeros(co))
    th = np.concatenate(parts)
    th = (th + 0.05 * rng.standard_normal(th.shape)).astype(np.float32)
    return th, env["torch"].from_numpy(th).to(env["dev"])


def test_forward_matches_oracle(env):
    m, o, torch = env["m"], env["o"], env["torch"]
    rng = np.random.default_rng(0)
    B, H, W = 2, 32, 48
    u = rng.uniform(size=(B, H, W)).astype(np.float32)
    th_host, th = _theta(env, 1)
    logits = torch.empty((B * H * W, 16), dtype=torch.float32, device=env["dev"])
    m.mf4d_net_forward(th, torch.from_numpy(u).to(env["dev"]), logits=logits)
    torch.cuda.synchronize()
    got = logits.cpu().numpy().reshape(B, H, W, 16)[..., :9].transpose(0, 3, 1, 2)
    ref = o.net_forward(_bf16(th_host), _bf16(u))
    e = _rel(got, ref)
    _log(f"forward rel-L2 vs oracle {e:.3e}")
    assert e <= 2e-2


def test_gradient_matches_oracle(env):
    m, o, torch = env["m"], env["o"], env["torch"]
    rng = np.random.default_rng(2)
    B, H, W = 2, 32, 32
    u = rng.uniform(size=(B, H, W)).astype(np.float32)
    lab = rng.integers(0, 8, size=(B, H, W)).astype(np.uint8)
    th_host, th = _theta(env, 3)
    grad = torch.zeros_like(th)
    stats = torch.zeros(2, dtype=torch.float32, device=env["dev"])
    m.mf4d_net_backward(th, torch.from_numpy(u).to(env["dev"]), torch.from_numpy(lab).to(env["dev"]), grad,
                        w_conf=0.3, stats_out=stats)
    torch.cuda.synchronize()
    loss_ref, g_ref = o.net_grad(_bf16(th_host), _bf16(u), lab, 0.3)
    g = grad.cpu().numpy().astype(np.float64)
    assert abs(float(stats[0]) - loss_ref) <= 2e-2 * abs(loss_ref)
    pos = 0
    for l, (ci, co) in enumerate(zip(o.NET_CHANNELS[:-1], o.NET_CHANNELS[1:])):
        nw = co * ci * 9
        ew, eb = _rel(g[pos:pos + nw], g_ref[pos:pos + nw]), _rel(g[pos + nw:pos + nw + co], g_ref[pos + nw:pos + nw + co])
        _log(f"layer {l}: weight-grad rel-L2 {ew:.3e}, bias-grad rel-L2 {eb:.3e}")
        assert ew <= 2e-2 and eb <= 2e-2, l
        pos += nw + co


def test_training_reduces_loss_on_exact_labels(env):
    m, torch, synth = env["m"], env["torch"], env["synth"]
    sig = [8.0 ** (k / 7.0) for k in range(8)]
    imgs, labs = [], []
    for sd in range(4):
        u = synth.fundus(128, 128, seed=70 + sd)
        ui = torch.from_numpy(u).to(env["dev"])
        idx = torch.empty((128, 128), dtype=torch.uint8, device=env["dev"])
        m.mf4d_scale_select(ui, m.Params(sig, mode=1), idx)
        imgs.append(ui)
        labs.append(idx)
    U, L = torch.stack(imgs), torch.stack(labs)
    th = m.net_init(5, env["dev"])
    g = torch.zeros_like(th)
    mm, vv = torch.zeros_like(th), torch.zeros_like(th)
    stats = torch.zeros(2, dtype=torch.float32, device=env["dev"])
    ws = m.net_workspace(4, 128, 128, True, env["dev"])
    first = None
    for step in range(1, 151):
        m.mf4d_net_backward(th, U, L, g, 0.1, stats, ws)
        m.mf4d_net_step(th, g, mm, vv, step, 3e-3)
        if step == 1:
            torch.cuda.synchronize()
            first = stats.cpu().numpy().copy()
    torch.cuda.synchronize()
    last = stats.cpu().numpy()
    _log(f"training: loss {first[0]:.3f} -> {last[0]:.3f}, accuracy {first[1]:.3f} -> {last[1]:.3f}")
    assert last[0] < 0.8 * first[0] and last[1] > first[1]


def test_learned_filter_extremes(env):
    """threshold 1 with an unsure net is the exact filter (bitwise); threshold 0
    uses the net's scale everywhere and every pixel-cycle is counted."""
    m, torch, synth = env["m"], env["torch"], env["synth"]
    sig = [8.0 ** (k / 7.0) for k in range(8)]
    H, W = 96, 112
    u = synth.fundus(H, W, seed=3)
    p = m.Params(sig, mode=1, cycles=3, substeps=6)
    ui = torch.from_numpy(u).to(env["dev"])
    ref = torch.empty_like(ui)
    m.mf4d_filter(ui, ref, p)
    th = m.net_init(7, env["dev"]) * 1e-3   # logits ~ 0: confidence ~ 0.5 everywhere
    out = torch.empty_like(ui)
    fb = torch.zeros(1, dtype=torch.int32, device=env["dev"])
    m.mf4d_filter_learned(ui, out, p, th, 1.0, fb)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    assert int(fb.item()) == 3 * H * W
    m.mf4d_filter_learned(ui, out, p, th, 0.0, fb)
    torch.cuda.synchronize()
    assert int(fb.item()) == 0
    assert torch.isfinite(out).all()
    assert abs(float(out.double().mean()) - float(ui.double().mean())) <= 1e-6   # mass is conserved
