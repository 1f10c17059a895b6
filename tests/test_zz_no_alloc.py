"""mf4d_filter_noalloc (the entry point for callers that cannot allocate)
against mf4d_filter, through the C ABI: the same values, bit for bit (the
same kernels; running every scale on the caller's stream changes no value),
on two calls in a row with the second on a smaller image, and the size limit
of its fixed scratch array."""
import ctypes
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


def _run(env, fn, u, p):
    torch = env["torch"]
    ui = torch.from_numpy(u).to(env["dev"])
    uo = torch.full_like(ui, float("nan"))
    fn(ui, uo, p)
    torch.cuda.synchronize()
    return uo.cpu().numpy()


def test_noalloc_equals_filter_two_calls(env):
    m, synth = env["m"], env["synth"]
    w = synth.ridges128()
    big = w.image()
    p_big = m.Params.from_workload(w)                      # 128 x 128, 4 scales, 5 x 10
    small = synth.creases(70, 93, 2, seed=9, signs="mixed")
    p_small = m.Params([1.0, 2.0, 3.0], mode=m.MF4D_BOTH, cycles=3, substeps=7)
    _log("noalloc: 128x128 then 70x93")
    a1 = _run(env, m.mf4d_filter_noalloc, big, p_big)
    a2 = _run(env, m.mf4d_filter_noalloc, small, p_small)
    b1 = _run(env, m.mf4d_filter, big, p_big)
    b2 = _run(env, m.mf4d_filter, small, p_small)
    assert np.array_equal(a1, b1)
    assert np.array_equal(a2, b2)
    # in place, and with the monitor
    torch = env["torch"]
    ui = torch.from_numpy(small).to(env["dev"])
    pc = m.Params([1.0, 2.0, 3.0], mode=m.MF4D_BOTH, cycles=3, substeps=7, check=1)
    m.mf4d_filter_noalloc(ui, ui, pc)
    torch.cuda.synchronize()
    assert np.array_equal(ui.cpu().numpy(), b2)


def test_noalloc_size_limit(env):
    m, torch = env["m"], env["torch"]
    cap = m.mf4d_noalloc_max_bytes()
    assert cap == 128 << 20
    p = m.Params([1.0, 2.0, 4.0, 8.0])
    # an image whose workspace exceeds the array is rejected before any launch
    H, W = 2048, 1024
    assert m.mf4d_workspace_bytes(H, W, p) > cap
    st = p.struct()
    rc = m.lib().mf4d_filter_noalloc(ctypes.c_void_p(256), ctypes.c_void_p(256), H, W, ctypes.byref(st), None)
    assert rc == m.MF4D_ENOMEM
    # the largest square image that fits still runs and matches
    n = 64
    while m.mf4d_workspace_bytes(2 * n, 2 * n, p) <= cap:
        n *= 2
    lo, hi = n, 2 * n
    while hi - lo > 1:
        mid = (lo + hi) // 2
        lo, hi = (mid, hi) if m.mf4d_workspace_bytes(mid, mid, p) <= cap else (lo, mid)
    u = env["synth"].creases(lo, lo, 4, seed=2)
    p.cycles, p.substeps = 1, 4
    _log(f"noalloc: largest square image {lo}x{lo}")
    assert np.array_equal(_run(env, m.mf4d_filter_noalloc, u, p), _run(env, m.mf4d_filter, u, p))
