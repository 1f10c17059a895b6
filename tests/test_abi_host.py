"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every symbol include/mf4d.h declares, the host FED schedule equals
the oracle's, and invalid arguments are rejected before any launch."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from conftest import ROOT


@pytest.fixture(scope="module")
def m():
    from paper_1611_06906_amd import mf4d
    mf4d.lib()
    return mf4d


def test_header_symbols_exported(m):
    hdr = open(os.path.join(ROOT, "include", "mf4d.h")).read()
    declared = set(re.findall(r"\b(mf4d(?:3d)?_[a-z0-9_]+)\s*\(", hdr))
    assert declared == set(m.EXPORTS)
    for name in declared:
        assert hasattr(m.lib(), name), name


def test_status_strings(m):
    for st in (0, -1, -2, -3, -4, -5, 7):
        assert len(m.status_string(st)) > 0
    assert m.status_string(-4) != m.status_string(7) and m.status_string(-5) != m.status_string(7)


def test_schedule_equals_oracle_bitwise(m, oracle_lib):
    for n in range(1, 65):
        taus, perm, k = m.mf4d_fed_schedule(n, 0.05)
        o_taus, o_perm, o_k = oracle_lib.fed_schedule(n, 0.05)
        assert k == o_k and np.array_equal(perm, o_perm), n
        assert np.array_equal(taus, o_taus), n
    for tmax in (1.0 / 17.0, 0.03):
        taus, _, _ = m.mf4d_fed_schedule(20, tmax)
        assert np.array_equal(taus, oracle_lib.fed_schedule(20, tmax)[0])


def test_substeps_and_plan_equal_oracle(m, oracle_lib):
    for T, M in [(500.0, 10000), (20.0, 1000), (12.0, 2), (5.0, 1), (80.0, 20), (7.3, 3)]:
        assert m.mf4d_fed_substeps(T, M, 0.05) == oracle_lib.fed_n(T, M, 0.05)
    p = m.Params([1.0, 2.0], cycles=2, substeps=0, stop_time=12.0)
    n, taus = m.mf4d_fed_plan(p)
    assert n == 19
    nat = oracle_lib.fed_taus(n, 12.0, 2)
    _, _, ordered = oracle_lib.kappa_order(nat, 0.05)
    assert np.array_equal(taus, ordered)
    assert math.isclose(taus.sum(), 6.0, rel_tol=1e-13)


def _raw_filter(m, H, W, p):
    st = p.struct()
    return m.lib().mf4d_filter(None, None, H, W, ctypes.byref(st), None, 0, None)


def test_validation_rejects_before_launch(m):
    good = dict(sigmas=[1.0, 2.0], mode=0, cycles=1, substeps=5)
    P = lambda **kw: m.Params(**{**good, **kw})
    assert m.mf4d_workspace_bytes(64, 64, P()) > 0
    bad = [
        (2, 64, P()), (64, 2, P()), (1 << 16, 1 << 15, P()),
        (64, 64, P(sigmas=[])), (64, 64, P(sigmas=[2.0, 1.0])), (64, 64, P(sigmas=[1.0, 1.0])),
        (64, 64, P(sigmas=[0.0, 1.0])), (64, 64, P(sigmas=[30.0])), (64, 64, P(sigmas=list(range(1, 18)))),
        (64, 64, P(mode=3)), (64, 64, P(lam=0.0)), (64, 64, P(lam=float("nan"))),
        (64, 64, P(rho=-1.0)), (64, 64, P(rho=5.0)), (64, 64, P(beta=0.0)),
        (64, 64, P(c=float("inf"))), (64, 64, P(cycles=-1)), (64, 64, P(tau_max=0.06)),
        (64, 64, P(tau_max=0.0)), (64, 64, P(substeps=0, stop_time=0.0)),
        (64, 64, P(substeps=2000)), (64, 64, P(reselect_each_cycle=2)), (64, 64, P(postprocess=2)),
        (64, 64, P(postprocess=1, theta=float("nan"))), (64, 64, P(check=2)), (64, 64, P(model=2)),
        (64, 64, P(model=1)),   # the isotropic model takes exactly one scale
    ]
    for H, W, p in bad:
        assert m.mf4d_workspace_bytes(H, W, p) == 0
        assert _raw_filter(m, H, W, p) == m.MF4D_EINVAL
    # valid parameters but missing buffers are rejected too
    assert _raw_filter(m, 64, 64, P()) == m.MF4D_EINVAL
    # lambda = +inf (linear isotropic) and rho = 0 are valid, and so are the
    # postprocessing, the check and the isotropic model with one scale
    assert m.mf4d_workspace_bytes(64, 64, P(lam=math.inf, rho=0.0)) > 0
    assert m.mf4d_workspace_bytes(64, 64, P(postprocess=1, theta=0.2, check=1)) > 0
    assert m.mf4d_workspace_bytes(64, 64, P(sigmas=[1.0], model=1)) > 0
    # l2 stopping: u_out must not alias the input or the ground truth
    st = P().struct()
    L = m.lib()
    for uo in (16, 32):
        assert L.mf4d_filter_l2stop(ctypes.c_void_p(16), ctypes.c_void_p(uo), 64, 64, ctypes.byref(st),
                                    ctypes.c_void_p(32), None, None, ctypes.c_void_p(64), 1 << 30,
                                    None) == m.MF4D_EINVAL
    # workspace too small
    st = P().struct()
    nb = m.mf4d_workspace_bytes(64, 64, P())
    assert m.lib().mf4d_filter(ctypes.c_void_p(16), ctypes.c_void_p(16), 64, 64, ctypes.byref(st),
                               ctypes.c_void_p(16), nb - 1, None) == m.MF4D_ENOMEM
    with pytest.raises(m.MF4DError):
        m.mf4d_fed_schedule(0)
    with pytest.raises(m.MF4DError):
        m.mf4d_fed_schedule(10, 0.07)


def test_volume_validation_rejects_before_launch(m):
    """The 3-D calls: the 2-D parameter checks, tau_max <= 1/27, and the
    options the volume filter does not take; sizes >= 3 per axis."""
    good = dict(sigmas=[1.0, 2.0], mode=0, cycles=1, substeps=5, tau_max=1.0 / 27.0)
    P = lambda **kw: m.Params(**{**good, **kw})
    assert m.mf4d3d_workspace_bytes(8, 9, 10, P()) > 0
    assert m.mf4d3d_workspace_bytes(3, 3, 3, P()) > 0
    bad = [
        ((2, 9, 10), P()), ((8, 2, 10), P()), ((8, 9, 2), P()), ((70000, 4, 4), P()),
        ((1 << 11, 1 << 10, 1 << 10), P()),
        ((8, 9, 10), P(tau_max=0.05)), ((8, 9, 10), P(tau_max=1.0 / 26.0)), ((8, 9, 10), P(tau_max=0.0)),
        ((8, 9, 10), P(model=1, sigmas=[1.0])), ((8, 9, 10), P(postprocess=1)), ((8, 9, 10), P(check=1)),
        ((8, 9, 10), P(reselect_each_cycle=0)), ((8, 9, 10), P(sigmas=[2.0, 1.0])), ((8, 9, 10), P(mode=3)),
        ((8, 9, 10), P(lam=0.0)), ((8, 9, 10), P(beta=0.0)), ((8, 9, 10), P(cycles=-1)),
    ]
    L = m.lib()
    one = ctypes.c_void_p(16)
    for (D, H, W), p in bad:
        assert m.mf4d3d_workspace_bytes(D, H, W, p) == 0
        st = p.struct()
        assert L.mf4d3d_filter(one, one, D, H, W, ctypes.byref(st), one, 1 << 40, None) == m.MF4D_EINVAL
        assert L.mf4d3d_scale_select(one, D, H, W, ctypes.byref(st), one, None, None, one, 1 << 40,
                                     None) == m.MF4D_EINVAL
    st = P().struct()
    nb = m.mf4d3d_workspace_bytes(8, 9, 10, P())
    assert L.mf4d3d_filter(one, one, 8, 9, 10, ctypes.byref(st), one, nb - 1, None) == m.MF4D_ENOMEM
    assert L.mf4d3d_filter(None, one, 8, 9, 10, ctypes.byref(st), one, nb, None) == m.MF4D_EINVAL
    two = ctypes.c_void_p(32)
    taus = (ctypes.c_double * 2)(0.01, -0.01)
    assert L.mf4d3d_fed_cycle_tensor(one, two, 8, 9, 10, one, taus, 2, None) == m.MF4D_EINVAL
    assert L.mf4d3d_fed_cycle_tensor(one, two, 8, 9, 10, one, taus, 0, None) == m.MF4D_EINVAL
    assert L.mf4d3d_fed_cycle_tensor(one, None, 8, 9, 10, one, taus, 1, None) == m.MF4D_EINVAL
    assert L.mf4d3d_fed_cycle_tensor(one, one, 8, 9, 10, one, taus, 1, None) == m.MF4D_EINVAL   # aliasing
    # the workspace grows with the volume and the number of scales
    a = m.mf4d3d_workspace_bytes(16, 16, 16, P())
    assert m.mf4d3d_workspace_bytes(32, 32, 32, P()) > 7.9 * a
    assert m.mf4d3d_workspace_bytes(16, 16, 16, P(sigmas=[1.0, 2.0, 3.0])) > a


def test_workspace_scales_with_image_and_scales(m):
    p1 = m.Params([1.0, 2.0])
    p2 = m.Params([1.0, 2.0, 3.0, 4.0])
    a = m.mf4d_workspace_bytes(256, 256, p1)
    assert m.mf4d_workspace_bytes(512, 512, p1) > 3.9 * a
    assert m.mf4d_workspace_bytes(256, 256, p2) > a


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1611_06906_amd import mf4d
    monkeypatch.setattr(mf4d, "_lib", None)
    monkeypatch.setattr(mf4d, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        mf4d.lib()


def test_batch_plan_validation(m):
    sig = [1.0, 2.0]
    P = m.Params
    shapes = [(32, 40), (20, 20)]
    b = m.Batch(shapes, [P(sig, mode=0, cycles=2), P(sig, mode=1, cycles=5)])
    assert b.workspace_bytes() > m.mf4d_workspace_bytes(32, 40, P(sig))
    assert b.tuning()[0] in (1, 2, 3, 4)
    b.set_tuning(2, 64)
    assert b.tuning() == (2, 64)
    with pytest.raises(m.MF4DError):
        b.set_tuning(5, 0)
    b.close()
    bad = [
        (shapes, [P(sig), P([1.0, 3.0])], None),                    # different scales
        (shapes, [P(sig), P(sig, lam=0.01)], None),                 # different lambda
        (shapes, [P(sig, substeps=5), P(sig, substeps=6)], None),   # different schedule
        (shapes, [P(sig), P(sig)], [0, 100]),                       # overlapping images
        ([(2, 40), (20, 20)], [P(sig), P(sig)], None),              # invalid size
        (shapes, [P(sig, postprocess=1), P(sig, postprocess=1)], None),   # batches do not postprocess
        (shapes, [P(sig, check=1), P(sig, check=1)], None),               # nor check
        (shapes, [P([1.0], model=1), P([1.0], model=1)], None),           # nor run the isotropic model
    ]
    for sh, prm, off in bad:
        with pytest.raises(m.MF4DError):
            m.Batch(sh, prm, offsets=off)
