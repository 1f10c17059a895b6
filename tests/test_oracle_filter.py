"""Whole-filter invariants of the oracle (Sec. 3.5 Eq. (21); rotational
invariance goal of Sec. 4.1)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.usefixtures("oracle_lib")

SIG = [1.0, 1.5, 2.5]


def _img(seed, H=28, W=28):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:H, 0:W].astype(float)
    u = 0.3 + 0.5 * np.exp(-((x - 0.4 * W - 0.3 * y) ** 2) / 6.0) + rng.normal(0, 0.05, (H, W))
    return np.clip(u, 0, 1).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_d4_equivariance(oracle_lib, mode):
    u = _img(1)
    f = lambda v: oracle_lib.filter(v, SIG, mode, cycles=2, substeps=6)
    out = f(u)
    for op in (lambda a: a.T, lambda a: a[::-1], lambda a: a[:, ::-1], lambda a: np.rot90(a)):
        assert np.allclose(f(np.ascontiguousarray(op(u))), op(out), atol=1e-10)


def test_mass_conserved_and_changes_image(oracle_lib):
    u = _img(2, 32, 40)
    out = oracle_lib.filter(u, SIG, 0, cycles=3, substeps=10)
    assert math.isclose(out.sum(), u.sum(), rel_tol=1e-12)
    assert np.abs(out - u).max() > 1e-2


def test_order_independence_within_a_cycle(oracle_lib):
    # P is frozen within a cycle, so the factors (I - tau_i P) commute
    rng = np.random.default_rng(3)
    u = rng.uniform(size=(20, 20))
    D = oracle_lib.dtensor(rng.normal(scale=0.01, size=(3, 20, 20)), 0.005, 2)
    ordered, _, _ = oracle_lib.fed_schedule(10, 0.05)
    a = oracle_lib.fed_cycle(u, D, ordered)
    b = oracle_lib.fed_cycle(u, D, np.sort(ordered))
    c = oracle_lib.fed_cycle(u, D, ordered[::-1])
    assert np.allclose(a, b, atol=1e-9) and np.allclose(a, c, atol=1e-9)


def test_affine_and_constant_images_are_stationary(oracle_lib):
    H, W = 24, 26
    y, x = np.mgrid[0:H, 0:W].astype(float)
    u = 0.25 + x / 1024 + y / 2048
    for mode in (0, 1, 2):
        assert np.array_equal(oracle_lib.filter(u, SIG, mode, cycles=2, substeps=5), u)
    c = np.full((H, W), 0.6)
    out, rec = oracle_lib.filter(c, SIG, 0, cycles=2, substeps=5, record=True)
    assert np.array_equal(out, c) and np.all(rec["idx"] == 0) and np.all(rec["c"] == 0)


def test_stop_time_path_matches_given_n(oracle_lib):
    u = _img(4, 20, 20)
    n, M = 6, 2
    T = M * 0.05 * (n * n + n) / 3
    a = oracle_lib.filter(u, SIG, 2, cycles=M, substeps=n)
    b = oracle_lib.filter(u, SIG, 2, cycles=M, substeps=0, stop_time=T)
    assert np.allclose(a, b, atol=1e-12)


def test_records_are_consistent(oracle_lib):
    u = _img(5, 24, 24)
    out, rec = oracle_lib.filter(u, SIG, 0, cycles=2, substeps=4, record=True)
    assert np.array_equal(rec["u"][-1], out)
    sel = oracle_lib.scale_select(u, SIG, 0)
    assert np.array_equal(rec["idx"][0], sel["idx"]) and rec["c"][0] == sel["c"]
    hr = oracle_lib.tensor(u, sel["idx"], SIG, 0.5)
    assert np.allclose(rec["hrho"][0], hr, atol=0)
    D = oracle_lib.dtensor(hr, float(np.float32(0.005)), 0)
    ordered, _, _ = oracle_lib.fed_schedule(4)
    assert np.allclose(rec["u"][0], oracle_lib.fed_cycle(u, D, ordered), atol=0)
