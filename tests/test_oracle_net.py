"""Pins of the FP64 oracle of the learned scale surrogate: the convolution
against a library 2-D correlation, the loss against its definition on a
hand-checked case, and every gradient against central finite differences."""
import math

import numpy as np
import pytest
from scipy import signal

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _theta(oracle_lib, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(scale=scale, size=oracle_lib.net_param_count())


def test_param_count(oracle_lib):
    c = oracle_lib.NET_CHANNELS
    assert oracle_lib.net_param_count() == sum(c[l + 1] * c[l] * 9 + c[l + 1] for l in range(5))


def test_forward_matches_scipy_correlation(oracle_lib):
    rng = np.random.default_rng(1)
    theta = _theta(oracle_lib, 2)
    u = rng.uniform(size=(2, 7, 9))
    z = oracle_lib.net_forward(theta, u)
    a = u[:, None]
    for l, (w, b) in enumerate(oracle_lib.net_unpack(theta)):
        out = np.zeros((a.shape[0], w.shape[0]) + u.shape[1:])
        for n in range(a.shape[0]):
            for co in range(w.shape[0]):
                out[n, co] = b[co] + sum(signal.correlate2d(a[n, ci], w[co, ci], mode="same", boundary="fill")
                                         for ci in range(w.shape[1]))
        a = np.maximum(out, 0) if l < 4 else out
    assert np.allclose(z, a, atol=1e-12)


def test_loss_definition(oracle_lib):
    # one pixel: logits (0, ..., 0, log 3 at k = 2), label 2, confidence logit 0
    z = np.zeros((1, 9, 1, 1))
    z[0, 2] = math.log(3.0)
    loss, dz = oracle_lib.net_loss(z, np.array([[[2]]]), w_conf=0.5)
    p2 = 3.0 / (3.0 + 7.0)
    assert math.isclose(loss, -math.log(p2) + 0.5 * math.log(2.0), rel_tol=1e-14)
    assert math.isclose(dz[0, 2, 0, 0], p2 - 1.0, rel_tol=1e-14)
    assert math.isclose(dz[0, 8, 0, 0], 0.5 * (0.5 - 1.0), rel_tol=1e-14)


def test_gradient_matches_finite_differences(oracle_lib):
    rng = np.random.default_rng(3)
    theta = _theta(oracle_lib, 4)
    u = rng.uniform(size=(2, 6, 5))
    lab = rng.integers(0, 8, size=(2, 6, 5)).astype(np.uint8)
    loss, g = oracle_lib.net_grad(theta, u, lab, 0.3)
    z = oracle_lib.net_forward(theta, u)
    assert math.isclose(loss, oracle_lib.net_loss(z, lab, 0.3)[0], rel_tol=1e-14)
    # the confidence target depends on the argmax: keep perturbations small
    idx = rng.choice(len(theta), size=60, replace=False)
    for l in range(5):   # include every bias vector
        off = sum(oracle_lib.NET_CHANNELS[k + 1] * (oracle_lib.NET_CHANNELS[k] * 9 + 1) for k in range(l))
        idx = np.append(idx, off + oracle_lib.NET_CHANNELS[l + 1] * oracle_lib.NET_CHANNELS[l] * 9)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (oracle_lib.net_loss(oracle_lib.net_forward(tp, u), lab, 0.3)[0]
              - oracle_lib.net_loss(oracle_lib.net_forward(tm, u), lab, 0.3)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(g[i])), (i, fd, g[i])
