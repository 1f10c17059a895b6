"""The seeded synthetic inputs (CPU): deterministic per seed, float32 in
[0, 1], and the workloads the tests and the bench name."""
import numpy as np
import pytest

from paper_1611_06906_amd import synth


@pytest.mark.parametrize("gen", [
    lambda s: synth.creases(96, 130, 4, s),
    lambda s: synth.creases(96, 130, 6, s, background=0.5, amplitude=0.4, width_range=(1.0, 16.0), signs="mixed"),
    lambda s: synth.fundus(160, 128, s),
    lambda s: synth.noise_image(50, 70, s),
])
def test_generators_are_seeded(gen):
    a, b, c = gen(3), gen(3), gen(4)
    assert a.dtype == np.float32 and a.flags["C_CONTIGUOUS"]
    assert np.array_equal(a, b)            # same seed, same bits
    assert not np.array_equal(a, c)        # another seed, another image
    assert a.min() >= 0.0 and a.max() <= 1.0
    assert a.std() > 0.01                  # structure, not a constant


def test_workloads():
    w = synth.creases4096()
    assert (w.H, w.W, w.cycles, w.substeps, w.mode) == (4096, 4096, 30, 20, synth.BOTH)
    assert np.allclose(w.sigmas, [16.0 ** (k / 7.0) for k in range(8)]) and w.sigmas[0] == 1.0
    assert w.px_substeps == 4096 * 4096 * 30 * 20
    r = synth.ridges128()
    assert (r.H, r.W, r.cycles, r.substeps, r.mode, r.sigmas) == (128, 128, 5, 10, synth.RIDGE, [1.0, 1.5, 2.0, 3.0])
    f = synth.fundus1024()
    assert (f.H, f.W, f.cycles, f.substeps, f.mode, len(f.sigmas)) == (1024, 1024, 20, 15, synth.VALLEY, 6)
    img = r.image()
    assert img.shape == (128, 128) and np.array_equal(img, synth.ridges128().image())


def test_batch_specs():
    specs = synth.batch_of_images()
    assert specs == synth.batch_of_images()
    assert len(specs) == 256
    assert all(256 <= s["H"] <= 1536 and 256 <= s["W"] <= 1536 and 5 <= s["cycles"] <= 25 for s in specs)
    assert {s["mode"] for s in specs} == {synth.RIDGE, synth.VALLEY}
    small = dict(specs[0], H=64, W=80)
    ridge, valley = dict(small, mode=synth.RIDGE), dict(small, mode=synth.VALLEY)
    assert np.allclose(synth.batch_image(valley), 1.0 - synth.batch_image(ridge).astype(np.float64), atol=1e-7)
