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


def test_ground_truth_outputs():
    """The noise-free image and centrelines come from the same draws: the
    noisy image is unchanged, the noise-free one differs from it by the
    noise only, and the centreline samples lie inside the image."""
    from paper_1611_06906_amd import synth
    w = synth.ridges128()
    img, clean, lines = w.ground_truth()
    assert np.array_equal(img, w.image())
    assert clean.dtype == np.float32 and clean.min() >= 0 and clean.max() <= 1
    d = img.astype(np.float64) - clean
    assert 0.04 < d.std() < 0.06 and abs(d.mean()) < 0.005
    assert len(lines) == 3
    for pts, sgn in lines:
        assert sgn == 1.0 and pts.shape[1] == 2
        assert np.all(np.linalg.norm(np.diff(pts, axis=0), axis=1) < 1.0)
    img2, clean2, lines2 = synth.fundus(256, 256, 5, ground_truth=True)
    assert np.array_equal(img2, synth.fundus(256, 256, 5))
    assert all(sgn == -1.0 for _, sgn in lines2) and len(lines2) >= 4
