"""The seeded input generators: determinism, value ranges and stacking order."""

import numpy as np

from synth import make_exact_rank, make_stereo_stack, serving_requests, haar_orthonormal
from synth.stack import _to_ycbcr, _to_ipt


def test_stack_is_deterministic_and_shaped():
    a = make_stereo_stack(40, 64, 3, "ycbcr", seed=5)
    b = make_stereo_stack(40, 64, 3, "ycbcr", seed=5)
    c = make_stereo_stack(40, 64, 3, "ycbcr", seed=6)
    assert a.shape == (40, 64, 3, 6) and a.dtype == np.float32
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_stack_ycbcr_ranges_and_exposure_order():
    x = make_stereo_stack(60, 96, 5, "ycbcr", seed=1)
    y, cb, cr = x[:, :, 0], x[:, :, 1], x[:, :, 2]
    assert y.min() >= 0.0 and y.max() <= 1.0 + 1e-6
    assert np.abs(cb).max() <= 0.5 + 1e-6 and np.abs(cr).max() <= 0.5 + 1e-6
    # within a view, luma grows with exposure (EV steps upward)
    for v in range(2):
        means = [y[:, :, v * 5 + e].mean() for e in range(5)]
        assert all(m1 > m0 for m0, m1 in zip(means, means[1:]))
    # the brightest exposure clips, the darkest much less and reaches dark values
    assert (y[:, :, 4] >= 1.0 - 1e-6).mean() > 0.01
    assert (y[:, :, 0] >= 1.0 - 1e-6).mean() < (y[:, :, 4] >= 1.0 - 1e-6).mean()
    assert y[:, :, 0].min() < 0.1


def test_stack_is_8bit_quantised_in_rgb():
    # Y'CbCr is linear in R'G'B', so invert it and check the 8-bit grid
    x = make_stereo_stack(32, 48, 3, "ycbcr", seed=2).astype(np.float64)
    y, cb, cr = x[:, :, 0], x[:, :, 1], x[:, :, 2]
    r = y + 1.402 * cr
    b = y + 1.772 * cb
    g = (y - 0.299 * r - 0.114 * b) / 0.587
    for ch in (r, g, b):
        q = ch * 255.0
        assert np.abs(q - np.round(q)).max() < 1e-3


def test_stereo_views_differ_by_horizontal_shift():
    x = make_stereo_stack(48, 128, 1, "ycbcr", seed=3)
    left, right = x[:, :, 0, 0], x[:, :, 0, 1]
    assert not np.array_equal(left, right)
    # some shift in [0, 32] explains the right view far better than no shift
    errs = [np.abs(left[:, s:s + 64] - right[:, 0:64]).mean() for s in range(0, 33)]
    assert min(errs) < 0.5 * errs[0] + 1e-9 or errs[0] < 1e-3


def test_colour_transforms_white_and_black():
    white = np.ones((3, 1, 1))
    ycc = _to_ycbcr(white)
    assert abs(ycc[0].item() - 1.0) < 1e-12 and abs(ycc[1].item()) < 1e-12 and abs(ycc[2].item()) < 1e-12
    ipt = _to_ipt(white)
    assert abs(ipt[1].item()) < 0.01 and abs(ipt[2].item()) < 0.01   # D65 white is achromatic
    assert np.allclose(_to_ipt(np.zeros((3, 1, 1))), 0.0)


def test_exact_rank_builder():
    x, core, fac = make_exact_rank((7, 6, 5), (2, 3, 2), seed=0)
    for u in fac:
        assert np.allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-13)
    for n, r in enumerate((2, 3, 2)):
        s = np.linalg.svd(np.moveaxis(x, n, 0).reshape(x.shape[n], -1), compute_uv=False)
        assert s[r] < 1e-12 * s[0]
    q = haar_orthonormal(np.random.default_rng(1), 5, 5)
    assert np.allclose(q @ q.T, np.eye(5), atol=1e-13)


def test_serving_requests():
    reqs = serving_requests(64, seed=3)
    assert len(reqs) == 64
    assert reqs[0]["t_arrive"] == 0.0
    assert all(b["t_arrive"] >= a["t_arrive"] for a, b in zip(reqs, reqs[1:]))
    for r in reqs:
        assert r["ranks"] == (r["H"] // 4, r["W"] // 4, 3, 2 * r["E"] - 1)
    assert serving_requests(64, seed=3) == reqs
