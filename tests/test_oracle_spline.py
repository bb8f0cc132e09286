"""Pins of the oracle's bicubic-spline shift (natural cubic spline per row and column).

* The paper's own check (Sec. 3.1.1): an image of cubic B-spline basis functions is
  reproduced exactly by cubic-spline interpolation, so its shifted image is known in
  closed form without interpolating.
* Linear images are reproduced exactly; integer shifts are exact copies.
* Along one line the oracle agrees with SciPy's natural cubic spline (an independent
  implementation of the same definition).
"""
import numpy as np
import pytest

import oracle


def bspline3(u):
    a = np.abs(np.asarray(u, dtype=np.float64))
    return np.where(a < 1.0, 2.0 / 3.0 - a * a + a ** 3 / 2.0, np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))


def _bspline_image(H, W, centres, amps):
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.zeros((H, W))
    for (cx, cy), a in zip(centres, amps):
        img += a * bspline3(x - cx) * bspline3(y - cy)
    return img


@pytest.mark.parametrize("s", [(0.6, 0.7), (-1.35, 2.25), (0.5, -0.5), (3.0, -2.0)])
def test_bspline_image_is_shifted_exactly(s):
    rng = np.random.default_rng(11)
    H, W = 40, 56
    # supports [c-2, c+2] inside the frame: the natural end conditions hold exactly
    centres = [(int(rng.integers(2, W - 2)), int(rng.integers(2, H - 2))) for _ in range(25)]
    amps = rng.uniform(100.0, 5000.0, len(centres))
    img = _bspline_image(H, W, centres, amps)
    offs = np.array([s], dtype=np.float32)
    rect = oracle.valid_rect(offs, W, H)
    x0, y0, w, h = (int(v) for v in rect)
    got = oracle.shift_spline(img[None], offs, rect)[0]
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    sx, sy = float(offs[0, 0]), float(offs[0, 1])
    want = np.zeros((h, w))
    for (cx, cy), a in zip(centres, amps):
        want += a * bspline3(x0 + xx + sx - cx) * bspline3(y0 + yy + sy - cy)
    assert np.abs(got - want).max() <= 1e-9 * amps.max()


def test_linear_images_and_integer_shifts():
    H, W = 23, 31
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    img = 3.5 + 0.25 * x - 1.75 * y
    offs = np.array([[0.3, -0.8]], dtype=np.float32)
    rect = oracle.valid_rect(offs, W, H)
    x0, y0, w, h = (int(v) for v in rect)
    got = oracle.shift_spline(img[None], offs, rect)[0]
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    want = 3.5 + 0.25 * (x0 + xx + float(offs[0, 0])) - 1.75 * (y0 + yy + float(offs[0, 1]))
    assert np.abs(got - want).max() < 1e-12
    rnd = np.random.default_rng(5).normal(size=(H, W))
    got = oracle.shift_spline(rnd[None], np.array([[2.0, -3.0]], np.float32), (0, 3, W - 2, H - 3))[0]
    assert np.array_equal(got, rnd[0:H - 3, 2:W])


def test_one_line_matches_scipy_natural_spline():
    interp = pytest.importorskip("scipy.interpolate")
    rng = np.random.default_rng(3)
    f = rng.normal(size=(5, 97)) * 30.0 + 1000.0
    x = rng.uniform(0.0, 96.0, 200)
    M = oracle.spline.second_derivatives(f)
    got = oracle.spline.evaluate(f, M, x)
    for r in range(f.shape[0]):
        cs = interp.CubicSpline(np.arange(97.0), f[r], bc_type="natural")
        np.testing.assert_allclose(got[r], cs(x), rtol=1e-13, atol=1e-10)
        np.testing.assert_allclose(M[r], cs(np.arange(97.0), 2), rtol=1e-9, atol=1e-9)
