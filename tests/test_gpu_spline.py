"""Parity of the HIP bicubic-spline shift (natural cubic spline per row and column)
against the FP64 oracle: several row and column tiles with ragged ends, frames whose
overlap touches the frame edges (end corrections), tiny lines, integer shifts (exact
copies) and the cubic B-spline image whose shifted version is known in closed form.
"""
import numpy as np
import pytest

import synth
from helpers import TOL, err_summary, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2008_11486_amd as rd
    rd.lib()
    return rd


def _run(rd, orc, frames, s, rect=None):
    N, H, W = frames.shape
    s = np.asarray(s, dtype=np.float32).reshape(N, 2)
    if rect is None:
        rect = orc.valid_rect(s, W, H)
    got = rd.shift_spline(to_dev(frames.astype(np.float32)), to_dev(s), rect).cpu().numpy()
    want = orc.shift_spline(frames.astype(np.float32).astype(np.float64), s, rect)
    return got, want, rect


@pytest.mark.parametrize("shape,seed", [((3, 530, 600), 1), ((2, 77, 300), 2), ((4, 130, 64), 3), ((2, 257, 257), 4)])
def test_spline_parity_sky_frames(rd, orc, shape, seed):
    N, H, W = shape
    spec = synth.small_spec(N, W, H, n_stars=max(10, W * H // 1500), shift_bound=6.0, seed=(seed, 9))
    st = synth.make_stack(spec)
    cal = orc.calibrate(st.raw, st.dark, st.flat).astype(np.float32)
    rng = np.random.default_rng(seed)
    s = np.zeros((N, 2), np.float32)
    s[1:] = rng.uniform(-6, 6, (N - 1, 2))
    got, want, rect = _run(rd, orc, cal, s)
    e = rel_err(got, want)
    print(f"spline {shape} rect {list(rect)}: {err_summary(e)}")
    assert e.max() <= TOL


def test_spline_edges_tiny_lines_and_integer_shifts(rd, orc):
    rng = np.random.default_rng(7)
    # a rect that reaches both ends of rows and columns (offsets within (-1, 1))
    f = (1000.0 + 50.0 * rng.normal(size=(2, 40, 70))).astype(np.float32)
    got, want, _ = _run(rd, orc, f, [[0.0, 0.0], [0.4, -0.3]], rect=(0, 0, 69, 39))
    assert rel_err(got, want).max() <= TOL
    # two- and three-pixel lines
    f = (1000.0 + 50.0 * rng.normal(size=(2, 3, 2))).astype(np.float32)
    got, want, _ = _run(rd, orc, f, [[0.25, 0.5], [0.75, 0.1]], rect=(0, 0, 1, 2))
    assert rel_err(got, want).max() <= TOL
    # integer shifts are exact copies
    f = (1000.0 + 50.0 * rng.normal(size=(2, 50, 90))).astype(np.float32)
    got, _, rect = _run(rd, orc, f, [[0.0, 0.0], [3.0, -2.0]])
    x0, y0, w, h = (int(v) for v in rect)
    assert np.array_equal(got[1], f[1, y0 - 2:y0 - 2 + h, x0 + 3:x0 + 3 + w])


def test_spline_reproduces_shifted_bspline_image(rd, orc):
    import test_oracle_spline as t
    rng = np.random.default_rng(12)
    H, W = 96, 300
    centres = [(int(rng.integers(2, W - 2)), int(rng.integers(2, H - 2))) for _ in range(60)]
    amps = rng.uniform(100.0, 5000.0, len(centres))
    img = t._bspline_image(H, W, centres, amps)
    s = np.array([[0.6, 0.7]], np.float32)
    rect = orc.valid_rect(s, W, H)
    x0, y0, w, h = (int(v) for v in rect)
    got = rd.shift_spline(to_dev(img.astype(np.float32)[None]), to_dev(s), rect).cpu().numpy()[0]
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    want = np.zeros((h, w))
    for (cx, cy), a in zip(centres, amps):
        want += a * t.bspline3(x0 + xx + 0.6000000238418579 - cx) * t.bspline3(y0 + yy + 0.699999988079071 - cy)
    assert np.abs(got - want).max() <= 1e-5 * amps.max()
