"""Pins of the FP64 oracle to facts outside itself (CPU only).

Each test ties one oracle function to a closed form, an invariant, a brute-force
evaluation or an independent library routine, chosen so that a dropped term, a
wrong sign or index or a transposed operand in the oracle fails at least one test.
"""
import math
import os

import numpy as np
import pytest
import scipy.ndimage
import scipy.signal
import scipy.stats

import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ----------------------------------------------------------------------------- calibrate
def _rand_raw(rng, N, H, W):
    return rng.integers(0, 65536, size=(N, H, W), dtype=np.uint16)


def test_calibrate_unit_flat_zero_dark_is_identity(orc):
    rng = np.random.default_rng(1)
    raw = _rand_raw(rng, 3, 17, 23)
    out = orc.calibrate(raw, np.zeros((17, 23)), np.ones((17, 23)))
    assert np.array_equal(out, raw.astype(np.float64))


def test_calibrate_recovers_exact_signal(orc):
    # raw = dark + flat * S with integer S, integer dark and power-of-two flat is exact,
    # so the calibrated value must be S itself.
    rng = np.random.default_rng(2)
    H, W = 19, 31
    S = 4.0 * rng.integers(0, 1000, size=(4, H, W))
    dark = rng.integers(90, 110, size=(H, W)).astype(np.float64)
    flat = rng.choice([0.25, 0.5, 1.0, 2.0, 4.0], size=(H, W))
    raw = (dark + flat * S).astype(np.uint16)
    assert np.array_equal(raw.astype(np.float64), dark + flat * S)
    assert np.array_equal(orc.calibrate(raw, dark, flat), S)


def test_calibrate_inverts_with_general_flat(orc):
    rng = np.random.default_rng(3)
    H, W = 13, 29
    raw = _rand_raw(rng, 2, H, W)
    dark = 100 + rng.normal(0, 3, size=(H, W))
    flat = rng.uniform(0.95, 1.05, size=(H, W))
    cal = orc.calibrate(raw, dark, flat)
    # multiplying back by the flat and adding the dark returns the raw counts
    np.testing.assert_allclose(cal * flat + dark, raw.astype(np.float64), rtol=1e-13, atol=1e-9)
    # a constant flat c scales the dark-subtracted frame by exactly 1/c
    c = 0.8
    cal_c = orc.calibrate(raw, dark, np.full((H, W), c))
    np.testing.assert_allclose(cal_c * c, raw - dark, rtol=1e-14, atol=1e-10)


def test_calibrate_pitched_roi_equals_cropped_copy(orc):
    # the overscan cut of Section 2.1 expressed as a view with a larger row pitch
    rng = np.random.default_rng(4)
    full = _rand_raw(rng, 3, 24, 40)
    roi = full[:, 2:22, 2:32]
    dark = rng.normal(100, 3, size=(24, 40))[2:22, 2:32]
    flat = rng.uniform(0.9, 1.1, size=(24, 40))[2:22, 2:32]
    a = orc.calibrate(roi, dark, flat)
    b = orc.calibrate(np.ascontiguousarray(roi), np.ascontiguousarray(dark), np.ascontiguousarray(flat))
    assert np.array_equal(a, b)


# ----------------------------------------------------------------------------- register
def _interior_canvas(rng, H, W, n_stars, lo, hi):
    """Noisy sky with every star stamp inside [lo, hi) on both axes."""
    m = synth.STAMP_HALF + 1
    stars = np.stack([rng.uniform(lo + m, hi - m, n_stars), rng.uniform(lo + m, hi - m, n_stars),
                      np.exp(rng.uniform(np.log(2e3), np.log(5e4), n_stars))], axis=1)
    sky = synth.render_sky(W, H, stars, (0.0, 0.0))
    return sky + rng.normal(0, 10, size=sky.shape)


@pytest.mark.parametrize("t", [(0, 0), (3, -2), (-5, 4), (1, 5), (-4, -4)])
def test_register_recovers_injected_integer_shift(orc, t):
    # The frame is cut from a larger canvas at an offset, so frame(x + t) = ref(x)
    # holds exactly.  Stars are kept clear of the template border: a star cut by the
    # fixed template biases an unnormalised correlation towards its centre.
    rng = np.random.default_rng(100 + t[0] * 7 + t[1])
    H = W = 96
    R = 6
    pad = R + 2
    C = _interior_canvas(rng, H + 2 * pad, W + 2 * pad, 14, pad + 2 * R, pad + W - 2 * R)
    x0 = y0 = pad
    ref = C[y0:y0 + H, x0:x0 + W]
    tx, ty = t
    # frame(x + t) = ref(x)  <=>  frame(x) = C(x0 + x - t)
    frame = C[y0 - ty:y0 - ty + H, x0 - tx:x0 - tx + W]
    res = orc.register(ref, np.stack([ref, frame]), R)
    assert (res["dx"][1], res["dy"][1]) == (tx, ty)
    assert (res["dx"][0], res["dy"][0]) == (0, 0)
    assert res["flags"][1] & (orc.EDGE_X | orc.EDGE_Y) == 0
    assert abs(res["sx"][1] - tx) < 0.5 and abs(res["sy"][1] - ty) < 0.5


@pytest.mark.parametrize("R,shape,tmpl", [(0, (9, 11), None), (1, (12, 10), None),
                                          (3, (16, 16), None), (2, (16, 20), (3, 4, 9, 7))])
def test_register_scores_match_scipy_correlate(orc, R, shape, tmpl):
    rng = np.random.default_rng(20 + R)
    H, W = shape
    Rmax = 3 if tmpl is not None else R
    ref = rng.normal(0, 1, size=(H, W)) + 5
    frame = rng.normal(0, 1, size=(H, W)) + 5
    res, S = orc.register(ref, frame[None], R, Rmax, tmpl=tmpl, want_scores=True)
    x0, y0, tw, th = tmpl if tmpl is not None else (Rmax, Rmax, W - 2 * Rmax, H - 2 * Rmax)
    rt = ref[y0:y0 + th, x0:x0 + tw]
    rp = rt - rt.mean()
    win = frame[y0 - R:y0 + th + R, x0 - R:x0 + tw + R]
    # correlate(in1, in2, 'valid')[j, i] = sum in1[j + y, i + x] * in2[y, x]  = S(dy=j-R, dx=i-R)
    ref_scores = scipy.signal.correlate(win, rp, mode="valid", method="direct")
    assert ref_scores.shape == S[0].shape
    np.testing.assert_allclose(S[0], ref_scores, rtol=1e-12, atol=1e-10 * np.abs(ref_scores).max())
    j, i = np.unravel_index(np.argmax(ref_scores), ref_scores.shape)
    assert (res["dx"][0], res["dy"][0]) == (i - R, j - R)
    srt = np.sort(ref_scores.ravel())
    assert res["peak"][0] == pytest.approx(srt[-1], rel=1e-12)
    if srt.size > 1:
        assert res["second"][0] == pytest.approx(srt[-2], rel=1e-12)
        assert res["margin"][0] == pytest.approx((srt[-1] - srt[-2]) / abs(srt[-1]), rel=1e-6, abs=1e-15)
    else:
        assert res["second"][0] == -np.inf and res["margin"][0] == np.inf


def _impulse_pair(H, W, p, a, b):
    ref = np.zeros((H, W))
    ref[p[1], p[0]] = 100.0
    frame = np.zeros((H, W))
    frame[p[1] + a[1], p[0] + a[0]] = 7.0
    frame[p[1] + b[1], p[0] + b[0]] = 7.0
    return ref, frame


@pytest.mark.parametrize("a,b,win", [((1, 0), (-1, 0), (-1, 0)), ((0, 1), (0, -1), (0, -1)),
                                     ((1, -1), (-1, 1), (1, -1)), ((2, 2), (-2, 2), (-2, 2))])
def test_register_tie_break_prefers_smaller_dy_then_dx(orc, a, b, win):
    H = W = 21
    ref, frame = _impulse_pair(H, W, (10, 10), a, b)
    res = orc.register(ref, frame[None], 3)
    assert (res["dx"][0], res["dy"][0]) == win
    assert res["margin"][0] == 0.0 and res["flags"][0] & orc.NEAR_TIE


def test_register_subpixel_recovery_bound(orc):
    # Analytically rendered sub-pixel shifts (no interpolation), noiseless sky, stars
    # clear of the template border.  The correlation peak of a Gaussian star of
    # sigma = FWHM / 2.355 is a Gaussian of sigma * sqrt(2); a 3-point parabola through
    # its integer samples is biased towards the sample by at most 0.015 px; overlapping
    # stars add cross terms of the same order, hence the 0.05 px bound.
    rng = np.random.default_rng(30)
    H = W = 160
    R = 6
    m = synth.STAMP_HALF + 1 + 2 * R
    errs = []
    for trial in range(12):
        stars = np.stack([rng.uniform(m, W - m, 30), rng.uniform(m, H - m, 30),
                          np.exp(rng.uniform(np.log(2e3), np.log(5e4), 30))], axis=1)
        t = rng.uniform(-5, 5, size=2)
        ref = synth.render_sky(W, H, stars, (0, 0))
        frame = synth.render_sky(W, H, stars, t)
        res = orc.register(ref, frame[None], R)
        errs.append(max(abs(res["sx"][0] - t[0]), abs(res["sy"][0] - t[1])))
        assert (res["dx"][0], res["dy"][0]) == (int(np.rint(t[0])), int(np.rint(t[1])))
    assert max(errs) < 0.05, errs


def test_register_vertex_matches_polyfit(orc):
    # the fraction is the vertex of the parabola through d* and its two neighbours
    rng = np.random.default_rng(33)
    H = W = 80
    R = 5
    stars = np.stack([rng.uniform(0, W, 25), rng.uniform(0, H, 25),
                      np.exp(rng.uniform(np.log(2e3), np.log(5e4), 25))], axis=1)
    ref = synth.render_sky(W, H, stars, (0, 0)) + rng.normal(0, 10, (H, W))
    ts = rng.uniform(-3.5, 3.5, size=(6, 2))
    frames = np.stack([synth.render_sky(W, H, stars, t) + rng.normal(0, 10, (H, W)) for t in ts])
    res, S = orc.register(ref, frames, R, want_scores=True)
    for k in range(6):
        dx, dy = int(res["dx"][k]), int(res["dy"][k])
        j, i = dy + R, dx + R
        px = np.polyfit([-1.0, 0.0, 1.0], S[k, j, i - 1:i + 2], 2)
        py = np.polyfit([-1.0, 0.0, 1.0], S[k, j - 1:j + 2, i], 2)
        vx, vy = -px[1] / (2 * px[0]), -py[1] / (2 * py[0])
        assert abs(vx) <= 0.5 and abs(vy) <= 0.5
        assert res["sx"][k] == pytest.approx(dx + vx, abs=2e-6)
        assert res["sy"][k] == pytest.approx(dy + vy, abs=2e-6)


def test_register_border_peak_sets_edge_and_zero_fraction(orc):
    # one star moved by 9.3 px: within the +-4 window the score rises monotonically
    # towards +x, so the maximum sits on the window border
    H = W = 96
    stars = np.array([[40.0, 48.0, 2e4]])
    ref = synth.render_sky(W, H, stars, (0, 0))
    frame = synth.render_sky(W, H, stars, (9.3, -0.4))
    res = orc.register(ref, frame[None], 4, 10)
    assert res["dx"][0] == 4 and res["flags"][0] & orc.EDGE_X
    assert res["sx"][0] == 4.0
    assert not res["flags"][0] & orc.EDGE_Y


def test_register_centred_window_matches_full_search(orc):
    rng = np.random.default_rng(32)
    H = W = 128
    stars = np.stack([rng.uniform(0, W, 40), rng.uniform(0, H, 40),
                      np.exp(rng.uniform(np.log(2e3), np.log(5e4), 40))], axis=1)
    ref = synth.render_sky(W, H, stars, (0, 0)) + rng.normal(0, 10, (H, W))
    ts = [(7.2, -3.6), (-9.8, 8.1), (0.4, 10.7)]
    frames = np.stack([synth.render_sky(W, H, stars, t) + rng.normal(0, 10, (H, W)) for t in ts])
    full = orc.register(ref, frames, 12)
    centers = np.array([[7, -4], [-9, 7], [1, 11]], dtype=np.int32)
    loc = orc.register(ref, frames, 2, 12, centers=centers)
    for k in range(3):
        assert (loc["dx"][k], loc["dy"][k]) == (full["dx"][k], full["dy"][k])
        assert loc["sx"][k] == full["sx"][k] and loc["sy"][k] == full["sy"][k]
        assert loc["peak"][k] == full["peak"][k]
    # a window clipped at +-Rmax is flagged
    clipped = orc.register(ref, frames[:1], 2, 12, centers=np.array([[11, 0]], dtype=np.int32))
    assert clipped["flags"][0] & orc.CLIPPED


def test_register_rejects_bad_template(orc):
    ref = np.zeros((16, 16))
    with pytest.raises(orc.OracleError):
        orc.register(ref, ref[None], 2, 2, tmpl=(1, 2, 8, 8))


# ----------------------------------------------------------------------------- valid rect
def test_valid_rect_brute_force(orc):
    rng = np.random.default_rng(40)
    for trial in range(20):
        W, H = int(rng.integers(20, 60)), int(rng.integers(20, 60))
        N = int(rng.integers(1, 6))
        offs = rng.uniform(-6, 6, size=(N, 2)).astype(np.float32)
        if trial % 3 == 0:
            offs = np.rint(offs)
        rect = orc.valid_rect(offs, W, H)
        xs = [x for x in range(-10, W + 10)
              if all(0 <= x + float(o[0]) <= W - 1 for o in offs)]
        ys = [y for y in range(-10, H + 10)
              if all(0 <= y + float(o[1]) <= H - 1 for o in offs)]
        assert (rect[0], rect[2]) == (xs[0], len(xs)) and xs[-1] == xs[0] + len(xs) - 1
        assert (rect[1], rect[3]) == (ys[0], len(ys))


# ----------------------------------------------------------------------------- shift
def test_shift_integer_offset_is_exact_copy(orc):
    rng = np.random.default_rng(50)
    f = rng.normal(1000, 30, size=(3, 30, 40))
    offs = np.array([[0, 0], [3, -2], [-4, 5]], dtype=np.float32)
    rect = orc.valid_rect(offs, 40, 30)
    out = orc.shift(f, offs, rect)
    x0, y0, w, h = rect
    for k in range(3):
        sx, sy = int(offs[k, 0]), int(offs[k, 1])
        assert np.array_equal(out[k], f[k, y0 + sy:y0 + sy + h, x0 + sx:x0 + sx + w])


def test_shift_reproduces_bilinear_functions_exactly(orc):
    # f = alpha + beta x + gamma y + eta x y lies in the bilinear space, so sampling it at
    # any shifted position gives the analytic value (the bilinear analogue of the
    # paper's exactly reproducible B-spline image, Section 3.1.1)
    H, W = 25, 33
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    al, be, ga, et = 1000.0, 3.25, -1.5, 0.0625
    f = al + be * xx + ga * yy + et * xx * yy
    offs = np.array([[0.3, 0.2], [-1.7, 2.45], [0.5, -0.5], [2.0, 0.125]], dtype=np.float32)
    rect = orc.valid_rect(offs, W, H)
    out = orc.shift(np.stack([f] * 4), offs, rect)
    x0, y0, w, h = rect
    v, u = np.mgrid[0:h, 0:w].astype(np.float64)
    for k in range(4):
        X = x0 + u + float(offs[k, 0])
        Y = y0 + v + float(offs[k, 1])
        np.testing.assert_allclose(out[k], al + be * X + ga * Y + et * X * Y, rtol=1e-14, atol=1e-11)


def test_shift_round_trip_closed_form(orc):
    # shifting by +a then by -a equals a 3-tap blur [a(1-a), a^2+(1-a)^2, a(1-a)] per axis
    # (the analogue of the paper's set B, Section 3.1.1)
    rng = np.random.default_rng(51)
    H, W = 20, 24
    f = rng.normal(1000, 50, size=(H, W))
    a, b = 0.6, 0.7
    g = orc.shift(f, np.array([[a, b]], dtype=np.float32), [0, 0, W - 1, H - 1])[0]
    back = orc.shift(g, np.array([[-a, -b]], dtype=np.float32), [1, 1, W - 2, H - 2])[0]
    a32, b32 = float(np.float32(a)), float(np.float32(b))
    kx = np.array([a32 * (1 - a32), a32 ** 2 + (1 - a32) ** 2, a32 * (1 - a32)])
    ky = np.array([b32 * (1 - b32), b32 ** 2 + (1 - b32) ** 2, b32 * (1 - b32)])
    expect = scipy.signal.convolve2d(f, np.outer(ky, kx), mode="valid")
    np.testing.assert_allclose(back, expect[:H - 2, :W - 2], rtol=1e-13)


def test_shift_matches_scipy_ndimage_order1(orc):
    rng = np.random.default_rng(52)
    H, W = 40, 50
    f = rng.normal(1000, 100, size=(H, W))
    for s in [(0.3, 0.2), (-2.6, 1.35), (4.75, -3.5)]:
        offs = np.array([[0.0, 0.0], s], dtype=np.float32)  # the reference keeps rect inside
        rect = orc.valid_rect(offs, W, H)
        out = orc.shift(np.stack([f, f]), offs, rect)[1]
        # ndimage.shift(f, shift) gives f(x - shift): pass -s to sample f(x + s)
        ref = scipy.ndimage.shift(f, (-float(offs[1, 1]), -float(offs[1, 0])), order=1, mode="nearest")
        x0, y0, w, h = rect
        np.testing.assert_allclose(out, ref[y0:y0 + h, x0:x0 + w], rtol=1e-12)


# ----------------------------------------------------------------------------- combine
def test_combine_identical_frames(orc):
    rng = np.random.default_rng(60)
    fr = rng.normal(1000, 30, size=(1, 9, 11))
    for N in (1, 2, 5, 16, 30):
        out, keep, nrej, _ = orc.combine(np.repeat(fr, N, axis=0))
        assert keep.all() and nrej == 0
        if N <= 2:  # v and v + v = 2v are exact, and so is the division
            assert np.array_equal(out, fr[0])
        else:  # N-fold sequential sum (kv rounds for k > 2), then one division
            np.testing.assert_allclose(out, fr[0], rtol=N * 2.3e-16, atol=0)


def test_combine_small_stacks_never_reject(orc):
    # Samuelson: |x - m| <= sigma sqrt(n - 1), so with k = 3 nothing is dropped for n <= 10
    rng = np.random.default_rng(61)
    for N in range(1, 11):
        a = rng.standard_cauchy(size=(N, 8, 8)) * 100 + 1000
        out, keep, nrej, _ = orc.combine(a)
        assert keep.all() and nrej == 0
        np.testing.assert_allclose(out, a.mean(axis=0), rtol=1e-14)


def test_combine_single_outlier_closed_form(orc):
    # 15 equal values v and one outlier o: z = sqrt(15) > 3 rejects o at iteration 1,
    # then sigma = 0 keeps the rest, so the output is exactly v
    v, o = 1234.5, 1.0e5
    for pos in (0, 7, 15):
        col = np.full(16, v)
        col[pos] = o
        out, keep, nrej, _ = orc.combine(col.reshape(16, 1, 1))
        assert out[0, 0] == v and nrej == 1
        assert keep[:, 0, 0].tolist() == [0 if k == pos else 1 for k in range(16)]


def test_combine_exact_threshold_is_kept(orc):
    # [0]*9 + [10]: mean 1, sigma 3, |10 - 1| = 9 = 3 sigma exactly; the strict test keeps it
    col = np.array([0.0] * 9 + [10.0]).reshape(10, 1, 1)
    out, keep, nrej, near = orc.combine(col)
    assert out[0, 0] == 1.0 and keep.all() and nrej == 0 and near[9, 0, 0] == 1
    lo, hi, _ = (None, None, None)
    c, lo, hi = scipy.stats.sigmaclip(col.ravel(), 3, 3)
    assert c.size == 10


def test_combine_matches_scipy_sigmaclip_when_converged(orc):
    rng = np.random.default_rng(62)
    checked = 0
    for trial in range(300):
        N = int(rng.integers(11, 40))
        col = rng.normal(1000, 10, size=N)
        nout = int(rng.integers(0, 5))
        col[:nout] += rng.uniform(100, 5e4, size=nout) * rng.choice([-1, 1], size=nout)
        rng.shuffle(col)
        out_lim, keep_lim, _, _ = orc.combine(col.reshape(N, 1, 1), max_iters=3)
        out_inf, keep_inf, _, _ = orc.combine(col.reshape(N, 1, 1), max_iters=1000)
        c, _, _ = scipy.stats.sigmaclip(col, 3, 3)
        assert keep_inf.sum() == c.size
        assert out_inf[0, 0] == pytest.approx(c.mean(), rel=1e-13)
        if np.array_equal(keep_lim, keep_inf):
            assert out_lim[0, 0] == out_inf[0, 0]
            checked += 1
    assert checked > 250


def test_combine_iteration_cap_and_zero_iterations(orc):
    # a column that needs several passes: each pass removes only the largest remaining outlier
    base = [0.0] * 30
    col = np.array(base + [1e6, 1e4, 1e2, 12.0])
    N = col.size
    passes = []
    for it in range(0, 6):
        _, keep, nrej, _ = orc.combine(col.reshape(N, 1, 1), max_iters=it)
        passes.append(nrej)
    assert passes[0] == 0
    assert passes == sorted(passes) and passes[1] >= 1 and passes[3] > passes[1]
    out0, _, _, _ = orc.combine(col.reshape(N, 1, 1), max_iters=0)
    assert out0[0, 0] == pytest.approx(col.mean(), rel=1e-15)


# ----------------------------------------------------------------------------- downsample
def test_downsample_constant_and_linear(orc):
    H, W = 16, 24
    assert np.array_equal(orc.downsample4(np.full((H, W), 3.5)), np.full((4, 6), 3.5))
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    f = 7.0 + 0.5 * xx - 0.25 * yy
    j, i = np.mgrid[0:4, 0:6].astype(np.float64)
    np.testing.assert_allclose(orc.downsample4(f), 7.0 + 0.5 * (4 * i + 1.5) - 0.25 * (4 * j + 1.5), rtol=1e-15)
    rng = np.random.default_rng(70)
    g = rng.normal(size=(H, W))
    np.testing.assert_allclose(orc.downsample4(g), g.reshape(4, 4, 6, 4).mean(axis=(1, 3)), rtol=1e-13, atol=1e-15)


# ----------------------------------------------------------------------------- end to end
def test_end_to_end_small_stack_recovers_integer_shifts(orc):
    st = synth.make_config(0)[0]
    res = orc.reduce_stack(st.raw, st.dark, st.flat, st.spec.radius, integer_mode=True)
    assert np.array_equal(np.stack([res["offsets"]["dx"], res["offsets"]["dy"]], 1)[1:],
                          st.shifts[1:].astype(np.int64))
    assert res["n_rej"] == 0  # N = 5 can never reject


def test_combine_golden_closed_forms(orc):
    """Hand-derived cases in tests/golden/sigma_clip_closed_forms.txt."""
    path = os.path.join(os.path.dirname(__file__), "golden", "sigma_clip_closed_forms.txt")
    n = 0
    for line in open(path):
        if not line.strip() or line.startswith("#"):
            continue
        want, mask, vals = [p.strip() for p in line.split("|")]
        v = np.array([float(t) for t in vals.split()])
        out, keep, nrej, _ = orc.combine(v.reshape(-1, 1, 1), 3.0, 3)
        assert out[0, 0] == float(want)
        assert "".join(str(int(b)) for b in keep[:, 0, 0]) == mask
        assert nrej == mask.count("0")
        n += 1
    assert n == 5


# ----------------------------------------------------------------------------- bias, bad pixels
def test_calibrate_bias_then_dark_then_flat(orc):
    """Section 2.1's order: the cast at the bias subtraction, then dark, then flat.  With
    integer bias, dark and signal and a power-of-two flat every step is exact."""
    rng = np.random.default_rng(81)
    N, H, W = 3, 9, 13
    bias = rng.integers(200, 400, size=(H, W)).astype(np.float32)
    dark = rng.integers(10, 90, size=(H, W)).astype(np.float32)
    flat = rng.choice([0.5, 1.0, 2.0], size=(H, W)).astype(np.float32)
    S = 2 * rng.integers(0, 10000, size=(N, H, W))  # flat * S is an integer
    raw = (bias + dark + flat * S).astype(np.uint16)
    assert np.array_equal(orc.calibrate(raw, dark, flat, bias=bias), S.astype(np.float64))
    # without a bias frame, a dark that carries the bias gives the same frames
    assert np.array_equal(orc.calibrate(raw, dark + bias, flat), S.astype(np.float64))


@pytest.mark.parametrize("s", [(0.0, 0.0), (3.0, -2.0), (0.25, 0.0), (0.0, -0.75), (1.5, 2.25)])
def test_shift_bad_pixel_reaches_exactly_its_taps(orc, s):
    """A bad pixel at (px, py) makes missing exactly the outputs whose bilinear taps
    include it: columns i with px in {i, i + 1 if the x fraction is non-zero}, rows
    likewise; every other output equals the unmasked shift."""
    rng = np.random.default_rng(82)
    H, W = 24, 30
    f = rng.normal(1000, 20, size=(1, H, W))
    mask = np.zeros((H, W), np.uint8)
    px, py = 14, 11
    mask[py, px] = 1
    offs = np.array([s], np.float32)
    rect = orc.valid_rect(offs, W, H)
    x0, y0, w, h = (int(v) for v in rect)
    got = orc.shift(f, offs, rect, mask)[0]
    plain = orc.shift(f, offs, rect)[0]
    fx, fy = np.floor(s[0]), np.floor(s[1])
    cols = {px - (x0 + int(fx))} | ({px - 1 - (x0 + int(fx))} if s[0] != fx else set())
    rows = {py - (y0 + int(fy))} | ({py - 1 - (y0 + int(fy))} if s[1] != fy else set())
    want = np.zeros((h, w), bool)
    for v in rows:
        for u in cols:
            if 0 <= v < h and 0 <= u < w:
                want[v, u] = True
    assert np.array_equal(np.isnan(got), want)
    assert want.sum() == len(rows) * len(cols)
    assert np.array_equal(got[~want], plain[~want])


def test_combine_missing_values_are_left_out(orc):
    """NaN values are missing: the clip runs over the other values of the pixel.  Pinned
    against numpy's nanmean where no clip can reject (n <= 10, A10), against
    scipy.stats.sigmaclip of the remaining values, and all-missing pixels give NaN."""
    rng = np.random.default_rng(83)
    N, h, w = 24, 6, 50
    vals = rng.normal(1000, 10, size=(N, h, w))
    hits = rng.random(size=vals.shape) < 0.05
    vals[hits] += rng.uniform(500, 5e4, size=hits.sum())
    miss = rng.random(size=vals.shape) < 0.3
    miss[:, 0, 0] = True                      # a pixel without any value
    miss[:, 0, 1] = True
    miss[:7, 0, 1] = False                    # a pixel with 7 values: a plain mean
    vals[miss] = np.nan
    out, keep, nrej, _ = orc.combine(vals, max_iters=1000, missing=True)
    assert np.isnan(out[0, 0]) and not keep[:, 0, 0].any()
    assert out[0, 1] == pytest.approx(np.nanmean(vals[:, 0, 1]), rel=1e-15)
    assert not keep[miss].any()
    total = 0
    for y in range(h):
        for x in range(w):
            if (y, x) in ((0, 0), (0, 1)):
                continue
            col = vals[:, y, x]
            c, _, _ = scipy.stats.sigmaclip(col[~np.isnan(col)], 3, 3)
            assert keep[:, y, x].sum() == c.size
            assert out[y, x] == pytest.approx(c.mean(), rel=1e-13)
            total += int((~np.isnan(col)).sum()) - c.size
    assert nrej == total > 0
    # without the missing rule a NaN poisons its pixel, as IEEE arithmetic does
    out2, _, _, _ = orc.combine(vals[:, :2, :3], missing=False)
    assert np.isnan(out2).all()
