"""The end-to-end offset tolerance of the GPU parity tests, checked on the CPU with the
oracle alone: searching single-precision calibrated frames (computed the way the GPU does,
one correctly rounded float operation per step) instead of the oracle's FP64 calibration
moves each parabola offset by no more than offset_bound (+ 2 float ulps), and the bound is
tight enough to catch a real error (well under 1e-4 px on these stacks)."""
import numpy as np
import pytest

import synth
from helpers import offset_bound, ulp32


@pytest.mark.parametrize("seed,with_bias", [(0, False), (1, True), (2, True)])
def test_offset_bound_covers_single_precision_calibration(orc, seed, with_bias):
    spec = synth.small_spec(9, 160, 128, n_stars=30, shift_bound=5.0, seed=(77, seed))
    st = synth.make_stack(spec)
    rng = np.random.default_rng(seed)
    bias = (250 + rng.normal(0, 2, size=(spec.H, spec.W))).astype(np.float32) if with_bias else None
    raw = st.raw.astype(np.int64) + (0 if bias is None else np.round(bias).astype(np.int64))
    raw = np.clip(raw, 0, 65535).astype(np.uint16)
    cal_a = orc.calibrate(raw, st.dark, st.flat, bias)
    # float32 chain: cast, (bias,) dark, flat, each step rounded once
    v = raw.astype(np.float32)
    if bias is not None:
        v = v - bias
    cal_b = ((v - st.dark) / st.flat).astype(np.float32)
    assert not np.array_equal(cal_b.astype(np.float64), cal_a)
    R = spec.radius
    oa = orc.register(cal_a[0], cal_a, R)
    ob, sb = orc.register(cal_b[0].astype(np.float64), cal_b.astype(np.float64), R, want_scores=True)
    assert np.array_equal(oa["dx"], ob["dx"]) and np.array_equal(oa["dy"], ob["dy"])
    bound = offset_bound(cal_a, cal_b, 0, R, ob, sb)
    s_a = np.stack([oa["sx"], oa["sy"]], 1).astype(np.float64)
    s_b = np.stack([ob["sx"], ob["sy"]], 1).astype(np.float64)
    d = np.abs(s_a - s_b)
    assert np.all(d <= bound + 2 * ulp32(s_a)), (d, bound)
    assert np.all(bound[1:] < 1e-4), bound
    print(f"largest offset change {d.max():.3g} px, largest bound {bound[1:].max():.3g} px")
