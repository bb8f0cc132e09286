"""Stage-isolated parity of the HIP path against the FP64 oracle.

Each oracle stage receives exactly the GPU's inputs to that stage (float32 promoted
to float64), so the comparison isolates the stage's own arithmetic.  Bars: integer
offsets and keep masks bit-exact (masks except values within 1e-6 of the clip
threshold, which are counted), sub-pixel offsets within 2 float ulp, pixel values
within 2e-6 relative (1 ADU floor).
"""
import os

import numpy as np
import pytest

import synth
from helpers import TOL, err_summary, rel_err, to_dev, ulp32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2008_11486_amd as rd
    rd.lib()
    return rd


def _stack_dev(st):
    return to_dev(st.raw), to_dev(st.dark), to_dev(st.flat)


# ----------------------------------------------------------------------------- calibrate
@pytest.mark.parametrize("shape", [(5, 512, 512), (3, 37, 53), (2, 64, 24), (1, 1, 1), (4, 9, 8)])
def test_calibrate_parity(rd, orc, shape):
    N, H, W = shape
    rng = np.random.default_rng(sum(shape))
    raw = rng.integers(0, 65536, size=shape, dtype=np.uint16)
    dark = (100 + rng.normal(0, 3, size=(H, W))).astype(np.float32)
    flat = rng.uniform(0.95, 1.05, size=(H, W)).astype(np.float32)
    cal = rd.calibrate(to_dev(raw), to_dev(dark), to_dev(flat)).cpu().numpy()
    ref = orc.calibrate(raw, dark, flat)
    e = rel_err(cal, ref)
    print(f"calibrate {shape}: {err_summary(e)}")
    assert e.max() <= TOL


def test_calibrate_identity_and_pitched_roi(rd, orc):
    rng = np.random.default_rng(5)
    full = rng.integers(0, 65536, size=(3, 40, 72), dtype=np.uint16)
    zero = np.zeros((40, 72), np.float32)
    one = np.ones((40, 72), np.float32)
    cal = rd.calibrate(to_dev(full), to_dev(zero), to_dev(one)).cpu().numpy()
    assert np.array_equal(cal, full.astype(np.float32))
    # overscan-style region of interest through the row and frame pitches (vector path)
    dev = to_dev(full)
    roi = dev[:, 4:36, 8:64]
    dark = (100 + rng.normal(0, 3, size=(40, 72))).astype(np.float32)
    flat = rng.uniform(0.95, 1.05, size=(40, 72)).astype(np.float32)
    d, f = to_dev(dark)[4:36, 8:64], to_dev(flat)[4:36, 8:64]
    got = rd.calibrate(roi, d, f).cpu().numpy()
    ref = orc.calibrate(full[:, 4:36, 8:64], dark[4:36, 8:64], flat[4:36, 8:64])
    assert rel_err(got, ref).max() <= TOL
    # unaligned region (scalar path)
    got2 = rd.calibrate(dev[:, 3:30, 5:60], to_dev(dark)[3:30, 5:60], to_dev(flat)[3:30, 5:60]).cpu().numpy()
    ref2 = orc.calibrate(full[:, 3:30, 5:60], dark[3:30, 5:60], flat[3:30, 5:60])
    assert rel_err(got2, ref2).max() <= TOL


@pytest.mark.parametrize("shape", [(4, 96, 128), (3, 37, 53)])
def test_calibrate_with_bias_parity(rd, orc, shape):
    """Bias, then dark, then flat (Section 2.1), on the vector and the scalar paths."""
    N, H, W = shape
    rng = np.random.default_rng(W + 7)
    raw = rng.integers(0, 65536, size=shape, dtype=np.uint16)
    bias = (300 + rng.normal(0, 2, size=(H, W))).astype(np.float32)
    dark = (20 + rng.normal(0, 3, size=(H, W))).astype(np.float32)
    flat = rng.uniform(0.95, 1.05, size=(H, W)).astype(np.float32)
    cal = rd.calibrate(to_dev(raw), to_dev(dark), to_dev(flat), bias=to_dev(bias)).cpu().numpy()
    e = rel_err(cal, orc.calibrate(raw, dark, flat, bias=bias))
    print(f"calibrate+bias {shape}: {err_summary(e)}")
    assert e.max() <= TOL
    # an overscan cut (50 columns and a 2-pixel border, as Section 2.1) through the pitches
    full = rng.integers(0, 65536, size=(2, H + 4, W + 54), dtype=np.uint16)
    roi = to_dev(full)[:, 2:H + 2, 2:W + 2]
    got = rd.calibrate(roi, to_dev(dark), to_dev(flat), bias=to_dev(bias)).cpu().numpy()
    assert rel_err(got, orc.calibrate(full[:, 2:H + 2, 2:W + 2], dark, flat, bias=bias)).max() <= TOL


# ----------------------------------------------------------------------------- register
def _check_offsets(g, o, label):
    tie = (o["flags"] & 4) != 0
    same = (g["dx"] == o["dx"]) & (g["dy"] == o["dy"])
    assert np.all(same | tie), f"{label}: integer offsets differ: gpu {g[['dx','dy']]} oracle {o[['dx','dy']]}"
    for ax in ("sx", "sy"):
        d = np.abs(g[ax].astype(np.float64) - o[ax].astype(np.float64))
        assert np.all((d <= 2 * ulp32(o[ax])) | tie), f"{label}: {ax} gpu {g[ax]} oracle {o[ax]}"
    np.testing.assert_allclose(g["peak"], o["peak"], rtol=1e-10)
    fin = np.isfinite(o["second"])
    np.testing.assert_allclose(g["second"][fin], o["second"][fin], rtol=1e-10)
    assert np.array_equal(g["flags"] & ~4, o["flags"] & ~4), f"{label}: flags {g['flags']} vs {o['flags']}"
    return int(tie.sum())


@pytest.mark.parametrize("R,shape", [(0, (3, 40, 48)), (1, (3, 33, 41)), (2, (4, 64, 64)),
                                     # small windows over several 256-column tiles, 240-row
                                     # strips and 15-row chunks, with ragged last ones
                                     (2, (2, 530, 600)), (1, (2, 497, 700)), (0, (2, 260, 513)),
                                     (3, (2, 45, 70)),
                                     (5, (3, 96, 80)), (8, (3, 120, 100)), (12, (2, 90, 150)),
                                     (17, (2, 130, 140)), (21, (2, 150, 128))])
def test_register_parity_random_shapes(rd, orc, R, shape):
    N, H, W = shape
    spec = synth.small_spec(N, W, H, n_stars=max(6, W * H // 800), shift_bound=max(R - 1, 0.4), radius=R,
                            seed=(R, N))
    st = synth.make_stack(spec)
    raw, dark, flat = _stack_dev(st)
    cal = rd.calibrate(raw, dark, flat)
    out, S = rd.register(cal[0].contiguous(), cal, R, want_scores=True)
    g = rd.offsets_to_numpy(out)
    cal64 = cal.cpu().numpy().astype(np.float64)
    o, So = orc.register(cal64[0], cal64, R, want_scores=True)
    S = S.cpu().numpy()
    fin = np.isfinite(So)
    assert np.array_equal(np.isfinite(S), fin)
    np.testing.assert_allclose(S[fin], So[fin], rtol=1e-11, atol=1e-11 * np.abs(So[fin]).max())
    _check_offsets(g, o, f"R={R} {shape}")


def test_register_template_and_centres(rd, orc):
    spec = synth.small_spec(4, 160, 140, n_stars=40, shift_bound=9.0, radius=10, seed=(77,))
    st = synth.make_stack(spec)
    cal = rd.calibrate(*_stack_dev(st))
    cal64 = cal.cpu().numpy().astype(np.float64)
    tmpl = (14, 12, 120, 100)
    g = rd.offsets_to_numpy(rd.register(cal[0].contiguous(), cal, 10, 12, tmpl=tmpl))
    o = orc.register(cal64[0], cal64, 10, 12, tmpl=tmpl)
    _check_offsets(g, o, "template")
    # +-2 windows around given centres, some clipped at +-Rmax
    centers = np.array([[0, 0], [int(o["dx"][1]), int(o["dy"][1])], [12, -11], [-3, 12]], dtype=np.int32)
    cd = to_dev(centers)
    g2, S2 = rd.register(cal[0].contiguous(), cal, 2, 12, centers=cd, tmpl=tmpl, want_scores=True)
    o2, So2 = orc.register(cal64[0], cal64, 2, 12, centers=centers, tmpl=tmpl, want_scores=True)
    _check_offsets(rd.offsets_to_numpy(g2), o2, "centres")
    S2 = S2.cpu().numpy()
    assert np.array_equal(np.isfinite(S2), np.isfinite(So2))
    fin = np.isfinite(So2)
    np.testing.assert_allclose(S2[fin], So2[fin], rtol=1e-11)


def test_register_workload0_integer_shifts(rd, orc):
    st = synth.make_config(0)[0]
    cal = rd.calibrate(*_stack_dev(st))
    g = rd.offsets_to_numpy(rd.register(cal[0].contiguous(), cal, st.spec.radius))
    assert np.array_equal(np.stack([g["dx"], g["dy"]], 1), st.shifts.astype(np.int64))
    cal64 = cal.cpu().numpy().astype(np.float64)
    o = orc.register(cal64[0], cal64, st.spec.radius)
    assert _check_offsets(g, o, "workload 0") == 0


def test_register_errors(rd):
    cal = torch.zeros((2, 32, 32), dtype=torch.float32, device="cuda:0")
    with pytest.raises(rd.ReduceError) as e:
        rd.register(cal[0].contiguous(), cal, 2, 16)
    assert e.value.status == rd.ERR_RANGE
    with pytest.raises(rd.ReduceError) as e:
        rd.register(cal[0].contiguous(), cal, 2, 4, tmpl=(1, 4, 10, 10))
    assert e.value.status == rd.ERR_RANGE
    with pytest.raises(rd.ReduceError) as e:
        rd.register(cal[0].contiguous(), cal, 2, ws=torch.empty(8, dtype=torch.uint8, device="cuda:0"))
    assert e.value.status == rd.ERR_WORKSPACE


# ----------------------------------------------------------------------------- shift
@pytest.mark.parametrize("W,H,N", [(64, 48, 4), (37, 29, 3), (128, 128, 6)])
def test_shift_parity(rd, orc, W, H, N):
    rng = np.random.default_rng(W * H + N)
    frames = rng.normal(1000, 300, size=(N, H, W)).astype(np.float32)
    frames[:, ::7, ::5] += rng.uniform(2e3, 5e4, size=frames[:, ::7, ::5].shape).astype(np.float32)
    offs = np.zeros((N, 2), np.float32)
    offs[1:] = rng.uniform(-6, 6, size=(N - 1, 2))
    offs[-1] = (-0.25 - 2 ** -20, 3.0)  # a negative fraction close to an integer, an exact integer
    rect = orc.valid_rect(offs, W, H)
    assert np.array_equal(rd.valid_rect(offs, W, H), rect)
    got = rd.shift(to_dev(frames), to_dev(offs), rect).cpu().numpy()
    ref = orc.shift(frames.astype(np.float64), offs, rect)
    e = rel_err(got, ref)
    print(f"shift {W}x{H}x{N}: {err_summary(e)}")
    assert e.max() <= TOL


def test_shift_integer_mode_is_exact_copy(rd, orc):
    rng = np.random.default_rng(9)
    frames = rng.normal(1000, 30, size=(3, 50, 61)).astype(np.float32)
    offs = np.array([[0, 0], [4, -3], [-5, 2]], np.float32)
    rect = orc.valid_rect(offs, 61, 50)
    for mode in (True, False):
        got = rd.shift(to_dev(frames), to_dev(offs), rect, integer_mode=mode).cpu().numpy()
        x0, y0, w, h = rect
        for k in range(3):
            sx, sy = int(offs[k, 0]), int(offs[k, 1])
            assert np.array_equal(got[k], frames[k, y0 + sy:y0 + sy + h, x0 + sx:x0 + sx + w])


@pytest.mark.parametrize("integer_mode", [False, True])
def test_mask_shifted_marks_exactly_the_oracle_outputs(rd, orc, integer_mode):
    """Bad pixels (0.3% of a 97x131 map) reach exactly the outputs whose taps read them;
    every other value equals the unmasked shift."""
    rng = np.random.default_rng(91 + integer_mode)
    N, H, W = 5, 97, 131
    frames = rng.normal(1000, 30, size=(N, H, W)).astype(np.float32)
    mask = (rng.random(size=(H, W)) < 0.003).astype(np.uint8)
    s = rng.uniform(-6, 6, size=(N, 2)).astype(np.float32)
    s[0] = 0.0
    s[1] = (2.0, -3.0)        # an integer offset: one tap
    s[2] = (0.5, 0.0)         # a fraction on one axis only
    if integer_mode:
        s = np.round(s).astype(np.float32)
    rect = rd.valid_rect(s, W, H)
    dev = to_dev(frames)
    offs = to_dev(s)
    al = rd.shift(dev, offs, rect, integer_mode=integer_mode)
    rd.mask_shifted(to_dev(mask), al, offs, rect, W, H, integer_mode=integer_mode)
    got = al.cpu().numpy()
    want = orc.shift(frames.astype(np.float64), s, rect, mask)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want)
    assert rel_err(got[ok], want[ok]).max() <= TOL
    assert np.isnan(want).sum() > 20


@pytest.mark.parametrize("N", [5, 16, 40, 97])
def test_combine_missing_values_parity(rd, orc, N):
    rng = np.random.default_rng(4000 + N)
    h, w = 19, 157
    vals = rng.normal(1000, 30, size=(N, h, w)).astype(np.float32)
    hits = rng.random(size=vals.shape) < 0.02
    vals[hits] += rng.uniform(5e3, 6e4, size=hits.sum()).astype(np.float32)
    vals[rng.random(size=vals.shape) < 0.2] = np.nan
    vals[:, 0, :3] = np.nan                       # pixels without any value
    out, keep, nrej = rd.combine(to_dev(vals), want_keep=True, want_nrej=True, missing=True)
    out, keep, nrej = out.cpu().numpy(), keep.cpu().numpy(), int(nrej.cpu().numpy()[0])
    o_out, o_keep, o_nrej, near = orc.combine(vals.astype(np.float64), 3.0, 3, missing=True)
    assert np.array_equal(np.isnan(out), np.isnan(o_out)) and np.isnan(out[0, :3]).all()
    flips = keep != o_keep
    assert np.all(~flips | (near == 1))
    good = ~flips.any(axis=0) & ~np.isnan(o_out)
    e = rel_err(out[good], o_out[good])
    print(f"combine missing N={N}: rejected {o_nrej}, flips {int(flips.sum())}, {err_summary(e)}")
    assert e.max() <= TOL
    if not flips.any():
        assert nrej == o_nrej
    assert not keep[np.isnan(vals)].any()


# ----------------------------------------------------------------------------- combine
def _combine_check(rd, orc, vals, ksigma=3.0, iters=3, lanes=None):
    if lanes:
        os.environ["REDUCE_COMBINE_LANES"] = str(lanes)
    try:
        out, keep, nrej = rd.combine(to_dev(vals), ksigma, iters, want_keep=True, want_nrej=True)
    finally:
        os.environ.pop("REDUCE_COMBINE_LANES", None)
    out, keep, nrej = out.cpu().numpy(), keep.cpu().numpy(), int(nrej.cpu().numpy()[0])
    o_out, o_keep, o_nrej, near = orc.combine(vals.astype(np.float64), float(np.float32(ksigma)), iters)
    flips = (keep != o_keep)
    assert np.all(~flips | (near == 1)), "keep mask differs away from the threshold"
    bad_px = flips.any(axis=0)
    e = rel_err(out, o_out)[~bad_px]
    assert e.max() <= TOL, err_summary(e)
    if not flips.any():
        assert nrej == o_nrej
    return int(flips.sum()), o_nrej, e


@pytest.mark.parametrize("N", [1, 2, 5, 10, 11, 16, 30, 48])
@pytest.mark.parametrize("lanes", [1, 4, 16])
def test_combine_parity_with_outliers(rd, orc, N, lanes):
    rng = np.random.default_rng(N * 100 + lanes)
    h, w = 37, 301
    vals = rng.normal(1000, 30, size=(N, h, w)).astype(np.float32)
    hits = rng.random(size=vals.shape) < 0.02
    vals[hits] += rng.uniform(5e3, 6e4, size=hits.sum()).astype(np.float32)
    flips, nrej, e = _combine_check(rd, orc, vals, lanes=lanes)
    print(f"combine N={N} L={lanes}: rejected {nrej}, mask flips {flips}, {err_summary(e)}")
    if N <= 10:
        assert nrej == 0


@pytest.mark.parametrize("shape", [(16, 10, 64), (16, 10, 61), (16, 9, 63), (5, 11, 62), (12, 7, 66)])
@pytest.mark.parametrize("missing", [False, True])
def test_combine_pixel_groups_every_plane_alignment(rd, orc, shape, missing):
    """Planes of length 0, 1, 2, 3 mod 4: four pixels per thread with 16- or 8-byte loads
    per frame, two, or one, and the ragged last group."""
    N, h, w = shape
    rng = np.random.default_rng(h * w + N)
    vals = rng.normal(1000, 30, size=shape).astype(np.float32)
    vals[rng.random(size=shape) < 0.03] += 2e4
    if missing:
        vals[rng.random(size=shape) < 0.1] = np.nan
    out, keep, nrej = rd.combine(to_dev(vals), want_keep=True, want_nrej=True, missing=missing)
    out, keep = out.cpu().numpy(), keep.cpu().numpy()
    o_out, o_keep, o_nrej, near = orc.combine(vals.astype(np.float64), 3.0, 3, missing=missing)
    flips = keep != o_keep
    assert np.all(~flips | (near == 1))
    good = ~flips.any(axis=0) & ~np.isnan(o_out)
    assert np.array_equal(np.isnan(out), np.isnan(o_out))
    assert rel_err(out[good], o_out[good]).max() <= TOL


@pytest.mark.parametrize("N", [49, 64, 65, 97, 128])
def test_combine_parity_deep_stacks(rd, orc, N):
    """Stacks past the LDS tile's depth (the paper's sets reach 97 frames): the one-lane
    path with the column in LDS, across a ragged last block of 64 pixels."""
    rng = np.random.default_rng(7000 + N)
    h, w = 23, 171
    vals = rng.normal(1000, 30, size=(N, h, w)).astype(np.float32)
    hits = rng.random(size=vals.shape) < 0.02
    vals[hits] += rng.uniform(5e3, 6e4, size=hits.sum()).astype(np.float32)
    flips, nrej, e = _combine_check(rd, orc, vals)
    print(f"combine N={N}: rejected {nrej}, mask flips {flips}, {err_summary(e)}")
    assert nrej > 0
    for iters in (0, 1, 2, 5):
        _combine_check(rd, orc, vals[:, :4, :70].copy(), iters=iters)
    one = np.full((N, 1, 5), 1234.5, np.float32)
    one[N - 1, 0, 2] = 1.0e5  # the last frame's value sits in the second kept word
    out, keep, nr = rd.combine(to_dev(one), want_keep=True, want_nrej=True)
    assert np.array_equal(out.cpu().numpy(), np.full((1, 5), 1234.5, np.float32))
    assert int(nr.cpu()[0]) == 1 and keep.cpu().numpy()[N - 1, 0, 2] == 0 and keep.cpu().numpy().sum() == 5 * N - 1


def test_combine_closed_forms(rd, orc):
    col = np.full((16, 1, 3), 1234.5, np.float32)
    col[7, 0, 1] = 1.0e5
    out, keep, nrej = rd.combine(to_dev(col), want_keep=True, want_nrej=True)
    assert np.array_equal(out.cpu().numpy(), np.full((1, 3), 1234.5, np.float32))
    assert int(nrej.cpu()[0]) == 1 and keep.cpu().numpy()[7, 0, 1] == 0
    thr = np.array([0.0] * 9 + [10.0], np.float32).reshape(10, 1, 1)
    out, keep, _ = rd.combine(to_dev(thr), want_keep=True)
    assert out.cpu().numpy()[0, 0] == 1.0 and keep.cpu().numpy().all()
    for iters in (0, 1, 2, 5):
        v = np.array([0.0] * 30 + [1e6, 1e4, 1e2, 12.0], np.float32).reshape(-1, 1, 1)
        _combine_check(rd, orc, v, iters=iters)


# ----------------------------------------------------------------------------- autotuner
def test_tuned_shapes_keep_results(rd, orc, tmp_path):
    spec = synth.small_spec(3, 200, 180, n_stars=40, shift_bound=7.0, radius=8, seed=(5,))
    st = synth.make_stack(spec)
    cal = rd.calibrate(*_stack_dev(st))
    ref = cal[0].contiguous()
    rd.tune_clear()
    base = rd.offsets_to_numpy(rd.register(ref, cal, 8))
    plan = rd.tune_register(ref, cal, 8, reps=1)
    assert rd.register_plan(200, 180, 3, 8) == plan
    tuned = rd.offsets_to_numpy(rd.register(ref, cal, 8))
    assert np.array_equal(base[["dx", "dy"]], tuned[["dx", "dy"]])
    cal64 = cal.cpu().numpy().astype(np.float64)
    _check_offsets(tuned, orc.register(cal64[0], cal64, 8), "tuned")
    path = str(tmp_path / "tuned.json")
    rd.tune_save(path)
    rd.tune_clear()
    rd.tune_load(path)
    assert rd.register_plan(200, 180, 3, 8) == plan
    lanes = rd.tune_combine(cal[:, :64, :64].contiguous(), reps=1)
    assert lanes in (1, 2, 4, 8, 16)
    rd.tune_clear()


def test_tuner_finds_shapes_for_wide_windows(rd):
    """The +-65 px search of 6144x6160 frames: the cost model's own tiles are taller than
    the cap on the tuner's tile-height variants, and the tuner must still find a shape
    (a cap on every candidate once left none)."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(4)
    fr = 1000.0 + 30.0 * torch.randn((3, 6160, 6144), generator=g, device=dev)
    rd.tune_clear()
    plan = rd.tune_register(fr[0].contiguous(), fr[1:].contiguous(), 65, reps=1)
    print("tuned plan for 6144x6160, R = 65:", plan)
    assert plan == rd.register_plan(6144, 6160, 2, 65)
    rd.tune_clear()
    for W, H, R in ((2048, 2048, 17), (4096, 4096, 17)):
        # the chunk-count variants stay within the cap: radius 17 tiles of at most 150 rows
        fr = 1000.0 + 30.0 * torch.randn((3, H, W), generator=g, device=dev)
        plan = rd.tune_register(fr[0].contiguous(), fr[1:].contiguous(), R, reps=1)
        print(f"tuned plan for {W}x{H}, R = {R}:", plan)
        assert plan["BR"] <= 150 or plan["BR"] == plan["TY"]
        rd.tune_clear()


@pytest.mark.parametrize("N", [12, 16, 30, 45])
@pytest.mark.parametrize("missing", [False, True])
def test_combine_every_column_drops(rd, orc, N, missing):
    """Every column holds an outlier, so every column leaves the first iteration for the
    workgroup's queue: more queued columns than the queue keeps in LDS (the rest are
    loaded again), on planes with a ragged last workgroup."""
    rng = np.random.default_rng(9100 + N)
    h, w = 13, 389
    vals = rng.normal(1000, 30, size=(N, h, w)).astype(np.float32)
    k = rng.integers(0, N, size=(h, w))
    np.put_along_axis(vals, k[None], 1.0e5, axis=0)
    if missing:
        vals[rng.random(size=vals.shape) < 0.1] = np.nan
    out, keep, nrej = rd.combine(to_dev(vals), want_keep=True, want_nrej=True, missing=missing)
    out, keep, nrej = out.cpu().numpy(), keep.cpu().numpy(), int(nrej.cpu().numpy()[0])
    o_out, o_keep, o_nrej, near = orc.combine(vals.astype(np.float64), 3.0, 3, missing=missing)
    flips = keep != o_keep
    assert np.all(~flips | (near == 1))
    good = ~flips.any(axis=0) & ~np.isnan(o_out)
    assert np.array_equal(np.isnan(out), np.isnan(o_out))
    e = rel_err(out[good], o_out[good])
    print(f"combine every column drops, N={N}, missing={missing}: rejected {o_nrej}, {err_summary(e)}")
    assert e.max() <= TOL
    if not flips.any():
        assert nrej == o_nrej
