"""The batched path (one launch per phase over all stacks) against the stage-wise chain
(bit-identical) and the oracle."""
import numpy as np
import pytest

import synth
from helpers import assert_end_to_end, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2008_11486_amd as rd
    rd.lib()
    return rd


def stagewise(rd, raw, dark, flat, R, ref=0, integer_mode=False, bias=None, mask=None):
    """The same chain through the stage-wise entry points."""
    N, H, W = raw.shape
    cal = rd.calibrate(raw, dark, flat, bias=bias)
    offs = np.zeros(N, dtype=rd.OFFSET_DTYPE)
    offs["second"] = -np.inf
    offs["margin"] = np.inf
    s = np.zeros((N, 2), np.float32)
    if N > 1:
        others = [k for k in range(N) if k != ref]
        frames = torch.stack([cal[k] for k in others]).contiguous()
        o = rd.offsets_to_numpy(rd.register(cal[ref].contiguous(), frames, R))
        for i, k in enumerate(others):
            offs[k] = o[i]
            s[k] = (o["dx"][i], o["dy"][i]) if integer_mode else (o["sx"][i], o["sy"][i])
    rect = rd.valid_rect(s, W, H)
    al = rd.shift(cal, to_dev(s), rect, integer_mode=integer_mode)
    if mask is not None:
        rd.mask_shifted(mask, al, to_dev(s), rect, W, H, integer_mode=integer_mode)
    out, _, nrej = rd.combine(al, want_nrej=True, missing=mask is not None)
    return out.cpu().numpy(), rect, offs, int(nrej.cpu()[0])


SPECS = [  # (N, W, H, radius, ref, integer_mode, cosmic)
    (5, 128, 96, 4, 0, False, False),
    (11, 160, 160, 6, 3, False, True),
    (3, 96, 128, 3, 0, True, False),
    (16, 200, 152, 5, 7, False, True),
    (1, 64, 64, 2, 0, False, False),
    (2, 72, 40, 0, 1, False, False),
]


def _make(i, N, W, H, R, cosmic, seed=0):
    spec = synth.small_spec(N, W, H, n_stars=max(8, W * H // 1000), shift_bound=max(R - 1, 0.3), radius=R,
                            cosmic=cosmic, seed=(i, seed))
    if R == 0:
        spec = synth.small_spec(N, W, H, n_stars=8, shift_kind="zero", radius=0, seed=(i, seed))
    return synth.make_stack(spec)


def test_batch_bit_identical_to_stagewise(rd, orc):
    stacks = [_make(i, N, W, H, R, cos) for i, (N, W, H, R, _, _, cos) in enumerate(SPECS)]
    dev = [(to_dev(st.raw), to_dev(st.dark), to_dev(st.flat), sp[3]) for st, sp in zip(stacks, SPECS)]
    batch = rd.StackBatch(dev, ref_index=[sp[4] for sp in SPECS], integer_mode=[sp[5] for sp in SPECS])
    batch.run()
    for i, ((raw, dark, flat, R), sp) in enumerate(zip(dev, SPECS)):
        img, rect, offs, nrej = batch.result(i)
        ref_img, ref_rect, ref_offs, ref_nrej = stagewise(rd, raw, dark, flat, R, sp[4], sp[5])
        assert np.array_equal(rect, ref_rect), (i, rect, ref_rect)
        assert np.array_equal(img.cpu().numpy(), ref_img), f"stack {i}: image differs"
        assert offs.tobytes() == ref_offs.tobytes(), f"stack {i}: offsets differ\n{offs}\n{ref_offs}"
        assert nrej == ref_nrej
    # the stacks with cosmic rays really exercised the clip
    assert batch.result(1)[3] > 0 and batch.result(3)[3] > 0


def test_batch_reruns_follow_new_data(rd):
    specs = SPECS[:4]
    A = [_make(i, N, W, H, R, cos, seed=1) for i, (N, W, H, R, _, _, cos) in enumerate(specs)]
    B = [_make(i, N, W, H, R, cos, seed=2) for i, (N, W, H, R, _, _, cos) in enumerate(specs)]
    dev = [(to_dev(st.raw), to_dev(st.dark), to_dev(st.flat), sp[3]) for st, sp in zip(A, specs)]
    batch = rd.StackBatch(dev, ref_index=[sp[4] for sp in specs], integer_mode=[sp[5] for sp in specs])
    for rep, src in enumerate([A, B, A, B]):
        for (raw, dark, flat, _), st in zip(dev, src):  # new inputs in place between runs
            raw.copy_(to_dev(st.raw))
            dark.copy_(to_dev(st.dark))
            flat.copy_(to_dev(st.flat))
        torch.cuda.synchronize()
        batch.run()
        for i, ((raw, dark, flat, R), sp) in enumerate(zip(dev, specs)):
            img, rect, offs, nrej = batch.result(i)
            ref_img, ref_rect, ref_offs, ref_nrej = stagewise(rd, raw, dark, flat, R, sp[4], sp[5])
            assert np.array_equal(rect, ref_rect) and np.array_equal(img.cpu().numpy(), ref_img), (rep, i)
            assert offs.tobytes() == ref_offs.tobytes() and nrej == ref_nrej, (rep, i)


def test_batch_matches_oracle_end_to_end(rd, orc):
    st = _make(9, 16, 180, 140, 6, True, seed=3)
    batch = rd.StackBatch([(to_dev(st.raw), to_dev(st.dark), to_dev(st.flat), 6)])
    batch.run()
    img, rect, offs, nrej = batch.result(0)
    o = orc.reduce_stack(st.raw, st.dark, st.flat, 6)
    assert np.array_equal(offs["dx"][1:], o["offsets"]["dx"][1:]) and np.array_equal(offs["dy"][1:], o["offsets"]["dy"][1:])
    assert np.array_equal(rect, o["rect"])
    s = np.stack([offs["sx"], offs["sy"]], 1).astype(np.float32)
    cal_gpu = rd.calibrate(to_dev(st.raw), to_dev(st.dark), to_dev(st.flat)).cpu().numpy()
    assert_end_to_end(orc, o["cal"], cal_gpu, offs, s, o["s"], rect, img.cpu().numpy(), 6, "batch vs oracle")


def test_batch_workload1_three_bands(rd):
    stacks = synth.make_config(1)
    dev = [(to_dev(st.raw), to_dev(st.dark), to_dev(st.flat), st.spec.radius) for st in stacks]
    batch = rd.StackBatch(dev)
    batch.run()
    for i, (raw, dark, flat, R) in enumerate(dev):
        img, rect, offs, nrej = batch.result(i)
        ref_img, ref_rect, ref_offs, _ = stagewise(rd, raw, dark, flat, R)
        assert np.array_equal(rect, ref_rect) and np.array_equal(img.cpu().numpy(), ref_img)
        assert offs.tobytes() == ref_offs.tobytes()
        err = np.abs(np.stack([offs["sx"], offs["sy"]], 1) - stacks[i].shifts)[1:]
        assert err.max() < 0.1


def test_batch_deep_stacks(rd, orc):
    """Stacks of 60 and 97 frames (the paper's co-adding sets reach 97) beside a short
    one in one call: bit-identical to the stage-wise chain, and the 97-frame stack
    against the oracle end to end."""
    specs = [(97, 96, 80, 3, True), (60, 112, 72, 4, True), (10, 64, 64, 2, False)]
    stacks = [_make(20 + i, N, W, H, R, cos, seed=4) for i, (N, W, H, R, cos) in enumerate(specs)]
    dev = [(to_dev(st.raw), to_dev(st.dark), to_dev(st.flat), sp[3]) for st, sp in zip(stacks, specs)]
    batch = rd.StackBatch(dev)
    batch.run()
    for i, (raw, dark, flat, R) in enumerate(dev):
        img, rect, offs, nrej = batch.result(i)
        ref_img, ref_rect, ref_offs, ref_nrej = stagewise(rd, raw, dark, flat, R)
        assert np.array_equal(rect, ref_rect) and np.array_equal(img.cpu().numpy(), ref_img), i
        assert offs.tobytes() == ref_offs.tobytes() and nrej == ref_nrej, i
    assert batch.result(0)[3] > 0 and batch.result(1)[3] > 0
    img, rect, offs, _ = batch.result(0)
    st = stacks[0]
    o = orc.reduce_stack(st.raw, st.dark, st.flat, specs[0][3])
    assert np.array_equal(offs["dx"][1:], o["offsets"]["dx"][1:]) and np.array_equal(offs["dy"][1:], o["offsets"]["dy"][1:])
    s = np.stack([offs["sx"], offs["sy"]], 1).astype(np.float32)
    assert np.array_equal(rect, o["rect"])
    cal_gpu = rd.calibrate(dev[0][0], dev[0][1], dev[0][2]).cpu().numpy()
    assert_end_to_end(orc, o["cal"], cal_gpu, offs, s, o["s"], rect, img.cpu().numpy(), specs[0][3],
                      "97-frame batch vs oracle")


def test_batch_bias_and_bad_pixels(rd, orc):
    """Stacks with a bias frame and a bad-pixel map beside plain ones: bit-identical to
    the stage-wise chain (bias calibrate, shift, masking, missing-value combine), and
    against the oracle end to end."""
    rng = np.random.default_rng(95)
    specs = [(12, 120, 100, 4, True), (6, 96, 80, 3, False), (60, 64, 72, 3, True), (9, 80, 64, 3, False)]
    dev, stacks, extras = [], [], []
    for i, (N, W, H, R, cos) in enumerate(specs):
        st = _make(30 + i, N, W, H, R, cos, seed=5)
        bias = (250 + rng.normal(0, 2, size=(H, W))).astype(np.float32) if i != 3 else None
        raw = st.raw.astype(np.int64) + (0 if bias is None else np.round(bias).astype(np.int64))
        raw = np.clip(raw, 0, 65535).astype(np.uint16)
        mask = (rng.random(size=(H, W)) < 0.004).astype(np.uint8) if i in (0, 2, 3) else None
        stacks.append((raw, st.dark, st.flat, R, bias, mask))
        extras.append(i % 2 == 1)
        dev.append((to_dev(raw), to_dev(st.dark), to_dev(st.flat), R, None if bias is None else to_dev(bias),
                    None if mask is None else to_dev(mask)))
    batch = rd.StackBatch(dev, integer_mode=extras)
    batch.run()
    for i, (raw, dark, flat, R, bias, mask) in enumerate(dev):
        img, rect, offs, nrej = batch.result(i)
        ref_img, ref_rect, ref_offs, ref_nrej = stagewise(rd, raw, dark, flat, R, integer_mode=extras[i], bias=bias,
                                                          mask=mask)
        assert np.array_equal(rect, ref_rect), i
        assert np.array_equal(img.cpu().numpy(), ref_img, equal_nan=True), i
        assert offs.tobytes() == ref_offs.tobytes() and nrej == ref_nrej, i
    for i in (0, 2):
        raw, dark, flat, R, bias, mask = stacks[i]
        img, rect, offs, _ = batch.result(i)
        o = orc.reduce_stack(raw, dark, flat, R, bias=bias, mask=mask, integer_mode=extras[i])
        assert np.array_equal(offs["dx"][1:], o["offsets"]["dx"][1:]) and np.array_equal(offs["dy"][1:], o["offsets"]["dy"][1:])
        s = (np.stack([offs["dx"], offs["dy"]], 1) if extras[i] else np.stack([offs["sx"], offs["sy"]], 1))
        s = s.astype(np.float32)
        assert np.array_equal(rect, o["rect"]), (i, rect, o["rect"])
        cal_gpu = rd.calibrate(dev[i][0], dev[i][1], dev[i][2], bias=dev[i][4]).cpu().numpy()
        assert_end_to_end(orc, o["cal"], cal_gpu, offs, s, o["s"], rect, img.cpu().numpy(), R,
                          f"stack {i} with bias and bad pixels vs oracle", integer_mode=extras[i], mask=mask,
                          missing=True)


def test_batch_rejects_bad_stacks(rd):
    st = _make(4, 5, 128, 96, 4, False, seed=6)
    raw = to_dev(st.raw)
    batch = rd.StackBatch([(raw, to_dev(st.dark), to_dev(st.flat), 60)])  # no template left
    with pytest.raises(rd.ReduceError):
        batch.run()


def test_batch_spectral_search_bit_identical_to_stagewise(rd, orc):
    """Stacks that register through row spectra beside a direct-search stack in one call:
    each bit-identical to the stage-wise chain with reduce_register_fft (offsets of every
    frame but the reference, the overlap, the image, the rejected count), and one of them
    against the oracle end to end."""
    specs = [(8, 200, 171, 6, False), (12, 160, 160, 6, True), (5, 300, 261, 17, False), (6, 128, 96, 4, False)]
    search = ["spectral", "spectral", "spectral", "direct"]
    stacks = [_make(40 + i, N, W, H, R, cos, seed=7) for i, (N, W, H, R, cos) in enumerate(specs)]
    dev = [(to_dev(st.raw), to_dev(st.dark), to_dev(st.flat), sp[3]) for st, sp in zip(stacks, specs)]
    batch = rd.StackBatch(dev, search=search)
    batch.run()
    for i, (raw, dark, flat, R) in enumerate(dev):
        img, rect, offs, nrej = batch.result(i)
        if search[i] == "direct":
            ref_img, ref_rect, ref_offs, ref_nrej = stagewise(rd, raw, dark, flat, R)
            assert np.array_equal(img.cpu().numpy(), ref_img) and offs.tobytes() == ref_offs.tobytes(), i
            continue
        cal = rd.calibrate(raw, dark, flat)
        o = rd.offsets_to_numpy(rd.register_fft(cal[0].contiguous(), cal, R))
        s = np.stack([o["sx"], o["sy"]], 1).astype(np.float32)
        s[0] = 0.0
        r2 = rd.valid_rect(s, cal.shape[2], cal.shape[1])
        al = rd.shift(cal, to_dev(s), r2)
        ref_img, _, ref_nrej = rd.combine(al, want_nrej=True)
        assert np.array_equal(rect, r2), i
        assert offs[1:].tobytes() == o[1:].tobytes(), i
        assert np.array_equal(img.cpu().numpy(), ref_img.cpu().numpy()), i
        assert nrej == int(ref_nrej.cpu()[0]), i
    img, rect, offs, _ = batch.result(1)
    st = stacks[1]
    o = orc.reduce_stack(st.raw, st.dark, st.flat, specs[1][3])
    assert np.array_equal(offs["dx"][1:], o["offsets"]["dx"][1:]) and np.array_equal(offs["dy"][1:], o["offsets"]["dy"][1:])
    assert np.array_equal(rect, o["rect"])
    s = np.stack([offs["sx"], offs["sy"]], 1).astype(np.float32)
    cal_gpu = rd.calibrate(dev[1][0], dev[1][1], dev[1][2]).cpu().numpy()
    assert_end_to_end(orc, o["cal"], cal_gpu, offs, s, o["s"], rect, img.cpu().numpy(), specs[1][3],
                      "spectral batch vs oracle")
