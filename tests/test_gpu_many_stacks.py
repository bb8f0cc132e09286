"""Sampled parity of the many-stack workload (64 stacks of 3-30 frames, sides 512-4096,
sub-pixel shifts within +-16 px, search radius 17) in the launch configuration the
benchmark times: the same GPU-rendered inputs, search shapes tuned per frame size the
same way, all stacks in one batched call.  The oracle checks, on stacks of every size
(the largest stack of each size and the smallest stack): the overlap rectangle, the
integer and sub-pixel offsets of sampled frames (the oracle's 3x3 window around the
GPU's maximum on the same calibrated frames must peak at the same offset with the same
parabola; for one frame of every stack the oracle searches the whole +-17 px window and
must find the same maximum, flags and parabola), and whole rows of the combined image
(the oracle's shift and clipped mean of the GPU's calibrated frames with the GPU's
offsets).
"""
import numpy as np
import pytest

from helpers import TOL, err_summary, rel_err, ulp32

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2008_11486_amd as rd
    rd.lib()
    return rd


@pytest.fixture(scope="module")
def many(rd):
    import bench
    import synth
    specs = synth.config_specs(2)
    store = {}
    stacks, shifts = bench.many_stack_inputs(torch, rd, specs, bench.tuning_hook(store))
    plans = bench.tune_many_stacks(torch, rd, specs, store)
    batch = rd.StackBatch(stacks)
    batch.run()
    torch.cuda.synchronize()
    picks = sorted({max((i for i, sp in enumerate(specs) if sp.W == W), key=lambda i: specs[i].N)
                    for W in {sp.W for sp in specs}} | {min(range(len(specs)), key=lambda i: specs[i].N)})
    results = {i: batch.result(i) for i in picks}
    torch.cuda.synchronize()
    return dict(specs=specs, stacks=stacks, shifts=shifts, plans=plans, batch=batch, picks=picks,
                results=results)


def _calibrated(rd, stack):
    raw, dark, flat, _ = stack
    return rd.calibrate(raw, dark, flat)


def test_many_stack_offsets_and_rectangles(rd, orc, many):
    specs, picks = many["specs"], many["picks"]
    checked = full = 0
    for i in picks:
        sp = specs[i]
        img, rect, offs, nrej = many["results"][i]
        s = np.stack([offs["sx"], offs["sy"]], 1).astype(np.float32)
        assert np.array_equal(rect, orc.valid_rect(s, sp.W, sp.H)), (i, rect)
        truth = many["shifts"][i]
        assert np.all(np.abs(s[1:] - truth[1:]) < 0.1), (i, s[1:], truth[1:])
        assert offs["dx"][0] == 0 and offs["dy"][0] == 0 and s[0, 0] == 0 and s[0, 1] == 0
        cal = _calibrated(rd, many["stacks"][i])
        ref = cal[0].cpu().numpy().astype(np.float64)
        for k in sorted({1, sp.N // 2, sp.N - 1}):
            frame = cal[k].cpu().numpy().astype(np.float64)
            d = np.array([[int(offs["dx"][k]), int(offs["dy"][k])]], dtype=np.int32)
            o = orc.register(ref, frame, 1, sp.radius, centers=d)
            assert (o["dx"][0], o["dy"][0]) == (d[0, 0], d[0, 1]) or (o["flags"][0] & 4), (i, k, o, d)
            for ax in ("sx", "sy"):
                diff = abs(float(o[ax][0]) - float(offs[ax][k]))
                assert diff <= 2 * ulp32(o[ax][0]), (i, k, ax, o[ax][0], offs[ax][k])
            np.testing.assert_allclose(offs["peak"][k], o["peak"][0], rtol=1e-10)
            checked += 1
        # the whole window on the first frame of the stack
        frame = cal[1].cpu().numpy().astype(np.float64)
        o = orc.register(ref, frame, sp.radius)
        assert (o["dx"][0], o["dy"][0]) == (offs["dx"][1], offs["dy"][1]), (i, o, offs[1])
        assert o["flags"][0] == offs["flags"][1], (i, o["flags"][0], offs["flags"][1])
        for ax in ("sx", "sy"):
            assert abs(float(o[ax][0]) - float(offs[ax][1])) <= 2 * ulp32(o[ax][0]), (i, ax, o[ax][0], offs[ax][1])
        np.testing.assert_allclose(offs["peak"][1], o["peak"][0], rtol=1e-10)
        np.testing.assert_allclose(offs["second"][1], o["second"][0], rtol=1e-10)
        full += 1
        del cal
    print(f"{len(picks)} stacks, {checked} frames checked locally, {full} over the whole window; "
          f"plans {many['plans']}")


def test_many_stack_combined_rows(rd, orc, many):
    specs, picks = many["specs"], many["picks"]
    rng = np.random.default_rng(7)
    for i in picks:
        sp = specs[i]
        img, rect, offs, _ = many["results"][i]
        x0, y0, w, h = (int(v) for v in rect)
        s = np.stack([offs["sx"], offs["sy"]], 1).astype(np.float32)
        cal = _calibrated(rd, many["stacks"][i])
        for v in rng.choice(h, 2, replace=False):
            rows = []
            for k in range(sp.N):
                iy = int(np.floor(s[k, 1]))
                lo = max(y0 + v + iy - 1, 0)
                hi = min(y0 + v + iy + 3, sp.H)
                crop = cal[k, lo:hi].cpu().numpy().astype(np.float64)
                rows.append(orc.shift(crop[None], s[k:k + 1], (x0, y0 + v - lo, w, 1))[0, 0])
            al = np.stack(rows)[:, None, :]
            oo, _, _, near = orc.combine(al)
            got = img[v].cpu().numpy().astype(np.float64)
            band = near.any(axis=0)[0]
            e = rel_err(got, oo[0])
            assert e[~band].max() <= TOL, (i, int(v), err_summary(e[~band]))
        del cal
