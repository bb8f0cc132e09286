"""End-to-end parity from raw frames: calibrate -> register -> shift -> combine.

Two comparisons per stack: (a) from the raw frames: integer offsets and the overlap
bit-exact against the oracle's whole chain; sub-pixel offsets within 2 float ulps of the
oracle's search of the GPU's own calibrated frames, and within the bound that single-
precision calibration can move them of the oracle's whole chain; the combined image
within 2e-6 of the oracle's shift and clip at the GPU's offsets (the oracle's whole chain
itself wherever the offsets agree bit for bit; the frames that differ are counted);
(b) stage-isolated, where the oracle combines the GPU's aligned frames.
"""
import numpy as np
import pytest

import synth
from helpers import TOL, assert_end_to_end, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2008_11486_amd as rd
    rd.lib()
    return rd


def gpu_chain(rd, st, integer_mode=False):
    R = st.spec.radius
    cal = rd.calibrate(to_dev(st.raw), to_dev(st.dark), to_dev(st.flat))
    offs = rd.offsets_to_numpy(rd.register(cal[0].contiguous(), cal, R))
    if integer_mode:
        s = np.stack([offs["dx"], offs["dy"]], 1).astype(np.float32)
    else:
        s = np.stack([offs["sx"], offs["sy"]], 1).astype(np.float32)
    s[0] = 0.0
    rect = rd.valid_rect(s, st.spec.W, st.spec.H)
    al = rd.shift(cal, to_dev(s), rect, integer_mode=integer_mode)
    out, keep, nrej = rd.combine(al, want_keep=True, want_nrej=True)
    return dict(cal=cal, offsets=offs, s=s, rect=rect, aligned=al, out=out.cpu().numpy(),
                keep=keep.cpu().numpy(), n_rej=int(nrej.cpu()[0]))


def _compare(orc, st, g, integer_mode=False):
    o = orc.reduce_stack(st.raw, st.dark, st.flat, st.spec.radius, integer_mode=integer_mode)
    go, oo = g["offsets"], o["offsets"]
    assert np.array_equal(go["dx"][1:], oo["dx"][1:]) and np.array_equal(go["dy"][1:], oo["dy"][1:])
    assert np.array_equal(g["rect"], o["rect"])
    e = assert_end_to_end(orc, o["cal"], g["cal"].cpu().numpy(), go, g["s"], o["s"], g["rect"], g["out"],
                          st.spec.radius, f"end-to-end {st.spec.N}x{st.spec.H}x{st.spec.W}",
                          integer_mode=integer_mode)
    # stage-isolated combine of the GPU's aligned frames
    oc, okeep, _, near = orc.combine(g["aligned"].cpu().numpy().astype(np.float64))
    flips = g["keep"] != okeep
    assert np.all(~flips | (near == 1))
    bad = flips.any(axis=0)
    print(f"stage-isolated combine: {int(flips.sum())} keep flips inside the threshold band")
    assert rel_err(g["out"], oc)[~bad].max() <= TOL
    return e


def test_workload0_integer_mode(rd, orc):
    st = synth.make_config(0)[0]
    g = gpu_chain(rd, st, integer_mode=True)
    assert np.array_equal(np.stack([g["offsets"]["dx"], g["offsets"]["dy"]], 1), st.shifts.astype(np.int64))
    _compare(orc, st, g, integer_mode=True)
    assert g["n_rej"] == 0


@pytest.mark.slow
def test_workload1_three_bands(rd, orc):
    for st in synth.make_config(1):
        g = gpu_chain(rd, st)
        truth = st.shifts
        err = np.abs(np.stack([g["offsets"]["sx"], g["offsets"]["sy"]], 1) - truth)[1:]
        print(f"sub-pixel error vs truth: max {err.max():.3f} px")
        assert err.max() < 0.1
        _compare(orc, st, g)


def test_small_stack_with_outliers(rd, orc):
    spec = synth.small_spec(16, 200, 160, n_stars=40, shift_bound=6.0, cosmic=True, seed=(3,))
    st = synth.make_stack(spec)
    g = gpu_chain(rd, st)
    _compare(orc, st, g)
    assert g["n_rej"] > 0
