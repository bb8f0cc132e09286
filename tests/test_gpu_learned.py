"""The offset-proposal network on the GPU against the FP64 oracle.

Each stage is checked in isolation: the oracle gets the GPU's bfloat16 input to the
stage.  The GPU accumulates in FP32 where the oracle uses FP64, so a stored bfloat16
value may differ by one bfloat16 unit when the exact value lies near a rounding
boundary; such values are counted and must be rare.
"""
import numpy as np
import pytest

import synth
from helpers import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2008_11486_amd as rd
    rd.lib()
    return rd


def bf16_ulp(v):
    v = np.abs(np.asarray(v, dtype=np.float64))
    e = np.floor(np.log2(np.maximum(v, 2.0 ** -126)))
    return 2.0 ** (e - 7)


def compare_bf16(gpu, ref, label, max_frac=0.01):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    diff = np.abs(gpu - ref)
    assert np.all(diff <= bf16_ulp(ref) * 1.0001 + 1e-30), f"{label}: max diff {diff.max()}"
    frac = np.mean(diff > 0)
    print(f"{label}: {frac:.2e} of values one bfloat16 unit apart")
    assert frac <= max_frac
    return frac


def random_params(orc, rng):
    p = np.empty(orc.cnn_num_params())
    parts = orc.cnn_split(p)
    for i, cin in enumerate(orc.CNN_CIN):
        parts[f"w{i + 1}"][...] = rng.normal(size=(9, cin, 32)) * np.sqrt(2.0 / (9 * cin))
        parts[f"b{i + 1}"][...] = rng.normal(size=32) * 0.05
    parts["wl"][...] = rng.normal(size=(2, 32)) * 0.3
    parts["bl"][...] = rng.normal(size=2) * 0.1
    return p.astype(np.float32).astype(np.float64)


def test_network_input_parity(rd, orc):
    spec = synth.small_spec(3, 256, 192, n_stars=60, shift_bound=10.0, seed=(41,))
    st = synth.make_stack(spec)
    cal = orc.calibrate(st.raw, st.dark, st.flat).astype(np.float32)
    got = rd.bf16_bits_to_float(rd.cnn_input(to_dev(cal))).cpu().numpy()
    for k in range(3):
        compare_bf16(got[k], orc.cnn_input(cal[k].astype(np.float64)), f"input frame {k}", max_frac=1e-3)


@pytest.mark.parametrize("B,h,w,shared", [(3, 64, 64, True), (2, 48, 80, False), (1, 128, 96, True)])
def test_network_forward_parity(rd, orc, B, h, w, shared):
    rng = np.random.default_rng(B * 1000 + h)
    params = random_params(orc, rng)
    ref = orc.bf16_round(rng.normal(size=(h, w) if shared else (B, h, w)))
    img = orc.bf16_round(rng.normal(size=(B, h, w)))
    pdev = to_dev(params.astype(np.float32))
    rdev = torch.from_numpy(ref.astype(np.float32)).to("cuda:0").to(torch.bfloat16).view(torch.int16)
    idev = torch.from_numpy(img.astype(np.float32)).to("cuda:0").to(torch.bfloat16).view(torch.int16)
    cws = rd.CnnWorkspace(B, h, w)
    pred = rd.cnn_forward(rdev, idev, pdev, cws, ref_shared=shared).cpu().numpy()
    parts = orc.cnn_split(params)
    refb = np.broadcast_to(ref, (B, h, w)) if shared else ref
    x = np.stack([refb, img], axis=-1)
    for layer in range(1, 5):
        got = rd.bf16_bits_to_float(cws.activation(layer)).cpu().numpy()
        want = orc.bf16_round(orc.conv_forward(x, orc.bf16_round(parts[f"w{layer}"]), parts[f"b{layer}"]))
        compare_bf16(got, want, f"layer {layer}")
        x = got.astype(np.float64)  # the next stage gets the GPU's own input
    pool = x.reshape(B, -1, 32).mean(axis=1)
    want_pred = pool @ parts["wl"].T + parts["bl"]
    np.testing.assert_allclose(pred, want_pred, rtol=1e-5, atol=1e-5)
