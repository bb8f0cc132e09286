"""The search entry point that allocates nothing (reduce_register_static: its workspace is
the library's fixed per-device array) against reduce_register with a caller workspace, on
two calls in a row, the second with smaller frames, fewer frames and a smaller window:
offsets and score planes bit-identical (same kernels, same launch shapes, same summation
order), and sizes beyond the fixed array rejected before any launch."""
import ctypes

import numpy as np
import pytest

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


def _frames(seed, N, H, W):
    import synth
    spec = synth.small_spec(N, W, H, n_stars=max(8, W * H // 1500), shift_bound=3.0, seed=(61, seed))
    st = synth.make_stack(spec)
    return (st.raw.astype(np.float32) - st.dark) / st.flat


@pytest.mark.parametrize("centred", [False, True])
def test_static_search_matches_workspace_search(rd, centred):
    cases = [(12, 224, 256, 9, 9), (5, 128, 160, 6, 8)]  # (N, H, W, R, Rmax): the second call is smaller
    for i, (N, H, W, R, Rmax) in enumerate(cases):
        cal = to_dev(_frames(i + (10 if centred else 0), N + 1, H, W))
        ref, frames = cal[0].contiguous(), cal[1:].contiguous()
        centres = None
        if centred:
            rng = np.random.default_rng(i)
            centres = to_dev(rng.integers(-Rmax, Rmax + 1, size=(N, 2)).astype(np.int32))
        want, want_sc = rd.register(ref, frames, R, Rmax, centers=centres, want_scores=True)
        out = torch.full((N, rd.OFFSET_BYTES), 0xAB, dtype=torch.uint8, device=cal.device)
        sc = torch.full((N, 2 * R + 1, 2 * R + 1), float("nan"), dtype=torch.float64, device=cal.device)
        rd.register_static(ref, frames, R, Rmax, centers=centres, out=out, scores=sc)
        torch.cuda.synchronize()
        assert torch.equal(out, want), (i, rd.offsets_to_numpy(out), rd.offsets_to_numpy(want))
        a, b = sc.cpu().numpy(), want_sc.cpu().numpy()
        assert np.array_equal(a, b), (i, np.nanmax(np.abs(a - b)))
        print(f"call {i}: {N} frames {W}x{H}, R={R}, Rmax={Rmax}: identical to the workspace search")


def test_static_search_rejects_sizes_beyond_its_array(rd):
    L = rd.lib()
    cap = int(L.reduce_register_static_max())
    assert cap == 64 << 20
    N, H, W, R = 64, 1024, 1024, 21
    assert int(L.reduce_register_ws(W, H, N, R, R)) > cap
    ref = torch.zeros((H, W), dtype=torch.float32, device="cuda:0")
    frames = torch.zeros((N, H, W), dtype=torch.float32, device="cuda:0")
    out = torch.empty((N, rd.OFFSET_BYTES), dtype=torch.uint8, device="cuda:0")
    rc = L.reduce_register_static(ctypes.c_void_p(ref.data_ptr()), ctypes.c_void_p(frames.data_ptr()), W, H, N, R, R,
                                  None, None, ctypes.c_void_p(out.data_ptr()), None, None)
    assert rc == rd.ERR_UNSUPPORTED, rc
    assert b"reduce_register_static" in L.reduce_last_error()
