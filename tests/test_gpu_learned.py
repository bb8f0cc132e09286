"""The offset-proposal network on the GPU against the FP64 oracle.

Each stage is checked in isolation: the oracle gets the GPU's bfloat16 input to the
stage.  The GPU accumulates in FP32 where the oracle uses FP64, so a stored bfloat16
value may differ by one bfloat16 unit when the exact value lies near a rounding
boundary; such values are counted and must be rare.
"""
import os

import numpy as np
import pytest

import synth
from helpers import to_dev, ulp32

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


def _bf16_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0").to(torch.bfloat16) \
        .view(torch.int16)


def _net_case(rd, orc, B, h, w, seed):
    rng = np.random.default_rng(seed)
    params = random_params(orc, rng)
    ref = orc.bf16_round(rng.normal(size=(h, w)))
    img = orc.bf16_round(rng.normal(size=(B, h, w)))
    target = rng.normal(size=(B, 2)) * 2.0  # a share beyond the Huber threshold
    pdev = to_dev(params.astype(np.float32))
    rdev, idev = _bf16_dev(ref), _bf16_dev(img)
    cws = rd.CnnWorkspace(B, h, w)
    pred = rd.cnn_forward(rdev, idev, pdev, cws)
    tdev = to_dev(target.astype(np.float32))
    loss, grad = rd.cnn_backward(rdev, idev, pdev, pred, tdev, cws, huber_delta=1.0)
    x = np.stack([np.broadcast_to(ref, (B, h, w)), img], axis=-1)
    return dict(params=params, x=x, target=target, pred=pred.cpu().numpy().astype(np.float64),
                loss=float(loss.cpu()[0]), grad=grad.cpu().numpy().astype(np.float64), cws=cws)


@pytest.mark.parametrize("B,h,w", [(3, 64, 64), (2, 48, 80), (5, 37, 53)])
def test_network_backward_stages(rd, orc, B, h, w):
    """Each backward stage against the oracle, given the GPU's own stage inputs."""
    c = _net_case(rd, orc, B, h, w, seed=B * 7 + h)
    parts = orc.cnn_split(c["params"])
    g = orc.cnn_split(c["grad"])
    acts = [c["x"]] + [rd.bf16_bits_to_float(c["cws"].activation(l)).cpu().numpy().astype(np.float64)
                       for l in range(1, 5)]
    # head: Huber derivative, pool of the GPU's X4
    e = c["pred"] - c["target"]
    dpred = np.where(np.abs(e) <= 1.0, e, np.sign(e)) / e.size
    pool = acts[4].reshape(B, -1, 32).mean(axis=1)
    np.testing.assert_allclose(g["wl"], dpred.T @ pool, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(g["bl"], dpred.sum(axis=0), rtol=1e-5, atol=1e-7)
    hub = np.where(np.abs(e) <= 1.0, 0.5 * e * e, np.abs(e) - 0.5).mean()
    assert c["loss"] == pytest.approx(hub, rel=1e-5)
    # conv layers 1 and 2: weight and bias gradients from the GPU's dZ, and dZ1 from dZ2
    dz = {l: rd.bf16_bits_to_float(c["cws"].grad_z(l)).cpu().numpy().astype(np.float64) for l in (1, 2)}
    for l in (1, 2):
        dx, dw, db = orc.conv_backward(acts[l - 1], orc.bf16_round(parts[f"w{l}"]), dz[l], want_dx=(l == 2))
        scale = np.abs(dw).max()
        np.testing.assert_allclose(g[f"w{l}"], dw, rtol=1e-4, atol=1e-4 * scale)
        np.testing.assert_allclose(g[f"b{l}"], db, rtol=1e-4, atol=1e-4 * np.abs(db).max())
        if l == 2:
            want = orc.bf16_round(dx * (acts[1] > 0))
            compare_bf16(dz[1], want, "dZ1 from dZ2")


@pytest.mark.parametrize("B,h,w", [(4, 64, 64), (2, 40, 72)])
def test_network_gradient_vs_oracle(rd, orc, B, h, w):
    """The whole gradient against the oracle's bfloat16-mode backward on the same input."""
    c = _net_case(rd, orc, B, h, w, seed=100 + B)
    loss, grad = orc.cnn_loss_backward(c["x"], c["params"], c["target"], 1.0, bf16=True)
    assert c["loss"] == pytest.approx(loss, rel=1e-3)
    got, want = orc.cnn_split(c["grad"]), orc.cnn_split(grad)
    for k in want:
        a, b = got[k].ravel(), want[k].ravel()
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        print(f"{k}: relative L2 {rel:.2e}, cosine {cos:.6f}")
        assert rel <= 2e-2 and cos >= 0.999, k


def test_adamw_matches_torch(rd):
    rng = np.random.default_rng(5)
    n = 1000
    p0 = rng.normal(size=n).astype(np.float32)
    grads = [rng.normal(size=n).astype(np.float32) for _ in range(3)]
    pt = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.AdamW([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.05)
    pd = to_dev(p0)
    m = torch.zeros_like(pd)
    v = torch.zeros_like(pd)
    for step, gr in enumerate(grads, start=1):
        pt.grad = torch.from_numpy(gr)
        opt.step()
        rd.cnn_adamw(pd, m, v, to_dev(gr), lr=1e-2, step=step, weight_decay=0.05)
    np.testing.assert_allclose(pd.cpu().numpy(), pt.detach().numpy(), rtol=1e-5, atol=1e-6)


def test_adamw_matches_oracle(rd, orc):
    """Stage-isolated per step: from the GPU's single-precision state (p, m, v) before each
    step, the FP64 oracle takes the same AdamW step with the same (float-rounded) hyper-
    parameters.  Bound from the arithmetic, u = 2^-24: the moments take 3 and 4 correctly
    rounded operations (|dm| <= 3u(|b1 m| + |(1 - b1) g|), |dv| <= 4u(|b2 v| + |(1 - b2) g^2|)),
    the step r = mhat / (sqrt(vhat) + eps) carries at most 16u relative error including the
    moments', and the update two more roundings: |dp| <= 2u|p'| + 16u lr (|r| + wd |p|)."""
    rng = np.random.default_rng(6)
    n = 4096
    f = lambda x: float(np.float32(x))  # noqa: E731
    lr, b1, b2, eps, wd = f(3e-3), f(0.9), f(0.999), f(1e-8), f(0.05)
    u = 2.0 ** -24
    p = rng.normal(size=n).astype(np.float32)
    pd = to_dev(p)
    m = torch.zeros_like(pd)
    v = torch.zeros_like(pd)
    for step in range(1, 6):
        g = (rng.normal(size=n) * np.exp(rng.uniform(-4, 2, size=n))).astype(np.float32)
        p0, m0, v0 = (t.cpu().numpy().astype(np.float64) for t in (pd, m, v))
        rd.cnn_adamw(pd, m, v, to_dev(g), lr=lr, step=step, beta1=b1, beta2=b2, eps=eps, weight_decay=wd)
        po, mo, vo = orc.adamw(p0, m0, v0, g, lr, step, beta1=b1, beta2=b2, eps=eps, weight_decay=wd)
        gd = g.astype(np.float64)
        r = (mo / (1 - b1 ** step)) / (np.sqrt(vo / (1 - b2 ** step)) + eps)
        tol_m = 3 * u * (np.abs(b1 * m0) + np.abs((1 - b1) * gd))
        tol_v = 4 * u * (np.abs(b2 * v0) + np.abs((1 - b2) * gd * gd))
        tol_p = 2 * u * np.abs(po) + 16 * u * lr * (np.abs(r) + wd * np.abs(p0))
        for name, got, want, tol in (("m", m, mo, tol_m), ("v", v, vo, tol_v), ("p", pd, po, tol_p)):
            d = np.abs(got.cpu().numpy().astype(np.float64) - want)
            assert np.all(d <= tol), (step, name, float((d / np.maximum(tol, 1e-300)).max()))


# ---- rendered training frames --------------------------------------------------------------
def _render_np(stars, W, H, sky, fwhm):
    sig = fwhm / (2 * np.sqrt(2 * np.log(2)))
    out = np.full((stars.shape[0], H, W), sky, dtype=np.float64)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    for f in range(stars.shape[0]):
        for x, y, a, _ in stars[f].astype(np.float64):
            m = (np.abs(xx - x) <= 8) & (np.abs(yy - y) <= 8)
            out[f][m] += a * np.exp(-((xx[m] - x) ** 2 + (yy[m] - y) ** 2) / (2 * sig * sig))
    return out


def test_render_noise_free_matches_numpy(rd):
    rng = np.random.default_rng(3)
    F, S, W, H = 3, 300, 200, 136
    stars = np.zeros((F, S, 4), np.float32)
    stars[..., 0] = rng.uniform(-20, W + 20, (F, S))
    stars[..., 1] = rng.uniform(-20, H + 20, (F, S))
    stars[..., 2] = rng.uniform(100, 5e4, (F, S))
    keys = torch.arange(F, dtype=torch.int64, device="cuda:0")
    got = rd.render_frames(to_dev(stars), keys, W, H, sky=1000.0, fwhm=3.0, noise=False).cpu().numpy()
    want = _render_np(stars, W, H, 1000.0, 3.0)
    np.testing.assert_allclose(got, want, rtol=2e-6, atol=1e-3)


def test_render_noise_matches_philox_reference(rd):
    from philox_ref import philox4x32_10, std_normal
    W, H, F = 96, 40, 2
    stars = np.zeros((F, 1, 4), np.float32)
    stars[:, 0] = (50.3, 20.7, 3e4, 0)
    keys = np.array([5, (1 << 48) | 77], np.int64)
    seed = 0x1234_5678_9ABC_DEF0
    got = rd.render_frames(to_dev(stars), torch.from_numpy(keys).to("cuda:0"), W, H, sky=1000.0, fwhm=3.0,
                           read_noise=10.0, seed=seed).cpu().numpy().astype(np.float64)
    clean = _render_np(stars, W, H, 1000.0, 3.0)
    pix = np.arange(W * H, dtype=np.uint64)
    for f in range(F):
        k = int(keys[f])
        r = philox4x32_10(pix & 0xFFFFFFFF, pix >> 32, np.full(pix.shape, k & 0xFFFFFFFF, np.uint64),
                          np.full(pix.shape, k >> 32, np.uint64), seed & 0xFFFFFFFF, seed >> 32)
        z = std_normal(r[0], r[1]).reshape(H, W)
        want = clean[f] + np.sqrt(clean[f] + 100.0) * z
        np.testing.assert_allclose(got[f], want, rtol=1e-5, atol=1e-3)
    # the noise is standard normal after scaling
    zz = (got - clean) / np.sqrt(clean + 100.0)
    assert abs(zz.mean()) < 0.05 and abs(zz.std() - 1.0) < 0.05


def test_render_is_reproducible_and_keyed(rd):
    stars = torch.zeros((2, 0, 4), dtype=torch.float32, device="cuda:0")
    a = rd.render_frames(stars, torch.tensor([1, 2], device="cuda:0"), 64, 64, seed=9)
    b = rd.render_frames(stars, torch.tensor([1, 3], device="cuda:0"), 64, 64, seed=9)
    assert torch.equal(a[0], b[0]) and not torch.equal(a[1], b[1])


def test_centres(rd):
    pred = np.array([[0.1, -0.124], [0.125, 0.375], [-16.2, 17.0], [np.nan, 2.5]], np.float32)
    got = rd.cnn_centres(to_dev(pred), 4.0, 64).cpu().numpy()
    want = np.clip(np.rint(pred.astype(np.float32) * np.float32(4.0)), -64, 64)
    want[3, 0] = -64
    np.testing.assert_array_equal(got, want.astype(np.int32))


# ---- training and the narrowed search ---------------------------------------------------------
TRAIN_W, TRAIN_BOUND, TRAIN_RMAX = 512, 12, 16


@pytest.fixture(scope="module")
def trained(rd):
    from paper_2008_11486_amd import learned
    tr = learned.ProposalTrainer(TRAIN_W, TRAIN_W, batch=16, shift_bound=TRAIN_BOUND, lr=2e-3, seed=0)
    untrained = tr.params.clone()
    hist = tr.train(n_pairs=2048, epochs=3, warmup=20, log_every=8)
    print("loss history", hist[:3], "...", hist[-3:])
    return learned, untrained, tr.params.clone(), hist


def test_training_lowers_the_loss(trained):
    _, _, _, hist = trained
    losses = np.array([l for _, l in hist])
    first, last = losses[:4].mean(), losses[-4:].mean()
    print(f"loss {first:.3f} -> {last:.3f}")
    assert last < 0.5 * first


def test_trained_proposals_need_fewer_fallbacks(trained):
    learned, p0, p1, _ = trained
    M = 24
    frames, t = learned.render_stack(0, M + 1, TRAIN_W, TRAIN_W, TRAIN_BOUND)
    ref, rest = frames[0], frames[1:].contiguous()
    import paper_2008_11486_amd as rd
    full = rd.offsets_to_numpy(learned.full_search(ref, rest, TRAIN_RMAX))
    out = {}
    for name, p in (("untrained", p0), ("trained", p1)):
        reg = learned.LearnedRegistrar(p, TRAIN_W, TRAIN_W, M, radius_max=TRAIN_RMAX)
        res = reg.register(ref, rest)
        # the fallback keeps the result identical to the full search
        np.testing.assert_array_equal(res.offsets["dx"], full["dx"])
        np.testing.assert_array_equal(res.offsets["dy"], full["dy"])
        err = np.abs(res.centres - np.stack([full["dx"], full["dy"]], 1)).max(axis=1)
        out[name] = (int(res.fallback.sum()), float(np.median(err)))
        print(name, "fallbacks", out[name][0], "of", M, "median centre error", out[name][1], res.reason)
    assert out["trained"][0] < out["untrained"][0]
    assert out["trained"][1] < out["untrained"][1]


def test_recentre_moves_border_windows_only(rd):
    o = np.zeros(5, dtype=rd.OFFSET_DTYPE)
    o["dx"] = [5, -62, 3, 9, 64]
    o["dy"] = [-2, 1, 4, 63, 10]
    o["flags"] = [rd.EDGE_X, rd.EDGE_Y | rd.CLIPPED, 0, rd.EDGE_X | rd.EDGE_Y, rd.EDGE_X | rd.CLIPPED]
    raw = torch.from_numpy(o.view(np.uint8).reshape(5, -1).copy()).to("cuda:0")
    c = torch.tensor([[3, -2], [-62, 0], [1, 1], [7, 61], [63, 10]], dtype=torch.int32, device="cuda:0")
    rd.recentre(raw, c, 64)
    # the last window's maximum is on the +64 border, which the full search shares: it stays
    np.testing.assert_array_equal(c.cpu().numpy(), [[5, -2], [-62, 1], [1, 1], [9, 63], [63, 10]])


def _host_flow(rd, learned, params, ref, frames, rmax, r=2, ratio=0.5, moves=4):
    """The proposal -> narrowed search -> window moves -> fallback decisions taken on the
    host, one stage-wise call at a time (the reference for the device-side call)."""
    M, H, W = frames.shape
    inp_ref = rd.cnn_input(ref.reshape(1, H, W))
    inp = rd.cnn_input(frames)
    cws = rd.CnnWorkspace(M, H // 4, W // 4)
    pred = rd.cnn_forward(inp_ref[0], inp, torch.from_numpy(np.asarray(params, np.float32)).to("cuda:0"), cws)
    cen = rd.cnn_centres(pred, 4.0, rmax)
    o = rd.offsets_to_numpy(rd.register(ref, frames, r, rmax, centers=cen))
    s_auto = float(rd.offsets_to_numpy(rd.register(ref, ref.reshape(1, H, W), 0, rmax))["peak"][0])

    def inner(o):
        ix = (o["dx"] > -rmax) & (o["dx"] < rmax)
        iy = (o["dy"] > -rmax) & (o["dy"] < rmax)
        return (((o["flags"] & rd.EDGE_X) != 0) & ix) | (((o["flags"] & rd.EDGE_Y) != 0) & iy)

    n_moves = np.zeros(M, np.int32)
    c = cen.cpu().numpy().copy()
    for _ in range(moves):
        walk = np.nonzero(inner(o))[0]
        for k in walk:
            c[k] = (o["dx"][k], o["dy"][k])
            o[k] = rd.offsets_to_numpy(rd.register(ref, frames[k:k + 1], r, rmax,
                                                   centers=torch.from_numpy(c[k:k + 1].copy()).to("cuda:0")))[0]
            n_moves[k] += 1
    fb = inner(o) | ~(o["peak"] >= ratio * s_auto)
    for k in np.nonzero(fb)[0]:
        o[k] = rd.offsets_to_numpy(rd.register(ref, frames[k:k + 1], rmax, rmax))[0]
        o["flags"][k] |= rd.FALLBACK
    return o, cen.cpu().numpy(), fb, n_moves


def test_propose_matches_the_host_flow(rd, trained):
    """reduce_propose takes every decision on the device; the same decisions taken on the
    host with the stage-wise calls give the same bytes, for trained and untrained weights."""
    learned, p0, p1, _ = trained
    M = 24
    frames, _ = learned.render_stack(3, M + 1, TRAIN_W, TRAIN_W, TRAIN_BOUND)
    ref, rest = frames[0], frames[1:].contiguous()
    for name, p in (("untrained", p0), ("trained", p1)):
        o_dev, c_dev, info = rd.propose(ref, rest, p, radius_max=TRAIN_RMAX)
        got = rd.offsets_to_numpy(o_dev)
        want, c_host, fb, n_moves = _host_flow(rd, learned, p.cpu().numpy(), ref, rest, TRAIN_RMAX)
        info = info.cpu().numpy()
        print(f"{name}: {int(fb.sum())} fallbacks, {int(n_moves.sum())} moves")
        np.testing.assert_array_equal(c_dev.cpu().numpy(), c_host)
        np.testing.assert_array_equal(info & 255, n_moves)
        np.testing.assert_array_equal((info >> 8) & 3 != 0, fb)
        assert got.tobytes() == want.tobytes(), name


@pytest.mark.slow
def test_trained_weights_at_4096_match_the_full_search(rd, orc):
    """The shipped network (trained on the GPU by these kernels on 4096x4096 pairs with
    shifts within +-64 px) on two evaluation stacks of 16 frames each: the learned call's
    integer offsets equal the full +-64 px search on every frame, with no fallback; the
    untrained network needs the fallback far more often; the full search itself matches
    the oracle's whole window on one frame."""
    from paper_2008_11486_amd import learned
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    trained_p = learned.load_params(os.path.join(root, "paper_2008_11486_amd", "weights", "proposal_4096.npy"))
    M, S = 16, 4096
    stats = {"trained": [0, 0, []], "untrained": [0, 0, []]}
    for index in (0, 1):
        frames, t = learned.render_stack(index, M + 1, S, S, 64.0)
        ref, rest = frames[0], frames[1:].contiguous()
        full = rd.offsets_to_numpy(learned.full_search(ref, rest, 64))
        for name, p in (("trained", trained_p), ("untrained", learned.init_params(0))):
            res = learned.LearnedRegistrar(p, S, S, M, radius_max=64).register(ref, rest)
            np.testing.assert_array_equal(res.offsets["dx"], full["dx"])
            np.testing.assert_array_equal(res.offsets["dy"], full["dy"])
            err = np.abs(res.centres - np.stack([full["dx"], full["dy"]], 1)).max(axis=1)
            stats[name][0] += int(res.fallback.sum())
            stats[name][1] += M
            stats[name][2] += list(err)
        if index == 0:
            o = orc.register(ref.cpu().numpy().astype(np.float64), rest[0].cpu().numpy().astype(np.float64), 64)
            assert (o["dx"][0], o["dy"][0]) == (full["dx"][0], full["dy"][0])
            for ax in ("sx", "sy"):
                assert abs(float(o[ax][0]) - float(full[ax][0])) <= 2 * ulp32(o[ax][0])
            np.testing.assert_allclose(full["peak"][0], o["peak"][0], rtol=1e-10)
        del frames, ref, rest
    for name, (nfb, n, err) in stats.items():
        print(f"{name}: fallback rate {nfb / n:.3f} ({nfb} of {n}), centre error median {np.median(err):.1f} px, "
              f"max {np.max(err):.0f} px")
    assert stats["trained"][0] == 0
    assert stats["untrained"][0] > stats["trained"][0]
