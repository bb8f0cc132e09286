"""Pins of the network oracle: torch float64 conv2d and autograd (an independent
implementation), central finite differences, and bfloat16 rounding against torch's
conversion."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import torch.nn.functional as F  # noqa: E402


def _torch_weight(w):  # [9][cin][cout] -> [cout][cin][3][3]
    w = torch.as_tensor(np.asarray(w, dtype=np.float64))
    return w.reshape(3, 3, w.shape[1], w.shape[2]).permute(3, 2, 0, 1).contiguous()


def _nchw(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64)).permute(0, 3, 1, 2).contiguous()


def _nhwc(t):
    return t.permute(0, 2, 3, 1).contiguous().detach().numpy()


@pytest.mark.parametrize("cin,H,W", [(2, 16, 16), (32, 9, 14), (3, 7, 5)])
def test_conv_forward_and_backward_match_torch(orc, cin, H, W):
    rng = np.random.default_rng(cin * 100 + H)
    B, cout = 2, 32
    x = rng.normal(size=(B, H, W, cin))
    w = rng.normal(size=(9, cin, cout)) * 0.2
    b = rng.normal(size=cout)
    for relu in (False, True):
        y = orc.conv_forward(x, w, b, relu=relu)
        ref = F.conv2d(_nchw(x), _torch_weight(w), torch.as_tensor(b), stride=2, padding=1)
        if relu:
            ref = torch.relu(ref)
        np.testing.assert_allclose(y, _nhwc(ref), rtol=1e-12, atol=1e-12)
    dz = rng.normal(size=y.shape)
    dx, dw, db = orc.conv_backward(x, w, dz)
    xt = _nchw(x).requires_grad_(True)
    wt = _torch_weight(w).requires_grad_(True)
    bt = torch.as_tensor(b).requires_grad_(True)
    z = F.conv2d(xt, wt, bt, stride=2, padding=1)
    (z * _nchw(dz)).sum().backward()
    np.testing.assert_allclose(dx, _nhwc(xt.grad), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dw, wt.grad.permute(2, 3, 1, 0).reshape(9, cin, cout).numpy(), rtol=1e-11,
                               atol=1e-11)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-11, atol=1e-11)


def _torch_net(orc, x, params, target, delta):
    p = orc.cnn_split(torch.as_tensor(params))
    h = _nchw(x)
    for i in range(1, 5):
        h = torch.relu(F.conv2d(h, _torch_weight_t(p[f"w{i}"]), p[f"b{i}"], stride=2, padding=1))
    pool = h.mean(dim=(2, 3))
    pred = pool @ p["wl"].T + p["bl"]
    loss = F.huber_loss(pred, torch.as_tensor(target), delta=delta, reduction="mean")
    return pred, loss


def _torch_weight_t(w):
    return w.reshape(3, 3, w.shape[1], w.shape[2]).permute(3, 2, 0, 1)


def _params(orc, rng):
    n = orc.cnn_num_params()
    p = np.empty(n)
    parts = orc.cnn_split(p)
    for i, cin in enumerate(orc.CNN_CIN):
        parts[f"w{i + 1}"][...] = rng.normal(size=(9, cin, 32)) * np.sqrt(2.0 / (9 * cin))
        parts[f"b{i + 1}"][...] = rng.normal(size=32) * 0.05
    parts["wl"][...] = rng.normal(size=(2, 32)) * 0.3
    parts["bl"][...] = rng.normal(size=2) * 0.1
    return p


def test_network_forward_and_gradient_match_torch_autograd(orc):
    rng = np.random.default_rng(7)
    B, H, W = 3, 32, 48
    x = rng.normal(size=(B, H, W, 2))
    params = _params(orc, rng)
    target = rng.normal(size=(B, 2)) * 2
    pred = orc.cnn_forward(x, params, bf16=False)
    loss, grad = orc.cnn_loss_backward(x, params, target, 1.0, bf16=False)
    pt = torch.as_tensor(params).requires_grad_(True)
    tpred, tloss = _torch_net(orc, x, pt, target, 1.0)
    tloss.backward()
    np.testing.assert_allclose(pred, tpred.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert loss == pytest.approx(float(tloss.detach()), rel=1e-12)
    np.testing.assert_allclose(grad, pt.grad.numpy(), rtol=1e-9, atol=1e-12)
    # some targets beyond the Huber threshold exercise the linear branch
    assert np.any(np.abs(pred - target) > 1.0)


def test_network_gradient_central_differences(orc):
    rng = np.random.default_rng(8)
    B, H, W = 2, 16, 16
    x = rng.normal(size=(B, H, W, 2))
    params = _params(orc, rng)
    target = rng.normal(size=(B, 2))
    _, grad = orc.cnn_loss_backward(x, params, target, 1.0, bf16=False)
    idx = rng.choice(params.size, size=40, replace=False)
    h = 1e-5
    for i in idx:
        p1, p2 = params.copy(), params.copy()
        p1[i] += h
        p2[i] -= h
        l1, _ = orc.cnn_loss_backward(x, p1, target, 1.0, bf16=False)
        l2, _ = orc.cnn_loss_backward(x, p2, target, 1.0, bf16=False)
        fd = (l1 - l2) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(abs(fd), 1e-3), (i, fd, grad[i])


def test_bf16_rounding_matches_torch(orc):
    rng = np.random.default_rng(9)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-8, 8, size=5000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, -2.5, 3.0e38, 1e-40])])
    # exact halfway points between bfloat16 neighbours: ties go to even
    base = np.float32(rng.uniform(1, 2, size=100)).view(np.uint32) & np.uint32(0xffff0000)
    halfway = (base | np.uint32(0x8000)).view(np.float32).astype(np.float64)
    x = np.concatenate([x, halfway])
    ref = torch.as_tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(orc.bf16_round(x), ref)


def test_bf16_mode_rounds_at_the_storage_points(orc):
    rng = np.random.default_rng(10)
    B, H, W = 2, 16, 16
    x = orc.bf16_round(rng.normal(size=(B, H, W, 2)))
    params = _params(orc, rng)
    pred, acts = orc.cnn_forward(x, params, bf16=True, want_acts=True)
    n_act = acts.size - B * 32
    np.testing.assert_array_equal(acts[:n_act], orc.bf16_round(acts[:n_act]))  # stored activations
    pred_exact = orc.cnn_forward(x, params, bf16=False)
    assert np.all(np.abs(pred - pred_exact) < 0.05 * (1 + np.abs(pred_exact)))  # rounding only perturbs


def test_network_input_normalisation(orc):
    rng = np.random.default_rng(11)
    img = 1000 + rng.normal(0, 30, size=(64, 96))
    img[10:14, 20:24] += 5e4
    z = orc.cnn_input(img)
    d = orc.downsample4(img)
    ref = np.arcsinh((d - d.mean()) / d.std())
    np.testing.assert_allclose(z, ref, rtol=2 ** -8, atol=2 ** -8)  # bfloat16 has 8 significant bits
    np.testing.assert_array_equal(z, orc.bf16_round(z))
    assert np.array_equal(orc.cnn_input(np.full((32, 32), 7.0)), np.zeros((8, 8)))


def test_adamw_constant_gradient_closed_form(orc):
    """With the same gradient g at every step the bias-corrected moments are exactly g and
    g^2, so every step is p <- (1 - lr wd) p - lr g / (|g| + eps): after T steps
    p_T = q^T p_0 - c (1 - q^T) / (1 - q) with q = 1 - lr wd, c = lr g / (|g| + eps).
    A coupled (L2-in-the-gradient) decay, a missing bias correction or eps inside the
    square root all break it."""
    rng = np.random.default_rng(12)
    n, lr, wd, eps, T = 64, 1e-2, 0.1, 1e-3, 7
    p0 = rng.normal(size=n)
    g = rng.normal(size=n) * np.exp(rng.uniform(-3, 3, size=n))
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, T + 1):
        p, m, v = orc.adamw(p, m, v, g, lr, t, beta1=0.9, beta2=0.99, eps=eps, weight_decay=wd)
    q = 1.0 - lr * wd
    c = lr * g / (np.abs(g) + eps)
    want = q ** T * p0 - c * (1.0 - q ** T) / (1.0 - q)
    np.testing.assert_allclose(p, want, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(m, (1 - 0.9 ** T) * g, rtol=1e-13)
    np.testing.assert_allclose(v, (1 - 0.99 ** T) * g * g, rtol=1e-13)


def test_adamw_first_step_by_hand(orc):
    """Step 1 from zero moments, worked by hand: m = 0.1 g, v = 0.001 g^2, mhat = g,
    vhat = g^2; for g = 2, p = 3, lr = 0.5, wd = 0.25, eps = 1:
    p <- 3 - 0.5 (2 / (2 + 1) + 0.25 * 3) = 3 - 0.5 * (17 / 12) = 2.291666..."""
    p, m, v = orc.adamw([3.0], [0.0], [0.0], [2.0], 0.5, 1, beta1=0.9, beta2=0.999, eps=1.0, weight_decay=0.25)
    assert p[0] == pytest.approx(3.0 - 0.5 * 17.0 / 12.0, rel=1e-15)
    assert m[0] == pytest.approx(0.2, rel=1e-15) and v[0] == pytest.approx(0.004, rel=1e-13)


def test_adamw_matches_torch_float64(orc):
    """Independent implementation of the same rule: torch.optim.AdamW in float64 on the CPU."""
    rng = np.random.default_rng(13)
    n = 200
    p0 = rng.normal(size=n)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.AdamW([tp], lr=3e-3, betas=(0.8, 0.95), eps=1e-6, weight_decay=0.02)
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        g = rng.normal(size=n)
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = orc.adamw(p, m, v, g, 3e-3, t, beta1=0.8, beta2=0.95, eps=1e-6, weight_decay=0.02)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)
