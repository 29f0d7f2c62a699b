"""Pins of the proposal-network oracle (oracle/nn_oracle.py) and of the proposal
steps on the method side (oracle/proposal.py).

The network oracle is pinned to torch's float64 CPU routines (convolution,
pooling, nearest upsampling, autograd, Adam) and to central finite differences;
the proposal steps to closed forms and exact special cases.  Nothing here uses
the GPU library."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import nn_oracle as nn



def rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co, k in nn.LAYERS:
        p[name] = (rng.standard_normal((co, k, k, ci)) * scale * np.sqrt(2.0 / (k * k * ci)),
                   rng.standard_normal(co) * 0.1)
    return p


def nchw(x):
    return torch.from_numpy(np.ascontiguousarray(x.transpose(0, 3, 1, 2)))


def nhwc(t):
    return t.detach().numpy().transpose(0, 2, 3, 1)


def torch_w(W):
    return torch.from_numpy(np.ascontiguousarray(W.transpose(0, 3, 1, 2)))


def test_param_count():
    assert nn.param_count() == 196341
    th = np.arange(nn.param_count(), dtype=np.float64)
    np.testing.assert_array_equal(nn.flatten(nn.unflatten(th)), th)


@pytest.mark.parametrize("k,ci,co", [(3, 16, 16), (3, 112, 48), (3, 5, 7), (1, 16, 5)])
def test_conv_matches_torch(k, ci, co):
    rng = np.random.default_rng(k * 100 + ci)
    x = rng.standard_normal((2, 6, 10, ci))
    W = rng.standard_normal((co, k, k, ci))
    b = rng.standard_normal(co)
    ref = F.conv2d(nchw(x), torch_w(W), torch.from_numpy(b), padding=k // 2)
    np.testing.assert_allclose(nn.conv(x, W, b), nhwc(ref), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("k", [3, 1])
def test_conv_backward_matches_autograd(k):
    rng = np.random.default_rng(5 + k)
    x = rng.standard_normal((2, 4, 6, 8))
    W = rng.standard_normal((12, k, k, 8))
    b = rng.standard_normal(12)
    g = rng.standard_normal((2, 4, 6, 12))
    xt, Wt, bt = nchw(x).requires_grad_(), torch_w(W).requires_grad_(), torch.from_numpy(b).requires_grad_()
    y = F.conv2d(xt, Wt, bt, padding=k // 2)
    (y * nchw(g)).sum().backward()
    dx, dW, db = nn.conv_backward(x, W, g)
    np.testing.assert_allclose(dx, nhwc(xt.grad), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dW, Wt.grad.numpy().transpose(0, 2, 3, 1), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-11, atol=1e-11)


def test_pool_and_up_match_torch():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 6, 8, 3))
    np.testing.assert_allclose(nn.pool(x), nhwc(F.avg_pool2d(nchw(x), 2)), atol=1e-14)
    np.testing.assert_allclose(nn.up(x), nhwc(F.interpolate(nchw(x), scale_factor=2, mode="nearest")), atol=0)
    xt = nchw(x).requires_grad_()
    g = rng.standard_normal((2, 3, 3, 4))
    (F.avg_pool2d(xt, 2) * torch.from_numpy(g)).sum().backward()
    np.testing.assert_allclose(nn.pool_backward(nhwc(torch.from_numpy(g))), nhwc(xt.grad), atol=1e-14)
    xt = nchw(x).requires_grad_()
    g2 = rng.standard_normal((2, 3, 12, 16))
    (F.interpolate(xt, scale_factor=2, mode="nearest") * torch.from_numpy(g2)).sum().backward()
    np.testing.assert_allclose(nn.up_backward(nhwc(torch.from_numpy(g2))), nhwc(xt.grad), atol=1e-13)


def small_batch(seed, n=1, h=8, w=16):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, h, w, nn.IN_CHANNELS))
    t = np.zeros((n, h, w, 6))
    t[..., 0] = rng.uniform(2.0, 6.0, (n, h, w))
    nt = rng.standard_normal((n, h, w, 3))
    t[..., 1:4] = nt / np.linalg.norm(nt, axis=-1, keepdims=True)
    t[..., 4] = rng.uniform(0, 1, (n, h, w))
    t[..., 5] = (rng.uniform(0, 1, (n, h, w)) < 0.8).astype(float)
    q_ref = rng.uniform(1.0 / 6.0, 0.5, (n, h, w))
    return x, q_ref, t


def test_network_gradient_matches_finite_differences():
    x, q_ref, t = small_batch(1)
    theta = nn.flatten(rand_params(2))
    L, g = nn.loss_and_grads(theta, x, q_ref, t, 2.0, 6.0)
    rng = np.random.default_rng(4)
    # a few parameters of every layer
    offs, o = [], 0
    for name, ci, co, k in nn.LAYERS:
        nw = co * k * k * ci
        offs += list(o + rng.integers(0, nw, 3)) + [o + nw + int(rng.integers(0, co))]
        o += nw + co
    h = 1e-6
    for i in offs:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (nn.loss_and_grads(tp, x, q_ref, t, 2.0, 6.0)[0] - nn.loss_and_grads(tm, x, q_ref, t, 2.0, 6.0)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=2e-4, abs=1e-8), i


def test_network_gradient_matches_autograd():
    """Whole network in torch float64 autograd (a second, library implementation)."""
    x, q_ref, t = small_batch(7, n=2, h=16, w=8)
    params = rand_params(8)
    z, a = nn.forward(params, x)
    L, dz = nn.loss(z, q_ref, t, 2.0, 6.0)
    grads = nn.backward(params, a, dz)
    tp = {k: (torch_w(W).requires_grad_(), torch.from_numpy(b).requires_grad_()) for k, (W, b) in params.items()}

    def c(name, inp, act=True):
        y = F.conv2d(inp, tp[name][0], tp[name][1], padding=tp[name][0].shape[2] // 2)
        return torch.relu(y) if act else y

    xt = nchw(x)
    e0 = c("enc0b", c("enc0a", xt))
    e1 = c("enc1b", c("enc1a", F.avg_pool2d(e0, 2)))
    e2 = c("enc2b", c("enc2a", F.avg_pool2d(e1, 2)))
    e3 = c("enc3b", c("enc3a", F.avg_pool2d(e2, 2)))
    upn = lambda v: F.interpolate(v, scale_factor=2, mode="nearest")
    d2 = c("dec2", torch.cat([upn(e3), e2], 1))
    d1 = c("dec1", torch.cat([upn(d2), e1], 1))
    d0 = c("dec0", torch.cat([upn(d1), e0], 1))
    zt = c("head", d0, act=False)
    np.testing.assert_allclose(nhwc(zt), z, rtol=1e-10, atol=1e-10)
    T = nchw(t)
    R = (0.5 - 1.0 / 6.0) / 12.0
    q = torch.clamp(torch.from_numpy(q_ref) + R * torch.tanh(zt[:, 0]), 1.0 / 6.0, 0.5)
    s = (1.0 / q - 2.0) / 4.0
    td = (T[:, 0] - 2.0) / 4.0
    nh = zt[:, 1:4] / zt[:, 1:4].norm(dim=1, keepdim=True)
    w = T[:, 5]
    Lt = (w * ((s - td).abs() + 1 - (nh * T[:, 1:4]).sum(1)) + F.softplus(zt[:, 4]) - T[:, 4] * zt[:, 4]).mean()
    assert float(Lt.detach()) == pytest.approx(L, rel=1e-12)
    Lt.backward()
    for name, (dW, db) in grads.items():
        np.testing.assert_allclose(dW, tp[name][0].grad.numpy().transpose(0, 2, 3, 1), rtol=1e-8, atol=1e-12)
        np.testing.assert_allclose(db, tp[name][1].grad.numpy(), rtol=1e-8, atol=1e-12)


def test_loss_closed_forms_and_gradient():
    z = np.zeros((1, 1, 2, 5))
    z[0, 0, :, 1:4] = [0.0, 0.0, -2.0]
    q_ref = np.full((1, 1, 2), 0.25)  # z0 = 0 keeps the sweep's inverse depth: depth 4
    t = np.zeros((1, 1, 2, 6))
    t[..., 0] = 4.0
    t[..., 1:4] = [0.0, 0.0, -1.0]
    t[..., 4] = 0.0
    t[..., 5] = 1.0
    L, dz = nn.loss(z, q_ref, t, 2.0, 6.0)
    assert L == pytest.approx(np.log(2.0), abs=1e-15)  # depth and normal terms vanish; BCE(1/2, 0) = log 2
    assert np.all(dz[..., 0] == 0) and np.allclose(dz[..., 1:4], 0) and np.allclose(dz[..., 4], 0.25)
    d, _, _ = nn.decode(z, q_ref, 2.0, 6.0)
    np.testing.assert_allclose(d, 4.0, rtol=1e-15)
    # the correction saturates at one twelfth of the inverse-depth range, and the range clamps it
    zbig = z.copy()
    zbig[..., 0] = 50.0
    d, _, _ = nn.decode(zbig, q_ref, 2.0, 6.0)
    np.testing.assert_allclose(d, 1.0 / (0.25 + (0.5 - 1.0 / 6.0) / 12.0), rtol=1e-12)
    d, _, _ = nn.decode(zbig, np.full((1, 1, 2), 0.49), 2.0, 6.0)
    np.testing.assert_allclose(d, 2.0, rtol=1e-15)
    q, dq = nn.inverse_depth(np.array([3.0]), np.array([0.49]), 2.0, 6.0)
    assert q[0] == 0.5 and dq[0] == 0.0
    rng = np.random.default_rng(9)
    z = rng.standard_normal((1, 3, 4, 5))
    _, q_ref, t = small_batch(10, 1, 3, 4)
    L, dz = nn.loss(z, q_ref, t, 2.0, 6.0)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (0, 1, 2, 0), (0, 2, 1, 0), (0, 1, 2, 1), (0, 2, 3, 3), (0, 1, 1, 4), (0, 2, 0, 2)]:
        zp, zm = z.copy(), z.copy()
        zp[idx] += h
        zm[idx] -= h
        fd = (nn.loss(zp, q_ref, t, 2.0, 6.0)[0] - nn.loss(zm, q_ref, t, 2.0, 6.0)[0]) / (2 * h)
        assert dz[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_decode_ranges():
    rng = np.random.default_rng(0)
    z = rng.standard_normal((2, 4, 4, 5)) * 5
    d, n, c = nn.decode(z, rng.uniform(1 / 6, 0.5, (2, 4, 4)), 2.0, 6.0)
    assert d.min() >= 2.0 and d.max() <= 6.0
    np.testing.assert_allclose(np.linalg.norm(n, axis=-1), 1.0, rtol=1e-14)
    assert c.min() > 0 and c.max() < 1
    assert nn.confidence_target(0.0) == 1.0 and nn.confidence_target(0.3) == pytest.approx(np.exp(-0.5))


def test_adam_first_step_closed_form_and_torch():
    rng = np.random.default_rng(1)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = nn.adam_step(p0, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    np.testing.assert_allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    pt = torch.from_numpy(p0.copy()).requires_grad_()
    opt = torch.optim.Adam([pt], lr=2e-3, betas=(0.8, 0.99), eps=1e-6)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for s in range(1, 6):
        gs = rng.standard_normal(50)
        pt.grad = torch.from_numpy(gs.copy())
        opt.step()
        p, m, v = nn.adam_step(p, gs, m, v, s, 2e-3, 0.8, 0.99, 1e-6)
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_bf16_round():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 1e-3, 65504.0])
    out = nn.bf16_round(vals)
    np.testing.assert_array_equal(out[:4], [1.0, 1.0, 1.0 + 2.0 ** -6, -2.5])  # ties to even
    assert abs(out[4] - 1e-3) <= 1e-3 * 2.0 ** -8
    # bf16 keeps 8 significant bits: round trip of a representable value is exact
    np.testing.assert_array_equal(nn.bf16_round(out), out)
    assert out.dtype == np.float64


# ------------------------------------------------------------------------------------------
# proposal steps on the method side
# ------------------------------------------------------------------------------------------

def disparity_pair(oracle_mod, W=64, H=40, Z=4.0):
    """Fronto-parallel plane at Z seen by a source translated by B = 0.12 with f = 100:
    disparity exactly 3 px, so the true plane costs 0 (the exact special case of Eq. 8)."""
    from test_oracle_geometry_ncc import cam

    rng = np.random.default_rng(11)
    f, B = 100.0, 0.12
    K = np.array([[f, 0, (W - 1) / 2], [0, f, (H - 1) / 2], [0, 0, 1]])
    ref = rng.uniform(0, 255, (H, W)).astype(np.float32)
    src = np.zeros_like(ref)
    src[:, :W - 3] = ref[:, 3:] * 1.07 + 5.0
    return oracle_mod.Views([ref, src], [cam(K, np.eye(3), np.zeros(3), W, H), cam(K, np.eye(3), [-B, 0, 0], W, H)])


@pytest.mark.parametrize("W,fine", [(64, 5), (320, 11)])
def test_sweep_features_find_the_true_depth(oracle_mod, W, fine):
    """Exact case of Eq. 8: the sweep plane through the true depth costs 0, so it wins."""
    from oracle import proposal

    V = disparity_pair(oracle_mod, W=W)
    m = proposal.sub_bins(W)
    D = 12 * m
    assert (m, D) == ((1, 12) if W == 64 else (2, 24))
    # depth range chosen so that sweep plane `fine` sits exactly at Z = 4
    qz, span = 0.25, 0.14
    qf = qz - (fine + 0.5) * span / D
    P = oracle_mod.Params(d_min=1.0 / (qf + span), d_max=1.0 / qf)
    assert proposal.sweep_planes(P, W)[fine][3] == pytest.approx(4.0, rel=1e-12)
    Fm = proposal.sweep_features(V, P)
    assert Fm.shape == proposal.grid(40, W) + (16,) == (16, 8 * -(-W // 32), 16)
    inner = Fm[2:8, 2:W // 4 - 5]  # cells whose window and warped window stay inside both images
    np.testing.assert_allclose(inner[..., 2], 2.0 * (fine + 0.5) / D - 1.0, atol=1e-12)
    np.testing.assert_allclose(inner[..., 3], 1.0, atol=1e-9)
    np.testing.assert_allclose(inner[..., 4 + fine // m], 1.0, atol=1e-9)
    assert np.all(np.argmax(inner[..., 4:], axis=-1) == fine // m)
    ref = V.images[0].astype(np.float64)
    blk = ref[12:16, 20:24]
    assert Fm[3, 5, 0] == pytest.approx((blk.mean() - 127.5) / 64, rel=1e-12)
    assert Fm[3, 5, 1] == pytest.approx(np.sqrt(((blk - blk.mean()) ** 2).mean()) / 32, rel=1e-12)


def test_proposal_low_confidence_is_random_init(oracle_mod, scene_128x96):
    from oracle import proposal

    sc = scene_128x96
    img = [im[:32, :48] for im in sc.images]
    V = oracle_mod.Views(img, sc.cams)
    P = oracle_mod.Params(seed=3)
    h, w = 8, 12
    st, used = proposal.proposal_state(V, P, np.full((h, w), 4.0), np.tile([0.0, 0.0, -1.0], (h, w, 1)),
                                       np.full((h, w), 0.49))
    ref = oracle_mod.init(V, P)
    assert not used.any()
    np.testing.assert_array_equal(st.plane, ref.plane)
    np.testing.assert_array_equal(st.cost, ref.cost)


def test_proposal_at_the_true_plane(oracle_mod):
    from oracle import proposal

    V = disparity_pair(oracle_mod)
    P = oracle_mod.Params()
    h, w = 10, 16
    n = np.tile([0.0, 0.0, -1.0], (h, w, 1))
    st, used = proposal.proposal_state(V, P, np.full((h, w), 4.0), n, np.full((h, w), 0.9))
    assert used.all()
    np.testing.assert_allclose(st.plane[..., 3], 4.0, rtol=1e-14)
    np.testing.assert_allclose(st.plane[..., 2], -1.0)
    assert np.all(st.cost[8:32, 8:53] < 1e-9)  # the true plane costs 0 where the window stays inside
    # the opposite normal describes the same plane and is turned to face the camera
    st2, _ = proposal.proposal_state(V, P, np.full((h, w), 4.0), -n, np.full((h, w), 0.9))
    np.testing.assert_array_equal(st2.plane, st.plane)
    # a slanted plane: every pixel lies on the plane of its cell
    nt = np.array([0.3, -0.2, -1.0])
    nt /= np.linalg.norm(nt)
    st3, used3 = proposal.proposal_state(V, P, np.full((h, w), 4.0), np.tile(nt, (h, w, 1)), np.full((h, w), 0.9))
    Ki = proposal._kinv(V)
    for (y, x) in [(0, 0), (13, 37), (39, 63)]:
        i, j = y // 4, x // 4
        Xc = 4.0 * (Ki @ np.array([4 * j + 2, 4 * i + 2, 1.0]))
        if used3[y, x]:
            assert st3.plane[y, x, :3] @ Xc + st3.plane[y, x, 3] == pytest.approx(0.0, abs=1e-12)
            assert st3.plane[y, x, :3] @ (Ki @ np.array([x, y, 1.0])) < 0


def test_sweep_grid_of_a_ragged_image(oracle_mod):
    """Grid 8 ceil(H/32) x 8 ceil(W/32): cells past the image repeat its edge (clamped sample pixel and block)."""
    from oracle import proposal

    V = disparity_pair(oracle_mod, W=70, H=36)
    P = oracle_mod.Params()
    Fm = proposal.sweep_features(V, P)
    assert Fm.shape == (16, 24, 16)
    assert proposal.sample_pixel(36, 70, 15, 23) == (69, 35)
    # the last column of cells inside the image ends at x = 69: cells 17.. repeat column 69 / row 35
    ref = V.images[0].astype(np.float64)
    blk = ref[np.ix_([35, 35, 35, 35], [69, 69, 69, 69])]
    assert Fm[12, 20, 0] == pytest.approx((blk.mean() - 127.5) / 64, rel=1e-12)
    assert Fm[12, 20, 1] == 0.0
    np.testing.assert_array_equal(Fm[12, 20], Fm[15, 23])
