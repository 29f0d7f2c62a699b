"""GPU parity of the stage after the depth maps (amh_median_filter4, amh_fuse)
against the oracle (oracle/fusion.py).

Bars:
  * median filter: bit-exact (a selection, and the mean of two float32 values,
    which rounds the same in float32 and float64), NaN where the oracle has NaN;
  * fusion, first reference view (nothing consumed yet): on every pixel whose
    decisions clear the float32 margins the oracle reports (disparity 1e-3 px,
    normal cosine 1e-5, projection 1e-3 px from a rounding boundary) the same
    decision and witness count, and the point and normal within 1e-4;
  * whole clouds: a decision flipped inside a margin changes which witnesses
    are consumed, so later views are compared as sets: totals within 0.5 %,
    >= 99.5 % of either cloud's origins in the other, common points within 1e-4.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def amh():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_07920_amd as amh

    amh.lib()
    return amh


def method_maps(amh, sc, iters=3):
    """Depth and normal maps of every view of the scene (each view the reference, the others its sources)."""
    import torch

    ctx = amh.Context(seed=0)
    ctx.init_views([torch.from_numpy(np.ascontiguousarray(im)).cuda() for im in sc.images], sc.cams)
    V = len(sc.images)
    ctx.run_batch([dict(ref=i, srcs=[j for j in range(V) if j != i], iters=iters) for i in range(V)])
    depths, normals = [], []
    for i in range(V):
        d = torch.empty((sc.height, sc.width), dtype=torch.float32, device="cuda")
        n = torch.empty((sc.height, sc.width, 3), dtype=torch.float32, device="cuda")
        ctx.get_job_result(i, depth=d, normal=n)
        depths.append(d)
        normals.append(n)
    torch.cuda.synchronize()
    return ctx, depths, normals


@pytest.mark.parametrize("H,W", [(29, 37), (1, 1), (1, 9), (7, 1), (64, 96)])
def test_median_bit_exact(amh, H, W):
    import torch

    from oracle import fusion

    say("case median", H, W)
    rng = np.random.default_rng(H * 100 + W)
    d = rng.uniform(2.0, 6.0, (H, W)).astype(np.float32)
    if H * W > 10:
        d[rng.integers(0, H, 5), rng.integers(0, W, 5)] = np.nan
    want = fusion.median_filter4(d)
    with amh.Context() as ctx:
        got = ctx.median_filter4(torch.from_numpy(d).cuda()).cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want)
    assert np.array_equal(got[ok].view(np.uint32), want[ok].view(np.uint32))


def test_median_bit_exact_fullsize(amh):
    import torch

    from oracle import fusion

    say("case median 1920x1280")
    rng = np.random.default_rng(5)
    d = rng.uniform(2.0, 6.0, (1280, 1920)).astype(np.float32)
    want = fusion.median_filter4(d)
    with amh.Context() as ctx:
        got = ctx.median_filter4(torch.from_numpy(d).cuda()).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_median_rejects_in_place(amh):
    import torch

    x = torch.ones((8, 8), device="cuda")
    with amh.Context() as ctx:
        with pytest.raises(amh.AmhError) as e:
            ctx.median_filter4(x, x)
        assert e.value.status == amh.AMH_E_INVALID_ARG


def test_fusion_of_ground_truth_one_plane_world(amh):
    import torch

    import scenegen
    from oracle import fusion

    say("case fusion one-plane world, ground-truth maps")
    sc = scenegen.make_scene(96, 64, 4, 30.0, 0, 5, supersample=2, all_views=True)
    with amh.Context() as ctx:
        ctx.init_views([np.ascontiguousarray(im) for im in sc.images], sc.cams)
        d = [torch.from_numpy(x).cuda() for x in sc.depth_views]
        n = [torch.from_numpy(x).cuda() for x in sc.normal_views]
        P, N, O, total = ctx.fuse(list(range(len(d))), d, n)
    P, N = P.cpu().numpy(), N.cpu().numpy()
    np.testing.assert_allclose(P[:, 2], scenegen.BACKGROUND_Z, atol=2e-5)
    np.testing.assert_allclose(N, np.tile([0.0, 0.0, -1.0], (len(N), 1)), atol=1e-5)
    Po, _, _ = fusion.fuse(sc.cams, sc.depth_views, sc.normal_views)
    say(f"  {total} points, oracle {len(Po)}")
    assert abs(total - len(Po)) <= 0.005 * len(Po)


def _compare_first_view(sc, depths_np, normals_np, P, N, O, pixels, **kw):
    from oracle import fusion

    W = sc.width
    first = {int(o[1]): k for k, o in enumerate(O) if o[0] == 0}
    checked = fragile = 0
    for x, y in pixels:
        r = fusion.fuse_pixel(sc.cams, depths_np, normals_np, 0, x, y, **kw)
        if r["fragile"]:
            fragile += 1
            continue
        checked += 1
        k = first.get(y * W + x)
        assert r["emitted"] == (k is not None), (x, y, r["count"])
        if k is not None:
            assert O[k, 2] == r["count"], (x, y)
            np.testing.assert_allclose(P[k], r["point"], atol=1e-4, rtol=0)
            np.testing.assert_allclose(N[k], r["normal"], atol=1e-4, rtol=0)
    return checked, fragile


def test_fusion_parity_small(amh):
    import torch

    import scenegen
    from oracle import fusion

    say("case fusion 96x64, 5 views, method depth maps")
    sc = scenegen.make_scene(96, 64, 4, 30.0, 3, 7, supersample=2)
    ctx, depths, normals = method_maps(amh, sc)
    with ctx:
        filt = [ctx.median_filter4(d) for d in depths]
        P, N, O, total = ctx.fuse(list(range(len(filt))), filt, normals)
        P2, N2, O2, total2 = ctx.fuse(list(range(len(filt))), filt, normals)
        half = total // 2
        P3, _, O3, total3 = ctx.fuse(list(range(len(filt))), filt, normals, capacity=half)
    torch.cuda.synchronize()
    # deterministic, and a smaller capacity writes a prefix of the same cloud
    assert total2 == total and torch.equal(P, P2) and torch.equal(N, N2) and torch.equal(O, O2)
    assert total3 == total and len(P3) == half and torch.equal(P3, P[:half]) and torch.equal(O3, O[:half])
    dn = [d.cpu().numpy() for d in filt]
    nn = [n.cpu().numpy() for n in normals]
    P, N, O = P.cpu().numpy(), N.cpu().numpy(), O.cpu().numpy()
    pix = [(x, y) for y in range(sc.height) for x in range(sc.width)]
    checked, fragile = _compare_first_view(sc, dn, nn, P, N, O, pix)
    say(f"  first view: {checked} pixels checked, {fragile} within a margin")
    assert checked >= 0.98 * len(pix)
    Po, No, Oo = fusion.fuse(sc.cams, dn, nn)
    key_g = {(int(a), int(b)): k for k, (a, b, _) in enumerate(O)}
    key_o = {(int(a), int(b)): k for k, (a, b, _) in enumerate(Oo)}
    common = key_g.keys() & key_o.keys()
    say(f"  points {total} vs oracle {len(Po)}, common {len(common)}")
    assert abs(total - len(Po)) <= 0.005 * len(Po)
    assert len(common) >= 0.995 * max(len(key_g), len(key_o))
    g = np.array([key_g[c] for c in sorted(common)])
    o = np.array([key_o[c] for c in sorted(common)])
    same = np.all(np.abs(P[g] - Po[o]) <= 1e-4, axis=1) & (O[g, 2] == Oo[o, 2])
    assert same.mean() >= 0.995


def test_fusion_fullsize_sampled(amh):
    """11 views of 1920x1280 (the measured scene): the first view's decisions on sampled pixels."""
    import scenegen

    say("case fusion 1920x1280, 11 views, sampled pixels of the first view")
    sc = scenegen.config_scene("1920x1280_n10", 1, device="cuda")
    ctx, depths, normals = method_maps(amh, sc)
    with ctx:
        filt = [ctx.median_filter4(d) for d in depths]
        P, N, O, total = ctx.fuse(list(range(len(filt))), filt, normals)
    say(f"  {total} points from {len(filt)} views")
    dn = [d.cpu().numpy() for d in filt]
    nn = [n.cpu().numpy() for n in normals]
    P, N, O = P.cpu().numpy(), N.cpu().numpy(), O.cpu().numpy()
    rng = np.random.default_rng(3)
    pix = [(int(rng.integers(0, sc.width)), int(rng.integers(0, sc.height))) for _ in range(1500)]
    pix += [(0, 0), (sc.width - 1, sc.height - 1)]
    checked, fragile = _compare_first_view(sc, dn, nn, P, N, O, pix)
    say(f"  {checked} checked, {fragile} within a margin")
    # each pixel makes 20 projections (10 views x 2 coordinates), each with a 2e-3 chance of landing within
    # 1e-3 px of a rounding boundary: ~4 % of the pixels are left unchecked
    assert checked >= 0.94 * len(pix)
    assert total > 0.5 * sc.width * sc.height


def test_fusion_errors(amh):
    import torch

    import scenegen

    sc = scenegen.make_scene(32, 24, 2, 20.0, 1, 1, supersample=1)
    d = torch.ones((24, 32), device="cuda")
    n = torch.zeros((24, 32, 3), device="cuda")
    with amh.Context() as ctx:
        ctx.init_views([np.ascontiguousarray(im) for im in sc.images], sc.cams)
        for kw, views in ((dict(), [5]), (dict(f_con=-1), [0]), (dict(f_eps=0.0), [0]), (dict(f_ang_deg=200.0), [0])):
            with pytest.raises(amh.AmhError) as e:
                ctx.fuse(views, [d] * len(views), [n] * len(views), **kw)
            assert e.value.status == amh.AMH_E_INVALID_ARG
        with pytest.raises(amh.AmhError):
            ctx.fuse([0] * 129, [d] * 129, [n] * 129)
        # one view, f_con 0: every pixel with a depth yields its own back-projection
        P, N, O, total = ctx.fuse([0], [d], [n], f_con=0)
        assert total == 32 * 24


@pytest.mark.parametrize("W,H", [(1, 1), (1, 7), (9, 1), (65, 3)])
def test_fusion_tiny_views(amh, W, H):
    """Views of 1 to a few pixels (ragged 64-pixel blocks): the cloud equals the vectorised oracle's."""
    import torch

    import scenegen
    from oracle import fusion

    say("case fusion tiny", W, H)
    sc = scenegen.make_scene(W, H, 2, 10.0, 0, 3, supersample=1, all_views=True)
    with amh.Context() as ctx:
        ctx.init_views([np.ascontiguousarray(im) for im in sc.images], sc.cams)
        d = [torch.from_numpy(x).cuda() for x in sc.depth_views]
        n = [torch.from_numpy(x).cuda() for x in sc.normal_views]
        P, N, O, total = ctx.fuse([0, 1, 2], d, n, f_con=1)
    Po, _, Oo = fusion.fuse(sc.cams, sc.depth_views, sc.normal_views, f_con=1)
    assert total == len(Po)
    assert np.array_equal(O.cpu().numpy()[:, :2], Oo[:, :2].astype(np.int32))
    np.testing.assert_allclose(P.cpu().numpy(), Po, atol=1e-4)


def test_fusion_views_of_different_sizes(amh):
    """Two parallel cameras of different image sizes looking at one fronto-parallel plane: the cloud equals the
    oracle's, point for point."""
    import torch

    from oracle import fusion

    class Cam:
        def __init__(self, K, t, w, h):
            self.K, self.R, self.t, self.width, self.height = K, np.eye(3), np.asarray(t, float), w, h

    say("case fusion different sizes")
    cams, depths, normals = [], [], []
    for (w, h, tx) in ((40, 24, 0.0), (56, 30, -0.52)):
        K = np.array([[100.0, 0, (w - 1) / 2], [0, 100.0, (h - 1) / 2], [0, 0, 1.0]])
        cams.append(Cam(K, [tx, 0, 0], w, h))
        depths.append(np.full((h, w), 4.0, np.float32))
        normals.append(np.tile(np.array([0, 0, -1], np.float32), (h, w, 1)))
    imgs = [np.full((c.height, c.width), 100.0, np.float32) for c in cams]
    with amh.Context() as ctx:
        ctx.init_views(imgs, cams)
        P, N, O, total = ctx.fuse([0, 1], [torch.from_numpy(d).cuda() for d in depths],
                                  [torch.from_numpy(n).cuda() for n in normals], f_con=1)
    Po, _, Oo = fusion.fuse(cams, depths, normals, f_con=1)
    say(f"  {total} points, oracle {len(Po)}")
    assert total == len(Po) > 0
    assert np.array_equal(O.cpu().numpy()[:, :2], Oo[:, :2].astype(np.int32))
    np.testing.assert_allclose(P.cpu().numpy(), Po, atol=1e-4)
