"""Pins of the oracle's post-processing and fusion (oracle/fusion.py).

* Median filter: against a per-pixel sort of the clipped window (ragged
  image), a constant image, a removed spike, and the closed form on a ramp.
* Fusion on the ground-truth maps of a one-plane world: every point lies on the
  plane z = 5.9 with normal (0, 0, -1).
* Two parallel cameras (closed form): a pixel of view 0 at depth z0 lands
  fB/z0 = 13 px to the left in view 1; with view 1 at z0 + delta the disparity
  difference is fB |1/z0 - 1/(z0 + delta)|, fused just below f_eps and not just
  above; normals 29 vs 31 degrees apart decide the same way.
* f_con = 0 yields every valid pixel, a pixel without witnesses at its own
  back-projection; identical cameras consume every pixel of the second view;
  pixels without depth yield nothing and witness nothing.
"""
import math

import numpy as np
import pytest

from oracle import fusion


def test_median_matches_sorted_window():
    rng = np.random.default_rng(0)
    d = rng.uniform(2.0, 6.0, (9, 13)).astype(np.float32)
    got = fusion.median_filter4(d)
    H, W = d.shape
    for y in range(H):
        for x in range(W):
            vals = sorted(float(d[yy, xx]) for yy in range(y - 1, y + 3) for xx in range(x - 1, x + 3)
                          if 0 <= yy < H and 0 <= xx < W)
            n = len(vals)
            want = vals[n // 2] if n % 2 else 0.5 * (vals[n // 2 - 1] + vals[n // 2])
            assert got[y, x] == np.float32(want), (x, y)


def test_median_constant_spike_ramp():
    c = np.full((8, 10), 3.25, np.float32)
    assert np.array_equal(fusion.median_filter4(c), c)
    s = c.copy()
    s[4, 5] = 5.9
    assert np.array_equal(fusion.median_filter4(s), c)
    x = np.arange(12, dtype=np.float64)
    ramp = np.tile(2.0 + 0.125 * x, (7, 1)).astype(np.float32)
    got = fusion.median_filter4(ramp)
    # interior columns: the window holds columns x-1..x+2 four times each; the middle pair is x, x+1
    np.testing.assert_array_equal(got[:, 1:10], np.tile(2.0 + 0.125 * (x[1:10] + 0.5), (7, 1)).astype(np.float32))


def test_fusion_of_one_plane_world_lies_on_the_plane():
    import scenegen

    sc = scenegen.make_scene(96, 64, 4, 30.0, 0, 5, supersample=2, all_views=True)
    P, N, O = fusion.fuse(sc.cams, sc.depth_views, sc.normal_views)
    assert len(P) > 0.9 * 96 * 64
    np.testing.assert_allclose(P[:, 2], scenegen.BACKGROUND_Z, atol=1e-5)
    np.testing.assert_allclose(N, np.tile([0.0, 0.0, -1.0], (len(N), 1)), atol=1e-6)
    assert np.all(O[:, 2] >= fusion.F_CON)


class _Cam:
    def __init__(self, K, R, t, w, h):
        self.K, self.R, self.t, self.width, self.height = K, R, np.asarray(t, float), w, h


def _two_views(z0=4.0, delta=0.0, rot1_deg=0.0, W=40, H=24):
    f, B = 100.0, 0.52  # f B / z0 = 13 px
    K = np.array([[f, 0, (W - 1) / 2], [0, f, (H - 1) / 2], [0, 0, 1.0]])
    cams = [_Cam(K, np.eye(3), [0, 0, 0], W, H), _Cam(K, np.eye(3), [-B, 0, 0], W, H)]
    n0 = np.tile([0.0, 0.0, -1.0], (H, W, 1))
    a = math.radians(rot1_deg)
    n1 = np.tile([math.sin(a), 0.0, -math.cos(a)], (H, W, 1))
    d = [np.full((H, W), z0), np.full((H, W), z0 + delta)]
    return cams, d, [n0, n1], f * B


def _delta_for(disp, z0, fB):
    # fB (1/z0 - 1/(z0 + delta)) = disp
    return 1.0 / (1.0 / z0 - disp / fB) - z0


@pytest.mark.parametrize("scale,fused", [(0.98, True), (1.02, False)])
def test_disparity_threshold_closed_form(scale, fused):
    z0 = 4.0
    cams, d, n, fB = _two_views(z0)
    delta = _delta_for(fusion.F_EPS * scale, z0, fB)
    cams, d, n, fB = _two_views(z0, delta)
    P, N, O = fusion.fuse(cams, d, n, f_con=1)
    from0 = O[O[:, 0] == 0]
    W, H = 40, 24
    if fused:
        assert len(from0) == (W - 13) * H
        assert set((from0[:, 1] % W).tolist()) == set(range(13, W))
    else:
        assert len(from0) == 0


@pytest.mark.parametrize("deg,fused", [(29.0, True), (31.0, False)])
def test_normal_threshold(deg, fused):
    cams, d, n, _ = _two_views(rot1_deg=deg)
    _, _, O = fusion.fuse(cams, d, n, f_con=1)
    assert (np.sum(O[:, 0] == 0) > 0) == fused


def test_fcon_zero_and_own_back_projection():
    z0 = 4.0
    cams, d, n, fB = _two_views(z0, delta=1.0)  # far beyond f_eps: no witnesses
    P, N, O = fusion.fuse(cams, d, n, f_con=0)
    W, H = 40, 24
    assert len(P) == 2 * W * H and np.all(O[:, 2] == 0)
    ys, xs = np.divmod(O[O[:, 0] == 0, 1], W)
    np.testing.assert_allclose(P[O[:, 0] == 0], fusion.back_project(cams[0], xs, ys, np.full(len(xs), z0)),
                               atol=1e-12)
    # back-projection: (x - cx) z / f, (y - cy) z / f, z
    np.testing.assert_allclose(P[0], [(0 - 19.5) * z0 / 100.0, (0 - 11.5) * z0 / 100.0, z0], atol=1e-12)


def test_identical_cameras_consume_the_second_view():
    cams, d, n, _ = _two_views()
    cams[1] = cams[0]
    P, N, O = fusion.fuse(cams, [d[0], d[0].copy()], [n[0], n[0].copy()], f_con=1)
    assert np.all(O[:, 0] == 0) and len(P) == 40 * 24


def test_pixels_without_depth():
    cams, d, n, _ = _two_views()
    d0 = d[0].copy()
    d0[5, 20] = 0.0
    d0[6, 20] = np.nan
    d1 = d[1].copy()
    d1[7, 20 - 13] = -1.0  # the witness of view 0's pixel (20, 7)
    P, N, O = fusion.fuse(cams, [d0, d1], n, f_con=1)
    from0 = set(O[O[:, 0] == 0, 1].tolist())
    for y in (5, 6, 7):
        assert y * 40 + 20 not in from0
    assert 8 * 40 + 20 in from0


def test_vectorised_fusion_equals_the_per_pixel_definition():
    """View 0 (nothing consumed yet) of a rendered scene with noisy depths: both formulations agree."""
    import scenegen

    sc = scenegen.make_scene(48, 32, 3, 30.0, 3, 2, supersample=2, all_views=True)
    rng = np.random.default_rng(1)
    depths = [d * (1 + rng.normal(scale=2e-3, size=d.shape)) for d in sc.depth_views]
    P, N, O = fusion.fuse(sc.cams, depths, sc.normal_views)
    first = {int(o[1]): k for k, o in enumerate(O) if o[0] == 0}
    emitted = 0
    for y in range(32):
        for x in range(48):
            r = fusion.fuse_pixel(sc.cams, depths, sc.normal_views, 0, x, y)
            k = first.get(y * 48 + x)
            assert r["emitted"] == (k is not None), (x, y)
            if k is not None:
                emitted += 1
                assert r["count"] == O[k, 2]
                np.testing.assert_allclose(P[k], r["point"], atol=1e-12)
                np.testing.assert_allclose(N[k], r["normal"], atol=1e-12)
    assert 0.3 * 48 * 32 < emitted < 48 * 32
