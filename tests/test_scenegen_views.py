"""Invariants of the per-view ground truth of the scene generator (all_views=True), which the fusion pins
and the fusion benchmark use: view 0 equals the reference's ground truth; every view's depth, back-projected
into the world and projected into another camera, lands on that camera's rendered surface wherever the
other camera sees the same point; normals are unit and face their camera."""
import numpy as np


def test_per_view_ground_truth_is_consistent():
    import scenegen

    sc = scenegen.make_scene(64, 48, 3, 30.0, 3, 11, supersample=1, all_views=True)
    assert np.array_equal(sc.depth_views[0], sc.depth_gt)
    assert np.array_equal(sc.normal_views[0], sc.normal_gt)
    H, W = sc.height, sc.width
    ys, xs = np.mgrid[0:H, 0:W]
    for i, ci in enumerate(sc.cams):
        n = sc.normal_views[i].astype(np.float64)
        np.testing.assert_allclose(np.linalg.norm(n, axis=-1), 1.0, atol=1e-6)
        ray = np.stack([xs, ys, np.ones_like(xs)], -1).astype(np.float64) @ np.linalg.inv(ci.K).T
        assert np.all((n * ray).sum(-1) <= 1e-9)  # facing the camera
        X = (ray * sc.depth_views[i][..., None] - ci.t) @ ci.R  # world points, R^T (X_cam - t)
        for j, cj in enumerate(sc.cams):
            if j == i:
                continue
            Xj = X @ cj.R.T + cj.t
            p = Xj @ cj.K.T
            u, v = p[..., 0] / p[..., 2], p[..., 1] / p[..., 2]
            ui, vi = np.floor(u + 0.5).astype(int), np.floor(v + 0.5).astype(int)
            inside = (Xj[..., 2] > 0) & (ui >= 0) & (ui < W) & (vi >= 0) & (vi < H)
            dj = np.where(inside, sc.depth_views[j][np.clip(vi, 0, H - 1), np.clip(ui, 0, W - 1)], np.nan)
            seen = inside & (np.abs(dj - Xj[..., 2]) < 0.05 * Xj[..., 2])
            # most points a camera can see land on its surface (the rest are occluded or at edges)
            assert seen.sum() >= 0.5 * inside.sum()
            # and where they do, within the depth change of half a pixel of the surface
            assert np.median(np.abs(dj - Xj[..., 2])[seen] / Xj[..., 2][seen]) < 2e-3
