"""Whole-method pins of the oracle on rendered scenes.

* Order independence (Sec. 3.1): a half-pass updated in place gives the same
  result in any pixel order, because every candidate has the other colour.
* Ground truth: after 3 iterations most visible pixels of the tiny
  configuration recover the rendered depth (threshold calibrated once on seeds
  0-2 and frozen).
* Brute force: with a static objective (plain mean over the views) the cost
  PatchMatch reaches is, on most pixels, within a small margin of an
  exhaustive plane sweep's minimum.
"""
import math

import numpy as np
import pytest


def test_half_pass_order_independent(oracle_mod, scene_128x96):
    O = oracle_mod
    V = O.Views.from_scene(scene_128x96)
    P = O.Params(refine=1, seed=9)
    base = O.init(V, P)
    for t, colour in [(0, 0), (3, 1)]:
        a = base.copy()
        b = base.copy()
        raster = np.array([i for i in range(V.W * V.H) if ((i % V.W) + (i // V.W)) % 2 == colour], np.int32)
        shuffled = np.random.default_rng(1).permutation(raster).astype(np.int32)
        O.run_pass(V, P, a, t, colour, order=raster)
        O.run_pass(V, P, b, t, colour, order=shuffled)
        assert np.array_equal(a.plane, b.plane) and np.array_equal(a.cost, b.cost)
        assert np.array_equal(a.S, b.S) and np.array_equal(a.v, b.v)
        # and the other colour is untouched
        other = np.array([((i % V.W) + (i // V.W)) % 2 != colour for i in range(V.W * V.H)]).reshape(V.H, V.W)
        assert np.array_equal(a.plane[other], base.plane[other])


@pytest.mark.parametrize("seed,frac_1pct", [(0, 0.75), (1, 0.70), (2, 0.65)])
def test_recovers_rendered_depth(oracle_mod, seed, frac_1pct):
    import scenegen

    sc = scenegen.config_scene("128x96_n4", seed)
    O = oracle_mod
    V = O.Views.from_scene(sc)
    st = O.run(V, O.Params(refine=1), 3)
    d, n = O.depth_normal(V, st)
    vis = sc.vis_count >= 2
    rel = np.abs(d - sc.depth_gt) / sc.depth_gt
    assert (rel[vis] < 0.01).mean() >= frac_1pct
    # the kept planes face the camera and have depths inside the range
    assert np.all(d >= 2.0 - 1e-9) and np.all(d <= 6.0 + 1e-9)
    np.testing.assert_allclose(np.linalg.norm(n, axis=-1), 1.0, atol=1e-9)


def _fib_hemisphere(n):
    i = np.arange(n) + 0.5
    z = -(i / n)  # normals facing the camera: n_z < 0
    phi = math.pi * (1 + 5 ** 0.5) * i
    r = np.sqrt(1 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], -1)


def test_patchmatch_reaches_plane_sweep_minimum(oracle_mod):
    import scenegen

    sc = scenegen.make_scene(40, 30, 2, 15.0, 2, seed=4, supersample=4)
    O = oracle_mod
    V = O.Views.from_scene(sc)
    P = O.Params(refine=1, view_mode=1)
    st = O.run(V, P, 6)
    Kinv = np.linalg.inv(sc.cams[0].K)
    depths = np.linspace(2.0, 6.0, 48)
    normals = _fib_hemisphere(24)
    rng = np.random.default_rng(0)
    gaps = []
    near_gt = 0
    pix = [(int(rng.integers(6, 34)), int(rng.integers(6, 24))) for _ in range(40)]
    for x, y in pix:
        r = Kinv @ np.array([x, y, 1.0])
        best = math.inf
        best_d = None
        for n in normals:
            for d in depths:
                pl = np.r_[n, -d * (n @ r)]
                c = 0.5 * (O.matching_cost(V, P, x, y, pl, 0) + O.matching_cost(V, P, x, y, pl, 1))
                if c < best:
                    best, best_d = c, d
        ng = sc.normal_gt[y, x].astype(float)
        gt = np.r_[ng, -float(sc.depth_gt[y, x]) * (ng @ r)]
        best = min(best, 0.5 * (O.matching_cost(V, P, x, y, gt, 0) + O.matching_cost(V, P, x, y, gt, 1)))
        gaps.append(st.cost[y, x] - best)
        near_gt += abs(best_d - sc.depth_gt[y, x]) < 0.15
    gaps = np.array(gaps)
    # local search: most pixels reach the sweep minimum (or beat its discretisation); a few stay in
    # local minima on an image this small (calibrated once: 90 % within 0.02 at 6 iterations)
    assert (gaps <= 0.02).mean() >= 0.85
    assert np.median(gaps) <= 0.005
    assert near_gt >= 0.6 * len(pix)
