"""Pins of the oracle's plane-induced warp and of its matching cost (Sec. 3.3, Eq. 8).

* The warp (ray-plane intersection, then projection) must agree with the
  closed-form plane-induced homography K_j (R - t n^T / d) K_ref^-1 built from
  the relative pose, for random cameras and planes, and with the renderer:
  reference pixels seen by a source land on the same intensity there.
* The cost reduces to library routines: with uniform weights it is
  1 - numpy.corrcoef; with two weight levels fixed by the paper's sigma_I it is
  the weighted correlation of numpy.cov(aweights=...).
* Invariances: an affine source with positive gain costs 0, negative gain 2.
* Exact special case: a fronto-parallel plane seen by a source translated along
  x with integer disparity f B / Z costs 0 at the true plane.
"""
import math
from types import SimpleNamespace

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st
from scipy.ndimage import map_coordinates


def cam(K, R, t, W, H):
    return SimpleNamespace(K=np.asarray(K, float), R=np.asarray(R, float), t=np.asarray(t, float), width=W, height=H)


def rand_rot(rng, scale=0.3):
    a = rng.normal(size=3) * scale
    th = np.linalg.norm(a)
    k = a / th
    Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * Kx + (1 - math.cos(th)) * Kx @ Kx


def test_warp_matches_closed_form_homography(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(3)
    W, H = 64, 48
    for trial in range(40):
        Kr = np.array([[rng.uniform(40, 80), rng.uniform(-1, 1), rng.uniform(20, 40)],
                       [0, rng.uniform(40, 80), rng.uniform(15, 30)], [0, 0, 1]])
        Ks = np.array([[rng.uniform(40, 80), 0, rng.uniform(20, 40)], [0, rng.uniform(40, 80), rng.uniform(15, 30)],
                       [0, 0, 1]])
        Rr, Rs = rand_rot(rng), rand_rot(rng)
        tr, ts = rng.normal(size=3) * 0.3, rng.normal(size=3) * 0.3
        img = np.zeros((H, W), np.float32)
        V = O.Views([img, img], [cam(Kr, Rr, tr, W, H), cam(Ks, Rs, ts, W, H)])
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        n[2] = -abs(n[2]) - 0.5
        n /= np.linalg.norm(n)
        dp = rng.uniform(2, 5)
        # homography from the relative pose (a different derivation from the oracle's)
        Rrel = Rs @ Rr.T
        trel = ts - Rrel @ tr
        Hm = Ks @ (Rrel - np.outer(trel, n) / dp) @ np.linalg.inv(Kr)
        for _ in range(5):
            x, y = rng.uniform(0, W), rng.uniform(0, H)
            h = Hm @ np.array([x, y, 1.0])
            o = O.project(V, x, y, np.r_[n, dp], 0)
            np.testing.assert_allclose(o[:2] / o[2], h[:2] / h[2], rtol=1e-9, atol=1e-9)


def test_warp_agrees_with_rendered_views(oracle_mod, scene_128x96):
    """Ground-truth planes warp reference pixels onto matching source intensities."""
    O, sc = oracle_mod, scene_128x96
    V = O.Views.from_scene(sc)
    Kinv = np.linalg.inv(sc.cams[0].K)
    rng = np.random.default_rng(0)
    H, W = sc.height, sc.width
    diffs, wrong = [], []
    for _ in range(300):
        x, y = int(rng.integers(8, W - 8)), int(rng.integers(8, H - 8))
        if sc.vis_count[y, x] < sc.meta["n_src"]:
            continue
        n = sc.normal_gt[y, x].astype(float)
        d = float(sc.depth_gt[y, x])
        pl = np.r_[n, -n @ (d * (Kinv @ [x, y, 1.0]))]
        for j in range(sc.meta["n_src"]):
            o = O.project(V, x, y, pl, j)
            u, v = o[0] / o[2], o[1] / o[2]
            diffs.append(abs(map_coordinates(sc.srcs[j].astype(float), [[v], [u]], order=1)[0] - sc.ref[y, x]))
            wrong.append(abs(map_coordinates(sc.srcs[j].astype(float), [[v], [u + 3]], order=1)[0] - sc.ref[y, x]))
    assert len(diffs) > 200
    assert np.median(diffs) < 3.0
    assert np.median(wrong) > 4 * np.median(diffs)


# ------------------------------------------------------------------------------------------
# matching cost
# ------------------------------------------------------------------------------------------

OFFS = [-5, -3, -1, 1, 3, 5]


def identity_pair(oracle_mod, ref, src):
    """Source camera == reference camera: a fronto-parallel plane warps pixels onto themselves."""
    H, W = ref.shape
    K = np.array([[50.0, 0, (W - 1) / 2], [0, 50.0, (H - 1) / 2], [0, 0, 1]])
    c = cam(K, np.eye(3), np.zeros(3), W, H)
    return oracle_mod.Views([ref, src], [c, c]), np.array([0.0, 0.0, -1.0, 4.0])


def window(img, x, y):
    return np.array([img[y + dy, x + dx] for dy in OFFS for dx in OFFS], float)


@settings(max_examples=40, deadline=None)
@given(st.integers(0, 2**32 - 1))
def test_uniform_weights_reduce_to_corrcoef(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    ref = rng.uniform(0, 255, (16, 16)).astype(np.float32)
    src = rng.uniform(0, 255, (16, 16)).astype(np.float32)
    V, pl = identity_pair(oracle_mod, ref, src)
    P = oracle_mod.Params(sigma_color=1e12, sigma_spatial=1e12)
    m = oracle_mod.matching_cost(V, P, 8, 8, pl, 0)
    expect = 1.0 - np.corrcoef(window(ref, 8, 8), window(src, 8, 8))[0, 1]
    assert m == pytest.approx(min(max(expect, 0.0), 2.0), abs=1e-12)


def test_colour_weights_two_levels_match_weighted_cov(oracle_mod):
    """sigma_I = 3 (the paper's value): a sample 36 grey levels from the centre weighs e^-2 (36 / (2 * 3^2))."""
    rng = np.random.default_rng(5)
    ref = np.full((16, 16), 100.0, np.float32)
    far = rng.random((16, 16)) < 0.5
    ref[far] = 136.0
    ref[8, 8] = 100.0
    src = rng.uniform(0, 255, (16, 16)).astype(np.float32)
    V, pl = identity_pair(oracle_mod, ref, src)
    P = oracle_mod.Params(sigma_color=3.0, sigma_spatial=1e12)
    a, b = window(ref, 8, 8), window(src, 8, 8)
    w = np.where(a == 136.0, math.exp(-2.0), 1.0)
    c = np.cov(np.stack([a, b]), aweights=w, bias=True)
    expect = 1.0 - c[0, 1] / math.sqrt(c[0, 0] * c[1, 1])
    assert oracle_mod.matching_cost(V, P, 8, 8, pl, 0) == pytest.approx(expect, abs=1e-12)


def test_spatial_weights_match_weighted_cov(oracle_mod):
    """sigma_x = 1, no colour term: weight exp(-distance / 2) with the Euclidean pixel distance."""
    rng = np.random.default_rng(6)
    ref = rng.uniform(0, 255, (16, 16)).astype(np.float32)
    src = (0.5 * ref + rng.uniform(0, 80, (16, 16))).astype(np.float32)
    V, pl = identity_pair(oracle_mod, ref, src)
    P = oracle_mod.Params(sigma_color=1e12, sigma_spatial=1.0)
    w = np.array([math.exp(-math.hypot(dx, dy) / 2.0) for dy in OFFS for dx in OFFS])
    c = np.cov(np.stack([window(ref, 8, 8), window(src, 8, 8)]), aweights=w, bias=True)
    expect = 1.0 - c[0, 1] / math.sqrt(c[0, 0] * c[1, 1])
    assert oracle_mod.matching_cost(V, P, 8, 8, pl, 0) == pytest.approx(expect, abs=1e-12)


@settings(max_examples=40, deadline=None)
@given(st.integers(0, 2**32 - 1), st.floats(0.05, 20.0), st.floats(-100.0, 100.0))
def test_affine_invariance(oracle_mod, seed, gain, offset):
    rng = np.random.default_rng(seed)
    ref = rng.uniform(0, 255, (16, 16)).astype(np.float64)
    P = oracle_mod.Params()
    for g, expect in ((gain, 0.0), (-gain, 2.0)):
        src = (g * ref + offset).astype(np.float32)
        V, pl = identity_pair(oracle_mod, ref.astype(np.float32), src)
        # ref is cast to float32 for the oracle; rebuild src from the same float32 values
        src = (g * V.images[0].astype(np.float64) + offset).astype(np.float32)
        V, pl = identity_pair(oracle_mod, V.images[0], src)
        assert oracle_mod.matching_cost(V, P, 8, 8, pl, 0) == pytest.approx(expect, abs=2e-6)


@settings(max_examples=60, deadline=None)
@given(st.integers(0, 2**32 - 1), st.floats(1.0, 5.0), st.floats(-0.9, 0.9), st.floats(-0.9, 0.9))
def test_cost_range(oracle_mod, seed, depth, nx, ny):
    rng = np.random.default_rng(seed)
    ref = rng.uniform(0, 255, (24, 24)).astype(np.float32)
    src = rng.uniform(0, 255, (24, 24)).astype(np.float32)
    V, _ = identity_pair(oracle_mod, ref, src)
    n = np.array([nx, ny, -1.0])
    n /= np.linalg.norm(n)
    m = oracle_mod.matching_cost(V, oracle_mod.Params(d_min=0.5, d_max=10), 12, 12, np.r_[n, 4.0 * -n[2]], 0)
    assert 0.0 <= m <= 2.0


def test_degenerate_and_invalid_cost_two(oracle_mod):
    rng = np.random.default_rng(1)
    ref = rng.uniform(0, 255, (16, 16)).astype(np.float32)
    V, pl = identity_pair(oracle_mod, ref, np.full((16, 16), 77.0, np.float32))
    P = oracle_mod.Params()
    assert oracle_mod.matching_cost(V, P, 8, 8, pl, 0) == 2.0  # constant source patch
    V, pl = identity_pair(oracle_mod, ref, ref)
    assert oracle_mod.matching_cost(V, P, 8, 8, pl, 0) == pytest.approx(0.0, abs=1e-12)
    assert oracle_mod.matching_cost(V, oracle_mod.Params(d_min=4.5, d_max=6.0), 8, 8, pl, 0) == 2.0  # depth 4 out
    behind = np.array([0.0, 0.0, 1.0, -4.0])  # same plane, normal facing away: depth still 4
    assert oracle_mod.matching_cost(V, P, 8, 8, behind, 0) == pytest.approx(0.0, abs=1e-12)


def test_integer_disparity_true_plane_costs_zero(oracle_mod):
    """Fronto-parallel plane at Z = 4, source shifted by B = 0.12 with f = 100: disparity exactly 3 px."""
    rng = np.random.default_rng(11)
    W, H, f, Z, B = 64, 40, 100.0, 4.0, 0.12
    K = np.array([[f, 0, (W - 1) / 2], [0, f, (H - 1) / 2], [0, 0, 1]])
    ref = rng.uniform(0, 255, (H, W)).astype(np.float32)
    src = np.zeros_like(ref)
    src[:, :W - 3] = ref[:, 3:] * 1.07 + 5.0  # pixel u in the source shows the reference pixel u + 3
    V = oracle_mod.Views([ref, src], [cam(K, np.eye(3), np.zeros(3), W, H), cam(K, np.eye(3), [-B, 0, 0], W, H)])
    pl = np.array([0.0, 0.0, -1.0, Z])
    P = oracle_mod.Params()
    for x, y in [(20, 10), (30, 20), (40, 30), (12, 15)]:
        o = oracle_mod.project(V, x, y, pl, 0)
        assert o[0] / o[2] == pytest.approx(x - 3, abs=1e-12)
        assert oracle_mod.matching_cost(V, P, x, y, pl, 0) == pytest.approx(0.0, abs=1e-9)
        wrong = np.array([0.0, 0.0, -1.0, Z * 1.2])
        assert oracle_mod.matching_cost(V, P, x, y, wrong, 0) > 0.3


def test_squared_bilateral_weights_match_weighted_cov(oracle_mod):
    """The squared form: sigma_I = 3 and a 6-level step weigh e^-2 (36 / 18); sigma_x = 1 weighs
    exp(-(dx^2 + dy^2) / 2)."""
    rng = np.random.default_rng(8)
    ref = np.full((16, 16), 100.0, np.float32)
    far = rng.random((16, 16)) < 0.5
    ref[far] = 106.0
    ref[8, 8] = 100.0
    src = rng.uniform(0, 255, (16, 16)).astype(np.float32)
    V, pl = identity_pair(oracle_mod, ref, src)
    a, b = window(ref, 8, 8), window(src, 8, 8)
    P = oracle_mod.Params(sigma_color=3.0, sigma_spatial=1e12, bilateral_sq=1)
    w = np.where(a == 106.0, math.exp(-2.0), 1.0)
    c = np.cov(np.stack([a, b]), aweights=w, bias=True)
    assert oracle_mod.matching_cost(V, P, 8, 8, pl, 0) == pytest.approx(1.0 - c[0, 1] / math.sqrt(c[0, 0] * c[1, 1]),
                                                                       abs=1e-12)
    ref2 = rng.uniform(0, 255, (16, 16)).astype(np.float32)
    V, pl = identity_pair(oracle_mod, ref2, src)
    P = oracle_mod.Params(sigma_color=1e12, sigma_spatial=1.0, bilateral_sq=1)
    w = np.array([math.exp(-(dx * dx + dy * dy) / 2.0) for dy in OFFS for dx in OFFS])
    c = np.cov(np.stack([window(ref2, 8, 8), b]), aweights=w, bias=True)
    assert oracle_mod.matching_cost(V, P, 8, 8, pl, 0) == pytest.approx(1.0 - c[0, 1] / math.sqrt(c[0, 0] * c[1, 1]),
                                                                       abs=1e-12)


def test_short_predicate_matches_oracle_early_exits():
    """The predicate used to check the library's short-evaluation counters marks exactly the evaluations that
    the oracle ends with cost 2 on its range and visibility tests (R3); on random initial planes of the
    128x96 scene every other evaluation reaches the NCC (none here has a flat window)."""
    import oracle as O
    import scenegen
    from short_predicate import short_mask
    sc = scenegen.config_scene("128x96_n4", seed=0)
    V = O.Views(sc.images, sc.cams)
    P = O.Params(seed=5, refine=0)
    st = O.init(V, P)
    ys, xs = np.mgrid[0:sc.height, 0:sc.width]
    xy = np.c_[xs.ravel(), ys.ravel()]
    pl = st.plane.reshape(-1, 4)
    m = short_mask(sc, xy, pl, P.d_min, P.d_max)
    assert 0.02 < m.mean() < 0.3
    idx = np.random.default_rng(0).choice(len(xy), 400, replace=False)
    for i in idx:
        for j in range(len(sc.srcs)):
            c = O.matching_cost(V, P, int(xy[i, 0]), int(xy[i, 1]), pl[i], j)
            assert (c == 2.0) == bool(m[i, j]), (xy[i], j, c)


def test_sample_f32_probe_only_rounds_positions_and_samples(oracle_mod, scene_128x96):
    """The conditioning probe (sample_f32 = 1) changes nothing but the precision of the samples' source
    positions (relative to the centre's texel) and interpolated values: where every sample lands on a texel
    (integer disparity) both are float32 numbers already and the cost is unchanged; elsewhere it moves by no
    more than float32 rounding of them can move a correlation (~1e-5 on the rendered scene), and it does move."""
    rng = np.random.default_rng(11)
    W, H, f, Z, B = 64, 40, 100.0, 4.0, 0.12
    K = np.array([[f, 0, (W - 1) / 2], [0, f, (H - 1) / 2], [0, 0, 1]])
    ref = rng.uniform(0, 255, (H, W)).astype(np.float32)
    src = np.zeros_like(ref)
    src[:, :W - 3] = ref[:, 3:] * 1.07 + 5.0
    V = oracle_mod.Views([ref, src], [cam(K, np.eye(3), np.zeros(3), W, H), cam(K, np.eye(3), [-B, 0, 0], W, H)])
    pl = np.array([0.0, 0.0, -1.0, Z * 1.3])  # disparity 3 / 1.3: samples between texels
    exact = np.array([0.0, 0.0, -1.0, Z / 2.0])  # disparity 6: samples on texels
    P0, P1 = oracle_mod.Params(), oracle_mod.Params(sample_f32=1)
    for x, y in [(20, 10), (30, 20), (40, 30)]:
        # (the warped positions are texel centres up to double rounding)
        assert oracle_mod.matching_cost(V, P1, x, y, exact, 0) == pytest.approx(
            oracle_mod.matching_cost(V, P0, x, y, exact, 0), abs=1e-12)
    V = oracle_mod.Views.from_scene(scene_128x96)
    diffs = []
    for _ in range(300):
        x, y = int(rng.integers(0, V.W)), int(rng.integers(0, V.H))
        plane = oracle_mod.random_plane(V, P0, x, y, 5, 0)
        for j in range(V.n_src):
            a, b = oracle_mod.matching_cost(V, P0, x, y, plane, j), oracle_mod.matching_cost(V, P1, x, y, plane, j)
            if a < 2.0:
                diffs.append(abs(a - b))
    diffs = np.array(diffs)
    assert diffs.max() <= 1e-4 and diffs.max() > 0.0


def test_sample_f32_probe_level_two_rounds_the_moments(oracle_mod, scene_128x96):
    """Level 2 of the probe also forms the weights' sums and the NCC's moments in float32.  On samples that
    land on texels (nothing for level 1 to round) it moves the cost by float32 rounding of the moments only
    (< 1e-5, and it does move); a constant source window stays at cost 2 (zero variance is exact in float32
    as well); on the rendered scene it stays within 1e-4 of level 1 and of the exact cost."""
    O = oracle_mod
    rng = np.random.default_rng(12)
    W, H, f, Z, B = 64, 40, 100.0, 4.0, 0.12
    K = np.array([[f, 0, (W - 1) / 2], [0, f, (H - 1) / 2], [0, 0, 1]])
    ref = rng.uniform(0, 255, (H, W)).astype(np.float32)
    src = np.zeros_like(ref)
    src[:, :W - 6] = ref[:, 6:] * 0.93 + 11.0
    V = O.Views([ref, src], [cam(K, np.eye(3), np.zeros(3), W, H), cam(K, np.eye(3), [-B, 0, 0], W, H)])
    exact = np.array([0.0, 0.0, -1.0, Z / 2.0])  # disparity 6: samples on texels
    P0, P1, P2 = O.Params(), O.Params(sample_f32=1), O.Params(sample_f32=2)
    moved = []
    for x, y in [(20, 10), (30, 20), (40, 30), (25, 15)]:
        c0, c1, c2 = (O.matching_cost(V, P, x, y, exact, 0) for P in (P0, P1, P2))
        assert c1 == pytest.approx(c0, abs=1e-12)
        assert abs(c2 - c0) < 1e-5
        moved.append(abs(c2 - c0))
    assert max(moved) > 0.0
    flat = O.Views([ref, np.full_like(ref, 77.0)], [cam(K, np.eye(3), np.zeros(3), W, H),
                                                   cam(K, np.eye(3), [-B, 0, 0], W, H)])
    assert O.matching_cost(flat, P2, 30, 20, exact, 0) == 2.0
    V = O.Views.from_scene(scene_128x96)
    d1, d0 = [], []
    for _ in range(200):
        x, y = int(rng.integers(0, V.W)), int(rng.integers(0, V.H))
        plane = O.random_plane(V, P0, x, y, 5, 0)
        for j in range(V.n_src):
            a, b, c = (O.matching_cost(V, P, x, y, plane, j) for P in (P0, P1, P2))
            if a < 2.0 and b < 2.0 and c < 2.0:
                d1.append(abs(c - b))
                d0.append(abs(c - a))
    assert max(d1) <= 1e-4 and max(d0) <= 1e-4 and max(d1) > 0.0


def test_sample_f32_probe_level_three_is_the_first_order_worst_case(oracle_mod, scene_128x96):
    """Level 3 moves every sample value by the first-order bound of rounding its position and value to float32,
    in the direction that moves the cost towards 1: the cost moves towards 1 (never away, never past it), by
    no more than 1e-4 with the printed weights, and by at least what the actual rounding (level 1) moves it in
    nearly every case -- a worst case bounds the actual rounding to first order."""
    O = oracle_mod
    V = O.Views.from_scene(scene_128x96)
    P0, P1, P3 = O.Params(), O.Params(sample_f32=1), O.Params(sample_f32=3)
    rng = np.random.default_rng(13)
    d1, d3 = [], []
    for _ in range(200):
        x, y = int(rng.integers(0, V.W)), int(rng.integers(0, V.H))
        plane = O.random_plane(V, P0, x, y, 5, 0)
        for j in range(V.n_src):
            c0, c1, c3 = (O.matching_cost(V, P, x, y, plane, j) for P in (P0, P1, P3))
            if not (c0 < 2.0 and c1 < 2.0 and c3 < 2.0):
                continue
            if c0 >= 1.0:
                assert c3 <= c0 + 1e-15
            else:
                assert c3 >= c0 - 1e-15
            assert abs(c3 - c0) <= 1e-4
            d1.append(abs(c1 - c0))
            d3.append(abs(c3 - c0))
    d1, d3 = np.array(d1), np.array(d3)
    assert len(d3) > 500 and d3.max() > 0.0
    assert np.mean(d3 >= d1) >= 0.9


def test_cost_noise_probe_is_bounded_deterministic_and_centred(oracle_mod, scene_128x96):
    """The second conditioning probe (cost_noise = e) moves every scored cost by a fixed offset in
    [-e/2, e/2) that depends only on (pixel, view, plane); cost 2 and the clamp are untouched."""
    O = oracle_mod
    V = O.Views.from_scene(scene_128x96)
    P0, P1 = O.Params(), O.Params(cost_noise=2e-4)
    rng = np.random.default_rng(3)
    d = []
    for _ in range(300):
        x, y = int(rng.integers(5, V.W - 5)), int(rng.integers(5, V.H - 5))
        plane = O.random_plane(V, P0, x, y, 7, 0)
        for j in range(V.n_src):
            a = O.matching_cost(V, P0, x, y, plane, j)
            b = O.matching_cost(V, P1, x, y, plane, j)
            assert b == O.matching_cost(V, P1, x, y, plane, j)
            if a == 2.0:
                assert b == 2.0
            elif 1e-4 < a < 2.0 - 1e-4:
                d.append(b - a)
    d = np.array(d)
    assert len(d) > 200 and np.all(np.abs(d) <= 1e-4)
    assert abs(d.mean()) < 1e-5 and d.std() > 4e-5  # uniform on +-1e-4: std 5.8e-5
