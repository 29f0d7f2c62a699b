"""Pins of the oracle's random initialisation and refinement step.

The paper draws random planes (PatchMatch initialisation, Sec. 2 and 3) and
ends every pixel update with a refinement whose details it defers to an
earlier system (Sec. 3.3).  The readings R1 and R13 fix them; these tests pin
the oracle to what those readings state, through properties that any correct
implementation has and that a plausible slip breaks:

* random planes: depth uniform on [d_min, d_max], normal uniform on the sphere
  and turned to face the reference camera (Kolmogorov-Smirnov tests, plus exact
  range and unit-length checks);
* initial cost (R1): the mean of the min(k, N) lowest per-view costs of the
  pixel's random plane, recomputed here with a numpy sort;
* refinement candidates (R13): three for t < 3 and six from t = 3; the
  perturbed depth lies within 2^-(t+2) (d_max - d_min) of the current depth and
  inside the range (clamped at its ends), and that bound is reached; the
  perturbed normal differs from the current one by at most 2 * 2^-(t+2) per
  component before normalisation, and that bound is reached too; shared draws
  are shared ((d_prt, n_prt) reuses both); random depths are uniform on the range;
* scoring and acceptance: a candidate costs the weighted mean of its costs on
  the views with positive weight (Eq. 7 with the pixel's weights); candidates
  are accepted in order only when strictly lower, so a tie keeps the current
  plane (checked on a view that sees nothing, where every cost is 2).
"""
import numpy as np
import pytest
from scipy import stats

D_MIN, D_MAX = 2.0, 6.0


def depth_of(Kinv, x, y, pl):
    r = Kinv @ np.array([x, y, 1.0])
    return -pl[3] / (pl[:3] @ r), r


def cheb_residual(a, b):
    """min over real s of max_i |s a_i - b_i| (a convex piecewise-linear function of s: its minimum
    lies where two of the lines meet, or where one crosses zero)."""
    cands = [b[i] / a[i] for i in range(3) if a[i] != 0.0]
    for i in range(3):
        for k in range(i + 1, 3):
            for sg in (1.0, -1.0):
                den = a[i] - sg * a[k]
                if den != 0.0:
                    cands.append((b[i] - sg * b[k]) / den)
    return min(np.max(np.abs(s * a - b)) for s in cands)


@pytest.fixture(scope="module")
def views(oracle_mod, scene_128x96):
    return oracle_mod.Views.from_scene(scene_128x96)


def test_random_planes_are_uniform_and_face_the_camera(oracle_mod, views):
    O, V = oracle_mod, views
    st = O.init(V, O.Params(seed=21))
    Kinv = np.linalg.inv(np.array(V.c.Kref[:]).reshape(3, 3))
    ys, xs = np.mgrid[0:V.H, 0:V.W]
    r = np.einsum("ij,hwj->hwi", Kinv, np.stack([xs, ys, np.ones_like(xs)], -1).astype(np.float64))
    n = st.plane[..., :3]
    nr = np.einsum("hwi,hwi->hw", n, r)
    depth = -st.plane[..., 3] / nr
    np.testing.assert_allclose(np.linalg.norm(n, axis=-1), 1.0, atol=1e-12)
    assert np.all(nr < 0)
    assert np.all((depth >= D_MIN - 1e-12) & (depth <= D_MAX + 1e-12))
    # depth ~ U[d_min, d_max]; the cosine between a uniform direction and any fixed axis is U[-1, 1],
    # and turning it to face the camera makes it U[-1, 0]
    assert stats.kstest(depth.ravel(), stats.uniform(D_MIN, D_MAX - D_MIN).cdf).pvalue > 1e-4
    cos = (nr / np.linalg.norm(r, axis=-1)).ravel()
    assert stats.kstest(cos, stats.uniform(-1.0, 1.0).cdf).pvalue > 1e-4
    # a uniform direction turned to face r is uniform on that hemisphere: its azimuth about r, in a
    # frame (e1, e2) perpendicular to r, is uniform on [0, 2 pi)
    rh = r / np.linalg.norm(r, axis=-1, keepdims=True)
    e1 = np.array([1.0, 0.0, 0.0]) - rh[..., :1] * rh
    e1 /= np.linalg.norm(e1, axis=-1, keepdims=True)
    e2 = np.cross(rh, e1)
    az = np.arctan2(np.einsum("hwi,hwi->hw", n, e2), np.einsum("hwi,hwi->hw", n, e1)).ravel() % (2 * np.pi)
    assert stats.kstest(az, stats.uniform(0.0, 2 * np.pi).cdf).pvalue > 1e-4
    # the generator is keyed by the seed: another seed gives other planes
    assert not np.array_equal(st.plane, O.init(V, O.Params(seed=22)).plane)


@pytest.mark.parametrize("k,n_src", [(4, 4), (2, 4), (1, 4), (4, 2), (3, 3)])
def test_initial_cost_is_mean_of_k_lowest(oracle_mod, scene_128x96, k, n_src):
    O, sc = oracle_mod, scene_128x96
    V = O.Views(sc.images[: n_src + 1], sc.cams[: n_src + 1])
    P = O.Params(seed=5, k=k)
    st = O.init(V, P)
    assert np.all(st.S == 0) and np.all(st.v == -1)
    rng = np.random.default_rng(k * 10 + n_src)
    kk = min(k, n_src)
    for _ in range(150):
        x, y = int(rng.integers(0, V.W)), int(rng.integers(0, V.H))
        pl = st.plane[y, x]
        assert np.array_equal(pl, O.random_plane(V, P, x, y, 0, 0))
        c = np.array([O.matching_cost(V, P, x, y, pl, j) for j in range(n_src)])
        assert st.cost[y, x] == pytest.approx(np.sort(c)[:kk].mean(), rel=1e-12, abs=1e-15)


def _refined_pass(O, sc, t, seed):
    V = O.Views.from_scene(sc)
    P = O.Params(refine=1, seed=seed)
    st = O.init(V, P)
    O.run_pass(V, P, st, 0, 0)  # a realistic state: view sets and best views from an earlier pass
    O.run_pass(V, P, st, 0, 1)
    pre = st.copy()
    order = np.array([i for i in range(V.W * V.H) if ((i % V.W) + (i // V.W)) % 2 == 0], np.int32)
    dg = O.run_pass(V, P, st, t, 0, order=order, diag=True)
    return V, P, pre, st, order, dg


def _current_plane(d, pre, x, y, odx, ody):
    """The hypothesis that refinement starts from: the argmin of the unified costs (own row first on
    ties, then region order)."""
    best = None
    for r in (8, 0, 1, 2, 3, 4, 5, 6, 7):
        if d.row_valid[r] and (best is None or d.mfinal[r] < d.mfinal[best]):
            best = r
    if best == 8:
        return best, pre.plane[y, x].copy()
    ci = d.cand_index[best]
    return best, pre.plane[y + ody[ci], x + odx[ci]].copy()


@pytest.mark.parametrize("t", [0, 1, 2, 3, 4])
def test_refinement_candidates(oracle_mod, scene_128x96, t):
    O = oracle_mod
    V, P, pre, st, order, dg = _refined_pass(O, scene_128x96, t, seed=7 + t)
    odx, ody, _ = O.acp_offsets()
    Kinv = np.linalg.inv(np.array(V.c.Kref[:]).reshape(3, 3))
    rho = 2.0 ** -(t + 2)
    span = rho * (D_MAX - D_MIN)
    N = V.n_src
    dratio, nratio, drnd, nrnd_cos, pairs = [], [], [], [], []
    n_checked_costs = 0
    for q, idx in enumerate(order):
        d = dg[q]
        x, y = int(idx % V.W), int(idx // V.W)
        assert d.n_cand == (3 if t < 3 else 6)
        best, cur = _current_plane(d, pre, x, y, odx, ody)
        d_cur, r = depth_of(Kinv, x, y, cur)
        n_face = cur[:3] if cur[:3] @ r <= 0 else -cur[:3]
        cand = [np.array(d.cand_plane[c][:4]) for c in range(d.n_cand)]
        dep = [depth_of(Kinv, x, y, c)[0] for c in cand]
        for c in cand:
            np.testing.assert_allclose(np.linalg.norm(c[:3]), 1.0, atol=1e-12)
            assert c[:3] @ r < 0
        # (d_prt, n): the current normal, a depth within the perturbation range, clamped to [d_min, d_max]
        np.testing.assert_allclose(cand[0][:3], n_face, atol=1e-15)
        assert D_MIN - 1e-12 <= dep[0] <= D_MAX + 1e-12
        if abs(dep[0] - D_MIN) < 1e-12:
            assert d_cur - span <= D_MIN + 1e-9
        elif abs(dep[0] - D_MAX) < 1e-12:
            assert d_cur + span >= D_MAX - 1e-9
        else:
            assert abs(dep[0] - d_cur) <= span * (1 + 1e-9)
        unclamped = D_MIN + span < d_cur < D_MAX - span  # the draw is seen whole
        if unclamped:
            dratio.append((dep[0] - d_cur) / span)
        # (d, n_prt): the current depth, the normal moved by at most 2 rho per component before
        # normalisation (either orientation, as the plane is turned to face the camera)
        assert dep[1] == pytest.approx(d_cur, rel=1e-9)
        nratio.append(cheb_residual(cand[1][:3], cur[:3]) / (2.0 * rho))
        # (d_prt, n_prt) reuses both draws
        assert dep[2] == pytest.approx(dep[0], rel=1e-9)
        np.testing.assert_allclose(cand[2][:3], cand[1][:3], atol=1e-12)
        if t >= 3:
            # (d_rnd, n), (d, n_rnd), (d_rnd, n_rnd)
            np.testing.assert_allclose(cand[3][:3], n_face, atol=1e-15)
            assert D_MIN - 1e-12 <= dep[3] <= D_MAX + 1e-12
            assert dep[4] == pytest.approx(d_cur, rel=1e-9)
            assert dep[5] == pytest.approx(dep[3], rel=1e-9)
            np.testing.assert_allclose(cand[5][:3], cand[4][:3], atol=1e-12)
            drnd.append(dep[3])
            nrnd_cos.append(cand[4][:3] @ r / np.linalg.norm(r))
            pairs.append((dep[0] - d_cur) / span if unclamped else np.nan)
        # scoring: Eq. 7 with the pixel's weights, on the views that carry weight
        w = np.array(d.w[:N])
        if n_checked_costs < 40 and q % 7 == 0:
            n_checked_costs += 1
            for c in range(d.n_cand):
                m = np.array([O.matching_cost(V, P, x, y, cand[c], j) if w[j] > 0 else 0.0 for j in range(N)])
                assert d.cand_cost[c] == pytest.approx((w * m).sum() / w.sum(), rel=1e-12, abs=1e-15)
        # acceptance: in candidate order, strictly lower only
        cost, chosen, plane = d.mfinal[best], best, cur
        for c in range(d.n_cand):
            if d.cand_cost[c] < cost:
                cost, chosen, plane = d.cand_cost[c], 9 + c, cand[c]
        assert d.chosen == chosen
        assert st.cost[y, x] == cost
        assert np.array_equal(st.plane[y, x], plane)
    dratio, nratio = np.array(dratio), np.array(nratio)
    # the bounds hold, and the draws reach them (a range off by a power of two fails one side)
    assert np.all(np.abs(dratio) <= 1.0 + 1e-9) and np.abs(dratio).max() >= 0.97
    assert stats.kstest(dratio, stats.uniform(-1.0, 2.0).cdf).pvalue > 1e-4
    assert np.all(nratio <= 1.0 + 1e-9) and nratio.max() >= 0.75
    if t >= 3:
        assert stats.kstest(drnd, stats.uniform(D_MIN, D_MAX - D_MIN).cdf).pvalue > 1e-4
        assert stats.kstest(nrnd_cos, stats.uniform(-1.0, 1.0).cdf).pvalue > 1e-4
        # the random depth is a fresh draw, independent of the perturbation's
        pairs, drnd = np.array(pairs), np.array(drnd)
        ok = np.isfinite(pairs)
        assert abs(np.corrcoef(pairs[ok], drnd[ok])[0, 1]) < 0.1


def test_refinement_keeps_the_plane_on_exact_ties(oracle_mod, scene_128x96):
    """A source that sees nothing (turned away from the scene): every cost is 2, the joint selection
    is empty and falls back to uniform weights, every row and candidate costs exactly 2, so the own
    plane stays (ties keep it) and no candidate is accepted (strictly lower only)."""
    import dataclasses

    O, sc = oracle_mod, scene_128x96
    # the reference camera is the world frame; a source at its centre looking down -z sees every point
    # in front of the reference behind itself
    assert np.allclose(sc.cams[0].R, np.eye(3)) and np.allclose(sc.cams[0].t, 0.0)
    away = dataclasses.replace(sc.cams[1], R=np.diag([-1.0, 1.0, -1.0]), t=np.zeros(3))
    V = O.Views(sc.images[:2], [sc.cams[0], away])
    for t in (1, 3):
        P = O.Params(refine=1, seed=3)
        st = O.init(V, P)
        assert np.all(st.cost == 2.0)
        pre = st.copy()
        order = np.array([i for i in range(V.W * V.H) if ((i % V.W) + (i // V.W)) % 2 == 1], np.int32)
        dg = O.run_pass(V, P, st, t, 1, order=order, diag=True)
        for d in dg:
            assert d.n_cand == (3 if t < 3 else 6)
            assert all(d.cand_cost[c] == 2.0 for c in range(d.n_cand))
            assert d.chosen == 8 and d.S == 0 and d.v == -1
        assert np.array_equal(st.plane, pre.plane)
        assert np.all(st.cost == 2.0)


def test_per_pixel_hypotheses_pass_through_their_point(oracle_mod, scene_128x96):
    """Initial hypotheses from per-pixel estimates (cells of one pixel): a confident, in-range pixel's plane
    passes through the point at its depth on its own ray with its normal (unit, facing the camera); the
    others keep the random plane; the cost is the initial cost of that plane."""
    from oracle import proposal

    O, sc = oracle_mod, scene_128x96
    V = O.Views.from_scene(sc)
    P = O.Params(seed=4)
    H, W = sc.height, sc.width
    rng = np.random.default_rng(5)
    depth = sc.depth_gt.astype(np.float64) * (1 + rng.uniform(-0.01, 0.01, (H, W)))
    depth[3, 4] = 7.0  # out of range
    depth[5, 6] = np.nan
    normal = sc.normal_gt.astype(np.float64) * rng.choice([-2.0, 0.5], (H, W, 1))  # any length, either sign
    normal[7, 8] = 0.0
    conf = rng.uniform(0, 1, (H, W))
    st, used = proposal.proposal_state(V, P, depth, normal, conf, conf_min=0.5, cell=1)
    Kinv = np.linalg.inv(sc.cams[0].K)
    for y, x in [(3, 4), (5, 6), (7, 8)]:
        assert not used[y, x]
    assert np.array_equal(used, (conf >= 0.5) & used)
    assert 0.4 < used.mean() < 0.6
    for y in range(0, H, 5):
        for x in range(0, W, 3):
            pl = st.plane[y, x]
            if used[y, x]:
                d, r = depth_of(Kinv, x, y, pl)
                assert d == pytest.approx(depth[y, x], rel=1e-12)
                n = normal[y, x] / np.linalg.norm(normal[y, x])
                np.testing.assert_allclose(np.abs(pl[:3] @ n), 1.0, atol=1e-12)
                assert pl[:3] @ r < 0
            else:
                assert np.array_equal(pl, O.random_plane(V, P, x, y, 0, 0))
            c = np.sort([O.matching_cost(V, P, x, y, pl, j) for j in range(V.n_src)])[:4].mean()
            assert st.cost[y, x] == pytest.approx(c, rel=1e-12, abs=1e-15)
