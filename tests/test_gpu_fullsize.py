"""GPU parity at the measured sizes, 1920x1280 with 10 sources and 3200x2130 with
20 float16 sources, in the launch configuration bench.py times.

Whole depth maps against whole oracle runs are in test_gpu_fullmap.py (1920x1280
in full; the 3200x2130 recipe at 800x532, as the oracle's whole run at full
size takes minutes).  Here the oracle recomputes sampled pixels of one
half-pass at full size, one by one, from the GPU's pre-pass state (the update of
a pixel only reads its neighbourhood), plus sampled fixed-hypothesis costs;
whole runs are checked through properties that hold at any size.
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


@pytest.fixture(scope="module", params=["1920x1280_n10", "3200x2130_n20"])
def big_scene(request):
    import scenegen

    say("rendering", request.param)
    return request.param, scenegen.config_scene(request.param, 0, device="cuda")


def _ctx(amh, sc, refine, seed=0):
    ctx = amh.Context(refine=refine, seed=seed)
    store = amh.AMH_F16 if sc.srcs[0].dtype == np.float16 else amh.AMH_F32
    ctx.init_views([np.ascontiguousarray(im) for im in sc.images], sc.cams, store_as=store)
    return ctx


def _sample_pixels(W, H, colour, n, rng):
    pts = set()
    while len(pts) < n:
        x, y = int(rng.integers(0, W)), int(rng.integers(0, H))
        if (x + y) % 2 == colour:
            pts.add(y * W + x)
    # image corners and borders of this colour
    for x, y in [(0, 0), (W - 1, H - 1), (1, 0), (0, 1), (W - 2, H - 1), (W - 1, H - 2), (W // 2, 0), (0, H // 2)]:
        if (x + y) % 2 == colour:
            pts.add(y * W + x)
    return np.array(sorted(pts), np.int32)


def test_sampled_half_pass_matches_oracle(amh, oracle_mod, big_scene):
    name, sc = big_scene
    O = oracle_mod
    n = len(sc.srcs)
    cfg_refine = sc.meta["refine"]
    W, H = sc.width, sc.height
    say(f"case sampled pass {name} {W}x{H} n={n}")
    with _ctx(amh, sc, cfg_refine) as ctx:
        ctx.begin(0, list(range(1, n + 1)))
        ctx.init_hypotheses()
        ctx.pass_(0, 0)
        ctx.pass_(0, 1)
        pl0, c0, S0, v0 = ctx.get_state()  # state before the t = 1 red pass
        ctx.pass_(1, 0)
        pl1, c1, S1, v1 = ctx.get_state()
    V = O.Views.from_scene(sc)
    P = O.Params(refine=cfg_refine, seed=0)
    st = O.State.from_arrays(pl0, c0, S0, v0)
    order = _sample_pixels(W, H, 0, 300, np.random.default_rng(3))
    dg = O.run_pass(V, P, st, 1, 0, order=order, delta=1e-5, diag=True)
    bits = np.array([d.robust for d in dg])
    robust = (bits & 29) == 29
    chosen = np.array([d.chosen for d in dg])
    gp = pl1.reshape(-1, 4)[order]
    gc = c1.ravel()[order]
    gS = S1.ravel()[order]
    op = st.plane.reshape(-1, 4)[order]
    oc = st.cost.ravel()[order]
    oS = st.S.ravel()[order]
    exact = np.all(gp == op.astype(np.float32), axis=-1)
    close = np.all(np.abs(gp - op) <= 1e-5 * (1 + np.abs(op)), axis=-1)
    ok_plane = np.where(chosen < 9, exact, close)
    ok = ok_plane & (gS == oS) & (np.abs(gc - oc) <= 1e-4)
    say(f"  robust {robust.mean():.3f}, agree on robust {ok[robust].mean():.4f}, plane agreement {ok_plane.mean():.4f}")
    assert robust.mean() >= 0.5
    assert ok[robust].all()
    assert ok_plane.mean() >= 0.99  # the one-half-pass bar: >= 99 % of all pixels keep the oracle's plane


def test_sampled_fixed_costs_match_oracle(amh, oracle_mod, big_scene):
    name, sc = big_scene
    O = oracle_mod
    n = len(sc.srcs)
    W, H = sc.width, sc.height
    say(f"case sampled fixed costs {name}")
    rng = np.random.default_rng(4)
    Kinv = np.linalg.inv(sc.cams[0].K)
    pix, planes = [], []
    for _ in range(60):
        x, y = int(rng.integers(0, W)), int(rng.integers(0, H))
        nrm = sc.normal_gt[y, x].astype(np.float64)
        d = float(sc.depth_gt[y, x]) * (1 + rng.uniform(-0.01, 0.01))
        planes.append(np.r_[nrm, -d * (nrm @ (Kinv @ [x, y, 1.0]))])
        pix.append((x, y))
    planes = np.array(planes, np.float32)
    with _ctx(amh, sc, 0) as ctx:
        ctx.begin(0, list(range(1, n + 1)))
        got = ctx.score_fixed(planes, np.array(pix, np.int32))
    V = O.Views.from_scene(sc)
    # the cost-2 decisions (weighted variance at the 1e-5 threshold) against the oracle's own with its
    # positions, samples and moments in float32 (conditioning probe, level 2): a decision that rounding can
    # flip there may flip on the GPU too
    want, probe = (np.array([[O.matching_cost(V, Q, x, y, pl.astype(np.float64), j) for j in range(n)]
                             for (x, y), pl in zip(pix, planes)]) for Q in (O.Params(), O.Params(sample_f32=2)))
    both = (want < 2) & (got < 2)
    err = np.abs(got - want)[both]
    flips, probe_flips = ((want < 2) != (got < 2)).mean(), ((want < 2) != (probe < 2)).mean()
    say(f"  max err {err.max():.2e} over {both.sum()} scored pairs; cost-2 decisions differing: gpu {flips:.4f}, "
        f"probe {probe_flips:.4f}")
    assert flips <= probe_flips + 5e-3
    assert err.max() <= 1e-4


def test_full_run_properties(amh, big_scene):
    """A whole run at full size: outputs are finite, in range, unit normals facing the camera, and accurate."""
    name, sc = big_scene
    n = len(sc.srcs)
    iters = sc.meta["iters"]
    say(f"case full run properties {name} iters={iters}")
    with _ctx(amh, sc, sc.meta["refine"]) as ctx:
        ctx.run_checkerboard(0, list(range(1, n + 1)), iters)
        depth, normal, cost = ctx.get_depth_normal_cost()
        pl, c, S, v = ctx.get_state()
        st = ctx.get_stats()
    assert np.all(np.isfinite(depth)) and np.all(np.isfinite(normal)) and np.all(np.isfinite(cost))
    assert depth.min() >= 2.0 * (1 - 1e-5) and depth.max() <= 6.0 * (1 + 1e-5)
    np.testing.assert_allclose(np.linalg.norm(normal, axis=-1), 1.0, atol=1e-5)
    Kinv = np.linalg.inv(sc.cams[0].K)
    ys, xs = np.mgrid[0:sc.height, 0:sc.width]
    rx = Kinv[0, 0] * xs + Kinv[0, 1] * ys + Kinv[0, 2]
    ry = Kinv[1, 1] * ys + Kinv[1, 2]
    assert np.all(normal[..., 0] * rx + normal[..., 1] * ry + normal[..., 2] < 0)
    assert cost.min() >= 0.0 and cost.max() <= 2.0
    assert np.all(S < (1 << n)) and np.all((v >= -1) & (v < n))
    # every pixel's propagation rows: 8 neighbours (fewer at the border) + its own plane, on n views
    P = sc.width * sc.height
    assert st["evals_init"] == P * n
    assert 2 * iters * (P // 2) * 8 * n < st["evals_propagation"] <= 2 * iters * ((P + 1) // 2) * 9 * n
    rel = np.abs(depth - sc.depth_gt) / sc.depth_gt
    vis = sc.vis_count >= 2
    acc = (rel[vis] < 0.01).mean()
    say(f"  accuracy within 1% of ground truth: {acc:.4f}; evals {st['evals_total']}")
    # calibrated once (seed 0): 0.995 at 1920x1280 after 3 iterations; 0.41 at 3200x2130 after 4
    # iterations, where 30 % of the reference is constant-intensity planes and the propagation reach
    # (23 px per half-pass) covers less of the image
    assert acc >= (0.97 if name == "1920x1280_n10" else 0.38)
