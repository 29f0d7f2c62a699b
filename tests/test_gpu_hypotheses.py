"""Initial hypotheses from per-pixel estimates (amh_set_initial_hypotheses)
against the oracle's initialisation from cells of one pixel, from host and from
device buffers, and one iteration on from a near-truth start."""
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


def _estimates(sc, seed):
    rng = np.random.default_rng(seed)
    H, W = sc.height, sc.width
    depth = (sc.depth_gt * (1 + rng.uniform(-0.005, 0.005, (H, W)))).astype(np.float32)
    depth[3, 4] = 7.0
    depth[5, 6] = np.nan
    normal = (sc.normal_gt * rng.choice([-2.0, 0.5], (H, W, 1))).astype(np.float32)
    normal[7, 8] = 0.0
    conf = rng.uniform(0, 1, (H, W)).astype(np.float32)
    return depth, normal, conf


def test_set_initial_hypotheses_matches_oracle(amh, oracle_mod, scene_128x96):
    import torch
    from oracle import proposal

    say("case per-pixel initial hypotheses 128x96_n4")
    sc = scene_128x96
    depth, normal, conf = _estimates(sc, 3)
    ctx = amh.Context(seed=13, conf_min=0.5)
    ctx.init_views([np.ascontiguousarray(im) for im in sc.images], sc.cams)
    with ctx:
        ctx.begin(0, [1, 2, 3, 4])
        ctx.set_initial_hypotheses(depth, normal, conf)
        pl, cost, S, v = ctx.get_state()
        fallbacks = ctx.get_stats()["fallback_pixels"]
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        ctx.begin(0, [1, 2, 3, 4])
        ctx.set_initial_hypotheses(dev(depth), dev(normal), dev(conf))
        torch.cuda.synchronize()
        pl2, cost2, S2, v2 = ctx.get_state()
        ctx.begin(0, [1, 2, 3, 4])
        ctx.set_initial_hypotheses(depth, normal)  # no confidence: every estimate counts
        _, _, _, _ = ctx.get_state()
        all_fb = ctx.get_stats()["fallback_pixels"]
        with pytest.raises(ValueError):
            ctx.set_initial_hypotheses(depth[:-1], normal, conf)
        assert ctx.L.amh_set_initial_hypotheses(ctx.h, None, None, None, 0) == amh.AMH_E_INVALID_ARG
        assert ctx.L.amh_set_initial_hypotheses(ctx.h, depth.ctypes.data, normal.ctypes.data, None, 2) == \
            amh.AMH_E_INVALID_ARG
    for a, b in zip((pl, cost, S, v), (pl2, cost2, S2, v2)):
        assert np.array_equal(a, b)  # host and device inputs give the same state
    V = oracle_mod.Views.from_scene(sc)
    P = oracle_mod.Params(seed=13)
    f64 = lambda a: a.astype(np.float64)
    ost, used = proposal.proposal_state(V, P, f64(depth), f64(normal), f64(conf), conf_min=0.5, cell=1)
    near = np.abs(depth - 2.0) < 6e-4 * 2.0
    near |= np.abs(depth - 6.0) < 6e-4 * 6.0
    ok = ~near
    say(f"  estimate used on {used.mean():.3f} of the pixels; fallbacks {fallbacks}, without confidence {all_fb}")
    np.testing.assert_allclose(pl[ok], ost.plane[ok], atol=2e-5, rtol=2e-5)
    assert (np.abs(cost - ost.cost)[ok] <= 1e-4).mean() >= 0.999
    assert np.all(S == 0) and np.all(v == -1)
    assert abs(int(fallbacks) - int((~used).sum())) <= int(near.sum())
    assert all_fb < fallbacks


def test_one_iteration_from_near_truth(amh, scene_128x96):
    """From estimates within 0.5 % of the rendered depth, one iteration keeps the depth map that accurate."""
    say("case one iteration from near-truth hypotheses")
    sc = scene_128x96
    depth, normal, _ = _estimates(sc, 4)
    with amh.Context(seed=2, refine=1) as ctx:
        ctx.init_views([np.ascontiguousarray(im) for im in sc.images], sc.cams)
        ctx.begin(0, [1, 2, 3, 4])
        ctx.set_initial_hypotheses(depth, normal)
        ctx.pass_(0, 0)
        ctx.pass_(0, 1)
        d, _, _ = ctx.get_depth_normal_cost()
    vis = sc.vis_count >= 2
    acc = float((np.abs(d - sc.depth_gt)[vis] < 0.01 * sc.depth_gt[vis]).mean())
    say(f"  within 1 % after one iteration: {acc:.4f}")
    assert acc >= 0.9
