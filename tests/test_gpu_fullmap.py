"""Whole depth maps against the oracle at the measured workloads' recipes.

The bar of the method: after the full schedule of iterations (Sec. 3, with the
parameters of Sec. 4), the GPU's depth agrees with the oracle's within 0.1 %
relative on at least 99.5 % of the pixels; the rest are argmin near-ties that
flip under rounding and spread through propagation.

Cases (the oracle runs whole, on all host cores):
  * 1920x1280 reference + 10 sources, 20-plane scene with occlusions and
    +-5 % per-view gain, 3 iterations + refinement -- the throughput workload
    itself, at full size, in the launch configuration the autotuner picks (the
    one the benchmark times);
  * 800x532 reference + 20 sources stored in float16, 30 % of the area
    low-texture planes, 4 iterations + refinement -- the 3200x2130 recipe at a
    quarter of its side: the initialisation and the source loop at 20 sources,
    the float16 gather layout and the random refinement candidates of t >= 3
    all run.

Both sides' accuracy against the rendered depth is printed and compared, which
separates what the method reaches from what the kernels do.

Textured pixels must meet the bar.  On the constant-intensity planes of the
second case the images do not determine the depth: the oracle itself, with only
its interpolated source samples rounded to float32 (its conditioning probe),
keeps its double-precision depth on about 95 % of those pixels, so no
single-precision kernel can meet the bar there.  The test checks that premise on
every run and compares the GPU with the oracle on those pixels by the
distribution of their depth error and final cost.
"""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DEPTH_REL = 1e-3
MIN_AGREE = 0.995


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


CASES = {
    "1920x1280_n10_3it_refine": dict(cfg="1920x1280_n10", seed=0, overrides={}),
    "800x532_n20_fp16_lowtex_4it_refine": dict(cfg="3200x2130_n20", seed=0, overrides=dict(width=800, height=532)),
}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("key", list(CASES))
def test_whole_depth_map_matches_oracle(amh, oracle_mod, key):
    import scenegen

    spec = CASES[key]
    sc = scenegen.config_scene(spec["cfg"], spec["seed"], device="cuda", **spec["overrides"])
    iters, refine = sc.meta["iters"], sc.meta["refine"]
    n = len(sc.srcs)
    srcs = list(range(1, n + 1))
    W, H = sc.width, sc.height
    say(f"case whole map {key}: {W}x{H}, {n} sources, {iters} iterations, refine {refine}")
    store = amh.AMH_F16 if sc.srcs[0].dtype == np.float16 else amh.AMH_F32
    with amh.Context(refine=refine, seed=spec["seed"]) as ctx:
        ctx.init_views([np.ascontiguousarray(im) for im in sc.images], sc.cams, store_as=store)
        best, _ = ctx.tune([dict(ref=0, srcs=srcs, iters=iters)])
        ctx.run_checkerboard(0, srcs, iters)
        depth, normal, cost = ctx.get_depth_normal_cost()
        st = ctx.get_stats()
    say(f"  gpu done (launch configuration {best}, {st['evals_total']} evaluations)")
    O = oracle_mod
    V = O.Views.from_scene(sc)
    t0 = time.time()
    ost = O.run(V, O.Params(refine=refine, seed=spec["seed"]), iters)
    od, on = O.depth_normal(V, ost)
    say(f"  oracle done in {time.time() - t0:.1f} s on {O.num_threads()} threads")
    same = np.abs(depth - od) / od <= DEPTH_REL
    agree = float(same.mean())
    low = sc.low_texture
    vis = sc.vis_count >= 2
    acc_g = float((np.abs(depth - sc.depth_gt)[vis] < 0.01 * sc.depth_gt[vis]).mean())
    acc_o = float((np.abs(od - sc.depth_gt)[vis] < 0.01 * sc.depth_gt[vis]).mean())
    cost_close = float((np.abs(cost - ost.cost) <= 1e-4).mean())
    say(f"  depth agreement {agree:.5f} (bar {MIN_AGREE}): textured pixels {same[~low].mean():.5f}, "
        f"low-texture pixels {same[low].mean() if low.any() else float('nan'):.5f} ({low.mean():.3f} of the image); "
        f"cost within 1e-4 on {cost_close:.5f}; within 1 % of the rendered depth: gpu {acc_g:.4f}, oracle {acc_o:.4f}")
    assert np.all(np.isfinite(depth)) and np.all(np.isfinite(cost))
    assert abs(acc_g - acc_o) <= 0.005
    assert same[~low].mean() >= MIN_AGREE
    if not low.any():
        assert agree >= MIN_AGREE
        return
    # Constant-intensity planes: the conditioning probe (the oracle with only its interpolated source
    # samples rounded to float32) shows how far the method's result moves there under single-precision
    # samples alone
    t0 = time.time()
    pst = O.run(V, O.Params(refine=refine, seed=spec["seed"], sample_f32=1), iters)
    pd, _ = O.depth_normal(V, pst)
    psame = np.abs(pd - od) / od <= DEPTH_REL
    lv = low & vis

    def stats(d, c):
        e = np.abs(d - sc.depth_gt)[lv] / sc.depth_gt[lv]
        return [float((e < tol).mean()) for tol in (0.01, 0.05, 0.2)] + [float(c[low].mean())]

    sg, so, sp = stats(depth, cost), stats(od, ost.cost), stats(pd, pst.cost)
    say(f"  probe (float32 samples) done in {time.time() - t0:.1f} s: agreement with the oracle {psame.mean():.5f}, "
        f"textured {psame[~low].mean():.5f}, low-texture {psame[low].mean():.5f}")
    say(f"  low-texture pixels, within 1 % / 5 % / 20 % of the rendered depth and mean cost: gpu {np.round(sg, 4)}, "
        f"oracle {np.round(so, 4)}, probe {np.round(sp, 4)}")
    # The premise: float32 samples alone move the result on those planes below the bar (measured: 95 % of
    # their pixels keep the oracle's depth, textured pixels 100 %), so no single-precision kernel can meet it
    # there; the images do not determine the depth of a constant plane, and which of the near-equal noise
    # costs wins is decided by rounding and then spread by propagation.  There the GPU must reach the
    # oracle's result statistically: the fractions of pixels within 1 %, 5 % and 20 % of the rendered depth
    # within half a point of the oracle's (the equal-accuracy margin), and the mean final cost within 0.002
    # (float32 samples alone move these by 0.0002 and 0.00001).
    assert psame[low].mean() < MIN_AGREE
    for g, o in zip(sg[:3], so[:3]):
        assert abs(g - o) <= 0.005
    assert abs(sg[3] - so[3]) <= 0.002
