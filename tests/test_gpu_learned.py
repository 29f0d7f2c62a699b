"""What the trained proposal network gains over the method without it.

On a held-out 1920 x 1280 scene with 10 sources (the training scenes are
640 x 480, seeds from 1000), three runs from the same views:
  * proposal + 1 iteration (amh_run_proposal),
  * random initialisation + 1 iteration (the same iteration budget),
  * random initialisation + 3 iterations (the plain method's schedule).
The gain test requires the proposal run to resolve at least 10 points more of
the visible pixels to 1 % relative depth than random + 1 iteration, and to
stay within 3 points of the plain 3-iteration result.  Accuracy is measured
against the scene's ground truth on pixels seen by at least two sources.
The weights are the committed result of paper_1805_07920_amd.train_proposal.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.environ.get("AMH_PROPOSAL_WEIGHTS",
                         os.path.join(ROOT, "paper_1805_07920_amd", "weights", "proposal.bin"))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def accuracy(depth, sc):
    vis = sc.vis_count >= 2
    e = np.abs(depth - sc.depth_gt)[vis]
    gt = sc.depth_gt[vis]
    return dict(rel1=float((e < 0.01 * gt).mean()), cm2=float((e < 0.02).mean()), cm10=float((e < 0.10).mean()))


def nearest_first(sc):
    """Source indices ordered by the angle between source and reference camera (nearest first)."""
    import scenegen

    ang = scenegen.source_angles(len(sc.srcs), sc.meta["arc_deg"])
    return [int(i) + 1 for i in np.argsort(np.abs(ang), kind="stable")]


def test_learned_proposal_gain():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_07920_amd as amh
    import scenegen

    assert os.path.exists(WEIGHTS), f"missing trained weights {WEIGHTS}"
    sc = scenegen.config_scene("1920x1280_n10", 1, device="cuda")
    srcs = nearest_first(sc)
    say(f"case learned gain 1920x1280_n10 seed 1, sources {srcs}")
    res = {}
    with amh.Context(seed=5) as ctx:
        ctx.init_views([torch.from_numpy(np.ascontiguousarray(im)).cuda() for im in sc.images], sc.cams)
        ctx.nn_load(WEIGHTS)
        for name, run in (("proposal+1", lambda: ctx.run_proposal(0, srcs, 1)),
                          ("random+1", lambda: ctx.run_checkerboard(0, srcs, 1)),
                          ("random+3", lambda: ctx.run_checkerboard(0, srcs, 3))):
            run()
            d, _, _ = ctx.get_depth_normal_cost()
            res[name] = accuracy(d, sc)
            say(f"  {name}: {res[name]}")
    p, r1, r3 = res["proposal+1"], res["random+1"], res["random+3"]
    assert p["rel1"] >= r1["rel1"] + 0.10
    assert p["rel1"] >= r3["rel1"] - 0.03
