"""The paper's two ablation claims (Sec. 4), measured on a synthetic 1920x1280 scene
with 10 sources (seed 1, nearest sources first) against its rendered depth:

* Fig. 4: asymmetric propagation reaches accurate depths in fewer iterations
  than the symmetric checkerboard, fast or standard pattern (after 1 and 2
  iterations the fraction of visible pixels within 2 cm is far higher);
* Table 1: the method with both contributions ends at least as accurate as
  either ablation (6 iterations, the paper's setting).

Margins are set from the measured curves (seeds 1-3, all of which show the
same ordering): at 1 iteration 0.64 vs 0.18 (fast) and 0.36 (standard), at 2
iterations 0.994 vs 0.80 and 0.955.
Parity of the ablation modes with the oracle is in tests/test_gpu_parity.py.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def curves():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_07920_amd as amh
    import scenegen

    say("rendering 1920x1280_n10 seed 1")
    sc = scenegen.config_scene("1920x1280_n10", 1, device="cuda")
    ang = scenegen.source_angles(len(sc.srcs), sc.meta["arc_deg"])
    srcs = [int(i) + 1 for i in np.argsort(np.abs(ang), kind="stable")]
    gt = torch.from_numpy(sc.depth_gt).cuda()
    vis = torch.from_numpy(sc.vis_count >= 2).cuda()
    depth = torch.empty_like(gt)
    out = {}
    with amh.Context(seed=0) as ctx:
        ctx.init_views([torch.from_numpy(np.ascontiguousarray(im)).cuda() for im in sc.images], sc.cams)
        for name, sym, heur in (("full", 0, 0), ("no_acp", 1, 0), ("no_acp_standard", 2, 0), ("no_mhj", 0, 1),
                                ("neither", 1, 1)):
            ctx.set_params(amh.params_default(seed=0, sym_prop=sym, heuristic_views=heur))
            ctx.begin(0, srcs)
            ctx.init_hypotheses()
            cm2 = []
            for t in range(6):
                ctx.pass_(t, 0)
                ctx.pass_(t, 1)
                ctx.get_depth_normal_cost(depth=depth)
                cm2.append(float(((depth - gt).abs()[vis] < 0.02).float().mean()))
            say(f"  {name}: within 2 cm per iteration {np.round(cm2, 4).tolist()}")
            out[name] = np.array(cm2)
    return out


def test_asymmetric_propagation_converges_faster(curves):
    full, scp, std = curves["full"], curves["no_acp"], curves["no_acp_standard"]
    assert full[0] >= scp[0] + 0.3
    assert full[1] >= scp[1] + 0.1
    assert np.all(full >= scp)
    # the standard pattern's 20 neighbours spread a hypothesis further per step than the fast one's 8, but
    # still within 5 px
    assert full[0] >= std[0] + 0.15 and std[0] >= scp[0] + 0.1
    assert full[1] >= std[1] + 0.02
    assert np.all(full >= std - 1e-3)


def test_both_contributions_beat_each_ablation(curves):
    final = {k: v[-1] for k, v in curves.items()}
    assert final["full"] >= final["no_acp"]
    assert final["full"] >= final["no_acp_standard"]
    assert final["full"] >= final["no_mhj"]
    assert final["full"] >= final["neither"]
    assert final["full"] >= 0.99
