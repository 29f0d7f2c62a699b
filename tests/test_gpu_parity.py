"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Bars (written here, derived in the design notes):
  * fixed hypotheses: |cost_gpu - cost_oracle| <= 1e-4 per hypothesis and view;
  * one half-pass from the same state: on every pixel whose decisions clear a
    margin of 1e-5 in the oracle (robust pixels; measured GPU cost errors are
    ~1e-6), the GPU keeps exactly the oracle's plane (bit-exact when it is a
    propagated one, 1e-5 when refined), the same view set S_t, and a cost
    within 1e-4; v_t agrees wherever its own argmax clears the margin;
  * full runs: >= 99.5 % of pixels within 0.1 % relative depth.
"""
import sys

import numpy as np
import pytest
from short_predicate import short_mask

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


def gt_planes(sc, pix, jitter=0.0, rng=None):
    Kinv = np.linalg.inv(sc.cams[0].K)
    out = []
    for x, y in pix:
        n = sc.normal_gt[y, x].astype(np.float64)
        d = float(sc.depth_gt[y, x])
        if jitter and rng is not None:
            d *= 1 + rng.uniform(-jitter, jitter)
            n = n + rng.normal(scale=jitter, size=3)
            n /= np.linalg.norm(n)
        out.append(np.r_[n, -d * (n @ (Kinv @ [x, y, 1.0]))])
    return np.array(out, np.float32)


def random_planes(sc, pix, rng):
    Kinv = np.linalg.inv(sc.cams[0].K)
    out = []
    for x, y in pix:
        r = Kinv @ [x, y, 1.0]
        d = rng.uniform(1.8, 6.2)
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        if n @ r > 0:
            n = -n
        out.append(np.r_[n, -d * (n @ r)])
    return np.array(out, np.float32)


def make_ctx(amh, sc, **kw):
    ctx = amh.Context(**kw)
    store = amh.AMH_F16 if sc.srcs[0].dtype == np.float16 else amh.AMH_F32
    ctx.init_views([np.ascontiguousarray(im) for im in sc.images], sc.cams, store_as=store)
    return ctx


SCENES = {
    "128x96_n4": dict(name="128x96_n4", seed=0),
    "ragged_131x77_n5": dict(w=131, h=77, n=5, arc=20.0, planes=4, seed=7),
    "fp16_96x64_n6": dict(w=96, h=64, n=6, arc=30.0, planes=3, seed=3, src_dtype="f16", low=0.3),
}


def build_scene(spec):
    import scenegen

    if "name" in spec:
        return scenegen.config_scene(spec["name"], spec["seed"])
    return scenegen.make_scene(spec["w"], spec["h"], spec["n"], spec["arc"], spec["planes"], spec["seed"],
                               src_dtype=spec.get("src_dtype", "f32"), low_texture_frac=spec.get("low", 0.0),
                               gain=0.05, supersample=2)


@pytest.mark.parametrize("key", list(SCENES))
def test_score_fixed_matches_oracle(amh, oracle_mod, key):
    say("case score_fixed", key)
    sc = build_scene(SCENES[key])
    O = oracle_mod
    rng = np.random.default_rng(1)
    W, H = sc.width, sc.height
    pix = [(int(rng.integers(0, W)), int(rng.integers(0, H))) for _ in range(300)]
    pix += [(0, 0), (W - 1, H - 1), (0, H - 1), (W - 1, 0), (2, 3), (W - 3, H - 2)]
    planes = np.concatenate([gt_planes(sc, pix), gt_planes(sc, pix, 0.02, rng), random_planes(sc, pix, rng)])
    pix3 = np.array(pix * 3, np.int32)
    n = len(sc.srcs)
    with make_ctx(amh, sc) as ctx:
        ctx.begin(0, list(range(1, n + 1)))
        got = ctx.score_fixed(planes, pix3)
    V = O.Views.from_scene(sc)
    P = O.Params()
    want = np.array([[O.matching_cost(V, P, int(x), int(y), pl.astype(np.float64), j) for j in range(n)]
                     for (x, y), pl in zip(pix3, planes)])
    err = np.abs(got - want)
    say("  max err", err.max(), "valid frac", (want < 2).mean())
    # validity decisions (cost 2 vs scored) agree, and scored costs agree to 1e-4
    both = (want < 2) & (got < 2)
    assert ((want < 2) != (got < 2)).mean() < 1e-3
    assert err[both].max() <= 1e-4
    assert np.all(np.isfinite(got))


def _centre_in_source(sc, xy, planes):
    """[M, N, 2] position of each window centre in each source (camera conventions of the scenes)."""
    ref = sc.cams[0]
    pl = planes.astype(np.float64)
    r = np.linalg.solve(ref.K, np.c_[xy.astype(np.float64), np.ones(len(xy))].T).T
    q = -np.einsum("ij,ij->i", pl[:, :3], r) / pl[:, 3]
    out = []
    for cam in sc.cams[1:]:
        R_rel = cam.R @ ref.R.T
        h = r @ (cam.K @ R_rel).T + q[:, None] * (cam.K @ (cam.t - R_rel @ ref.t))
        out.append(h[:, :2] / h[:, 2:3])
    return np.stack(out, axis=1)


def test_score_fixed_windows_crossing_source_edges(amh, oracle_mod, scene_128x96):
    """Windows whose centre lies within 6 px inside a source's edge read texels beyond it: through the
    gather layout's clamped border (up to 16 texels) or the clamped path.  Their costs must equal the
    oracle's, which clamps every texel index."""
    say("case score_fixed near source edges")
    sc, O = scene_128x96, oracle_mod
    rng = np.random.default_rng(4)
    W, H, n = sc.width, sc.height, len(sc.srcs)
    pix = [(int(rng.integers(0, W)), int(rng.integers(0, H))) for _ in range(4000)]
    planes = np.concatenate([gt_planes(sc, pix, 0.01, rng), random_planes(sc, pix, rng)])
    xy = np.array(pix * 2, np.int32)
    c = _centre_in_source(sc, xy, planes)
    Ws = np.array([cam.width for cam in sc.cams[1:]]) - 1
    Hs = np.array([cam.height for cam in sc.cams[1:]]) - 1
    inside = (c[..., 0] >= 0) & (c[..., 0] <= Ws) & (c[..., 1] >= 0) & (c[..., 1] <= Hs)
    edge = np.minimum(np.minimum(c[..., 0], Ws - c[..., 0]), np.minimum(c[..., 1], Hs - c[..., 1]))
    near = inside & (edge < 6.0)
    sel = np.nonzero(near.any(axis=1))[0][:400]
    assert len(sel) >= 100
    with make_ctx(amh, sc) as ctx:
        ctx.begin(0, list(range(1, n + 1)))
        got = ctx.score_fixed(planes[sel], xy[sel])
    V = O.Views.from_scene(sc)
    P = O.Params()
    want = np.array([[O.matching_cost(V, P, int(x), int(y), pl.astype(np.float64), j) for j in range(n)]
                     for (x, y), pl in zip(xy[sel], planes[sel])])
    m = near[sel] & (want < 2)
    err = np.abs(got - want)
    say(f"  {int(m.sum())} scored evaluations near an edge, max err {err[m].max():.2e}")
    assert m.sum() >= 100
    assert err[m].max() <= 1e-4
    assert ((want < 2) != (got < 2)).mean() < 1e-3


def _init_cost_bar(O, sc, ost, d, seed):
    """Initial costs (mean of the k lowest per-view costs, a continuous function of them) within the per-cost
    bar 1e-4 on every pixel, except where a per-view cost-2 decision sits on its threshold: there the oracle's
    own initialisation with float32 positions, samples and moments (conditioning probe, level 2) misses the
    bar too."""
    probe = O.init(O.Views.from_scene(sc), O.Params(seed=seed, sample_f32=2))
    unsure = np.abs(probe.cost - ost.cost) > 1e-4
    say(f"  pixels where the float32 probe misses the bar: {int(unsure.sum())}")
    assert np.all((d <= 1e-4) | unsure)
    assert unsure.mean() <= 1e-3


def test_init_matches_oracle(amh, oracle_mod, scene_128x96):
    say("case init 128x96_n4")
    O = oracle_mod
    sc = scene_128x96
    with make_ctx(amh, sc, seed=11) as ctx:
        ctx.begin(0, [1, 2, 3, 4])
        ctx.init_hypotheses()
        pl, cost, S, v = ctx.get_state()
        st = ctx.get_stats()
    ost = O.init(O.Views.from_scene(sc), O.Params(seed=11))
    assert np.all(S == 0) and np.all(v == -1)
    np.testing.assert_allclose(pl, ost.plane, atol=2e-5, rtol=2e-5)
    d = np.abs(cost - ost.cost)
    say(f"  initial cost within 1e-4 on {(d <= 1e-4).mean():.5f}, max diff {d.max():.2e}")
    _init_cost_bar(O, sc, ost, d, 11)
    assert st["evals_init"] == sc.width * sc.height * 4


@pytest.mark.parametrize("n", [1, 5, 8, 9, 17, 32])
def test_init_matches_oracle_source_counts(amh, oracle_mod, n):
    """Initialisation with 1, 5, 8, 9, 17 and 32 sources (up to the largest view set, one LDS row of costs per
    source) on a ragged 61x37 image: the colour's last workgroup is partial and rows end mid-block."""
    say("case init n", n)
    import scenegen

    O = oracle_mod
    sc = scenegen.make_scene(61, 37, n, 40.0, 2, seed=20 + n, supersample=1)
    with make_ctx(amh, sc, seed=13) as ctx:
        ctx.begin(0, list(range(1, n + 1)))
        ctx.init_hypotheses()
        pl, cost, S, v = ctx.get_state()
        st = ctx.get_stats()
    ost = O.init(O.Views.from_scene(sc), O.Params(seed=13))
    assert np.all(S == 0) and np.all(v == -1)
    np.testing.assert_allclose(pl, ost.plane, atol=2e-5, rtol=2e-5)
    d = np.abs(cost - ost.cost)
    say(f"  initial cost within 1e-4 on {(d <= 1e-4).mean():.5f}, max diff {d.max():.2e}")
    _init_cost_bar(O, sc, ost, d, 13)
    assert st["evals_init"] == sc.width * sc.height * n
    ys, xs = np.mgrid[0:sc.height, 0:sc.width]
    want = int(short_mask(sc, np.c_[xs.ravel(), ys.ravel()], pl.reshape(-1, 4), 2.0, 6.0).sum())
    assert abs(st["evals_init_short"] - want) <= 2 + 0.002 * want


def _pass_parity(amh, O, sc, t, colour, seed, refine, n_src=None, include_self=1, sym_prop=0, heuristic=0,
                 bil_sq=0, delta=1e-5, ctol=1e-4, min_plane=0.99):
    n = len(sc.srcs) if n_src is None else n_src
    V = O.Views(sc.images[: n + 1], sc.cams[: n + 1])
    P = O.Params(refine=refine, seed=seed, include_self=include_self, prop_mode=sym_prop,
                 view_mode=2 if heuristic else 0, bilateral_sq=bil_sq)
    with make_ctx(amh, sc, refine=refine, seed=seed, include_self=include_self, sym_prop=sym_prop,
                  heuristic_views=heuristic, bilateral_squared=bil_sq) as ctx:
        ctx.begin(0, list(range(1, n + 1)))
        ctx.init_hypotheses()
        # earlier passes give a realistic state (non-empty S, v)
        for tt in range(t):
            ctx.pass_(tt, 0)
            ctx.pass_(tt, 1)
        if colour == 1:
            ctx.pass_(t, 0)
        pl0, c0, S0, v0 = ctx.get_state()
        ctx.pass_(t, colour)
        pl1, c1, S1, v1 = ctx.get_state()
    st = O.State.from_arrays(pl0, c0, S0, v0)
    Wd, Hd = sc.width, sc.height
    order = np.array([i for i in range(Wd * Hd) if ((i % Wd) + (i // Wd)) % 2 == colour], np.int32)
    dg = O.run_pass(V, P, st, t, colour, order=order, delta=delta, diag=True)
    bits = np.array([d.robust for d in dg])
    # the plane and the cost depend on the view tests, the top-k cut, the argmin and refinement;
    # v_t additionally on its own argmax (ORC_ROBUST_* bits of the oracle)
    robust = (bits & 29) == 29
    v_robust = (bits & 3) == 3
    chosen = np.array([d.chosen for d in dg])
    flat = lambda a: a.reshape(Wd * Hd, *a.shape[2:])[order]
    gp, gc, gS, gv = flat(pl1), flat(c1), flat(S1), flat(v1)
    op, oc, oS, ov = flat(st.plane), flat(st.cost), flat(st.S), flat(st.v)
    propagated = chosen <= np.array([d.n_prop for d in dg])  # a propagated row or the own plane
    exact = np.all(gp == op.astype(np.float32), axis=-1)
    close = np.all(np.abs(gp - op) <= 1e-5 * (1 + np.abs(op)), axis=-1)
    ok_plane = np.where(propagated, exact, close)
    ok = ok_plane & (gS == oS) & (np.abs(gc - oc) <= ctol)
    frac_robust = robust.mean()
    say(f"  t={t} colour={colour}: robust {frac_robust:.4f}, agree on robust {ok[robust].mean():.5f}, "
        f"plane agreement overall {ok_plane.mean():.5f}, S {np.mean(gS == oS):.4f}, v {np.mean(gv == ov):.4f}, "
        f"max cost diff on robust {np.abs(gc - oc)[robust].max():.2e}")
    bad = np.nonzero(robust & ~ok)[0][:5]
    for q in bad:
        d = dg[q]
        say(f"    pixel {order[q] % Wd},{order[q] // Wd}: chosen {d.chosen} gpu cost {gc[q]:.6f} oracle {oc[q]:.6f} "
            f"S {gS[q]:#x}/{oS[q]:#x} v {gv[q]}/{ov[q]} mfinal {[round(d.mfinal[r], 6) for r in range(d.n_prop + 1)]} "
            f"cand {[round(d.cand_cost[c], 6) for c in range(d.n_cand)]}")
    vbad = np.nonzero(v_robust & (gv != ov))[0][:5]
    for q in vbad:
        d = dg[q]
        say(f"    v mismatch at {order[q] % Wd},{order[q] // Wd}: gpu {gv[q]} oracle {ov[q]} S {gS[q]:#x}/{oS[q]:#x} "
            f"M {[[round(d.M[r][j], 5) for j in range(n)] for r in range(d.n_prop + 1) if d.row_valid[r]]}")
    assert np.all(gv[v_robust] == ov[v_robust])
    # the other colour is untouched by the pass
    other = ~np.isin(np.arange(Wd * Hd), order)
    assert np.array_equal(pl1.reshape(-1, 4)[other], pl0.reshape(-1, 4)[other])
    # every robust pixel must agree, and almost every pixel keeps the same plane
    assert frac_robust >= 0.5
    assert ok[robust].all()
    assert ok_plane.mean() >= min_plane
    return ok, robust, float(ok_plane.mean())


@pytest.mark.parametrize("t,colour,refine", [(0, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1), (3, 0, 1)])
def test_single_pass_matches_oracle(amh, oracle_mod, scene_128x96, t, colour, refine):
    say("case pass 128x96_n4", t, colour, refine)
    _pass_parity(amh, oracle_mod, scene_128x96, t, colour, seed=3, refine=refine)


@pytest.mark.parametrize("key", ["ragged_131x77_n5", "fp16_96x64_n6"])
def test_single_pass_other_shapes(amh, oracle_mod, key):
    say("case pass", key)
    sc = build_scene(SCENES[key])
    _pass_parity(amh, oracle_mod, sc, 1, 0, seed=8, refine=1)


def test_single_pass_without_self_row(amh, oracle_mod, scene_128x96):
    say("case pass include_self=0")
    _pass_parity(amh, oracle_mod, scene_128x96, 0, 0, seed=2, refine=0, include_self=0)



def test_short_evaluation_counters(amh, oracle_mod, scene_128x96):
    """evals_init_short / evals_short count the evaluations whose cost was decided before sampling:
    compared with the same predicate evaluated on the planes the oracle's pass actually scores."""
    say("case short-evaluation counters 128x96_n4")
    sc, O = scene_128x96, oracle_mod
    Wd, Hd, n = sc.width, sc.height, len(sc.srcs)
    with make_ctx(amh, sc, refine=0, seed=5) as ctx:
        ctx.begin(0, list(range(1, n + 1)))
        ctx.init_hypotheses()
        s_init = ctx.get_stats()
        pl_init, _, _, _ = ctx.get_state()
        ctx.pass_(0, 0)
        ctx.pass_(0, 1)
        s0 = ctx.get_stats()
        pl0, c0, S0, v0 = ctx.get_state()
        ctx.pass_(1, 0)
        s1 = ctx.get_stats()
    ys, xs = np.mgrid[0:Hd, 0:Wd]
    xy = np.c_[xs.ravel(), ys.ravel()]
    want_init = int(short_mask(sc, xy, pl_init.reshape(-1, 4), 2.0, 6.0).sum())
    say(f"  init: gpu {s_init['evals_init_short']} of {s_init['evals_init']}, predicate {want_init}")
    assert s_init["evals_init"] == Wd * Hd * n
    assert abs(s_init["evals_init_short"] - want_init) <= 2 + 0.002 * want_init
    # the pass at t = 1, colour 0: rows of every pixel as the oracle forms them from the same state
    V = O.Views(sc.images, sc.cams)
    P = O.Params(refine=0, seed=5)
    st = O.State.from_arrays(pl0, c0, S0, v0)
    order = np.array([i for i in range(Wd * Hd) if ((i % Wd) + (i // Wd)) % 2 == 0], np.int32)
    dg = O.run_pass(V, P, st, 1, 0, order=order, diag=True)
    odx, ody, _ = O.acp_offsets()
    flat_pl = pl0.reshape(-1, 4)
    rows_xy, rows_pl = [], []
    for q, d in zip(order, dg):
        x, y = q % Wd, q // Wd
        for r in range(8):
            if d.row_valid[r]:
                ci = d.cand_index[r]
                rows_xy.append((x, y))
                rows_pl.append(flat_pl[(y + ody[ci]) * Wd + x + odx[ci]])
        if d.row_valid[8]:
            rows_xy.append((x, y))
            rows_pl.append(flat_pl[q])
    want = int(short_mask(sc, np.array(rows_xy), np.array(rows_pl), 2.0, 6.0).sum())
    got = s1["evals_short"] - s0["evals_short"]
    evals = s1["evals_propagation"] - s0["evals_propagation"]
    say(f"  pass: gpu {got} short of {evals}, predicate {want} of {len(rows_xy) * n}")
    assert evals == len(rows_xy) * n
    assert abs(got - want) <= 2 + 0.002 * want
    assert 0 < got < evals


# ablation modes of Sec. 4 (symmetric propagation, fast (sym 1) and standard (sym 2) pattern; heuristic best-k
# view selection), same bars
@pytest.mark.parametrize("sym,heur,t,colour,refine", [(1, 0, 0, 0, 1), (1, 0, 1, 1, 1), (0, 1, 0, 1, 0),
                                                      (0, 1, 1, 0, 1), (1, 1, 3, 1, 1), (2, 0, 0, 0, 1),
                                                      (2, 0, 1, 1, 1), (2, 0, 3, 0, 1), (2, 1, 1, 0, 1)])
def test_ablation_pass_matches_oracle(amh, oracle_mod, scene_128x96, sym, heur, t, colour, refine):
    say("case ablation pass 128x96_n4", sym, heur, t, colour, refine)
    _pass_parity(amh, oracle_mod, scene_128x96, t, colour, seed=6, refine=refine, sym_prop=sym, heuristic=heur)


@pytest.mark.parametrize("key,sym,heur", [("ragged_131x77_n5", 1, 1), ("fp16_96x64_n6", 0, 1),
                                          ("ragged_131x77_n5", 2, 0), ("fp16_96x64_n6", 2, 1)])
def test_ablation_pass_other_shapes(amh, oracle_mod, key, sym, heur):
    say("case ablation pass", key, sym, heur)
    _pass_parity(amh, oracle_mod, build_scene(SCENES[key]), 1, 1, seed=8, refine=1, sym_prop=sym, heuristic=heur)


@pytest.mark.parametrize("sym,heur", [(1, 0), (0, 1), (1, 1), (2, 0), (2, 1)])
def test_ablation_full_run_depth_parity(amh, oracle_mod, scene_128x96, sym, heur):
    say("case ablation full run 128x96_n4", sym, heur)
    O = oracle_mod
    with make_ctx(amh, scene_128x96, refine=1, seed=4, sym_prop=sym, heuristic_views=heur) as ctx:
        ctx.run_checkerboard(0, [1, 2, 3, 4], 3)
        depth, _, _ = ctx.get_depth_normal_cost()
        _, _, S, v = ctx.get_state()
    V = O.Views.from_scene(scene_128x96)
    st = O.run(V, O.Params(refine=1, seed=4, prop_mode=sym, view_mode=2 if heur else 0), 3)
    od, _ = O.depth_normal(V, st)
    frac = (np.abs(depth - od) / od <= 1e-3).mean()
    say(f"  depth agreement {frac:.5f}")
    assert frac >= 0.995
    if heur:
        assert np.all(S == 0) and np.all(v == -1)


# Squared bilateral weights (reading R5's alternative, Sec. 3.3): exp(-dI^2 / 18) leaves weight only on the few
# samples closest in intensity to the centre, and the NCC of so few effective samples is far worse conditioned
# than with the printed weights.  Two conditioning probes of the oracle measure that, and the bars below are
# derived from them, not from the kernel's errors:
#  * sample_f32 (sample positions and values in float32, nothing else): costs move by up to ~4e-5 with squared
#    weights against ~2e-7 with the printed ones, and whole runs keep only 70-80 % of their depths (100 %);
#    its level 2 also forms the NCC's sums and moments in float32, which a kernel cannot avoid either, and its
#    level 3 moves every sample by the first-order bound of that rounding in the worst direction (one rounding
#    pattern can miss a sensitive eval: one moved 1.6e-8 by level 1 moves 2e-6 at level 3);
#  * cost_noise = 2e-4 (every cost moved by a fixed offset within +-1e-4, the per-hypothesis cost bar): what a
#    kernel whose costs all meet the bar may produce.  With squared weights it keeps fewer planes per pass and
#    ends 1-3 points less accurate than the exact oracle (cost errors within the bar pick worse near-ties in
#    this flat objective); with the printed weights it changes nothing measurable.
NOISE_AT_BAR = 2e-4


@pytest.mark.parametrize("key", list(SCENES))
def test_score_fixed_squared_weights(amh, oracle_mod, key):
    """Fixed hypotheses with squared weights.  Where float32 positions, samples and moments (the probe at
    level 2) and the first-order worst case of rounding the samples (level 3) both move the oracle's cost by
    less than 1e-6 the 1e-4 bar holds as for the printed weights; the ill-conditioned rest (a probe moves them
    by more) must stay within 1e-3, and the cost-2 decisions (weighted variance at the 1e-5 threshold) may
    differ only as often as the level-2 probe's do, plus 0.5 %."""
    say("case score_fixed squared weights", key)
    sc = build_scene(SCENES[key])
    O = oracle_mod
    rng = np.random.default_rng(2)
    W, H = sc.width, sc.height
    pix = [(int(rng.integers(0, W)), int(rng.integers(0, H))) for _ in range(200)]
    planes = np.concatenate([gt_planes(sc, pix), gt_planes(sc, pix, 0.02, rng), random_planes(sc, pix, rng)])
    pix3 = np.array(pix * 3, np.int32)
    n = len(sc.srcs)
    with make_ctx(amh, sc, bilateral_squared=1) as ctx:
        ctx.begin(0, list(range(1, n + 1)))
        got = ctx.score_fixed(planes, pix3)
    V = O.Views.from_scene(sc)
    P, Pp, Pw = O.Params(bilateral_sq=1), O.Params(bilateral_sq=1, sample_f32=2), O.Params(bilateral_sq=1, sample_f32=3)
    want, probe, worst = (np.array([[O.matching_cost(V, Q, int(x), int(y), pl.astype(np.float64), j) for j in range(n)]
                                    for (x, y), pl in zip(pix3, planes)]) for Q in (P, Pp, Pw))
    both = (want < 2) & (got < 2) & (probe < 2) & (worst < 2)
    err, cond = np.abs(got - want), np.maximum(np.abs(probe - want), np.abs(worst - want))
    well = both & (cond < 1e-6)
    flips, probe_flips = ((want < 2) != (got < 2)).mean(), ((want < 2) != (probe < 2)).mean()
    say(f"  well-conditioned {well.sum()} of {both.sum()}: max err {err[well].max():.2e}; ill-conditioned: max err "
        f"{err[both & ~well].max() if (both & ~well).any() else 0:.2e} (probe {cond[both].max():.2e}); "
        f"cost-2 decisions differing: gpu {flips:.4f}, probe {probe_flips:.4f}")
    assert well.sum() >= 0.5 * both.sum()
    assert err[well].max() <= 1e-4
    assert err[both].max() <= 1e-3
    assert flips <= probe_flips + 5e-3


@pytest.mark.parametrize("t,colour,include_self", [(0, 0, 1), (1, 1, 0)])
def test_squared_bilateral_pass_matches_oracle(amh, oracle_mod, scene_128x96, t, colour, include_self):
    """One half-pass with squared weights: a decision must clear the cost bar itself (1e-4) to count as robust;
    on robust pixels exact agreement and the 1e-4 cost bar hold.  Over all pixels the GPU keeps the oracle's
    plane at least as often as the oracle with costs moved within the bar does (cost_noise), less 0.5 %."""
    say("case pass squared bilateral", t, colour, include_self)
    _, _, gpu_keeps = _pass_parity(amh, oracle_mod, scene_128x96, t, colour, seed=9, refine=1,
                                   include_self=include_self, bil_sq=1, delta=1e-4, ctol=1e-4, min_plane=0.0)
    O, sc = oracle_mod, scene_128x96
    V = O.Views.from_scene(sc)
    P = O.Params(refine=1, seed=9, include_self=include_self, bilateral_sq=1)
    Pn = O.Params(refine=1, seed=9, include_self=include_self, bilateral_sq=1, cost_noise=NOISE_AT_BAR)
    st = O.init(V, P)
    for tt in range(t):
        O.run_pass(V, P, st, tt, 0)
        O.run_pass(V, P, st, tt, 1)
    if colour == 1:
        O.run_pass(V, P, st, t, 0)
    a, b = st.copy(), st.copy()
    O.run_pass(V, P, a, t, colour)
    O.run_pass(V, Pn, b, t, colour)
    sel = (np.add.outer(np.arange(sc.height), np.arange(sc.width)) % 2) == colour
    pa, pb = a.plane[sel], b.plane[sel]
    noisy = float(np.all(np.abs(pa - pb) <= 1e-5 * (1 + np.abs(pa)), axis=-1).mean())
    say(f"  oracle with costs within the bar keeps the plane on {noisy:.4f} of the pixels")
    assert gpu_keeps >= noisy - 0.005


@pytest.mark.parametrize("include_self", [1, 0])
def test_squared_bilateral_full_run_accuracy(amh, oracle_mod, include_self):
    """Full runs with squared weights, scene seeds 0-2: the probes show the method's result is not fixed at
    float32 precision there (sample_f32 keeps < 99.5 % of the oracle's depths), so runs are compared by
    accuracy against the rendered depth, within 1 % and within 5 %: on each seed the GPU's accuracy differs from
    the exact oracle's by no more than the oracle's own with costs moved within the bar (cost_noise) does, plus
    half a point."""
    say("case full run squared bilateral, include_self", include_self)
    import scenegen

    O = oracle_mod
    probe_agree = []
    for seed in (0, 1, 2):
        sc = scenegen.config_scene("128x96_n4", seed)
        with make_ctx(amh, sc, refine=1, seed=4, bilateral_squared=1, include_self=include_self) as ctx:
            ctx.run_checkerboard(0, [1, 2, 3, 4], 3)
            depth, _, _ = ctx.get_depth_normal_cost()
        V = O.Views.from_scene(sc)
        run = lambda **kw: O.depth_normal(V, O.run(V, O.Params(refine=1, seed=4, bilateral_sq=1,
                                                                   include_self=include_self, **kw), 3))[0]
        od, pd, nd = run(), run(sample_f32=1), run(cost_noise=NOISE_AT_BAR)
        vis = sc.vis_count >= 2
        acc = lambda d, tol: float((np.abs(d - sc.depth_gt)[vis] < tol * sc.depth_gt[vis]).mean())
        probe_agree.append(float((np.abs(pd - od) / od <= 1e-3).mean()))
        for tol in (0.01, 0.05):
            g, o, nz = acc(depth, tol), acc(od, tol), acc(nd, tol)
            say(f"  seed {seed}, within {tol:.0%}: gpu {g:.4f}, oracle {o:.4f}, oracle with costs within the bar "
                f"{nz:.4f}; float32 probe keeps {probe_agree[-1]:.4f} of the depths")
            assert abs(g - o) <= abs(nz - o) + 0.005
        if include_self:  # without the own plane a pixel can be left with a neighbour's plane out of range here
            assert np.all((depth >= 2.0 - 1e-5) & (depth <= 6.0 + 1e-5))
    assert min(probe_agree) < 0.995  # the premise


def test_ablation_rejected_by_the_batched_path(amh, scene_128x96):
    say("case ablation batch rejected")
    with make_ctx(amh, scene_128x96, sym_prop=1) as ctx:
        with pytest.raises(amh.AmhError) as e:
            ctx.run_batch([dict(ref=0, srcs=[1, 2, 3, 4], iters=1)])
        assert e.value.status == amh.AMH_E_UNSUPPORTED

def test_full_run_depth_parity(amh, oracle_mod, scene_128x96):
    """3 iterations + refinement: GPU and oracle depth maps agree on >= 99.5 % of pixels (0.1 % relative)."""
    say("case full run 128x96_n4")
    O = oracle_mod
    sc = scene_128x96
    with make_ctx(amh, sc, refine=1, seed=4) as ctx:
        ctx.run_checkerboard(0, [1, 2, 3, 4], 3)
        depth, normal, cost = ctx.get_depth_normal_cost()
        stats = ctx.get_stats()
    V = O.Views.from_scene(sc)
    st = O.run(V, O.Params(refine=1, seed=4), 3)
    od, on = O.depth_normal(V, st)
    rel = np.abs(depth - od) / od
    frac = (rel <= 1e-3).mean()
    say(f"  depth agreement {frac:.5f}; evals {stats}")
    assert frac >= 0.995
    gt = np.abs(depth - sc.depth_gt) / sc.depth_gt
    assert (gt[sc.vis_count >= 2] < 0.01).mean() >= 0.7
    assert stats["evals_propagation"] > 0 and stats["evals_refine"] > 0


def test_run_is_deterministic_and_composes(amh, scene_128x96):
    say("case determinism")
    sc = scene_128x96
    outs = []
    for mode in range(3):
        with make_ctx(amh, sc, refine=1, seed=9) as ctx:
            if mode < 2:
                ctx.run_checkerboard(0, [1, 2, 3, 4], 2)
            else:
                ctx.begin(0, [1, 2, 3, 4])
                ctx.init_hypotheses()
                for t in range(2):
                    ctx.pass_(t, 0)
                    ctx.pass_(t, 1)
            outs.append(ctx.get_state())
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
    for a, b in zip(outs[0], outs[2]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("W,H,n,sym,heur", [(1, 1, 1, 0, 0), (2, 3, 2, 0, 0), (7, 5, 3, 0, 0), (16, 1, 2, 0, 0),
                                           (30, 30, 1, 0, 0), (1, 1, 1, 1, 1), (7, 5, 3, 1, 0), (16, 1, 2, 0, 1)])
def test_degenerate_sizes(amh, oracle_mod, W, H, n, sym, heur):
    say("case tiny", W, H, n, "ablation" if sym or heur else "")
    import scenegen

    sc = scenegen.make_scene(W, H, n, 15.0, 1, seed=1, supersample=1)
    with make_ctx(amh, sc, refine=1, seed=1, sym_prop=sym, heuristic_views=heur) as ctx:
        ctx.run_checkerboard(0, list(range(1, n + 1)), 2)
        d, nn, c = ctx.get_depth_normal_cost()
    O = oracle_mod
    V = O.Views.from_scene(sc)
    st = O.run(V, O.Params(refine=1, seed=1, prop_mode=sym, view_mode=2 if heur else 0), 2)
    od, _ = O.depth_normal(V, st)
    assert np.all(np.isfinite(d)) and np.all(np.isfinite(c))
    agree = (np.abs(d - od) / od <= 1e-3).mean()
    say("agreement", agree)
    # the method's full-run bar: 99.5 % of the pixels within 0.1 % (on images this small: every pixel)
    assert agree >= 0.995


def test_many_sources(amh, oracle_mod):
    """N = 32, the largest view set (one 32-bit mask)."""
    say("case n=32")
    import scenegen

    sc = scenegen.make_scene(48, 40, 32, 40.0, 2, seed=5, supersample=1)
    _pass_parity(amh, oracle_mod, sc, 1, 0, seed=5, refine=1)


def test_errors_on_device(amh, scene_128x96):
    say("case errors")
    sc = scene_128x96
    ctx = amh.Context()
    with pytest.raises(amh.AmhError) as e:
        ctx.begin(0, [1])
    assert e.value.status == amh.AMH_E_STATE
    ctx.init_views([np.ascontiguousarray(im) for im in sc.images], sc.cams)
    for srcs in ([], [0], [1, 1], [9], list(range(1, 5)) * 9):
        with pytest.raises(amh.AmhError) as e:
            ctx.begin(0, srcs)
        assert e.value.status == amh.AMH_E_INVALID_ARG
    ctx.begin(0, [1, 2])
    with pytest.raises(amh.AmhError) as e:
        ctx.pass_(0, 0)
    assert e.value.status == amh.AMH_E_STATE
    with pytest.raises(amh.AmhError) as e:
        ctx.get_depth_normal_cost()
    assert e.value.status == amh.AMH_E_STATE
    with pytest.raises(amh.AmhError):
        ctx.score_fixed(np.zeros((1, 4), np.float32), np.array([[sc.width, 0]], np.int32))
    ctx.init_hypotheses()
    with pytest.raises(amh.AmhError) as e:
        ctx.pass_(0, 2)
    assert e.value.status == amh.AMH_E_INVALID_ARG
    bad = [np.zeros((4, 4), np.float32)]
    with pytest.raises(amh.AmhError):
        ctx.init_views(bad, sc.cams[:1])  # camera size differs from the image
    # the widest image the 32-bit gather offsets allow (16351 with the layout's 16-texel border), and one more
    import dataclasses
    for w, ok in ((16352, False), (16351, True)):
        cam = dataclasses.replace(sc.cams[0], width=w, height=2)
        if ok:
            ctx.init_views([np.zeros((2, w), np.float32)], [cam])
        else:
            with pytest.raises(amh.AmhError) as e:
                ctx.init_views([np.zeros((2, w), np.float32)], [cam])
            assert e.value.status == amh.AMH_E_INVALID_ARG
    ctx.close()
