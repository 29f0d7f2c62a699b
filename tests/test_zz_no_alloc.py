"""The allocation-free entry point (amh_run_checkerboard_static) against the
allocating one (amh_run_checkerboard + amh_get_depth_normal_cost): bit-equal
depth, normal and cost on two calls in a row, the second on a smaller
reference, then the size limit and the state it leaves behind."""
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


def _scene(W, H, n, seed):
    import scenegen

    return scenegen.make_scene(W, H, n, 30.0, 3, seed, gain=0.05, supersample=1)


def _static_run(amh, ctx, ref, srcs, iters, H, W):
    import torch

    d = torch.full((H, W), float("nan"), device="cuda")
    nm = torch.full((H, W, 3), float("nan"), device="cuda")
    c = torch.full((H, W), float("nan"), device="cuda")
    ctx.run_checkerboard_static(ref, srcs, iters, d, nm, c)
    torch.cuda.synchronize()
    return d.cpu().numpy(), nm.cpu().numpy(), c.cpu().numpy()


def test_static_run_equals_allocating_run_twice(amh):
    cases = [(160, 112, 5, 2, 31), (96, 64, 3, 3, 32)]  # the second call on a smaller reference
    scenes = [_scene(W, H, n, seed) for W, H, n, _, seed in cases]
    images, cams, refs = [], [], []
    for sc in scenes:
        refs.append(len(images))
        images += [np.ascontiguousarray(im) for im in sc.images]
        cams += sc.cams
    with amh.Context(refine=1, seed=11) as ctx:
        ctx.init_views(images, cams)
        for (W, H, n, iters, _), ref in zip(cases, refs):
            srcs = list(range(ref + 1, ref + n + 1))
            say(f"case static run {W}x{H}, {n} sources, {iters} iterations")
            got = _static_run(amh, ctx, ref, srcs, iters, H, W)
            st_static = ctx.get_stats()
            ctx.run_checkerboard(ref, srcs, iters)
            want = ctx.get_depth_normal_cost()
            st = ctx.get_stats()
            for g, w, name in zip(got, want, ("depth", "normal", "cost")):
                assert np.array_equal(g, w), f"{name} differs from the allocating run"
            for k in ("evals_init", "evals_propagation", "evals_refine", "evals_short", "evals_init_short"):
                assert st_static[k] == st[k], k


def test_static_run_limits_and_released_reference(amh):
    import dataclasses

    import torch

    sc = _scene(64, 48, 2, 33)
    images = [np.ascontiguousarray(im) for im in sc.images]
    # a reference one row past the limit is refused before any work
    big_w = 2048
    big_h = amh.AMH_STATIC_MAX_PIXELS // big_w + 1
    big_cam = dataclasses.replace(sc.cams[0], width=big_w, height=big_h)
    with amh.Context(refine=0, seed=1) as ctx:
        ctx.init_views(images + [np.zeros((big_h, big_w), np.float32)], sc.cams + [big_cam])
        with pytest.raises(amh.AmhError) as e:
            ctx.run_checkerboard_static(3, [1, 2], 1)
        assert e.value.status == amh.AMH_E_INVALID_ARG and "at most" in str(e.value)
        with pytest.raises(amh.AmhError) as e:
            ctx.run_checkerboard_static(0, [0, 1], 1)  # the reference listed as a source
        assert e.value.status == amh.AMH_E_INVALID_ARG
        with pytest.raises(ValueError):
            ctx.run_checkerboard_static(0, [1, 2], 1, depth=torch.zeros(10, device="cuda"))
        # the context's reference is released by a static run: its state is not readable any more
        ctx.run_checkerboard(0, [1, 2], 1)
        ctx.get_state()
        ctx.run_checkerboard_static(0, [1, 2], 1)
        with pytest.raises(amh.AmhError) as e:
            ctx.get_state()
        assert e.value.status == amh.AMH_E_STATE
        torch.cuda.synchronize()
