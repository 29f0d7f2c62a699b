"""C-ABI checks that need no GPU: the library loads, exports every function
include/amhmvs.h declares, and validates arguments before any HIP call."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def amh():
    import paper_1805_07920_amd as amh

    if not os.path.exists(amh.LIB_PATH):
        from paper_1805_07920_amd import build

        build.build()
    return amh


def header_functions():
    txt = open(os.path.join(ROOT, "include", "amhmvs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(amh_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_function(amh):
    L = amh.lib()
    declared = header_functions()
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(L, name), f"{name} declared in the header but not exported"
    assert sorted(amh.EXPORTS) == declared


def test_params_default_are_the_papers(amh):
    p = amh.params_default()
    assert (p.tau_mc_init, p.alpha, p.beta, p.tau_up) == pytest.approx((0.8, 90.0, 0.3, 1.2))
    assert (p.n1, p.n2, p.k) == (2, 3, 4)
    assert (p.sigma_color, p.sigma_spatial) == (3.0, 30.0)
    assert (p.depth_min, p.depth_max, p.refine, p.include_self) == (2.0, 6.0, 1, 1)
    assert amh.lib().amh_params_default(None) == amh.AMH_E_INVALID_ARG


@pytest.mark.parametrize("field,value", [("depth_min", -1.0), ("depth_max", 1.0), ("sigma_color", 0.0),
                                         ("beta", 0.0), ("k", 0), ("k", 33), ("n1", -1), ("refine", 2),
                                         ("alpha", -3.0), ("depth_max", float("inf"))])
def test_create_rejects_bad_params_before_touching_hip(amh, field, value):
    p = amh.params_default()
    setattr(p, field, value)
    h = C.c_void_p()
    assert amh.lib().amh_create(C.byref(h), C.byref(p), None) == amh.AMH_E_INVALID_ARG
    assert not h.value


def test_null_arguments(amh):
    L = amh.lib()
    p = amh.params_default()
    assert L.amh_create(None, C.byref(p), None) == amh.AMH_E_INVALID_ARG
    assert L.amh_create(C.byref(C.c_void_p()), None, None) == amh.AMH_E_INVALID_ARG
    for call in (lambda: L.amh_set_params(None, C.byref(p)), lambda: L.amh_init_views(None, 1, None, None, 0),
                 lambda: L.amh_begin(None, 0, None, 1), lambda: L.amh_init_hypotheses(None),
                 lambda: L.amh_pass(None, 0, 0), lambda: L.amh_run_checkerboard(None, 0, None, 1, 3),
                 lambda: L.amh_get_depth_normal_cost(None, None, None, None, 0),
                 lambda: L.amh_get_state(None, None, None, None, None, 0),
                 lambda: L.amh_set_state(None, None, None, None, None, 0),
                 lambda: L.amh_score_fixed(None, None, None, 0, None, 0), lambda: L.amh_run_batch(None, 0, None),
                 lambda: L.amh_get_job_result(None, 0, None, None, None, 0),
                 lambda: L.amh_get_job_times(None, 0, None), lambda: L.amh_tune(None, 0, None, None, None),
                 lambda: L.amh_get_stats(None, None), lambda: L.amh_set_launch_config(None, 0),
                 lambda: L.amh_run_batch_proposal(None, 0, None)):
        assert call() == amh.AMH_E_INVALID_ARG
    L.amh_destroy(None)
    assert L.amh_last_error(None) == b"NULL context"


def test_status_strings(amh):
    L = amh.lib()
    assert L.amh_status_str(0) == b"ok"
    assert L.amh_status_str(amh.AMH_E_OOM) == b"out of device memory"
    assert L.amh_status_str(123) == b"unknown status"


def test_no_gpu_means_hip_error(amh):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(amh.AmhError) as e:
        amh.Context()
    assert e.value.status == amh.AMH_E_HIP


def test_nn_null_arguments_and_count(amh):
    L = amh.lib()
    n = C.c_int64()
    assert L.amh_nn_param_count(C.byref(n)) == 0 and n.value == 196341
    assert L.amh_nn_param_count(None) == amh.AMH_E_INVALID_ARG
    for call in (lambda: L.amh_nn_init(None, 0), lambda: L.amh_nn_get_params(None, None, 0),
                 lambda: L.amh_nn_set_params(None, None, 0), lambda: L.amh_nn_get_grads(None, None, 0),
                 lambda: L.amh_nn_forward(None, None, None, 1, 8, 8, None), lambda: L.amh_nn_backward(None, None, None),
                 lambda: L.amh_nn_adam_step(None, 1e-3, 0.9, 0.999, 1e-8), lambda: L.amh_nn_save(None, b"x"),
                 lambda: L.amh_nn_load(None, b"x"), lambda: L.amh_sweep_features(None, None, None),
                 lambda: L.amh_init_from_proposal(None, None, 1, 1), lambda: L.amh_run_proposal(None, 0, None, 1, 1)):
        assert call() == amh.AMH_E_INVALID_ARG


def test_conf_min_validated(amh):
    p = amh.params_default()
    assert p.conf_min == 0.0
    for bad in (-0.1, 1.5, float("nan")):
        p.conf_min = bad
        assert amh.lib().amh_create(C.byref(C.c_void_p()), C.byref(p), None) == amh.AMH_E_INVALID_ARG


def test_ablation_switches_validated(amh):
    p = amh.params_default()
    assert p.sym_prop == 0 and p.heuristic_views == 0
    for field, bads in (("sym_prop", (-1, 3)), ("heuristic_views", (-1, 2)), ("sweep_sources", (-1, 33))):
        for bad in bads:
            q = amh.params_default(**{field: bad})
            assert amh.lib().amh_create(C.byref(C.c_void_p()), C.byref(q), None) == amh.AMH_E_INVALID_ARG


def test_fusion_arguments_validated(amh):
    L = amh.lib()
    fp = amh.amh_fusion_params()
    assert L.amh_fusion_params_default(C.byref(fp)) == amh.AMH_OK
    assert (fp.f_eps, fp.f_ang_deg, fp.f_con) == (pytest.approx(0.3), 30.0, 2)
    assert L.amh_fusion_params_default(None) == amh.AMH_E_INVALID_ARG
    assert L.amh_median_filter4(None, None, None, 4, 4) == amh.AMH_E_INVALID_ARG
    n = C.c_int64(0)
    assert L.amh_fuse(None, 1, None, None, None, C.byref(fp), None, None, None, 0, C.byref(n)) == amh.AMH_E_INVALID_ARG


def test_bilateral_switch_validated(amh):
    assert amh.params_default().bilateral_squared == 0
    for bad in (-1, 2):
        q = amh.params_default(bilateral_squared=bad)
        assert amh.lib().amh_create(C.byref(C.c_void_p()), C.byref(q), None) == amh.AMH_E_INVALID_ARG


def test_probe_arguments_validated(amh):
    L = amh.lib()
    ms = C.c_float()
    for kind, blocks, iters in ((-1, 1, 1), (8, 1, 1), (0, 0, 1), (0, 65537, 1), (0, 1, 0), (0, 1, 65537)):
        assert L.amh_probe_valu(kind, blocks, iters, C.byref(ms)) == amh.AMH_E_INVALID_ARG
    assert L.amh_probe_valu(0, 1, 1, None) == amh.AMH_E_INVALID_ARG
    assert len(amh.PROBE_KINDS) == 8
