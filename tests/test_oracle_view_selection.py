"""Pins of the oracle's multi-hypothesis joint view selection (Sec. 3.2, Eq. 2-7).

The paper prints no worked example, so every expectation below is computed by
hand from the equations and the paper's parameters (tau_mc_init 0.8, alpha 90,
beta 0.3, n1 2, n2 3, tau_up 1.2, k 4), with the readings R8-R12 for the
points the garbled Eq. 5/6 leave open.  Matrices are 8 rows (propagated
hypotheses) by N columns (source views); entries sit well away from every
threshold so that no case depends on rounding.
"""
import math

import numpy as np
import pytest


def C(m, beta=0.3):
    return math.exp(-m * m / (2 * beta * beta))  # Eq. 3


def test_tau_closed_form(oracle_mod):
    P = oracle_mod.Params()
    assert oracle_mod.tau(P, 0) == pytest.approx(0.8, abs=1e-15)
    assert oracle_mod.tau(P, 2) == pytest.approx(0.8 * math.exp(-4 / 90), abs=1e-15)  # 0.76522...
    assert oracle_mod.tau(P, 5) == pytest.approx(0.60597, abs=1e-5)  # 0.8 * e^(-25/90)


def test_constant_matrix_selects_all_views(oracle_mod):
    P = oracle_mod.Params()
    M = np.full((8, 4), 0.1)
    S, v, w = oracle_mod.view_selection(P, 0, M, [1] * 8)
    assert S == 0b1111
    assert v == 0  # equal importance: lowest index
    np.testing.assert_allclose(w, [C(0.1)] * 4, rtol=1e-13)  # psi_j = (1/8) sum_i C(0.1)


def test_good_view_counts_are_strict(oracle_mod):
    P = oracle_mod.Params()
    M = np.full((8, 5), 0.95)  # between tau (0.8) and tau_up (1.2): neither count
    M[:3, 0] = 0.1   # 3 costs < tau: 3 > n1 = 2 -> good
    M[:2, 1] = 0.1   # only 2 < tau: not good
    M[:3, 2] = 0.1
    M[3:6, 2] = 1.5  # 3 costs > tau_up: not fewer than n2 = 3 -> not good
    M[:3, 3] = 0.1
    M[3:5, 3] = 1.5  # 2 costs > tau_up -> good
    M[:, 4] = 1.0    # nothing below tau
    S, v, w = oracle_mod.view_selection(P, 0, M, [1] * 8)
    assert S == 0b01001
    psi0 = (3 * C(0.1) + 5 * C(0.95)) / 8
    psi3 = (3 * C(0.1) + 3 * C(0.95) + 2 * C(1.5)) / 8
    assert v == (0 if psi0 >= psi3 else 3)
    np.testing.assert_allclose(w, [psi0, 0, 0, psi3, 0], rtol=1e-13)


def test_threshold_decreases_with_iteration(oracle_mod):
    """Costs of 0.7 pass at t = 0 (tau 0.8) but not at t = 5 (tau 0.606)."""
    P = oracle_mod.Params()
    M = np.full((8, 2), 0.7)
    assert oracle_mod.view_selection(P, 0, M, [1] * 8)[0] == 0b11
    S, v, w = oracle_mod.view_selection(P, 5, M, [1] * 8)
    assert S == 0 and v == -1
    np.testing.assert_allclose(w, [1.0, 1.0])  # empty selection, empty memory: plain mean (R12)


def test_topk_truncation_and_previous_best_doubled(oracle_mod):
    P = oracle_mod.Params()
    costs = [0.10, 0.15, 0.20, 0.25, 0.30, 0.35]  # all good; importance decreases with j
    M = np.tile(np.array(costs), (8, 1))
    psi = [C(c) for c in costs]
    S, v, w = oracle_mod.view_selection(P, 1, M, [1] * 8)
    assert S == 0b111111 and v == 0
    np.testing.assert_allclose(w, psi[:4] + [0, 0], rtol=1e-13)
    # the most important view of the previous iteration is view 5: doubled, it enters the top 4
    assert 2 * psi[5] > psi[3]
    S, v, w = oracle_mod.view_selection(P, 1, M, [1] * 8, S_prev=0b100000, v_prev=5)
    assert v == 0  # v_t uses the unmodified importance
    np.testing.assert_allclose(w, [psi[0], psi[1], psi[2], 0, 0, 2 * psi[5]], rtol=1e-13)


def test_views_that_left_the_selection_weigh_point_two(oracle_mod):
    P = oracle_mod.Params()
    M = np.full((8, 4), 1.0)
    M[:, 0] = 0.2
    M[:, 1] = 0.3
    S, v, w = oracle_mod.view_selection(P, 2, M, [1] * 8, S_prev=0b1110, v_prev=2)
    assert S == 0b0011 and v == 0
    np.testing.assert_allclose(w, [C(0.2), C(0.3), 0.2, 0.2], rtol=1e-13)


def test_ties_break_to_lower_index(oracle_mod):
    P = oracle_mod.Params()
    M = np.full((8, 6), 0.2)
    S, v, w = oracle_mod.view_selection(P, 0, M, [1] * 8)
    assert S == 0b111111 and v == 0
    np.testing.assert_allclose(w, [C(0.2)] * 4 + [0, 0], rtol=1e-13)


def test_invalid_rows_excluded(oracle_mod):
    """Rows without a candidate (image border) count in neither the tests nor the mean."""
    P = oracle_mod.Params()
    M = np.full((8, 2), 0.1)
    M[5:, :] = 2.0
    S, v, w = oracle_mod.view_selection(P, 0, M, [1, 1, 1, 1, 1, 0, 0, 0])
    assert S == 0b11
    np.testing.assert_allclose(w, [C(0.1), C(0.1)], rtol=1e-13)  # (1/5) * 5 C(0.1)
    S, _, _ = oracle_mod.view_selection(P, 0, M, [1] * 8)
    assert S == 0  # the three cost-2 rows now count: 3 > tau_up is not fewer than n2


def test_unified_cost_is_weighted_mean(oracle_mod, scene_128x96):
    """Eq. 7 on a real pixel: the kept cost equals sum_j w_j m_ij / sum_j w_j of the chosen row."""
    O = oracle_mod
    V = O.Views.from_scene(scene_128x96)
    P = O.Params(refine=0)
    st = O.init(V, P)
    order = np.array([y * V.W + x for y in range(20, 40) for x in range(20, 60) if (x + y) % 2 == 0], np.int32)
    dg = O.run_pass(V, P, st, 0, 0, order=order, diag=True)
    for q, idx in enumerate(order[:200]):
        d = dg[q]
        N = V.n_src
        w = np.array(d.w[:N])
        for r in range(9):
            if d.row_valid[r]:
                m = np.array(d.M[r][:N])
                assert d.mfinal[r] == pytest.approx((w * m).sum() / w.sum(), rel=1e-12)
        best = min((d.mfinal[r], 0 if r == 8 else r + 1) for r in range(9) if d.row_valid[r])
        assert st.cost.ravel()[idx] == pytest.approx(best[0], rel=1e-12)
        assert st.cost.ravel()[idx] <= d.mfinal[8] + 1e-15  # never worse than keeping the own plane
