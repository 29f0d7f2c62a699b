"""Pins of the oracle's ablation modes (Sec. 4: the method with symmetric
checkerboard propagation instead of ACP, and with heuristic view selection
instead of MHJ).

* Symmetric table: 8 other-colour neighbours, closed under reflection and
  90-degree rotation, each inside the asymmetric region of the same index.
* Reach (Sec. 3.1: a symmetric checkerboard spreads a hypothesis only a
  limited distance per step): a single true plane planted in a wrong-plane
  field reaches, in one half-pass, exactly the pixels whose candidate set holds
  it -- 8 pixels within 5 px symmetrically, up to 23 px asymmetrically.
* Selection by brute force: every propagated row of the symmetric mode is the
  plane of the fixed neighbour, scored view by view by the matching cost.
* Standard symmetric pattern (Fig. 2(b), reading R15): 20 other-colour
  neighbours (every one within L1 distance 3, and the four axial ones at
  distance 5), closed under reflection and quarter turns, containing the fast
  pattern; a planted plane reaches exactly them in one half-pass; every one of
  the 20 rows is its fixed neighbour's plane; the view selection over 20 rows
  equals a brute-force count with n1, n2 taken as the same fractions of the
  rows (n 20 / 8), and with 8 rows the general function equals the method's.
* Heuristic view selection against numpy: a hypothesis costs the mean of its
  k lowest per-view costs; k >= N is the plain mean over the views and k = 1
  the minimum; no selection memory is kept.
"""
import numpy as np
import pytest


def test_scp_table_invariants(oracle_mod):
    dx, dy, reg = oracle_mod.scp_offsets()
    assert len(dx) == 8 and reg.tolist() == list(range(8))
    offs = list(zip(dx.tolist(), dy.tolist()))
    assert len(set(offs)) == 8 and (0, 0) not in offs
    assert np.all((np.abs(dx) + np.abs(dy)) % 2 == 1)  # the other colour
    s = set(offs)
    assert {(-a, -b) for a, b in s} == s  # symmetric
    assert {(b, -a) for a, b in s} == s  # invariant under a quarter turn
    assert sorted(np.abs(dx) + np.abs(dy)) == [1, 1, 1, 1, 5, 5, 5, 5]
    # each symmetric neighbour lies in the asymmetric region of the same index and direction
    adx, ady, areg = oracle_mod.acp_offsets()
    for r in range(8):
        members = set(zip(adx[areg == r].tolist(), ady[areg == r].tolist()))
        assert offs[r] in members


def _planted(oracle_mod, prop_mode, view_mode=0):
    import scenegen

    O = oracle_mod
    sc = scenegen.make_scene(64, 64, 3, 15.0, 0, seed=2, supersample=2)  # one fronto-parallel plane
    V = O.Views.from_scene(sc)
    P = O.Params(refine=0, prop_mode=prop_mode, view_mode=view_mode)
    true = np.array([0.0, 0.0, -1.0, scenegen.BACKGROUND_Z])
    wrong = np.array([0.0, 0.0, -1.0, 2.5])
    st = O.State.empty(V.H, V.W)
    st.plane[:] = wrong
    st.cost[:] = 2.0
    cx, cy = 32, 32  # red
    st.plane[cy, cx] = true
    st.cost[cy, cx] = 0.0
    O.run_pass(V, P, st, 0, 1)
    took = np.all(st.plane == true, axis=-1)
    kept = np.all(st.plane == wrong, axis=-1)
    assert np.all(took | kept)
    took[cy, cx] = False
    return {(x - cx, y - cy) for y, x in zip(*np.nonzero(took))}


@pytest.mark.parametrize("view_mode", [0, 2])
def test_symmetric_reach_is_its_neighbour_set(oracle_mod, view_mode):
    got = _planted(oracle_mod, 1, view_mode)
    dx, dy, _ = oracle_mod.scp_offsets()
    assert got == set(zip(dx.tolist(), dy.tolist()))


def test_asymmetric_reach_extends_to_23_px(oracle_mod):
    got = _planted(oracle_mod, 0)
    dx, dy, _ = oracle_mod.acp_offsets()
    allowed = set(zip(dx.tolist(), dy.tolist()))
    assert got <= allowed
    assert len(got) >= 0.9 * len(allowed)
    assert {(0, -23), (0, 23), (-23, 0), (23, 0)} <= got
    assert max(abs(a) + abs(b) for a, b in got) == 23


def _diag_pass(oracle_mod, scene, **kw):
    O = oracle_mod
    V = O.Views.from_scene(scene)
    P = O.Params(**kw)
    st = O.init(V, P)
    before = st.copy()
    order = np.array([y * V.W + x for y in range(2, 30) for x in range(2, 70) if (x + y) % 2 == 0], np.int32)
    dg = O.run_pass(V, P, st, 1, 0, order=order, diag=True)
    return V, P, before, st, order, dg


def test_symmetric_rows_are_the_fixed_neighbours(oracle_mod, scene_128x96):
    O = oracle_mod
    V, P, before, st, order, dg = _diag_pass(O, scene_128x96, refine=0, prop_mode=1, seed=3)
    dx, dy, _ = O.scp_offsets()
    N = V.n_src
    rng = np.random.default_rng(0)
    for q in rng.choice(len(order), 40, replace=False):
        idx = int(order[q])
        x, y = idx % V.W, idx // V.W
        d = dg[q]
        for r in range(8):
            nx, ny = x + dx[r], y + dy[r]
            inside = 0 <= nx < V.W and 0 <= ny < V.H
            assert d.row_valid[r] == inside
            if not inside:
                assert d.cand_index[r] == -1
                continue
            assert d.cand_index[r] == r
            pl = before.plane[ny, nx]
            want = [O.matching_cost(V, P, x, y, pl, j) for j in range(N)]
            np.testing.assert_allclose(np.array(d.M[r][:N]), want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_heuristic_cost_is_mean_of_k_lowest(oracle_mod, scene_128x96, k):
    O = oracle_mod
    V, P, before, st, order, dg = _diag_pass(O, scene_128x96, refine=1, view_mode=2, k=k, seed=4)
    N = V.n_src
    for q, idx in enumerate(order[:300]):
        d = dg[q]
        assert d.S == 0 and d.v == -1
        for r in range(9):
            if d.row_valid[r]:
                m = np.sort(np.array(d.M[r][:N]))
                assert d.mfinal[r] == pytest.approx(m[:min(k, N)].mean(), rel=1e-12, abs=1e-15)
                if k == 1:
                    assert d.mfinal[r] == min(d.M[r][:N])
        best = min(d.mfinal[r] for r in range(9) if d.row_valid[r])
        y, x = divmod(int(idx), V.W)
        # refinement candidates are scored the same way, each on its own k lowest views
        for c in range(d.n_cand):
            cc = np.sort([O.matching_cost(V, P, x, y, np.array(d.cand_plane[c][:]), j) for j in range(N)])
            assert d.cand_cost[c] == pytest.approx(cc[:min(k, N)].mean(), rel=1e-12, abs=1e-15)
        kept = min([best] + [d.cand_cost[c] for c in range(d.n_cand)])
        assert st.cost[y, x] == pytest.approx(kept, rel=1e-12)
    assert np.all(st.S == 0) and np.all(st.v == -1)


def test_heuristic_with_k_at_least_n_is_the_plain_mean(oracle_mod, scene_128x96):
    O = oracle_mod
    N = len(scene_128x96.srcs)
    a = _diag_pass(O, scene_128x96, refine=1, view_mode=2, k=N + 3, seed=5)
    b = _diag_pass(O, scene_128x96, refine=1, view_mode=1, k=N + 3, seed=5)
    for q in range(len(a[4])):
        for r in range(9):
            assert a[5][q].mfinal[r] == pytest.approx(b[5][q].mfinal[r], rel=1e-13)
    np.testing.assert_allclose(a[3].cost, b[3].cost, rtol=1e-13)


def test_standard_scp_table_invariants(oracle_mod):
    dx, dy, reg = oracle_mod.sscp_offsets()
    assert len(dx) == 20 and reg.tolist() == list(range(20))
    offs = set(zip(dx.tolist(), dy.tolist()))
    assert len(offs) == 20 and (0, 0) not in offs
    l1 = np.abs(dx) + np.abs(dy)
    assert np.all(l1 % 2 == 1)  # the other colour
    assert {(-a, -b) for a, b in offs} == offs and {(b, -a) for a, b in offs} == offs
    # every other-colour pixel within L1 distance 3 (4 + 12), and the four axial pixels at 5
    inner = {(a, b) for a in range(-3, 4) for b in range(-3, 4) if (abs(a) + abs(b)) in (1, 3)}
    assert len(inner) == 16 and inner <= offs
    assert offs - inner == {(0, -5), (0, 5), (-5, 0), (5, 0)}
    fx, fy, _ = oracle_mod.scp_offsets()
    assert set(zip(fx.tolist(), fy.tolist())) <= offs  # the fast version is a subset


@pytest.mark.parametrize("view_mode", [0, 2])
def test_standard_symmetric_reach_is_its_neighbour_set(oracle_mod, view_mode):
    got = _planted(oracle_mod, 2, view_mode)
    dx, dy, _ = oracle_mod.sscp_offsets()
    assert got == set(zip(dx.tolist(), dy.tolist()))


def test_standard_symmetric_rows_and_selection(oracle_mod, scene_128x96):
    O = oracle_mod
    V, P, before, st, order, dg = _diag_pass(O, scene_128x96, refine=1, prop_mode=2, seed=3)
    dx, dy, _ = O.sscp_offsets()
    N = V.n_src
    rng = np.random.default_rng(1)
    tau = O.tau(P, 1)
    checked = 0
    for q in rng.choice(len(order), 40, replace=False):
        idx = int(order[q])
        x, y = idx % V.W, idx // V.W
        d = dg[q]
        assert d.n_prop == 20
        for r in range(20):
            nx, ny = x + dx[r], y + dy[r]
            inside = 0 <= nx < V.W and 0 <= ny < V.H
            assert d.row_valid[r] == inside and d.cand_index[r] == (r if inside else -1)
            if inside:
                pl = before.plane[ny, nx]
                want = [O.matching_cost(V, P, x, y, pl, j) for j in range(N)]
                np.testing.assert_allclose(np.array(d.M[r][:N]), want, rtol=0, atol=1e-12)
        assert d.row_valid[20] == 1  # the pixel's own plane
        # good views by brute force over the 20 rows, thresholds n1 20 / 8 and n2 20 / 8
        M = np.array([d.M[r][:N] for r in range(20)])
        rv = np.array([d.row_valid[r] for r in range(20)], bool)
        S = 0
        for j in range(N):
            lt = int((M[rv, j] < tau).sum())
            gt = int((M[rv, j] > P.tau_up).sum())
            if rv.any() and lt > P.n1 * 2.5 and gt < P.n2 * 2.5:
                S |= 1 << j
        assert d.S == S
        checked += S != 0
        # the argmin: self first, then the rows in order; strictly lower wins
        best = 20
        for r in range(20):
            if d.row_valid[r] and d.mfinal[r] < d.mfinal[best]:
                best = r
        if d.chosen <= 20:
            assert d.chosen == best
        else:
            assert d.cand_cost[d.chosen - 21] < d.mfinal[best]
    assert checked > 0


def test_view_selection_rows_generalises_the_method(oracle_mod):
    O = oracle_mod
    P = O.Params()
    rng = np.random.default_rng(5)
    for _ in range(50):
        M = rng.uniform(0.0, 2.0, (8, 6))
        rv = rng.integers(0, 2, 8)
        a = O.view_selection(P, 1, M, rv, 0b101, 2)
        b = O.lib()  # the general entry point at 8 rows, called directly
        import ctypes as C
        Mc = np.ascontiguousarray(M)
        rvc = np.ascontiguousarray(rv, np.int32)
        S = C.c_uint32(0)
        v = C.c_int(0)
        w = np.zeros(6)
        b.orc_view_selection_rows(C.byref(P.c()), 1, Mc.ctypes.data_as(C.POINTER(C.c_double)),
                                  rvc.ctypes.data_as(C.POINTER(C.c_int)), 8, 6, 0b101, 2, C.byref(S), C.byref(v),
                                  w.ctypes.data_as(C.POINTER(C.c_double)))
        assert a[0] == S.value and a[1] == v.value and np.array_equal(a[2], w)
