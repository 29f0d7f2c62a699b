"""CPU oracle for the two method-side steps of the learned proposal.

TEST INFRASTRUCTURE ONLY (same rules as the rest of ``oracle``).

1. ``sweep_features``: the network's input at 1/4 resolution, on a grid of
   8 ceil(H / 32) x 8 ceil(W / 32) cells (the network halves it three times).
   Cell (i, j) covers reference pixels x in [4j, 4j + 4), y in [4i, 4i + 4),
   coordinates clamped to the image (cells past the right or bottom edge repeat
   the edge pixels), and is sampled at pixel (min(4j + 2, W - 1),
   min(4i + 2, H - 1)).  A plane sweep scores D = 12 m fronto-parallel
   planes, m = max(1, floor((W + 80) / 160)) sub-planes per coarse bin (so one step
   moves a near source's warp by ~2 px at any image width), at inverse depths
   q_i = 1/d_max + (i + 0.5) (1/d_min - 1/d_max) / D; the aggregated cost of
   plane i is the mean of the min(2, n) lowest matching costs (Eq. 8) over the
   first n = min(n_sweep, N) sources (n_sweep = 4 unless given).  Channels:
     0: (mean of the cell's 16 reference intensities - 127.5) / 64;
     1: population standard deviation of those 16 intensities / 32;
     2: position of the lowest aggregated cost, 2 (i* + 0.5) / D - 1 (ties: lowest i);
     3: 1 - that lowest aggregated cost;
     4 + c, c = 0..11: 1 - the lowest aggregated cost among planes c m .. c m + m - 1.
   ``sweep_reference_q`` gives the winning plane's inverse depth, the base that
   the network's depth head corrects.
2. ``proposal_state``: the initial PatchMatch state built from per-cell
   predictions (depth, unit normal, confidence) on the same grid of 4 x 4 cells.
   Pixel (x, y) takes the plane of its cell (y // 4, x // 4): through the 3-D
   point at the predicted depth on the ray of the cell's sample pixel, with the
   predicted normal, turned to face the pixel's own ray.  It is used when the confidence is at least
   ``conf_min``, the normal is non-zero and the plane's depth along the pixel's
   ray lies in [d_min, d_max]; otherwise the pixel keeps the random plane of
   random initialisation (Sec. 3: random plane per pixel).  The initial cost is
   the mean of the k lowest per-view costs over all N sources, S = 0, v = -1.
"""
from __future__ import annotations

import numpy as np

from . import Params, State, Views, matching_cost, random_plane

N_COARSE = 12
N_NET_SRC = 4
K_SWEEP = 2
CELL = 4


def _kinv(views: Views) -> np.ndarray:
    return np.linalg.inv(np.array(views.c.Kref[:], np.float64).reshape(3, 3))


def grid(H: int, W: int):
    """Cell grid (h4, w4) of an H x W reference: 1/4 resolution rounded up to multiples of 8."""
    return 8 * -(-H // 32), 8 * -(-W // 32)


def sample_pixel(H: int, W: int, i: int, j: int):
    return min(CELL * j + CELL // 2, W - 1), min(CELL * i + CELL // 2, H - 1)


def sub_bins(width: int) -> int:
    return max(1, (width + 80) // 160)


def sweep_planes(params: Params, width: int) -> list:
    D = N_COARSE * sub_bins(width)
    qf, qn = 1.0 / params.d_max, 1.0 / params.d_min
    return [np.array([0.0, 0.0, -1.0, 1.0 / (qf + (i + 0.5) * (qn - qf) / D)]) for i in range(D)]


def sweep_costs(views: Views, params: Params, x: int, y: int, n_sweep: int = N_NET_SRC) -> np.ndarray:
    """Aggregated cost of every sweep plane at reference pixel (x, y) over the first n_sweep sources."""
    n = min(n_sweep, views.n_src)
    kk = min(K_SWEEP, n)
    out = []
    for pl in sweep_planes(params, views.W):
        c = sorted(matching_cost(views, params, x, y, pl, jv) for jv in range(n))
        out.append(float(np.mean(c[:kk])))
    return np.array(out)


def sweep_features(views: Views, params: Params, n_sweep: int = N_NET_SRC) -> np.ndarray:
    """(h4, w4, 16) float64 network input of the reference of ``views`` (sweep over the first n_sweep sources)."""
    H, W = views.H, views.W
    h4, w4 = grid(H, W)
    m = sub_bins(W)
    D = N_COARSE * m
    ref = views.images[0].astype(np.float64)
    F = np.zeros((h4, w4, 4 + N_COARSE))
    for i in range(h4):
        for j in range(w4):
            ys = np.minimum(np.arange(CELL * i, CELL * i + CELL), H - 1)
            xs = np.minimum(np.arange(CELL * j, CELL * j + CELL), W - 1)
            blk = ref[np.ix_(ys, xs)]
            F[i, j, 0] = (blk.mean() - 127.5) / 64.0
            F[i, j, 1] = blk.std() / 32.0
            a = sweep_costs(views, params, *sample_pixel(H, W, i, j), n_sweep=n_sweep)
            best = int(np.argmin(a))
            F[i, j, 2] = 2.0 * (best + 0.5) / D - 1.0
            F[i, j, 3] = 1.0 - a[best]
            F[i, j, 4:] = 1.0 - a.reshape(N_COARSE, m).min(axis=1)
    return F


def sweep_reference_q(views: Views, params: Params, n_sweep: int = N_NET_SRC) -> np.ndarray:
    """(h4, w4) inverse depth of each cell's winning sweep plane (the network's depth base)."""
    H, W = views.H, views.W
    h4, w4 = grid(H, W)
    D = N_COARSE * sub_bins(W)
    qf, qn = 1.0 / params.d_max, 1.0 / params.d_min
    out = np.zeros((h4, w4))
    for i in range(h4):
        for j in range(w4):
            x, y = sample_pixel(H, W, i, j)
            best = int(np.argmin(sweep_costs(views, params, x, y, n_sweep=n_sweep)))
            out[i, j] = qf + (best + 0.5) * (qn - qf) / D
    return out


def proposal_plane(views: Views, params: Params, x: int, y: int, depth, normal, conf, conf_min: float = 0.5,
                   cell: int = CELL):
    """(plane, used) for pixel (x, y) from per-cell maps (h, w) and (h, w, 3) of cell x cell pixels (cell 1:
    per-pixel hypotheses)."""
    H, W = views.H, views.W
    i, j = y // cell, x // cell
    nv = np.asarray(normal[i, j], np.float64)
    nn = float(np.linalg.norm(nv))
    if conf[i, j] >= conf_min and np.isfinite(nn) and nn > 0.0 and np.isfinite(depth[i, j]):
        Ki = _kinv(views)
        n = nv / nn
        sx, sy = min(cell * j + cell // 2, W - 1), min(cell * i + cell // 2, H - 1)
        Xc = float(depth[i, j]) * (Ki @ np.array([sx, sy, 1.0]))
        dp = -float(n @ Xc)
        r = Ki @ np.array([x, y, 1.0])
        nr = float(n @ r)
        if nr > 0.0:
            n, dp, nr = -n, -dp, -nr
        if nr < 0.0:
            d = -dp / nr
            if params.d_min <= d <= params.d_max:
                return np.array([n[0], n[1], n[2], dp]), True
    return random_plane(views, params, x, y, 0, 0), False


def proposal_state(views: Views, params: Params, depth, normal, conf, conf_min: float = 0.5, cell: int = CELL):
    """(State, used mask) of proposal initialisation (cell 1: from per-pixel hypotheses)."""
    H, W, N = views.H, views.W, views.n_src
    kk = min(params.k, N)
    st = State.empty(H, W)
    used = np.zeros((H, W), bool)
    for y in range(H):
        for x in range(W):
            pl, u = proposal_plane(views, params, x, y, depth, normal, conf, conf_min, cell)
            st.plane[y, x] = pl
            used[y, x] = u
            c = sorted(matching_cost(views, params, x, y, pl, jv) for jv in range(N))
            st.cost[y, x] = float(np.mean(c[:kk]))
    return st, used
