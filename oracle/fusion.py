"""CPU oracle for the stage after the depth maps: the 4 x 4 median filter and the
consistency-check fusion into a point cloud.

TEST INFRASTRUCTURE ONLY (same rules as the rest of ``oracle``): only the tests,
the smoke check and the benchmark's CPU-baseline leg use it.

1. ``median_filter4`` (Sec. 3.3, last sentence of the refinement paragraph: a
   4 x 4 median filter post-processes each depth map).  Reading R17: the window
   of pixel (x, y) covers columns x-1..x+2 and rows y-1..y+2 (an even window has
   no centre; this is the placement of the usual convention, one before and two
   after), clipped to the image; the median of an even count is the mean of the
   two middle values.  Depth maps are float32; the result is rounded to float32.

2. ``fuse`` (Sec. 3.3, fusion paragraph: a consistency check on depth and normal
   as in Gipuma, with f_eps = 0.3 for the disparity difference, f_ang = 30 degrees
   for the normal difference and f_con = 2 consistent views).  Reading R18:
   views are reference views in the order given.  A pixel p of view i that no
   earlier view has consumed back-projects to X = R_i^T (d K_i^-1 [x, y, 1] - t_i)
   with world normal R_i^T n.  For every other view j: X's camera depth z_j in
   j must be positive; X projects to the nearest pixel q = (round u, round v),
   which must be inside view j; with view j's depth d_j(q) and normal n_j(q)
   the view is consistent when the disparity difference
   f_j B_ij |1 / z_j - 1 / d_j(q)| is below f_eps (f_j the focal length of view
   j along x, B_ij the distance between the camera centres) and the angle
   between the two world normals is below f_ang.  When at least f_con views are
   consistent, p yields a point: the mean of X and the back-projections of the
   consistent q, with the normalised sum of the normals, and every consistent q
   is consumed (it yields no point when its own view becomes the reference).
   Consumed pixels still count as consistent witnesses.  Rounding to the
   nearest pixel is floor(u + 0.5).  A depth that is not finite or not positive
   marks a pixel without depth: it yields no point and witnesses nothing.
"""
from __future__ import annotations

import numpy as np

F_EPS = 0.3
F_ANG_DEG = 30.0
F_CON = 2


def median_filter4(depth) -> np.ndarray:
    """(H, W) float32 -> (H, W) float32 4x4 median (window x-1..x+2, y-1..y+2, clipped)."""
    d = np.asarray(depth, np.float64)
    H, W = d.shape
    pad = np.full((H + 3, W + 3), np.nan)
    pad[1:H + 1, 1:W + 1] = d
    stack = np.stack([pad[dy:dy + H, dx:dx + W] for dy in range(4) for dx in range(4)])
    return np.nanmedian(stack, axis=0).astype(np.float32)


def _cam(c):
    K = np.asarray(c.K, np.float64)
    R = np.asarray(c.R, np.float64)
    t = np.asarray(c.t, np.float64).reshape(3)
    return K, R, t, -R.T @ t


def back_project(cam, x, y, depth):
    """World points of pixels (x, y) at camera depth ``depth`` (arrays of equal shape)."""
    K, R, t, _ = _cam(cam)
    Ki = np.linalg.inv(K)
    rays = np.stack([x, y, np.ones_like(x)], -1).astype(np.float64) @ Ki.T
    return (rays * np.asarray(depth, np.float64)[..., None] - t) @ R  # R^T (X_cam - t)


def fuse(cams, depths, normals, f_eps: float = F_EPS, f_ang_deg: float = F_ANG_DEG, f_con: int = F_CON):
    """Point cloud of the views ``cams`` with per-view (H, W) depth and (H, W, 3) camera-frame unit normals.

    Returns (points (P, 3), normals (P, 3), origin (P, 3) int: view slot, pixel index y W + x, number of
    consistent views), in view order, then raster order."""
    V = len(cams)
    used = [np.zeros(np.shape(d), bool) for d in depths]
    pts, nrm, org = [], [], []
    for i in range(V):
        H, W = np.shape(depths[i])
        _, Ri, _, Ci = _cam(cams[i])
        ys, xs = np.mgrid[0:H, 0:W]
        d = np.asarray(depths[i], np.float64)
        valid = np.isfinite(d) & (d > 0)
        d = np.where(valid, d, 1.0)
        X = back_project(cams[i], xs, ys, d)
        nw = np.asarray(normals[i], np.float64) @ Ri  # R^T n
        acc_X = X.copy()
        acc_n = nw.copy()
        count = np.zeros((H, W), np.int64)
        matches = []
        for j in range(V):
            if j == i:
                continue
            Kj, Rj, tj, Cj = _cam(cams[j])
            Hj, Wj = np.shape(depths[j])
            Xj = X @ Rj.T + tj
            z = Xj[..., 2]
            p = Xj @ Kj.T
            with np.errstate(divide="ignore", invalid="ignore"):
                u = p[..., 0] / p[..., 2]
                v = p[..., 1] / p[..., 2]
            ui = np.floor(u + 0.5)
            vi = np.floor(v + 0.5)
            inside = valid & (z > 0) & (ui >= 0) & (ui <= Wj - 1) & (vi >= 0) & (vi <= Hj - 1)
            ui = np.where(inside, ui, 0).astype(np.int64)
            vi = np.where(inside, vi, 0).astype(np.int64)
            dj = np.asarray(depths[j], np.float64)[vi, ui]
            inside &= np.isfinite(dj) & (dj > 0)
            nj = np.asarray(normals[j], np.float64)[vi, ui] @ Rj
            fB = Kj[0, 0] * np.linalg.norm(Ci - Cj)
            with np.errstate(divide="ignore", invalid="ignore"):
                disp = fB * np.abs(1.0 / z - 1.0 / dj)
                ang = np.degrees(np.arccos(np.clip((nw * nj).sum(-1), -1.0, 1.0)))
            ok = inside & (disp < f_eps) & (ang < f_ang_deg)
            Xq = back_project(cams[j], ui, vi, dj)
            acc_X += np.where(ok[..., None], Xq, 0.0)
            acc_n += np.where(ok[..., None], nj, 0.0)
            count += ok
            matches.append((j, ok, vi, ui))
        emit = valid & (~used[i]) & (count >= f_con)
        for j, ok, vi, ui in matches:
            m = emit & ok
            used[j][vi[m], ui[m]] = True
        idx = np.nonzero(emit.ravel())[0]
        P = acc_X.reshape(-1, 3)[idx] / (count.ravel()[idx] + 1)[:, None]
        Nn = acc_n.reshape(-1, 3)[idx]
        Nn = Nn / np.linalg.norm(Nn, axis=1, keepdims=True)
        pts.append(P)
        nrm.append(Nn)
        org.append(np.stack([np.full(len(idx), i), idx, count.ravel()[idx]], 1))
    return np.concatenate(pts), np.concatenate(nrm), np.concatenate(org).astype(np.int64)


def fuse_pixel(cams, depths, normals, i: int, x: int, y: int, used: bool = False, f_eps: float = F_EPS,
               f_ang_deg: float = F_ANG_DEG, f_con: int = F_CON):
    """The fusion decision of one pixel (x, y) of reference view i, written out view by view.

    ``used``: whether an earlier view consumed the pixel.  Returns a dict: emitted, point, normal, count,
    witnesses [(j, q)], and fragile -- whether a decision lies within the margins of a float32 evaluation
    (disparity within 1e-3 px of f_eps, normal cosine within 1e-5 of cos f_ang, or a projection within
    1e-3 px of a rounding boundary)."""
    K, R, t, C = _cam(cams[i])
    d = float(np.asarray(depths[i])[y, x])
    out = dict(emitted=False, point=None, normal=None, count=0, witnesses=[], fragile=False)
    if not (np.isfinite(d) and d > 0) or used:
        return out
    X = R.T @ (d * (np.linalg.inv(K) @ [x, y, 1.0]) - t)
    nw = R.T @ np.asarray(normals[i], np.float64)[y, x]
    cos_ang = np.cos(np.radians(f_ang_deg))
    acc, accn = X.copy(), nw.copy()
    for j in range(len(cams)):
        if j == i:
            continue
        Kj, Rj, tj, Cj = _cam(cams[j])
        Hj, Wj = np.shape(depths[j])
        Xj = Rj @ X + tj
        if not Xj[2] > 0:
            continue
        p = Kj @ Xj
        u, v = p[0] / p[2], p[1] / p[2]
        for c in (u, v):
            f = (c + 0.5) - np.floor(c + 0.5)
            if min(f, 1.0 - f) < 1e-3:
                out["fragile"] = True
        ui, vi = int(np.floor(u + 0.5)), int(np.floor(v + 0.5))
        if not (0 <= ui <= Wj - 1 and 0 <= vi <= Hj - 1):
            continue
        dj = float(np.asarray(depths[j])[vi, ui])
        if not (np.isfinite(dj) and dj > 0):
            continue
        nj = Rj.T @ np.asarray(normals[j], np.float64)[vi, ui]
        disp = Kj[0, 0] / Kj[2, 2] * np.linalg.norm(C - Cj) * abs(1.0 / Xj[2] - 1.0 / dj)
        cosn = float(nw @ nj)
        if abs(disp - f_eps) < 1e-3 or abs(cosn - cos_ang) < 1e-5:
            out["fragile"] = True
        if disp < f_eps and np.degrees(np.arccos(np.clip(cosn, -1.0, 1.0))) < f_ang_deg:
            acc += Rj.T @ (dj * (np.linalg.inv(Kj) @ [ui, vi, 1.0]) - tj)
            accn += nj
            out["count"] += 1
            out["witnesses"].append((j, vi * Wj + ui))
    if out["count"] >= f_con:
        out.update(emitted=True, point=acc / (out["count"] + 1), normal=accn / np.linalg.norm(accn))
    return out
