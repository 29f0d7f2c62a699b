"""Which (pixel, plane, view) evaluations end with cost 2 before any sample is taken (reading R3 of the
range and visibility tests): a predicate for the tests of the library's short-evaluation counters."""
import numpy as np


def short_mask(sc, xy, planes, d_min, d_max):
    """[M, N] mask of (pixel, plane, view) whose cost is 2 before any sample is taken (R3): the plane's depth
    at the pixel outside [d_min, d_max] (relative slack 1e-5), a corner (x +- 5, y +- 5) of the window whose
    ray meets the plane behind the reference camera, the window centre behind the source camera or
    projecting outside its image, or a window corner not in front of the source camera.
    Positions in the source are h = A r + b q per unit inverse depth q = -(n . r) / d_p along the pixel ray
    r = K_ref^-1 (x, y, 1), with A = K_j R_rel, b = K_j t_rel: written from the camera conventions, not
    from either implementation."""
    ref = sc.cams[0]
    pl = planes.astype(np.float64)

    def ray_q(px, py):
        r = np.linalg.solve(ref.K, np.c_[px, py, np.ones(len(px))].T).T
        return r, -np.einsum("ij,ij->i", pl[:, :3], r) / pl[:, 3]

    x, y = xy[:, 0].astype(np.float64), xy[:, 1].astype(np.float64)
    r, q = ray_q(x, y)
    with np.errstate(invalid="ignore", divide="ignore"):
        lam = 1.0 / q
        bad = ~(lam > 0) | (lam < d_min * (1 - 1e-5)) | (lam > d_max * (1 + 1e-5))
    corners = [ray_q(x + dx, y + dy) for dx in (-5, 5) for dy in (-5, 5)]
    for _, qc in corners:
        bad |= ~(qc > 0)
    out = []
    for cam in sc.cams[1:]:
        R_rel = cam.R @ ref.R.T
        A, b = cam.K @ R_rel, cam.K @ (cam.t - R_rel @ ref.t)
        h = r @ A.T + q[:, None] * b
        with np.errstate(invalid="ignore", divide="ignore"):
            cu, cv = h[:, 0] / h[:, 2], h[:, 1] / h[:, 2]
            inside = (h[:, 2] > 0) & (cu >= 0) & (cu <= cam.width - 1) & (cv >= 0) & (cv <= cam.height - 1)
        for rc, qc in corners:
            inside &= (rc @ A.T + qc[:, None] * b)[:, 2] > 0
        out.append(bad | ~inside)
    return np.stack(out, axis=1)
