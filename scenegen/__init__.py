"""Seeded synthetic multi-view scenes with ground truth.

This module only *generates inputs*: calibrated pinhole cameras and grayscale
images of a piecewise-planar, textured world, rendered by ray casting, plus the
reference view's ground-truth depth, normal and visibility.  It contains none
of the stereo method's arithmetic (no matching cost, no view selection, no
propagation).  Both the GPU library's tests and the CPU oracle's tests feed it
the same seeds, so both sides see identical images.

Conventions (shared by every consumer because they describe the *data*):
  * world = reference camera frame; every camera maps X_cam = R X_world + t;
  * pixel (x, y) has its centre at integer (x, y); y points down; depth is the
    camera-frame z;
  * intensities are floats on the [0, 255] scale.

The world follows the recipe of the configurations the method is measured on:
cameras on a horizontal circle of radius 4 around (0, 0, 4) looking at its
centre, rectangles with random tilt (< 50 deg from facing the reference)
at depths 2.5..5.5, a fronto-parallel textured background, view-consistent
texture from a hashed lattice attached to each plane, optional per-view gain
and optional constant-intensity ("low texture") planes with per-view noise.

Rendering runs in torch float64 on whatever device is asked for (CPU in the
CPU test-suite, the GPU in benchmarks so that large scenes take milliseconds).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

__all__ = ["Camera", "Scene", "make_scene", "config_scene", "batch_job_specs", "CONFIGS"]

D_MIN, D_MAX = 2.0, 6.0
BACKGROUND_Z = 5.9


@dataclass
class Camera:
    K: np.ndarray  # 3x3 float64
    R: np.ndarray  # 3x3 float64, world -> camera
    t: np.ndarray  # 3 float64
    width: int
    height: int

    @property
    def center(self) -> np.ndarray:
        return -self.R.T @ self.t


@dataclass
class Scene:
    images: list  # list of (H, W) numpy arrays; [0] is the reference (float32), sources float32 or float16
    cams: list  # list of Camera, same order
    depth_gt: np.ndarray  # (H, W) float32 z-depth of the reference view
    normal_gt: np.ndarray  # (H, W, 3) float32, unit, facing the reference camera
    vis_count: np.ndarray  # (H, W) int32: sources that see the reference pixel's surface point
    label_gt: np.ndarray  # (H, W) int32 plane id seen at each reference pixel
    low_texture: np.ndarray  # (H, W) bool, reference pixels on constant-intensity planes
    d_min: float = D_MIN
    d_max: float = D_MAX
    meta: dict = field(default_factory=dict)
    # with all_views=True: per camera (same order as cams) the z-depth and the unit normal (camera frame,
    # facing that camera) of the surface at each pixel centre, float32
    depth_views: list = None
    normal_views: list = None

    @property
    def ref(self) -> np.ndarray:
        return self.images[0]

    @property
    def srcs(self) -> list:
        return self.images[1:]

    @property
    def width(self) -> int:
        return self.cams[0].width

    @property
    def height(self) -> int:
        return self.cams[0].height


# --------------------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------------------

def _intrinsics(width: int, height: int) -> np.ndarray:
    f = 100.0 * width / 128.0
    return np.array([[f, 0.0, (width - 1) / 2.0], [0.0, f, (height - 1) / 2.0], [0.0, 0.0, 1.0]])


def _circle_camera(theta: float, width: int, height: int) -> Camera:
    """Camera on the circle of radius 4 about (0, 0, 4), looking at that centre, y down."""
    c = np.array([0.0, 0.0, 4.0])
    pos = c + 4.0 * np.array([math.sin(theta), 0.0, -math.cos(theta)])
    z = (c - pos) / np.linalg.norm(c - pos)
    y = np.array([0.0, 1.0, 0.0])
    x = np.cross(y, z)
    R = np.stack([x, y, z])
    t = -R @ pos
    return Camera(_intrinsics(width, height), R, t, width, height)


def source_angles(n_src: int, arc_deg: float) -> np.ndarray:
    """Source angles spread evenly over the arc with the reference in the middle."""
    a = np.linspace(-arc_deg / 2.0, arc_deg / 2.0, n_src + 1)
    a = np.delete(a, int(np.argmin(np.abs(a))))
    return np.deg2rad(a)


# --------------------------------------------------------------------------------------
# world: planes
# --------------------------------------------------------------------------------------

@dataclass
class _Plane:
    n: np.ndarray  # unit normal (world), n.X + o = 0
    o: float
    p0: np.ndarray  # rectangle centre
    e1: np.ndarray  # in-plane axes
    e2: np.ndarray
    hu: float  # half sizes (inf for the background)
    hv: float
    const: float = -1.0  # >= 0: constant intensity (low texture)


def _make_planes(rng: np.random.Generator, n_planes: int, K: np.ndarray, width: int, height: int) -> list:
    Kinv = np.linalg.inv(K)
    planes = []
    tries = 0
    while len(planes) < n_planes and tries < 100 * max(n_planes, 1):
        tries += 1
        px = rng.uniform(0, width - 1)
        py = rng.uniform(0, height - 1)
        ray = Kinv @ np.array([px, py, 1.0])
        depth = rng.uniform(2.5, 5.5)
        p0 = ray * depth
        # normal within 50 deg of -z (facing the reference camera)
        tilt = math.radians(rng.uniform(0.0, 50.0))
        az = rng.uniform(0.0, 2.0 * math.pi)
        n = np.array([math.sin(tilt) * math.cos(az), math.sin(tilt) * math.sin(az), -math.cos(tilt)])
        a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e1 = np.cross(n, a)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(n, e1)
        hu = rng.uniform(0.5, 1.5)
        hv = rng.uniform(0.5, 1.5)
        corners = [p0 + su * hu * e1 + sv * hv * e2 for su in (-1, 1) for sv in (-1, 1)]
        if min(c[2] for c in corners) < 2.2 or max(c[2] for c in corners) > 5.8:
            continue
        planes.append(_Plane(n, float(-n @ p0), p0, e1, e2, hu, hv))
    # background: fronto-parallel, unbounded, facing the cameras
    nb = np.array([0.0, 0.0, -1.0])
    planes.append(_Plane(nb, BACKGROUND_Z, np.array([0.0, 0.0, BACKGROUND_Z]), np.array([1.0, 0.0, 0.0]),
                         np.array([0.0, 1.0, 0.0]), math.inf, math.inf))
    return planes


# --------------------------------------------------------------------------------------
# texture: hashed value lattice, bilinear in plane coordinates (view-consistent)
# --------------------------------------------------------------------------------------

_M32 = 0xFFFFFFFF


def _hash32(x: torch.Tensor) -> torch.Tensor:
    """32-bit integer mix on int64 tensors holding values < 2**32."""
    x = x & _M32
    x = x ^ (x >> 16)
    x = (x * 0x7FEB352D) & _M32
    x = x ^ (x >> 15)
    x = (x * 0x846CA68B) & _M32
    x = x ^ (x >> 16)
    return x


def _salt(seed: int, pid: int) -> int:
    return int(_hash32(torch.tensor((seed * 0x27D4EB2F + pid * 0x165667B1) & _M32)).item())


def _lattice_value(salt: torch.Tensor, i: torch.Tensor, j: torch.Tensor) -> torch.Tensor:
    h = _hash32(i ^ salt)
    h = _hash32(h ^ (j & _M32))
    h = _hash32(h + 0x5BD1E995)
    return h.to(torch.float64) * (255.0 / 4294967295.0)


def _texture(salt: torch.Tensor, u: torch.Tensor, v: torch.Tensor, spacing: float) -> torch.Tensor:
    su = u / spacing
    sv = v / spacing
    fi = torch.floor(su)
    fj = torch.floor(sv)
    fu = su - fi
    fv = sv - fj
    i = fi.to(torch.int64) + (1 << 30)
    j = fj.to(torch.int64) + (1 << 30)
    v00 = _lattice_value(salt, i, j)
    v10 = _lattice_value(salt, i + 1, j)
    v01 = _lattice_value(salt, i, j + 1)
    v11 = _lattice_value(salt, i + 1, j + 1)
    return (v00 * (1 - fu) + v10 * fu) * (1 - fv) + (v01 * (1 - fu) + v11 * fu) * fv


# --------------------------------------------------------------------------------------
# ray casting
# --------------------------------------------------------------------------------------

def _cast(cams: list, planes: list, xs: torch.Tensor, ys: torch.Tensor, ci: torch.Tensor, seed: int,
          spacing: float):
    """Intersect the rays through pixel coords (xs, ys) of cameras cams[ci] with the world (flat tensors).

    Returns (intensity, camera z-depth, plane id) tensors shaped like xs.  Element-wise arithmetic on
    the three coordinates (no small matrix products); per-camera and per-plane constants are gathered
    per ray, so one call covers every camera and every plane."""
    dev = xs.device
    nc = len(cams)

    def per_cam(vals):
        return torch.tensor(vals, dtype=torch.float64, device=dev)[ci]

    Kis = [np.linalg.inv(c.K) for c in cams]
    Cs = [c.center for c in cams]
    # camera-frame ray with z = 1, then its world direction R^T r (the hit distance is the camera z)
    rx = per_cam([K[0, 0] for K in Kis]) * xs + per_cam([K[0, 1] for K in Kis]) * ys + per_cam([K[0, 2] for K in Kis])
    ry = per_cam([K[1, 1] for K in Kis]) * ys + per_cam([K[1, 2] for K in Kis])
    dw = [per_cam([c.R[0, i] for c in cams]) * rx + per_cam([c.R[1, i] for c in cams]) * ry
          + per_cam([c.R[2, i] for c in cams]) for i in range(3)]
    del rx, ry
    best_t = torch.full_like(xs, math.inf)
    best_id = torch.full(xs.shape, -1, dtype=torch.int64, device=dev)
    for pid, pl in enumerate(planes):
        den = pl.n[0] * dw[0] + pl.n[1] * dw[1] + pl.n[2] * dw[2]
        num = per_cam([-(float(pl.n @ C) + pl.o) for C in Cs])
        tt = num / den
        ok = (tt > 1e-6) & (tt < best_t)
        if math.isfinite(pl.hu):
            d = [per_cam([C[i] - pl.p0[i] for C in Cs]) + tt * dw[i] for i in range(3)]
            u = pl.e1[0] * d[0] + pl.e1[1] * d[1] + pl.e1[2] * d[2]
            v = pl.e2[0] * d[0] + pl.e2[1] * d[1] + pl.e2[2] * d[2]
            ok = ok & (u.abs() <= pl.hu) & (v.abs() <= pl.hv)
        best_t = torch.where(ok, tt, best_t)
        best_id = torch.where(ok, torch.full_like(best_id, pid), best_id)
    tcl = best_t.clamp(max=1e6)
    # texture of the plane each ray hit, with that plane's constants gathered per ray
    hit = best_id.clamp(min=0)
    slot = hit * nc + ci

    def per_plane(vals):
        return torch.tensor(vals, dtype=torch.float64, device=dev)[hit]

    d = [torch.tensor([C[i] - pl.p0[i] for pl in planes for C in Cs], dtype=torch.float64, device=dev)[slot]
         + tcl * dw[i] for i in range(3)]
    u = per_plane([pl.e1[0] for pl in planes]) * d[0] + per_plane([pl.e1[1] for pl in planes]) * d[1] \
        + per_plane([pl.e1[2] for pl in planes]) * d[2]
    v = per_plane([pl.e2[0] for pl in planes]) * d[0] + per_plane([pl.e2[1] for pl in planes]) * d[1] \
        + per_plane([pl.e2[2] for pl in planes]) * d[2]
    del d
    salt = torch.tensor([_salt(seed, pid) for pid in range(len(planes))], dtype=torch.int64, device=dev)[hit]
    const = per_plane([pl.const for pl in planes])
    val = torch.where(const >= 0, const, _texture(salt, u, v, spacing))
    inten = torch.where(best_id >= 0, val, torch.zeros_like(val))
    return inten, best_t, best_id


def _render(cams: list, planes: list, seed: int, spacing: float, ss: int, device) -> list:
    """Render every camera (same size) with ss x ss supersampling.
    Returns [(image, depth at pixel centres, id at centres)] per camera."""
    W, H = cams[0].width, cams[0].height
    nc = len(cams)
    imgs = [torch.zeros((H, W), dtype=torch.float64, device=device) for _ in cams]
    depths = [torch.zeros((H, W), dtype=torch.float64, device=device) for _ in cams]
    ids = [torch.zeros((H, W), dtype=torch.int64, device=device) for _ in cams]
    xs0 = torch.arange(W, dtype=torch.float64, device=device)
    offs = [(k + 0.5) / ss - 0.5 for k in range(ss)]
    grid = [(oy, ox) for oy in offs for ox in offs] + [(0.0, 0.0)]  # samples, then the pixel centre
    ng = len(grid)
    rows_per_chunk = max(1, (1 << 23) // max(1, W * ng * nc))
    for y0 in range(0, H, rows_per_chunk):
        y1 = min(H, y0 + rows_per_chunk)
        ys0 = torch.arange(y0, y1, dtype=torch.float64, device=device)
        # ray layout (camera, grid point, row, column)
        ys = torch.stack([ys0 + oy for oy, _ in grid])[:, :, None].expand(ng, y1 - y0, W)
        xs = torch.stack([xs0 + ox for _, ox in grid])[:, None, :].expand(ng, y1 - y0, W)
        ys = ys[None].expand(nc, ng, y1 - y0, W).reshape(-1)
        xs = xs[None].expand(nc, ng, y1 - y0, W).reshape(-1)
        ci = torch.arange(nc, device=device)[:, None].expand(nc, ng * (y1 - y0) * W).reshape(-1)
        val, dep, pid = _cast(cams, planes, xs, ys, ci, seed, spacing)
        val = val.view(nc, ng, y1 - y0, W)
        dep = dep.view(nc, ng, y1 - y0, W)
        pid = pid.view(nc, ng, y1 - y0, W)
        for c in range(nc):
            acc = torch.zeros((y1 - y0, W), dtype=torch.float64, device=device)
            for g in range(ng - 1):
                acc += val[c, g]
            imgs[c][y0:y1] = acc / (ss * ss)
            depths[c][y0:y1] = dep[c, ng - 1]
            ids[c][y0:y1] = pid[c, ng - 1]
    return list(zip(imgs, depths, ids))


def make_scene(width: int, height: int, n_src: int, arc_deg: float, n_planes: int, seed: int, *,
               gain: float = 0.0, low_texture_frac: float = 0.0, src_dtype: str = "f32",
               supersample: int = 4, device="cpu", all_views: bool = False) -> Scene:
    """Render one reference + n_src source views of a seeded piecewise-planar world."""
    rng = np.random.default_rng(seed)
    ref_cam = Camera(_intrinsics(width, height), np.eye(3), np.zeros(3), width, height)
    cams = [ref_cam] + [_circle_camera(th, width, height) for th in source_angles(n_src, arc_deg)]
    planes = _make_planes(rng, n_planes, ref_cam.K, width, height)
    spacing = 8.0 / ref_cam.K[0, 0]  # 2 px at depth 4
    device = torch.device(device)

    # low-texture planes: mark planes (front to back in the id order) until ~frac of the reference is covered
    low_ids = []
    ys, xs = torch.meshgrid(torch.arange(height, dtype=torch.float64, device=device),
                            torch.arange(width, dtype=torch.float64, device=device), indexing="ij")
    if low_texture_frac > 0:
        ci0 = torch.zeros(width * height, dtype=torch.int64, device=device)
        _, _, ids0 = _cast([ref_cam], planes, xs.reshape(-1), ys.reshape(-1), ci0, seed, spacing)
        counts = torch.bincount(ids0.flatten().clamp(min=0), minlength=len(planes)).cpu().numpy()
        covered = 0
        for pid in range(len(planes) - 1):
            if covered >= low_texture_frac * width * height:
                break
            if counts[pid] == 0:
                continue
            planes[pid].const = float(rng.uniform(50.0, 200.0))
            low_ids.append(pid)
            covered += counts[pid]

    gains = [1.0] + [float(rng.uniform(1.0 - gain, 1.0 + gain)) if gain > 0 else 1.0 for _ in range(n_src)]
    images = []
    ref_depth = ref_ids = None
    src_depths = []
    depth_views, normal_views = ([], []) if all_views else (None, None)
    rendered = _render(cams, planes, seed, spacing, supersample, device)
    for vi, cam in enumerate(cams):
        img, depth, ids = rendered[vi]
        if low_ids:
            noise_gen = torch.Generator(device="cpu").manual_seed(seed * 1000 + vi + 7)
            noise = (torch.rand((height, width), generator=noise_gen, dtype=torch.float64) * 2 - 1).to(device)
            for pid in low_ids:
                m = ids == pid
                img = torch.where(m, img + 0.01 * planes[pid].const * noise, img)
        img = (img * gains[vi]).clamp(0.0, 255.0)
        a = img.to(torch.float32).cpu().numpy()
        if vi > 0 and src_dtype == "f16":
            a = a.astype(np.float16)
        images.append(a)
        if vi == 0:
            ref_depth, ref_ids = depth, ids
        else:
            src_depths.append(depth)
        if all_views:
            depth_views.append(depth.to(torch.float32).cpu().numpy())
            idn = ids.cpu().numpy()
            nv = np.zeros((height, width, 3))
            for pid, pl in enumerate(planes):
                nv[idn == pid] = cam.R @ pl.n
            Ki = np.linalg.inv(cam.K)
            gy, gx = np.mgrid[0:height, 0:width]
            ray = np.stack([Ki[0, 0] * gx + Ki[0, 1] * gy + Ki[0, 2], Ki[1, 1] * gy + Ki[1, 2],
                            np.ones_like(gx, dtype=np.float64)], -1)
            nv = np.where(((nv * ray).sum(-1) > 0)[..., None], -nv, nv)
            normal_views.append(nv.astype(np.float32))

    # ground truth for the reference: depth, normal, visibility
    depth_gt = ref_depth.to(torch.float32).cpu().numpy()
    ids_np = ref_ids.cpu().numpy().astype(np.int32)
    normal_gt = np.zeros((height, width, 3), np.float32)
    for pid, pl in enumerate(planes):
        normal_gt[ids_np == pid] = pl.n  # every plane normal faces -z, i.e. the reference camera
    low_mask = np.isin(ids_np, np.array(low_ids, dtype=np.int32)) if low_ids else np.zeros_like(ids_np, bool)
    Kinv = np.linalg.inv(ref_cam.K)
    Xr = torch.stack([(Kinv[0, 0] * xs + Kinv[0, 1] * ys + Kinv[0, 2]) * ref_depth,
                      (Kinv[1, 1] * ys + Kinv[1, 2]) * ref_depth, ref_depth], dim=-1)
    vis = torch.zeros((height, width), dtype=torch.int32, device=device)
    for cam, sd in zip(cams[1:], src_depths):
        R = torch.tensor(cam.R, dtype=torch.float64, device=device)
        t = torch.tensor(cam.t, dtype=torch.float64, device=device)
        K = torch.tensor(cam.K, dtype=torch.float64, device=device)
        Xc = Xr @ R.T + t
        p = Xc @ K.T
        z = p[..., 2]
        u = p[..., 0] / z
        v = p[..., 1] / z
        ui = torch.round(u).clamp(0, cam.width - 1).to(torch.int64)
        vi_ = torch.round(v).clamp(0, cam.height - 1).to(torch.int64)
        inside = (z > 0) & (u >= 0) & (u <= cam.width - 1) & (v >= 0) & (v <= cam.height - 1)
        dz = sd[vi_, ui]
        vis += (inside & ((dz - z).abs() < 0.02 * z)).to(torch.int32)
    meta = dict(width=width, height=height, n_src=n_src, arc_deg=arc_deg, n_planes=n_planes, seed=seed,
                gain=gain, low_texture_frac=low_texture_frac, src_dtype=src_dtype, supersample=supersample,
                gains=gains)
    return Scene(images, cams, depth_gt, normal_gt, vis.cpu().numpy(), ids_np, low_mask, meta=meta,
                 depth_views=depth_views, normal_views=normal_views)


# --------------------------------------------------------------------------------------
# the measured workloads
# --------------------------------------------------------------------------------------

CONFIGS = {
    # tiny: 128x96, 4 sources, 15 deg arc, 3 planes, fp32, 3 iterations, no refinement
    "128x96_n4": dict(width=128, height=96, n_src=4, arc_deg=15.0, n_planes=3, gain=0.0, low_texture_frac=0.0,
               src_dtype="f32", supersample=4, iters=3, refine=0),
    # 1920x1280, 10 sources, 40 deg arc, 20 planes with occlusions, +-5 % per-view gain, 3 iterations + refinement
    "1920x1280_n10": dict(width=1920, height=1280, n_src=10, arc_deg=40.0, n_planes=20, gain=0.05, low_texture_frac=0.0,
               src_dtype="f32", supersample=2, iters=3, refine=1),
    # 3200x2130, 20 sources stored fp16, 30 % low texture, 4 iterations + refinement
    "3200x2130_n20": dict(width=3200, height=2130, n_src=20, arc_deg=40.0, n_planes=20, gain=0.0, low_texture_frac=0.30,
               src_dtype="f16", supersample=2, iters=4, refine=1),
    # training scenes of the learned proposal (seeds 1000-2999): 640x480, 8 sources, the 1920x1280 recipe
    "640x480_n8": dict(width=640, height=480, n_src=8, arc_deg=40.0, n_planes=20, gain=0.05, low_texture_frac=0.0,
               src_dtype="f32", supersample=2, iters=3, refine=1),
}


def config_scene(name: str, seed: int = 0, device="cpu", **overrides) -> Scene:
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    iters = cfg.pop("iters")
    refine = cfg.pop("refine")
    sc = make_scene(cfg.pop("width"), cfg.pop("height"), cfg.pop("n_src"), cfg.pop("arc_deg"), cfg.pop("n_planes"),
                    seed, device=device, **cfg)
    sc.meta.update(iters=iters, refine=refine, config=name)
    return sc


def batch_job_specs(n_jobs: int = 32, seed0: int = 100) -> list:
    """Uneven batch: size scale s ~ U(0,1), W = 640 + 2560 s, H = 480 + 1650 s (even), N ~ U{4..16}."""
    specs = []
    for i in range(n_jobs):
        rng = np.random.default_rng(seed0 + i)
        s = rng.uniform()
        w = int(round((640 + 2560 * s) / 2)) * 2
        h = int(round((480 + 1650 * s) / 2)) * 2
        n = int(rng.integers(4, 17))
        specs.append(dict(width=w, height=h, n_src=n, arc_deg=40.0, n_planes=20, gain=0.05, seed=seed0 + i))
    return specs
