"""Seeded synthetic rectified-stereo disparity scenes.

These scenes stand in for the datasets the paper evaluates on (3F2N, Middlebury,
Cityscapes), none of which is available here: only image sizes, disparity ranges
and camera scales are borrowed, never any dataset content.

This module is shared input plumbing: the FP64 oracle and the GPU path both take
their inputs from it, and it contains none of the method's arithmetic (no filter,
no gradient, no affine or normal estimation, no labelling).  It only ray-casts
analytic surfaces through the rectified pin-hole pair of the paper's Sec. 2
(left projection Pi_1, right projection Pi_2 shifted by the baseline b) to obtain

* the clean disparity D = u_L - u_R = f_x * b / z  (float64),
* the noisy float32 disparity with additive N(0, sigma) noise (Sec. 4, noise model)
  and NaN at invalid pixels,
* the analytic ground-truth unit normal (camera-facing, float64) and a patch id.

Pixel centres sit at integer (u, v); u is the column, v the row (downwards); the
camera frame has x right, y down, z forward.  The principal point defaults to the
image centre ((W-1)/2, (H-1)/2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Camera:
    fx: float
    fy: float
    baseline: float
    u0: float
    v0: float

    @staticmethod
    def centred(width: int, height: int, f: float, baseline: float) -> "Camera":
        return Camera(float(f), float(f), float(baseline),
                      (width - 1) / 2.0, (height - 1) / 2.0)


@dataclass
class Scene:
    disp: np.ndarray          # float32 (H, W); NaN = invalid
    clean: np.ndarray         # float64 (H, W); NaN where no surface
    normal: np.ndarray        # float64 (H, W, 3); NaN where no surface
    patch: np.ndarray         # int32 (H, W); -1 where no surface
    cam: Camera
    sigma: float
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.disp.shape


# ----------------------------------------------------------------------------
# geometry helpers (ray casting only)
# ----------------------------------------------------------------------------

def _rays(width, height, cam):
    """Unnormalised viewing rays r = ((u-u0)/fx, (v-v0)/fy, 1), shape (H, W, 3)."""
    u = np.arange(width, dtype=np.float64)
    v = np.arange(height, dtype=np.float64)
    ru = (u - cam.u0) / cam.fx
    rv = (v - cam.v0) / cam.fy
    r = np.empty((height, width, 3), np.float64)
    r[..., 0] = ru[None, :]
    r[..., 1] = rv[:, None]
    r[..., 2] = 1.0
    return r


def cone_normal(rng, max_angle_deg):
    """Unit normal uniform on the spherical cap of half-angle max_angle about the
    optical axis, oriented towards the camera (negative z)."""
    cmin = np.cos(np.deg2rad(max_angle_deg))
    ct = rng.uniform(cmin, 1.0)
    st = np.sqrt(max(0.0, 1.0 - ct * ct))
    ph = rng.uniform(0.0, 2.0 * np.pi)
    return -np.array([st * np.cos(ph), st * np.sin(ph), ct])


def _plane_depth(rays, n, rho):
    """z of the ray/plane n.X = rho intersection (r_z = 1 so t = z)."""
    den = rays @ n
    with np.errstate(divide="ignore", invalid="ignore"):
        z = rho / den
    return z, den


def _sphere_depth(rays, centre, radius):
    """Near intersection depth and outward normal of rays with a sphere."""
    rr = np.einsum("...i,...i->...", rays, rays)
    rc = rays @ centre
    cc = float(centre @ centre) - radius * radius
    disc = rc * rc - rr * cc
    hit = disc > 0
    with np.errstate(invalid="ignore"):
        t = (rc - np.sqrt(np.where(hit, disc, 0.0))) / rr
    hit &= t > 0
    X = rays * t[..., None]
    nrm = (X - centre) / radius
    return np.where(hit, t, np.inf), nrm


def _box_depth(rays, lo, hi):
    """Slab-method near intersection of rays with an axis-aligned box."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / rays
        t1 = (lo - 0.0) * inv
        t2 = (hi - 0.0) * inv
    tmin = np.minimum(t1, t2)
    tmax = np.maximum(t1, t2)
    tn = np.max(tmin, axis=-1)
    tf = np.min(tmax, axis=-1)
    axis = np.argmax(tmin, axis=-1)
    hit = (tn <= tf) & (tn > 0)
    sign = np.take_along_axis(-np.sign(rays), axis[..., None], axis=-1)[..., 0]
    nrm = np.zeros(rays.shape, np.float64)
    np.put_along_axis(nrm, axis[..., None], sign[..., None], axis=-1)
    return np.where(hit, tn, np.inf), nrm


def _voronoi_cells(width, height, n_cells, rng):
    seeds = np.stack([rng.uniform(0, width, n_cells),
                      rng.uniform(0, height, n_cells)], axis=1)
    u = np.arange(width, dtype=np.float64)
    v = np.arange(height, dtype=np.float64)
    best = np.full((height, width), np.inf)
    cell = np.zeros((height, width), np.int32)
    for k, (su, sv) in enumerate(seeds):
        d2 = (u[None, :] - su) ** 2 + (v[:, None] - sv) ** 2
        m = d2 < best
        best[m] = d2[m]
        cell[m] = k
    return cell


def _voronoi_planes(rays, n_cells, rng, cone_deg, z_centroid, z_ok,
                    max_tries=200):
    """Piecewise-planar surface: one plane per image-space Voronoi cell.

    Each cell gets a cap-uniform normal and a depth at its centroid pixel; a
    plane is resampled until every pixel of its cell is front-facing and has
    depth inside z_ok."""
    H, W, _ = rays.shape
    cell = _voronoi_cells(W, H, n_cells, rng)
    z = np.full((H, W), np.nan)
    nrm = np.full((H, W, 3), np.nan)
    for k in range(n_cells):
        m = cell == k
        if not m.any():
            continue
        vv, uu = np.nonzero(m)
        rc = rays[int(round(vv.mean())), int(round(uu.mean()))]
        cell_rays = rays[m]
        for _ in range(max_tries):
            n = cone_normal(rng, cone_deg)
            z0 = rng.uniform(*z_centroid)
            rho = float(n @ (z0 * rc))
            zc, den = _plane_depth(cell_rays, n, rho)
            if np.all(den < 0) and rho < 0 and zc.min() >= z_ok[0] and zc.max() <= z_ok[1]:
                break
        else:  # fall back to a fronto-parallel plane at the centroid depth
            n = np.array([0.0, 0.0, -1.0])
            rho = float(n @ (z0 * rc))
            zc, _ = _plane_depth(cell_rays, n, rho)
        z[m] = zc
        nrm[m] = n
    return z, nrm, cell


def _occlusion_mask(clean_disp):
    """Left-image pixels not visible in the right image: pixel u on a row is
    occluded when some pixel further right maps to the same or a further-left
    right-image column u_R = u - D."""
    H, W = clean_disp.shape
    u = np.arange(W, dtype=np.float64)[None, :]
    ur = np.where(np.isfinite(clean_disp), u - clean_disp, np.inf)
    # running minimum of u_R over columns strictly to the right
    rev = np.minimum.accumulate(ur[:, ::-1], axis=1)[:, ::-1]
    right_min = np.concatenate([rev[:, 1:], np.full((H, 1), np.inf)], axis=1)
    return right_min <= ur


def _invalidate(clean_disp, target_frac, rng, bands=True):
    """Boolean invalid mask: occlusion bands (optionally) widened leftwards one
    pixel at a time, then i.i.d. top-up, to exactly round(target*H*W) pixels
    (or more when the scene's own holes already exceed the target)."""
    H, W = clean_disp.shape
    target = int(round(target_frac * H * W))
    inv = ~np.isfinite(clean_disp)
    if bands:
        occ = _occlusion_mask(clean_disp) & ~inv
        inv = inv | occ
        band = occ.copy()
        grow_iter = 0
        while inv.sum() < target and band.any() and grow_iter < 6:
            grown = band.copy()
            grown[:, :-1] |= band[:, 1:]
            new = grown & ~inv
            need = target - int(inv.sum())
            nn = int(new.sum())
            if nn == 0:
                break
            if nn > need:
                idx = np.flatnonzero(new)
                pick = rng.choice(idx, size=need, replace=False)
                new = np.zeros(H * W, bool)
                new[pick] = True
                new = new.reshape(H, W)
            inv |= new
            band = grown
            grow_iter += 1
    need = target - int(inv.sum())
    if need > 0:
        idx = np.flatnonzero(~inv)
        pick = rng.choice(idx, size=need, replace=False)
        flat = inv.reshape(-1).copy()
        flat[pick] = True
        inv = flat.reshape(H, W)
    return inv


def _finish(z, nrm, patch, cam, sigma, invalid, rng, seed, meta):
    with np.errstate(divide="ignore", invalid="ignore"):
        clean = cam.fx * cam.baseline / z
    clean = np.where(np.isfinite(z) & (z > 0), clean, np.nan)
    noisy = clean + rng.normal(0.0, sigma, clean.shape)
    disp = noisy.astype(np.float32)
    disp[invalid | ~np.isfinite(clean)] = np.nan
    nrm = np.where(np.isfinite(clean)[..., None], nrm, np.nan)
    patch = np.where(np.isfinite(clean), patch, -1).astype(np.int32)
    return Scene(disp=disp, clean=clean, normal=nrm, patch=patch, cam=cam,
                 sigma=float(sigma), seed=int(seed), meta=meta)


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def planes_scene(width=640, height=480, f=500.0, baseline=0.12, n_planes=3,
                 cone_deg=60.0, z_centroid=(2.0, 10.0), z_ok=(1.5, 15.0),
                 sigma=0.25, invalid_frac=0.05, seed=0, cam=None):
    """Voronoi-cell planes (jump edges between cells), i.i.d. invalid pixels.
    Defaults: the 640x480, 3-plane, f=500, b=0.12 m, sigma=0.25 px, 5% workload."""
    rng = np.random.default_rng(seed)
    cam = cam or Camera.centred(width, height, f, baseline)
    rays = _rays(width, height, cam)
    z, nrm, cell = _voronoi_planes(rays, n_planes, rng, cone_deg, z_centroid, z_ok)
    with np.errstate(divide="ignore", invalid="ignore"):
        clean = cam.fx * cam.baseline / z
    invalid = _invalidate(clean, invalid_frac, rng, bands=False)
    return _finish(z, nrm, cell, cam, sigma, invalid, rng, seed,
                   {"kind": "planes", "n_planes": n_planes})


def _add_spheres(rays, z, nrm, patch, n_spheres, rng, z_range, first_id):
    H, W, _ = rays.shape
    for k in range(n_spheres):
        uc, vc = rng.uniform(0, W), rng.uniform(0, H)
        zc = rng.uniform(*z_range)
        rc = rays[min(H - 1, int(vc)), min(W - 1, int(uc))]
        centre = zc * rc
        radius = rng.uniform(0.05, 0.2) * zc
        t, sn = _sphere_depth(rays, centre, radius)
        m = t < np.where(np.isfinite(z), z, np.inf)
        z[m] = t[m]
        nrm[m] = sn[m]
        patch[m] = first_id + k
    return z, nrm, patch


def planes_quadrics_scene(width=1920, height=1080, f=1400.0, baseline=0.2,
                          n_planes=40, n_spheres=10, cone_deg=60.0,
                          z_range=(2.0, 50.0), sigma=0.5, invalid_frac=0.08,
                          seed=0, cam=None):
    """Voronoi planes plus z-buffered sphere caps, occlusion-band invalids.
    Defaults: the 1920x1080, 40 planes + 10 quadrics, f=1400, b=0.2 m,
    sigma=0.5 px, 8% invalid workload."""
    rng = np.random.default_rng(seed)
    cam = cam or Camera.centred(width, height, f, baseline)
    rays = _rays(width, height, cam)
    zlo, zhi = z_range
    z, nrm, patch = _voronoi_planes(rays, n_planes, rng, cone_deg,
                                    (zlo * 1.5, zhi * 0.6), (zlo, zhi))
    z, nrm, patch = _add_spheres(rays, z, nrm, patch, n_spheres, rng,
                                 (zlo * 1.5, zhi * 0.5), n_planes)
    with np.errstate(divide="ignore", invalid="ignore"):
        clean = cam.fx * cam.baseline / z
    invalid = _invalidate(clean, invalid_frac, rng, bands=True)
    return _finish(z, nrm, patch, cam, sigma, invalid, rng, seed,
                   {"kind": "planes+quadrics", "n_planes": n_planes,
                    "n_spheres": n_spheres})


def uneven_batch_specs(n_frames=64, seed=0, w_range=(640, 2880), h_range=(480, 1988),
                       f_range=(500.0, 3000.0), b_range=(0.1, 0.3), d_max=280.0,
                       sigma_range=(0.25, 1.0), invalid_range=(0.05, 0.10),
                       size_scale=1.0):
    """Per-frame arguments of uneven_batch (so frames can be generated apart)."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_frames):
        W = int(rng.integers(w_range[0], w_range[1] + 1) * size_scale)
        H = int(rng.integers(h_range[0], h_range[1] + 1) * size_scale)
        W, H = max(W, 8), max(H, 8)
        f = rng.uniform(*f_range)
        b = rng.uniform(*b_range)
        sigma = rng.uniform(*sigma_range)
        inv = rng.uniform(*invalid_range)
        z_min = f * b / d_max
        z_max = max(z_min * 40.0, 60.0)
        specs.append(dict(width=W, height=H, f=f, baseline=b,
                          n_planes=int(rng.integers(8, 41)), n_spheres=int(rng.integers(2, 11)),
                          z_range=(z_min * 1.2, z_max), sigma=sigma, invalid_frac=inv,
                          seed=int(rng.integers(0, 2**31 - 1))))
    return specs


def uneven_frame(spec):
    return planes_quadrics_scene(**spec)


def uneven_batch(n_frames=64, seed=0, **kw):
    """Frames of uneven resolution (planes + spheres), disparity in (0, d_max].
    size_scale < 1 shrinks every frame (for quick tests) keeping the recipe."""
    return [uneven_frame(sp) for sp in uneven_batch_specs(n_frames, seed, **kw)]


def road_scene(width=2048, height=1024, f=2260.0, baseline=0.22, sigma=0.75,
               invalid_frac=0.10, seed=0, cam=None):
    """Street-like frame: ground plane, two facades, up to 8 boxes, invalid sky.
    Defaults: 2048x1024, f=2260, b=0.22 m, sigma=0.75 px, 10% invalid."""
    rng = np.random.default_rng(seed)
    cam = cam or Camera.centred(width, height, f, baseline)
    rays = _rays(width, height, cam)
    H, W = height, width
    z = np.full((H, W), np.inf)
    nrm = np.full((H, W, 3), np.nan)
    patch = np.full((H, W), -1, np.int32)
    z_far = 120.0
    z_min = f * baseline / 128.0  # keep D <= 128 px

    def put(t, n, pid):
        m = (t < z) & (t >= z_min) & (t <= z_far)
        z[m] = t[m]
        nrm[m] = n[m] if n.ndim == 3 else n
        patch[m] = pid[m] if np.ndim(pid) == 2 else pid

    h_cam = rng.uniform(1.2, 1.7)
    tg, _ = _plane_depth(rays, np.array([0.0, -1.0, 0.0]), -h_cam)
    tg = np.where(tg > 0, tg, np.inf)
    put(tg, np.array([0.0, -1.0, 0.0]), 0)
    for side, pid in ((-1.0, 1), (1.0, 2)):
        a = rng.uniform(4.0, 12.0)
        top = rng.uniform(8.0, 25.0)
        n = np.array([-side, 0.0, 0.0])
        tf, _ = _plane_depth(rays, n, -a)
        tf = np.where(tf > 0, tf, np.inf)
        y = rays[..., 1] * tf
        tf = np.where(y >= -top, tf, np.inf)  # facade ends at its roof line
        put(tf, n, pid)
    for k in range(int(rng.integers(0, 9))):
        sx, sy, sz = rng.uniform(1.5, 4.0, 3)
        cx = rng.uniform(-3.0, 3.0)
        cz = rng.uniform(6.0, 60.0)
        lo = np.array([cx - sx / 2, h_cam - sy, cz - sz / 2])
        hi = np.array([cx + sx / 2, h_cam, cz + sz / 2])
        tb, nb = _box_depth(rays, lo, hi)
        # one patch id per box face (faces meet at creases)
        face = np.argmax(np.abs(nb), axis=-1) * 2 + (nb.sum(-1) > 0)
        put(tb, nb, 3 + 6 * k + face)
    z = np.where(np.isfinite(z), z, np.nan)
    with np.errstate(divide="ignore", invalid="ignore"):
        clean = cam.fx * cam.baseline / z
    invalid = _invalidate(clean, invalid_frac, rng, bands=True)
    return _finish(z, nrm, patch, cam, sigma, invalid, rng, seed,
                   {"kind": "road"})


def road_batch(n_frames=256, seed=0, **kw):
    return [road_scene(seed=seed * 100003 + i, **kw) for i in range(n_frames)]


def sphere_scene(size=1024, f=500.0, baseline=0.3, radius=1.4, distance=3.0,
                 sigma=0.2, seed=0):
    """Ray-cast sphere straight ahead of the camera, background invalid
    (the paper's noise-robustness setup; the focal length is an assumption)."""
    rng = np.random.default_rng(seed)
    cam = Camera.centred(size, size, f, baseline)
    rays = _rays(size, size, cam)
    t, nrm = _sphere_depth(rays, np.array([0.0, 0.0, distance]), radius)
    z = np.where(np.isfinite(t), t, np.nan)
    patch = np.zeros((size, size), np.int32)
    invalid = np.zeros((size, size), bool)
    return _finish(z, nrm, patch, cam, sigma, invalid, rng, seed,
                   {"kind": "sphere"})


def training_crop(index, crop=256, frame_w=2048, frame_h=1024, f=2260.0,
                  baseline=0.22, sigma_range=(0.1, 1.5), invalid_range=(0.0, 0.15),
                  base_seed=1_000_000):
    """One piecewise-planar training crop cut from a virtual frame: the crop keeps
    the frame's principal point, so (u-u0, v-v0) vary across crops."""
    seed = base_seed + int(index)
    rng = np.random.default_rng(seed)
    ox = int(rng.integers(0, frame_w - crop + 1))
    oy = int(rng.integers(0, frame_h - crop + 1))
    cam = Camera(f, f, baseline, (frame_w - 1) / 2.0 - ox, (frame_h - 1) / 2.0 - oy)
    sigma = rng.uniform(*sigma_range)
    inv = rng.uniform(*invalid_range)
    rays = _rays(crop, crop, cam)
    z, nrm, cell = _voronoi_planes(rays, int(rng.integers(2, 7)), rng, 60.0,
                                   (4.0, 30.0), (3.0, 60.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        clean = cam.fx * cam.baseline / z
    invalid = _invalidate(clean, inv, rng, bands=False)
    return _finish(z, nrm, cell, cam, sigma, invalid, rng, seed,
                   {"kind": "crop", "origin": (ox, oy)})


def road_crop(index, crop=256, frame_w=2048, frame_h=1024, f=2260.0, baseline=0.22,
              sigma_range=(0.1, 1.5), invalid_range=(0.0, 0.15), base_seed=2_000_000):
    """One road-like training crop (ground plane, facades, boxes, sky) cut from a
    virtual frame, the crop keeping the frame's principal point."""
    seed = base_seed + int(index)
    rng = np.random.default_rng(seed)
    ox = int(rng.integers(0, frame_w - crop + 1))
    oy = int(rng.integers(0, frame_h - crop + 1))
    cam = Camera(f, f, baseline, (frame_w - 1) / 2.0 - ox, (frame_h - 1) / 2.0 - oy)
    sc = road_scene(width=crop, height=crop, f=f, baseline=baseline,
                    sigma=float(rng.uniform(*sigma_range)),
                    invalid_frac=float(rng.uniform(*invalid_range)), seed=seed, cam=cam)
    sc.meta.update(kind="road_crop", origin=(ox, oy))
    return sc


def workload(name, seed=None):
    """The named single-frame workloads with their evaluation seeds."""
    if name == "planes_640x480":
        return planes_scene(seed=1000 if seed is None else seed)
    if name == "planes_quadrics_1920x1080":
        return planes_quadrics_scene(seed=2000 if seed is None else seed)
    if name == "road_2048x1024":
        return road_scene(seed=5000 if seed is None else seed)
    raise KeyError(name)
