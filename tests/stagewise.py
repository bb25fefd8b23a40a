"""Stage-wise comparison of one frame's point records with the FP64 oracle.

Used by the GPU tests of calls that write only the record array (batch plans):
each stage gets the same upstream input on both sides, so each stage's error is
isolated.

  filter     the GPU's D~ against the oracle's filter of the raw input,
             |err| <= 2^-22 |D~| (FP64 solve rounded once to float32); skipped
             for the learned filter, whose D~ is checked against the network
             oracle elsewhere
  slope      definedness (record flag bit 0) identical to the oracle's on the
             GPU's own D~ (exact integer tests on both sides)
  normals    the record's normal within 1e-4 rad of the oracle's
  labels     bit-exact (raw float32 input), count exact
  points     x, y, z relative error <= 1e-5; flags and labels exact
"""
import numpy as np


def _valid(D):
    with np.errstate(invalid="ignore"):
        return np.isfinite(D) & (D > 0)


def check_records(oracle, D, cam, ng, dn, lab, cnt, pts, nf=None, k=0.1, t=1.0):
    """D raw (H, W) float32; dn, lab, pts the GPU's D~, labels and records
    (host arrays); cnt the GPU's component count or None; nf the LSQ filter
    window (None: learned filter, D~ not compared).  Returns the largest normal
    angle in radians."""
    H, W = D.shape
    valid = _valid(D)
    dn64 = dn.astype(np.float64)
    if nf is not None:
        ref = oracle.denoise(D.astype(np.float64), nf)
        if nf == 1:
            dn64 = np.where(valid, dn64, np.nan)      # window 1 writes valid pixels only
        assert np.array_equal(np.isnan(ref), np.isnan(dn64)), "filter definedness"
        m = np.isfinite(ref)
        err = np.abs(dn64[m] - ref[m])
        assert np.all(err <= 2.0 ** -22 * np.abs(ref[m])), ("filter", float(err.max()))
    else:
        assert np.array_equal(np.isnan(dn64), ~valid), "learned filter definedness"
    a1, a2, dfn = oracle.affine(dn64, ng)
    nref = oracle.normals(dn64, a1, a2, dfn, cam)
    li = pts.view(np.int32)
    flags = li[..., 7]
    assert np.array_equal((flags & 1).astype(bool), dfn), \
        ("slope definedness", int(((flags & 1).astype(bool) != dfn).sum()))
    n = pts[..., 3:6].astype(np.float64)
    assert np.all(np.isnan(n[~dfn])), "normal written where the slope is undefined"
    ng_, nr = n[dfn], nref[dfn]
    ang = np.arctan2(np.linalg.norm(np.cross(ng_, nr), axis=-1), (ng_ * nr).sum(-1))
    max_ang = float(ang.max()) if ang.size else 0.0
    assert max_ang <= 1e-4, ("normals", max_ang)
    lref, cref = oracle.components(D, k, t)
    assert np.array_equal(lab, lref), ("labels", int((lab != lref).sum()))
    if cnt is not None:
        assert cnt == cref, ("count", cnt, cref)
    np.testing.assert_array_equal(li[..., 6], lref)
    np.testing.assert_array_equal(flags, dfn.astype(np.int32) + 2 * (lref >= 0))
    pref = oracle.point_cloud(dn64, nref, cam)
    xyz = pts[..., :3].astype(np.float64)
    assert np.all(np.isnan(xyz[~dfn])), "point written where the slope is undefined"
    rel = np.abs(xyz[dfn] - pref[..., :3][dfn]) / np.maximum(np.abs(pref[..., :3][dfn]), 1e-6)
    assert rel.size == 0 or rel.max() <= 1e-5, ("points", float(rel.max()))
    return max_ang
