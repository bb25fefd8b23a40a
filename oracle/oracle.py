"""Python face of the FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares nothing with the GPU package:
it loads ``oracle/libsnx_oracle.so`` (plain C, gcc) through ctypes and works on
numpy arrays.

Stage functions (the C file cites the paper's passage for each):
  denoise(D, nf)            masked LSQ plane-fit intercept (filter)
  affine(Dt, ng)            a1, a2 and definedness (anchored masked LSQ)
  normals(Dt, a1, a2, ...)  normal from the constraint-vector cross product
  components(D, k, t)       min-index labels of covered-depth components
  components_crease(D, n, ...) the same with a normal-crease test on every edge
  components_edges(flags)   the same on an explicitly given 4-neighbour graph
  point_cloud(Dt, n, cam)   back-projected points with normals
  affine_labels(Dt, lab, ng) a1, a2 over the window restricted to the centre's component
  compact_points(rec)       the defined records of a dense cloud in raster order
  star_mask(Dt, u, v, ...)  star-fill support of one pixel (adaptive region)
  star_affine(Dt, ...)      a1, a2 and definedness over the star-fill support
  pipeline(D, cam, ...)     all of the above, in order
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsnx_oracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_i32 = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build  # compile the oracle library on first use
        _build.build()
    lib = C.CDLL(_LIB_PATH)
    lib.snxo_denoise.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_int, _dp]
    lib.snxo_affine.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, _u8]
    lib.snxo_normals.argtypes = [_dp, _dp, _dp, _u8, C.c_int, C.c_int] + [C.c_double] * 5 + [_dp]
    lib.snxo_components.argtypes = [_fp, C.c_int, C.c_int, C.c_float, C.c_float, _i32,
                                    C.POINTER(C.c_int64)]
    lib.snxo_components_edges.argtypes = [_u8, C.c_int, C.c_int, _i32, C.POINTER(C.c_int64)]
    lib.snxo_point_cloud.argtypes = [_dp, _dp, C.c_int, C.c_int] + [C.c_double] * 5 + [_dp]
    lib.snxo_num_threads.argtypes = []
    lib.snxo_set_threads.argtypes = [C.c_int]
    lib.snxo_components_crease.argtypes = [_fp, _fp, C.c_int, C.c_int, C.c_float, C.c_float,
                                           C.c_double, _i32, C.POINTER(C.c_int64)]
    lib.snxo_affine_labels.argtypes = [_dp, _i32, C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp,
                                       _u8]
    lib.snxo_star_mask.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_double, C.c_double, _u8]
    lib.snxo_star_affine.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                     C.c_double, C.c_double, C.c_int, _dp, _dp, _u8]
    for f in ("snxo_denoise", "snxo_affine", "snxo_normals", "snxo_components",
              "snxo_point_cloud", "snxo_num_threads", "snxo_star_mask", "snxo_star_affine",
              "snxo_affine_labels", "snxo_components_crease", "snxo_components_edges",
              "snxo_set_threads"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


def num_threads() -> int:
    return int(load().snxo_num_threads())


def set_threads(n: int) -> int:
    """OpenMP threads of later calls; returns the count now in effect."""
    return int(load().snxo_set_threads(int(n)))


def default_min_support(ng: int) -> int:
    """Default minimum support of the gradient window: half the window, rounded up."""
    return int(math.ceil(ng * ng / 2.0))


def _as_f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def denoise(D, nf: int, min_support: int = 0) -> np.ndarray:
    D = _as_f64(D)
    H, W = D.shape
    out = np.empty_like(D)
    if load().snxo_denoise(D, W, H, int(nf), int(min_support), out) != 0:
        raise ValueError("oracle denoise: bad arguments")
    return out


def affine(Dt, ng: int, min_support: int | None = None):
    Dt = _as_f64(Dt)
    H, W = Dt.shape
    ms = default_min_support(ng) if min_support is None else int(min_support)
    a1 = np.empty_like(Dt)
    a2 = np.empty_like(Dt)
    d = np.empty((H, W), np.uint8)
    if load().snxo_affine(Dt, W, H, int(ng), ms, a1, a2, d) != 0:
        raise ValueError("oracle affine: bad arguments")
    return a1, a2, d.astype(bool)


def normals(Dt, a1, a2, defined, cam) -> np.ndarray:
    Dt = _as_f64(Dt)
    H, W = Dt.shape
    out = np.empty((H, W, 3), np.float64)
    load().snxo_normals(Dt, _as_f64(a1), _as_f64(a2),
                        np.ascontiguousarray(defined, dtype=np.uint8), W, H,
                        cam.fx, cam.fy, cam.baseline, cam.u0, cam.v0, out)
    return out


def components(D, k_rel: float = 0.1, t_abs: float = 1.0):
    D = np.ascontiguousarray(D, dtype=np.float32)
    H, W = D.shape
    lab = np.empty((H, W), np.int32)
    n = C.c_int64(0)
    if load().snxo_components(D, W, H, C.c_float(k_rel), C.c_float(t_abs), lab,
                              C.byref(n)) != 0:
        raise MemoryError("oracle components")
    return lab, int(n.value)



def components_edges(flags):
    """Labels and count of the 4-neighbour graph given by per-pixel bits:
    bit 0 present, bit 1 edge to the left neighbour, bit 2 edge to the upper
    neighbour (an edge counts between two present pixels)."""
    flags = np.ascontiguousarray(flags, dtype=np.uint8)
    H, W = flags.shape
    lab = np.empty((H, W), np.int32)
    n = C.c_int64(0)
    if load().snxo_components_edges(flags, W, H, lab, C.byref(n)) != 0:
        raise MemoryError("oracle components_edges")
    return lab, int(n.value)

def point_cloud(Dt, nrm, cam) -> np.ndarray:
    Dt = _as_f64(Dt)
    H, W = Dt.shape
    out = np.empty((H, W, 6), np.float64)
    load().snxo_point_cloud(Dt, _as_f64(nrm), W, H, cam.fx, cam.fy,
                            cam.baseline, cam.u0, cam.v0, out)
    return out


def components_crease(D, nrm, k_rel: float = 0.1, t_abs: float = 1.0, cos_min: float = 0.9):
    """Labels and count of the components whose edges pass both the covered-depth
    predicate and n_p . n_q >= cos_min (nrm: float32 [3, H, W]; NaN = undefined)."""
    D = np.ascontiguousarray(D, dtype=np.float32)
    H, W = D.shape
    n = np.ascontiguousarray(nrm, dtype=np.float32).reshape(3, H, W)
    lab = np.empty((H, W), np.int32)
    cnt = C.c_int64(0)
    if load().snxo_components_crease(D, n, W, H, C.c_float(k_rel), C.c_float(t_abs),
                                     float(cos_min), lab, C.byref(cnt)) != 0:
        raise MemoryError("oracle components_crease")
    return lab, int(cnt.value)


def affine_labels(Dt, lab, ng: int, min_support: int | None = None):
    """a1, a2 and definedness with the n_g window restricted to the pixels of
    the centre's component (labels as from components())."""
    Dt = _as_f64(Dt)
    H, W = Dt.shape
    ms = default_min_support(ng) if min_support is None else int(min_support)
    a1 = np.empty_like(Dt)
    a2 = np.empty_like(Dt)
    d = np.empty((H, W), np.uint8)
    if load().snxo_affine_labels(Dt, np.ascontiguousarray(lab, dtype=np.int32), W, H, int(ng),
                                 ms, a1, a2, d) != 0:
        raise ValueError("oracle affine_labels: bad arguments")
    return a1, a2, d.astype(bool)


POINT_DEFINED = 1


def compact_points(records):
    """The compacted oriented point cloud: the records whose flags hold the
    defined bit, in raster order.  records: [H, W, 8] float32 (x, y, z, nx, ny,
    nz, label bits, flag bits); returns [n, 8] float32."""
    r = np.ascontiguousarray(records, dtype=np.float32).reshape(-1, 8)
    flags = r[:, 7].view(np.uint32)
    return r[(flags & POINT_DEFINED) != 0]


STOP_CD, STOP_ST = 0, 1


def _fxb(cam):
    """f_x * baseline in binary64 from the float32 camera fields."""
    if cam is None:
        return 1.0
    return float(np.float32(cam.fx)) * float(np.float32(cam.baseline))


def star_mask(Dt, u: int, v: int, dirs: int = 8, steps: int = 10, stop: int = STOP_CD,
              thr: float = 0.05, cam=None):
    """Support of the star-fill at pixel (u, v) as a (2s+1)^2 boolean array
    indexed [dy + s, dx + s] (centre not marked), or None for an invalid centre."""
    Dt = _as_f64(Dt)
    H, W = Dt.shape
    side = 2 * steps + 1
    m = np.zeros(side * side, np.uint8)
    n = load().snxo_star_mask(Dt, W, H, int(u), int(v), int(dirs), int(steps), int(stop),
                              float(thr), _fxb(cam), m)
    if n < 0:
        return None
    return m.reshape(side, side).astype(bool)


def star_affine(Dt, dirs: int = 8, steps: int = 10, stop: int = STOP_CD, thr: float = 0.05,
                cam=None, min_support: int = 0):
    """a1, a2 and definedness over the star-fill support; min_support <= 0
    selects the default (the number of directions)."""
    Dt = _as_f64(Dt)
    H, W = Dt.shape
    ms = int(dirs) if min_support <= 0 else int(min_support)
    a1 = np.empty_like(Dt)
    a2 = np.empty_like(Dt)
    d = np.empty((H, W), np.uint8)
    if load().snxo_star_affine(Dt, W, H, int(dirs), int(steps), int(stop), float(thr),
                               _fxb(cam), ms, a1, a2, d) != 0:
        raise ValueError("oracle star_affine: bad arguments")
    return a1, a2, d.astype(bool)


def pipeline(D, cam, nf: int = 3, ng: int = 9, min_support_f: int = 0,
             min_support_g: int | None = None, k_rel: float = 0.1,
             t_abs: float = 1.0) -> dict:
    """Every stage in the paper's order on one float32 disparity map."""
    D32 = np.ascontiguousarray(D, dtype=np.float32)
    Dt = denoise(D32.astype(np.float64), nf, min_support_f)
    a1, a2, dfn = affine(Dt, ng, min_support_g)
    nrm = normals(Dt, a1, a2, dfn, cam)
    lab, ncomp = components(D32, k_rel, t_abs)
    pts = point_cloud(Dt, nrm, cam)
    return {"denoised": Dt, "a1": a1, "a2": a2, "defined": dfn, "normals": nrm,
            "labels": lab, "num_components": ncomp, "points": pts}
