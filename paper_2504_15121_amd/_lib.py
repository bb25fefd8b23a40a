"""ctypes binding of libsnx.so: argument marshalling only.

Every function here has the name of the C entry point it calls and forwards
torch device tensors as raw pointers plus strides; all computation happens in the
HIP kernels.  The library must have been built (``__graft_entry__.build()``);
there is no fallback of any kind: a missing library raises at load time.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsnx.so")

SNX_OK = 0
STATUS = {0: "SNX_OK", 1: "SNX_ERR_ARG", 2: "SNX_ERR_UNSUPPORTED", 3: "SNX_ERR_WORKSPACE",
          4: "SNX_ERR_HIP", 5: "SNX_ERR_MODEL", 6: "SNX_ERR_IO"}

POINT_DEFINED = 1
POINT_LABELLED = 2


class SnxError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class snx_camera(C.Structure):
    _fields_ = [("fx", C.c_float), ("fy", C.c_float), ("baseline", C.c_float),
                ("u0", C.c_float), ("v0", C.c_float)]


class snx_denoise_params(C.Structure):
    _fields_ = [("window", C.c_int32), ("min_support", C.c_int32), ("mode", C.c_int32),
                ("reserved", C.c_int32), ("model", C.c_void_p)]


class snx_cnn_model(C.Structure):
    _fields_ = [("params", C.c_void_p), ("packed", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t)]


class snx_model_info(C.Structure):
    _fields_ = [("step", C.c_int64), ("normal_window", C.c_int32), ("seed", C.c_int32),
                ("fidelity", C.c_float), ("has_moments", C.c_int32)]


class snx_frame(C.Structure):
    _fields_ = [("disp", C.c_void_p), ("stride", C.c_int64), ("width", C.c_int32),
                ("height", C.c_int32), ("cam", snx_camera), ("disp_dn", C.c_void_p),
                ("dn_stride", C.c_int64), ("labels", C.c_void_p), ("label_stride", C.c_int64),
                ("points", C.c_void_p), ("num_components", C.c_void_p)]


class snx_normal_params(C.Structure):
    _fields_ = [("window", C.c_int32), ("min_support", C.c_int32)]


class snx_star_params(C.Structure):
    _fields_ = [("directions", C.c_int32), ("steps", C.c_int32), ("stop", C.c_int32),
                ("min_support", C.c_int32), ("threshold", C.c_double)]


STOP_CD, STOP_ST = 0, 1


class snx_component_params(C.Structure):
    _fields_ = [("k_rel", C.c_float), ("t_abs", C.c_float)]


_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32
_SZ = C.c_size_t

SIGNATURES = {
    "snx_denoise": (_I32, [_P, _I64, _P, _I64, _I32, _I32, C.POINTER(snx_denoise_params), _P]),
    "snx_affine_normals": (_I32, [_P, _I64, _I32, _I32, C.POINTER(snx_camera),
                                  C.POINTER(snx_normal_params), _P, _P, _I64, _P]),
    "snx_components_creases": (_I32, [_P, _I64, _P, _I64, _I32, _I32,
                                      C.POINTER(snx_component_params), C.c_double, _P, _I64, _P,
                                      _P, _SZ, _P]),
    "snx_compact_points_workspace_size": (_SZ, [_I32, _I32]),
    "snx_compact_points": (_I32, [_P, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "snx_affine_normals_labels": (_I32, [_P, _I64, _P, _I64, _I32, _I32, C.POINTER(snx_camera),
                                         C.POINTER(snx_normal_params), _P, _P, _I64, _P]),
    "snx_affine_normals_star": (_I32, [_P, _I64, _I32, _I32, C.POINTER(snx_camera),
                                       C.POINTER(snx_star_params), _P, _P, _I64, _P]),
    "snx_components_workspace_size": (_SZ, [_I32, _I32]),
    "snx_components": (_I32, [_P, _I64, _I32, _I32, C.POINTER(snx_component_params), _P, _I64,
                              _P, _P, _SZ, _P]),
    "snx_point_cloud": (_I32, [_P, _I64, _P, _I64, _P, _I64, _I32, _I32, C.POINTER(snx_camera),
                               _P, _P]),
    "snx_oriented_point_cloud": (_I32, [_P, _I64, _I32, _I32, C.POINTER(snx_camera),
                                        C.POINTER(snx_denoise_params),
                                        C.POINTER(snx_normal_params), _P, _I64, _P, _P, _P,
                                        _I64, _P, _P]),
    "snx_pipeline_workspace_size": (_SZ, [_I32, _I32]),
    "snx_pipeline": (_I32, [_P, _I64, _I32, _I32, C.POINTER(snx_camera),
                            C.POINTER(snx_denoise_params), C.POINTER(snx_normal_params),
                            C.POINTER(snx_component_params), _P, _P, _P, _I64, _P, _I64, _P, _P,
                            _P, _SZ, _P]),
    "snx_pipeline_part": (_I32, [_P, _I64, _I32, _I32, C.POINTER(snx_camera),
                                 C.POINTER(snx_denoise_params), C.POINTER(snx_normal_params),
                                 C.POINTER(snx_component_params), _P, _P, _P, _I64, _P, _I64,
                                 _P, _P, _P, _SZ, _I32, _P]),
    "snx_autotune": (_I32, [_I32, _I32, C.POINTER(snx_denoise_params),
                            C.POINTER(snx_normal_params), _P, _P]),
    "snx_tune_set": (_I32, [_I32, _I32, _I32, _I32, _I32]),
    "snx_cnn_param_count": (_I32, []),
    "snx_cnn_packed_bytes": (_SZ, []),
    "snx_cnn_workspace_size": (_SZ, [_I32, _I32, _I32, _I32]),
    "snx_cnn_pack": (_I32, [_P, _P, _P]),
    "snx_cnn_denoise": (_I32, [_P, _I64, _I32, _I32, _P, _P, _I64, _P]),
    "snx_cnn_train_step": (_I32, [_P, _P, _P, C.c_float, _P, _I32, _I32, _I32, _I32, _P, _P,
                                  _P, _P, _P, _I32, C.c_float, C.c_float, C.c_float, C.c_float,
                                  _P, _P, _SZ, _P]),
    "snx_components_from_edges": (_I32, [_P, _I64, _I32, _I32, _P, _I64, _P, _P, _SZ, _P]),
    "snx_compact_points_noalloc": (_I32, [_P, _I32, _I32, _P, _P, _P]),
    "snx_model_create": (_I32, [_P, _P, _P, C.POINTER(snx_model_info), C.POINTER(C.c_void_p)]),
    "snx_model_load": (_I32, [C.c_char_p, C.POINTER(C.c_void_p)]),
    "snx_model_save": (_I32, [_P, C.c_char_p]),
    "snx_model_read": (_I32, [_P, _P, _P, _P, C.POINTER(snx_model_info)]),
    "snx_model_bind": (_I32, [_P, _I32, _I32, _P, C.POINTER(snx_cnn_model)]),
    "snx_model_destroy": (_I32, [_P]),
    "snx_plan_create": (_I32, [_P, _I32, C.POINTER(snx_denoise_params),
                               C.POINTER(snx_normal_params), C.POINTER(snx_component_params),
                               C.POINTER(C.c_void_p)]),
    "snx_plan_run": (_I32, [_P, _P]),
    "snx_plan_destroy": (_I32, [_P]),
    "snx_status_string": (C.c_char_p, [_I32]),
    "snx_last_error": (C.c_char_p, []),
    "snx_version": (_I32, []),
}

_lib = None


def load():
    """Load libsnx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first "
                          "(there is no non-HIP fallback)")
    # torch brings its own HIP runtime; load it first so that libsnx binds to the
    # same runtime instance that owns the tensors' memory and streams
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != SNX_OK:
        raise SnxError(status, load().snx_last_error().decode())


_current_raw_stream = None


def _stream(stream):
    """The raw HIP stream handle: the given stream, else torch's current stream
    (read without building a Stream object: this runs on every call)."""
    global _current_raw_stream
    if stream is None:
        if _current_raw_stream is None:
            import torch
            raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
            if raw is not None:
                dev = torch.cuda.current_device
                _current_raw_stream = lambda: raw(dev())
            else:
                _current_raw_stream = lambda: torch.cuda.current_stream().cuda_stream
        return _current_raw_stream()
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def _img(t, dtype, name):
    import torch
    if t.dtype != dtype or t.dim() != 2 or not t.is_cuda or t.stride(1) != 1:
        raise ValueError(f"{name}: need a CUDA {dtype} (H, W) tensor with unit column stride")
    return t.stride(0)


def _planes(t, n, H, W, name):
    import torch
    if t is None:
        return None
    if (t.dtype != torch.float32 or t.dim() != 3 or t.shape[0] != n or t.shape[1] != H
            or t.shape[2] < W or not t.is_cuda or t.stride(2) != 1
            or t.stride(0) != t.shape[1] * t.stride(1)):
        raise ValueError(f"{name}: need a CUDA float32 ({n}, H, S) plane tensor, S >= W")
    return t.stride(1)


def _dense(t, dtype, shape, name):
    """Pointer of a contiguous CUDA tensor of the given dtype and shape (None = any size)."""
    if (t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.dim() != len(shape)
            or any(s is not None and s != d for s, d in zip(shape, t.shape))):
        want = "x".join("?" if s is None else str(s) for s in shape)
        raise ValueError(f"{name}: need a contiguous CUDA {dtype} tensor of shape {want}, "
                         f"got {t.dtype} {tuple(t.shape)} strides {t.stride()}")
    return t.data_ptr()


def camera(cam) -> snx_camera:
    """snx_camera from anything with fx, fy, baseline, u0, v0 attributes."""
    return snx_camera(cam.fx, cam.fy, cam.baseline, cam.u0, cam.v0)


def snx_denoise(disp, out, window=3, min_support=0, stream=None):
    H, W = disp.shape
    p = snx_denoise_params(window, min_support, 0, 0, None)
    _check(load().snx_denoise(_ptr(disp), _img(disp, disp.dtype, "disp"), _ptr(out),
                              _img(out, disp.dtype, "out"), W, H, C.byref(p), _stream(stream)))


def snx_affine_normals(disp_dn, cam, affine=None, normals=None, window=9, min_support=0,
                       stream=None):
    import torch
    H, W = disp_dn.shape
    ld = _img(disp_dn, torch.float32, "disp_dn")
    la = _planes(affine, 2, H, W, "affine")
    ln = _planes(normals, 3, H, W, "normals")
    if la is not None and ln is not None and la != ln:
        raise ValueError("affine and normals must share one row stride")
    out_ld = la if la is not None else (ln if ln is not None else W)
    p = snx_normal_params(window, min_support)
    c = camera(cam)
    _check(load().snx_affine_normals(_ptr(disp_dn), ld, W, H, C.byref(c), C.byref(p),
                                     _ptr(affine), _ptr(normals), out_ld, _stream(stream)))


def snx_components_creases(disp, normals, labels, workspace, num_components=None, k_rel=0.1,
                           t_abs=1.0, crease_cos=0.9, stream=None):
    """Components whose edges pass covered depth and n_p . n_q >= crease_cos."""
    import torch
    H, W = disp.shape
    ln = _planes(normals, 3, H, W, "normals")
    p = snx_component_params(k_rel, t_abs)
    _check(load().snx_components_creases(_ptr(disp), _img(disp, torch.float32, "disp"),
                                         _ptr(normals), ln if ln is not None else W, W, H,
                                         C.byref(p), float(crease_cos), _ptr(labels),
                                         _img(labels, torch.int32, "labels"), _ptr(num_components),
                                         _ptr(workspace),
                                         workspace.numel() * workspace.element_size(),
                                         _stream(stream)))


def snx_compact_points_workspace_size(width, height):
    return int(load().snx_compact_points_workspace_size(width, height))


def snx_compact_points(points, out, count, workspace, stream=None):
    """Defined records of `points` ([H, W, 8] float32 records, contiguous)
    packed into `out` (at least H*W records, contiguous) in raster order; the
    number goes to `count` (int32 device tensor)."""
    import torch
    if points.dim() != 3 or points.shape[2] != 8 or points.dtype != torch.float32:
        raise ValueError("points must be [H, W, 8] float32 records")
    if not points.is_contiguous() or not out.is_contiguous():
        raise ValueError("points and out must be contiguous")
    H, W = points.shape[0], points.shape[1]
    if out.dtype != torch.float32 or out.numel() < H * W * 8:
        raise ValueError("out must be float32 with room for H*W records")
    if count.dtype != torch.int32 or count.numel() < 1:
        raise ValueError("count must be an int32 tensor")
    for t in (points, out, count, workspace):
        if t.device.type != "cuda":
            raise ValueError("tensors must be on the GPU")
    _check(load().snx_compact_points(_ptr(points), W, H, _ptr(out), _ptr(count), _ptr(workspace),
                                     workspace.numel() * workspace.element_size(),
                                     _stream(stream)))


def snx_compact_points_noalloc(points, out, count, stream=None):
    """snx_compact_points without a workspace: the library's own static device
    scratch (allocates nothing; frames up to 33 554 432 records; calls that
    overlap on one GPU race)."""
    import torch
    if points.dim() != 3 or points.shape[2] != 8 or points.dtype != torch.float32:
        raise ValueError("points must be [H, W, 8] float32 records")
    if not points.is_contiguous() or not out.is_contiguous():
        raise ValueError("points and out must be contiguous")
    H, W = points.shape[0], points.shape[1]
    if out.dtype != torch.float32 or out.numel() < H * W * 8:
        raise ValueError("out must be float32 with room for H*W records")
    if count.dtype != torch.int32 or count.numel() < 1:
        raise ValueError("count must be an int32 tensor")
    for t in (points, out, count):
        if t.device.type != "cuda":
            raise ValueError("tensors must be on the GPU")
    _check(load().snx_compact_points_noalloc(_ptr(points), W, H, _ptr(out), _ptr(count),
                                             _stream(stream)))


def snx_affine_normals_labels(disp_dn, labels, cam, affine=None, normals=None, window=9,
                              min_support=0, stream=None):
    """Gradients, A and normals over the window restricted to the centre's component."""
    import torch
    H, W = disp_dn.shape
    ld = _img(disp_dn, torch.float32, "disp_dn")
    ll = _img(labels, torch.int32, "labels")
    if tuple(labels.shape) != (H, W):
        raise ValueError("labels must have the shape of disp_dn")
    la = _planes(affine, 2, H, W, "affine")
    ln = _planes(normals, 3, H, W, "normals")
    if la is not None and ln is not None and la != ln:
        raise ValueError("affine and normals must share one row stride")
    out_ld = la if la is not None else (ln if ln is not None else W)
    p = snx_normal_params(window, min_support)
    c = camera(cam)
    _check(load().snx_affine_normals_labels(_ptr(disp_dn), ld, _ptr(labels), ll, W, H,
                                            C.byref(c), C.byref(p), _ptr(affine), _ptr(normals),
                                            out_ld, _stream(stream)))


def snx_affine_normals_star(disp_dn, cam, affine=None, normals=None, directions=8, steps=10,
                            stop=STOP_CD, threshold=0.05, min_support=0, stream=None):
    """Gradients, A and normals over the adaptive star-fill support."""
    import torch
    H, W = disp_dn.shape
    ld = _img(disp_dn, torch.float32, "disp_dn")
    la = _planes(affine, 2, H, W, "affine")
    ln = _planes(normals, 3, H, W, "normals")
    if la is not None and ln is not None and la != ln:
        raise ValueError("affine and normals must share one row stride")
    out_ld = la if la is not None else (ln if ln is not None else W)
    p = snx_star_params(directions, steps, stop, min_support, threshold)
    c = camera(cam)
    _check(load().snx_affine_normals_star(_ptr(disp_dn), ld, W, H, C.byref(c), C.byref(p),
                                          _ptr(affine), _ptr(normals), out_ld, _stream(stream)))


def snx_components_workspace_size(width, height):
    return int(load().snx_components_workspace_size(width, height))


def snx_components(disp, labels, workspace, num_components=None, k_rel=0.1, t_abs=1.0,
                   stream=None):
    import torch
    H, W = disp.shape
    p = snx_component_params(k_rel, t_abs)
    _check(load().snx_components(_ptr(disp), _img(disp, torch.float32, "disp"), W, H,
                                 C.byref(p), _ptr(labels), _img(labels, torch.int32, "labels"),
                                 _ptr(num_components), _ptr(workspace),
                                 workspace.numel() * workspace.element_size(), _stream(stream)))


def snx_components_from_edges(edges, labels, workspace, num_components=None, stream=None):
    """Components of the 4-neighbour graph given by per-pixel bits (uint8 (H, W):
    bit 0 present, bit 1 edge left, bit 2 edge up); the labelling's test hook."""
    import torch
    H, W = edges.shape
    _check(load().snx_components_from_edges(
        _ptr(edges), _img(edges, torch.uint8, "edges"), W, H, _ptr(labels),
        _img(labels, torch.int32, "labels"), _ptr(num_components), _ptr(workspace),
        workspace.numel() * workspace.element_size(), _stream(stream)))


def _points(t, H, W):
    if t.numel() * t.element_size() < H * W * 32 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("points: need a contiguous CUDA buffer of width*height*32 bytes")


def snx_point_cloud(disp_dn, normals, labels, cam, out, stream=None):
    import torch
    H, W = disp_dn.shape
    ld = _img(disp_dn, torch.float32, "disp_dn")
    ln = _planes(normals, 3, H, W, "normals")
    ll = _img(labels, torch.int32, "labels") if labels is not None else 0
    _points(out, H, W)
    c = camera(cam)
    _check(load().snx_point_cloud(_ptr(disp_dn), ld, _ptr(normals), ln, _ptr(labels), ll, W, H,
                                  C.byref(c), _ptr(out), _stream(stream)))


def _out_stride(disp_dn, affine, normals, H, W):
    import torch
    lds = []
    if disp_dn is not None:
        lds.append(_img(disp_dn, torch.float32, "disp_dn"))
    for t, n, name in ((affine, 2, "affine"), (normals, 3, "normals")):
        if t is not None:
            lds.append(_planes(t, n, H, W, name))
    if len(set(lds)) > 1:
        raise ValueError("disp_dn, affine and normals must share one row stride")
    return lds[0] if lds else W


def snx_oriented_point_cloud(disp, cam, points, labels=None, disp_dn=None, affine=None,
                             normals=None, filter_window=3, filter_min_support=0,
                             normal_window=9, normal_min_support=0, stream=None):
    import torch
    H, W = disp.shape
    ld = _img(disp, torch.float32, "disp")
    out_ld = _out_stride(disp_dn, affine, normals, H, W)
    ll = _img(labels, torch.int32, "labels") if labels is not None else 0
    _points(points, H, W)
    dp = snx_denoise_params(filter_window, filter_min_support, 0, 0, None)
    np_ = snx_normal_params(normal_window, normal_min_support)
    c = camera(cam)
    _check(load().snx_oriented_point_cloud(_ptr(disp), ld, W, H, C.byref(c), C.byref(dp),
                                           C.byref(np_), _ptr(labels), ll, _ptr(disp_dn),
                                           _ptr(affine), _ptr(normals), out_ld, _ptr(points),
                                           _stream(stream)))


def snx_pipeline_workspace_size(width, height):
    return int(load().snx_pipeline_workspace_size(width, height))


PART_FOREST = 1
PART_POINTS = 2


def snx_pipeline_part(disp, cam, labels, points, workspace, parts=3, num_components=None,
                      disp_dn=None, affine=None, normals=None, filter_window=3,
                      filter_min_support=0, normal_window=9, normal_min_support=0, k_rel=0.1,
                      t_abs=1.0, stream=None, cnn=None):
    """cnn: None (LSQ filter) or an snx_cnn_model (learned filter)."""
    import torch
    H, W = disp.shape
    ld = _img(disp, torch.float32, "disp")
    out_ld = _out_stride(disp_dn, affine, normals, H, W)
    _points(points, H, W)
    dp = snx_denoise_params(filter_window, filter_min_support, 0 if cnn is None else 1, 0,
                            None if cnn is None else C.cast(C.pointer(cnn), C.c_void_p))
    np_ = snx_normal_params(normal_window, normal_min_support)
    cp = snx_component_params(k_rel, t_abs)
    c = camera(cam)
    _check(load().snx_pipeline_part(_ptr(disp), ld, W, H, C.byref(c), C.byref(dp), C.byref(np_),
                                    C.byref(cp), _ptr(disp_dn), _ptr(affine), _ptr(normals),
                                    out_ld, _ptr(labels), _img(labels, torch.int32, "labels"),
                                    _ptr(num_components), _ptr(points), _ptr(workspace),
                                    workspace.numel() * workspace.element_size(), int(parts),
                                    _stream(stream)))


def snx_pipeline(disp, cam, labels, points, workspace, num_components=None, disp_dn=None,
                 affine=None, normals=None, filter_window=3, filter_min_support=0,
                 normal_window=9, normal_min_support=0, k_rel=0.1, t_abs=1.0, stream=None,
                 cnn=None):
    snx_pipeline_part(disp, cam, labels, points, workspace, 3, num_components, disp_dn, affine,
                      normals, filter_window, filter_min_support, normal_window,
                      normal_min_support, k_rel, t_abs, stream, cnn)


def snx_autotune(width, height, filter_window=3, normal_window=9, filter_min_support=0,
                 normal_min_support=0, stream=None):
    """Returns the tile heights chosen (fused, gradient-only)."""
    dp = snx_denoise_params(filter_window, filter_min_support, 0, 0, None)
    np_ = snx_normal_params(normal_window, normal_min_support)
    out = (C.c_int32 * 2)()
    _check(load().snx_autotune(width, height, C.byref(dp), C.byref(np_), C.cast(out, C.c_void_p),
                               _stream(stream)))
    return int(out[0]), int(out[1])


def snx_tune_set(width, height, filter_window, normal_window, tile_height):
    _check(load().snx_tune_set(width, height, filter_window, normal_window, tile_height))


FILTER_LSQ = 0
FILTER_CNN = 1


def snx_cnn_param_count():
    return int(load().snx_cnn_param_count())


def snx_cnn_packed_bytes():
    return int(load().snx_cnn_packed_bytes())


def snx_cnn_workspace_size(width, height, batch=1, training=False):
    return int(load().snx_cnn_workspace_size(width, height, batch, int(bool(training))))


def _params(t, name="params"):
    import torch
    return _dense(t, torch.float32, (snx_cnn_param_count(),), name)


def _packed(t):
    if not t.is_cuda or not t.is_contiguous() or t.numel() * t.element_size() < snx_cnn_packed_bytes():
        raise ValueError(f"packed: need a contiguous CUDA buffer of {snx_cnn_packed_bytes()} bytes")
    return t.data_ptr()


def snx_cnn_pack(params, packed, stream=None):
    _check(load().snx_cnn_pack(_params(params), _packed(packed), _stream(stream)))


def cnn_model(params, packed, workspace):
    """snx_cnn_model for the C calls (keep the returned object alive)."""
    if not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace: need a contiguous CUDA buffer")
    return snx_cnn_model(_params(params), _packed(packed), workspace.data_ptr(),
                         workspace.numel() * workspace.element_size())


def snx_cnn_denoise(disp, model, out, stream=None):
    import torch
    H, W = disp.shape
    _check(load().snx_cnn_denoise(_ptr(disp), _img(disp, torch.float32, "disp"), W, H,
                                  C.byref(model), _ptr(out), _img(out, torch.float32, "out"),
                                  _stream(stream)))


def snx_cnn_train_step(disp, normals, cams, params, packed, grad, adam_m, adam_v, step, lr,
                       loss_out, workspace, normal_window=9, beta1=0.9, beta2=0.999, eps=1e-8,
                       stream=None, clean=None, fidelity=0.0):
    """disp (B, H, W) and normals (B, 3, H, W) device float32; cams: list of objects with
    fx, fy, baseline, u0, v0; loss_out device float64[4]; clean (B, H, W) float32 or None."""
    import torch
    B, H, W = disp.shape
    if len(cams) != B:
        raise ValueError("one camera per batch item")
    carr = (snx_camera * B)(*[camera(c) for c in cams])
    if not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace: need a contiguous CUDA buffer")
    _check(load().snx_cnn_train_step(
        _dense(disp, torch.float32, (B, H, W), "disp"),
        _dense(normals, torch.float32, (B, 3, H, W), "normals"),
        None if clean is None else _dense(clean, torch.float32, (B, H, W), "clean"),
        float(fidelity), C.cast(carr, C.c_void_p),
        W, H, B, normal_window, _params(params), _packed(packed), _params(grad, "grad"),
        None if adam_m is None else _params(adam_m, "adam_m"),
        None if adam_v is None else _params(adam_v, "adam_v"), int(step),
        float(lr), float(beta1), float(beta2), float(eps),
        _dense(loss_out, torch.float64, (4,), "loss_out"), workspace.data_ptr(),
        workspace.numel() * workspace.element_size(), _stream(stream)))


def model_save(path, params, adam_m=None, adam_v=None, step=0, normal_window=0, seed=0,
               fidelity=0.0):
    """Writes a model file (snx_model_create + snx_model_save) from host float32
    arrays of snx_cnn_param_count() values; the moments both or neither."""
    import numpy as np
    n = snx_cnn_param_count()
    arrs = []
    for a in (params, adam_m, adam_v):
        if a is None:
            arrs.append(None)
            continue
        a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
        if a.size != n:
            raise ValueError(f"need {n} values, got {a.size}")
        arrs.append(a)
    info = snx_model_info(int(step), int(normal_window), int(seed), float(fidelity), 0)
    h = C.c_void_p()
    lib = load()
    _check(lib.snx_model_create(*[None if a is None else a.ctypes.data for a in arrs],
                                C.byref(info), C.byref(h)))
    try:
        _check(lib.snx_model_save(h, os.fsencode(path)))
    finally:
        lib.snx_model_destroy(h)


def model_load(path):
    """Reads a model file (snx_model_load + snx_model_read): dict with params, m,
    v (None without Adam state), step, normal_window, seed, fidelity."""
    import numpy as np
    lib = load()
    h = C.c_void_p()
    _check(lib.snx_model_load(os.fsencode(path), C.byref(h)))
    try:
        n = snx_cnn_param_count()
        info = snx_model_info()
        _check(lib.snx_model_read(h, None, None, None, C.byref(info)))
        p = np.empty(n, np.float32)
        m = np.empty(n, np.float32) if info.has_moments else None
        v = np.empty(n, np.float32) if info.has_moments else None
        _check(lib.snx_model_read(h, p.ctypes.data, None if m is None else m.ctypes.data,
                                  None if v is None else v.ctypes.data, None))
    finally:
        lib.snx_model_destroy(h)
    return dict(params=p, m=m, v=v, step=int(info.step), normal_window=int(info.normal_window),
                seed=int(info.seed), fidelity=float(info.fidelity))


class Plan:
    """A batch plan over frames given as dicts of device tensors:
    disp (H, W) f32, cam, labels (H, W) int32, points (H, W, 8) f32, optional
    disp_dn (H, W) f32 and num_components (1,) int32.  Keep the tensors alive."""

    def __init__(self, frames, filter_window=3, normal_window=9, k_rel=0.1, t_abs=1.0,
                 cnn=None, normal_min_support=0):
        import torch
        arr = (snx_frame * len(frames))()
        for i, f in enumerate(frames):
            d = f["disp"]
            H, W = d.shape
            _points(f["points"], H, W)
            dn = f.get("disp_dn")
            arr[i] = snx_frame(d.data_ptr(), _img(d, torch.float32, "disp"), W, H,
                               camera(f["cam"]), 0 if dn is None else dn.data_ptr(),
                               0 if dn is None else _img(dn, torch.float32, "disp_dn"),
                               f["labels"].data_ptr(), _img(f["labels"], torch.int32, "labels"),
                               f["points"].data_ptr(),
                               0 if f.get("num_components") is None else
                               f["num_components"].data_ptr())
        self._model = cnn
        dp = snx_denoise_params(filter_window, 0, 0 if cnn is None else 1, 0,
                                None if cnn is None else C.cast(C.pointer(cnn), C.c_void_p))
        np_ = snx_normal_params(normal_window, normal_min_support)
        cp = snx_component_params(k_rel, t_abs)
        h = C.c_void_p()
        _check(load().snx_plan_create(C.cast(arr, C.c_void_p), len(frames), C.byref(dp),
                                      C.byref(np_), C.byref(cp), C.byref(h)))
        self.handle = h

    def run(self, stream=None):
        _check(load().snx_plan_run(self.handle, _stream(stream)))

    def close(self):
        if self.handle:
            load().snx_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
