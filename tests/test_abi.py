"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid arguments before any HIP call."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "snx.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(snx_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2504_15121_amd import _lib
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) == 36
    for n in names:
        assert hasattr(lib, n), n
    from paper_2504_15121_amd import _lib
    assert set(_lib.SIGNATURES) == set(names)


def test_status_strings(lib):
    assert lib.snx_status_string(0) == b"SNX_OK"
    assert lib.snx_status_string(3) == b"SNX_ERR_WORKSPACE"
    assert lib.snx_version() >= 100


def test_workspace_sizes(lib):
    assert lib.snx_components_workspace_size(640, 480) == 256 + 640 * 480 * 4
    assert lib.snx_pipeline_workspace_size(1920, 1080) >= 1920 * 1080 * 4
    assert lib.snx_components_workspace_size(1 << 16, 1 << 16) == 0   # too large


FAKE = C.c_void_p(0x1000)   # never dereferenced: every call below fails validation first


def _dn(window=3, mode=0):
    from paper_2504_15121_amd._lib import snx_denoise_params
    return snx_denoise_params(window, 0, mode, 0, None)


def _cam(fx=500.0, b=0.1):
    from paper_2504_15121_amd._lib import snx_camera
    return snx_camera(fx, fx, b, 10.0, 10.0)


@pytest.mark.parametrize("args,status", [
    (dict(disp=None), 1),
    (dict(stride=10), 1),
    (dict(window=4), 1),
    (dict(window=0), 1),
    (dict(window=65), 2),
    (dict(mode=1), 5),          # learned filter without a model
    (dict(mode=2), 2),
    (dict(w=-1), 1),
    (dict(w=70000, h=70000), 1),
])
def test_denoise_validation(lib, args, status):
    p = _dn(args.get("window", 3), args.get("mode", 0))
    disp = args.get("disp", FAKE)
    st = lib.snx_denoise(disp, args.get("stride", 64), FAKE, 64, args.get("w", 64),
                         args.get("h", 8), C.byref(p), None)
    assert st == status
    assert lib.snx_last_error() != b""


def test_empty_calls_are_ok(lib):
    p = _dn()
    assert lib.snx_denoise(None, 0, None, 0, 0, 5, C.byref(p), None) == 0
    assert lib.snx_denoise(None, 0, None, 0, 7, 0, C.byref(p), None) == 0


def test_affine_normals_validation(lib):
    from paper_2504_15121_amd._lib import snx_normal_params
    ok = snx_normal_params(9, 0)
    cam = _cam()
    assert lib.snx_affine_normals(FAKE, 64, 64, 8, C.byref(cam), C.byref(snx_normal_params(1, 0)),
                                  FAKE, FAKE, 64, None) == 1
    assert lib.snx_affine_normals(FAKE, 64, 64, 8, C.byref(_cam(fx=-1.0)), C.byref(ok),
                                  FAKE, FAKE, 64, None) == 1
    assert lib.snx_affine_normals(FAKE, 64, 64, 8, C.byref(_cam(b=float("nan"))), C.byref(ok),
                                  FAKE, FAKE, 64, None) == 1
    assert lib.snx_affine_normals(FAKE, 64, 64, 8, C.byref(cam), C.byref(ok),
                                  None, None, 64, None) == 1
    assert lib.snx_affine_normals(FAKE, 64, 64, 8, C.byref(cam), C.byref(ok),
                                  FAKE, FAKE, 32, None) == 1
    assert lib.snx_affine_normals(FAKE, 64, 64, 8, None, C.byref(ok), FAKE, FAKE, 64, None) == 1


def test_compact_validation(lib):
    cnt = FAKE
    # 256 bytes of alignment slack, then one int32 count per 4096-record chunk
    assert lib.snx_compact_points_workspace_size(1920, 1080) == 256 + 4 * ((1920 * 1080 + 4095) // 4096)
    ws = lib.snx_compact_points_workspace_size(64, 64)
    assert lib.snx_compact_points(FAKE, 64, 64, FAKE, None, FAKE, ws, None) == 1       # no count
    assert lib.snx_compact_points(None, 64, 64, FAKE, cnt, FAKE, ws, None) == 1
    assert lib.snx_compact_points(FAKE, 64, 64, FAKE, cnt, FAKE, ws, None) == 1        # overlap
    assert lib.snx_compact_points(FAKE, 64, 64, C.c_void_p(0x10000000), cnt, FAKE, ws - 1,
                                  None) == 3
    assert lib.snx_compact_points(FAKE, -1, 64, FAKE, cnt, FAKE, ws, None) == 1


def test_labels_validation(lib):
    from paper_2504_15121_amd._lib import snx_normal_params
    cam = _cam()
    ok = snx_normal_params(9, 0)

    def call(p=ok, lab=FAKE, ll=64, out=64, c=cam, aff=FAKE, nrm=FAKE, w=64):
        return lib.snx_affine_normals_labels(FAKE, 64, lab, ll, w, 8,
                                             C.byref(c) if c is not None else None,
                                             C.byref(p) if p is not None else None, aff, nrm, out,
                                             None)
    assert call(p=snx_normal_params(4, 0)) == 1       # even window
    assert call(p=snx_normal_params(65, 0)) != 0
    assert call(lab=None) == 1
    assert call(ll=32) == 1
    assert call(c=None) == 1
    assert call(aff=None, nrm=None) == 1
    assert call(out=32) == 1
    assert call(w=0) == 0                             # empty call


def test_star_validation(lib):
    from paper_2504_15121_amd._lib import snx_star_params
    cam = _cam()
    ok = snx_star_params(8, 10, 0, 0, 0.05)

    def call(p, w=64, h=8, aff=FAKE, nrm=FAKE, out=64, c=cam):
        return lib.snx_affine_normals_star(FAKE, 64, w, h, C.byref(c) if c is not None else None,
                                           C.byref(p) if p is not None else None, aff, nrm, out,
                                           None)
    assert call(snx_star_params(12, 10, 0, 0, 0.05)) == 2        # unsupported direction count
    assert call(snx_star_params(0, 10, 0, 0, 0.05)) == 1
    assert call(snx_star_params(8, 0, 0, 0, 0.05)) == 1
    assert call(snx_star_params(8, 33, 0, 0, 0.05)) == 1
    assert call(snx_star_params(8, 10, 2, 0, 0.05)) == 1
    assert call(snx_star_params(8, 10, 0, 0, -1.0)) == 1
    assert call(snx_star_params(8, 10, 1, 0, float("nan"))) == 1
    assert call(None) == 1
    assert call(ok, c=None) == 1
    assert call(ok, aff=None, nrm=None) == 1
    assert call(ok, out=32) == 1
    assert call(ok, w=0, h=0) == 0                                # empty call


def test_components_validation(lib):
    from paper_2504_15121_amd._lib import snx_component_params
    p = snx_component_params(0.1, 1.0)
    need = lib.snx_components_workspace_size(64, 8)
    assert lib.snx_components(FAKE, 64, 64, 8, C.byref(p), FAKE, 64, None, None, need, None) == 3
    assert lib.snx_components(FAKE, 64, 64, 8, C.byref(p), FAKE, 64, None, FAKE, need - 1,
                              None) == 3
    assert lib.snx_components(FAKE, 64, 64, 8, C.byref(snx_component_params(-0.1, 1.0)), FAKE,
                              64, None, FAKE, need, None) == 1
    assert lib.snx_components(FAKE, 64, 64, 8, C.byref(p), None, 64, None, FAKE, need, None) == 1
    assert lib.snx_components(FAKE, 64, 64, 8, C.byref(p), FAKE, 63, None, FAKE, need, None) == 1


def test_point_cloud_and_pipeline_validation(lib):
    from paper_2504_15121_amd._lib import snx_component_params, snx_normal_params
    cam = _cam()
    assert lib.snx_point_cloud(FAKE, 64, FAKE, 64, None, 0, 64, 8, C.byref(cam), None, None) == 1
    assert lib.snx_point_cloud(FAKE, 64, FAKE, 64, FAKE, 10, 64, 8, C.byref(cam), FAKE, None) == 1
    dn, nr, cp = _dn(), snx_normal_params(9, 0), snx_component_params(0.1, 1.0)
    need = lib.snx_pipeline_workspace_size(64, 8)
    args = [FAKE, 64, 64, 8, C.byref(cam), C.byref(dn), C.byref(nr), C.byref(cp), None, None,
            None, 64, FAKE, 64, None, FAKE, FAKE, need, None]
    bad = list(args)
    bad[15] = None                                  # points
    assert lib.snx_pipeline(*bad) == 1
    bad = list(args)
    bad[17] = need - 4                              # workspace too small
    assert lib.snx_pipeline(*bad) == 3
    bad = list(args)
    bad[6] = C.byref(snx_normal_params(2, 0))       # even window
    assert lib.snx_pipeline(*bad) == 1


def test_pipeline_part_validation(lib):
    from paper_2504_15121_amd._lib import snx_component_params, snx_normal_params
    cam = _cam()
    dn, nr, cp = _dn(), snx_normal_params(9, 0), snx_component_params(0.1, 1.0)
    need = lib.snx_pipeline_workspace_size(64, 8)
    assert need >= 256 + 2 * 64 * 8 * 4
    for parts in (0, 4, -1):
        assert lib.snx_pipeline_part(FAKE, 64, 64, 8, C.byref(cam), C.byref(dn), C.byref(nr),
                                     C.byref(cp), None, None, None, 64, FAKE, 64, None, FAKE,
                                     FAKE, need, parts, None) == 1


def test_autotune_validation(lib):
    from paper_2504_15121_amd._lib import snx_normal_params
    dn, nr = _dn(), snx_normal_params(9, 0)
    assert lib.snx_autotune(0, 10, C.byref(dn), C.byref(nr), None, None) == 1
    assert lib.snx_autotune(10, 10, C.byref(_dn(window=2)), C.byref(nr), None, None) == 1
    assert lib.snx_autotune(10, 10, C.byref(dn), C.byref(snx_normal_params(65, 0)), None, None) == 2


def test_tune_set(lib):
    assert lib.snx_tune_set(640, 480, 1, 9, 32) == 0      # compiled candidate
    assert lib.snx_tune_set(640, 480, 1, 9, 5) == 2       # not compiled
    assert lib.snx_tune_set(640, 480, 2, 9, 16) == 1      # even window
    assert lib.snx_tune_set(640, 480, 1, 9, 0) == 0       # clear


def test_cnn_sizes_and_validation(lib):
    assert lib.snx_cnn_param_count() == 37889
    assert lib.snx_cnn_packed_bytes() == 2 * 80384
    assert lib.snx_cnn_workspace_size(256, 256, 8, 1) > lib.snx_cnn_workspace_size(256, 256, 8, 0)
    assert lib.snx_cnn_workspace_size(0, 256, 1, 0) == 0
    assert lib.snx_cnn_pack(None, FAKE, None) == 1
    assert lib.snx_cnn_denoise(FAKE, 64, 64, 8, None, FAKE, 64, None) == 5
    from paper_2504_15121_amd._lib import snx_camera
    cams = (snx_camera * 1)(snx_camera(500.0, 500.0, 0.1, 10.0, 10.0))
    args = [FAKE, FAKE, None, C.c_float(0.0), C.cast(cams, C.c_void_p), 64, 64, 1, 9, FAKE,
            FAKE, FAKE, FAKE, FAKE, 1, C.c_float(1e-3), C.c_float(0.9), C.c_float(0.999),
            C.c_float(1e-8), FAKE, FAKE, 10, None]
    assert lib.snx_cnn_train_step(*args) == 3          # workspace too small
    bad = list(args); bad[8] = 4                         # even window
    assert lib.snx_cnn_train_step(*bad) == 1
    bad = list(args); bad[12] = None                     # Adam moments missing
    assert lib.snx_cnn_train_step(*bad) == 1
    bad = list(args); bad[3] = C.c_float(-1.0)           # negative fidelity weight
    assert lib.snx_cnn_train_step(*bad) == 1


def test_plan_validation(lib):
    from paper_2504_15121_amd._lib import (snx_component_params, snx_frame, snx_normal_params,
                                           snx_camera)
    out = C.c_void_p()
    cp = snx_component_params(0.1, 1.0)
    nr = snx_normal_params(9, 0)
    fr = (snx_frame * 1)(snx_frame(0x1000, 64, 64, 8, snx_camera(500.0, 500.0, 0.1, 3.0, 3.0),
                                   0, 0, 0x2000, 64, 0x3000, 0))
    assert lib.snx_plan_create(C.cast(fr, C.c_void_p), 0, C.byref(_dn()), C.byref(nr),
                               C.byref(cp), C.byref(out)) == 1                  # n < 1
    assert lib.snx_plan_create(C.cast(fr, C.c_void_p), 1, C.byref(_dn(window=5)), C.byref(nr),
                               C.byref(cp), C.byref(out)) == 2                  # window 5
    bad = (snx_frame * 1)(snx_frame(0x1000, 32, 64, 8, snx_camera(500.0, 500.0, 0.1, 3.0, 3.0),
                                    0, 0, 0x2000, 64, 0x3000, 0))
    assert lib.snx_plan_create(C.cast(bad, C.c_void_p), 1, C.byref(_dn()), C.byref(nr),
                               C.byref(cp), C.byref(out)) == 1                  # stride < width
    assert lib.snx_plan_run(None, None) == 1


def test_compact_noalloc_validation(lib):
    """The allocation-free compaction refuses frames over its static scratch
    (33 554 432 records) and bad arguments before any HIP call."""
    assert lib.snx_compact_points_noalloc(FAKE, 8192, 4097, C.c_void_p(0x900000000), FAKE,
                                          None) == 2
    assert b"allocation-free limit" in lib.snx_last_error()
    assert lib.snx_compact_points_noalloc(FAKE, 64, 8, FAKE, None, None) == 1     # no count
    assert lib.snx_compact_points_noalloc(None, 64, 8, FAKE, FAKE, None) == 1     # no points
    assert lib.snx_compact_points_noalloc(FAKE, -1, 8, FAKE, FAKE, None) == 1
    assert lib.snx_compact_points_noalloc(FAKE, 64, 8, FAKE, FAKE, None) == 1     # overlap


# ---------------------------------------------------------------- model files
def _model_file(tmp_path, moments=True, seed=3):
    import numpy as np
    from paper_2504_15121_amd import _lib
    n = _lib.snx_cnn_param_count()
    rng = np.random.default_rng(seed)
    p, m, v = (rng.normal(0, 1, n).astype(np.float32) for _ in range(3))
    path = str(tmp_path / "m.snxm")
    _lib.model_save(path, p, m if moments else None, v if moments else None, step=1234,
                    normal_window=9, seed=seed, fidelity=0.25)
    return path, p, m, v


@pytest.mark.parametrize("moments", [True, False])
def test_model_file_round_trip_and_layout(lib, tmp_path, moments):
    import struct
    import zlib
    import numpy as np
    from paper_2504_15121_amd import _lib
    path, p, m, v = _model_file(tmp_path, moments)
    raw = open(path, "rb").read()
    n = _lib.snx_cnn_param_count()
    assert len(raw) == 40 + (3 if moments else 1) * 4 * n + 4
    magic, ver, cnt, flags, step, ng, seed, fid, res = struct.unpack("<4sIIIqiifI", raw[:40])
    assert (magic, ver, cnt, flags, step, ng, seed, res) == (b"SNXM", 1, n, int(moments), 1234,
                                                             9, 3, 0)
    assert fid == np.float32(0.25)
    # the library's CRC-32 is zlib's
    assert struct.unpack("<I", raw[-4:])[0] == zlib.crc32(raw[:-4])
    assert np.array_equal(np.frombuffer(raw[40:40 + 4 * n], np.float32), p)
    st = _lib.model_load(path)
    assert np.array_equal(st["params"], p)
    if moments:
        assert np.array_equal(st["m"], m) and np.array_equal(st["v"], v)
    else:
        assert st["m"] is None and st["v"] is None
    assert (st["step"], st["normal_window"], st["seed"]) == (1234, 9, 3)
    assert not os.path.exists(path + ".tmp")       # written to .tmp, then renamed


def _status_of_load(lib, path):
    h = C.c_void_p(0x1234)
    st = lib.snx_model_load(os.fsencode(path), C.byref(h))
    if st == 0:
        lib.snx_model_destroy(h)
    else:
        assert h.value is None                     # no model on failure
    return st


def test_model_file_corruption_is_refused(lib, tmp_path):
    import struct
    import zlib
    path, _, _, _ = _model_file(tmp_path)
    raw = open(path, "rb").read()
    bad = str(tmp_path / "bad.snxm")

    def status(data):
        open(bad, "wb").write(data)
        return _status_of_load(lib, bad)

    assert status(raw) == 0
    for cut in (0, 3, 39, 40, 44, len(raw) // 2, len(raw) - 5, len(raw) - 1):
        assert status(raw[:cut]) == 5, cut                       # truncated
    assert status(raw + b"\0") == 5                               # trailing bytes
    flip = bytearray(raw)
    flip[40 + 1000] ^= 0x10
    assert status(bytes(flip)) == 5                               # CRC
    assert b"CRC" in lib.snx_last_error()
    assert status(b"SNXX" + raw[4:]) == 5                         # magic

    def with_header(off, fmt, val):
        b = bytearray(raw)
        struct.pack_into(fmt, b, off, val)
        struct.pack_into("<I", b, len(b) - 4, zlib.crc32(bytes(b[:-4])))
        return bytes(b)

    assert status(with_header(4, "<I", 2)) == 5                   # version
    assert status(with_header(8, "<I", 100)) == 5                 # parameter count
    assert status(with_header(12, "<I", 2)) == 5                  # unknown flag
    assert status(with_header(12, "<I", 0)) == 5                  # size disagrees with flags
    assert _status_of_load(lib, str(tmp_path / "missing.snxm")) == 6
    assert lib.snx_model_save(None, os.fsencode(bad)) == 1


def test_model_read_without_moments(lib, tmp_path):
    path, _, _, _ = _model_file(tmp_path, moments=False)
    h = C.c_void_p()
    assert lib.snx_model_load(os.fsencode(path), C.byref(h)) == 0
    buf = (C.c_float * 64)()
    assert lib.snx_model_read(h, None, buf, buf, None) == 5
    assert lib.snx_model_destroy(h) == 0
    assert lib.snx_model_destroy(None) == 0


def test_committed_model_loads():
    from paper_2504_15121_amd import learned
    st = learned.load_checkpoint(learned.DEFAULT_MODEL)
    assert st["m"] is not None and st["step"] > 0 and st["normal_window"] == 9
