"""GPU parity of crease-aware components: covered depth plus the normal-crease
test on every 4-neighbour edge, bit-exact labels and counts against the
oracle's flood fill with the same float32 normals on both sides."""
import numpy as np
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NAN = float("nan")


def _snx():
    import paper_2504_15121_amd as snx
    snx.load()
    return snx


def _run(snx, D, N, cos, pad=0, k=0.1, t=1.0):
    H, W = D.shape
    d = torch.from_numpy(np.ascontiguousarray(D, np.float32)).to(DEV)
    n = torch.full((3, H, W + pad), NAN, device=DEV)
    n[:, :, :W] = torch.from_numpy(np.ascontiguousarray(N, np.float32))
    lab = torch.full((H, W), -9, dtype=torch.int32, device=DEV)
    cnt = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    ws = torch.empty(snx.snx_components_workspace_size(W, H), dtype=torch.uint8, device=DEV)
    snx.snx_components_creases(d, n, lab, ws, num_components=cnt, k_rel=k, t_abs=t,
                               crease_cos=cos)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), int(cnt.item())


def _gpu_normals(snx, D, cam):
    H, W = D.shape
    dn = torch.empty((H, W), device=DEV)
    nrm = torch.empty((3, H, W), device=DEV)
    snx.snx_denoise(torch.from_numpy(D).to(DEV), dn, window=3)
    snx.snx_affine_normals(dn, cam, normals=nrm, window=9)
    torch.cuda.synchronize()
    return nrm.cpu().numpy()


@pytest.mark.parametrize("W,H,cos,pad", [(200, 150, 0.9, 0), (130, 70, 0.99, 3), (70, 37, 0.5, 0),
                                         (1920, 1080, 0.95, 0), (64, 32, 0.9, 0), (1, 1, 0.9, 0),
                                         (129, 65, -1.0, 1)])
def test_crease_components_match_oracle(oracle, W, H, cos, pad):
    snx = _snx()
    print(f"case crease components {W}x{H} cos {cos} pad {pad}", flush=True)
    if (W, H) == (1920, 1080):
        sc = scenes.workload("planes_quadrics_1920x1080")
    else:
        sc = scenes.planes_quadrics_scene(width=max(W, 8), height=max(H, 8), f=300.0,
                                          n_planes=8, n_spheres=2, seed=W * 3 + H)
    D = np.ascontiguousarray(sc.disp[:H, :W])
    N = _gpu_normals(snx, D, sc.cam)
    lab, cnt = _run(snx, D, N, cos, pad)
    ref, rcnt = oracle.components_crease(D, N, 0.1, 1.0, cos)
    assert np.array_equal(lab, ref), (lab != ref).sum()
    assert cnt == rcnt
    if cos == -1.0:                       # no crease test: the plain components
        plain, pc = oracle.components(D, 0.1, 1.0)
        assert np.array_equal(lab, plain) and cnt == pc


def test_crease_roof_and_random_normals(oracle):
    snx = _snx()
    print("case crease roof / random normals", flush=True)
    # a roof spanning two component tiles and a seam: one covered-depth component,
    # two crease components
    H, W = 40, 150
    u = np.arange(W, dtype=np.float64)[None, :].repeat(H, 0)
    D = np.where(u < 70, 20.0 + 0.25 * u, 20.0 + 0.25 * 70 - 0.25 * (u - 70)).astype(np.float32)
    N = np.where((u < 70)[None], np.array([-0.6, 0.0, -0.8])[:, None, None],
                 np.array([0.6, 0.0, -0.8])[:, None, None]).astype(np.float32)
    lab, cnt = _run(snx, D, N, 0.9)
    assert cnt == 2 and np.all(lab[:, :70] == 0) and np.all(lab[:, 70:] == 70)
    # random unit normals with NaN holes on a constant frame: labels by the
    # crease test alone, across tile seams
    rng = np.random.default_rng(4)
    H, W = 96, 200
    D = np.full((H, W), 30.0, np.float32)
    v = rng.normal(size=(3, H, W))
    v[2] = -np.abs(v[2]) - 2.0
    N = (v / np.linalg.norm(v, axis=0)).astype(np.float32)
    N[:, rng.random((H, W)) < 0.1] = np.nan
    for cos in (0.9, 0.97):
        lab, cnt = _run(snx, D, N, cos)
        ref, rcnt = oracle.components_crease(D, N, 0.1, 1.0, cos)
        assert np.array_equal(lab, ref) and cnt == rcnt
