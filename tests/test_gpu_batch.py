"""Batch plans: every frame of an uneven batch is bit-identical to snx_pipeline on
that frame alone, on direct runs and on graph replays with fresh inputs."""
import numpy as np
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _snx():
    import paper_2504_15121_amd as snx
    snx.load()
    return snx


def _frames(specs, seed):
    out = []
    for k, (W, H) in enumerate(specs):
        sc = scenes.planes_quadrics_scene(width=W, height=H, f=0.8 * W, n_planes=6, n_spheres=2,
                                          seed=seed + k)
        out.append(sc)
    return out


def _alloc(sc, label_pad=0, dn=True, count=True):
    H, W = sc.disp.shape
    lab_full = torch.full((H, W + label_pad), -7, dtype=torch.int32, device=DEV)
    f = dict(disp=torch.from_numpy(sc.disp).to(DEV), cam=sc.cam,
             labels=lab_full[:, :W], points=torch.empty((H, W, 8), device=DEV))
    if dn:
        f["disp_dn"] = torch.empty((H, W), device=DEV)
    if count:
        f["num_components"] = torch.zeros(1, dtype=torch.int32, device=DEV)
    return f


def _reference(snx, f, filter_window, normal_window, cnn=None):
    d = f["disp"]
    H, W = d.shape
    lab = torch.empty((H, W), dtype=torch.int32, device=DEV)
    pts = torch.empty((H, W, 8), device=DEV)
    dn = torch.empty((H, W), device=DEV)
    cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = torch.empty(snx.snx_pipeline_workspace_size(W, H), dtype=torch.uint8, device=DEV)
    snx.snx_pipeline(d, f["cam"], lab, pts, ws, num_components=cnt, disp_dn=dn,
                     filter_window=filter_window, normal_window=normal_window, cnn=cnn)
    return lab, pts, dn, cnt


def _check(snx, frames, filter_window, normal_window, cnn=None):
    for i, f in enumerate(frames):
        lab, pts, dn, cnt = _reference(snx, f, filter_window, normal_window, cnn)
        torch.cuda.synchronize()
        assert torch.equal(f["labels"], lab), i
        assert torch.equal(f["points"].view(torch.int32), pts.view(torch.int32)), i
        if "disp_dn" in f:
            H, W = f["disp"].shape
            valid = torch.isfinite(f["disp"]) & (f["disp"] > 0)
            a, b = f["disp_dn"], dn
            if filter_window == 1 and cnn is None:
                a, b = a[valid], b[valid]      # window 1 writes only valid pixels
            assert torch.equal(a.view(torch.int32), b.view(torch.int32)), i
        if "num_components" in f:
            assert int(f["num_components"].item()) == int(cnt.item()), i


SPECS = [(300, 170), (64, 32), (1, 1), (517, 333), (65, 33), (1280, 720)]


@pytest.mark.parametrize("filter_window,normal_window", [(3, 9), (1, 5), (3, 21), (3, 45), (1, 61)])
def test_plan_direct_matches_pipeline(filter_window, normal_window):
    snx = _snx()
    print(f"case plan direct f{filter_window} g{normal_window}", flush=True)
    scs = _frames(SPECS, 100)
    frames = [_alloc(sc, label_pad=(5 if k % 2 else 0), dn=(k != 2), count=(k != 3))
              for k, sc in enumerate(scs)]
    plan = snx.Plan(frames, filter_window=filter_window, normal_window=normal_window)
    plan.run()
    torch.cuda.synchronize()
    _check(snx, frames, filter_window, normal_window)
    plan.close()


def test_plan_graph_replays_with_new_inputs():
    snx = _snx()
    print("case plan graph replay", flush=True)
    scs = _frames(SPECS[:4], 200)
    frames = [_alloc(sc, label_pad=3 * (k % 2)) for k, sc in enumerate(scs)]
    plan = snx.Plan(frames, filter_window=3, normal_window=9)
    st = torch.cuda.Stream()
    for rep in range(4):
        new = _frames(SPECS[:4], 300 + 10 * rep)
        for f, sc in zip(frames, new):
            f["disp"].copy_(torch.from_numpy(sc.disp))
            f["labels"].fill_(-9)
            f["points"].zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            plan.run(st)
        st.synchronize()
        # eager work between replays
        junk = torch.randn(1 << 20, device=DEV).sum()
        torch.cuda.synchronize()
        _check(snx, frames, 3, 9)
        del junk
    plan.close()


def test_plan_learned_filter_matches_pipeline():
    snx = _snx()
    from paper_2504_15121_amd import learned
    print("case plan learned", flush=True)
    rng = np.random.default_rng(4)
    flat = learned.init_params(4)
    flat[-33:-1] = rng.normal(0, 0.05, 32).astype(np.float32)   # non-zero last layer
    P = torch.from_numpy(flat).to(DEV)
    packed = torch.empty(snx.snx_cnn_packed_bytes() // 2, dtype=torch.int16, device=DEV)
    snx.snx_cnn_pack(P, packed)
    specs = [(300, 170), (129, 70), (64, 64)]
    ws = torch.empty(snx.snx_cnn_workspace_size(300, 170, 1, 0), dtype=torch.uint8, device=DEV)
    model = snx.cnn_model(P, packed, ws)
    frames = [_alloc(sc) for sc in _frames(specs, 400)]
    plan = snx.Plan(frames, normal_window=9, cnn=model)
    st = torch.cuda.Stream()
    for rep in range(2):
        with torch.cuda.stream(st):
            plan.run(st)
        st.synchronize()
        _check(snx, frames, 3, 9, cnn=model)
    plan.close()


def test_plan_rejects_incomplete_model():
    snx = _snx()
    from paper_2504_15121_amd import learned
    from paper_2504_15121_amd._lib import snx_cnn_model
    P = torch.from_numpy(learned.init_params(0)).to(DEV)
    frames = [_alloc(sc) for sc in _frames([(100, 60)], 500)]
    with pytest.raises(snx.SnxError) as ei:
        snx.Plan(frames, cnn=snx_cnn_model(P.data_ptr(), None, None, 0))   # no packed weights
    assert ei.value.status == 5
