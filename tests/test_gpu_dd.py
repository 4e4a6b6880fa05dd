"""GPU parity of the domain-decomposition inference (apmg_dd_forward) against the oracle:
48 brick models over a 100 x 120 x 90 volume (bricks of 32 voxels, one ghost voxel)."""
import numpy as np
import pytest
import torch

import synth
from oracle import apmg_oracle as O

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda"
SHAPE = (100, 120, 90)   # nx, ny, nz


def A():
    import paper_2308_02494_amd as mod
    return mod


def _setup(M=8, C=2, R=12, H=64, mlp=None, seed=0):
    A_ = A()
    table, bricks = A_.apmg_make_bricks(*SHAPE, 32, 1)
    nb = len(bricks)
    rng = np.random.default_rng(seed)
    hosts = []
    for b in range(nb):
        h = synth.init_model(M, C, R, [M * C, H, H, 1], seed=100 + b, grid_range=0.5, extra_translation=0.2)
        bricks[b].vmin, bricks[b].vmax = float(rng.uniform(-1, 0)), float(rng.uniform(1, 2))
        hosts.append(h)
    G = torch.stack([torch.from_numpy(h["G"]) for h in hosts]).to(DEV)
    F = torch.stack([torch.from_numpy(h["F"]) for h in hosts]).contiguous().to(DEV)
    W = torch.stack([torch.cat([torch.from_numpy(w).reshape(-1) for w in h["W"]]) for h in hosts]).to(DEV)
    models = A_.DDModels(G, F, W, [M * C, H, H, 1], table, bricks, A_.F32 if mlp is None else mlp)
    obricks = [{"e0": list(br.e0), "e1": list(br.e1), "vmin": br.vmin, "vmax": br.vmax} for br in bricks]
    omodels = [{"G": h["G"].astype(np.float64), "F": h["F"].astype(np.float64),
                "W": [w.astype(np.float64) for w in h["W"]], "vmin": 0.0, "vmax": 1.0} for h in hosts]
    return models, omodels, obricks, (table.dims[0], table.dims[1], table.dims[2])


def _points(n, seed):
    x = synth.uniform_points_host(n, seed=seed)
    x[:6] = [[1.0, 1.0, 1.0], [-1.0, -1.0, -1.0], [0.0, 0.0, 0.0], [1.2, 0.0, -1.3], [np.nan, 0.2, 0.1],
             [-0.36, 0.0667, 1.0]]
    return x


def test_dd_forward_matches_oracle_fp32():
    models, omodels, obricks, dims = _setup()
    assert models.struct.nb == 48
    x = _points(20000, 8)
    got = A().apmg_dd_forward(models, torch.from_numpy(np.ascontiguousarray(x.T)).to(DEV)).cpu().numpy()
    want, ids = O.dd_forward(omodels, obricks, SHAPE, 32, dims, x)
    assert len(np.unique(ids)) == 48
    ok = np.isfinite(want)
    assert np.array_equal(np.isfinite(got), ok)
    err = np.linalg.norm(got[ok] - want[ok]) / np.linalg.norm(want[ok])
    mx = np.max(np.abs(got[ok] - want[ok])) / np.max(np.abs(want[ok]))
    print(f"dd forward fp32: normwise {err:.2e} max {mx:.2e}")
    assert err < 1e-5 and mx < 1e-5


def test_dd_forward_brick_ids_and_assignment_agree():
    # the hash inside the DD call is apmg_assign_bricks: equal ids for every point
    models, _, _, dims = _setup()
    x = _points(5000, 9)
    pts = torch.from_numpy(np.ascontiguousarray(x.T)).to(DEV)
    ids = A().apmg_assign_bricks(models.table, pts).cpu().numpy()
    assert np.array_equal(ids, O.brick_assign(x, SHAPE, 32, dims))


def test_dd_forward_bf16_stated_and_empty():
    models, omodels, obricks, dims = _setup(mlp=A().BF16)
    x = _points(8000, 10)
    got = A().apmg_dd_forward(models, torch.from_numpy(np.ascontiguousarray(x.T)).to(DEV)).cpu().numpy()
    want, _ = O.dd_forward(omodels, obricks, SHAPE, 32, dims, x)
    ok = np.isfinite(want)
    err = np.linalg.norm(got[ok] - want[ok]) / np.linalg.norm(want[ok])
    print(f"dd forward bf16 MLP: normwise {err:.2e}")
    assert err < 3e-2
    empty = A().apmg_dd_forward(models, torch.zeros((3, 0), device=DEV))
    assert empty.numel() == 0


def test_ghost_cells_seam_error():
    # Sec. 5.1 ghost cells, Sec. 7.2 study: a 2 x 2 x 2 brick split of a 128^3 volume trained
    # with one ghost voxel and with 16, then queried globally (apmg_dd_forward).  The error
    # against the volume (the oracle's trilinear sample) on points within one voxel of an
    # internal brick face, against interior points: with 16 ghost voxels the seam error is
    # not worse than with one.
    A_ = A()
    n_vox = 128
    vol = synth.make_volume("blobs_sine", (n_vox, n_vox, n_vox))
    vol_np = vol.numpy().astype(np.float64)
    rng = np.random.default_rng(5)
    # seam points: one coordinate within one voxel of the face at voxel 63.5 (bricks of 64)
    m = 20000
    seam = rng.uniform(-1, 1, size=(m, 3))
    axis = rng.integers(0, 3, size=m)
    u_face = rng.uniform(62.5, 64.5, size=m)
    seam[np.arange(m), axis] = u_face / ((n_vox - 1) * 0.5) - 1.0
    inner = rng.uniform(-1, 1, size=(m, 3))
    u_in = (inner + 1.0) * ((n_vox - 1) * 0.5)
    inner = inner[np.all(np.abs(u_in - 63.5) > 8.0, axis=1)]
    seam, inner = seam.astype(np.float32), inner.astype(np.float32)
    v_seam = O.gt_sample(vol_np, seam.astype(np.float64))
    v_inner = O.gt_sample(vol_np, inner.astype(np.float64))
    results = {}
    for ghost in (1, 16):
        table, bricks = A_.apmg_make_bricks(n_vox, n_vox, n_vox, 64, ghost)
        hosts = [synth.init_model(8, 2, 16, [16, 64, 64, 1], seed=200 + b) for b in range(len(bricks))]
        tr = A_.Trainer(hosts, vol.to(DEV), bricks, 1 << 14, seed=21)
        tr.density_active.fill_(0)
        for _ in range(300):
            tr.step()
        dd = A_.DDModels.from_trainer(tr, table, bricks)
        f_seam = A_.apmg_dd_forward(dd, torch.from_numpy(np.ascontiguousarray(seam.T)).to(DEV)).cpu().numpy()
        f_in = A_.apmg_dd_forward(dd, torch.from_numpy(np.ascontiguousarray(inner.T)).to(DEV)).cpu().numpy()
        rs = float(np.sqrt(np.mean((f_seam - v_seam) ** 2)))
        ri = float(np.sqrt(np.mean((f_in - v_inner) ** 2)))
        results[ghost] = (rs, ri)
        print(f"ghost {ghost}: seam RMSE {rs:.4e}, interior RMSE {ri:.4e}, ratio {rs / ri:.3f}")
    assert results[16][0] <= results[1][0]
