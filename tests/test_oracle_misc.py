"""Pins for the oracle's point generator, ground-truth sampling, brick
partition and assignment (Sec. 5.1, Sec. 5.3), Adam (Sec. 7) and the
constants the paper states."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage
import torch

import synth
from oracle import apmg_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


# ---------------------------------------------------------------- RNG
def test_philox_matches_numpy_bit_generator():
    rng = np.random.default_rng(30)
    for _ in range(20):
        ctr = rng.integers(0, 2 ** 63, size=4, dtype=np.uint64)
        ctr[0] |= np.uint64(1)                   # numpy pre-increments word 0
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64)
        before = ctr.copy()
        before[0] -= np.uint64(1)
        bg = np.random.Philox(key=key, counter=before)
        ref = bg.random_raw(4).astype(np.uint64)
        got = O.philox4x64_10(ctr[None], key)[0]
        assert np.array_equal(got, ref)


def test_points_are_exact_lattice_values_in_range():
    x = O.uniform_points(seed=7, step=3, stream=1, n=20000)
    assert x.shape == (20000, 3)
    assert x.min() >= -1.0 and x.max() < 1.0
    assert np.array_equal(x.astype(np.float32).astype(np.float64), x)
    k = (x + 1.0) * 2 ** 23
    assert np.array_equal(k, np.round(k))
    assert abs(x.mean()) < 0.02 and abs(x.var() - 1.0 / 3.0) < 0.01
    # distinct steps and streams give distinct batches; a sub-range is a slice
    assert not np.array_equal(x, O.uniform_points(7, 4, 1, 20000))
    assert not np.array_equal(x, O.uniform_points(7, 3, 2, 20000))
    np.testing.assert_array_equal(O.uniform_points(7, 3, 1, 100, start=500), x[500:600])


# ---------------------------------------------------------------- GT sampling
def test_gt_sample_matches_scipy_map_coordinates():
    vol = synth.make_volume("blobs_sine", (17, 23, 29)).numpy().astype(np.float64)
    x = O.uniform_points(seed=1, step=0, stream=0, n=3000)
    x = np.concatenate([x, [[1.0, 1.0, 1.0], [-1.0, -1.0, -1.0], [1.0, -1.0, 0.0]]])
    v = O.gt_sample(vol, x)
    nz, ny, nx = vol.shape
    coords = np.stack([(x[:, 2] + 1) / 2 * (nz - 1), (x[:, 1] + 1) / 2 * (ny - 1),
                       (x[:, 0] + 1) / 2 * (nx - 1)])
    ref = scipy.ndimage.map_coordinates(vol, coords, order=1, mode="nearest")
    np.testing.assert_allclose(v, ref, rtol=0, atol=1e-12)


def test_reconstruction_loss_closed_form():
    f = np.array([1.0, 2.0, -1.0])
    v = np.array([0.5, 2.0, 1.0])
    L, df, h = O.reconstruction_loss(f, v)
    assert L == pytest.approx((0.25 + 0 + 4) / 3)
    np.testing.assert_allclose(df, [1.0 / 3, 0, -4.0 / 3])
    np.testing.assert_allclose(h, [0.25, 0, 4])


# ---------------------------------------------------------------- bricks
def test_brick_partition_by_brute_force():
    shape = (1000, 1200, 900)
    dims, bricks = O.brick_partition(shape, 256, 1)
    assert dims == (4, 5, 4) and len(bricks) == 80
    for d, n in enumerate(shape):
        owner = np.full(n, -1)
        for i in range(dims[d]):
            b = next(b for b in bricks if b["ijk"][d] == i)
            assert owner[b["base0"][d]:b["base1"][d]].max() == -1
            owner[b["base0"][d]:b["base1"][d]] = i
            assert b["e0"][d] == max(b["base0"][d] - 1, 0)
            assert b["e1"][d] == min(b["base1"][d], n - 1)
        assert owner.min() == 0                       # every voxel owned exactly once
    edge = bricks[-1]
    assert [edge["base1"][d] - edge["base0"][d] for d in range(3)] == [232, 176, 132]
    # brick ids in x, y, z order: id = i + I j + I J k
    for bid, b in enumerate(bricks):
        i, j, k = b["ijk"]
        assert bid == i + 4 * j + 20 * k
    # 16 ghost cells give 256 + 2*16 = 288 voxels for an interior brick (Sec. 7.2)
    _, b16 = O.brick_partition((1024, 1024, 1024), 256, 16)
    inner = b16[1 + 4 + 16]
    assert [inner["e1"][d] - inner["e0"][d] + 1 for d in range(3)] == [288, 288, 288]


def test_brick_assignment_by_exact_arithmetic():
    shape = (1000, 1200, 900)
    dims, bricks = O.brick_partition(shape, 256, 1)
    x = O.uniform_points(seed=3, step=0, stream=0, n=4000)
    x = np.concatenate([x, [[1.0, 1.0, 1.0], [-1.0, -1.0, -1.0]]]).astype(np.float32)
    ids = O.brick_assign(x, shape, 256, dims)
    for n in range(x.shape[0]):
        ijk = []
        for d in range(3):
            u = (Fraction(float(x[n, d])) + 1) * Fraction(shape[d] - 1, 2)
            ijk.append(min(int(u) // 256, dims[d] - 1))
        assert ids[n] == ijk[0] + dims[0] * ijk[1] + dims[0] * dims[1] * ijk[2]


def test_equal_bricks_agree_with_paper_hash_up_to_a_ghost_sliver():
    # Sec. 5.3: i = floor(I (p+1)/2), clamped below I.  With equal bricks the
    # voxel-based rule differs only where both bricks' ghost extents hold p.
    shape, B = (512, 512, 512), 128
    dims, bricks = O.brick_partition(shape, B, 1)
    x = O.uniform_points(seed=4, step=0, stream=0, n=20000)
    ids = O.brick_assign(x, shape, B, dims)
    paper = np.minimum(np.floor(4 * (x + 1) / 2), 3).astype(np.int64)
    pid = paper[:, 0] + 4 * paper[:, 1] + 16 * paper[:, 2]
    differ = ids != pid
    assert differ.mean() < 0.02
    for n in np.nonzero(differ)[0]:
        for b in (bricks[ids[n]], bricks[pid[n]]):
            u = (x[n] + 1) / 2 * (np.array(shape) - 1)
            assert np.all(u >= b["e0"]) and np.all(u <= b["e1"])


def test_brick_local_frame_round_trip():
    _, bricks = O.brick_partition((1000, 1200, 900), 256, 1)
    b = bricks[17]
    u = O.brick_local_to_voxel(np.array([[-1.0, -1.0, -1.0], [1.0, 1.0, 1.0]]), b["e0"], b["e1"])
    np.testing.assert_array_equal(u[0], b["e0"])
    np.testing.assert_array_equal(u[1], b["e1"])


def test_brick_gt_sample_matches_global_sampling():
    vol = synth.make_volume("blobs_turb", (40, 50, 60)).numpy().astype(np.float64)
    shape = (60, 50, 40)
    dims, bricks = O.brick_partition(shape, 16, 1)
    b = bricks[5]
    l = O.uniform_points(seed=5, step=0, stream=0, n=500)
    v_local = O.brick_gt_sample(vol, b, l)
    u = O.brick_local_to_voxel(l, b["e0"], b["e1"])
    coords = np.stack([u[:, 2], u[:, 1], u[:, 0]])
    ref = scipy.ndimage.map_coordinates(vol, coords, order=1, mode="nearest")
    np.testing.assert_allclose(v_local, ref, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- Adam
def test_adam_matches_torch_optim():
    rng = np.random.default_rng(31)
    theta = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    p = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.01, betas=(0.9, 0.99), eps=1e-8)
    for t in range(1, 6):
        g = rng.normal(size=50)
        theta, m, v = O.adam_update(theta, g, m, v, t, 0.01)
        p.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(theta, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_train_step_first_update_is_lr_times_sign():
    # Adam's first step moves each parameter by lr * g / (|g| + eps).
    model = synth.init_model(2, 2, 4, [4, 8, 8, 1], seed=3)
    model = {k: (np.asarray(v, np.float64) if k != "W" else [np.asarray(w, np.float64) for w in v])
             for k, v in model.items()}
    model["F"] = model["F"] * 1e3
    x = O.uniform_points(seed=1, step=0, stream=0, n=256)
    v = np.sin(3 * x[:, 0]) * 0.5 + 0.5
    st = O.zero_adam_state(model)
    m1, s1, info = O.train_step(model, st, x, v, density_active=False)
    g = info["dF"]
    np.testing.assert_allclose(m1["F"] - model["F"], -0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)
    assert np.array_equal(np.asarray(m1["G"]), np.asarray(model["G"])) and s1["tG"] == 0
    m2, s2, info2 = O.train_step(model, st, x, v, density_active=True)
    gG = info2["dG_density"]
    np.testing.assert_allclose(m2["G"] - model["G"][:, :3], -0.001 * gG / (np.abs(gG) + 1e-8),
                               atol=1e-15)
    assert s2["tG"] == 1 and info2["L_density"] > 0


# ---------------------------------------------------------------- paper constants
def test_constants_match_the_paper():
    c = {k: v["value"] for k, v in json.load(open(GOLDEN)).items() if not k.startswith("_")}
    assert O.P_FLATTOP == c["p_flattop"]
    assert O.ADAM_BETAS == (c["adam_beta1"], c["adam_beta2"])
    assert O.LR_DEFAULT == c["lr"] and O.LR_TRANSFORM == c["lr_transform"]
    model = synth.init_model(4000, 1, 2, [4000, 1], seed=9)
    G = model["G"].astype(np.float64)
    diag = G[:, [0, 1, 2], [0, 1, 2]]
    off = np.concatenate([G[:, 0, 1:], G[:, 1, [0, 2, 3]], G[:, 2, [0, 1, 3]]], axis=1)
    assert abs(diag.mean() - c["init_diag_mean"]) < 0.005
    assert abs(diag.std() - c["init_std"]) < 0.005 and abs(off.std() - c["init_std"]) < 0.005
    assert np.abs(model["F"]).max() <= c["init_grid_range"]
