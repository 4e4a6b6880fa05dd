"""Pins of the oracle's domain-decomposition inference (Sec. 5.3): the local frame inverts
the training map, one brick spanning the volume is the identity frame, and every point is
evaluated by the brick the hash assigns it to."""
import numpy as np

import synth
from oracle import apmg_oracle as O


def test_local_frame_inverts_the_training_map():
    shape = (100, 120, 90)
    dims, bricks = O.brick_partition(shape, 32, 1)
    x = synth.uniform_points_host(20000, seed=4)
    ids = O.brick_assign(x, shape, 32, dims)
    for b in np.unique(ids)[:20]:
        sel = ids == b
        lc = O.dd_local_coords(x[sel], shape, bricks[b])
        u_back = O.brick_local_to_voxel(lc, bricks[b]["e0"], bricks[b]["e1"])
        u_true = (x[sel].astype(np.float64) + 1.0) * 0.5 * (np.array(shape) - 1)
        assert np.max(np.abs(u_back - u_true)) < 1e-3          # float32 rounding of ~100-voxel coordinates
        # the assigned brick's base extent holds the point: local coordinates stay inside [-1, 1]
        assert np.all(np.abs(lc) <= 1.0)


def test_one_brick_spanning_the_volume_is_the_identity_frame():
    shape = (64, 48, 40)
    dims, bricks = O.brick_partition(shape, 64, 0)
    assert dims == (1, 1, 1)
    x = synth.uniform_points_host(5000, seed=5)
    lc = O.dd_local_coords(x, shape, bricks[0])
    assert np.max(np.abs(lc.astype(np.float64) - x)) < 4e-7
    assert np.all(O.brick_assign(x, shape, 64, dims) == 0)


def test_each_point_is_evaluated_by_its_brick():
    # models whose output is the constant vmin (zero MLP): f equals the brick's vmin, which is
    # set to the brick id, so f must equal the id of the brick holding floor(u) on every axis
    shape = (70, 50, 40)
    dims, bricks = O.brick_partition(shape, 16, 2)
    host = synth.init_model(2, 1, 4, [2, 64, 64, 1], seed=1)
    models = []
    for b, br in enumerate(bricks):
        m = {"G": host["G"].astype(np.float64), "F": host["F"].astype(np.float64),
             "W": [np.zeros_like(w, dtype=np.float64) for w in host["W"]], "vmin": 0.0, "vmax": 1.0}
        models.append(m)
        br["vmin"], br["vmax"] = float(b), float(b) + 1.0
    x = synth.uniform_points_host(4000, seed=6)
    x[:3] = [[1.0, 1.0, 1.0], [-1.0, -1.0, -1.0], [0.0, 0.0, 0.0]]
    f, ids = O.dd_forward(models, bricks, shape, 16, dims, x)
    # brute force: the base extent [iB, min((i+1)B, n)) holding floor(u), u in float64
    u = (x.astype(np.float64) + 1.0) * 0.5 * (np.array(shape) - 1)
    ijk = np.minimum(np.floor(u).astype(np.int64) // 16, np.array(dims) - 1)
    want = ijk[:, 0] + dims[0] * ijk[:, 1] + dims[0] * dims[1] * ijk[:, 2]
    agree = want == ids
    assert agree.mean() > 0.999                                    # float32 u may differ on a sliver
    assert np.array_equal(f, ids.astype(np.float64))
