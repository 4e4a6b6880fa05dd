"""Pins for the oracle of the two encoder variants of Sec. 9 (a hash grid inside each
adaptive grid; 4-D time grids), against what their definitions fix independently of
the code: the dense-grid limits (checked against the pinned dense encoder), the hash
function's published constants, partition of unity, interpolation at vertices and
linearity in time, central differences, and torch autograd through grid_sample."""
import numpy as np
import torch

from oracle import apmg_oracle as O
from oracle import apmg_variants as V


def _G(rng, M, shear=0.05, scale=0.8):
    G = np.zeros((M, 3, 4))
    G[:, [0, 1, 2], [0, 1, 2]] = rng.normal(1.0, 0.05, size=(M, 3)) * scale
    G += rng.normal(0, shear, size=G.shape) * (1 - np.eye(3, 4)[None])
    return G


def _mlp(rng, K, hidden=8):
    return [rng.normal(size=(hidden, K)), rng.normal(size=(hidden, hidden)) / 3, rng.normal(size=(1, hidden)) / 3]


def _points(rng, N):
    x = rng.uniform(-1.2, 1.2, size=(N, 3))
    x[0] = [np.nan, 0.0, 0.0]
    x[1] = [1.0, 1.0, 1.0]
    x[2] = [-1.0, -1.0, -1.0]
    return x


# ------------------------------------------------------------------ hash grid

def test_hash_index_published_constants_and_wrap():
    # Mueller et al. 2022: h(v) = (v_x * 1 ^ v_y * 2654435761 ^ v_z * 805459861) mod 2^32 mod T
    T = 1 << 19
    v = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [3, 5, 7], [0, 2, 0], [0, 0, 9]])
    got = V.hash_index(v, T)
    assert got[0] == 1
    assert got[1] == 2654435761 % T
    assert got[2] == 805459861 % T
    assert got[3] == ((3 ^ ((5 * 2654435761) % 2 ** 32) ^ ((7 * 805459861) % 2 ** 32)) % T)
    assert got[4] == ((2 * 2654435761) % 2 ** 32) % T          # wraps mod 2^32
    assert got[5] == ((9 * 805459861) % 2 ** 32) % T
    # XOR-linear in the per-axis terms, for any vertex
    rng = np.random.default_rng(1)
    w = rng.integers(0, 4096, size=(200, 3))
    hx = V.hash_index(w * [1, 0, 0], 1 << 32)
    hy = V.hash_index(w * [0, 1, 0], 1 << 32)
    hz = V.hash_index(w * [0, 0, 1], 1 << 32)
    np.testing.assert_array_equal(V.hash_index(w, 1 << 32), hx ^ hy ^ hz)


def test_level_entries_one_to_one_until_the_table_is_full():
    # (N + 1)^3 <= T: one entry per vertex, x fastest; one vertex more: hashed
    N, T = 7, 512
    v = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij"), -1).reshape(-1, 3)[:, ::-1]
    e = V.level_entries(v, N, T)
    np.testing.assert_array_equal(np.sort(e), np.arange(512))
    np.testing.assert_array_equal(e, v[:, 0] + 8 * (v[:, 1] + 8 * v[:, 2]))
    np.testing.assert_array_equal(V.level_entries(v, 8, 512), V.hash_index(v, 512))


def test_hash_one_dense_level_equals_the_dense_encoder():
    # L = 1, N_0 = R - 1, T >= R^3: the level is the dense grid of Eq. (2), entry x + R(y + Rz)
    rng = np.random.default_rng(2)
    M, C, R, N = 3, 2, 5, 300
    G = _G(rng, M)
    F = rng.normal(size=(M, C, R, R, R))
    Theta = np.zeros((M, 1, 128, C))
    Theta[:, 0, :R ** 3, :] = F.transpose(0, 2, 3, 4, 1).reshape(M, R ** 3, C)
    x = _points(rng, N)
    e_hash = V.hash_encode(G, Theta, [R - 1], x)
    e_dense = O.encode(G, F, x)
    np.testing.assert_array_equal(e_hash["inside"], e_dense["inside"])
    np.testing.assert_allclose(e_hash["y"], e_dense["y"], rtol=0, atol=1e-14)
    # and the adjoint: dTheta is dF laid out as the table, dG and dW agree
    W = _mlp(rng, M * C)
    df = rng.normal(size=N)
    gh = V.hash_backward({"G": G, "Theta": Theta, "res": [R - 1], "W": W, "vmin": -1.0, "vmax": 2.0}, x, df)
    gd = O.backward({"G": G, "F": F, "W": W, "vmin": -1.0, "vmax": 2.0}, x, df)
    np.testing.assert_allclose(gh["dTheta"][:, 0, :R ** 3, :], gd["dF"].transpose(0, 2, 3, 4, 1).reshape(M, R ** 3, C),
                               rtol=0, atol=1e-12)
    assert np.all(gh["dTheta"][:, 0, R ** 3:, :] == 0)
    np.testing.assert_allclose(gh["dG"], gd["dG"], rtol=1e-12, atol=1e-12)
    for a, b in zip(gh["dW"], gd["dW"]):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)


def test_hash_levels_concatenate_grid_major_then_level():
    # two dense levels of different resolution = two dense encoders, features (i L + k) C + c
    rng = np.random.default_rng(3)
    M, C, N = 2, 2, 200
    res = [3, 6]
    G = _G(rng, M)
    T = 7 ** 3
    Theta = np.zeros((M, 2, T, C))
    F = []
    for k, Nk in enumerate(res):
        R = Nk + 1
        Fk = rng.normal(size=(M, C, R, R, R))
        Theta[:, k, :R ** 3, :] = Fk.transpose(0, 2, 3, 4, 1).reshape(M, R ** 3, C)
        F.append(Fk)
    x = _points(rng, N)
    y = V.hash_encode(G, Theta, res, x)["y"].reshape(N, M, 2, C)
    for k in range(2):
        yk = O.encode(G, F[k], x)["y"].reshape(N, M, C)
        np.testing.assert_allclose(y[:, :, k, :], yk, rtol=0, atol=1e-14)


def test_hash_partition_of_unity_with_collisions():
    # every table entry = the same vector: each inside level gives that vector, whatever collides
    rng = np.random.default_rng(4)
    M, L, T, C = 3, 3, 64, 2
    G = _G(rng, M)
    Theta = np.broadcast_to(np.array([0.25, -1.5]), (M, L, T, C)).copy()
    x = _points(rng, 400)
    enc = V.hash_encode(G, Theta, [2, 9, 40], x)
    y = enc["y"].reshape(-1, M, L, C)
    ins = enc["inside"]
    np.testing.assert_allclose(y[ins], np.broadcast_to([0.25, -1.5], y[ins].shape), rtol=0, atol=1e-14)
    assert np.all(y[~ins] == 0)
    assert (~ins).sum() > 10 and ins.sum() > 100


def test_hash_vertex_reads_its_entry():
    # a point on a vertex of a hashed level reads exactly that vertex's entry
    rng = np.random.default_rng(5)
    M, L, T, C = 1, 1, 32, 2
    G = np.zeros((1, 3, 4))
    G[0, [0, 1, 2], [0, 1, 2]] = 1.0
    Theta = rng.normal(size=(M, L, T, C))
    Nk = 16                                     # 17^3 vertices > 32: hashed
    v = rng.integers(0, Nk + 1, size=(50, 3))
    x = -1.0 + 2.0 * v / Nk                     # exact in binary (Nk a power of two)
    y = V.hash_encode(G, Theta, [Nk], x)["y"].reshape(-1, C)
    np.testing.assert_allclose(y, Theta[0, 0, V.hash_index(v, T)], rtol=0, atol=1e-15)


def _hash_model(rng, M=2, L=2, T=16, C=2, res=(2, 5)):
    G = _G(rng, M)
    return {"G": G, "Theta": rng.normal(size=(M, L, T, C)), "res": list(res), "W": _mlp(rng, M * L * C),
            "vmin": -0.5, "vmax": 3.0}


def test_hash_backward_matches_central_differences():
    # T = 16 forces collisions on the second level (6^3 vertices): their gradients add
    rng = np.random.default_rng(6)
    model = _hash_model(rng)
    N = 24
    x = rng.uniform(-1, 1, size=(N, 3))
    df = rng.normal(size=N)
    g = V.hash_backward(model, x, df)

    def pattern(m):
        _, c = V.hash_forward(m, x)
        e = c["enc"]
        return [e["inside"].copy()] + [i.copy() for i in e["i0"]] + [(z > 0).copy() for z in c["z"][:-1]]

    base = pattern(model)
    hstep = 1e-5
    checked = skipped = 0
    for name in ("Theta", "G"):
        arr = model[name]
        for fi in range(arr.size):
            idx = np.unravel_index(fi, arr.shape)
            vals = []
            ok = True
            for sgn in (+1, -1):
                m2 = dict(model)
                m2[name] = arr.copy()
                m2[name][idx] += sgn * hstep
                if not all(np.array_equal(a, b) for a, b in zip(pattern(m2), base)):
                    ok = False
                    break
                vals.append(float(np.dot(df, V.hash_forward(m2, x)[0])))
            if not ok:
                skipped += 1
                continue
            fd = (vals[0] - vals[1]) / (2 * hstep)
            grad = g["dTheta"][idx] if name == "Theta" else g["dG"][idx]
            assert abs(fd - grad) <= 1e-7 * (1 + abs(grad)), (name, idx, fd, grad)
            checked += 1
    assert checked > 80 and skipped < 0.2 * checked
    assert np.count_nonzero(g["dTheta"][:, 1]) > 0


def test_hash_backward_matches_torch_autograd():
    # independent adjoint: torch autograd through the gather-and-interpolate of every level
    # (entries from the oracle's index function), points strictly inside every grid
    rng = np.random.default_rng(7)
    model = _hash_model(rng, M=3, L=3, T=32, C=2, res=(2, 3, 7))
    model["G"][:, :, :3] *= 0.7
    model["G"][:, :, 3] *= 0.4
    N = 64
    x = rng.uniform(-1, 1, size=(N, 3))
    df = rng.normal(size=N)
    g = V.hash_backward(model, x, df)
    M, L, T, C = model["Theta"].shape
    Gt = torch.tensor(model["G"], requires_grad=True)
    Tt = torch.tensor(model["Theta"], requires_grad=True)
    Wt = [torch.tensor(w, requires_grad=True) for w in model["W"]]
    l = torch.einsum("mrk,nk->nmr", Gt[:, :, :3], torch.tensor(x)) + Gt[None, :, :, 3]
    assert float(l.detach().abs().max()) < 1.0
    feats = []
    for k, Nk in enumerate(model["res"]):
        u = (l + 1.0) * (Nk / 2.0)
        i0 = torch.clamp(torch.floor(u.detach()), 0, Nk - 1)
        w = u - i0
        e = torch.zeros((N, M, C), dtype=torch.float64)
        for q in range(8):
            off = torch.tensor([q & 1, (q >> 1) & 1, (q >> 2) & 1], dtype=torch.float64)
            vtx = (i0 + off).long().numpy()
            ent = torch.from_numpy(V.level_entries(vtx, Nk, T))
            wq = torch.where(off.bool(), w, 1.0 - w).prod(-1)
            vals = Tt[torch.arange(M)[None, :], k, ent, :]
            e = e + wq[..., None] * vals
        feats.append(e)
    y = torch.stack(feats, 2).reshape(N, M * L * C)
    h = torch.relu(y @ Wt[0].T)
    h = torch.relu(h @ Wt[1].T)
    f = (h @ Wt[2].T)[:, 0] * (model["vmax"] - model["vmin"]) + model["vmin"]
    (f * torch.tensor(df)).sum().backward()
    np.testing.assert_allclose(g["dTheta"], Tt.grad.numpy(), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(g["dG"], Gt.grad.numpy(), rtol=1e-10, atol=1e-10)
    for a, b in zip(g["dW"], Wt):
        np.testing.assert_allclose(a, b.grad.numpy(), rtol=1e-10, atol=1e-10)


# ------------------------------------------------------------------ 4-D grids

def test_time_grid_with_equal_slices_is_the_dense_grid():
    rng = np.random.default_rng(8)
    M, C, R, Rt, N = 3, 2, 5, 4, 300
    G = _G(rng, M)
    F = rng.normal(size=(M, C, R, R, R))
    F4 = np.repeat(F[:, :, None], Rt, axis=2)
    x = _points(rng, N)
    tau = rng.uniform(-1, 1, size=N)
    e4 = V.time_encode(G, F4, x, tau)
    e3 = O.encode(G, F, x)
    np.testing.assert_array_equal(e4["inside"], e3["inside"])
    np.testing.assert_allclose(e4["y"], e3["y"], rtol=0, atol=1e-13)
    # a time outside [-1, 1] (or NaN) masks every grid
    tau_out = np.full(N, 1.5)
    tau_out[::2] = np.nan
    assert np.all(V.time_encode(G, F4, x, tau_out)["y"] == 0)


def test_time_grid_at_time_vertices_is_that_slice():
    rng = np.random.default_rng(9)
    M, C, R, Rt, N = 2, 2, 4, 5, 200
    G = _G(rng, M)
    F4 = rng.normal(size=(M, C, Rt, R, R, R))
    x = _points(rng, N)
    for k in range(Rt):
        tau = np.full(N, -1.0 + 2.0 * k / (Rt - 1))          # -1, -0.5, 0, 0.5, 1: exact
        e4 = V.time_encode(G, F4, x, tau)["y"]
        e3 = O.encode(G, F4[:, :, k], x)["y"]
        np.testing.assert_allclose(e4, e3, rtol=0, atol=1e-14)


def test_time_grid_is_linear_in_time_inside_a_time_cell():
    rng = np.random.default_rng(10)
    M, C, R, Rt, N = 2, 2, 4, 3, 100
    G = _G(rng, M)
    F4 = rng.normal(size=(M, C, Rt, R, R, R))
    x = rng.uniform(-0.9, 0.9, size=(N, 3))
    a, b = -1.0, 0.0                                          # the first time cell
    ts = [a + (b - a) * s for s in (0.1, 0.35, 0.8)]
    ys = [V.time_encode(G, F4, x, np.full(N, t))["y"] for t in ts]
    # three points on a line: y(t2) - y(t1) = (t2 - t1)/(t1 - t0) (y(t1) - y(t0))
    np.testing.assert_allclose(ys[2] - ys[1], (ts[2] - ts[1]) / (ts[1] - ts[0]) * (ys[1] - ys[0]),
                               rtol=1e-10, atol=1e-12)


def test_time_backward_matches_torch_autograd_with_grid_sample():
    # independent adjoint: the two time slices through grid_sample, mixed by the time
    # weight, torch autograd in float64; points strictly inside every grid
    rng = np.random.default_rng(11)
    M, C, R, Rt, N = 3, 2, 5, 4, 64
    G = _G(rng, M, scale=0.7)
    G[:, :, 3] *= 0.4
    F4 = rng.normal(size=(M, C, Rt, R, R, R))
    W = _mlp(rng, M * C)
    model = {"G": G, "F4": F4, "W": W, "vmin": -1.0, "vmax": 2.5}
    x = rng.uniform(-1, 1, size=(N, 3))
    tau = rng.uniform(-0.99, 0.99, size=N)
    df = rng.normal(size=N)
    g = V.time_backward(model, x, tau, df)
    Gt = torch.tensor(G, requires_grad=True)
    Ft = torch.tensor(F4, requires_grad=True)
    Wt = [torch.tensor(w, requires_grad=True) for w in W]
    l = torch.einsum("mrk,nk->mnr", Gt[:, :, :3], torch.tensor(x)) + Gt[:, None, :, 3]
    assert float(l.detach().abs().max()) < 1.0
    ut = (torch.tensor(tau) + 1.0) * ((Rt - 1) / 2.0)
    t0 = torch.clamp(torch.floor(ut), 0, Rt - 2).long()
    wt = ut - t0
    y = torch.zeros((N, M, C), dtype=torch.float64)
    for k in range(Rt):
        e = torch.nn.functional.grid_sample(Ft[:, :, k], l[:, None, None], mode="bilinear", align_corners=True)
        e = e[:, :, 0, 0, :].permute(2, 0, 1)                  # [N, M, C]
        wk = torch.where(t0 == k, 1.0 - wt, torch.where(t0 + 1 == k, wt, torch.zeros_like(wt)))
        y = y + wk[:, None, None] * e
    y = y.reshape(N, M * C)
    h = torch.relu(y @ Wt[0].T)
    h = torch.relu(h @ Wt[1].T)
    f = (h @ Wt[2].T)[:, 0] * (model["vmax"] - model["vmin"]) + model["vmin"]
    (f * torch.tensor(df)).sum().backward()
    np.testing.assert_allclose(g["dF4"], Ft.grad.numpy(), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(g["dG"], Gt.grad.numpy(), rtol=1e-10, atol=1e-10)
    for a, b in zip(g["dW"], Wt):
        np.testing.assert_allclose(a, b.grad.numpy(), rtol=1e-10, atol=1e-10)


def test_time_backward_matches_central_differences_at_the_mask():
    # points near and beyond the faces of the space-time cube: the mask contributes nothing
    rng = np.random.default_rng(12)
    M, C, R, Rt, N = 2, 2, 4, 3, 20
    G = _G(rng, M)
    model = {"G": G, "F4": rng.normal(size=(M, C, Rt, R, R, R)), "W": _mlp(rng, M * C), "vmin": 0.0, "vmax": 1.0}
    x = rng.uniform(-1.1, 1.1, size=(N, 3))
    tau = rng.uniform(-1.05, 1.05, size=N)
    df = rng.normal(size=N)
    g = V.time_backward(model, x, tau, df)

    def pattern(m):
        _, c = V.time_forward(m, x, tau)
        e = c["enc"]
        return [e["inside"].copy(), e["i0"].copy(), e["t0"].copy()] + [(z > 0).copy() for z in c["z"][:-1]]

    base = pattern(model)
    hstep = 1e-5
    checked = 0
    for name, grad in (("G", g["dG"]), ("F4", g["dF4"])):
        arr = model[name]
        idxs = range(arr.size) if name == "G" else rng.choice(arr.size, size=80, replace=False)
        for fi in idxs:
            idx = np.unravel_index(fi, arr.shape)
            vals = []
            for sgn in (+1, -1):
                m2 = dict(model)
                m2[name] = arr.copy()
                m2[name][idx] += sgn * hstep
                if not all(np.array_equal(a, b) for a, b in zip(pattern(m2), base)):
                    break
                vals.append(float(np.dot(df, V.time_forward(m2, x, tau)[0])))
            if len(vals) < 2:
                continue
            fd = (vals[0] - vals[1]) / (2 * hstep)
            assert abs(fd - grad[idx]) <= 1e-7 * (1 + abs(grad[idx])), (name, idx, fd, grad[idx])
            checked += 1
    assert checked > 80
