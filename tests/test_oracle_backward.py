"""Pins for the oracle's decoder (Sec. 4.1.2) and its hand-derived adjoint.

The model is piecewise linear in every single parameter (trilinear weights
are linear per axis inside a cell, transforms are affine, ReLU is piecewise
linear), so central finite differences are exact up to rounding unless the
stencil crosses a kink; crossings are detected and skipped."""
import numpy as np

import synth
import torch

from oracle import apmg_oracle as O


def _tiny_model(rng, M=2, C=2, R=4, hidden=8, grid_scale=1.0):
    G = np.zeros((M, 3, 4))
    G[:, [0, 1, 2], [0, 1, 2]] = rng.normal(1.0, 0.05, size=(M, 3))
    G += rng.normal(0, 0.05, size=G.shape) * (1 - np.eye(3, 4)[None])
    F = rng.normal(size=(M, C, R, R, R)) * grid_scale
    W = [rng.normal(size=(hidden, M * C)), rng.normal(size=(hidden, hidden)) / 3,
         rng.normal(size=(1, hidden)) / 3]
    return {"G": G, "F": F, "W": W, "vmin": -3.5, "vmax": 12.25}


def _pattern(model, x):
    f, cache = O.forward(model, x)
    enc = cache["enc"]
    return (enc["inside"].copy(), enc["cell"].copy(), [(z > 0).copy() for z in cache["z"][:-1]])


def _same(p, q):
    return (np.array_equal(p[0], q[0]) and np.array_equal(p[1], q[1])
            and all(np.array_equal(a, b) for a, b in zip(p[2], q[2])))


def test_mlp_matches_torch_and_scaling():
    rng = np.random.default_rng(10)
    W = [rng.normal(size=(16, 6)), rng.normal(size=(16, 16)), rng.normal(size=(1, 16))]
    y = rng.normal(size=(50, 6))
    m, _, _ = O.mlp_forward(W, y)
    net = torch.nn.Sequential(torch.nn.Linear(6, 16, bias=False), torch.nn.ReLU(),
                              torch.nn.Linear(16, 16, bias=False), torch.nn.ReLU(),
                              torch.nn.Linear(16, 1, bias=False)).double()
    with torch.no_grad():
        for lin, w in zip([net[0], net[2], net[4]], W):
            lin.weight.copy_(torch.from_numpy(w))
        ref = net(torch.from_numpy(y))[:, 0].numpy()
    np.testing.assert_allclose(m, ref, rtol=1e-13, atol=1e-13)


def test_all_outside_gives_vmin_exactly():
    rng = np.random.default_rng(11)
    model = _tiny_model(rng)
    x = np.array([[5.0, 5.0, 5.0], [np.nan, 0.0, 0.0], [-7.0, 0.0, 0.0]])
    f, _ = O.forward(model, x)
    assert np.all(f == -3.5)


def test_output_linear_in_last_layer():
    rng = np.random.default_rng(12)
    model = _tiny_model(rng)
    x = rng.uniform(-1, 1, size=(20, 3))
    f1, _ = O.forward(model, x)
    m2 = dict(model)
    m2["W"] = [model["W"][0], model["W"][1], 2.0 * model["W"][2]]
    f2, _ = O.forward(m2, x)
    # f = m (vmax - vmin) + vmin, so f2 - vmin = 2 (f1 - vmin)
    np.testing.assert_allclose(f2 + 3.5, 2 * (f1 + 3.5), rtol=1e-12, atol=1e-12)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(13)
    model = _tiny_model(rng)
    N = 16
    x = rng.uniform(-1, 1, size=(N, 3))
    df = rng.normal(size=N)
    g = O.backward(model, x, df)
    base = _pattern(model, x)

    def L(m):
        return float(np.dot(df, O.forward(m, x)[0]))

    hstep = 1e-4
    checked = skipped = 0
    params = [("G", None), ("F", None)] + [("W", k) for k in range(3)]
    for name, k in params:
        arr = model[name] if k is None else model[name][k]
        grad = {"G": g["dG"], "F": g["dF"]}[name] if k is None else g["dW"][k]
        flat_idx = range(arr.size)
        if name == "F":
            flat_idx = rng.choice(arr.size, size=60, replace=False)
        for fi in flat_idx:
            idx = np.unravel_index(fi, arr.shape)
            vals = []
            ok = True
            for sgn in (+1, -1):
                m2 = {kk: (vv.copy() if isinstance(vv, np.ndarray) else vv) for kk, vv in model.items()}
                m2["W"] = [w.copy() for w in model["W"]]
                tgt = m2[name] if k is None else m2[name][k]
                tgt[idx] += sgn * hstep
                if not _same(_pattern(m2, x), base):
                    ok = False
                    break
                vals.append(L(m2))
            if not ok:
                skipped += 1
                continue
            fd = (vals[0] - vals[1]) / (2 * hstep)
            assert abs(fd - grad[idx]) <= 1e-8 * (1 + abs(grad[idx])), (name, k, idx, fd, grad[idx])
            checked += 1
    assert checked > 150 and skipped < 0.1 * checked


def test_backward_matches_torch_autograd_with_grid_sample():
    # Independent adjoint: torch autograd through grid_sample for points that
    # lie strictly inside every grid (no mask), in float64.
    rng = np.random.default_rng(14)
    M, C, R, N = 3, 2, 6, 64
    model = _tiny_model(rng, M=M, C=C, R=R)
    model["G"][:, :, :3] *= 0.7
    model["G"][:, :, 3] *= 0.5
    x = rng.uniform(-1, 1, size=(N, 3))
    df = rng.normal(size=N)
    g = O.backward(model, x, df)
    assert g["dy"].shape == (N, M * C)

    Gt = torch.tensor(model["G"], requires_grad=True)
    Ft = torch.tensor(model["F"], requires_grad=True)
    Wt = [torch.tensor(w, requires_grad=True) for w in model["W"]]
    xt = torch.tensor(x)
    l = torch.einsum("mrk,nk->mnr", Gt[:, :, :3], xt) + Gt[:, None, :, 3]   # [M, N, 3]
    assert float(l.detach().abs().max()) < 1.0
    e = torch.nn.functional.grid_sample(Ft, l[:, None, None], mode="bilinear", align_corners=True)
    y = e[:, :, 0, 0, :].permute(2, 0, 1).reshape(N, M * C)
    h = torch.relu(y @ Wt[0].T)
    h = torch.relu(h @ Wt[1].T)
    f = (h @ Wt[2].T)[:, 0] * (model["vmax"] - model["vmin"]) + model["vmin"]
    (f * torch.tensor(df)).sum().backward()
    np.testing.assert_allclose(g["dG"], Gt.grad.numpy(), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(g["dF"], Ft.grad.numpy(), rtol=1e-10, atol=1e-10)
    for k in range(3):
        np.testing.assert_allclose(g["dW"][k], Wt[k].grad.numpy(), rtol=1e-10, atol=1e-10)


def test_outside_points_give_no_gradient():
    rng = np.random.default_rng(15)
    model = _tiny_model(rng)
    x = np.array([[3.0, 0.0, 0.0], [0.0, -2.5, 0.1], [np.nan, 0.2, 0.1]])
    g = O.backward(model, x, np.ones(3))
    assert np.all(g["dF"] == 0) and np.all(g["dG"] == 0)


def test_backward_magnitudes_bound_and_equal_the_gradient_when_signs_agree():
    rng = np.random.default_rng(60)
    host = synth.init_model(3, 2, 4, [6, 8, 8, 1], seed=61, grid_range=0.5)
    model = {"G": host["G"].astype(np.float64), "F": host["F"].astype(np.float64),
             "W": [w.astype(np.float64) for w in host["W"]], "vmin": -1.0, "vmax": 2.0}
    x = rng.uniform(-0.9, 0.9, size=(40, 3))
    df = rng.normal(size=40)
    g = O.backward(model, x, df)
    mag = O.backward_magnitudes(model, x, df)
    assert np.all(mag["dF"] >= np.abs(g["dF"]) - 1e-15)
    for a, b in zip(mag["dW"], g["dW"]):
        assert np.all(a >= np.abs(b) - 1e-15)
    # opening every unit can only enlarge the envelope
    _, cache = O.forward(model, x)
    opened = O.backward_magnitudes(model, x, df, cache,
                                   open_units=[np.ones_like(z, bool) for z in cache["z"][:-1]])
    assert np.all(opened["dF"] >= mag["dF"] - 1e-15)
    # one point, positive grids, weights and dL/df: every term is positive, so the sums of
    # absolute values are the gradient itself
    pos = dict(model, F=np.abs(model["F"]) + 0.1, W=[np.abs(w) + 0.01 for w in model["W"]], vmin=0.0, vmax=1.0)
    x1 = np.array([[0.05, -0.1, 0.2]])
    g1 = O.backward(pos, x1, np.array([0.7]))
    m1 = O.backward_magnitudes(pos, x1, np.array([0.7]))
    np.testing.assert_allclose(m1["dF"], g1["dF"], rtol=1e-14, atol=0)
    for a, b in zip(m1["dW"], g1["dW"]):
        np.testing.assert_allclose(a, b, rtol=1e-14, atol=0)
