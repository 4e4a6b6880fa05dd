"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars (float32 arithmetic): per output tensor, normwise relative error
||x - x*|| / ||x*|| <= 1e-5 and max |x - x*| <= 1e-5 ||x*||_inf.  Integer
outputs (mask, cells, brick ids, random points) are bit-exact: both sides
take those decisions in float32 with the same fma order.  For adjoint
tests, points whose hidden pre-activations come within 1e-4 (relative) of
a ReLU kink are dropped from the input set, since there the gradient is
not determined to float32 precision.  bf16/fp16 variants are stated, with
a loose sanity bound.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import apmg_oracle as O

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda"
TOL = 1e-5


def A():
    import paper_2308_02494_amd as mod
    return mod


def errs(got, want):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    nrm = np.linalg.norm(want)
    norm_rel = np.linalg.norm(got - want) / nrm if nrm > 0 else np.linalg.norm(got - want)
    inf = np.max(np.abs(want)) if want.size else 0.0
    max_rel = np.max(np.abs(got - want)) / inf if inf > 0 else (np.max(np.abs(got - want)) if got.size else 0.0)
    return norm_rel, max_rel


def assert_close(name, got, want, tol=TOL):
    a, b = errs(got, want)
    print(f"{name}: normwise {a:.2e}, max {b:.2e}", flush=True)
    assert a <= tol and b <= tol, (name, a, b)


def host_model(M, C, R, H, seed=1, grid_range=0.5, vmin=-3.5, vmax=12.25, extra_t=0.0):
    return synth.init_model(M, C, R, [M * C, H, H, 1], seed=seed, grid_range=grid_range,
                            extra_translation=extra_t, vmin=vmin, vmax=vmax)


def f64(model):
    return {"G": model["G"].astype(np.float64), "F": model["F"].astype(np.float64),
            "W": [w.astype(np.float64) for w in model["W"]], "vmin": float(model["vmin"]),
            "vmax": float(model["vmax"])}


def make_points(n, seed=3, special=True):
    x = synth.uniform_points_host(n, seed=seed).astype(np.float32)
    if special and n >= 16:
        x[0] = [1.0, 1.0, 1.0]
        x[1] = [-1.0, -1.0, -1.0]
        x[2] = [np.nan, 0.1, 0.2]
        x[3] = [1.3, 0.0, 0.0]
        x[4] = [0.0, -1.7, 0.4]
        x[5] = [0.0, 0.0, 0.0]
    return x


def soa(x):
    return torch.from_numpy(np.ascontiguousarray(x.T)).to(DEV)


SHAPES = [  # (M, C, R, H)
    (16, 2, 16, 64),
    (5, 1, 7, 64),
    (8, 4, 9, 128),
    (3, 2, 4, 64),
    (32, 2, 32, 64),
]


# --------------------------------------------------------------------------- decisions
@pytest.mark.parametrize("M,C,R,H", SHAPES[:3])
def test_cells_bit_exact(M, C, R, H):
    host = host_model(M, C, R, H, extra_t=0.2)
    x = make_points(5000)
    cell, inside = A().apmg_cells(A().Model.from_host(host, DEV), soa(x))
    oin, ocell = O.cell_decision_f32(O.local_coords_f32(host["G"], x), R)
    assert np.array_equal(inside.cpu().numpy().astype(bool), oin)
    assert np.array_equal(cell.cpu().numpy(), ocell.astype(np.int32))


def test_uniform_points_bit_exact():
    for step, stream, start, n in [(0, 0, 0, 1000), (5, 3, 123, 777), (2 ** 40, 79, 2 ** 33, 64)]:
        got = A().apmg_uniform_points(7, step, stream, start, n, DEV).cpu().numpy().T
        want = O.uniform_points(7, step, stream, n, start=start)
        assert np.array_equal(got.astype(np.float64), want)


def test_assign_bricks_bit_exact():
    shape = (1000, 1200, 900)
    t, _ = A().apmg_make_bricks(*shape, 256, 1)
    x = make_points(20000, special=False)
    x = np.concatenate([x, [[1, 1, 1], [-1, -1, -1], [np.nan, 0, 0], [2, -3, 0.5]]]).astype(np.float32)
    got = A().apmg_assign_bricks(t, soa(x)).cpu().numpy()
    dims, _ = O.brick_partition(shape, 256, 1)
    assert np.array_equal(got, O.brick_assign(x, shape, 256, dims))


def test_gt_sample():
    vol = synth.make_volume("blobs_turb", (37, 29, 41))
    x = make_points(8000, special=False)
    x = np.concatenate([x, [[1, 1, 1], [-1, -1, -1], [1, -1, 0]]]).astype(np.float32)
    got = A().apmg_gt_sample(vol.to(DEV), soa(x)).cpu().numpy()
    want = O.gt_sample(vol.numpy().astype(np.float64), x.astype(np.float64))
    assert_close("gt", got, want, 2e-6)


# --------------------------------------------------------------------------- forward
@pytest.mark.parametrize("M,C,R,H", SHAPES)
def test_forward_fp32(M, C, R, H):
    host = host_model(M, C, R, H)
    n = 4099
    x = make_points(n)
    got = A().apmg_forward(A().Model.from_host(host, DEV), soa(x)).cpu().numpy()
    want, _ = O.forward(f64(host), x.astype(np.float64))
    assert got[2] == np.float32(-3.5)                   # NaN point: outside every grid -> vmin
    assert_close(f"forward {M},{C},{R},{H}", got, want)


def test_forward_paper_init_c1():
    host = synth.init_model(16, 2, 16, [32, 64, 64, 1], seed=42)
    x = make_points(65536)
    got = A().apmg_forward(A().Model.from_host(host, DEV), soa(x)).cpu().numpy()
    want, _ = O.forward(f64(host), x.astype(np.float64))
    assert_close("forward c1 init", got - 0.0, want)


def test_forward_edge_sizes():
    host = host_model(6, 2, 8, 64)
    model = A().Model.from_host(host, DEV)
    for n in (1, 31, 32, 33, 63, 64, 65):
        x = make_points(n, seed=n, special=False)
        got = A().apmg_forward(model, soa(x)).cpu().numpy()
        want, _ = O.forward(f64(host), x.astype(np.float64))
        assert_close(f"forward n={n}", got, want)
    empty = torch.empty((3, 0), dtype=torch.float32, device=DEV)
    assert A().apmg_forward(model, empty).numel() == 0


def test_forward_spatially_sorted_path_equals_direct_bitwise():
    # from 2^15 points on the forward sorts the points into spatial bins first and scatters
    # the outputs back: every point's arithmetic is unchanged, so the values are the same bits
    # as chunks below the threshold; strided input (ld > n), NaN and outside points included
    host = host_model(16, 2, 16, 64, extra_t=0.1)
    model = A().Model.from_host(host, DEV)
    n, ld = 40000, 40017
    x = make_points(n)
    x[7:1000] *= 1.4
    pts = torch.zeros((3, ld), dtype=torch.float32, device=DEV)
    pts[:, :n] = soa(x)
    big = A().apmg_forward(model, pts, n=n, ld=ld)
    parts = [A().apmg_forward(model, soa(x[i:i + 20000])) for i in range(0, n, 20000)]
    assert torch.equal(big, torch.cat(parts))
    idx = np.random.default_rng(3).choice(n, 3000, replace=False)
    want, _ = O.forward(f64(host), x[idx].astype(np.float64))
    assert_close("forward sorted path, sample", big.cpu().numpy()[idx], want)


@pytest.mark.parametrize("grid16,bf", [(False, True), (True, False), (True, True)])
def test_forward_mixed_precision_stated(grid16, bf):
    host = host_model(16, 2, 16, 64)
    x = make_points(8192)
    model = A().Model.from_host(host, DEV, grid_dtype=torch.float16 if grid16 else torch.float32,
                                mlp_dtype=A().BF16 if bf else A().F32)
    got = A().apmg_forward(model, soa(x)).cpu().numpy()
    want, _ = O.forward(f64(host), x.astype(np.float64))
    a, b = errs(got, want)
    print(f"forward grid16={grid16} bf16={bf}: normwise {a:.2e} max {b:.2e}")
    assert a < 3e-2


# --------------------------------------------------------------------------- adjoint
def kink_free_mask(host, x, tau=1e-4):
    _, cache = O.forward(f64(host), x.astype(np.float64))
    keep = np.ones(x.shape[0], bool)
    for z in cache["z"][:-1]:
        scale = np.sqrt(np.mean(z * z, axis=1, keepdims=True)) + 1e-30
        keep &= np.all(np.abs(z) / scale > tau, axis=1)
    return keep


def kink_free(host, x, tau=1e-4):
    return x[kink_free_mask(host, x, tau)]


@pytest.mark.parametrize("M,C,R,H", SHAPES[:4] + [(32, 2, 8, 64), (32, 2, 32, 64), (24, 1, 6, 64)])
def test_backward_fp32(M, C, R, H):
    host = host_model(M, C, R, H, extra_t=0.1)
    x = kink_free(host, make_points(3001))
    n = x.shape[0]
    df = np.random.default_rng(4).normal(size=n).astype(np.float32)
    model = A().Model.from_host(host, DEV)
    dF, dG, dW = A().apmg_backward(model, soa(x), torch.from_numpy(df).to(DEV))
    go = O.backward(f64(host), x.astype(np.float64), df.astype(np.float64))
    assert_close("dF", dF.cpu().numpy(), go["dF"])
    assert_close("dG", dG.cpu().numpy(), go["dG"])
    for k in range(3):
        assert_close(f"dW{k + 1}", dW[k].cpu().numpy(), go["dW"][k])


@pytest.mark.parametrize("M,C,R,H", SHAPES + [(32, 2, 8, 64), (7, 4, 5, 64)])
def test_grid_gradient_gathers_agree_and_match_oracle(M, C, R, H):
    # the wave gather with and without the transform gradient gives the same grid gradient
    # bits, and is bitwise reproducible; the one-thread-per-cell gather is compared in the
    # training-step tests (it sums the same terms in another fixed order)
    host = host_model(M, C, R, H, extra_t=0.1)
    x = make_points(6001)
    df = np.random.default_rng(5).normal(size=x.shape[0]).astype(np.float32)
    model = A().Model.from_host(host, DEV)
    dF_w, _, _ = A().apmg_backward(model, soa(x), torch.from_numpy(df).to(DEV), want_dG=False)
    dF_w2, _, _ = A().apmg_backward(model, soa(x), torch.from_numpy(df).to(DEV), want_dG=False)
    dF_c, _, _ = A().apmg_backward(model, soa(x), torch.from_numpy(df).to(DEV), want_dG=True)
    assert torch.equal(dF_w, dF_w2)
    assert torch.equal(dF_w, dF_c)
    xk = kink_free(host, x)
    dfk = np.random.default_rng(6).normal(size=xk.shape[0]).astype(np.float32)
    dF_k, _, _ = A().apmg_backward(model, soa(xk), torch.from_numpy(dfk).to(DEV), want_dG=False)
    go = O.backward(f64(host), xk.astype(np.float64), dfk.astype(np.float64))
    assert_close("dF (wave gather)", dF_k.cpu().numpy(), go["dF"])


def _rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def test_grid_gradient_under_rotated_scaled_sheared_transforms():
    # grids turned by any angle, scaled 0.3x..2.5x, sheared and moved (one with exact zeros
    # off the diagonal): the gathers' spatial culling (bin rows, per-row x-ranges) must keep
    # every point of every cell; points outside the domain included
    rng = np.random.default_rng(21)
    M, C, R, H = 12, 2, 9, 64
    host = host_model(M, C, R, H, grid_range=0.5)
    for i in range(M):
        A_ = np.diag(rng.uniform(0.3, 2.5, 3)) @ _rotation(rng) + rng.normal(0.0, 0.1, (3, 3))
        if i == 0:
            A_ = np.diag([1.7, 0.6, 1.1])
        host["G"][i, :, :3] = A_
        host["G"][i, :, 3] = rng.normal(0.0, 0.5, 3)
    host["G"] = host["G"].astype(np.float32)
    x = make_points(20000)
    x[6:2000] *= 1.5
    df = np.random.default_rng(8).normal(size=x.shape[0]).astype(np.float32)
    model = A().Model.from_host(host, DEV)
    dF_w, _, _ = A().apmg_backward(model, soa(x), torch.from_numpy(df).to(DEV), want_dG=False)
    dF_c, _, _ = A().apmg_backward(model, soa(x), torch.from_numpy(df).to(DEV), want_dG=True)
    assert torch.equal(dF_w, dF_c)
    xk = kink_free(host, x)
    dfk = np.random.default_rng(9).normal(size=xk.shape[0]).astype(np.float32)
    dF_k, dG_k, _ = A().apmg_backward(model, soa(xk), torch.from_numpy(dfk).to(DEV))
    go = O.backward(f64(host), xk.astype(np.float64), dfk.astype(np.float64))
    assert_close("dF (wave gather, turned grids)", dF_k.cpu().numpy(), go["dF"])
    assert_close("dG (wave gather, turned grids)", dG_k.cpu().numpy(), go["dG"])
    # the one-thread-per-cell gather (reached through the training step's launch shapes) on the
    # same turned grids: the grids' first moments (0.1 * gradient) agree with the wave gather's
    vol = synth.make_volume("blobs_sine", (30, 34, 38)).to(DEV)
    nz, ny, nx = vol.shape
    _, bricks = A().apmg_make_bricks(nx, ny, nz, max(nx, ny, nz), 0)
    host["vmin"], host["vmax"] = np.float32(0.0), np.float32(1.0)
    steps = []
    for ck in (1, 2):
        tr = A().Trainer([host], vol, bricks, 20000, seed=5, tuning={"cell_kernel": ck})
        tr.step()
        steps.append(tr)
    torch.cuda.synchronize()
    assert_close("mF wave vs per-cell gather (turned grids)", steps[0].mF.cpu().numpy(),
                 steps[1].mF.cpu().numpy(), 1e-6)


@pytest.mark.parametrize("bf", [False, True])
def test_backward_activation_path_is_bitwise_reproducible(bf):
    # H = 128 with 256 input features: weight gradients from stored activations and the
    # chunked matrix-core products, no float atomics
    host = host_model(64, 4, 9, 128, grid_range=0.3)
    x = make_points(40000)
    df = torch.from_numpy(np.random.default_rng(2).normal(size=x.shape[0]).astype(np.float32)).to(DEV)
    model = A().Model.from_host(host, DEV, mlp_dtype=A().BF16 if bf else A().F32)
    r1 = A().apmg_backward(model, soa(x), df)
    r2 = A().apmg_backward(model, soa(x), df)
    assert torch.equal(r1[0], r2[0]) and torch.equal(r1[1], r2[1])
    for k in range(3):
        assert torch.equal(r1[2][k], r2[2][k])


def test_backward_accumulate_and_partial_outputs():
    host = host_model(4, 2, 6, 64)
    x = kink_free(host, make_points(500))
    df = np.ones(x.shape[0], np.float32)
    model = A().Model.from_host(host, DEV)
    dF, dG, dW = A().apmg_backward(model, soa(x), torch.from_numpy(df).to(DEV))
    dF2, dG2, dW2 = A().apmg_backward(model, soa(x), torch.from_numpy(df).to(DEV), flags=A().ACCUMULATE,
                                      dF=dF.clone(), dG=dG.clone(), dW=[w.clone() for w in dW])
    assert_close("dF x2", dF2.cpu().numpy(), 2 * dF.cpu().numpy(), 1e-6)
    assert_close("dG x2", dG2.cpu().numpy(), 2 * dG.cpu().numpy(), 1e-6)
    assert_close("dW1 x2", dW2[0].cpu().numpy(), 2 * dW[0].cpu().numpy(), 1e-6)
    only_w = A().apmg_backward(model, soa(x), torch.from_numpy(df).to(DEV), want_dF=False, want_dG=False)
    assert_close("dW2 alone", only_w[2][1].cpu().numpy(), dW[1].cpu().numpy(), 1e-6)


def test_backward_empty_batch():
    # an empty batch: the gradients of an empty sum are zero (outputs pre-filled with 7 so the
    # clearing is seen), and under ACCUMULATE the outputs keep their values bit for bit
    host = host_model(4, 2, 6, 64)
    model = A().Model.from_host(host, DEV)
    empty = torch.empty((3, 0), dtype=torch.float32, device=DEV)
    no_df = torch.empty(0, dtype=torch.float32, device=DEV)
    dF0 = torch.full(model.F.shape, 7.0, dtype=torch.float32, device=DEV)
    dG0 = torch.full(tuple(model.G.shape), 7.0, dtype=torch.float64, device=DEV)
    dW0 = [torch.full_like(w, 7.0) for w in model.W]
    dF, dG, dW = A().apmg_backward(model, empty, no_df, dF=dF0, dG=dG0, dW=dW0)
    torch.cuda.synchronize()
    assert not dF.any() and not dG.any() and not any(w.any() for w in dW)
    x = make_points(300, special=False)
    dF1, dG1, dW1 = A().apmg_backward(model, soa(x), torch.ones(x.shape[0], device=DEV))
    dF2, dG2, dW2 = A().apmg_backward(model, empty, no_df, flags=A().ACCUMULATE, dF=dF1.clone(),
                                      dG=dG1.clone(), dW=[w.clone() for w in dW1])
    assert torch.equal(dF2, dF1) and torch.equal(dG2, dG1)
    assert all(torch.equal(a, b) for a, b in zip(dW2, dW1))


def test_backward_wide_first_layer_activation_path():
    # 256 input features and 128 hidden: outside the register-resident adjoint, so the weight
    # gradients come from the stored activations and the matrix-core products
    host = host_model(64, 4, 5, 128, grid_range=0.3)
    x = kink_free(host, make_points(1500))
    df = np.random.default_rng(5).normal(size=x.shape[0]).astype(np.float32)
    model = A().Model.from_host(host, DEV, mlp_dtype=A().F32)
    dF, dG, dW = A().apmg_backward(model, soa(x), torch.from_numpy(df).to(DEV))
    go = O.backward(f64(host), x.astype(np.float64), df.astype(np.float64))
    assert_close("dF", dF.cpu().numpy(), go["dF"])
    assert_close("dG", dG.cpu().numpy(), go["dG"])
    for k in range(3):
        assert_close(f"dW{k + 1}", dW[k].cpu().numpy(), go["dW"][k])


def test_autograd_function_matches_oracle():
    host = host_model(6, 2, 8, 64)
    x = kink_free(host, make_points(700))
    model = A().Model.from_host(host, DEV)
    G = model.G.clone().requires_grad_(True)
    F = model.F.clone().requires_grad_(True)
    Ws = [w.clone().requires_grad_(True) for w in model.W]
    f = A().APMGFunction.apply(torch.from_numpy(x).to(DEV), G, F, *Ws, model.vmin, model.vmax, A().F32)
    wts = torch.linspace(-1, 1, x.shape[0], device=DEV)
    (f * wts).sum().backward()
    go = O.backward(f64(host), x.astype(np.float64), wts.cpu().numpy().astype(np.float64))
    assert_close("autograd dG", G.grad.cpu().numpy(), go["dG"])
    assert_close("autograd dF", F.grad.cpu().numpy(), go["dF"])
    assert_close("autograd dW1", Ws[0].grad.cpu().numpy(), go["dW"][0])


# --------------------------------------------------------------------------- density
@pytest.mark.parametrize("M,n", [(16, 4099), (5, 1000), (32, 65536)])
def test_density_loss_same_err(M, n):
    host = host_model(M, 2, 8, 64, seed=M, extra_t=0.3)
    x = make_points(n, special=False)
    err = (np.random.default_rng(6).uniform(0, 1, n) ** 3).astype(np.float32)
    model = A().Model.from_host(host, DEV)
    loss, dG, rho = A().apmg_density_loss(model, soa(x), torch.from_numpy(err).to(DEV), eps=1e-12, p=10,
                                          want_rho=True)
    r = O.density_loss(host["G"].astype(np.float64), x.astype(np.float64), err.astype(np.float64), eps=1e-12)
    assert_close("rho", rho.cpu().numpy(), r["rho"])
    assert_close("L_density", loss.cpu().numpy(), [r["loss"]])
    assert_close("dG_density", dG.cpu().numpy(), r["dG"])


def test_density_loss_edge_cases():
    host = host_model(3, 2, 4, 64)
    model = A().Model.from_host(host, DEV)
    empty = torch.empty((3, 0), dtype=torch.float32, device=DEV)
    loss, dG, _ = A().apmg_density_loss(model, empty, torch.empty(0, device=DEV))
    assert loss.item() == 0.0 and torch.all(dG == 0)
    # every point far outside every grid: S = 0 -> loss 0, gradient 0
    x = np.full((100, 3), 5.0, np.float32)
    loss, dG, _ = A().apmg_density_loss(model, soa(x), torch.ones(100, device=DEV))
    assert loss.item() == 0.0 and torch.all(dG == 0)


# --------------------------------------------------------------------------- training step
def oracle_step(host, vol_np, brick, seed, step, stream, n, active, flags_rec=False):
    x = O.uniform_points(seed, step, stream, n)
    v = O.brick_gt_sample(vol_np, brick, x)
    st = O.zero_adam_state(f64(host))
    m2 = dict(f64(host))
    m2["vmin"], m2["vmax"] = 0.0, 1.0
    return O.train_step(m2, st, x, v, density_active=active, add_rec_dG=flags_rec)


@pytest.mark.parametrize("nb_shape", [(1, None), (3, (40, 50, 60))])
def test_batched_step_matches_oracle(nb_shape):
    nb_req, shape = nb_shape
    vol = synth.make_volume("blobs_sine", (48, 40, 36) if shape is None else shape[::-1])
    nz, ny, nx = vol.shape
    if nb_req == 1:
        _, bricks = A().apmg_make_bricks(nx, ny, nz, max(nx, ny, nz), 0)
    else:
        _, bricks = A().apmg_make_bricks(nx, ny, nz, 32, 1)
        bricks = bricks[:nb_req]
    nb = len(bricks)
    hosts = [host_model(8, 2, 8, 64, seed=10 + b, grid_range=0.2, vmin=0.0, vmax=1.0) for b in range(nb)]
    n = 2000
    tr = A().Trainer(hosts, vol.to(DEV), bricks, n, seed=7)
    tr.density_active.fill_(1)
    tr.step()
    torch.cuda.synchronize()
    vol_np = vol.numpy().astype(np.float64)
    _, obricks = O.brick_partition((nx, ny, nz), 32 if nb_req > 1 else max(nx, ny, nz), 1 if nb_req > 1 else 0)
    for b in range(nb):
        new_m, new_s, info = oracle_step(hosts[b], vol_np, obricks[b], 7, 0, b, n, True)
        L = tr.losses[b].cpu().numpy()
        assert_close(f"L_rec[{b}]", [L[0]], [info["L_rec"]])
        # density loss depends on h = (f - v)^2 computed in float32: stated, loose bar
        a, _ = errs([L[1]], [info["L_density"]])
        print(f"L_density[{b}] rel err {a:.2e}")
        assert a < 1e-3
        # Adam first moments are (1 - beta1) * gradient
        assert_close(f"mF[{b}]", tr.mF[b].cpu().numpy(), new_s["mF"])
        mW = tr.mW[b].cpu().numpy()
        o = 0
        for k, w in enumerate(new_s["mW"]):
            assert_close(f"mW{k + 1}[{b}]", mW[o:o + w.size].reshape(w.shape), w)
            o += w.size
        a, _ = errs(tr.mG[b].cpu().numpy(), new_s["mG"])
        print(f"mG[{b}] rel err {a:.2e}")
        assert a < 1e-3
    assert int(tr.step_ctr.item()) == 1 and int(tr.t[0].item()) == 1 and int(tr.tG[0].item()) == 1


def test_batched_step_activation_path_matches_oracle_and_is_reproducible():
    # H = 128 with 32 input features: outside the register-resident adjoint, the step takes
    # its weight gradients from stored activations and matrix-core products (two models)
    vol = synth.make_volume("blobs_sine", (40, 44, 36))
    nz, ny, nx = vol.shape
    _, bricks = A().apmg_make_bricks(nx, ny, nz, 24, 1)
    bricks = bricks[:2]
    hosts = [host_model(8, 4, 8, 128, seed=30 + b, grid_range=0.2, vmin=0.0, vmax=1.0) for b in range(2)]
    n = 2500
    trs = []
    for _ in range(2):
        tr = A().Trainer(hosts, vol.to(DEV), bricks, n, seed=9)
        tr.density_active.fill_(1)
        tr.step()
        trs.append(tr)
    torch.cuda.synchronize()
    for x, y in zip((trs[0].F, trs[0].W, trs[0].G, trs[0].mW), (trs[1].F, trs[1].W, trs[1].G, trs[1].mW)):
        assert torch.equal(x, y)
    tr = trs[0]
    vol_np = vol.numpy().astype(np.float64)
    _, obricks = O.brick_partition((nx, ny, nz), 24, 1)
    for b in range(2):
        new_m, new_s, info = oracle_step(hosts[b], vol_np, obricks[b], 9, 0, b, n, True)
        assert_close(f"L_rec[{b}]", [tr.losses[b, 0].item()], [info["L_rec"]])
        assert_close(f"mF[{b}]", tr.mF[b].cpu().numpy(), new_s["mF"])
        mW = tr.mW[b].cpu().numpy()
        o = 0
        for k, w in enumerate(new_s["mW"]):
            assert_close(f"mW{k + 1}[{b}]", mW[o:o + w.size].reshape(w.shape), w)
            o += w.size


@pytest.mark.parametrize("cell_kernel", [1, 2])
def test_batched_step_with_rec_transform_gradient_matches_oracle(cell_kernel):
    # APMG_ADD_REC_DG: L_rec's transform gradient (through the trilinear weights) is added to
    # the density gradient, from the wave gather (1) or the one-thread-per-cell gather (2)
    vol = synth.make_volume("blobs_sine", (48, 40, 36))
    nz, ny, nx = vol.shape
    _, bricks = A().apmg_make_bricks(nx, ny, nz, max(nx, ny, nz), 0)
    host = host_model(8, 2, 8, 64, seed=12, grid_range=0.2, vmin=0.0, vmax=1.0, extra_t=0.1)
    n = 3000
    tr = A().Trainer([host], vol.to(DEV), bricks, n, seed=7, flags=A().ADD_REC_DG,
                     tuning={"cell_kernel": cell_kernel})
    tr.density_active.fill_(1)
    tr.step()
    torch.cuda.synchronize()
    _, obricks = O.brick_partition((nx, ny, nz), max(nx, ny, nz), 0)
    new_m, new_s, info = oracle_step(host, vol.numpy().astype(np.float64), obricks[0], 7, 0, 0, n, True,
                                     flags_rec=True)
    assert_close("mF", tr.mF[0].cpu().numpy(), new_s["mF"])
    a, _ = errs(tr.mG[0].cpu().numpy(), new_s["mG"])
    print(f"mG (density + L_rec transform gradient), gather {cell_kernel}: rel err {a:.2e}")
    assert a < 1e-3


# --------------------------------------------------------------------------- graphs, determinism
def _trainer(A_, vol, nb=2, n=3000, mlp=None):
    nz, ny, nx = vol.shape
    _, bricks = A_.apmg_make_bricks(nx, ny, nz, 24, 1)
    bricks = bricks[:nb]
    hosts = [host_model(8, 2, 8, 64, seed=20 + b, grid_range=0.2, vmin=0.0, vmax=1.0) for b in range(nb)]
    tr = A_.Trainer(hosts, vol, bricks, n, seed=3, mlp_dtype=A_.F32 if mlp is None else mlp)
    tr.density_active.fill_(1)
    return tr


def _state(tr):
    return [t.clone() for t in (tr.G, tr.F, tr.W, tr.mG, tr.vG, tr.mF, tr.vF, tr.mW, tr.vW, tr.losses)]


def test_training_step_is_bitwise_deterministic():
    vol = synth.make_volume("blobs_turb", (40, 48, 44)).to(DEV)
    a, b = _trainer(A(), vol), _trainer(A(), vol)
    for _ in range(3):
        a.step()
        b.step()
    torch.cuda.synchronize()
    for x, y in zip(_state(a), _state(b)):
        assert torch.equal(x, y)


def test_graph_replay_matches_eager_steps():
    # the step records no memset, so it can be captured; replays advance the device step
    # counter, and every replay must equal the corresponding eager step
    vol = synth.make_volume("blobs_turb", (40, 48, 44)).to(DEV)
    eager, graphed = _trainer(A(), vol), _trainer(A(), vol)
    eager.step()
    graphed.step()                    # warm-up outside the capture (same first step)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            graphed.step()
    torch.cuda.synchronize()
    # capture does not execute: replay now performs step 2, then 3, 4
    for k in range(3):
        g.replay()
        eager.step()
        torch.cuda.synchronize()
        _ = (eager.W * 2).sum().item()  # unrelated eager work between replays
        for x, y in zip(_state(eager), _state(graphed)):
            assert torch.equal(x, y), k
    assert int(graphed.step_ctr.item()) == 4


# --------------------------------------------------------------------------- large model (render workload shape)
def test_forward_wide_fp32_weights_outside_lds():
    # 256 input features, 128 hidden, fp32: the operands exceed the LDS budget and are read
    # from global memory
    host = host_model(64, 4, 9, 128, grid_range=0.3)
    x = make_points(3000)
    got = A().apmg_forward(A().Model.from_host(host, DEV), soa(x)).cpu().numpy()
    want, _ = O.forward(f64(host), x.astype(np.float64))
    assert_close("forward 64x4 fp32", got, want)


def test_render_model_bf16_forward_sampled():
    # 64 grids at 64^3 x 4 features, MLP 256-128-128-1 in bf16; render-style points
    host = synth.init_model(64, 4, 64, [256, 128, 128, 1], seed=5, grid_range=1.0, extra_translation=0.3)
    pts = synth.ray_points(160, 90, 8)
    model = A().Model.from_host(host, DEV, mlp_dtype=A().BF16)
    got = A().apmg_forward(model, soa(pts)).cpu().numpy()
    idx = np.random.default_rng(0).choice(pts.shape[0], 2048, replace=False)
    want, _ = O.forward(f64(host), pts[idx].astype(np.float64))
    a, b = errs(got[idx], want)
    print(f"render bf16 forward: normwise {a:.2e} max {b:.2e}")
    assert a < 3e-2


def _perturbed(host, dirs, t):
    out = dict(host)
    out["G"] = (host["G"].astype(np.float64) + t * dirs["G"]).astype(np.float32)
    out["F"] = (host["F"].astype(np.float64) + t * dirs["F"]).astype(np.float32)
    out["W"] = [(w.astype(np.float64) + t * d).astype(np.float32) for w, d in zip(host["W"], dirs["W"])]
    return out


def _smooth_segment_points(hosts, x, margin=1e-6):
    # points whose mask, interpolation cell and ReLU pattern are the same at every model of the
    # segment: along the segment f is then a polynomial of degree <= 3 in t
    keep = np.ones(x.shape[0], bool)
    ref = None
    for h in hosts:
        _, c = O.forward(f64(h), x.astype(np.float64))
        sig = (c["enc"]["inside"], c["enc"]["cell"], [z > 0 for z in c["z"][:-1]])
        for z in c["z"][:-1]:
            keep &= np.all(np.abs(z) > margin, axis=1)
        if ref is None:
            ref = sig
            continue
        keep &= np.all(sig[0] == ref[0], axis=1)
        keep &= np.all((sig[1] == ref[1]).reshape(x.shape[0], -1), axis=1)
        for a, b in zip(sig[2], ref[2]):
            keep &= np.all(a == b, axis=1)
    return x[keep]


def _central_difference_check(host, dirs, h, x, wts_seed, tol, name):
    hp, hm = _perturbed(host, dirs, h), _perturbed(host, dirs, -h)
    x = _smooth_segment_points([hm, host, hp], x)
    n = x.shape[0]
    wts = (np.random.default_rng(wts_seed).normal(size=n) / n).astype(np.float32)
    pts, wd = soa(x), torch.from_numpy(wts).to(DEV)
    dF, dG, dW = A().apmg_backward(A().Model.from_host(host, DEV), pts, wd)
    # the step actually taken, after float32 rounding of the perturbed parameters
    step = {"G": hp["G"].astype(np.float64) - hm["G"], "F": hp["F"].astype(np.float64) - hm["F"],
            "W": [a.astype(np.float64) - b for a, b in zip(hp["W"], hm["W"])]}
    pred = float((dG.cpu().numpy().astype(np.float64) * step["G"]).sum()
                 + (dF.cpu().numpy().astype(np.float64) * step["F"]).sum()
                 + sum((g.cpu().numpy().astype(np.float64) * d).sum() for g, d in zip(dW, step["W"])))

    def L(hh):
        f = A().apmg_forward(A().Model.from_host(hh, DEV), pts).cpu().numpy().astype(np.float64)
        return float((f * wts.astype(np.float64)).sum())

    fd = L(hp) - L(hm)
    rel = abs(fd - pred) / abs(pred)
    print(f"{name}: points {n} adjoint {pred:.6e} central difference {fd:.6e} rel {rel:.2e}")
    assert n > 1000
    assert rel < tol


def test_adjoint_central_differences():
    # The adjoint applied to a random step equals the change of sum_n w_n f(x_n) over that step,
    # on points that cross no ReLU kink, cell face or mask face along it (there f is a cubic in
    # the step, and a central difference is exact up to O(h^2) and rounding).  Steps along F,
    # along the three MLP matrices, and along the 32 transforms, at the 32-grid, 32^3 shape.
    host = synth.init_model(32, 2, 32, [64, 64, 64, 1], seed=9, grid_range=0.3)
    rng = np.random.default_rng(21)
    zero = {"G": np.zeros(host["G"].shape), "F": np.zeros(host["F"].shape),
            "W": [np.zeros(w.shape) for w in host["W"]]}
    x = synth.uniform_points_host(32768, seed=13)
    dirs = dict(zero, F=0.3 * rng.normal(size=host["F"].shape))
    _central_difference_check(host, dirs, 1e-3, x, 1, 1e-3, "F")
    dirs = dict(zero, W=[np.abs(w).max() * rng.normal(size=w.shape) for w in host["W"]])
    _central_difference_check(host, dirs, 1e-3, x, 2, 1e-3, "W")
    dirs = dict(zero, G=rng.normal(size=host["G"].shape))
    _central_difference_check(host, dirs, 1e-4, x, 3, 1e-3, "G")


def test_adjoint_2e20_points_sampled_vertices_and_partition():
    # 2^20 points at the 32-grid, 32^3 shape.  dF at sampled vertices equals the oracle's sum
    # over the points of the vertex's 8 cells; the gradients over the whole batch equal the sum
    # of the gradients over four quarter batches (each sorted and reduced on its own), and one
    # quarter matches the oracle on all of dF, dG and dW.
    host = synth.init_model(32, 2, 32, [64, 64, 64, 1], seed=9, grid_range=0.3)
    model = A().Model.from_host(host, DEV)
    n, R = 1 << 20, 32
    pts = A().apmg_uniform_points(17, 0, 0, 0, n, DEV)
    x = pts.cpu().numpy().T.astype(np.float32).copy()
    rng = np.random.default_rng(3)
    wa = (rng.normal(size=n) / n).astype(np.float32)
    dF, dG, dW = A().apmg_backward(model, pts, torch.from_numpy(wa).to(DEV))
    parts = []
    q = n // 4
    for k in range(4):
        parts.append(A().apmg_backward(model, pts[:, k * q:(k + 1) * q].contiguous(),
                                       torch.from_numpy(wa[k * q:(k + 1) * q]).to(DEV)))
    assert_close("partition dF", dF.cpu().numpy(), sum(p[0] for p in parts).cpu().numpy())
    assert_close("partition dG", dG.cpu().numpy(), sum(p[1] for p in parts).cpu().numpy())
    for k in range(3):
        assert_close(f"partition dW{k + 1}", dW[k].cpu().numpy(), sum(p[2][k] for p in parts).cpu().numpy())
    # one 2^16 slice of the first quarter against the oracle
    s = 1 << 16
    keep = kink_free_mask(host, x[:s])
    sub = x[:s][keep]
    dFs, dGs, dWs = A().apmg_backward(model, soa(sub), torch.from_numpy(wa[:s][keep]).to(DEV))
    go = O.backward(f64(host), sub.astype(np.float64), wa[:s][keep].astype(np.float64))
    assert_close("slice dF", dFs.cpu().numpy(), go["dF"])
    assert_close("slice dG", dGs.cpu().numpy(), go["dG"])
    for k in range(3):
        assert_close(f"slice dW{k + 1}", dWs[k].cpu().numpy(), go["dW"][k])
    dF = dF.cpu().numpy()
    scale = np.abs(dF).max()
    checked = 0
    decisions = {}
    for trial in range(40):
        g = int(rng.integers(0, 32))
        v = rng.integers(1, R - 1, size=3)          # (vx, vy, vz), interior
        if g not in decisions:
            decisions[g] = O.cell_decision_f32(O.local_coords_f32(host["G"][g:g + 1], x), R)
        inside, cell = decisions[g]
        sel = inside[:, 0] & np.all((cell[:, 0, :] == v) | (cell[:, 0, :] == v - 1), axis=1)
        sub = x[sel]
        _, cache = O.forward(f64(host), sub.astype(np.float64))
        if any(np.any(np.abs(z) < 1e-6) for z in cache["z"][:-1]):
            continue                                # a pre-activation within float32 reach of 0
        go = O.backward(f64(host), sub.astype(np.float64), wa[sel].astype(np.float64), cache)
        want = go["dF"][g, :, v[2], v[1], v[0]]
        got = dF[g, :, v[2], v[1], v[0]]
        err = np.max(np.abs(got - want))
        print(f"vertex g={g} v={tuple(v)} points={sel.sum()} want={want} err={err:.2e}")
        assert err <= 1e-5 * max(np.max(np.abs(want)), 1e-2 * scale)
        checked += 1
        if checked == 8:
            break
    assert checked >= 6


def test_render_shape_backward_2e20_points():
    # the render workload's model (64 grids at 64^3 x 4 features, MLP 256-128-128-1) with a
    # 2^20-point backward: FP32 MLP against the oracle on a slice and by batch partition,
    # central differences along F on kink-free segments; the BF16 MLP's gradient error stated
    host = synth.init_model(64, 4, 64, [256, 128, 128, 1], seed=5, grid_range=1.0, extra_translation=0.3)
    n = 1 << 20
    pts = A().apmg_uniform_points(23, 0, 0, 0, n, DEV)
    x = pts.cpu().numpy().T.astype(np.float32).copy()
    w = (np.random.default_rng(8).normal(size=n) / n).astype(np.float32)
    model = A().Model.from_host(host, DEV)
    dF, dG, dW = A().apmg_backward(model, pts, torch.from_numpy(w).to(DEV))
    half = n // 2
    p1 = A().apmg_backward(model, pts[:, :half].contiguous(), torch.from_numpy(w[:half]).to(DEV))
    p2 = A().apmg_backward(model, pts[:, half:].contiguous(), torch.from_numpy(w[half:]).to(DEV))
    assert_close("partition dF", dF.cpu().numpy(), (p1[0] + p2[0]).cpu().numpy())
    assert_close("partition dG", dG.cpu().numpy(), (p1[1] + p2[1]).cpu().numpy())
    for k in range(3):
        assert_close(f"partition dW{k + 1}", dW[k].cpu().numpy(), (p1[2][k] + p2[2][k]).cpu().numpy())
    s = 4096
    keep = kink_free_mask(host, x[:s])
    sub, ws_ = x[:s][keep], w[:s][keep]
    g_ = A().apmg_backward(model, soa(sub), torch.from_numpy(ws_).to(DEV))
    go = O.backward(f64(host), sub.astype(np.float64), ws_.astype(np.float64))
    assert_close("slice dF", g_[0].cpu().numpy(), go["dF"])
    assert_close("slice dG", g_[1].cpu().numpy(), go["dG"])
    for k in range(3):
        assert_close(f"slice dW{k + 1}", g_[2][k].cpu().numpy(), go["dW"][k])
    rng = np.random.default_rng(31)
    zero = {"G": np.zeros(host["G"].shape), "F": np.zeros(host["F"].shape),
            "W": [np.zeros(wk.shape) for wk in host["W"]]}
    _central_difference_check(host, dict(zero, F=0.3 * rng.normal(size=host["F"].shape)), 1e-3,
                              synth.uniform_points_host(16384, seed=17), 4, 1e-3, "render F")
    # BF16 operands (8-bit mantissas) through a 256-128-128 MLP: the error is stated, with a
    # sanity bound only
    mb = A().Model.from_host(host, DEV, mlp_dtype=A().BF16)
    gb = A().apmg_backward(mb, soa(sub), torch.from_numpy(ws_).to(DEV))
    for name, got, want in (("dF", gb[0].cpu().numpy(), go["dF"]),
                            ("dG", gb[1].cpu().numpy(), go["dG"]),
                            ("dW1", gb[2][0].cpu().numpy(), go["dW"][0]),
                            ("dW2", gb[2][1].cpu().numpy(), go["dW"][1]),
                            ("dW3", gb[2][2].cpu().numpy(), go["dW"][2])):
        a, _ = errs(got, want)
        print(f"render bf16 backward {name}: normwise {a:.2e}")
        assert a < 0.2


# --------------------------------------------------------------------------- boundary layouts
def test_abi_paper_order_grids_and_4x4_transforms():
    # The boundary takes the encoder tensor in the paper's [M, C, D, H, W] order (Sec. 4.1.1)
    # and the full 4x4 matrices of Eq. (1) (row 3 is never read: filled with junk here), and
    # returns dF and dG in those shapes (row 3 of dG zero).  A caller that keeps its grids
    # channel-last and its transforms as 3x4 gets bitwise the same values.
    A_ = A()
    host = host_model(8, 2, 8, 64, extra_t=0.1)
    x = kink_free(host, make_points(3001))
    n = x.shape[0]
    df = np.random.default_rng(41).normal(size=n).astype(np.float32)
    G4 = np.zeros((8, 4, 4), np.float32)
    G4[:, :3, :] = host["G"]
    G4[:, 3, :] = [7.0, -3.0, np.nan, 2.0]
    W = [torch.from_numpy(w).to(DEV) for w in host["W"]]
    F = torch.from_numpy(host["F"]).to(DEV)
    m4 = A_.Model(torch.from_numpy(G4).to(DEV), F, W, host["vmin"], host["vmax"])
    pts, dft = soa(x), torch.from_numpy(df).to(DEV)
    f = A_.apmg_forward(m4, pts)
    want, _ = O.forward(f64(host), x.astype(np.float64))
    assert_close("forward (paper order, 4x4)", f.cpu().numpy(), want)
    dF, dG, dW = A_.apmg_backward(m4, pts, dft)
    assert tuple(dF.shape) == (8, 2, 8, 8, 8) and tuple(dG.shape) == (8, 4, 4)
    assert torch.all(dG[:, 3, :] == 0)
    go = O.backward(f64(host), x.astype(np.float64), df.astype(np.float64))
    assert_close("dF (paper order)", dF.cpu().numpy(), go["dF"])
    assert_close("dG (4x4)", dG[:, :3, :].cpu().numpy(), go["dG"])
    for k in range(3):
        assert_close(f"dW{k + 1}", dW[k].cpu().numpy(), go["dW"][k])
    # channel-last grids, 3x4 transforms
    Fcl = A_.apmg_convert_grids(F, True)
    mcl = A_.Model(torch.from_numpy(host["G"]).to(DEV), Fcl, W, host["vmin"], host["vmax"], layout=A_.GRIDS_MRRRC)
    assert torch.equal(A_.apmg_forward(mcl, pts), f)
    dF2, dG2, dW2 = A_.apmg_backward(mcl, pts, dft)
    assert torch.equal(A_.apmg_convert_grids(dF2, False), dF)
    assert torch.equal(dG2, dG[:, :3, :])
    for k in range(3):
        assert torch.equal(dW2[k], dW[k])
    # the density loss with 4x4 transforms
    err = torch.from_numpy((np.random.default_rng(42).uniform(0, 1, n) ** 2).astype(np.float32)).to(DEV)
    l4, g4, _ = A_.apmg_density_loss(m4, pts, err)
    l3, g3, _ = A_.apmg_density_loss(mcl, pts, err)
    assert l4.item() == l3.item()
    assert torch.equal(g4[:, :3, :], g3) and torch.all(g4[:, 3, :] == 0)
    # autograd with paper-order grids and 4x4 transforms
    Gp = torch.from_numpy(G4).to(DEV).requires_grad_(True)
    Fp = F.clone().requires_grad_(True)
    Wp = [w.clone().requires_grad_(True) for w in W]
    out = A_.APMGFunction.apply(torch.from_numpy(x).to(DEV), Gp, Fp, *Wp, float(host["vmin"]),
                                float(host["vmax"]), A_.F32)
    (out * dft).sum().backward()
    assert torch.equal(Fp.grad, dF) and torch.all(Gp.grad[:, 3, :] == 0)
    assert_close("autograd dG (4x4)", Gp.grad[:, :3, :].cpu().numpy(), go["dG"])


def test_backward_large_batch_bin_starts_by_search():
    # more than 8 points per spatial bin (2^21 + 4096 points): the bin starts come from one
    # binary search per bin instead of one thread per position; the gradients equal the sum
    # of the two halves' (each under the per-position path), to float32 rounding of the sums
    host = host_model(8, 2, 16, 64, extra_t=0.1)
    n = (1 << 21) + 4096
    x = synth.uniform_points_host(n, seed=41).astype(np.float32)
    x[:4096] = 0.02 * x[:4096] + 0.5                   # a dense clump, so that many bins stay empty
    # positive weights: the sums do not cancel, so their float32 rounding stays far below the bar
    df = np.random.default_rng(42).uniform(0.5, 1.5, size=n).astype(np.float32)
    model = A().Model.from_host(host, DEV)
    xd, dfd = soa(x), torch.from_numpy(df).to(DEV)
    dF, dG, dW = A().apmg_backward(model, xd, dfd)
    h = n // 2
    xa, xb = soa(x[:h]), soa(x[h:])
    dFa, dGa, dWa = A().apmg_backward(model, xa, dfd[:h].contiguous())
    dFb, dGb, dWb = A().apmg_backward(model, xb, dfd[h:].contiguous())
    assert_close("dF (one call vs halves)", dF.cpu().numpy(), (dFa + dFb).cpu().numpy())
    assert_close("dG (one call vs halves)", dG.cpu().numpy(), (dGa + dGb).cpu().numpy())
    for k in range(3):
        assert_close(f"dW{k + 1} (one call vs halves)", dW[k].cpu().numpy(), (dWa[k] + dWb[k]).cpu().numpy())
