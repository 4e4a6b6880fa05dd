"""Pins for the oracle's feature density and density loss (Sec. 4.2,
Eqs. (7)-(9)) and its gradient with the target density held constant."""
import decimal
from decimal import Decimal

import numpy as np
import torch

from oracle import apmg_oracle as O


def _scaled_identity(s, M=1):
    G = np.zeros((M, 3, 4))
    G[:, [0, 1, 2], [0, 1, 2]] = s
    return G


def test_density_closed_forms():
    s = 1.7
    G = _scaled_identity(s)
    x = np.array([[0.0, 0.0, 0.0], [1.0 / s, 0.0, 0.0], [0.0, -1.0 / s, 0.0]])
    rho, _, _, _ = O.density_terms(G, x)
    np.testing.assert_allclose(rho[0], s ** 3, rtol=1e-15)            # centre
    np.testing.assert_allclose(rho[1:], s ** 3 * np.exp(-1.0), rtol=1e-15)  # face centres


def test_flat_top_approaches_box_of_eq5():
    # For |l|_inf <= 1/2 the flat-top density is within 3*2^-20 of det (Eq. (5));
    # far outside it vanishes.
    rng = np.random.default_rng(20)
    G = _scaled_identity(1.0)
    G[0, :3, :3] = np.eye(3) + rng.normal(0, 0.05, (3, 3))
    det = np.linalg.det(G[0, :3, :3])
    l_in = rng.uniform(-0.5, 0.5, size=(200, 3))
    x_in = np.linalg.solve(G[0, :3, :3], l_in.T).T
    rho, _, _, _ = O.density_terms(G, x_in)
    assert np.all(np.abs(1 - rho / det) < 3 * 2.0 ** -20)
    x_out = np.linalg.solve(G[0, :3, :3], np.array([[1.5, 0, 0], [0, 0, -2.0]]).T).T
    rho_o, _, _, _ = O.density_terms(G, x_out)
    assert np.all(rho_o < 1e-30 * det)


def test_uniform_error_gives_zero_loss_and_gradient():
    rng = np.random.default_rng(21)
    G = _scaled_identity(1.0, M=3) + rng.normal(0, 0.1, (3, 3, 4))
    x = rng.uniform(-1, 1, size=(64, 3))
    h = np.full(64, 0.37)
    r = O.density_loss(G, x, h, eps=0.0)
    assert abs(r["loss"]) < 1e-15
    assert np.max(np.abs(r["dG"])) < 1e-13


def test_two_point_closed_form_in_50_digit_decimal():
    decimal.getcontext().prec = 50
    s, a, h1, h2, eps = 1.3, 0.93, 0.02, 0.35, 1e-12
    G = _scaled_identity(s)
    x = np.array([[0.0, 0.0, 0.0], [a / s, 0.0, 0.0]])
    r = O.density_loss(G, x, np.array([h1, h2]), eps=eps)
    D = Decimal
    S3 = D(s) ** 3
    rho = [S3, S3 * (-(D(a / s) * D(s)) ** 20).exp()]
    S = rho[0] + rho[1]
    rs = [v / S for v in rho]
    hb = (D(h1) + D(h2)) / 2
    L = D(0)
    for j, hj in enumerate((h1, h2)):
        lt = hb / (D(hj) + D(eps)) * (rs[j] + D(eps)).ln()
        L += lt.exp() * (lt - (rs[j] + D(eps)).ln())
    L /= 2
    np.testing.assert_allclose(r["loss"], float(L), rtol=1e-13)


def test_duplicated_grids_leave_loss_and_halve_gradient():
    rng = np.random.default_rng(22)
    G = _scaled_identity(1.1, M=2) + rng.normal(0, 0.08, (2, 3, 4))
    x = rng.uniform(-1, 1, size=(50, 3))
    h = rng.uniform(0, 1, 50) ** 3
    r1 = O.density_loss(G, x, h)
    r2 = O.density_loss(np.concatenate([G, G]), x, h)
    np.testing.assert_allclose(r2["loss"], r1["loss"], rtol=1e-12)
    np.testing.assert_allclose(r2["dG"][:2], 0.5 * r1["dG"], rtol=1e-10, atol=1e-15)
    np.testing.assert_allclose(r2["dG"][2:], 0.5 * r1["dG"], rtol=1e-10, atol=1e-15)


def test_single_pass_gradient_equals_bruteforce_double_sum():
    rng = np.random.default_rng(23)
    G = _scaled_identity(1.0, M=3) + rng.normal(0, 0.15, (3, 3, 4))
    x = rng.uniform(-1, 1, size=(7, 3))
    h = rng.uniform(0, 1, 7) ** 2
    r = O.density_loss(G, x, h, eps=1e-6)
    bf = O.density_grad_bruteforce(G, x, h, eps=1e-6)
    np.testing.assert_allclose(r["dG"], bf, rtol=1e-11, atol=1e-14)


def test_gradient_matches_torch_autograd_with_detached_target():
    rng = np.random.default_rng(24)
    M, N, eps = 3, 40, 1e-9
    G = _scaled_identity(1.0, M=M) + rng.normal(0, 0.1, (M, 3, 4))
    x = rng.uniform(-1, 1, size=(N, 3))
    h = rng.uniform(0, 1, N) ** 2
    r = O.density_loss(G, x, h, eps=eps)
    Gt = torch.tensor(G, requires_grad=True)
    xt, ht = torch.tensor(x), torch.tensor(h)
    l = torch.einsum("mrk,nk->nmr", Gt[:, :, :3], xt) + Gt[None, :, :, 3]
    rho = (torch.linalg.det(Gt[:, :, :3])[None] * torch.exp(-(l ** 20).sum(-1))).sum(-1)
    rs = rho / rho.sum()
    target = torch.exp(ht.mean() / (ht + eps) * torch.log(rs + eps)).detach()
    safe = torch.where(target > 0, target, torch.ones_like(target))
    L = torch.where(target > 0, target * (torch.log(safe) - torch.log(rs + eps)),
                    torch.zeros_like(target)).mean()
    L.backward()
    np.testing.assert_allclose(r["loss"], L.item(), rtol=1e-12)
    np.testing.assert_allclose(r["dG"], Gt.grad.numpy(), rtol=1e-9, atol=1e-14)


def test_gradient_matches_central_differences_with_fixed_target():
    rng = np.random.default_rng(25)
    M, N, eps = 2, 30, 1e-9
    G = _scaled_identity(1.0, M=M) + rng.normal(0, 0.1, (M, 3, 4))
    x = rng.uniform(-1, 1, size=(N, 3))
    h = rng.uniform(0, 1, N) ** 2
    r = O.density_loss(G, x, h, eps=eps)
    target = r["rho_star"]

    def L_fixed(Gp):
        rho, _, _, _ = O.density_terms(Gp, x)
        rs = rho / rho.sum()
        safe = np.where(target > 0, target, 1.0)
        return np.mean(np.where(target > 0, target * (np.log(safe) - np.log(rs + eps)), 0.0))

    hs = 1e-6
    for idx in np.ndindex(M, 3, 4):
        Gp, Gm = G.copy(), G.copy()
        Gp[idx] += hs
        Gm[idx] -= hs
        fd = (L_fixed(Gp) - L_fixed(Gm)) / (2 * hs)
        assert abs(fd - r["dG"][idx]) <= 1e-6 * (abs(r["dG"][idx]) + 1e-6 * np.abs(r["dG"]).max())


def test_empty_batch_and_nan_points():
    G = _scaled_identity(1.0, M=2)
    r = O.density_loss(G, np.zeros((0, 3)), np.zeros(0))
    assert r["loss"] == 0.0 and np.all(r["dG"] == 0)
    x = np.array([[0.1, 0.2, 0.3], [np.nan, 0, 0], [0.5, -0.5, 0.0]])
    rho, phi, _, _ = O.density_terms(G, x)
    assert rho[1] == 0.0 and np.all(phi[1] == 0)
    r = O.density_loss(G, x, np.array([0.1, 0.2, 0.3]))
    assert np.isfinite(r["loss"]) and np.all(np.isfinite(r["dG"]))


def test_all_points_outside_every_grid_is_zero():
    G = _scaled_identity(10.0, M=1)           # the grid covers only |x| < 0.1
    x = np.array([[0.9, 0.9, 0.9], [-0.8, 0.7, 0.95]])
    r = O.density_loss(G, x, np.array([0.1, 0.2]))
    assert r["loss"] == 0.0 and np.all(r["dG"] == 0)


# ---------------------------------------------------------------- alternative readings
# |det| in Eq. (7) (abs_det) and a target renormalised over the batch in Eq. (9)
# (norm_target); the literal reading stays the default of every function.

def _reflect_x(G):
    """The same grid placement with its local x axis reversed: l' = diag(-1,1,1) l."""
    Gr = G.copy()
    Gr[:, 0, :] = -Gr[:, 0, :]
    return Gr


def test_abs_det_reflected_grid_has_the_same_density():
    rng = np.random.default_rng(40)
    G = _scaled_identity(1.2, M=3) + rng.normal(0, 0.1, (3, 3, 4))
    x = rng.uniform(-1, 1, size=(100, 3))
    Gr = _reflect_x(G)
    rho_a, _, _, det_a = O.density_terms(G, x, abs_det=True)
    rho_r, _, _, det_r = O.density_terms(Gr, x, abs_det=True)
    np.testing.assert_allclose(rho_r, rho_a, rtol=1e-14)
    assert np.all(det_a > 0) and np.all(det_r > 0)
    # the literal (signed) reading negates the reflected grid's density
    rho_s, _, _, _ = O.density_terms(Gr, x)
    np.testing.assert_allclose(rho_s, -rho_a, rtol=1e-14)
    # and the losses agree under |det| (h independent of the placement's handedness)
    h = rng.uniform(0, 1, 100) ** 2
    la = O.density_loss(G, x, h, abs_det=True)["loss"]
    lr_ = O.density_loss(Gr, x, h, abs_det=True)["loss"]
    np.testing.assert_allclose(lr_, la, rtol=1e-12)


def test_abs_det_matches_signed_reading_for_positive_determinants():
    rng = np.random.default_rng(41)
    G = _scaled_identity(1.0, M=2) + rng.normal(0, 0.05, (2, 3, 4))
    assert np.all(np.linalg.det(G[:, :, :3]) > 0)
    x = rng.uniform(-1, 1, size=(60, 3))
    h = rng.uniform(0, 1, 60) ** 2
    r0 = O.density_loss(G, x, h)
    r1 = O.density_loss(G, x, h, abs_det=True)
    np.testing.assert_allclose(r1["loss"], r0["loss"], rtol=1e-14)
    np.testing.assert_allclose(r1["dG"], r0["dG"], rtol=1e-13, atol=1e-16)


def test_alternative_readings_uniform_error_gives_zero_loss_and_gradient():
    rng = np.random.default_rng(42)
    G = _scaled_identity(1.0, M=3) + rng.normal(0, 0.1, (3, 3, 4))
    G = _reflect_x(G)                                       # negative determinants
    x = rng.uniform(-1, 1, size=(64, 3))
    h = np.full(64, 0.37)
    for abs_det, norm in ((True, False), (False, True), (True, True)):
        r = O.density_loss(G, x, h, eps=0.0, abs_det=abs_det, norm_target=norm)
        assert abs(r["loss"]) < 1e-15, (abs_det, norm)
        assert np.max(np.abs(r["dG"])) < 1e-13, (abs_det, norm)


def test_normalised_target_loss_is_a_divergence():
    # with eps = 0 both arguments sum to one over the batch: Gibbs' inequality gives L >= 0,
    # and L equals the batch KL written out directly
    rng = np.random.default_rng(43)
    G = _scaled_identity(1.0, M=4) + rng.normal(0, 0.1, (4, 3, 4))
    x = rng.uniform(-1, 1, size=(80, 3))
    for trial in range(5):
        h = rng.uniform(0, 1, 80) ** (1 + trial)
        r = O.density_loss(G, x, h, eps=0.0, norm_target=True)
        tn = r["target"]
        np.testing.assert_allclose(tn.sum(), 1.0, rtol=1e-14)
        pos = tn > 0.0                                       # 0 log 0 = 0
        kl = np.sum(tn[pos] * np.log(tn[pos] / r["rho_s"][pos])) / 80
        np.testing.assert_allclose(r["loss"], kl, rtol=1e-12)
        assert r["loss"] >= 0.0


def test_alternative_readings_single_pass_gradient_equals_bruteforce():
    rng = np.random.default_rng(44)
    G = _scaled_identity(1.0, M=3) + rng.normal(0, 0.15, (3, 3, 4))
    G[1] = _reflect_x(G[1:2])[0]                             # one grid with det < 0
    x = rng.uniform(-1, 1, size=(7, 3))
    h = rng.uniform(0, 1, 7) ** 2
    for abs_det, norm in ((True, False), (False, True), (True, True)):
        r = O.density_loss(G, x, h, eps=1e-6, abs_det=abs_det, norm_target=norm)
        bf = O.density_grad_bruteforce(G, x, h, eps=1e-6, abs_det=abs_det, norm_target=norm)
        np.testing.assert_allclose(r["dG"], bf, rtol=1e-11, atol=1e-14)


def test_alternative_readings_match_torch_autograd_with_detached_target():
    rng = np.random.default_rng(45)
    M, N, eps = 3, 40, 1e-9
    G = _scaled_identity(1.0, M=M) + rng.normal(0, 0.1, (M, 3, 4))
    G[0] = _reflect_x(G[0:1])[0]
    x = rng.uniform(-1, 1, size=(N, 3))
    h = rng.uniform(0, 1, N) ** 2
    for abs_det, norm in ((True, False), (False, True), (True, True)):
        r = O.density_loss(G, x, h, eps=eps, abs_det=abs_det, norm_target=norm)
        Gt = torch.tensor(G, requires_grad=True)
        xt, ht = torch.tensor(x), torch.tensor(h)
        l = torch.einsum("mrk,nk->nmr", Gt[:, :, :3], xt) + Gt[None, :, :, 3]
        det = torch.linalg.det(Gt[:, :, :3])
        det = det.abs() if abs_det else det
        rho = (det[None] * torch.exp(-(l ** 20).sum(-1))).sum(-1)
        rs = rho / rho.sum()
        target = torch.exp(ht.mean() / (ht + eps) * torch.log(rs + eps)).detach()
        if norm:
            target = target / target.sum()
        safe = torch.where(target > 0, target, torch.ones_like(target))
        L = torch.where(target > 0, target * (torch.log(safe) - torch.log(rs + eps)),
                        torch.zeros_like(target)).mean()
        L.backward()
        np.testing.assert_allclose(r["loss"], L.item(), rtol=1e-12)
        np.testing.assert_allclose(r["dG"], Gt.grad.numpy(), rtol=1e-9, atol=1e-14)
