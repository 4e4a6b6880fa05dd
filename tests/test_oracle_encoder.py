"""Pins for the oracle's encoder (Sec. 4.1.1, Eqs. (1)-(3)) and its float32
decision arithmetic.  Each check is fixed by the paper or by mathematics, not
by re-typing the oracle's formula."""
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import apmg_oracle as O


def _round_f32_exact(q: Fraction) -> np.float32:
    """Correct round-to-nearest-even of an exact rational to float32."""
    r = np.float32(float(q))
    best = None
    for cand in (np.nextafter(r, np.float32(-np.inf)), r, np.nextafter(r, np.float32(np.inf))):
        d = abs(Fraction(float(cand)) - q)
        if best is None or d < best[0] or (d == best[0] and (np.float32(cand).view(np.uint32) & 1) == 0):
            best = (d, cand)
    return np.float32(best[1])


def test_fmaf_matches_exact_rational_rounding():
    rng = np.random.default_rng(0)
    a = rng.normal(size=4000).astype(np.float32)
    b = rng.normal(size=4000).astype(np.float32)
    c = rng.normal(size=4000).astype(np.float32)
    got = O._fmaf(a, b, c)
    for i in range(4000):
        q = Fraction(float(a[i])) * Fraction(float(b[i])) + Fraction(float(c[i]))
        assert got[i] == _round_f32_exact(q)


def test_fmaf_double_rounding_case():
    # a*b = 2^-24 - 2^-70 and c = 1 + 2^-23: the float64 sum lands on a float32
    # midpoint; the exact value is just below it, so the result rounds down.
    a = np.float32(1 + 2.0 ** -23)
    b = np.float32(2.0 ** -24 * (1 - 2.0 ** -23))
    c = np.float32(1 + 2.0 ** -23)
    q = Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c))
    naive = np.float32(float(a) * float(b) + float(c))
    assert naive != _round_f32_exact(q)            # the trap exists
    assert O._fmaf(a, b, c) == _round_f32_exact(q) == np.float32(1 + 2.0 ** -23)


def _identity_G(M):
    G = np.zeros((M, 3, 4))
    G[:, 0, 0] = G[:, 1, 1] = G[:, 2, 2] = 1.0
    return G


def test_vertices_reproduce_grid_values():
    rng = np.random.default_rng(1)
    M, C, R = 2, 3, 5
    F = rng.normal(size=(M, C, R, R, R))
    G = _identity_G(M)
    idx = rng.integers(0, R, size=(50, 3))          # (ix, iy, iz)
    x = -1.0 + 2.0 * idx / (R - 1)
    y = O.encode(G, F, x)["y"].reshape(50, M, C)
    for n in range(50):
        ix, iy, iz = idx[n]
        np.testing.assert_allclose(y[n], F[:, :, iz, iy, ix], rtol=0, atol=1e-14)


def test_affine_field_reproduced_exactly():
    # Trilinear interpolation reproduces any affine function of position.
    rng = np.random.default_rng(2)
    M, C, R = 3, 2, 7
    coef = rng.normal(size=(M, C, 4))
    pos = -1.0 + 2.0 * np.arange(R) / (R - 1)
    Z, Y, X = np.meshgrid(pos, pos, pos, indexing="ij")
    F = (coef[..., 0, None, None, None] * X + coef[..., 1, None, None, None] * Y
         + coef[..., 2, None, None, None] * Z + coef[..., 3, None, None, None])
    G = _identity_G(M) * 0.9
    G[:, :, 3] = rng.uniform(-0.05, 0.05, size=(M, 3))
    x = rng.uniform(-1, 1, size=(300, 3))
    enc = O.encode(G, F, x)
    l = enc["l"]
    want = (coef[None, :, :, 0] * l[:, :, None, 0] + coef[None, :, :, 1] * l[:, :, None, 1]
            + coef[None, :, :, 2] * l[:, :, None, 2] + coef[None, :, :, 3])
    want = np.where(enc["inside"][..., None], want, 0.0)
    np.testing.assert_allclose(enc["y"].reshape(300, M, C), want, rtol=0, atol=1e-13)


def test_identity_transform_equals_grid_sample():
    # torch grid_sample(align_corners=True) pins vertex alignment and the axis
    # order x->W, y->H, z->D of the [M, C, D, H, W] grid tensor.
    rng = np.random.default_rng(3)
    M, C, R = 3, 2, 9
    F = rng.normal(size=(M, C, R, R, R))
    G = _identity_G(M)
    x = rng.uniform(-1 + 2.0 / (R - 1), 1 - 2.0 / (R - 1), size=(400, 3))
    y = O.encode(G, F, x)["y"].reshape(400, M, C)
    inp = torch.from_numpy(F)                                  # [M, C, D, H, W]
    grid = torch.from_numpy(x)[None, None, None].expand(M, 1, 1, 400, 3).contiguous()
    ref = torch.nn.functional.grid_sample(inp, grid, mode="bilinear", align_corners=True)
    ref = ref[:, :, 0, 0, :].permute(2, 0, 1).numpy()          # [N, M, C]
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12)


def test_outside_is_exactly_zero_and_faces_inclusive():
    rng = np.random.default_rng(4)
    M, C, R = 1, 2, 4
    F = rng.normal(size=(M, C, R, R, R)) + 3.0
    G = _identity_G(M)
    x = np.array([[1.0, 0.0, 0.0], [-1.0, 1.0, -1.0], [1.0 + 2 ** -20, 0, 0],
                  [0, -1.0 - 2 ** -20, 0], [np.nan, 0, 0], [0.3, 0.2, np.inf]])
    enc = O.encode(G, F, x)
    assert enc["inside"][:, 0].tolist() == [True, True, False, False, False, False]
    assert np.all(enc["y"][2:] == 0.0)
    # l = 1 is the last vertex, reached from the last cell with weight 1
    # (u = 3, 1.5, 1.5): the average of the 4 vertices x = 3, y, z in {1, 2}
    want = F[0, :, 1:3, 1:3, 3].mean(axis=(1, 2))
    np.testing.assert_allclose(enc["y"][0], want, rtol=0, atol=1e-14)
    assert enc["cell"][0, 0].tolist() == [R - 2, 1, 1]
    assert np.all(enc["cell"][2:] == -1)


def test_cell_tie_breaks():
    # An integer vertex coordinate picks the upper cell with weight 0, except
    # the last vertex, which stays in the last cell.
    R = 5
    l = np.array([[[-1.0, -0.5, 0.0]], [[0.5, 1.0, -1.0]]], np.float32)
    inside, cell = O.cell_decision_f32(l, R)
    assert inside.all()
    assert cell[0, 0].tolist() == [0, 1, 2]
    assert cell[1, 0].tolist() == [3, 3, 0]


def test_translation_equivariance():
    # Shifting the transform's translation by k cells equals rolling F by k.
    rng = np.random.default_rng(5)
    M, C, R, k = 1, 2, 9, 2
    F = rng.normal(size=(M, C, R, R, R))
    G = _identity_G(M)
    G2 = G.copy()
    G2[0, 0, 3] = 2.0 * k / (R - 1)
    x = rng.uniform(-0.4, 0.4, size=(200, 3))
    y2 = O.encode(G2, F, x)["y"]
    Fr = np.roll(F, -k, axis=4)
    y1 = O.encode(G, Fr, x)["y"]
    np.testing.assert_allclose(y2, y1, rtol=0, atol=1e-12)


def test_grid_permutation_with_W1_columns_leaves_f_unchanged():
    # Pins the concatenation order y[i*C + c] of Eq. (3).
    rng = np.random.default_rng(6)
    M, C, R = 4, 2, 6
    F = rng.normal(size=(M, C, R, R, R))
    G = _identity_G(M) * rng.uniform(0.8, 1.2, size=(M, 1, 1))
    G[:, :, 3] = rng.normal(0, 0.1, size=(M, 3))
    W = [rng.normal(size=(8, M * C)), rng.normal(size=(8, 8)), rng.normal(size=(1, 8))]
    model = {"G": G, "F": F, "W": W, "vmin": -3.5, "vmax": 12.25}
    x = rng.uniform(-1, 1, size=(100, 3))
    f, _ = O.forward(model, x)
    perm = rng.permutation(M)
    cols = np.concatenate([np.arange(C) + C * p for p in perm])
    model2 = {"G": G[perm], "F": F[perm], "W": [W[0][:, cols], W[1], W[2]],
              "vmin": -3.5, "vmax": 12.25}
    f2, _ = O.forward(model2, x)
    np.testing.assert_allclose(f, f2, rtol=1e-13, atol=1e-13)


def test_decisions_match_float64_away_from_boundaries():
    # The float32 decisions equal the exact (float64) ones except within a
    # rounding band around cell faces and the cube faces.
    rng = np.random.default_rng(7)
    M, R = 8, 32
    G = _identity_G(M) * rng.uniform(0.9, 1.3, size=(M, 1, 1))
    G += rng.normal(0, 0.05, size=G.shape)
    G = G.astype(np.float32)
    x = (rng.integers(0, 1 << 24, size=(5000, 3)) * 2.0 ** -23 - 1.0).astype(np.float32)
    l64 = O.local_coords(G, x)
    u64 = (l64 + 1.0) * (R - 1) / 2
    inside, cell = O.cell_decision_f32(O.local_coords_f32(G, x), R)
    far = (np.abs(u64 - np.round(u64)) > 1e-4).all(-1) & (np.abs(np.abs(l64) - 1) > 1e-5).all(-1)
    in64 = np.all(np.abs(l64) <= 1.0, axis=-1)
    assert far.mean() > 0.95
    assert np.array_equal(inside[far], in64[far])
    c64 = np.clip(np.floor(u64), 0, R - 2)
    sel = far & in64
    assert np.array_equal(cell[sel], c64[sel])
