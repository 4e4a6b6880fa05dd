"""FP64 CPU oracle for the two encoder variants the paper names as future work
(Sec. 9, "Conclusion and future work"): (1) a hash-grid encoding queried inside each
adaptive grid instead of trilinear interpolation of a dense grid, and (2) feature grids
extended by a time axis (4-D grids, interpolated in time as well).

TEST INFRASTRUCTURE ONLY, like apmg_oracle: only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; it shares no code with the GPU library.

The paper gives no formulas for either variant.  The readings (collected with the other
readings in the design notes):

Hash grid inside grid i (extension (1); the hash grid is that of Mueller et al., "Instant
neural graphics primitives with a multiresolution hash encoding", 2022):
  * the point's local coordinate l = A_i x + t_i is that of Eq. (1), and the Eq. (2) mask
    applies unchanged: a point outside [-1, 1]^3 gets zero features from grid i;
  * grid i holds L levels; level k has N_k cells per axis across the local cube (the
    caller gives N_k), vertices 0..N_k, vertex coordinate u = (l + 1) N_k / 2, lower
    vertex floor(u) clamped to [0, N_k - 1] -- the dense grid's convention with R - 1 = N_k;
  * each level owns a table of T entries (T a power of two) of C features; vertex v of
    level k reads entry v_x + (N_k + 1)(v_y + (N_k + 1) v_z) when (N_k + 1)^3 <= T (one
    entry per vertex), else the spatial hash (v_x * 1 XOR v_y * 2654435761 XOR
    v_z * 805459861) mod 2^32, then mod T;
  * the level's C features are the trilinear interpolation of its 8 corner entries; grid i
    emits L * C features, index (i L + k) C + c, concatenated over the grids as in Eq. (3).
  Tables are [M, L, T, C].

4-D grid i (extension (2)):
  * the transform stays spatial (Eq. (1)); every point carries a normalised time
    tau in [-1, 1], the same for all grids;
  * grid i is [C, Rt, R, R, R]: Rt time vertices at -1 + 2k/(Rt - 1); the point is inside
    when the Eq. (2) test holds and -1 <= tau <= 1; the time vertex coordinate is
    u_t = (tau + 1)(Rt - 1)/2, lower vertex clamped to [0, Rt - 2];
  * the features are the linear interpolation in time of the trilinear interpolations of
    the two time slices (quadrilinear interpolation of 16 corners); grid i emits C
    features as in Eq. (3).
  Grids are [M, C, Rt, R, R, R].

The integer decisions (mask, cells) are taken in float32 with the fma conventions of
apmg_oracle (u = fma(l, h, h), h = N/2); the values that follow are float64.
"""
from __future__ import annotations

import numpy as np

from . import apmg_oracle as O

# Mueller et al. 2022, Sec. 3: the primes of the spatial hash (pi_1 = 1 keeps x coherent).
HASH_PRIMES = (1, 2654435761, 805459861)


# --------------------------------------------------------------------------
# Hash grid inside each adaptive grid (Sec. 9, extension (1))
# --------------------------------------------------------------------------

def hash_index(v, T):
    """Entry of integer vertices v [..., 3] (x, y, z) in a table of T = 2^k entries: the XOR
    of the coordinates times the primes, in uint32 arithmetic (wrapping mod 2^32), mod T."""
    v = np.asarray(v).astype(np.uint64)
    h = np.zeros(v.shape[:-1], np.uint64)
    for d, p in enumerate(HASH_PRIMES):
        h ^= (v[..., d] * np.uint64(p)) & np.uint64(0xFFFFFFFF)
    return (h & np.uint64(T - 1)).astype(np.int64)


def level_entries(vtx, Nk, T):
    """Entries of the vertices vtx [..., 3] of a level with Nk cells per axis: one entry per
    vertex when the level's (Nk + 1)^3 vertices fit the table, else the spatial hash."""
    n1 = Nk + 1
    if n1 ** 3 <= T:
        return vtx[..., 0] + n1 * (vtx[..., 1] + n1 * vtx[..., 2])
    return hash_index(vtx, T)


def hash_encode(G, Theta, res, x):
    """Features of every (grid, level): y [N, M*L*C] and the pieces the adjoint needs.

    G: [M, 3, 4] or [M, 4, 4]; Theta: [M, L, T, C]; res: the L per-level cell counts N_k;
    x: [N, 3].  Returns dict y, l [N, M, 3], inside [N, M], and per level k the lists
    i0[k] [N, M, 3] (lower vertex), w[k] [N, M, 3] (offsets), ent[k] [N, M, 8] (entries of
    the 8 corners, corner q = a + 2b + 4c).
    """
    Theta = np.asarray(Theta, np.float64)
    M, L, T, C = Theta.shape
    x = np.asarray(x, np.float64)
    N = x.shape[0]
    l = O.local_coords(G, x)
    l32 = O.local_coords_f32(G, x)
    y = np.zeros((N, M, L, C))
    inside = None
    i0s, ws, ents = [], [], []
    gidx = np.arange(M)[None, :]
    for k in range(L):
        Nk = int(res[k])
        ins, cell = O.cell_decision_f32(l32, Nk + 1)
        inside = ins if inside is None else inside
        i0 = np.where(cell >= 0, cell, 0)
        with np.errstate(invalid="ignore"):
            u = (l + 1.0) * (Nk * 0.5)
            w = np.where(ins[..., None], u - i0, 0.0)
        cw = O._corner_weights(w)
        ent = np.zeros((N, M, 8), np.int64)
        for q in range(8):
            off = np.array([q & 1, (q >> 1) & 1, (q >> 2) & 1])
            ent[..., q] = level_entries(i0 + off, Nk, T)
            y[:, :, k, :] += cw[..., q, None] * Theta[gidx, k, ent[..., q], :]
        y[:, :, k, :] = np.where(ins[..., None], y[:, :, k, :], 0.0)
        i0s.append(i0)
        ws.append(w)
        ents.append(ent)
    return {"y": y.reshape(N, M * L * C), "l": l, "inside": inside, "i0": i0s, "w": ws, "ent": ents}


def hash_forward(model, x):
    """f(x) = d(e(x)) with the hash encoder: model has G, Theta [M, L, T, C], res, W, vmin, vmax."""
    enc = hash_encode(model["G"], model["Theta"], model["res"], x)
    m, z, a = O.mlp_forward(model["W"], enc["y"])
    vmin, vmax = float(model["vmin"]), float(model["vmax"])
    return m * (vmax - vmin) + vmin, {"enc": enc, "z": z, "a": a, "x": np.asarray(x, np.float64)}


def _mlp_adjoint(model, cache, df):
    """dW and dL/dy of sum df f (the chain rule of the bias-free ReLU MLP, ReLU'(0) = 0)."""
    W = [np.asarray(w, np.float64) for w in model["W"]]
    z, a = cache["z"], cache["a"]
    scale = float(model["vmax"]) - float(model["vmin"])
    delta = (np.asarray(df, np.float64) * scale)[:, None]
    dW = [None] * len(W)
    for k in range(len(W) - 1, -1, -1):
        dW[k] = delta.T @ a[k]
        if k > 0:
            delta = (delta @ W[k]) * (z[k - 1] > 0.0)
    return dW, delta @ W[0]


def _trilinear_du(vals, w, dy):
    """d/du of sum_c dy_c trilerp_c for corner values vals [..., 8, C], offsets w [..., 3]."""
    du = np.zeros(w.shape)
    for q in range(8):
        a_, b_, c_ = q & 1, (q >> 1) & 1, (q >> 2) & 1
        g = np.sum(vals[..., q, :] * dy, axis=-1)
        wx = w[..., 0] if a_ else 1.0 - w[..., 0]
        wy = w[..., 1] if b_ else 1.0 - w[..., 1]
        wz = w[..., 2] if c_ else 1.0 - w[..., 2]
        sx, sy, sz = (1.0 if a_ else -1.0), (1.0 if b_ else -1.0), (1.0 if c_ else -1.0)
        du[..., 0] += g * sx * wy * wz
        du[..., 1] += g * wx * sy * wz
        du[..., 2] += g * wx * wy * sz
    return du


def _transform_grad(dl, x, M):
    """dL/dG [M, 3, 4] from dL/dl [N, M, 3] (Eq. (1): dl/dA = x^T, dl/dt = 1)."""
    dG = np.zeros((M, 3, 4))
    xs = np.where(np.isfinite(x), x, 0.0)
    dG[:, :, :3] = np.einsum("nmr,nk->mrk", dl, xs)
    dG[:, :, 3] = dl.sum(axis=0)
    return dG


def hash_backward(model, x, df, cache=None):
    """Gradients of sum_n df[n] f(x_n) for the hash encoder: dTheta [M, L, T, C] (colliding
    vertices add into their shared entry), dG [M, 3, 4] through every level's trilinear
    weights (du/dl = N_k / 2), dW.  Outside points give zero gradients."""
    if cache is None:
        _, cache = hash_forward(model, x)
    Theta = np.asarray(model["Theta"], np.float64)
    M, L, T, C = Theta.shape
    enc = cache["enc"]
    N = cache["x"].shape[0]
    dW, dy = _mlp_adjoint(model, cache, df)
    dy = dy.reshape(N, M, L, C)
    ins = enc["inside"]
    dy = np.where(ins[..., None, None], dy, 0.0)
    dTheta = np.zeros_like(Theta)
    dl = np.zeros((N, M, 3))
    gidx = np.broadcast_to(np.arange(M)[None, :], (N, M))
    for k in range(L):
        w, ent = enc["w"][k], enc["ent"][k]
        cw = O._corner_weights(w)
        vals = np.zeros((N, M, 8, C))
        for q in range(8):
            for c in range(C):
                np.add.at(dTheta, (gidx, k, ent[..., q], c), cw[..., q] * dy[:, :, k, c])
            vals[:, :, q, :] = Theta[gidx, k, ent[..., q], :]
        dl += _trilinear_du(vals, w, dy[:, :, k, :]) * (float(model["res"][k]) * 0.5)
    dl = np.where(ins[..., None], dl, 0.0)
    return {"dTheta": dTheta, "dG": _transform_grad(dl, cache["x"], M), "dW": dW,
            "dy": dy.reshape(N, M * L * C)}


# --------------------------------------------------------------------------
# 4-D (time) grids (Sec. 9, extension (2))
# --------------------------------------------------------------------------

def time_decision_f32(tau, Rt):
    """Time mask and lower time vertex in float32: inside = -1 <= tau <= 1 (NaN outside),
    u_t = fma(tau, h, h) with h = (Rt - 1)/2, lower vertex clamp(floor(u_t), 0, Rt - 2)."""
    t32 = np.asarray(tau, np.float32)
    h = np.float32((Rt - 1) * 0.5)
    inside = (t32 >= -1.0) & (t32 <= 1.0)
    with np.errstate(invalid="ignore"):
        u = O._fmaf(t32, h, h)
        u = np.where(np.isfinite(u), u, 0.0)
    return inside, np.clip(np.floor(u), 0, Rt - 2).astype(np.int64)


def time_encode(G, F4, x, tau):
    """Features of the 4-D grids: y [N, M*C] and the adjoint's pieces.

    F4: [M, C, Rt, R, R, R]; x: [N, 3]; tau: [N].  Returns dict y, l, inside [N, M] (space
    and time), i0 [N, M, 3], w [N, M, 3], t0 [N], wt [N].
    """
    F4 = np.asarray(F4, np.float64)
    M, C, Rt, R = F4.shape[0], F4.shape[1], F4.shape[2], F4.shape[3]
    x = np.asarray(x, np.float64)
    tau = np.asarray(tau, np.float64)
    N = x.shape[0]
    l = O.local_coords(G, x)
    ins_s, cell = O.cell_decision_f32(O.local_coords_f32(G, x), R)
    ins_t, t0 = time_decision_f32(tau, Rt)
    inside = ins_s & ins_t[:, None]
    i0 = np.where(cell >= 0, cell, 0)
    with np.errstate(invalid="ignore"):
        u = (l + 1.0) * ((R - 1) * 0.5)
        w = np.where(inside[..., None], u - i0, 0.0)
        wt = np.where(ins_t, (tau + 1.0) * ((Rt - 1) * 0.5) - t0, 0.0)
    cw = O._corner_weights(w)
    gidx = np.arange(M)[None, :]
    y = np.zeros((N, M, C))
    for s_, wts in ((0, 1.0 - wt), (1, wt)):
        ts = (t0 + s_)[:, None]
        for q in range(8):
            a, b, c = q & 1, (q >> 1) & 1, (q >> 2) & 1
            vals = F4[gidx, :, ts, i0[..., 2] + c, i0[..., 1] + b, i0[..., 0] + a]
            y += (wts[:, None] * cw[..., q])[..., None] * vals
    y = np.where(inside[..., None], y, 0.0)
    return {"y": y.reshape(N, M * C), "l": l, "inside": inside, "i0": i0, "w": w, "t0": t0, "wt": wt}


def time_forward(model, x, tau):
    """f(x, tau) = d(e(x, tau)) with 4-D grids: model has G, F4 [M, C, Rt, R, R, R], W, vmin, vmax."""
    enc = time_encode(model["G"], model["F4"], x, tau)
    m, z, a = O.mlp_forward(model["W"], enc["y"])
    vmin, vmax = float(model["vmin"]), float(model["vmax"])
    return m * (vmax - vmin) + vmin, {"enc": enc, "z": z, "a": a, "x": np.asarray(x, np.float64)}


def time_backward(model, x, tau, df, cache=None):
    """Gradients of sum_n df[n] f(x_n, tau_n) for 4-D grids: dF4 [M, C, Rt, R, R, R],
    dG [M, 3, 4] (spatial weights; the time weight scales them), dW."""
    if cache is None:
        _, cache = time_forward(model, x, tau)
    F4 = np.asarray(model["F4"], np.float64)
    M, C, Rt, R = F4.shape[0], F4.shape[1], F4.shape[2], F4.shape[3]
    enc = cache["enc"]
    N = cache["x"].shape[0]
    dW, dy = _mlp_adjoint(model, cache, df)
    dy = np.where(enc["inside"][..., None], dy.reshape(N, M, C), 0.0)
    i0, w, t0, wt = enc["i0"], enc["w"], enc["t0"], enc["wt"]
    cw = O._corner_weights(w)
    gidx = np.broadcast_to(np.arange(M)[None, :], (N, M))
    dF4 = np.zeros_like(F4)
    dl = np.zeros((N, M, 3))
    for s_, wts in ((0, 1.0 - wt), (1, wt)):
        ts = np.broadcast_to((t0 + s_)[:, None], (N, M))
        vals = np.zeros((N, M, 8, C))
        for q in range(8):
            a, b, c = q & 1, (q >> 1) & 1, (q >> 2) & 1
            zi, yi, xi = i0[..., 2] + c, i0[..., 1] + b, i0[..., 0] + a
            for ch in range(C):
                np.add.at(dF4, (gidx, ch, ts, zi, yi, xi), wts[:, None] * cw[..., q] * dy[..., ch])
            vals[:, :, q, :] = F4[gidx, :, ts, zi, yi, xi]
        dl += wts[:, None, None] * _trilinear_du(vals, w, dy)
    dl = np.where(enc["inside"][..., None], dl * ((R - 1) * 0.5), 0.0)
    return {"dF4": dF4, "dG": _transform_grad(dl, cache["x"], M), "dW": dW, "dy": dy.reshape(N, M * C)}
