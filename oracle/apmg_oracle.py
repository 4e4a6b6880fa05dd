"""FP64 CPU oracle for the APMGSRN hot path (Wurster et al., "Adaptively Placed
Multi-Grid Scene Representation Networks for Large-Scale Data Visualization").

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP library and imports nothing from it.

Notation follows the paper (Sec. 4.1): M feature grids of C channels at R^3
vertices, F with shape [M, C, R, R, R] (axes D=z, H=y, W=x), transforms
G with shape [M, 3, 4] (rows 0..2 of each 4x4 matrix of Eq. (1); row 3 is
fixed to (0, 0, 0, 1)).  Points are [N, 3] in the global cube [-1, 1]^3.

Arithmetic is numpy float64 throughout, except for the integer decisions
(inside-the-cube mask, interpolation cell, volume cell, brick index).  The
paper's own encoder ran in single precision (Sec. 7, "Training"), so those
decisions are taken in float32 with a fixed operation order, written out in
`_fmaf` below; the values that follow them are float64.

Readings of points the paper leaves open are listed at each function and
collected under "Readings of the paper" in the design notes.
"""
from __future__ import annotations

import numpy as np

# Sec. 4.2, Eq. (7): the flat-top exponent used in the paper.
P_FLATTOP = 10
# Sec. 7 "Training": Adam betas and learning rates.
ADAM_BETAS = (0.9, 0.99)
LR_DEFAULT = 0.01
LR_TRANSFORM = 0.001
# Not given by the paper: Kingma & Ba's default epsilon, no weight decay.
ADAM_EPS = 1e-8
# Eq. (8)/(9): "a small number"; must be far below 1/N because rho_scaled ~ 1/N.
EPS_DENSITY = 1e-12
# Flat-top cut-off: exp(-s) is taken as exactly 0 when s exceeds this (or is NaN).
S_MAX_F64 = 700.0


# --------------------------------------------------------------------------
# float32 decisions
# --------------------------------------------------------------------------

def _fmaf(a, b, c):
    """Correctly rounded float32 fused multiply-add, emulated in float64.

    a, b, c are float32 arrays (broadcastable).  a*b is exact in float64
    (24+24 bits).  s = a*b + c rounded to float64 can only mis-round to float32
    when s lands exactly on a float32 midpoint; the exact residual of the sum
    (Knuth's TwoSum) then decides the direction.
    """
    with np.errstate(invalid="ignore", over="ignore"):
        return _fmaf_impl(a, b, c)


def _fmaf_impl(a, b, c):
    a = np.asarray(a, np.float32).astype(np.float64)
    b = np.asarray(b, np.float32).astype(np.float64)
    c = np.asarray(c, np.float32).astype(np.float64)
    p = a * b
    s = p + c
    bb = s - p
    e = (p - (s - bb)) + (c - bb)             # exact: p + c == s + e
    r = s.astype(np.float32)
    r64 = r.astype(np.float64)
    d = s - r64                               # exact
    up = np.nextafter(r, np.float32(np.inf)).astype(np.float64)
    dn = np.nextafter(r, np.float32(-np.inf)).astype(np.float64)
    half_up = (up - r64) * 0.5
    half_dn = (r64 - dn) * 0.5
    mid = ((d > 0) & (d == half_up)) | ((d < 0) & (-d == half_dn))
    fix = mid & (e != 0) & (np.sign(e) == np.sign(d))
    if np.any(fix):
        other = np.where(d > 0, np.nextafter(r, np.float32(np.inf)),
                         np.nextafter(r, np.float32(-np.inf)))
        r = np.where(fix, other, r)
    return r.astype(np.float32)


def local_coords_f32(G, x):
    """Eq. (1) evaluated in float32 for the integer decisions.

    l_r = fma(G[r,2], x_z, fma(G[r,1], x_y, fma(G[r,0], x_x, G[r,3]))), each
    fma rounded once.  Returns float32 [N, M, 3].
    """
    G32 = np.asarray(G, np.float32)[:, :3, :]
    x32 = np.asarray(x, np.float32)
    acc = np.broadcast_to(G32[None, :, :, 3], (x32.shape[0],) + G32.shape[:2])
    for k in range(3):
        acc = _fmaf(G32[None, :, :, k], x32[:, None, None, k], acc)
    return acc


def cell_decision_f32(l32, R):
    """Eq. (2) mask and the interpolation cell, decided in float32.

    Reading: the test -1 <= l <= 1 is inclusive on every axis, so a NaN
    coordinate counts as outside.  The vertex coordinate is u = (l+1)(R-1)/2
    (vertices corner-aligned at +-1), rounded once: u = fma(l, h, h) with
    h = (R-1)/2.  The lower vertex is floor(u) clamped to [0, R-2], so u = R-1
    (l = 1) uses the last cell with weight 1, and an integer u picks the upper
    cell with weight 0.
    Returns (inside [..] bool, cell [.., 3] int64; -1 where outside).
    """
    h = np.float32((R - 1) * 0.5)
    inside = np.all((l32 >= -1.0) & (l32 <= 1.0), axis=-1)
    with np.errstate(invalid="ignore"):
        u32 = _fmaf(l32, h, h)
        u32 = np.where(np.isfinite(u32), u32, 0.0)
    i0 = np.clip(np.floor(u32), 0, R - 2).astype(np.int64)
    cell = np.where(inside[..., None], i0, -1)
    return inside, cell


# --------------------------------------------------------------------------
# Encoder: Sec. 4.1.1, Eqs. (1)-(3)
# --------------------------------------------------------------------------

def local_coords(G, x):
    """Eq. (1): l_i = G_i[0:3, 0:3] x + G_i[0:3, 3] for every grid, float64.

    G: [M, 3, 4] or [M, 4, 4]; x: [N, 3].  Returns [N, M, 3].
    """
    G = np.asarray(G, np.float64)[:, :3, :]
    x = np.asarray(x, np.float64)
    return np.einsum("mrk,nk->nmr", G[:, :, :3], x) + G[None, :, :, 3]


def _corner_weights(w):
    """The 8 trilinear weights for fractional offsets w [..., 3] (x, y, z).

    Corner index q = a + 2 b + 4 c for offsets (a, b, c) along (x, y, z).
    """
    out = []
    for q in range(8):
        a, b, c = q & 1, (q >> 1) & 1, (q >> 2) & 1
        wx = w[..., 0] if a else 1.0 - w[..., 0]
        wy = w[..., 1] if b else 1.0 - w[..., 1]
        wz = w[..., 2] if c else 1.0 - w[..., 2]
        out.append(wx * wy * wz)
    return np.stack(out, axis=-1)


def encode(G, F, x):
    """Eqs. (1)-(3): the concatenated feature vector y = e_0 + ... + e_{M-1}.

    F: [M, C, R, R, R].  Returns a dict with
      y      [N, M*C]  (index i*C + c, grid-major then channel),
      l      [N, M, 3] float64 local coordinates,
      inside [N, M] bool, cell [N, M, 3] int64 (float32 decisions),
      w      [N, M, 3] fractional offsets inside the cell (float64),
    Outside a grid all C features are exactly 0 (Eq. (2)).
    """
    F = np.asarray(F, np.float64)
    M, C, R = F.shape[0], F.shape[1], F.shape[2]
    x = np.asarray(x, np.float64)
    N = x.shape[0]
    l = local_coords(G, x)
    inside, cell = cell_decision_f32(local_coords_f32(G, x), R)
    i0 = np.where(cell >= 0, cell, 0)
    with np.errstate(invalid="ignore"):
        u = (l + 1.0) * ((R - 1) * 0.5)
        w = np.where(inside[..., None], u - i0, 0.0)
    cw = _corner_weights(w)                                  # [N, M, 8]
    y = np.zeros((N, M, C))
    gidx = np.arange(M)[None, :]
    for q in range(8):
        a, b, c = q & 1, (q >> 1) & 1, (q >> 2) & 1
        vals = F[gidx, :, i0[..., 2] + c, i0[..., 1] + b, i0[..., 0] + a]  # [N, M, C]
        y += cw[..., q, None] * vals
    y = np.where(inside[..., None], y, 0.0)
    return {"y": y.reshape(N, M * C), "l": l, "inside": inside, "cell": cell,
            "w": w, "i0": i0}


# --------------------------------------------------------------------------
# Decoder: Sec. 4.1.2
# --------------------------------------------------------------------------

def mlp_forward(W, y):
    """Bias-free MLP, ReLU after every layer except the last (Sec. 4.1.2).

    W: list of [out, in] matrices.  Returns (m [N], pre-activations z_k,
    activations a_k with a_0 = y).
    """
    a = [np.asarray(y, np.float64)]
    z = []
    for k, Wk in enumerate(W):
        zk = a[-1] @ np.asarray(Wk, np.float64).T
        z.append(zk)
        if k < len(W) - 1:
            a.append(np.maximum(zk, 0.0))
    return z[-1][:, 0], z, a


def forward(model, x):
    """f(x) = d(e(x)) with the output scaling d(y) = m(y)(max - min) + min
    (Sec. 4.1, Sec. 4.1.2 "Scaling").  Returns (f [N], cache)."""
    enc = encode(model["G"], model["F"], x)
    m, z, a = mlp_forward(model["W"], enc["y"])
    vmin, vmax = float(model["vmin"]), float(model["vmax"])
    f = m * (vmax - vmin) + vmin
    return f, {"enc": enc, "z": z, "a": a, "x": np.asarray(x, np.float64)}


# --------------------------------------------------------------------------
# Adjoint of the forward pass (hand-derived chain rule)
# --------------------------------------------------------------------------

def backward(model, x, df, cache=None):
    """Gradients of sum_n df[n] * f(x_n) with respect to F, G and the MLP.

    Readings: ReLU'(0) = 0; the mask's jump contributes nothing (outside
    points give zero dF and zero dG); at a vertex the derivative is the
    one-sided one of the cell chosen by the float32 decision.
    Returns dict dF [M,C,R,R,R], dG [M,3,4], dW list.
    """
    if cache is None:
        _, cache = forward(model, x)
    F = np.asarray(model["F"], np.float64)
    M, C, R = F.shape[0], F.shape[1], F.shape[2]
    W = [np.asarray(w, np.float64) for w in model["W"]]
    enc, z, a = cache["enc"], cache["z"], cache["a"]
    x = cache["x"]
    N = x.shape[0]
    df = np.asarray(df, np.float64)
    scale = float(model["vmax"]) - float(model["vmin"])

    delta = (df * scale)[:, None]                    # dL/dz_last  [N, 1]
    dW = [None] * len(W)
    for k in range(len(W) - 1, -1, -1):
        dW[k] = delta.T @ a[k]
        if k > 0:
            delta = (delta @ W[k]) * (z[k - 1] > 0.0)
    dy = (delta @ W[0]).reshape(N, M, C)
    dy = np.where(enc["inside"][..., None], dy, 0.0)

    i0, w = enc["i0"], enc["w"]
    cw = _corner_weights(w)
    dF = np.zeros_like(F)
    gidx = np.broadcast_to(np.arange(M)[None, :], (N, M))
    du = np.zeros((N, M, 3))
    for q in range(8):
        a_, b_, c_ = q & 1, (q >> 1) & 1, (q >> 2) & 1
        zi, yi, xi = i0[..., 2] + c_, i0[..., 1] + b_, i0[..., 0] + a_
        for c in range(C):
            np.add.at(dF, (gidx, c, zi, yi, xi), cw[..., q] * dy[..., c])
        vals = F[gidx, :, zi, yi, xi]                 # [N, M, C]
        g = np.sum(vals * dy, axis=-1)                # sum_c dy_c F_c(corner)
        wx = w[..., 0] if a_ else 1.0 - w[..., 0]
        wy = w[..., 1] if b_ else 1.0 - w[..., 1]
        wz = w[..., 2] if c_ else 1.0 - w[..., 2]
        sx, sy, sz = (1.0 if a_ else -1.0), (1.0 if b_ else -1.0), (1.0 if c_ else -1.0)
        du[..., 0] += g * sx * wy * wz
        du[..., 1] += g * wx * sy * wz
        du[..., 2] += g * wx * wy * sz
    dl = du * ((R - 1) * 0.5)                         # du/dl = (R-1)/2
    dl = np.where(enc["inside"][..., None], dl, 0.0)
    dG = np.zeros((M, 3, 4))
    xs = np.where(np.isfinite(x), x, 0.0)             # outside points add nothing
    dG[:, :, :3] = np.einsum("nmr,nk->mrk", dl, xs)
    dG[:, :, 3] = dl.sum(axis=0)
    return {"dF": dF, "dG": dG, "dW": dW, "dy": dy.reshape(N, M * C)}


def backward_magnitudes(model, x, df, cache=None, open_units=None):
    """Per gradient entry, the sum of the absolute values of the terms that backward()
    adds up: the same chain rule with every factor replaced by its absolute value.

    These sums set the scale of the float32 rounding error of each entry of a gradient
    that is reduced in float32 (the "noise level" of the rule for comparing Adam's
    first updates).  Two more sums cover the float32 encoder, whose corner weights carry
    an absolute error of a few (R-1) 2^-24 (u = (l + 1)(R-1)/2 is held to float32):
      dF_unit  per vertex, sum |dL/dy| over the points of its cells (weights taken as 1);
      dW_fabs  dW's sums with the features replaced by the interpolation of |F| (an upper
               bound of |y| and the scale of its float32 error).
    open_units: optional list, per hidden layer, of [N, H] boolean masks of units whose
    ReLU derivative is taken as 1 whatever the sign of the pre-activation -- an envelope
    of a point whose ReLU decisions a float32 forward pass may take either way.
    Returns dict dF [M,C,R,R,R], dF_unit, dW list, dW_fabs list.
    """
    if cache is None:
        _, cache = forward(model, x)
    F = np.asarray(model["F"], np.float64)
    M, C = F.shape[0], F.shape[1]
    W = [np.abs(np.asarray(w, np.float64)) for w in model["W"]]
    enc, z, a = cache["enc"], cache["z"], cache["a"]
    xs = cache["x"]
    N = xs.shape[0]
    y_fabs = encode(model["G"], np.abs(F), xs)["y"]
    scale = abs(float(model["vmax"]) - float(model["vmin"]))
    delta = np.abs(np.asarray(df, np.float64) * scale)[:, None]
    dW = [None] * len(W)
    dW_fabs = [None] * len(W)
    for k in range(len(W) - 1, -1, -1):
        dW[k] = delta.T @ np.abs(a[k])
        dW_fabs[k] = delta.T @ (y_fabs if k == 0 else np.abs(a[k]))
        if k > 0:
            on = z[k - 1] > 0.0
            if open_units is not None:
                on = on | open_units[k - 1]
            delta = (delta @ W[k]) * on
    dy = (delta @ W[0]).reshape(N, M, C)
    dy = np.where(enc["inside"][..., None], dy, 0.0)
    i0, cw = enc["i0"], _corner_weights(enc["w"])
    dF = np.zeros_like(F)
    dF_unit = np.zeros_like(F)
    gidx = np.broadcast_to(np.arange(M)[None, :], (N, M))
    for q in range(8):
        a_, b_, c_ = q & 1, (q >> 1) & 1, (q >> 2) & 1
        zi, yi, xi = i0[..., 2] + c_, i0[..., 1] + b_, i0[..., 0] + a_
        for c in range(C):
            np.add.at(dF, (gidx, c, zi, yi, xi), np.abs(cw[..., q]) * dy[..., c])
            np.add.at(dF_unit, (gidx, c, zi, yi, xi), dy[..., c])
    return {"dF": dF, "dF_unit": dF_unit, "dW": dW, "dW_fabs": dW_fabs}


# --------------------------------------------------------------------------
# Feature density and its loss: Sec. 4.2, Eqs. (7)-(9)
# --------------------------------------------------------------------------

def _det3(A):
    return (A[..., 0, 0] * (A[..., 1, 1] * A[..., 2, 2] - A[..., 1, 2] * A[..., 2, 1])
            - A[..., 0, 1] * (A[..., 1, 0] * A[..., 2, 2] - A[..., 1, 2] * A[..., 2, 0])
            + A[..., 0, 2] * (A[..., 1, 0] * A[..., 2, 1] - A[..., 1, 1] * A[..., 2, 0]))


def _cofactor3(A):
    """Cofactor matrix: d det(A) / dA."""
    cof = np.empty_like(A)
    for r in range(3):
        for c in range(3):
            rows = [i for i in range(3) if i != r]
            cols = [j for j in range(3) if j != c]
            minor = (A[..., rows[0], cols[0]] * A[..., rows[1], cols[1]]
                     - A[..., rows[0], cols[1]] * A[..., rows[1], cols[0]])
            cof[..., r, c] = ((-1) ** (r + c)) * minor
    return cof


def density_terms(G, x, p=P_FLATTOP, s_max=S_MAX_F64, abs_det=False):
    """Eq. (7): rho(x) = sum_i det(G_i[0:3,0:3]) exp(-sum_d l_d^{2p}).

    Reading: the determinant is signed, as written; no 1/2 or normaliser
    (Eq. (7) drops those of Eq. (6)); exp(-s) is exactly 0 when s > s_max or
    s is NaN.  With abs_det the alternative reading |det| is used instead: a
    grid's density is the number of its cells per unit of global volume
    (Sec. 4.2), which does not change sign when the grid is reflected.
    Returns (rho [N], phi [N, M], l [N, M, 3], det [M]) where det is the
    factor actually used (signed or absolute).
    """
    G = np.asarray(G, np.float64)
    det = _det3(G[:, :3, :3])
    if abs_det:
        det = np.abs(det)
    l = local_coords(G, x)
    with np.errstate(over="ignore", invalid="ignore"):
        s = np.sum(l ** (2 * p), axis=-1)
        keep = s <= s_max
        phi = np.where(keep, np.exp(-np.where(keep, s, 0.0)), 0.0)
    rho = phi @ det
    return rho, phi, l, det


def density_loss(G, x, h, eps=EPS_DENSITY, p=P_FLATTOP, s_max=S_MAX_F64, abs_det=False,
                 norm_target=False):
    """Eqs. (8)-(9) and the gradient of L_density with respect to G.

    h [N] is the per-point model error h(x).  Readings:
      * rho_scaled = rho / sum_X rho; h_bar = mean(h) over the batch.
      * rho* = exp( h_bar/(h+eps) * log(rho_scaled + eps) )        (Eq. (8))
      * L = (1/N) sum rho* (log rho* - log(rho_scaled + eps)), the same eps
        inside the second log as in Eq. (8), and 0*log 0 := 0.      (Eq. (9))
      * rho* is a target: it is held constant in the gradient.
    Alternative readings behind flags: abs_det takes |det| in Eq. (7) (see
    density_terms); norm_target replaces rho* by rho* / sum_X rho* in Eq. (9),
    so that both arguments of the divergence sum to one over the batch.
    The gradient uses a(x) = dL/drho_scaled(x) = -target/(N (rho_scaled+eps)),
    Q = sum_x a rho_scaled, dL/drho(y) = (a(y) - Q)/S, chained through
      d rho_i/dA = sgn exp(-s_i) cof(A_i) - rho_i 2p (l^{2p-1}) x^T,
      d rho_i/dt = -rho_i 2p l^{2p-1},
    with sgn = 1 (signed det) or sign(det(A_i)) (abs_det).
    Returns dict loss, dG [M,3,4], rho, rho_s, rho_star, S, h_bar.
    """
    G = np.asarray(G, np.float64)
    x = np.asarray(x, np.float64)
    h = np.asarray(h, np.float64)
    N = x.shape[0]
    M = G.shape[0]
    if N == 0:
        return {"loss": 0.0, "dG": np.zeros((M, 3, 4)), "rho": np.zeros(0),
                "rho_s": np.zeros(0), "rho_star": np.zeros(0), "S": 0.0, "h_bar": 0.0}
    rho, phi, l, det = density_terms(G, x, p, s_max, abs_det)
    S = rho.sum()
    if S == 0.0:
        # Reading: no grid has density at any point of the batch; the
        # normalisation of Eq. (8) is undefined and there is nothing to move.
        return {"loss": 0.0, "dG": np.zeros((M, 3, 4)), "rho": rho,
                "rho_s": np.zeros(N), "rho_star": np.zeros(N), "S": 0.0,
                "h_bar": float(h.mean())}
    rho_s = rho / S
    h_bar = h.mean()
    log_target = h_bar / (h + eps) * np.log(rho_s + eps)
    rho_star = np.exp(log_target)
    target = rho_star
    if norm_target:
        Z = rho_star.sum()
        target = rho_star / Z
        log_target = log_target - np.log(Z)
    terms = np.where(target > 0.0, target * (log_target - np.log(rho_s + eps)), 0.0)
    loss = terms.sum() / N

    a = -target / (N * (rho_s + eps))
    Q = np.sum(a * rho_s)
    dLdrho = (a - Q) / S                                     # [N]
    cof = _cofactor3(G[:, :3, :3])                           # [M, 3, 3]
    if abs_det:
        cof = cof * np.sign(_det3(G[:, :3, :3]))[:, None, None]
    rho_i = phi * det[None, :]                               # [N, M]
    with np.errstate(over="ignore", invalid="ignore"):
        q = np.where(phi[..., None] > 0.0, l ** (2 * p - 1), 0.0)   # [N, M, 3]
    coef = dLdrho[:, None] * rho_i * (2 * p)                 # [N, M]
    # a point without density (e.g. a NaN coordinate) contributes nothing
    xs = np.where(np.isfinite(x), x, 0.0)
    dG = np.zeros((M, 3, 4))
    dG[:, :, :3] = (np.einsum("n,nm->m", dLdrho, phi)[:, None, None] * cof
                    - np.einsum("nm,nmr,nk->mrk", coef, q, xs))
    dG[:, :, 3] = -np.einsum("nm,nmr->mr", coef, q)
    return {"loss": loss, "dG": dG, "rho": rho, "rho_s": rho_s, "rho_star": rho_star,
            "target": target, "S": S, "h_bar": h_bar, "Q": Q, "a": a}


def density_grad_bruteforce(G, x, h, eps=EPS_DENSITY, p=P_FLATTOP, abs_det=False, norm_target=False):
    """The literal double sum sum_x sum_y dL/drho_s(x) drho_s(x)/drho(y) drho(y)/dG.

    O(N^2): for tiny N only.  The target held constant, as in density_loss().
    """
    G = np.asarray(G, np.float64)
    x = np.asarray(x, np.float64)
    N, M = x.shape[0], G.shape[0]
    res = density_loss(G, x, h, eps, p, abs_det=abs_det, norm_target=norm_target)
    rho, rho_s, target, S = res["rho"], res["rho_s"], res["target"], res["S"]
    _, phi, l, det = density_terms(G, x, p, abs_det=abs_det)
    cof = _cofactor3(G[:, :3, :3])
    sgn = np.sign(_det3(G[:, :3, :3])) if abs_det else np.ones(M)
    dG = np.zeros((M, 3, 4))
    for xi in range(N):
        dL_drhos = -target[xi] / (N * (rho_s[xi] + eps))
        for yi in range(N):
            drhos_drho = ((1.0 if xi == yi else 0.0) / S) - rho[xi] / S ** 2
            for i in range(M):
                rho_i = det[i] * phi[yi, i]
                g = np.zeros((3, 4))
                for r in range(3):
                    qr = l[yi, i, r] ** (2 * p - 1)
                    for k in range(3):
                        g[r, k] = sgn[i] * phi[yi, i] * cof[i, r, k] - rho_i * 2 * p * qr * x[yi, k]
                    g[r, 3] = -rho_i * 2 * p * qr
                dG[i] += dL_drhos * drhos_drho * g
    return dG


# --------------------------------------------------------------------------
# Reconstruction loss and ground truth: Sec. 4.3.1
# --------------------------------------------------------------------------

def volume_cell_decision_f32(x, shape_zyx):
    """Float32 cell decision for trilinear sampling of a [Z][Y][X] volume.

    u_d = fma(x_d, h_d, h_d) with h_d = (n_d - 1)/2 (voxel k at -1 + 2k/(n-1)),
    lower voxel clamp(floor(u), 0, n-2).  Returns int64 [N, 3] (x, y, z).
    """
    x32 = np.asarray(x, np.float32)
    nz, ny, nx = shape_zyx
    out = np.empty(x32.shape, np.int64)
    for d, n in enumerate((nx, ny, nz)):
        h = np.float32((n - 1) * 0.5)
        with np.errstate(invalid="ignore"):
            u = _fmaf(x32[:, d], h, h)
            u = np.where(np.isfinite(u), u, 0.0)
        out[:, d] = np.clip(np.floor(u), 0, n - 2)
    return out


def gt_sample(volume, x):
    """v(x): trilinear interpolation of the volume at x (Sec. 4.3.1), with the
    volume's voxels corner-aligned at +-1 on every axis."""
    vol = np.asarray(volume)
    nz, ny, nx = vol.shape
    x = np.asarray(x, np.float64)
    i0 = volume_cell_decision_f32(x, vol.shape)
    u = np.stack([(x[:, 0] + 1.0) * ((nx - 1) * 0.5),
                  (x[:, 1] + 1.0) * ((ny - 1) * 0.5),
                  (x[:, 2] + 1.0) * ((nz - 1) * 0.5)], axis=-1)
    w = u - i0
    cw = _corner_weights(w)
    v = np.zeros(x.shape[0])
    for q in range(8):
        a, b, c = q & 1, (q >> 1) & 1, (q >> 2) & 1
        v += cw[:, q] * vol[i0[:, 2] + c, i0[:, 1] + b, i0[:, 0] + a].astype(np.float64)
    return v


def reconstruction_loss(f, v):
    """L_rec = (1/|X|) sum (f - v)^2 (Sec. 4.3.1), its gradient dL/df, and the
    per-point error h(x) = (f - v)^2 used by Eq. (8) (reading: h is the
    summand of L_rec)."""
    f = np.asarray(f, np.float64)
    v = np.asarray(v, np.float64)
    N = f.shape[0]
    e = f - v
    loss = float(np.sum(e * e) / N) if N else 0.0
    return loss, (2.0 * e / N if N else e), e * e


# --------------------------------------------------------------------------
# Optimiser: Sec. 7 "Training" (Adam, Kingma & Ba)
# --------------------------------------------------------------------------

def adam_update(theta, g, m, v, t, lr, betas=ADAM_BETAS, eps=ADAM_EPS):
    """One bias-corrected Adam step at step number t >= 1.  Returns new
    (theta, m, v) without modifying the inputs."""
    b1, b2 = betas
    theta = np.asarray(theta, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# --------------------------------------------------------------------------
# Point generator (Sec. 7 "Training": uniform samples in [-1, 1]^3)
# --------------------------------------------------------------------------

_PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
_PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
POINT_KEY_HI = 0x41504D47  # second key word of the point stream


def _mulhilo64(a, b):
    """64x64 -> 128-bit product of uint64 arrays, via 32-bit limbs."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a_lo, a_hi = a & m32, a >> s32
    b_lo, b_hi = b & m32, b >> s32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> s32) + (lh & m32) + (hl & m32)
    lo = (ll & m32) | ((mid & m32) << s32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    return hi, lo


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds (Salmon et al., SC'11), vectorised.

    ctr: uint64 [..., 4]; key: uint64 [..., 2].  Returns uint64 [..., 4].
    """
    c = [np.asarray(ctr, np.uint64)[..., i].copy() for i in range(4)]
    k = [np.asarray(key, np.uint64)[..., i].copy() for i in range(2)]
    k = [np.broadcast_to(kk, c[0].shape).copy() for kk in k]
    M0, M1 = np.uint64(_PHILOX_M[0]), np.uint64(_PHILOX_M[1])
    W0, W1 = np.uint64(_PHILOX_W[0]), np.uint64(_PHILOX_W[1])
    with np.errstate(over="ignore"):
        for r in range(10):
            hi0, lo0 = _mulhilo64(M0, c[0])
            hi1, lo1 = _mulhilo64(M1, c[2])
            c = [hi1 ^ c[1] ^ k[0], lo1, hi0 ^ c[3] ^ k[1], lo0]
            if r < 9:
                k = [k[0] + W0, k[1] + W1]
    return np.stack(c, axis=-1)


def uniform_points(seed, step, stream, n, start=0):
    """Batch of n uniform points in [-1, 1)^3 for training step `step` of
    model `stream`.  Point j uses one Philox4x64-10 block with counter
    (start + j, step, stream, 0) and key (seed, 0x41504D47); coordinate d is
    (word_d >> 40) * 2^-23 - 1, a 24-bit lattice value exact in float32."""
    j = np.arange(start, start + n, dtype=np.uint64)
    ctr = np.zeros((n, 4), np.uint64)
    ctr[:, 0] = j
    ctr[:, 1] = np.uint64(step)
    ctr[:, 2] = np.uint64(stream)
    key = np.array([seed, POINT_KEY_HI], np.uint64)
    blk = philox4x64_10(ctr, key)
    bits = (blk[:, :3] >> np.uint64(40)).astype(np.float64)
    return bits * 2.0 ** -23 - 1.0


# --------------------------------------------------------------------------
# Domain decomposition: Sec. 5.1 (partitioning, ghost cells), Sec. 5.3 (hash)
# --------------------------------------------------------------------------

def brick_partition(shape_xyz, B, ghost):
    """Bricks of edge B voxels over a volume of shape (nx, ny, nz).

    Readings: I = ceil(nx / B) etc. (edge bricks are smaller); the base extent
    of brick i is voxels [iB, min((i+1)B, n)); the extended (ghost) extent is
    [max(iB - g, 0), min((i+1)B - 1 + g, n - 1)] (inclusive voxel indices).
    Bricks are listed in x, y, z order, id = i + I j + I J k (Sec. 5.3).
    Returns (dims (I, J, K), list of dicts with ijk, base0, base1, e0, e1).
    """
    dims = tuple(-(-n // B) for n in shape_xyz)
    bricks = []
    for k in range(dims[2]):
        for j in range(dims[1]):
            for i in range(dims[0]):
                ijk = (i, j, k)
                b0 = [ijk[d] * B for d in range(3)]
                b1 = [min((ijk[d] + 1) * B, shape_xyz[d]) for d in range(3)]
                e0 = [max(ijk[d] * B - ghost, 0) for d in range(3)]
                e1 = [min((ijk[d] + 1) * B - 1 + ghost, shape_xyz[d] - 1) for d in range(3)]
                bricks.append({"ijk": ijk, "base0": b0, "base1": b1, "e0": e0, "e1": e1})
    return dims, bricks


def brick_assign(x, shape_xyz, B, dims):
    """Sec. 5.3 spatial hash generalised to uneven edge bricks.

    The float32 voxel coordinate u_d = fma(p_d, h_d, h_d), h_d = (n_d - 1)/2,
    selects the base brick containing floor(u_d): i = min(floor(u) div B, I-1),
    clamped to >= 0.  For equal bricks this is floor(I (p+1)/2) clamped to
    < I.  Returns int64 [N] ids i + I j + I J k.
    """
    x32 = np.asarray(x, np.float32)
    idx = []
    for d in range(3):
        h = np.float32((shape_xyz[d] - 1) * 0.5)
        with np.errstate(invalid="ignore"):
            u = _fmaf(x32[:, d], h, h)
            u = np.where(np.isfinite(u), u, 0.0)
        k = np.floor(u).astype(np.int64)
        idx.append(np.clip(k // B, 0, dims[d] - 1))
    I, J, _ = dims
    return idx[0] + I * idx[1] + I * J * idx[2]


def brick_local_to_voxel(l, e0, e1):
    """A brick model's local coordinate l in [-1, 1] maps corner-aligned onto
    its extended extent: voxel u = e0 + (l + 1)/2 (e1 - e0)."""
    return np.asarray(e0, np.float64) + (np.asarray(l, np.float64) + 1.0) * 0.5 * (
        np.asarray(e1, np.float64) - np.asarray(e0, np.float64))


def brick_gt_sample(volume_zyx, brick, l):
    """v(l) for a brick model: trilinear sampling of the brick's extended
    sub-volume at local coordinates l [N, 3]."""
    e0, e1 = brick["e0"], brick["e1"]
    sub = np.asarray(volume_zyx)[e0[2]:e1[2] + 1, e0[1]:e1[1] + 1, e0[0]:e1[0] + 1]
    return gt_sample(sub, l)


# --------------------------------------------------------------------------
# One training step: Sec. 4.3.2 (two-part step) with Sec. 7 hyper-parameters
# --------------------------------------------------------------------------

def train_step(model, state, x, v, density_active, add_rec_dG=False,
               eps=EPS_DENSITY, p=P_FLATTOP, lr=LR_DEFAULT, lr_G=LR_TRANSFORM,
               betas=ADAM_BETAS, adam_eps=ADAM_EPS, abs_det=False, norm_target=False):
    """Part (1): L_rec updates F and the MLP.  Part (2), when the density phase
    is active: L_density updates G only (L_rec gives G no gradient; its dG is
    added only when add_rec_dG is set).

    state holds Adam moments and step counters: mF, vF, mW[], vW[], mG, vG,
    t (F and MLP) and tG (transforms; counts only steps that update G).
    Returns (new_model, new_state, info) without modifying the inputs.
    """
    f, cache = forward(model, x)
    L_rec, df, h = reconstruction_loss(f, v)
    g = backward(model, x, df, cache)
    info = {"f": f, "L_rec": L_rec, "h": h, "dF": g["dF"], "dW": g["dW"],
            "dG_rec": g["dG"], "L_density": 0.0, "dG_density": np.zeros_like(g["dG"])}
    new_model = dict(model)
    new_state = dict(state)
    t = state["t"] + 1
    new_state["t"] = t
    new_model["F"], new_state["mF"], new_state["vF"] = adam_update(
        model["F"], g["dF"], state["mF"], state["vF"], t, lr, betas, adam_eps)
    Ws, mWs, vWs = [], [], []
    for k in range(len(model["W"])):
        w_, m_, v_ = adam_update(model["W"][k], g["dW"][k], state["mW"][k], state["vW"][k],
                                 t, lr, betas, adam_eps)
        Ws.append(w_)
        mWs.append(m_)
        vWs.append(v_)
    new_model["W"], new_state["mW"], new_state["vW"] = Ws, mWs, vWs
    if density_active:
        d = density_loss(model["G"], x, h, eps, p, abs_det=abs_det, norm_target=norm_target)
        info["L_density"] = d["loss"]
        info["dG_density"] = d["dG"]
        dG = d["dG"] + (g["dG"] if add_rec_dG else 0.0)
        tG = state["tG"] + 1
        new_state["tG"] = tG
        G_new, new_state["mG"], new_state["vG"] = adam_update(
            np.asarray(model["G"], np.float64)[:, :3, :], dG, state["mG"], state["vG"],
            tG, lr_G, betas, adam_eps)
        new_model["G"] = G_new
    return new_model, new_state, info


def zero_adam_state(model):
    """Adam moments at zero and both step counters at 0."""
    return {"mF": np.zeros_like(np.asarray(model["F"], np.float64)),
            "vF": np.zeros_like(np.asarray(model["F"], np.float64)),
            "mW": [np.zeros_like(np.asarray(w, np.float64)) for w in model["W"]],
            "vW": [np.zeros_like(np.asarray(w, np.float64)) for w in model["W"]],
            "mG": np.zeros((np.asarray(model["G"]).shape[0], 3, 4)),
            "vG": np.zeros((np.asarray(model["G"]).shape[0], 3, 4)),
            "t": 0, "tG": 0}


# --------------------------------------------------------------------------
# Training schedule: Sec. 4.3.2 "Delayed start", "Early stopping"; Sec. 5.2
# early stopping of brick models (plateau scheduler)
# --------------------------------------------------------------------------

CONTROL_DEFAULTS = {"delay": 500, "ma_window": 1000, "ma_rel": 1e-4, "stop_frac": 0.8, "patience": 500,
                    "plateau_rel": 1e-4, "plateau_factor": 0.1, "max_reductions": 3}


def control_initial(delay=CONTROL_DEFAULTS["delay"]):
    """Per-model schedule state before the first iteration, and the flags of the first
    iteration (transforms train in it only when delay is 0)."""
    return {"iter": 0, "density_done": 0, "ma_count": 0, "have_prev": 0, "bad": 0, "reductions": 0,
            "ma_sum": 0.0, "ma_prev": 0.0, "best": 0.0,
            "density_active": 1 if delay == 0 else 0, "frozen": 0, "lr_scale": np.float32(1.0)}


def control_update(st, L_rec, L_density, total_iters, **kw):
    """The schedule after one iteration with losses (L_rec, L_density); returns the new state.

    Readings:
    * Delayed start: transforms are not trained in iterations 1..delay (the
      paper's 500); iteration t trains them when t > delay.
    * Transform early stop: the paper's "1000-iteration moving average has not
      reduced by 0.01%" is read on consecutive non-overlapping blocks of
      ma_window density iterations: when a block's mean L_density is not below
      the previous block's mean times (1 - ma_rel), transform training stops for
      good.  It also stops for iterations beyond stop_frac * total_iters (80%),
      the product taken in float32 and truncated.
    * Plateau scheduler (Sec. 5.2): an iteration whose L_rec is below
      best * (1 - plateau_rel) becomes the best and resets the bad count;
      otherwise the bad count grows; more than `patience` bad iterations in a
      row multiply the learning rates by plateau_factor (float32) and restart
      the count; the max_reductions-th reduction retires the model.
    * A retired model's state no longer changes.
    """
    p = dict(CONTROL_DEFAULTS)
    p.update(kw)
    st = dict(st)
    if st["frozen"]:
        return st
    it = st["iter"] + 1
    if st["density_active"]:
        st["ma_sum"] = st["ma_sum"] + float(L_density)
        st["ma_count"] += 1
        if st["ma_count"] == p["ma_window"]:
            mean = st["ma_sum"] / float(p["ma_window"])
            if st["have_prev"] and not (mean < st["ma_prev"] * (1.0 - p["ma_rel"])):
                st["density_done"] = 1
            st["ma_prev"] = mean
            st["have_prev"] = 1
            st["ma_sum"] = 0.0
            st["ma_count"] = 0
    limit = int(np.float32(p["stop_frac"]) * np.float32(total_iters))
    if it + 1 > limit:
        st["density_done"] = 1
    if it == 1 or float(L_rec) < st["best"] * (1.0 - p["plateau_rel"]):
        st["best"] = float(L_rec)
        st["bad"] = 0
    else:
        st["bad"] += 1
    frozen = 0
    if st["bad"] > p["patience"]:
        st["lr_scale"] = np.float32(np.float32(st["lr_scale"]) * np.float32(p["plateau_factor"]))
        st["bad"] = 0
        st["reductions"] += 1
        if st["reductions"] >= p["max_reductions"]:
            frozen = 1
    st["iter"] = it
    st["density_active"] = 1 if (not frozen and it >= p["delay"] and not st["density_done"]) else 0
    st["frozen"] = frozen
    return st


# --------------------------------------------------------------------------
# Domain-decomposition inference: Sec. 5.3 (spatial hash, local frame)
# --------------------------------------------------------------------------

def dd_local_coords(x, shape_xyz, brick):
    """A global point's coordinates in a brick model's frame: the inverse of
    brick_local_to_voxel over the brick's extended extent.

    Reading: the paper scales the global coordinate into the network's local
    domain without giving the arithmetic; it is taken in float32, each step
    rounded once, so that the grids' integer decisions downstream are exact:
    u = fma(p, h, h) with h = (n - 1)/2 (the voxel coordinate of the hash),
    l = fma(u - e0, 2/(e1 - e0), -1).  Returns float32 [N, 3].
    """
    x32 = np.asarray(x, np.float32)
    out = np.empty_like(x32)
    for d in range(3):
        h = np.float32((shape_xyz[d] - 1) * 0.5)
        with np.errstate(invalid="ignore"):
            u = _fmaf(x32[:, d], h, h)
            span = int(brick["e1"][d]) - int(brick["e0"][d])
            sc = np.float32(2.0) / np.float32(span) if span > 0 else np.float32(0.0)
            diff = (u - np.float32(brick["e0"][d])).astype(np.float32)
            out[:, d] = _fmaf(diff, sc, np.float32(-1.0))
    return out


def dd_forward(models, bricks, shape_xyz, B, dims, x):
    """f at global points x [N, 3] over a domain decomposition: each point is
    hashed to its brick (brick_assign), mapped into that brick's frame
    (dd_local_coords) and evaluated by the brick's model with the brick's
    (vmin, vmax).  models[b]: a model dict; bricks[b]: dict with e0, e1, vmin,
    vmax.  Returns (f [N] float64, brick ids [N])."""
    ids = brick_assign(x, shape_xyz, B, dims)
    f = np.zeros(len(ids))
    for b in np.unique(ids):
        sel = ids == b
        lc = dd_local_coords(np.asarray(x)[sel], shape_xyz, bricks[b])
        m = dict(models[b])
        m["vmin"], m["vmax"] = float(bricks[b]["vmin"]), float(bricks[b]["vmax"])
        f[sel], _ = forward(m, lc.astype(np.float64))
    return f, ids
