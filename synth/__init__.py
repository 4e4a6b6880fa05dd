"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

Nothing here computes any part of the method: these are the stand-ins for the
paper's datasets (Table 1: plume, nyx, supernova, asteroid, isotropic, ... are
not available) and the paper's initial parameter distributions (Sec. 4.3.3).
Volumes are closed-form fields sampled at voxel k of an n-voxel axis placed at
-1 + 2k/(n-1), then normalised to [0, 1]:

* "blobs_sine": anisotropic, randomly rotated Gaussian blobs plus a low
  amplitude plane-wave (a "somewhat sparse" field);
* "blobs_turb": narrow blobs plus a localised turbulent patch (32 random-phase
  sine modes with |k| log-uniform in [8, 64] cycles per unit and amplitude
  |k|^(-5/6), i.e. a k^(-5/3) energy spectrum) covering 5% of the domain,
  windowed by a flat-top box (a "not sparse" region).

Volumes are built with torch in float32, on the CPU or on a GPU, slab by slab.
"""
from __future__ import annotations

import math

import numpy as np

SEED_VOLUME = 1234
SEED_MODEL = 42
SEED_POINTS = 7


# --------------------------------------------------------------------------
# volume parameters (numpy, seeded) and evaluation (torch, any device)
# --------------------------------------------------------------------------

def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def volume_params(kind, seed=SEED_VOLUME):
    """Seeded parameters of a closed-form synthetic field."""
    rng = np.random.default_rng(seed)
    if kind == "blobs_sine":
        nb, sig, c_rng = 8, (0.05, 0.3), 0.7
    elif kind == "blobs_turb":
        nb, sig, c_rng = 64, (0.01, 0.1), 0.9
    else:
        raise ValueError(kind)
    blobs = []
    for _ in range(nb):
        c = rng.uniform(-c_rng, c_rng, 3)
        s = rng.uniform(sig[0], sig[1], 3)
        a = rng.uniform(0.5, 1.0)
        Rm = _random_rotation(rng)
        # quadratic form (x-c)^T P (x-c), P = R^T D^-2 R
        P = Rm.T @ np.diag(1.0 / s ** 2) @ Rm
        blobs.append((c, P, a))
    out = {"kind": kind, "blobs": blobs}
    if kind == "blobs_sine":
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        kmag = rng.uniform(4.0, 8.0)
        out["sine"] = (0.05, d * kmag, rng.uniform(0, 2 * math.pi))
    else:
        edge = 2.0 * 0.05 ** (1.0 / 3.0)            # 5% of the [-1,1]^3 volume
        lo = rng.uniform(-1.0, 1.0 - edge, 3)
        modes = []
        for _ in range(32):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            kmag = math.exp(rng.uniform(math.log(8.0), math.log(64.0)))
            modes.append((d * kmag, rng.uniform(0, 2 * math.pi), kmag ** (-5.0 / 6.0)))
        norm = sum(m[2] for m in modes)
        out["turb"] = {"lo": lo, "hi": lo + edge, "modes": modes, "amp": 1.0 / norm}
    return out


def _eval_field(params, X, Y, Z, torch):
    """Field value at coordinates X, Y, Z (torch float32 tensors)."""
    val = torch.zeros_like(X)
    for c, P, a in params["blobs"]:
        dx, dy, dz = X - float(c[0]), Y - float(c[1]), Z - float(c[2])
        q = (P[0, 0] * dx * dx + P[1, 1] * dy * dy + P[2, 2] * dz * dz
             + 2.0 * P[0, 1] * dx * dy + 2.0 * P[0, 2] * dx * dz + 2.0 * P[1, 2] * dy * dz)
        val += float(a) * torch.exp(-0.5 * q)
    if "sine" in params:
        amp, k, ph = params["sine"]
        val += amp * torch.sin(2 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
    if "turb" in params:
        t = params["turb"]
        win = torch.ones_like(X)
        for d, C in enumerate((X, Y, Z)):
            ctr = 0.5 * (t["lo"][d] + t["hi"][d])
            half = 0.5 * (t["hi"][d] - t["lo"][d])
            win = win * torch.exp(-(((C - ctr) / half) ** 20))     # flat-top box window
        turb = torch.zeros_like(X)
        for k, ph, amp in t["modes"]:
            turb += amp * torch.sin(2 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
        val += t["amp"] * win * turb
    return val


def make_volume(kind, shape_zyx, seed=SEED_VOLUME, device="cpu", slab=None):
    """Synthetic volume [Z][Y][X] float32 torch tensor on `device`, in [0, 1]."""
    import torch
    nz, ny, nx = shape_zyx
    params = volume_params(kind, seed)
    vol = torch.empty((nz, ny, nx), dtype=torch.float32, device=device)
    xs = torch.linspace(-1.0, 1.0, nx, dtype=torch.float32, device=device)
    ys = torch.linspace(-1.0, 1.0, ny, dtype=torch.float32, device=device)
    zs = torch.linspace(-1.0, 1.0, nz, dtype=torch.float32, device=device)
    if slab is None:
        target = (1 << 22) if str(device) == "cpu" else (1 << 25)
        slab = max(1, target // (nx * ny))
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        Z, Y, X = torch.meshgrid(zs[z0:z1], ys, xs, indexing="ij")
        vol[z0:z1] = _eval_field(params, X, Y, Z, torch)
    lo, hi = vol.min(), vol.max()
    vol.sub_(lo).div_(hi - lo)
    return vol


# --------------------------------------------------------------------------
# model parameters: Sec. 4.3.3 initialisation
# --------------------------------------------------------------------------

def init_model(M, C, R, widths, seed=SEED_MODEL, grid_range=1e-4, extra_translation=0.0,
               vmin=0.0, vmax=1.0):
    """Initial APMGSRN parameters as float32 numpy arrays.

    Transforms: diagonal ~ N(1, 0.05), the other entries of rows 0..2
    (translation included) ~ N(0, 0.05), plus an optional uniform
    +-extra_translation.  Grids ~ U(-grid_range, grid_range).  MLP weights
    [out][in], Glorot-uniform, no biases.  widths = [M*C, h1, ..., 1].
    """
    rng = np.random.default_rng(seed)
    G = rng.normal(0.0, 0.05, size=(M, 3, 4))
    G[:, [0, 1, 2], [0, 1, 2]] = rng.normal(1.0, 0.05, size=(M, 3))
    if extra_translation:
        G[:, :, 3] += rng.uniform(-extra_translation, extra_translation, size=(M, 3))
    F = rng.uniform(-grid_range, grid_range, size=(M, C, R, R, R))
    W = []
    for k in range(len(widths) - 1):
        lim = math.sqrt(6.0 / (widths[k] + widths[k + 1]))
        W.append(rng.uniform(-lim, lim, size=(widths[k + 1], widths[k])).astype(np.float32))
    return {"G": G.astype(np.float32), "F": F.astype(np.float32), "W": W,
            "vmin": np.float32(vmin), "vmax": np.float32(vmax)}


def uniform_points_host(n, seed=SEED_POINTS):
    """Host-side uniform points in [-1, 1)^3 on a 2^-23 lattice (float32 [n, 3]);
    an input for calls that take caller-provided points."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 1 << 24, size=(n, 3))
    return (k * 2.0 ** -23 - 1.0).astype(np.float32)


def ray_points(width=1920, height=1080, samples=8, aspect_half=0.5625):
    """Render-style layout: an orthographic camera looking along z.  Pixel
    (px, py) maps to the pixel centre in x in [-1, 1], y in [-h, h]; samples at
    z_k = -1 + (2k+1)/samples.  Point index (py*width + px)*samples + k.
    Returns float32 [width*height*samples, 3]."""
    px = (-1.0 + (2.0 * np.arange(width) + 1.0) / width).astype(np.float32)
    py = (-aspect_half + (2.0 * np.arange(height) + 1.0) * aspect_half / height).astype(np.float32)
    pz = (-1.0 + (2.0 * np.arange(samples) + 1.0) / samples).astype(np.float32)
    Y, X, Z = np.meshgrid(py, px, pz, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)
