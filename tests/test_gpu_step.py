"""GPU parity of the training step (apmg_batched_step, Sec. 4.3.2 with the Sec. 7
optimiser) against the FP64 oracle's train_step, through the C ABI.

What each comparison covers, and its bar:
  * Gradients enter the step through Adam: after one step m = (1 - beta1) g and
    v = (1 - beta2) g^2, and later steps test the recurrences and the bias
    corrections at t = 2, 3.  Moments: normwise and max error <= 1e-5, plus the
    envelope of the points whose ReLU decisions float32 arithmetic may take either
    way (hidden pre-activations within 2e-6 of sum_j |W_kj a_j| of a kink), carried
    through the moment recurrences.
  * The transforms' step counter advances on density steps only.
  * Updated parameters: 1e-5 on the entries whose update is determined to float32
    precision by the gradients (the update's first-order sensitivity to the
    gradients' noise, accumulated over the steps, at most 1e-6 max|theta|); the others are
    counted and left out -- the first Adam update is about lr sign(g).
  * The density loss and the transforms' moments carry the stated float32 error of
    h (its conditioning through h_bar / h, stated, bar 1e-3).
  * BF16 MLP / FP16 grid steps have their errors against the FP64 oracle stated
    (printed, with sanity bounds), not barred.
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


def f64(h, vmin=0.0, vmax=1.0):
    return {"G": h["G"].astype(np.float64), "F": h["F"].astype(np.float64),
            "W": [w.astype(np.float64) for w in h["W"]], "vmin": vmin, "vmax": vmax}


def split_w(flat, shapes):
    out, o = [], 0
    for sh in shapes:
        k = int(np.prod(sh))
        out.append(flat[o:o + k].reshape(sh))
        o += k
    return out


def brick_setup(vol, nb, B, ghost):
    nz, ny, nx = vol.shape
    _, bricks = A().apmg_make_bricks(nx, ny, nz, B, ghost)
    _, obricks = O.brick_partition((nx, ny, nz), B, ghost)
    return bricks[:nb], obricks[:nb]


def oracle_steps(host, vol_np, obrick, seed, stream, n, actives, **kw):
    """The oracle's steps 0..len(actives)-1 of one brick model, chained on its own state."""
    model, st = f64(host), O.zero_adam_state(f64(host))
    out = []
    for step, act in enumerate(actives):
        x = O.uniform_points(seed, step, stream, n)
        v = O.brick_gt_sample(vol_np, obrick, x)
        model, st, info = O.train_step(model, st, x, v, density_active=act, **kw)
        out.append((model, st, info))
    return out


def snapshot(tr, b):
    return {k: getattr(tr, k)[b].detach().cpu().numpy().astype(np.float64).copy()
            for k in ("G", "F", "W", "mG", "vG", "mF", "vF", "mW", "vW")} | \
        {"losses": tr.losses[b].cpu().numpy().copy(), "t": int(tr.t[b]), "tG": int(tr.tG[b])}


U32 = 2.0 ** -24


def noise_levels(model64, x, v, tau=2e-6):
    """Per entry of L_rec's gradients dF and dW (flat W): the float32 noise level and the
    envelope of the points near a ReLU kink.
      round: 32 u sum|terms| (the reductions) plus 3 (R-1) u times the sums that carry the
             encoder's corner-weight error (dF: sum |dL/dy| per vertex; dW: the sums with
             the features replaced by the interpolation of |F|): the float32 encoder holds
             u = (l + 1)(R-1)/2, so each weight factor is known to about (R-1) u;
      env:   twice the sums of |terms|, ambiguous ReLU units open, over the points whose
             hidden pre-activations lie within tau * sum_j |W_kj a_j| of a kink, where the
             float32 forward may take the ReLU decision either way.  (The float32 error of
             a pre-activation of these models stays below 3.3e-7 sum_j |W_kj a_j|, measured
             against float64 over 2^16 points; tau = 2e-6 is six times that.)"""
    f, cache = O.forward(model64, x)
    _, df, _ = O.reconstruction_loss(f, v)
    mag = O.backward_magnitudes(model64, x, df, cache)
    R = np.asarray(model64["F"]).shape[2]
    near = np.zeros(x.shape[0], bool)
    opened = []
    for k in range(len(model64["W"]) - 1):
        scale = np.abs(cache["a"][k]) @ np.abs(np.asarray(model64["W"][k], np.float64)).T
        amb = np.abs(cache["z"][k]) <= tau * scale
        opened.append(amb)
        near |= amb.any(axis=1)
    envF = np.zeros_like(mag["dF"])
    envW = np.zeros(sum(m.size for m in mag["dW"]))
    if near.any():
        env = O.backward_magnitudes(model64, x[near], df[near], open_units=[o[near] for o in opened])
        envF = 2.0 * env["dF"]
        envW = 2.0 * np.concatenate([e.ravel() for e in env["dW"]])
    kw = 3.0 * (R - 1)
    roundF = U32 * (32.0 * mag["dF"] + kw * mag["dF_unit"])
    roundW = U32 * np.concatenate([(32.0 * m + kw * mf).ravel() for m, mf in zip(mag["dW"], mag["dW_fabs"])])
    return {"roundF": roundF, "roundW": roundW, "envF": envF, "envW": envW, "kinks": int(near.sum())}


def check_env(name, got, want, allowed, tol=TOL):
    """|got - want| <= tol max|want| + allowed per entry, and ||got - want|| <= tol ||want|| +
    ||allowed||: the FP32 bar plus the part that ambiguous ReLU decisions may move."""
    got, want, allowed = (np.asarray(a, np.float64).ravel() for a in (got, want, allowed))
    d = np.abs(got - want)
    a, b = errs(got, want)
    ok_max = np.all(d <= tol * np.abs(want).max() + allowed)
    ok_norm = np.linalg.norm(d) <= tol * np.linalg.norm(want) + np.linalg.norm(allowed)
    env = np.linalg.norm(allowed) / max(np.linalg.norm(want), 1e-300)
    print(f"{name}: normwise {a:.2e}, max {b:.2e}, kink envelope {env:.1e}", flush=True)
    assert ok_max and ok_norm, (name, a, b)


class Track:
    """The oracle's view of one model over consecutive steps, for the comparisons:
      * amF/avF, amW/avW: how far ambiguous ReLU decisions (the kink envelope) may move
        the Adam moments, propagated through their recurrences;
      * keep(): entries whose updated parameter is determined to float32 precision by
        the gradients.  With u_t = lr m_hat_t / (sqrt(v_hat_t) + eps) the update of step
        t, the parameter after step T moves by sum_s |d theta_T / d g_s| dg_s to first
        order under gradient changes dg_s, where d theta_T / d g_s = -sum_{t >= s} du_t / dg_s
        (signed: at t = 1 the m and v parts cancel to lr eps / (|g| + eps)^2) and dg_s is
        the gradient's noise level (noise_levels: rounding plus the kink envelope).  Entries where
        that exceeds 1e-6 max|theta| (a tenth of the bar), or whose gradient is within
        twice its noise of zero at some step (the sign of the first update, about
        lr sign(g), is then not determined), are left out and counted."""

    def __init__(self, nF, nW, lr=0.01, b1=0.9, b2=0.99, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps, self.t = lr, b1, b2, eps, 0
        self.st = {k: {"am": np.zeros(n), "av": np.zeros(n), "g": [], "noise": [], "D": [],
                       "ok": np.ones(n, bool)} for k, n in (("F", nF), ("W", nW))}

    def add(self, gF, gW, nl, ost):
        self.t += 1
        b1, b2, t, lr, eps = self.b1, self.b2, self.t, self.lr, self.eps
        bc1, bc2 = 1 - b1 ** t, 1 - b2 ** t
        for k, g, rnd, env, m, v in (("F", gF, nl["roundF"].ravel(), nl["envF"].ravel(), ost["mF"].ravel(),
                                      ost["vF"].ravel()),
                                     ("W", gW, nl["roundW"], nl["envW"], flat_w(ost["mW"]), flat_w(ost["vW"]))):
            d = self.st[k]
            g = np.asarray(g, np.float64)
            ag = np.abs(g)
            d["am"] = b1 * d["am"] + (1 - b1) * env
            d["av"] = b2 * d["av"] + (1 - b2) * (2 * ag * env + env * env)
            noise = rnd + env
            d["g"].append(g)
            d["noise"].append(noise)
            d["D"].append(np.zeros_like(g))
            d["ok"] &= (ag > 2.0 * noise) | ((g == 0.0) & (noise == 0.0))
            sv = np.sqrt(np.asarray(v, np.float64) / bc2)
            mh = np.asarray(m, np.float64) / bc1
            inv = 1.0 / (sv + eps)
            cv = np.where(sv > 0, mh / (2 * np.maximum(sv, 1e-300)) * inv * inv, 0.0)
            for s_ in range(t):
                dm = (1 - b1) * b1 ** (t - 1 - s_) / bc1
                dv = 2 * (1 - b2) * b2 ** (t - 1 - s_) * d["g"][s_] / bc2
                d["D"][s_] = d["D"][s_] + lr * (dm * inv - cv * dv)

    def keep(self, k, theta):
        """(entries with determined update signs, entries with determined updates)"""
        d = self.st[k]
        S = sum(np.abs(D) * nz for D, nz in zip(d["D"], d["noise"]))
        return d["ok"], d["ok"] & (S <= 1e-6 * np.abs(np.asarray(theta, np.float64)).max())

    @property
    def amF(self):
        return self.st["F"]["am"]

    @property
    def avF(self):
        return self.st["F"]["av"]

    @property
    def amW(self):
        return self.st["W"]["am"]

    @property
    def avW(self):
        return self.st["W"]["av"]



def compare_masked(name, got, want, masks, tol=TOL):
    """masks = (signs, keep): the normwise error over the entries whose update signs are
    determined at every step, the max error over those whose update is determined to
    float32 precision; both <= tol."""
    signs, keep = masks
    got, want = np.asarray(got, np.float64).ravel(), np.asarray(want, np.float64).ravel()
    a, _ = errs(got[signs], want[signs])
    _, b = errs(got[keep], want[keep])
    print(f"{name}: normwise {a:.2e} ({(~signs).sum()} of {signs.size} entries with undetermined signs left out), "
          f"max {b:.2e} ({(~keep).sum()} undetermined entries left out)", flush=True)
    assert a <= tol and b <= tol, (name, a, b)


def flat_w(ws):
    return np.concatenate([np.asarray(w, np.float64).ravel() for w in ws])


# ----------------------------------------------------------------------------------------- FP32
@pytest.mark.parametrize("nb", [1, 2])
def test_three_steps_match_oracle_moments_parameters_and_counters(nb):
    # three consecutive steps, the density phase on in steps 1 and 3 and off in step 2: the
    # first and second moments, the updated F/W/G, the bias corrections at t = 2, 3, and tG
    # advancing on density steps only
    vol = synth.make_volume("blobs_sine", (40, 44, 36))
    bricks, obricks = brick_setup(vol, nb, 24 if nb > 1 else 48, 1 if nb > 1 else 0)
    hosts = [synth.init_model(8, 2, 8, [16, 64, 64, 1], seed=50 + b, grid_range=0.2) for b in range(nb)]
    n = 2000
    actives = [True, False, True]
    tr = A().Trainer(hosts, vol.to(DEV), bricks, n, seed=7)
    snaps = []
    for act in actives:
        tr.density_active.fill_(1 if act else 0)
        tr.step()
        torch.cuda.synchronize()
        snaps.append([snapshot(tr, b) for b in range(nb)])
    vol_np = vol.numpy().astype(np.float64)
    for b in range(nb):
        model, st = f64(hosts[b]), O.zero_adam_state(f64(hosts[b]))
        trk = Track(model["F"].size, sum(w.size for w in model["W"]))
        for s, act in enumerate(actives):
            x = O.uniform_points(7, s, b, n)
            v = O.brick_gt_sample(vol_np, obricks[b], x)
            nl = noise_levels(model, x, v)
            model, st, info = O.train_step(model, st, x, v, density_active=act)
            trk.add(info["dF"].ravel(), flat_w(info["dW"]), nl, st)
            got = snaps[s][b]
            tag = f"[model {b}, step {s + 1}, {nl['kinks']} points near a kink]"
            assert got["t"] == s + 1 and got["tG"] == sum(actives[:s + 1]), (got["t"], got["tG"])
            assert_close("L_rec " + tag, [got["losses"][0]], [info["L_rec"]])
            if act:
                a, _ = errs([got["losses"][1]], [info["L_density"]])
                print(f"L_density {tag}: rel {a:.2e} (h in float32 on the GPU, stated)")
                assert a < 1e-3
            else:
                assert got["losses"][1] == 0.0
            check_env("mF " + tag, got["mF"], st["mF"], trk.amF)
            check_env("vF " + tag, got["vF"], st["vF"], trk.avF)
            check_env("mW " + tag, got["mW"], flat_w(st["mW"]), trk.amW)
            check_env("vW " + tag, got["vW"], flat_w(st["vW"]), trk.avW)
            compare_masked("F " + tag, got["F"], model["F"], trk.keep("F", model["F"]))
            compare_masked("W " + tag, got["W"], flat_w(model["W"]), trk.keep("W", flat_w(model["W"])))
            # transforms: the density gradient carries the stated error of h (float32 errors,
            # the conditioning rule for the density loss); its moments are compared at that
            # bar and the updates, about lr_G sign(g), at the FP32 bar
            a, _ = errs(got["mG"], st["mG"])
            print(f"mG {tag}: normwise {a:.2e} (density gradient, stated)")
            assert a < 1e-3
            a, _ = errs(got["G"], np.asarray(model["G"])[:, :3, :])
            print(f"G {tag}: normwise {a:.2e}")
            assert a < 1e-5
            if not act:
                prev = snaps[s - 1][b]
                for k in ("G", "mG", "vG"):
                    assert np.array_equal(got[k], prev[k]), k


def test_step_at_headline_shape_matches_oracle():
    # the headline model shape (32 grids at 32^3 x 2, MLP 64-64-64-1, density on) with 2^17
    # points: a multi-tile sort, the point regeneration with ground truth, the one-round
    # adjoint over all blocks, the wave gather and the density passes over a large batch
    vol = synth.make_volume("blobs_turb", (96, 96, 96))
    bricks, obricks = brick_setup(vol, 1, 96, 0)
    host = synth.init_model(32, 2, 32, [64, 64, 64, 1], seed=42)
    n = 1 << 17
    tr = A().Trainer([host], vol.to(DEV), bricks, n, seed=7)
    tr.density_active.fill_(1)
    tr.step()
    torch.cuda.synchronize()
    got = snapshot(tr, 0)
    model = f64(host)
    x = O.uniform_points(7, 0, 0, n)
    v = O.brick_gt_sample(vol.numpy().astype(np.float64), obricks[0], x)
    nl = noise_levels(model, x, v)
    om, ost, info = O.train_step(model, O.zero_adam_state(model), x, v, density_active=True)
    trk = Track(model["F"].size, sum(w.size for w in model["W"]))
    trk.add(info["dF"].ravel(), flat_w(info["dW"]), nl, ost)
    print(f"{nl['kinks']} of {n} points near a ReLU kink")
    assert_close("L_rec", [got["losses"][0]], [info["L_rec"]])
    a, _ = errs([got["losses"][1]], [info["L_density"]])
    print(f"L_density: rel {a:.2e} (stated)")
    assert a < 1e-3
    check_env("mF", got["mF"], ost["mF"], trk.amF)
    check_env("vF", got["vF"], ost["vF"], trk.avF)
    check_env("mW", got["mW"], flat_w(ost["mW"]), trk.amW)
    check_env("vW", got["vW"], flat_w(ost["vW"]), trk.avW)
    a, _ = errs(got["mG"], ost["mG"])
    print(f"mG: normwise {a:.2e} (stated)")
    assert a < 1e-3
    compare_masked("F", got["F"], om["F"], trk.keep("F", om["F"]))
    compare_masked("W", got["W"], flat_w(om["W"]), trk.keep("W", flat_w(om["W"])))


# ------------------------------------------------------------------------------ mixed precision
def _stated(name, got, want, bound):
    a, b = errs(got, want)
    print(f"{name}: normwise {a:.2e}, max {b:.2e} (stated)", flush=True)
    assert a < bound, (name, a)
    return a


def test_fp16_gathers_equal_the_rounded_masters():
    # grid_dtype F16: the encoder gathers the F16 rounding of the float32 masters, and the
    # gradients accumulate in float32 -- so the step equals, to the FP32 bar, the oracle's
    # step on the rounded grids
    vol = synth.make_volume("blobs_sine", (40, 44, 36))
    bricks, obricks = brick_setup(vol, 1, 48, 0)
    host = synth.init_model(8, 2, 8, [16, 64, 64, 1], seed=61, grid_range=0.3)
    n = 3000
    tr = A().Trainer([host], vol.to(DEV), bricks, n, seed=5, grid_dtype=torch.float16)
    tr.density_active.fill_(0)
    tr.step()
    torch.cuda.synchronize()
    got = snapshot(tr, 0)
    rounded = dict(host, F=host["F"].astype(np.float16).astype(np.float32))
    model = f64(rounded)
    x = O.uniform_points(5, 0, 0, n)
    v = O.brick_gt_sample(vol.numpy().astype(np.float64), obricks[0], x)
    nl = noise_levels(model, x, v)
    om, ost, info = O.train_step(model, O.zero_adam_state(model), x, v, density_active=False)
    trk = Track(model["F"].size, sum(w.size for w in model["W"]))
    trk.add(info["dF"].ravel(), flat_w(info["dW"]), nl, ost)
    assert_close("L_rec (F16 gathers)", [got["losses"][0]], [info["L_rec"]])
    check_env("mF (F16 gathers, float32 gradient)", got["mF"], ost["mF"], trk.amF)
    # the masters stay float32: F - F0 is the float32 Adam update, not an F16 rounding
    upd = got["F"] - host["F"].astype(np.float64)
    compare_masked("F update", upd, om["F"] - model["F"], trk.keep("F", om["F"]))


def test_mixed_precision_step_errors_stated():
    # the mixed-precision workload's model (32 grids at 32^3 x 2, BF16 MLP products with float32
    # accumulation, FP16 grid gathers, float32 masters), 2^17 points, density on: the error of
    # every output and gradient of the step against the FP64 oracle on the unrounded model
    vol = synth.make_volume("blobs_turb", (96, 96, 96))
    bricks, obricks = brick_setup(vol, 1, 96, 0)
    host = synth.init_model(32, 2, 32, [64, 64, 64, 1], seed=42)
    n = 1 << 17
    tr = A().Trainer([host], vol.to(DEV), bricks, n, seed=7, mlp_dtype=A().BF16, grid_dtype=torch.float16)
    tr.density_active.fill_(1)
    tr.step()
    torch.cuda.synchronize()
    got = snapshot(tr, 0)
    (om, ost, info), = oracle_steps(host, vol.numpy().astype(np.float64), obricks[0], 7, 0, n, [True])
    _stated("bf16+fp16 L_rec", [got["losses"][0]], [info["L_rec"]], 5e-2)
    _stated("bf16+fp16 L_density", [got["losses"][1]], [info["L_density"]], 5e-2)
    _stated("bf16+fp16 dF (from mF)", got["mF"] / 0.1, info["dF"], 0.2)
    wshapes = [w.shape for w in host["W"]]
    for k, m_ in enumerate(split_w(got["mW"], wshapes)):
        _stated(f"bf16+fp16 dW{k + 1} (from mW)", m_ / 0.1, info["dW"][k], 0.2)
    _stated("bf16+fp16 dG_density (from mG)", got["mG"] / 0.1, info["dG_density"], 0.2)
    _stated("bf16+fp16 updated F", got["F"], om["F"], 0.2)


def test_brick_step_bf16_errors_stated():
    # the batched-brick workload's per-brick model (16 grids at 32^3 x 2, MLP 32-64-64-1 in
    # BF16) over three uneven bricks with one ghost voxel, 2^15 points per brick
    vol = synth.make_volume("blobs_turb", (100, 120, 90))
    bricks, obricks = brick_setup(vol, 3, 64, 1)
    hosts = [synth.init_model(16, 2, 32, [32, 64, 64, 1], seed=70 + b) for b in range(3)]
    n = 1 << 15
    tr = A().Trainer(hosts, vol.to(DEV), bricks, n, seed=11, mlp_dtype=A().BF16)
    tr.density_active.fill_(1)
    tr.step()
    torch.cuda.synchronize()
    vol_np = vol.numpy().astype(np.float64)
    wshapes = [w.shape for w in hosts[0]["W"]]
    for b in range(3):
        got = snapshot(tr, b)
        (om, ost, info), = oracle_steps(hosts[b], vol_np, obricks[b], 11, b, n, [True])
        _stated(f"brick {b} bf16 L_rec", [got["losses"][0]], [info["L_rec"]], 5e-2)
        _stated(f"brick {b} bf16 L_density", [got["losses"][1]], [info["L_density"]], 5e-2)
        _stated(f"brick {b} bf16 dF", got["mF"] / 0.1, info["dF"], 0.2)
        for k, m_ in enumerate(split_w(got["mW"], wshapes)):
            _stated(f"brick {b} bf16 dW{k + 1}", m_ / 0.1, info["dW"][k], 0.2)
        _stated(f"brick {b} bf16 dG_density", got["mG"] / 0.1, info["dG_density"], 0.2)


# ------------------------------------------------------------------------------ batching
def test_brick_in_the_batch_equals_brick_alone_bitwise():
    # the domain decomposition's bricks are independent models (Sec. 5.2): with a fixed
    # launch shape, brick b stepped inside the batch and brick b stepped alone (drawing its
    # points from the same counter stream) end with bitwise equal parameters and moments
    vol = synth.make_volume("blobs_turb", (100, 120, 90)).to(DEV)
    bricks, _ = brick_setup(vol.cpu(), 4, 64, 1)
    hosts = [synth.init_model(8, 2, 16, [16, 64, 64, 1], seed=80 + b) for b in range(4)]
    n = 20000
    tune = {"tile_blocks": 16, "cell_kernel": 1, "cell_group": 4}
    batch = A().Trainer(hosts, vol, bricks, n, seed=3, tuning=tune)
    batch.density_active.fill_(1)
    for _ in range(2):
        batch.step()
    alone = []
    for b in range(4):
        tr = A().Trainer([hosts[b]], vol, [bricks[b]], n, seed=3, tuning=tune, stream0=b)
        tr.density_active.fill_(1)
        for _ in range(2):
            tr.step()
        alone.append(tr)
    torch.cuda.synchronize()
    for b in range(4):
        for k in ("G", "F", "W", "mG", "vG", "mF", "vF", "mW", "vW", "losses"):
            assert torch.equal(getattr(batch, k)[b], getattr(alone[b], k)[0]), (b, k)


# ------------------------------------------------------------------------------ density readings
@pytest.mark.parametrize("flags", ["abs", "norm", "abs+norm"])
def test_density_readings_match_oracle(flags):
    # the alternative readings of Eqs. (7) and (9) against the oracle, with the same err on
    # both sides; with |det|, on transforms that include reflected grids (negative
    # determinants, for which the signed reading gives negative densities)
    A_ = A()
    fl = (A_.DENSITY_ABS_DET if "abs" in flags else 0) | (A_.DENSITY_NORM_TARGET if "norm" in flags else 0)
    host = synth.init_model(12, 2, 8, [24, 64, 64, 1], seed=90, extra_translation=0.2)
    G = host["G"].copy()
    if "abs" in flags:
        G[::3, 0, :] *= -1.0                    # every third grid reflected (det < 0)
    host = dict(host, G=G)
    n = 20000
    x = synth.uniform_points_host(n, seed=91).astype(np.float32)
    err = (np.random.default_rng(92).uniform(0, 1, n) ** 3).astype(np.float32)
    model = A_.Model.from_host(host, DEV)
    pts = torch.from_numpy(np.ascontiguousarray(x.T)).to(DEV)
    loss, dG, rho = A_.apmg_density_loss(model, pts, torch.from_numpy(err).to(DEV), eps=1e-12, p=10,
                                         want_rho=True, flags=fl)
    r = O.density_loss(G.astype(np.float64), x.astype(np.float64), err.astype(np.float64), eps=1e-12,
                       abs_det="abs" in flags, norm_target="norm" in flags)
    assert_close(f"rho ({flags})", rho.cpu().numpy(), r["rho"])
    assert_close(f"L_density ({flags})", [loss.item()], [r["loss"]])
    assert_close(f"dG ({flags})", dG.cpu().numpy(), r["dG"])


def test_step_with_density_readings_matches_oracle():
    # a training step under |det| and the renormalised target, with two reflected grids
    A_ = A()
    vol = synth.make_volume("blobs_sine", (40, 44, 36))
    bricks, obricks = brick_setup(vol, 1, 48, 0)
    host = synth.init_model(8, 2, 8, [16, 64, 64, 1], seed=95, grid_range=0.2)
    G = host["G"].copy()
    G[[1, 5], 2, :] *= -1.0
    host = dict(host, G=G)
    n = 3000
    tr = A_.Trainer([host], vol.to(DEV), bricks, n, seed=9,
                    flags=A_.DENSITY_ABS_DET | A_.DENSITY_NORM_TARGET)
    tr.density_active.fill_(1)
    tr.step()
    torch.cuda.synchronize()
    got = snapshot(tr, 0)
    (om, ost, info), = oracle_steps(host, vol.numpy().astype(np.float64), obricks[0], 9, 0, n, [True],
                                    abs_det=True, norm_target=True)
    assert_close("L_rec", [got["losses"][0]], [info["L_rec"]])
    a, _ = errs([got["losses"][1]], [info["L_density"]])
    print(f"L_density (|det|, renormalised target): rel {a:.2e} (stated)")
    assert a < 1e-3
    a, _ = errs(got["mG"], ost["mG"])
    print(f"mG (|det|, renormalised target): normwise {a:.2e} (stated)")
    assert a < 1e-3


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_step_adjoint_kernel_variants_match_oracle(variant):
    # every fused-adjoint variant (eight-wave and four-wave tiled kernels, the one-wave-per-
    # SIMD register kernel) against the oracle's step, float32 MLP, two bricks with a ragged
    # tile count (3001 points) and 24 features (a partial dW1 column block)
    vol = synth.make_volume("blobs_sine", (40, 44, 36))
    bricks, obricks = brick_setup(vol, 2, 24, 1)
    hosts = [synth.init_model(12, 2, 8, [24, 64, 64, 1], seed=97 + b, grid_range=0.2) for b in range(2)]
    n = 3001
    tr = A().Trainer(hosts, vol.to(DEV), bricks, n, seed=13, tuning={"adjoint_kernel": variant})
    tr.density_active.fill_(0)
    tr.step()
    torch.cuda.synchronize()
    vol_np = vol.numpy().astype(np.float64)
    for b in range(2):
        got = snapshot(tr, b)
        model = f64(hosts[b])
        x = O.uniform_points(13, 0, b, n)
        v = O.brick_gt_sample(vol_np, obricks[b], x)
        nl = noise_levels(model, x, v)
        om, ost, info = O.train_step(model, O.zero_adam_state(model), x, v, density_active=False)
        trk = Track(model["F"].size, sum(w.size for w in model["W"]))
        trk.add(info["dF"].ravel(), flat_w(info["dW"]), nl, ost)
        tag = f"[variant {variant}, model {b}]"
        assert_close("L_rec " + tag, [got["losses"][0]], [info["L_rec"]])
        check_env("mF " + tag, got["mF"], ost["mF"], trk.amF)
        check_env("mW " + tag, got["mW"], flat_w(ost["mW"]), trk.amW)


def test_empty_batch_step_is_adam_on_zero_gradients():
    # a step over an empty batch (n = 0): both losses are 0 and every gradient is zero, so F
    # and W take the Adam update of a zero gradient from their current moments at t + 1, the
    # transforms do the same (at tG + 1) only where the density phase is on, and elsewhere
    # G, mG, vG and tG are left bit for bit
    vol = synth.make_volume("blobs_sine", (40, 44, 36))
    nb = 2
    bricks, _ = brick_setup(vol, nb, 24, 1)
    hosts = [synth.init_model(8, 2, 8, [16, 64, 64, 1], seed=70 + b, grid_range=0.2) for b in range(nb)]
    tr = A().Trainer(hosts, vol.to(DEV), bricks, 0, seed=7)
    rng = np.random.default_rng(17)
    for k in ("mF", "mW", "mG"):
        m = getattr(tr, k)
        vk = getattr(tr, "v" + k[1:])
        mv = rng.normal(0.0, 1e-3, tuple(m.shape))
        m.copy_(torch.from_numpy(mv.astype(np.float32)))
        vk.copy_(torch.from_numpy((mv * mv * rng.uniform(0.5, 2.0, mv.shape) + 1e-12).astype(np.float32)))
    t0, tG0 = 4, 2
    tr.t.fill_(t0)
    tr.tG.fill_(tG0)
    tr.density_active.copy_(torch.tensor([1, 0], dtype=torch.int32))
    before = [snapshot(tr, b) for b in range(nb)]
    tr.step()
    torch.cuda.synchronize()
    for b in range(nb):
        got, old = snapshot(tr, b), before[b]
        assert np.array_equal(got["losses"], [0.0, 0.0]), got["losses"]
        assert got["t"] == t0 + 1
        for k in ("F", "W"):
            want, wm, wv = O.adam_update(old[k], 0.0, old["m" + k], old["v" + k], t0 + 1, O.LR_DEFAULT)
            assert_close(f"{k} [model {b}]", got[k], want)
            assert_close(f"m{k} [model {b}]", got["m" + k], wm)
            assert_close(f"v{k} [model {b}]", got["v" + k], wv)
        if b == 0:
            assert got["tG"] == tG0 + 1
            want, wm, wv = O.adam_update(old["G"], 0.0, old["mG"], old["vG"], tG0 + 1, O.LR_TRANSFORM)
            assert_close(f"G [model {b}]", got["G"], want)
            assert_close(f"mG [model {b}]", got["mG"], wm)
            assert_close(f"vG [model {b}]", got["vG"], wv)
        else:
            assert got["tG"] == tG0
            for k in ("G", "mG", "vG"):
                assert np.array_equal(got[k], old[k]), k
