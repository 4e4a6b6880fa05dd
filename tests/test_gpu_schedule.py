"""GPU checks of the training schedule (apmg_train_control) against the oracle's rules,
of retired models and learning-rate scales in the batched step, and of the autotuner."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import apmg_oracle as O

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda"


def A():
    import paper_2308_02494_amd as mod
    return mod


def _control(nb, total, **kw):
    A_ = A()
    p = dict(O.CONTROL_DEFAULTS)
    p.update(kw)
    c = A_.ApmgControl()
    c.nb, c.delay, c.total_iters, c.ma_window = nb, p["delay"], total, p["ma_window"]
    c.patience, c.max_reductions = p["patience"], p["max_reductions"]
    c.stop_frac, c.plateau_factor, c.ma_rel, c.plateau_rel = p["stop_frac"], p["plateau_factor"], p["ma_rel"], \
        p["plateau_rel"]
    arrs = {"state": torch.zeros((nb, ctypes.sizeof(A_.ApmgCtlState)), dtype=torch.uint8, device=DEV),
            "density_active": torch.full((nb,), 1 if p["delay"] == 0 else 0, dtype=torch.int32, device=DEV),
            "frozen": torch.zeros(nb, dtype=torch.int32, device=DEV),
            "lr_scale": torch.ones(nb, dtype=torch.float32, device=DEV)}
    c.state = arrs["state"].data_ptr()
    c.density_active = arrs["density_active"].data_ptr()
    c.frozen = arrs["frozen"].data_ptr()
    c.lr_scale = arrs["lr_scale"].data_ptr()
    return c, arrs


def _dev_state(arrs, b):
    st = A().ApmgCtlState.from_buffer_copy(arrs["state"][b].cpu().numpy().tobytes())
    d = {k: getattr(st, k) for k, _ in A().ApmgCtlState._fields_}
    d["density_active"] = int(arrs["density_active"][b].item())
    d["frozen"] = int(arrs["frozen"][b].item())
    d["lr_scale"] = np.float32(arrs["lr_scale"][b].item())
    return d


def _losses(nb, T, seed):
    """Per-model loss sequences with descents, plateaus and noise (seeded)."""
    rng = np.random.default_rng(seed)
    out = np.zeros((T, nb, 2))
    for b in range(nb):
        t = np.arange(T)
        knee = rng.integers(20, 80)
        lrec = np.where(t < knee, 1.0 / (1.0 + 0.05 * t), 1.0 / (1.0 + 0.05 * knee))
        lrec = lrec * (1.0 + 1e-3 * b * rng.standard_normal(T))
        lden = 0.5 / (1.0 + 0.02 * t * (b % 3)) + 1e-4 * rng.standard_normal(T)
        out[:, b, 0], out[:, b, 1] = lrec, np.abs(lden)
    return out


@pytest.mark.parametrize("kw", [dict(delay=5, ma_window=7, ma_rel=1e-2, patience=4, plateau_rel=1e-3,
                                     plateau_factor=0.1, max_reductions=2, stop_frac=0.8),
                                dict(delay=0, ma_window=3, ma_rel=1e-4, patience=9, plateau_rel=1e-4,
                                     plateau_factor=0.5, max_reductions=3, stop_frac=0.5)])
def test_train_control_matches_oracle_every_iteration(kw):
    nb, T = 6, 150
    seq = _losses(nb, T, 5)
    ctl, arrs = _control(nb, T, **kw)
    losses = torch.zeros((nb, 2), dtype=torch.float64, device=DEV)
    ost = [O.control_initial(kw["delay"]) for _ in range(nb)]
    events = set()
    for t in range(T):
        losses.copy_(torch.from_numpy(seq[t]))
        A().train_control(ctl, losses)
        torch.cuda.synchronize()
        for b in range(nb):
            ost[b] = O.control_update(ost[b], seq[t, b, 0], seq[t, b, 1], T, **kw)
            got = _dev_state(arrs, b)
            for k, v in ost[b].items():
                assert got[k] == v, (t, b, k, got[k], v)
            events.update(k for k in ("density_done", "frozen", "reductions") if ost[b][k])
    print("events seen:", sorted(events))
    assert {"density_done", "reductions"} <= events


def _bricks_trainer(nb=3, n=4000, lr=0.01, lr_G=0.001, **kw):
    vol = synth.make_volume("blobs_turb", (40, 48, 44)).to(DEV)
    nz, ny, nx = vol.shape
    _, bricks = A().apmg_make_bricks(nx, ny, nz, 24, 1)
    bricks = bricks[:nb]
    hosts = [synth.init_model(8, 2, 8, [16, 64, 64, 1], seed=30 + b, grid_range=0.2) for b in range(nb)]
    tr = A().Trainer(hosts, vol, bricks, n, seed=11, lr=lr, lr_G=lr_G, **kw)
    if "control" not in kw:
        tr.density_active.fill_(1)
    return tr


def _params(tr, b):
    return [x[b].clone() for x in (tr.G, tr.F, tr.W, tr.mG, tr.vG, tr.mF, tr.vF, tr.mW, tr.vW)]


def test_frozen_model_is_untouched_and_others_unaffected():
    ref, frz = _bricks_trainer(), _bricks_trainer()
    frz.frozen[1] = 1
    before = _params(frz, 1)
    for _ in range(3):
        ref.step()
        frz.step()
    torch.cuda.synchronize()
    for x, y in zip(before, _params(frz, 1)):
        assert torch.equal(x, y)
    assert int(frz.t[1].item()) == 0 and int(frz.tG[1].item()) == 0
    for b in (0, 2):
        for x, y in zip(_params(ref, b), _params(frz, b)):
            assert torch.equal(x, y), b
    assert int(frz.t[0].item()) == 3 and int(frz.tG[2].item()) == 3


def test_lr_scale_equals_scaled_learning_rates():
    # halving is exact in float32, so lr * 0.5 in the kernel equals the halved rate bitwise
    a = _bricks_trainer(lr=0.01, lr_G=0.001)
    b = _bricks_trainer(lr=0.005, lr_G=0.0005)
    a.lr_scale.fill_(0.5)
    for _ in range(2):
        a.step()
        b.step()
    torch.cuda.synchronize()
    for m in range(3):
        for x, y in zip(_params(a, m), _params(b, m)):
            assert torch.equal(x, y)


def test_trainer_schedule_inside_a_graph_matches_eager():
    kw = dict(control=dict(total_iters=40, delay=2, ma_window=3, patience=3, plateau_rel=1e-2,
                           max_reductions=2))
    eager, graphed = _bricks_trainer(**kw), _bricks_trainer(**kw)
    eager.step()
    graphed.step()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            graphed.step()
    torch.cuda.synchronize()
    for k in range(12):
        g.replay()
        eager.step()
        torch.cuda.synchronize()
        for x, y in zip((eager.G, eager.F, eager.W, eager.density_active, eager.frozen, eager.lr_scale,
                         eager.ctl_state), (graphed.G, graphed.F, graphed.W, graphed.density_active,
                                            graphed.frozen, graphed.lr_scale, graphed.ctl_state)):
            assert torch.equal(x, y), k
    st = eager.control_state()
    assert all(s_["iter"] == 13 for s_ in st)
    assert int(eager.tG[0].item()) > 0


def test_autotune_returns_a_valid_shape_and_leaves_parameters():
    tr = _bricks_trainer(nb=2, n=20000)
    before = [x.clone() for x in (tr.G, tr.F, tr.W, tr.mF, tr.t, tr.step_ctr)]
    tune, ms = tr.autotune()
    torch.cuda.synchronize()
    print("autotune:", tune, f"{ms:.3f} ms")
    assert tune["cell_unroll"] in (2, 4, 8) and tune["tile_blocks"] >= 1 and tune["cell_kernel"] in (1, 2)
    assert tune["cell_group"] in (1, 2, 4, 8)
    assert ms > 0
    for x, y in zip(before, (tr.G, tr.F, tr.W, tr.mF, tr.t, tr.step_ctr)):
        assert torch.equal(x, y)
    # the tuned step against the default one: the same losses, and gradients (Adam's first
    # moments, 0.1 g after one step) equal up to the order of the weight-gradient sums
    ref = _bricks_trainer(nb=2, n=20000)
    tr.step()
    ref.step()
    torch.cuda.synchronize()
    assert torch.allclose(tr.losses, ref.losses, rtol=1e-6, atol=0)
    for x, y in zip((tr.mF, tr.mW, tr.mG), (ref.mF, ref.mW, ref.mG)):
        err = ((x - y).norm() / y.norm()).item()
        assert err <= 1e-5, err
    # bitwise reproducible with the tuned shape
    again = _bricks_trainer(nb=2, n=20000, tuning=tune)
    again.step()
    torch.cuda.synchronize()
    for x, y in zip((tr.F, tr.W, tr.G, tr.mF), (again.F, again.W, again.G, again.mF)):
        assert torch.equal(x, y)


def test_bad_tuning_is_rejected_before_launch():
    tr = _bricks_trainer(nb=1, n=4000)
    tr.set_tuning({"cell_unroll": 3})
    with pytest.raises(A().ApmgError):
        tr.step()
    tr.set_tuning({"tile_blocks": 1 << 20})
    with pytest.raises(A().ApmgError):
        tr.step()
    tr.set_tuning({"cell_kernel": 3})
    with pytest.raises(A().ApmgError):
        tr.step()
    tr.set_tuning({"cell_group": 3})
    with pytest.raises(A().ApmgError):
        tr.step()
    tr.set_tuning(None)
    tr.step()


def test_both_gathers_give_the_same_step():
    # one training step with the wave-cooperative gather and with the one-thread-per-cell
    # gather (every batch size).  The grid gradient is the same terms summed in a different
    # fixed order, so the grids' first moments (0.1 * gradient) agree to float32 rounding;
    # the per-cell gather's batch size does not change its order (bitwise equal); the MLP
    # and the transforms do not depend on the gather.
    ref = _bricks_trainer(nb=2, n=6000, tuning={"cell_kernel": 1})
    F0 = ref.F.clone()
    ref.step()
    first = None
    for unroll in (2, 4, 8):
        other = _bricks_trainer(nb=2, n=6000, tuning={"cell_kernel": 2, "cell_unroll": unroll})
        other.step()
        torch.cuda.synchronize()
        for x, y in zip((ref.W, ref.G), (other.W, other.G)):
            assert torch.equal(x, y), unroll
        rel = ((ref.mF - other.mF).norm() / ref.mF.norm()).item()
        assert rel < 1e-6, (unroll, rel)
        dref, doth = ref.F - F0, other.F - F0
        assert ((dref - doth).norm() / dref.norm()).item() < 1e-3, unroll
        if first is None:
            first = other
        else:
            for x, y in zip((first.F, first.mF), (other.F, other.mF)):
                assert torch.equal(x, y), unroll


@pytest.mark.parametrize("group", [1, 2, 8])
def test_wave_gather_lane_groups_give_the_same_step(group):
    # the wave gather with 1, 2 or 8 lanes per run against the one-thread-per-cell gather: the
    # same terms in another fixed order
    ref = _bricks_trainer(nb=2, n=6000, tuning={"cell_kernel": 2})
    ref.step()
    other = _bricks_trainer(nb=2, n=6000, tuning={"cell_kernel": 1, "cell_group": group})
    other.step()
    torch.cuda.synchronize()
    for x, y in zip((ref.W, ref.G), (other.W, other.G)):
        assert torch.equal(x, y), group
    rel = ((ref.mF - other.mF).norm() / ref.mF.norm()).item()
    print(f"lanes per run {group}: first moment rel {rel:.2e}")
    assert rel < 1e-6, (group, rel)


def test_steps_from_two_host_threads_match_sequential_steps():
    # two trainers stepping at the same time from two host threads, each on its own stream:
    # the library's per-device side stream is forked and joined under a lock, so each
    # trainer's parameters equal those of the same steps run one trainer after the other
    import threading
    seq = [_bricks_trainer(nb=2, n=6000), _bricks_trainer(nb=1, n=5000)]
    for tr in seq:
        for _ in range(3):
            tr.step()
    torch.cuda.synchronize()
    par = [_bricks_trainer(nb=2, n=6000), _bricks_trainer(nb=1, n=5000)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for st in streams:
        st.wait_stream(torch.cuda.current_stream())
    errors = []

    def run(i):
        try:
            with torch.cuda.stream(streams[i]):
                for _ in range(3):
                    par[i].step()
            streams[i].synchronize()
        except Exception as e:  # surfaced in the main thread
            errors.append(e)

    threads = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for a, b in zip(seq, par):
        for x, y in zip((a.F, a.W, a.G, a.mF, a.losses), (b.F, b.W, b.G, b.mF, b.losses)):
            assert torch.equal(x, y)
