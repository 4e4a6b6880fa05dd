"""Pins of the oracle's training schedule (Sec. 4.3.2 delayed start and transform early stop,
Sec. 5.2 plateau scheduler) on short hand-worked loss sequences."""
import numpy as np

from oracle import apmg_oracle as O


def run(seq, total, **kw):
    st = O.control_initial(kw.get("delay", O.CONTROL_DEFAULTS["delay"]))
    hist = []
    for lr, ld in seq:
        st = O.control_update(st, lr, ld, total, **kw)
        hist.append(st)
    return hist


def test_delayed_start_trains_transforms_from_iteration_delay_plus_one():
    h = run([(1.0, 1.0)] * 6, total=100, delay=3, ma_window=100, patience=100)
    # flags are those of the next iteration: iterations 1..3 frozen transforms, 4.. trained
    assert [s["density_active"] for s in h] == [0, 0, 1, 1, 1, 1]
    # the paper's default: 500 iterations without transform updates
    h = run([(1.0, 1.0)] * 501, total=10000, patience=10000)
    assert h[498]["density_active"] == 0 and h[499]["density_active"] == 1


def test_early_stop_when_block_mean_does_not_drop_enough():
    # delay 0: density from iteration 1; blocks of 2 density iterations, 10% required drop
    seq = [(1.0, 10.0), (1.0, 10.0), (1.0, 9.5), (1.0, 9.5), (1.0, 1.0)]
    h = run(seq, total=100, delay=0, ma_window=2, ma_rel=0.1, patience=100)
    assert [s["density_active"] for s in h[:3]] == [1, 1, 1]
    assert h[1]["have_prev"] == 1 and h[1]["ma_prev"] == 10.0
    assert h[3]["density_done"] == 1 and h[3]["density_active"] == 0   # 9.5 is not below 9.0
    assert h[4]["density_active"] == 0 and h[4]["ma_count"] == 0      # stopped for good
    # a sufficient drop keeps training
    seq = [(1.0, 10.0), (1.0, 10.0), (1.0, 8.0), (1.0, 8.0)]
    h = run(seq, total=100, delay=0, ma_window=2, ma_rel=0.1, patience=100)
    assert h[3]["density_done"] == 0 and h[3]["density_active"] == 1 and h[3]["ma_prev"] == 8.0


def test_transform_training_ends_at_80_percent_of_the_run():
    h = run([(1.0, 1.0)] * 10, total=10, delay=0, ma_window=100, patience=100)
    # iterations 1..8 may train transforms (8 = 0.8 * 10), 9 and 10 may not
    assert [s["density_active"] for s in h] == [1] * 7 + [0] * 3


def test_plateau_scheduler_reduces_and_retires():
    seq = [(10.0, 0.0), (9.5, 0.0), (9.4, 0.0), (9.3, 0.0), (9.2, 0.0), (9.1, 0.0), (9.0, 0.0), (1.0, 0.0)]
    h = run(seq, total=1000, delay=1000, ma_window=10, patience=2, plateau_rel=0.1, plateau_factor=0.5,
            max_reductions=2)
    assert [s["bad"] for s in h[:4]] == [0, 1, 2, 0]
    assert h[3]["reductions"] == 1 and h[3]["lr_scale"] == np.float32(0.5)
    assert h[3]["frozen"] == 0
    assert h[6]["reductions"] == 2 and h[6]["frozen"] == 1 and h[6]["lr_scale"] == np.float32(0.25)
    assert h[7] == h[6]                                                  # retired: no change
    # an improvement beyond the threshold resets the count
    h = run([(10.0, 0.0), (9.5, 0.0), (8.0, 0.0)], total=1000, delay=1000, patience=2, plateau_rel=0.1)
    assert h[2]["bad"] == 0 and h[2]["best"] == 8.0


def test_plateau_factor_is_applied_in_float32():
    h = run([(1.0, 0.0)] * 8, total=1000, delay=1000, patience=1, plateau_rel=0.0, max_reductions=5)
    # constant loss, patience 1: reductions after iterations 3, 5 and 7
    f = np.float32(0.1)
    want = [np.float32(1), np.float32(1), f, f, f * f, f * f, (f * f) * f, (f * f) * f]
    assert [s["lr_scale"] for s in h] == want
    assert all(isinstance(s["lr_scale"], np.float32) for s in h)
