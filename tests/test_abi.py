"""CPU checks of the C ABI: the library loads, exports every declared entry
point, validates arguments before launching anything, sizes workspaces, and
its host-side brick partition equals the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2308_02494_amd as A
from oracle import apmg_oracle as O

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "apmg.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:apmg_status|size_t|const char\*)\s+(apmg_\w+)\s*\(", txt, re.M)))


def test_every_declared_symbol_is_exported_and_bound():
    names = _declared()
    assert len(names) >= 12
    lib = ctypes.CDLL(A.LIB_PATH)
    for nm in names:
        assert hasattr(lib, nm), nm
        assert nm in A.EXPORTS, nm


def _model(M=32, C=2, R=32, H=64, grid=A.F32, mlp=A.F32):
    m = A.ApmgModel()
    m.M, m.C, m.R, m.n_layers = M, C, R, 3
    for k, w in enumerate([M * C, H, H, 1]):
        m.width[k] = w
    m.grid_dtype, m.mlp_dtype = grid, mlp
    return m


def test_status_strings():
    assert A.status_string(A.OK) == "ok"
    assert "workspace" in A.status_string(A.EWORKSPACE)
    assert A.status_string(7) == "unknown status"


@pytest.mark.parametrize("op", [A.OP_FORWARD, A.OP_BACKWARD, A.OP_DENSITY])
def test_workspace_sizes(op):
    m = _model()
    a = A._lib.apmg_workspace_bytes(op, ctypes.byref(m), 1 << 10)
    b = A._lib.apmg_workspace_bytes(op, ctypes.byref(m), 1 << 20)
    assert a > 0 and b >= a
    assert A._lib.apmg_workspace_bytes(op, ctypes.byref(m), -1) == 0
    bad = _model()
    bad.width[0] = 63
    assert A._lib.apmg_workspace_bytes(op, ctypes.byref(bad), 16) == 0


def test_forward_argument_validation_needs_no_gpu():
    m = _model()
    f = A._lib.apmg_forward
    assert f(None, None, 0, 0, None, None, 0, None) == A.EINVAL
    # missing parameter pointers
    assert f(ctypes.byref(m), None, 0, 0, None, None, 0, None) == A.EINVAL
    fake = ctypes.c_void_p(0x1000)
    m.G = m.F = 0x1000
    for k in range(3):
        m.W[k] = 0x1000
    assert f(ctypes.byref(m), fake, 4, 8, fake, fake, 1 << 30, None) == A.EINVAL   # ld < n
    assert f(ctypes.byref(m), fake, 8, -1, fake, fake, 1 << 30, None) == A.EINVAL  # n < 0
    assert f(ctypes.byref(m), fake, 8, 8, fake, fake, 16, None) == A.EWORKSPACE
    # the allocation-free variant checks the same arguments before sizing its scratch
    g = A._lib.apmg_forward_noalloc
    assert g(None, None, 0, 0, None, None) == A.EINVAL
    assert g(ctypes.byref(m), fake, 4, 8, fake, None) == A.EINVAL                   # ld < n
    assert g(ctypes.byref(m), fake, 8, -1, fake, None) == A.EINVAL                  # n < 0
    for field, val in [("C", 3), ("R", 1)]:
        bad = _model()
        setattr(bad, field, val)
        bad.width[0] = bad.M * bad.C
        bad.G = bad.F = 0x1000
        for k in range(3):
            bad.W[k] = 0x1000
        rc = f(ctypes.byref(bad), fake, 8, 8, fake, fake, 1 << 30, None)
        assert rc in (A.EINVAL, A.EUNSUPPORTED)
    unsup = _model(H=96)
    unsup.G = unsup.F = 0x1000
    for k in range(3):
        unsup.W[k] = 0x1000
    assert f(ctypes.byref(unsup), fake, 8, 8, fake, fake, 1 << 30, None) == A.EUNSUPPORTED
    big = _model(M=129, C=2)
    big.G = big.F = 0x1000
    for k in range(3):
        big.W[k] = 0x1000
    assert f(ctypes.byref(big), fake, 8, 8, fake, fake, 1 << 30, None) == A.EUNSUPPORTED


def test_backward_and_density_validation():
    m = _model()
    m.G = m.F = 0x1000
    for k in range(3):
        m.W[k] = 0x1000
    fake = ctypes.c_void_p(0x1000)
    assert A._lib.apmg_backward(ctypes.byref(m), fake, 8, 8, None, None, None, None, 0, fake, 1 << 30,
                                None) == A.EINVAL  # df missing
    assert A._lib.apmg_density_loss(ctypes.byref(m), fake, 8, 8, fake, 1e-12, 0, fake, None, None, 0, fake,
                                    1 << 30, None) == A.EINVAL  # p < 1
    assert A._lib.apmg_density_loss(ctypes.byref(m), fake, 8, 8, fake, -1.0, 10, fake, None, None, 0, fake,
                                    1 << 30, None) == A.EINVAL  # eps < 0
    assert A._lib.apmg_density_loss(ctypes.byref(m), fake, 8, 8, fake, 1e-12, 10, fake, None, None, 0, fake,
                                    16, None) == A.EWORKSPACE
    assert A._lib.apmg_batched_step(None, None, 0, None) == A.EINVAL
    assert A._lib.apmg_uniform_points(1, 0, 0, 0, -1, None, 0, None) == A.EINVAL
    assert A._lib.apmg_gt_sample(None, 4, 4, 4, None, 0, 0, None, None) == A.EINVAL
    assert A._lib.apmg_convert_grids(0, 1, 2, fake, 0, fake, 0, 1, None) == A.EINVAL


def test_zero_points_is_ok_without_launch():
    m = _model()
    m.G = m.F = 0x1000
    for k in range(3):
        m.W[k] = 0x1000
    ws = A._lib.apmg_workspace_bytes(A.OP_FORWARD, ctypes.byref(m), 0)
    assert A._lib.apmg_forward(ctypes.byref(m), None, 0, 0, None, ctypes.c_void_p(0x1000), ws, None) == A.OK
    assert A._lib.apmg_uniform_points(1, 0, 0, 0, 0, None, 0, None) == A.OK


@pytest.mark.parametrize("shape,B,g", [((1000, 1200, 900), 256, 1), ((1024, 1024, 1024), 256, 16),
                                       ((33, 17, 65), 16, 2), ((5, 5, 5), 8, 0)])
def test_make_bricks_equals_oracle_partition(shape, B, g):
    t, bricks = A.apmg_make_bricks(*shape, B, g)
    dims, ob = O.brick_partition(shape, B, g)
    assert tuple(t.dims) == dims and len(bricks) == len(ob)
    for b, o in zip(bricks, ob):
        assert tuple(b.ijk) == o["ijk"]
        assert list(b.e0) == o["e0"] and list(b.e1) == o["e1"]


def test_make_bricks_rejects_bad_arguments():
    t = A.ApmgBrickTable()
    assert A._lib.apmg_make_bricks(0, 4, 4, 2, 0, ctypes.byref(t), None, 0) == A.EINVAL
    assert A._lib.apmg_make_bricks(8, 8, 8, 0, 0, ctypes.byref(t), None, 0) == A.EINVAL
    assert A._lib.apmg_make_bricks(8, 8, 8, 2, -1, ctypes.byref(t), None, 0) == A.EINVAL
    arr = (A.ApmgBrick * 3)()
    assert A._lib.apmg_make_bricks(8, 8, 8, 2, 0, ctypes.byref(t), arr, 3) == A.EINVAL  # 64 bricks > cap


_LAYOUT_SRC = r"""
#include <cstdio>
#include <cstddef>
#include "apmg.h"
#define F(T, f) std::printf(#T " " #f " %zu\n", offsetof(T, f));
#define S(T) std::printf(#T " sizeof %zu\n", sizeof(T));
int main() {
  S(apmg_model) F(apmg_model, width) F(apmg_model, G) F(apmg_model, F) F(apmg_model, W) F(apmg_model, vmin)
  S(apmg_brick) F(apmg_brick, e1) F(apmg_brick, vmax)
  S(apmg_brick_table) F(apmg_brick_table, ghost)
  S(apmg_tuning) F(apmg_tuning, cell_unroll) F(apmg_tuning, cell_group)
  S(apmg_batch) F(apmg_batch, shape) F(apmg_batch, G) F(apmg_batch, density_active) F(apmg_batch, vol)
  F(apmg_batch, n) F(apmg_batch, step) F(apmg_batch, lr) F(apmg_batch, eps_density) F(apmg_batch, losses)
  F(apmg_batch, tuning) F(apmg_batch, frozen) F(apmg_batch, lr_scale)
  S(apmg_ctl_state) F(apmg_ctl_state, ma_sum) F(apmg_ctl_state, best)
  S(apmg_control) F(apmg_control, stop_frac) F(apmg_control, ma_rel) F(apmg_control, state)
  F(apmg_control, lr_scale)
  S(apmg_dd_models) F(apmg_dd_models, shape) F(apmg_dd_models, G) F(apmg_dd_models, bricks)
  return 0;
}
"""


def test_struct_layouts_match_the_header(tmp_path):
    """Every ctypes mirror has the size and field offsets the C compiler gives the header."""
    import shutil
    import subprocess
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    src = tmp_path / "layout.cpp"
    src.write_text(_LAYOUT_SRC)
    exe = tmp_path / "layout"
    inc = os.path.dirname(HEADER)
    r = subprocess.run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", f"-I{inc}", "-I/opt/rocm/include",
                        str(src), "-o", str(exe)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("header does not compile with the host compiler here: " + r.stderr[:200])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    mirrors = {"apmg_model": A.ApmgModel, "apmg_brick": A.ApmgBrick, "apmg_brick_table": A.ApmgBrickTable,
               "apmg_tuning": A.ApmgTuning, "apmg_batch": A.ApmgBatch, "apmg_ctl_state": A.ApmgCtlState,
               "apmg_control": A.ApmgControl, "apmg_dd_models": A.ApmgDdModels}
    checked = 0
    for line in out:
        if not line.strip():
            continue
        st, field, val = line.split()
        py = mirrors[st]
        got = ctypes.sizeof(py) if field == "sizeof" else getattr(py, field).offset
        assert got == int(val), (st, field, got, val)
        checked += 1
    assert checked >= 25


def test_new_entry_points_validate_without_gpu():
    b = A.ApmgBatch()
    t = A.ApmgTuning()
    ms = ctypes.c_float()
    # a batch with nb = 0 is rejected before anything is launched
    assert A._lib.apmg_autotune_batched_step(ctypes.byref(b), None, 0, None, ctypes.byref(t),
                                             ctypes.byref(ms)) == A.EINVAL
    assert A._lib.apmg_autotune_batched_step(None, None, 0, None, ctypes.byref(t), ctypes.byref(ms)) == A.EINVAL
    c = A.ApmgControl()
    assert A._lib.apmg_train_control(None, None, None) == A.EINVAL
    assert A._lib.apmg_train_control(ctypes.byref(c), None, None) == A.EINVAL
    c.nb = 1
    assert A._lib.apmg_train_control(ctypes.byref(c), 1, None) == A.EINVAL   # NULL state arrays


def test_batched_step_rejects_adam_settings_outside_their_range():
    # beta in [0, 1) (1 - beta^t divides the moments), adam_eps and the rates >= 0: checked on
    # the host before the workspace; with valid settings the missing workspace is reported
    b = A.ApmgBatch()
    b.nb, b.n = 1, 8
    s = b.shape
    s.M, s.C, s.R, s.n_layers = 8, 2, 8, 3
    for k, w in enumerate([16, 64, 64, 1]):
        s.width[k] = w
    s.grid_dtype, s.mlp_dtype = A.F32, A.F32
    for f in ("G", "F", "W", "mG", "vG", "mF", "vF", "mW", "vW", "t", "tG", "density_active", "volume",
              "bricks", "step", "losses"):
        setattr(b, f, 0x1000)
    b.vol[0], b.vol[1], b.vol[2] = 8, 8, 8
    b.p, b.eps_density = 10, 1e-12

    def rc(**kw):
        b.lr, b.lr_G, b.beta1, b.beta2, b.adam_eps = 0.01, 0.001, 0.9, 0.99, 1e-8
        for k, v in kw.items():
            setattr(b, k, v)
        return A._lib.apmg_batched_step(ctypes.byref(b), None, 0, None)

    assert rc() == A.EWORKSPACE
    for bad in ({"beta1": 1.0}, {"beta2": 1.5}, {"beta1": -0.1}, {"beta2": float("nan")},
                {"adam_eps": -1e-8}, {"lr": -0.01}, {"lr_G": float("nan")}):
        assert rc(**bad) == A.EINVAL, bad
