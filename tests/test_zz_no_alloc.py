"""The allocation-free forward entry point (apmg_forward_noalloc) against apmg_forward,
through the C ABI: two calls in a row, the second with fewer points, each equal to the
workspace entry point's output (bitwise: the same kernels and arithmetic per point); the
paper-order grids' copy and the 4x4 transforms' packing go through the static scratch too;
a model whose scratch exceeds the array is refused."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda"


def A():
    import paper_2308_02494_amd as mod
    return mod


def _pts(n, seed):
    x = synth.uniform_points_host(n, seed=seed)
    x[:4] = [[1.0, 1.0, 1.0], [-1.0, 0.5, 0.0], [np.nan, 0.0, 0.0], [1.5, 0.0, 0.0]]
    return torch.from_numpy(np.ascontiguousarray(x.T)).to(DEV)


@pytest.mark.parametrize("rows4,channel_last,bf16", [(False, False, False), (True, False, True), (False, True, False)])
def test_noalloc_forward_equals_workspace_forward_twice(rows4, channel_last, bf16):
    A_ = A()
    host = synth.init_model(32, 2, 32, [64, 64, 64, 1], seed=3, grid_range=0.5, extra_translation=0.1,
                            vmin=-1.0, vmax=2.0)
    model = A_.Model.from_host(host, DEV, mlp_dtype=A_.BF16 if bf16 else A_.F32)
    if rows4:
        G4 = torch.zeros((32, 4, 4), device=DEV)
        G4[:, :3, :] = model.G
        G4[:, 3, 3] = 1.0
        model = A_.Model(G4, model.F, model.W, model.vmin, model.vmax, model.mlp_dtype)
    if channel_last:
        model = A_.Model(model.G, A_.apmg_convert_grids(model.F, True), model.W, model.vmin, model.vmax,
                         model.mlp_dtype, layout=A_.GRIDS_MRRRC)
    for n, seed in ((70001, 1), (4099, 2)):          # the second call is smaller
        pts = _pts(n, seed)
        ref = A_.apmg_forward(model, pts)
        got = A_.apmg_forward_noalloc(model, pts)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (n, (got - ref).abs().max().item())
    assert A_._lib.apmg_forward_noalloc_scratch_bytes() == 16 << 20


def test_noalloc_forward_refuses_scratch_beyond_the_array():
    # paper-order grids of 64 x 4 x 64^3 float32 (256 MiB) would need a copy larger than the
    # 16 MiB scratch: refused before any launch; the same grids channel-last need no copy
    A_ = A()
    m = A_.ApmgModel()
    m.M, m.C, m.R, m.n_layers = 64, 4, 64, 3
    for k, w in enumerate([256, 128, 128, 1]):
        m.width[k] = w
    fake = ctypes.c_void_p(16)
    m.G, m.F = 16, 16
    for k in range(3):
        m.W[k] = 16
    rc = A_._lib.apmg_forward_noalloc(ctypes.byref(m), fake, 8, 8, fake, None)
    assert rc == A_.EWORKSPACE
    # invalid point counts are refused as invalid arguments before the scratch is sized or
    # touched (host-side checks; no launch)
    assert A_._lib.apmg_forward_noalloc(ctypes.byref(m), fake, 8, -1, fake, None) == A_.EINVAL
    assert A_._lib.apmg_forward_noalloc(ctypes.byref(m), fake, 4, 8, fake, None) == A_.EINVAL
