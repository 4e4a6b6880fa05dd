"""Training-step throughput of the APMGSRN hot path on one MI355X.

Workload (one model, "plain FP32 training step at paper-like scale"): a
256^3 float32 synthetic volume (64 Gaussian blobs of widths 0.01-0.1 plus a
turbulent patch on 5% of the domain), G = 32 grids at 32^3 with F = 2
features, MLP 64-64-64-1, 2^20 uniform points per step.  A step is the whole
hot path: point generation, ground-truth sampling, forward, L_rec and its
adjoint, the density loss (both passes) and its transform gradient, and Adam.

Prints one JSON line: train points/s of the fp32 step (value), plus the
roofline of the dominant kernel (the fused forward+adjoint tile kernel),
the FP64 oracle timed on a sample on the host, and extra figures
(inference points/s, the bf16-MLP step).
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0

COPY_PROBE_BYTES = 1 << 30

M, C, R, H = 32, 2, 32, 64
VOL = (256, 256, 256)
N = 1 << 20


def mlp_flops_fwd_bwd(K, Hd):
    """Algorithmic MLP flop per point of one forward + adjoint: forward
    2(KH + H^2 + H); adjoint dW1, dW2, dW3 (2KH + 2H^2 + 2H) and dL/dh1,
    dL/dy (2H^2 + 2KH)."""
    fwd = 2 * (K * Hd + Hd * Hd + Hd)
    bwd = 2 * (K * Hd + Hd * Hd + Hd) + 2 * (Hd * Hd + K * Hd)
    return fwd + bwd


COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_adjoint_train_c2_fp32_counters.txt")

# the sources the adjoint tile kernel is compiled from: its own file (with its launcher), the
# forward tile it recomputes and the shared device helpers
ADJOINT_SOURCES = ["apmg_adjoint.hip", "apmg_mlp.hip", "apmg_device.h", "apmg_kernels.h"]


def source_hash():
    """sha256 over the adjoint tile kernel's sources (path and content, in order)."""
    import hashlib
    h = hashlib.sha256()
    cdir = os.path.join("paper_2308_02494_amd", "csrc")
    files = [os.path.join(cdir, f) for f in ADJOINT_SOURCES]
    for rel in files:
        h.update(rel.encode() + b"\0")
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed FETCH_SIZE / WRITE_SIZE
    counter summary, each scaled by what the counter reads for a plain copy of known size;
    None when the summary is missing or was taken on other kernel sources."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    kv = {}
    with open(COUNTERS_FILE) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_hash():
        return None
    cb = float(kv["copy_bytes"])
    fetch = float(kv["fetch_kib_per_dispatch"]) * 1024 * cb / (float(kv["copy_fetch_kib"]) * 1024)
    write = float(kv["write_kib_per_dispatch"]) * 1024 * cb / (float(kv["copy_write_kib"]) * 1024)
    return fetch + write


def progress(msg):
    """A line on stderr after each finished phase (the JSON line stays alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def hip():
    lib = ctypes.CDLL("libamdhip64.so")
    lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
    lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
    return lib


def make_trainer(A, torch, synth, mlp_dtype, n):
    vol = synth.make_volume("blobs_turb", VOL, device="cuda")
    nz, ny, nx = vol.shape
    _, bricks = A.apmg_make_bricks(nx, ny, nz, max(nx, ny, nz), 0)
    host = synth.init_model(M, C, R, [M * C, H, H, 1], seed=synth.SEED_MODEL)
    tr = A.Trainer([host], vol, bricks, n, seed=synth.SEED_POINTS, mlp_dtype=mlp_dtype)
    tr.density_active.fill_(1)
    return tr, vol, host


def time_steps(A, torch, tr, steps, warmup, hl):
    """Whole-step wall time of `steps` steps, and the mean launch time (ms) of the adjoint
    tile kernel and of the grid-gradient gather, from HIP events the library records on the
    stream each is launched on."""
    for _ in range(warmup):
        tr.step()
    torch.cuda.synchronize()
    evs = []
    for _ in range(steps):
        pair = []
        for _k in range(2):
            a, b = ctypes.c_void_p(), ctypes.c_void_p()
            hl.hipEventCreate(ctypes.byref(a))
            hl.hipEventCreate(ctypes.byref(b))
            pair.append((a, b))
        evs.append(pair)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pair in evs:
        A.apmg_profile_kernel_events(A.PROF_ADJOINT, *pair[0])
        A.apmg_profile_kernel_events(A.PROF_GATHER, *pair[1])
        tr.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ks = [[], []]
    for pair in evs:
        for k, (a, b) in enumerate(pair):
            ms = ctypes.c_float()
            hl.hipEventElapsedTime(ctypes.byref(ms), a, b)
            ks[k].append(ms.value)
            hl.hipEventDestroy(a)
            hl.hipEventDestroy(b)
    return dt, sum(ks[0]) / len(ks[0]), sum(ks[1]) / len(ks[1])


def gather_bytes(n, Mg, Cg, Rg):
    """Algorithmic HBM bytes of one grid-gradient gather: dL/dy of every (point, grid) pair
    (4C bytes), each point once (a 16-byte record), and the gradient of every grid value."""
    return n * Mg * Cg * 4 + n * 16 + Mg * Rg ** 3 * Cg * 4


def time_forward(A, torch, host, n, reps=10):
    model = A.Model.from_host(host, "cuda")
    pts = A.apmg_uniform_points(11, 0, 0, 0, n)
    ws = torch.empty(A._lib.apmg_workspace_bytes(A.OP_FORWARD, ctypes.byref(model.struct()), n),
                     dtype=torch.uint8, device="cuda")
    out = torch.empty(n, device="cuda")
    for _ in range(3):
        A.apmg_forward(model, pts, out=out, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        A.apmg_forward(model, pts, out=out, ws=ws)
    torch.cuda.synchronize()
    return n * reps / (time.perf_counter() - t0)


def _time_trainer(torch, tr, steps, warmup):
    for _ in range(warmup):
        tr.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tr.step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def time_graph(torch, tr, reps):
    """One training step captured as a HIP graph (after an eager step) and replayed: ms per step."""
    tr.step()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tr.step()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3


def extra_c1(A, torch, synth, hl):
    """64^3 blobs+sine volume, 16 grids at 16^3 x 2, MLP 32-64-64-1, 65,536 points, fp32."""
    vol = synth.make_volume("blobs_sine", (64, 64, 64), device="cuda")
    _, bricks = A.apmg_make_bricks(64, 64, 64, 64, 0)
    host = synth.init_model(16, 2, 16, [32, 64, 64, 1], seed=synth.SEED_MODEL)
    tr = A.Trainer([host], vol, bricks, 65536, seed=synth.SEED_POINTS)
    tr.density_active.fill_(1)
    dt = _time_trainer(torch, tr, 20, 5)
    return {"train_pts_per_s": 65536 / dt, "ms_per_step": dt * 1e3}


def extra_c3(A, torch, synth, hl):
    """1024^3 volume, the 32-grid model with bf16 MLP and fp16 grids, 2^21 points."""
    vol = synth.make_volume("blobs_turb", (1024, 1024, 1024), device="cuda")
    _, bricks = A.apmg_make_bricks(1024, 1024, 1024, 1024, 0)
    host = synth.init_model(M, C, R, [M * C, H, H, 1], seed=synth.SEED_MODEL)
    n = 1 << 21
    tr = A.Trainer([host], vol, bricks, n, seed=synth.SEED_POINTS, mlp_dtype=A.BF16, grid_dtype=torch.float16)
    tr.density_active.fill_(1)
    dt = _time_trainer(torch, tr, 10, 3)
    return {"train_pts_per_s": n / dt, "ms_per_step": dt * 1e3, "mlp": "bf16", "grids": "fp16 (fp32 master)"}


def extra_c4(A, torch, synth, hl, B=256):
    """1000x1200x900 volume in B^3 bricks with one ghost voxel (B = 256: 4 x 5 x 4 = 80 bricks;
    B = 300: 4 x 4 x 3 = 48 bricks, the workload's stated model count), 16 grids at 32^3 x 2
    per brick, MLP 32-64-64-1 in bf16, 2^17 points per brick; all bricks per step, launch
    shapes from the autotuner, the step captured as a graph and replayed.  Then global-query
    inference over all brick models: 2^24 uniform points."""
    vol = synth.make_volume("blobs_turb", (900, 1200, 1000), device="cuda")
    table, bricks = A.apmg_make_bricks(1000, 1200, 900, B, 1)
    hosts = [synth.init_model(16, 2, 32, [32, 64, 64, 1], seed=synth.SEED_MODEL + b) for b in range(len(bricks))]
    n = 1 << 17
    tr = A.Trainer(hosts, vol, bricks, n, seed=synth.SEED_POINTS, mlp_dtype=A.BF16)
    tr.density_active.fill_(1)
    dt_eager = _time_trainer(torch, tr, 3, 1)
    tune, _ = tr.autotune()
    dt = time_graph(torch, tr, 5) * 1e-3
    out = {"bricks": len(bricks), "train_pts_per_s": len(bricks) * n / dt, "ms_per_step": dt * 1e3,
           "ms_per_step_eager_default_shapes": dt_eager * 1e3, "tuning": tune, "graph": True}
    dd = A.DDModels.from_trainer(tr, table, bricks)
    m = 1 << 24
    pts = A.apmg_uniform_points(99, 0, 0, 0, m)
    ws = torch.empty(A._lib.apmg_workspace_bytes(A.OP_DD_FORWARD, ctypes.byref(dd.struct), m), dtype=torch.uint8,
                     device="cuda")
    f = torch.empty(m, device="cuda")
    A.apmg_dd_forward(dd, pts, out=f, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        A.apmg_dd_forward(dd, pts, out=f, ws=ws)
    torch.cuda.synchronize()
    out["dd_infer_pts_per_s"] = 3 * m / (time.perf_counter() - t0)
    return out


def extra_c5(A, torch, synth, hl):
    """64 grids at 64^3 x 4 features, MLP 256-128-128-1 in bf16, a 1920x1080 ray layout
    with 8 samples per ray (16,588,800 points), forward only."""
    host = synth.init_model(64, 4, 64, [256, 128, 128, 1], seed=5, grid_range=1.0, extra_translation=0.3)
    model = A.Model.from_host(host, "cuda", mlp_dtype=A.BF16)
    pts = torch.from_numpy(synth.ray_points().T.copy()).cuda()
    n = pts.shape[1]
    ws = torch.empty(A._lib.apmg_workspace_bytes(A.OP_FORWARD, ctypes.byref(model.struct()), n),
                     dtype=torch.uint8, device="cuda")
    out_f = torch.empty(n, device="cuda")
    A.apmg_forward(model, pts, out=out_f, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        A.apmg_forward(model, pts, out=out_f, ws=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    fl = 2 * (256 * 128 + 128 * 128 + 128) * n
    out = {"infer_pts_per_s": n / dt, "ms_per_frame": dt * 1e3, "points": n,
           "bf16_mfma_frac_forward": fl / dt / 1e12 / PEAK_BF16_MFMA_TFLOPS,
           "logical_gather_TBps": n * 64 * 8 * 4 * 4 / dt / 1e12}
    # the same frame with the grids stored in fp16 (128 MiB instead of 256 MiB)
    model16 = A.Model.from_host(host, "cuda", grid_dtype=torch.float16, mlp_dtype=A.BF16)
    ws16 = torch.empty(A._lib.apmg_workspace_bytes(A.OP_FORWARD, ctypes.byref(model16.struct()), n),
                       dtype=torch.uint8, device="cuda")
    A.apmg_forward(model16, pts, out=out_f, ws=ws16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        A.apmg_forward(model16, pts, out=out_f, ws=ws16)
    torch.cuda.synchronize()
    dt16 = (time.perf_counter() - t0) / reps
    out["fp16_grids"] = {"infer_pts_per_s": n / dt16, "ms_per_frame": dt16 * 1e3,
                         "bf16_mfma_frac_forward": fl / dt16 / 1e12 / PEAK_BF16_MFMA_TFLOPS}
    del model16, ws16
    # the 2^20-point adjoint of the same model (dF, dG, dW), bf16 MLP
    nb_ = 1 << 20
    bp = A.apmg_uniform_points(13, 0, 0, 0, nb_)
    dfb = torch.full((nb_,), 1.0 / nb_, device="cuda")
    A.apmg_backward(model, bp, dfb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        A.apmg_backward(model, bp, dfb)
    torch.cuda.synchronize()
    out["backward_pts_per_s"] = 3 * nb_ / (time.perf_counter() - t0)
    return out


def extra_f4(A, torch, synth, hl, n=1 << 20, reps=5):
    """Sec. 9 encoder variants with the FP32 MLP 64-64-64-1 on 2^20 uniform points: (1) a hash
    grid inside each of 8 adaptive grids (4 levels at 16, 32, 64, 128 cells per axis, 2^16
    entries of 2 features per level, U(-1e-4, 1e-4) entries: 64 features); (2) 4-D grids,
    32 grids at 32^3 x 8 time vertices x 2 features, uniform times.  Forward and
    forward + adjoint (table / grid, transform and MLP gradients) points/s."""
    import numpy as np
    rng = np.random.default_rng(41)

    def glorot(i, o):
        lim = np.sqrt(6.0 / (i + o))
        return torch.from_numpy(rng.uniform(-lim, lim, size=(o, i)).astype(np.float32)).cuda()

    def run(model, pts):
        df = torch.full((n,), 1.0 / n, device="cuda")
        m, e = model.structs()
        wsf = A._variant_ws(A.OP_FORWARD, m, e, n, "cuda")
        wsb = A._variant_ws(A.OP_BACKWARD, m, e, n, "cuda")
        f = torch.empty(n, device="cuda")
        A.apmg_variant_forward(model, pts, out=f, ws=wsf)
        A.apmg_variant_backward(model, pts, df, ws=wsb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            A.apmg_variant_forward(model, pts, out=f, ws=wsf)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            A.apmg_variant_backward(model, pts, df, ws=wsb)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return {"infer_pts_per_s": n * reps / (t1 - t0), "ms_forward": (t1 - t0) / reps * 1e3,
                "fwd_bwd_pts_per_s": n * reps / (t2 - t1), "ms_forward_adjoint": (t2 - t1) / reps * 1e3}

    out = {}
    M, L, T = 8, 4, 1 << 16
    G = torch.from_numpy(synth.init_model(M, 2, 4, [2 * M, 64, 64, 1], seed=43)["G"]).cuda()
    Th = torch.from_numpy(rng.uniform(-1e-4, 1e-4, size=(M, L, T, 2)).astype(np.float32)).cuda()
    hm = A.VariantModel(A.ENC_HASH, G, Th, [glorot(M * L * 2, 64), glorot(64, 64), glorot(64, 1)],
                        level_res=[16, 32, 64, 128])
    pts = A.apmg_uniform_points(45, 0, 0, 0, n)
    out["hash_8x4_levels"] = run(hm, pts)
    del hm, Th
    M, R, Rt = 32, 32, 8
    G = torch.from_numpy(synth.init_model(M, 2, R, [2 * M, 64, 64, 1], seed=47)["G"]).cuda()
    F4 = torch.from_numpy(rng.uniform(-1e-4, 1e-4, size=(M, 2, Rt, R, R, R)).astype(np.float32)).cuda()
    tm = A.VariantModel(A.ENC_TIME, G, F4, [glorot(M * 2, 64), glorot(64, 64), glorot(64, 1)])
    pts4 = torch.cat([pts, torch.from_numpy(rng.uniform(-1, 1, size=(1, n)).astype(np.float32)).cuda()], 0)
    out["time_32x32cubed_x8"] = run(tm, pts4.contiguous())
    return out


def _oracle_chunk(args):
    """One FP64 oracle training step on a chunk of the sample (a worker of the CPU baseline)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import apmg_oracle as O
    host, vol_path, shape, start, count = args
    vol_np = np.memmap(vol_path, dtype=np.float64, mode="r", shape=shape)
    model = {"G": host["G"].astype(np.float64), "F": host["F"].astype(np.float64),
             "W": [w.astype(np.float64) for w in host["W"]], "vmin": 0.0, "vmax": 1.0}
    brick = {"e0": [0, 0, 0], "e1": [shape[2] - 1, shape[1] - 1, shape[0] - 1]}
    with threadpool_limits(limits=1):
        x = O.uniform_points(7, 0, 0, count, start=start)
        v = O.brick_gt_sample(vol_np, brick, x)
        O.train_step(model, O.zero_adam_state(model), x, v, density_active=True)
    return count


def cpu_baseline(vol_np, host, n_sample):
    """The FP64 oracle's training step on a bounded sample of the same workload, on the host's
    cores: the sample is split into one chunk per worker process (threads pinned to one per
    worker), each chunk a training step of its own -- the same per-point work (points, ground
    truth, forward, adjoint, density passes, Adam) as one step over the whole sample."""
    import multiprocessing as mp
    import tempfile

    import numpy as np
    cores = min(len(os.sched_getaffinity(0)), 16)
    chunk = (n_sample + cores - 1) // cores
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "volume.f64")
        mm = np.memmap(path, dtype=np.float64, mode="w+", shape=vol_np.shape)
        mm[:] = vol_np
        mm.flush()
        jobs = [(host, path, vol_np.shape, k * chunk, min(chunk, n_sample - k * chunk)) for k in range(cores)
                if k * chunk < n_sample]
        ctx = mp.get_context("spawn")
        with ctx.Pool(len(jobs)) as pool:
            pool.map(_oracle_chunk, [(host, path, vol_np.shape, 0, 8)] * len(jobs))   # workers up, imports done
            t0 = time.perf_counter()
            done = sum(pool.map(_oracle_chunk, jobs))
            dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "train pts/s", "cores": len(jobs), "kind": "oracle",
            "sample": f"FP64 oracle training steps (points, ground truth, forward, adjoint, density, Adam) on "
                      f"{done} of the {N} points of the headline step, same model and volume, split into "
                      f"{len(jobs)} chunks over {len(jobs)} worker processes (one thread each), {dt:.1f} s"}


def stated_errors(A, torch, synth, vol, host, n):
    """Error of one GPU training step (FP32, BF16 MLP, BF16 MLP + FP16 grids) against the FP64
    oracle's step on the same n points of the headline workload (step 0), and of one brick
    model's BF16 step of the brick workload, normwise relative: losses, and the gradients read
    off the first Adam moments (m = 0.1 g)."""
    import numpy as np

    from oracle import apmg_oracle as O
    model = {"G": host["G"].astype(np.float64), "F": host["F"].astype(np.float64),
             "W": [w.astype(np.float64) for w in host["W"]], "vmin": 0.0, "vmax": 1.0}
    vol_np = vol.cpu().numpy().astype(np.float64)
    brick = {"e0": [0, 0, 0], "e1": [VOL[2] - 1, VOL[1] - 1, VOL[0] - 1]}
    x = O.uniform_points(synth.SEED_POINTS, 0, 0, n)
    v = O.brick_gt_sample(vol_np, brick, x)
    _, st, info = O.train_step(model, O.zero_adam_state(model), x, v, density_active=True)

    def rel(a, b):
        a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    out = {"points": n}
    for name, mlp, gd in (("fp32", A.F32, torch.float32), ("bf16_mlp", A.BF16, torch.float32),
                          ("bf16_mlp_fp16_grids", A.BF16, torch.float16)):
        nz, ny, nx = vol.shape
        _, bricks = A.apmg_make_bricks(nx, ny, nz, max(nx, ny, nz), 0)
        tr = A.Trainer([host], vol, bricks, n, seed=synth.SEED_POINTS, mlp_dtype=mlp, grid_dtype=gd)
        tr.density_active.fill_(1)
        tr.step()
        torch.cuda.synchronize()
        L = tr.losses[0].cpu().numpy()
        mW = tr.mW[0].cpu().numpy().astype(np.float64)
        wflat = np.concatenate([w.ravel() for w in info["dW"]])
        out[name] = {"L_rec": rel([L[0]], [info["L_rec"]]), "L_density": rel([L[1]], [info["L_density"]]),
                     "dF": rel(tr.mF[0].cpu().numpy() / 0.1, info["dF"]), "dW": rel(mW / 0.1, wflat),
                     "dG_density": rel(tr.mG[0].cpu().numpy() / 0.1, info["dG_density"])}
        del tr
    # one brick model of the 80-brick workload (brick 21 of the 1000x1200x900 volume in 256^3
    # bricks, 16 grids at 32^3 x 2, MLP 32-64-64-1 in BF16), the same number of points
    del vol
    torch.cuda.empty_cache()
    vol4 = synth.make_volume("blobs_turb", (900, 1200, 1000), device="cuda")
    _, bricks = A.apmg_make_bricks(1000, 1200, 900, 256, 1)
    k = 21
    bk = bricks[k]
    e0, e1 = list(bk.e0), list(bk.e1)
    sub = vol4[e0[2]:e1[2] + 1, e0[1]:e1[1] + 1, e0[0]:e1[0] + 1].cpu().numpy().astype(np.float64)
    host4 = synth.init_model(16, 2, 32, [32, 64, 64, 1], seed=synth.SEED_MODEL + k)
    tr = A.Trainer([host4], vol4, [bk], n, seed=synth.SEED_POINTS, mlp_dtype=A.BF16)
    tr.density_active.fill_(1)
    tr.step()
    torch.cuda.synchronize()
    m4 = {"G": host4["G"].astype(np.float64), "F": host4["F"].astype(np.float64),
          "W": [w.astype(np.float64) for w in host4["W"]], "vmin": float(bk.vmin), "vmax": float(bk.vmax)}
    x4 = O.uniform_points(synth.SEED_POINTS, 0, 0, n)
    v4 = O.brick_gt_sample(sub, {"e0": [0, 0, 0], "e1": [e1[0] - e0[0], e1[1] - e0[1], e1[2] - e0[2]]}, x4)
    _, _, info4 = O.train_step(m4, O.zero_adam_state(m4), x4, v4, density_active=True)
    L = tr.losses[0].cpu().numpy()
    w4 = np.concatenate([w.ravel() for w in info4["dW"]])
    out["config4_brick_bf16_mlp"] = {
        "L_rec": rel([L[0]], [info4["L_rec"]]), "L_density": rel([L[1]], [info4["L_density"]]),
        "dF": rel(tr.mF[0].cpu().numpy() / 0.1, info4["dF"]),
        "dW": rel(tr.mW[0].cpu().numpy().astype(np.float64) / 0.1, w4),
        "dG_density": rel(tr.mG[0].cpu().numpy() / 0.1, info4["dG_density"])}
    del tr, vol4
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 19)
    ap.add_argument("--error-sample", type=int, default=1 << 17,
                    help="points of the GPU steps compared with the oracle for the stated errors")
    ap.add_argument("--skip-extra", action="store_true")
    ap.add_argument("--configs", default="config1,config3,config4,config5,f4",
                    help="extra workloads to time after the headline")
    ap.add_argument("--only", choices=["bf16", "config1", "config3", "config4", "config4_48", "config5", "f4"],
                    help="time one extra workload alone (no headline line; for profiling runs)")
    ap.add_argument("--source-hash", action="store_true",
                    help="print the hash of the adjoint kernel's sources and exit")
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with a plain 1 GiB device-to-device copy (the reference kernel that "
                         "calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.source_hash:
        print(source_hash())
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path is one GPU's "
              f"share; see the sharding notes in the design document)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2308_02494_amd as A
    import synth

    hl = hip()
    if args.only:
        if args.only == "bf16":
            trb, _, _ = make_trainer(A, torch, synth, A.BF16, N)
            dtb, kb, gbm = time_steps(A, torch, trb, args.steps, args.warmup, hl)
            res = {"train_pts_per_s": N * args.steps / dtb, "ms_per_step": dtb * 1e3 / args.steps,
                   "kernel_ms": kb, "gather_ms": gbm}
        else:
            fn = {"config1": extra_c1, "config3": extra_c3, "config4": extra_c4, "config5": extra_c5, "f4": extra_f4,
                  "config4_48": lambda A_, t_, s_, h_: extra_c4(A_, t_, s_, h_, B=300)}[args.only]
            res = fn(A, torch, synth, hl)
        print(json.dumps({"only": args.only, "result": res}), flush=True)
        return
    tr, vol, host = make_trainer(A, torch, synth, A.F32, N)
    dt, kern_ms, gather_ms = time_steps(A, torch, tr, args.steps, args.warmup, hl)
    ms_step = dt * 1e3 / args.steps
    progress(f"headline: {ms_step:.3f} ms per step")
    value = N * args.steps / dt
    flops = mlp_flops_fwd_bwd(M * C, H) * N
    achieved = flops / (kern_ms * 1e-3) / 1e12
    out = {
        "metric": "train pts/s (fwd+bwd), 32-grid APMGSRN, FP32",
        "value": value, "unit": "pts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded closed-form volume, paper initialisation)",
        "config": {"workload": "single-model training step: 256^3 blobs+turbulence volume, 32 grids "
                               "at 32^3 x 2 features, MLP 64-64-64-1, 2^20 points, density phase on",
                   "global_batch": N, "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA_TFLOPS, "traffic": measured_traffic(),
                     "kernel": "k_adjoint (fused forward + adjoint tile kernel, eight waves per block)",
                     "kernel_ms": kern_ms},
    }
    gb = gather_bytes(N, M, C, R)
    out["gather_roofline"] = {"bound": "hbm", "achieved": gb / (gather_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                              "unit": "GB/s", "frac": gb / (gather_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                              "kernel": "k_cell_pull_wave (grid-gradient gather)", "kernel_ms": gather_ms,
                              "algorithmic_bytes": gb}
    L = tr.losses.cpu().numpy()
    out["losses_last_step"] = {"L_rec": float(L[0, 0]), "L_density": float(L[0, 1])}
    if not args.skip_extra:
        extra = {}
        extra["infer_pts_per_s_fp32"] = time_forward(A, torch, host, N)
        progress("fp32 inference done")
        gms = time_graph(torch, tr, 20)
        extra["headline_graph"] = {"ms_per_step": gms, "train_pts_per_s": N / (gms * 1e-3)}
        progress("headline step as a replayed graph done")
        del tr
        torch.cuda.empty_cache()
        trb, _, _ = make_trainer(A, torch, synth, A.BF16, N)
        dtb, kb, gbm = time_steps(A, torch, trb, args.steps, args.warmup, hl)
        extra["train_pts_per_s_bf16_mlp"] = N * args.steps / dtb
        extra["bf16_ms_per_step"] = dtb * 1e3 / args.steps
        extra["bf16_kernel_ms"] = kb
        extra["bf16_gather_ms"] = gbm
        extra["bf16_kernel_roofline"] = {"bound": "mfma", "achieved": flops / (kb * 1e-3) / 1e12,
                                         "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                                         "frac": flops / (kb * 1e-3) / 1e12 / PEAK_BF16_MFMA_TFLOPS,
                                         "kernel": "k_adjoint (four waves per block, two blocks per CU)"}
        progress("bf16-MLP step done")
        del trb
        torch.cuda.empty_cache()
        c4_48 = lambda A_, t_, s_, h_: extra_c4(A_, t_, s_, h_, B=300)  # noqa: E731
        for name, fn in (("config1_tiny_fp32", extra_c1), ("config3_mixed_1024", extra_c3),
                         ("config4_bricks", extra_c4), ("config4_48bricks", c4_48),
                         ("config5_render_bf16", extra_c5), ("f4_variants", extra_f4)):
            if name.split("_")[0] in args.configs:
                try:
                    extra[name] = fn(A, torch, synth, hl)
                except Exception as e:  # an extra figure never hides the headline line
                    extra[name] = {"error": repr(e)[:200]}
                progress(f"{name} done")
                torch.cuda.empty_cache()
        out["extra"] = extra
    if args.copy_probe:
        src = torch.ones(COPY_PROBE_BYTES // 4, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(vol.cpu().numpy().astype("float64"), host, args.cpu_sample)
        progress("cpu baseline done")
        out["stated_errors_vs_oracle"] = stated_errors(A, torch, synth, vol, host, args.error_sample)
        progress("stated errors done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
