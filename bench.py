#!/usr/bin/env python3
"""End-to-end PCA throughput on one MI355X.

Workload: the 224-band radiance cube, 1024 x 1024 pixels (uint16 counts with
Poisson-like noise from the seeded generator, converted to float32 before
timing), k = 10 components. One step is the whole hot path on one cube:
fused centring + covariance, cyclic Jacobi eigendecomposition (with
eigenvector replay, sort and sign fix) and projection. The cube is resident in
HBM before timing starts.

The metric is Mpixel*band/s = pixels * bands * steps / time / 1e6, measured for
the plain float32 covariance and for the split-bfloat16 forms; `value` is the
fastest form whose eigenvalue error against the FP64 oracle is <= 1e-5
(normwise). Also reported: per-stage times from HIP events on the stream the
kernels run on, the roofline of the dominant kernel, the FP64 oracle timed
on the host cores, and (`stream`) the steady-state throughput of a stream of
such cubes with several in flight, where the single-CU Jacobi of one cube
overlaps the streaming passes of the others (every cube still runs the whole
pipeline; `value` stays the one-cube-at-a-time figure).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cube224|batch64]
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

# The stream measurement keeps several cubes in flight, one HIP stream each;
# HIP maps streams onto this many hardware queues per process (4 by default,
# which makes some of the streams share a queue and serialise). It must be
# set before the runtime starts, so here, before torch is imported; it only
# concerns this process, and the one-stream timings do not depend on it.
os.environ["GPU_MAX_HW_QUEUES"] = "8"

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "end-to-end PCA Mpixel·band/s; split-BF16 vs FP32 at ≤1e-5 eigval error"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, datasheet
MFMA_F32_PEAK_TFS = 157.3      # dense FP32 matrix
FP32_VECTOR_PEAK_TFS = 157.3   # FP32 vector (packed FMA counted), 256 CUs at 2.4 GHz
MFMA_BF16_PEAK_TFS = 2500.0    # dense BF16 matrix
EIG_TOL = 1e-5
# Covariance forms timed on the headline cube; the headline is the fastest of
# the metric's forms (float32 and split-bfloat16) within EIG_TOL.
DEFAULT_MODES = "f32,bf16x3,bf16x4,fp16x3"
HEADLINE_MODES = ("f32", "bf16x3", "bf16x4")
JACOBI_BLOCK_MIN_BANDS = 96    # the library's default form: block-cyclic from this band count


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_pipeline(P, torch, pipe, Yd, steps, warmup):
    for _ in range(warmup):
        pipe.forward(Yd)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        pipe.forward(Yd)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def time_stages(P, torch, pipe, Yd, steps):
    """Per-stage times from events recorded between the three C-ABI calls."""
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    torch.cuda.synchronize()
    for s in range(steps):
        ev[s][0].record(stream)
        pipe.covariance(Yd)
        ev[s][1].record(stream)
        pipe.eigh()
        ev[s][2].record(stream)
        pipe.project(Yd)
        ev[s][3].record(stream)
    torch.cuda.synchronize()
    names = ("covariance", "jacobi_eigh", "project")
    out = {}
    for i, nm in enumerate(names):
        out[nm] = statistics.mean(ev[s][i].elapsed_time(ev[s][i + 1]) for s in range(steps))
    return out


def time_stream(P, torch, n, m, k, mode, cubes, count, warmup, depth, chain=True, passes=1):
    """Steady-state throughput of a stream of cubes with `depth` in flight
    (PCAStream): `count` cubes, taken round-robin from `cubes` (distinct
    resident copies), after `warmup` untimed ones; with several `passes` of
    `count` cubes through the same PCAStream, the median pass. Returns
    (ms per cube, wall seconds of that pass, all converged, the PCAStream,
    ms per cube of every pass)."""
    ps = P.PCAStream(n, m, k, mode, depth=depth, chain=chain)
    for i in range(warmup):
        ps.submit(cubes[i % len(cubes)])
    ps.join()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    runs = []
    for _ in range(passes):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for i in range(count):
            ps.submit(cubes[i % len(cubes)])
        ps.join()
        e1.record(stream)
        torch.cuda.synchronize()
        runs.append((e0.elapsed_time(e1) / count, time.perf_counter() - t0))
    ok = all(P.read_info(p.info)["converged"] == 1 for p in ps.pipes)
    ms, wall = sorted(runs)[len(runs) // 2]
    return ms, wall, ok, ps, [round(r[0], 4) for r in runs]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(oracle, Y, k, budget_s=12.0, max_runs=3, one_thread_pixels=1 << 17):
    """The FP64 oracle on the same cube, repeated until ~budget_s of work with
    the host's BLAS threads, then once with one thread on a leading sample of
    one_thread_pixels pixels (the oracle's Jacobi is single-threaded C)."""
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threadpool_limits = None
        threads = os.cpu_count() or 1
    times = []
    t_all = time.perf_counter()
    while len(times) < max_runs and (time.perf_counter() - t_all) < budget_s:
        t0 = time.perf_counter()
        oracle.pca(Y, k)
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    n, m = Y.shape
    out = dict(value=round(n * m / med / 1e6, 3), unit="Mpixel·band/s", cores=int(threads), kind="oracle",
               sample=f"full cube {n} px x {m} bands, k={k}, float64 mean/covariance/row-cyclic Jacobi/"
                      f"projection; median of {len(times)} runs ({med:.2f} s each)",
               cpu_model=cpu_model())
    if threadpool_limits is not None:
        Ys = Y[:one_thread_pixels]
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            oracle.pca(Ys, k)
            t1 = time.perf_counter() - t0
        out["one_thread"] = dict(value=round(Ys.shape[0] * m / t1 / 1e6, 3), unit="Mpixel·band/s", cores=1,
                                 sample=f"leading {Ys.shape[0]} px x {m} bands, one run ({t1:.2f} s)")
    return out


def copy_check(torch, nbytes=1 << 30, reps=5):
    """A plain device copy of known size: the reference that scales the
    FETCH_SIZE / WRITE_SIZE counters, and the measured copy ceiling."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps(dict(copy_bytes=nbytes, ms=round(ms, 4), read_write_GBps=round(2 * nbytes / ms / 1e6, 1))),
          flush=True)
    return 0


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for name in t.get("sources", []):
        with open(os.path.join(ROOT, name), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != t.get("sources_sha256"):
        return None
    rec = t.get("kernels", {}).get(kernel)
    return None if rec is None else rec.get("bytes_per_launch")


def run_batch(P, synth, torch, steps, warmup, mode="f32", lanes=1, autotune=False, check=0):
    """The batched form: 64 cubes with square sides 64..512 and 64..256 bands,
    k = 5, through pca_batched calls (one per lane: sub-batches by band count
    on their own HIP streams) captured in one HIP graph. check > 0: the
    eigenvalues of that many cubes (the widest and the narrowest alternately)
    against the FP64 oracle."""
    import numpy as np
    log("generating the 64-cube batch ...")
    cubes = synth.make_batch(64, 4000)
    Yd = [torch.from_numpy(Y).cuda() for Y in cubes]
    b = P.BatchedPCA(Yd, 5, mode, lanes=lanes)
    tuning = None
    if autotune:
        from paper_2403_18321_amd import autotune as _at
        tuning, _ = _at.tune(b)
    g = b.capture()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    pb = b.pixel_bands()
    conv = sum(P.read_info(i)["converged"] for i in b.info)
    rec = dict(value=round(pb / (ms * 1e-3) / 1e6, 1), unit="Mpixel·band/s", ms_per_step=round(ms, 4),
               dtype="bf16" if mode.startswith("bf16") else "f32", cov_mode=mode, pixel_bands=pb, tuning=tuning,
               lanes=[len(gg) for gg in b.groups], converged=f"{conv}/{len(b.info)}",
               workload="64 cubes, square sides 64..512 px, 64..256 bands, k=5 (pca_batched per lane, graph replay)")
    if check > 0:
        import oracle
        order = sorted(range(len(cubes)), key=lambda i: cubes[i].shape[1] * cubes[i].shape[0])
        pick = []
        while len(pick) < min(check, len(order)):
            pick.append(order.pop(-1 if len(pick) % 2 == 0 else 0))
        errs = []
        for i in pick:
            lam_ref = oracle.pca(cubes[i], 5)["lam"]
            lam = b.eigvals[i].cpu().numpy().astype(np.float64)
            errs.append(float(np.max(np.abs(lam - lam_ref)) / abs(lam_ref[0])))
        rec["eig_err_max"] = max(errs)
        rec["checked_cubes"] = pick
    del Yd, cubes, b, g
    return rec


def bench_batch(P, synth, torch, args):
    mode = args.modes.split(",")[0] if args.modes != DEFAULT_MODES else "f32"
    rec = run_batch(P, synth, torch, args.steps, args.warmup, mode, args.lanes, args.autotune,
                    0 if args.no_accuracy else 8)
    out = dict(metric=METRIC, value=rec["value"], unit="Mpixel·band/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=rec["ms_per_step"], higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype=rec["dtype"], data="synthetic",
               config=dict(workload=rec["workload"], pixel_bands=rec["pixel_bands"], cov_mode=mode,
                           tuning=rec["tuning"], lanes=rec["lanes"], converged=rec["converged"]))
    if "eig_err_max" in rec:
        out["eig_err_max"] = rec["eig_err_max"]
    print(json.dumps(out), flush=True)
    return 0


def run_grad(P, synth, torch, steps, warmup, check=True):
    """The differentiation form: the planted 256x256-pixel, 128-band cube,
    k = 8, float32; one step = the forward pipeline plus pca_backward for the
    loss <W, Q> (W a fixed random [pixels, k] array), whose gradient goes
    through the projection, eigendecomposition, covariance and centring
    adjoints."""
    import numpy as np
    d = synth.make_config("c5")
    k = d["k"]
    Yh = d["Y"]
    n, m = Yh.shape
    Yd = torch.from_numpy(Yh).cuda()
    W = (np.random.default_rng(1006).standard_normal((n, k)) / np.sqrt(n)).astype(np.float32)
    Wd = torch.from_numpy(W).cuda()
    pipe = P.PCAPipeline(n, m, k, "f32")
    dY = torch.empty_like(Yd)
    ws = P.workspace(P.pca_workspace_size(P.PCA_OP_BACKWARD, n, m, k=k))

    def step():
        pipe.forward(Yd)
        P.pca_backward(Yd, pipe.mean, pipe.eigvals, pipe.V, k, dY, Wd, None, None, ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_fwd = t_bwd = 0.0
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    reps = max(3, min(steps, 10))
    for _ in range(reps):
        ev[0].record(stream)
        pipe.forward(Yd)
        ev[1].record(stream)
        P.pca_backward(Yd, pipe.mean, pipe.eigvals, pipe.V, k, dY, Wd, None, None, ws)
        ev[2].record(stream)
        torch.cuda.synchronize()
        t_fwd += ev[0].elapsed_time(ev[1]) / reps
        t_bwd += ev[1].elapsed_time(ev[2]) / reps
    rec = dict(value=round(n * m / (ms * 1e-3) / 1e6, 1), unit="Mpixel·band/s", ms_per_step=round(ms, 4),
               dtype="f32", workload="planted cube 256x256 px x 128 bands, k=8, loss <W, Q> (forward + pca_backward)",
               n_pixels=n, n_bands=m, k=k, stages_ms=dict(forward=round(t_fwd, 4), backward=round(t_bwd, 4)))
    if check:
        import oracle
        ref = oracle.backward(Yh.astype(np.float64), k, dQ=W.astype(np.float64))
        g = dY.cpu().numpy().astype(np.float64)
        rec["grad_rel_err"] = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
    return rec


def bench_grad(P, synth, torch, args):
    rec = run_grad(P, synth, torch, args.steps, args.warmup, not args.no_accuracy)
    out = dict(metric="forward + adjoint PCA Mpixel·band/s", value=rec["value"], unit="Mpixel·band/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=rec["ms_per_step"], higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=rec["workload"], n_pixels=rec["n_pixels"], n_bands=rec["n_bands"], k=rec["k"]),
               stages_ms=rec["stages_ms"])
    if "grad_rel_err" in rec:
        out["grad_rel_err"] = rec["grad_rel_err"]
    print(json.dumps(out), flush=True)
    return 0


def bench_sweep(P, synth, torch, args):
    """The paper's synthetic sweep shapes (Section 6): 100^2 .. 500^2 pixels x
    50 bands and 300^2 pixels x 20 .. 200 bands, 10-endmember mixtures at 70 dB
    SNR, projection onto the first eigenvector as in the paper's designs; the
    FP32 and split-bfloat16 pipelines, each cube resident in HBM."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity_utils import report
    oracle = None
    if not args.no_accuracy:
        import oracle as _oracle
        oracle = _oracle
    k = 1
    rows = []
    for i, (n, m) in enumerate(synth.SWEEP_SHAPES):
        Yh = synth.snr_mixture_cube(np.random.default_rng(5000 + i), n, m)
        Yd = torch.from_numpy(Yh).cuda()
        ref = oracle.pca(Yh, k) if oracle is not None else None
        rec = dict(pixels=n, bands=m)
        for mode in ("f32", "bf16x3"):
            pipe = P.PCAPipeline(n, m, k, mode)
            ms, _ = time_pipeline(P, torch, pipe, Yd, args.steps, args.warmup)
            info = P.read_info(pipe.info)
            rec[mode] = dict(ms=round(ms, 4), value=round(n * m / (ms * 1e-3) / 1e6, 1), sweeps=info["sweeps"])
            if ref is not None:
                r = report(pipe.eigvals.cpu().numpy(), pipe.V.cpu().numpy(), pipe.Q.cpu().numpy(), ref, k)
                rec[mode].update(eig_err=r["eig"], angle_err=r["angle"], proj_err=r["proj"])
        rows.append(rec)
        log("sweep", json.dumps(rec))
        del Yd, pipe
    out = dict(metric=METRIC, value=None, unit="Mpixel·band/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload="the paper's sweep shapes: 100^2..500^2 px x 50 bands, 300^2 px x 20..200 bands, "
                                    "70 dB SNR mixtures, k=1"),
               shapes=rows)
    print(json.dumps(out), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--modes", default=DEFAULT_MODES)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="cube224: skip the batch64 and grad sub-records")
    ap.add_argument("--workload", choices=("cube224", "batch64", "grad", "sweep"), default="cube224",
                    help="cube224: the 224-band 1024x1024 cube (the reported line); batch64: the 64-cube batch; "
                         "grad: the differentiation form (forward + adjoint); sweep: the paper's sweep shapes")
    ap.add_argument("--autotune", action="store_true", help="batch64: tune the tile shapes first")
    ap.add_argument("--lanes", type=int, default=1,
                    help="batch64: sub-batches by band count, one pca_batched call and HIP stream each")
    ap.add_argument("--stream-depth", type=int, default=6,
                    help="cube224: also time a stream of cubes with this many in flight (0: skip)")
    ap.add_argument("--copy-check", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration, copy ceiling)")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path, "
              "so runs on more than one GPU are not made.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.copy_check:
        return copy_check(torch)

    import paper_2403_18321_amd as P
    import synth

    P.library()  # fail loudly if the HIP library is missing
    if args.workload == "batch64":
        return bench_batch(P, synth, torch, args)
    if args.workload == "grad":
        return bench_grad(P, synth, torch, args)
    if args.workload == "sweep":
        return bench_sweep(P, synth, torch, args)
    log("generating the 224-band cube ...")
    d = synth.make_config("c3")
    k = d["k"]
    Yu = d["Y_u16"]
    n, m = Yu.shape
    Yd = torch.from_numpy(d["Y"]).cuda()
    torch.cuda.synchronize()

    ref = None
    oracle = None
    if not args.no_accuracy or not args.no_cpu_baseline:
        import oracle as _oracle
        oracle = _oracle
    if not args.no_accuracy:
        log("FP64 oracle for the accuracy report ...")
        ref = oracle.pca(Yu, k)
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from parity_utils import report

    modes = {}
    for mode in args.modes.split(","):
        pipe = P.PCAPipeline(n, m, k, mode)
        ms, wall = time_pipeline(P, torch, pipe, Yd, args.steps, args.warmup)
        stages = time_stages(P, torch, pipe, Yd, max(3, min(args.steps, 10)))
        info = pipe.forward(Yd).read_info()
        rec = dict(ms_per_step=round(ms, 4), value=round(n * m / (ms * 1e-3) / 1e6, 1),
                   wall_s=round(wall, 3), stages_ms={kk: round(v, 4) for kk, v in stages.items()},
                   sweeps=info["sweeps"], steps_jacobi=info["steps"], off_rel=info["off_rel"],
                   converged=info["converged"], jacobi_form="block" if m >= JACOBI_BLOCK_MIN_BANDS else "one_cu")
        if ref is not None:
            r = report(pipe.eigvals.cpu().numpy(), pipe.V.cpu().numpy(), pipe.Q.cpu().numpy(), ref, k)
            Cg = pipe.C.cpu().numpy().astype(np.float64)
            rec.update(eig_err=r["eig"], angle_err=r["angle"], proj_err=r["proj"], subspace_sin=r.get("subspace"),
                       cov_err_fro=float(np.linalg.norm(Cg - ref["C"]) / np.linalg.norm(ref["C"])),
                       cov_err_max=float(np.abs(Cg - ref["C"]).max() / np.abs(ref["C"]).max()))
        modes[mode] = rec
        log(mode, json.dumps(rec))

    # The headline is the metric's comparison (split-bfloat16 against
    # float32); the float16 split is measured and reported beside them.
    cand = [mm for mm in modes if mm in HEADLINE_MODES] or list(modes)
    ok = [mm for mm in cand if modes[mm].get("eig_err", 0.0) <= EIG_TOL]
    best = min(ok or cand, key=lambda mm: modes[mm]["ms_per_step"])
    br = modes[best]

    # Rooflines. End to end: the algorithmic bytes of the method (the cube
    # read twice, by the covariance with fused centring and by the
    # projection, plus Q' written) at the HBM peak, against the step time.
    b_in = 4
    e2e_bytes = 2 * n * m * b_in + n * k * 4
    t_roof = e2e_bytes / (HBM_PEAK_GBS * 1e9) * 1e3
    e2e = dict(bytes=e2e_bytes, t_roof_ms=round(t_roof, 4), ms_per_step=br["ms_per_step"],
               frac=round(t_roof / br["ms_per_step"], 4))
    stages = br["stages_ms"]
    me = m + (m & 1)
    kern = {}
    t_cov = stages["covariance"] * 1e-3
    if best == "f32":
        a = n * m * (m + 1) / t_cov / 1e12
        kern["covariance"] = dict(bound="mfma", achieved=round(a, 2), peak=MFMA_F32_PEAK_TFS, unit="TFLOP/s",
                                  frac=round(a / MFMA_F32_PEAK_TFS, 4))
    else:
        a = n * m * b_in / t_cov / 1e9
        kern["covariance"] = dict(bound="hbm", achieved=round(a, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                                  frac=round(a / HBM_PEAK_GBS, 4))
    a = (n * m * b_in + n * k * 4) / (stages["project"] * 1e-3) / 1e9
    kern["project"] = dict(bound="hbm", achieved=round(a, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                           frac=round(a / HBM_PEAK_GBS, 4))
    # Jacobi: about 6 M^3 flops per sweep (two-sided rotation of every index
    # pair once), against the chip's float32 vector peak.
    jac_flops = 6.0 * me ** 3 * max(br["sweeps"], 1)
    a = jac_flops / (stages["jacobi_eigh"] * 1e-3) / 1e12
    kern["jacobi_eigh"] = dict(bound="alu", achieved=round(a, 4), peak=FP32_VECTOR_PEAK_TFS, unit="TFLOP/s",
                               frac=round(a / FP32_VECTOR_PEAK_TFS, 5), flops=jac_flops, sweeps=br["sweeps"],
                               form=br["jacobi_form"])
    dom = max(stages, key=stages.get)
    roof = dict(kern[dom])
    roof["kernel"] = dom
    roof["traffic"] = measured_traffic(dom + ":" + best)

    out = dict(metric=METRIC, value=br["value"], unit="Mpixel·band/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=br["ms_per_step"], higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype={"f32": "f32", "bf16x3": "bf16", "bf16x4": "bf16", "fp16x3": "f16"}[best], data="synthetic",
               config=dict(workload="224-band radiance cube, 1024x1024 px (uint16 counts -> float32), k=10",
                           n_pixels=n, n_bands=m, k=k, cov_mode=best),
               roofline=roof, e2e_roofline=e2e, kernels=kern, modes=modes)
    # Other ingest forms of the same cube, best covariance form: the raw
    # uint16 counts read directly (half the bytes of the float32 cube), and
    # the band-sequential float32 layout of the paper's GPU design.
    ingest = {}
    for name, Yx, layout in (("u16_bip", torch.from_numpy(Yu).cuda(), "bip"),
                             ("f32_bsq", Yd.t().contiguous(), "bsq")):
        pipe = P.PCAPipeline(n, m, k, best, layout=layout)
        ms_x, _ = time_pipeline(P, torch, pipe, Yx, args.steps, args.warmup)
        stages_x = time_stages(P, torch, pipe, Yx, max(3, min(args.steps, 10)))
        rec = dict(ms_per_step=round(ms_x, 4), value=round(n * m / (ms_x * 1e-3) / 1e6, 1),
                   stages_ms={kk: round(v, 4) for kk, v in stages_x.items()})
        if ref is not None:
            r = report(pipe.eigvals.cpu().numpy(), pipe.V.cpu().numpy(), pipe.Q.cpu().numpy(), ref, k)
            rec.update(eig_err=r["eig"], angle_err=r["angle"], proj_err=r["proj"])
        ingest[name] = rec
        log(name, json.dumps(rec))
        del Yx, pipe
    out["ingest"] = ingest

    if args.stream_depth > 0:
        # Distinct resident cubes (the same pixels in another order, so the
        # same spectrum) so that no two cubes in flight share memory.
        D = args.stream_depth
        cubes = [Yd] + [torch.roll(Yd, shifts=(j * n) // D, dims=0) for j in range(1, D)]
        torch.cuda.synchronize()
        count = max(2 * args.steps, 4 * D)
        ms_c, wall_c, conv, ps, passes = time_stream(P, torch, n, m, k, best, cubes, count, 2 * D, D, chain=False,
                                                     passes=3)
        rec = dict(value=round(n * m / (ms_c * 1e-3) / 1e6, 1), ms_per_cube=round(ms_c, 4), passes_ms=passes, depth=D,
                   hw_queues=int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
                   cubes=count, wall_s=round(wall_c, 3), cov_mode=best, converged=conv,
                   vs_sequential=round(br["ms_per_step"] / ms_c, 3))
        if ref is not None:
            errs = [report(p.eigvals.cpu().numpy(), p.V.cpu().numpy(), None, ref, k) for p in ps.pipes]
            rec["eig_err_max"] = max(e["eig"] for e in errs)
            rec["angle_err_max"] = max(e["angle"] for e in errs)
        out["stream"] = rec
        log("stream", json.dumps(rec))
        del cubes, ps
    if not args.no_secondary:
        # The other workloads, each timed here under the same clock: the
        # 64-cube batch (float32, eigenvalues of 4 cubes against the oracle)
        # and the differentiation form (gradient against the oracle's).
        del Yd
        torch.cuda.empty_cache()
        out["batch64"] = run_batch(P, synth, torch, max(3, args.steps // 4), 2, "f32", check=0 if args.no_accuracy else 4)
        log("batch64", json.dumps(out["batch64"]))
        torch.cuda.empty_cache()
        out["grad"] = run_grad(P, synth, torch, args.steps, args.warmup, not args.no_accuracy)
        log("grad", json.dumps(out["grad"]))
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(oracle, Yu, k)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
