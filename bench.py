#!/usr/bin/env python
"""Throughput of the wide-band ADMM iteration on one MI355X.

One step = one full pass of Algorithm 1 (steps I-VI: row FFT, fused column
solve, inverse row FFT, fused spectral/prox/dual pass) over the whole cube.
Default workload: 1024 x 1024 x 64 bands, FP32, synthetic inputs (uv-track
PSFs, point + Gaussian sky, rho = 1, mu_s = mu_nu = 0.02, mu_eps = 1e-3).

Prints ONE JSON line: voxel-iterations/s, the roofline of the dominant
kernel (HIP-event timing of each kernel on the solver's stream, algorithmic
bytes per launch), the FP64 instantiation's rate, and the FP64 CPU oracle
timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-graph] [--no-batch]

Each pass is replayed from a HIP graph unless --no-graph is given.  The
16-cube batch (uneven sizes and band counts) is timed in its per-cube
sequential, grouped, grouped + graph and autotuned forms, and the paper's
spatial dictionary (Dirac + Db1..Db8) on the same cube and on the paper's
256 x 256 x 15 run shape (the `dictionary` object).  The `grad` object times
the reverse sweep of 20 unrolled passes at full size against 20 forward passes.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0      # MI355X HBM3E peak
METRIC = "voxel-iterations/s (FP32 vs FP64) at 1024²×64; HBM GB/s % of peak"

# algorithmic bytes per voxel and per pass of each kernel, in units of the
# element size (4 B in FP32): reads + writes of the arrays it must touch
#   row_fwd  : B_rest in, packed half spectrum out                     2
#   col_solve: spectrum in/out, conj(h) y_hat in, |h|^2 in (half)      3.5
#   row_inv  : spectrum in, X out                                      2
#   spectral : X, z_P, z_T, z_V, Gamma_S in;
#              z_P, z_T, z_V, Gamma_S, B_rest out                      10
#   fused    : Z, z_P, z_T, z_V, Gamma_S in;
#              Z, z_P, z_T, z_V, Gamma_S out                             10
#              (and X out, 11, in the last pass of a run only: the earlier
#              passes' X is overwritten unread; the profiled launches are
#              the steady-state ones)
KERNEL_ELEMS = {"row_fwd": 2.0, "col_solve": 3.5, "row_inv": 2.0, "spectral": 10.0, "fused": 10.0}
# minimum traffic of one pass of this algorithm: the 4-array state stream in
# and out plus the constants (38 B in FP32) and one transposition round trip
# of the 2-D FFT (16 B)
ITER_MIN_ELEMS = 13.5
# the same minimum for a 5-array state (46 + 16 = 62 B in FP32)
ITER_MIN5_ELEMS = 15.5
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash():
    """Hash of the sources of the iteration kernels (counters go stale with them)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("muffin_device.hpp", "muffin_kernels.hpp", "muffin_fft.hip", "muffin_spectral.hip", "muffin_fused.hip"):
        with open(os.path.join(ROOT, "paper_1504_06847_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counters, or None when the
    counters are missing or were taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get("kernels", {}).get(workload, {}).get(kernel)
    if not e or t.get("source_hash") != kernel_source_hash():
        return None
    return e["fetch_kib"] * t["fetch_scale"] * 1024 + e["write_kib"] * t["write_scale"] * 1024


def read_probe(mib=1024, reps=20):
    """A read-only pass of a known size: a sum over a device array (a second
    calibration of the FETCH counter, from another kernel than the copy)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.rand(n, device="cuda")
    for _ in range(3):
        a.sum()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        a.sum()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"read_probe_MiB": mib, "ms": round(ms, 4),
                      "GBps": round(mib * (1 << 20) / (ms * 1e-3) / 1e9, 1)}), flush=True)


def copy_probe(mib=256, reps=20):
    """Plain device copy of a known size (calibrates the FETCH/WRITE counters)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.rand(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_probe_MiB": mib, "ms": round(ms, 4),
                      "GBps": round(2 * mib * (1 << 20) / (ms * 1e-3) / 1e9, 1)}), flush=True)


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(inst, params, iters: int, workers: int):
    """Time the FP64 oracle (as it stands) on `iters` passes of the same cube."""
    import oracle as O
    O.set_workers(workers)
    prob = O.Problem(inst.psf, inst.dirty, params)
    st = O.State.zeros(prob.shape)
    st = O.admm_iteration(prob, st)          # first touch of every array, untimed
    t0 = time.perf_counter()
    for _ in range(iters):
        st = O.admm_iteration(prob, st)
    dt = time.perf_counter() - t0
    L, ny, nx = prob.shape
    return dict(value=L * ny * nx * iters / dt, unit="voxel-iterations/s", cores=workers,
                kind="oracle", cpu=cpu_model(),
                sample=f"{iters} FP64 passes of the full {nx}x{ny}x{L} cube after one untimed "
                       f"pass; scipy.fft with {workers} threads, {dt:.1f} s")


def run_gpu(inst, params, dtype, steps, warmup, profile_iters, graph=False):
    import torch
    from paper_1504_06847_amd import Solver
    kw = dict(mu_eps=params.mu_eps, mu_s=params.mu_s, mu_nu=params.mu_nu, rho_P=params.rho_P,
              rho_T=params.rho_T, rho_V=params.rho_V, rho_S=params.rho_S)
    s = Solver(inst.psf, inst.dirty, dtype=dtype, graph=graph, **kw)
    schedule = s.autotune(reps=5)             # tile schedules and pass form for this shape
    s.iterate(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    s.iterate(steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    prof = s.profile(profile_iters) if profile_iters > 0 else {}
    # the fused kernel in both forms (one or two pixels per thread), timed
    # the same way, whichever the autotuner kept
    forms = {}
    if profile_iters > 0 and s.fused_available:
        for form in (1, 2):
            s.set_schedule((schedule[0], schedule[1], form))
            forms[str(form)] = round(s.profile(profile_iters).get("fused", float("nan")), 5)
        s.set_schedule(schedule)
    s.close()
    if forms:
        prof = dict(prof)
        prof["_fused_forms_ms"] = forms
    return ms, prof, schedule


def run_grad(inst, params, K, ckpt_small=5):
    """The reverse sweep of K unrolled FP32 passes (MSE loss against the sky,
    gradient in mu_s, mu_nu, rho) at the cube's full size, timed once after
    an untimed sweep, against K forward passes: with the library's default
    checkpoint spacing (the largest whose scratch fits half the free HBM:
    every pass stored at this size) and with checkpoints every
    ``ckpt_small`` passes (a memory-bound setting: segments recomputed)."""
    import torch
    from paper_1504_06847_amd import Solver
    kw = dict(mu_eps=params.mu_eps, mu_s=params.mu_s, mu_nu=params.mu_nu, rho=params.rho_P)
    s = Solver(inst.psf, inst.dirty, graph=True, **kw)
    s.autotune(reps=3)
    C = s.sweep_ckpt_every(K)
    sky = torch.as_tensor(inst.sky, dtype=torch.float32, device=s.device)   # in HBM before the timed region

    def timed(c):
        s.grad(K, sky=sky, ckpt_every=c)               # workspace allocation, warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = s.grad(K, sky=sky, ckpt_every=c)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    t_grad, (loss, g) = timed(C)
    t_small, _ = timed(ckpt_small)
    s.reset()
    s.iterate(1)
    s.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(K)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    scratch = s.grad_workspace_bytes(K, C, False)
    scratch_small = s.grad_workspace_bytes(K, ckpt_small, False)
    s.close()
    return {"K": K, "ckpt_every": C, "ms": round(t_grad * 1e3, 2), "forward_ms": round(t_fwd * 1e3, 2),
            "ratio_to_forward": round(t_grad / t_fwd, 2), "scratch_GiB": round(scratch / 2**30, 2),
            "loss": loss, "grad": [float(v) for v in g],
            "recomputed": {"ckpt_every": ckpt_small, "ms": round(t_small * 1e3, 2),
                           "ratio_to_forward": round(t_small / t_fwd, 2),
                           "scratch_GiB": round(scratch_small / 2**30, 2)}}


# algorithmic elements per voxel of one wavelet basis in a pass: X read,
# the basis's coefficient cube read and written, B_rest read and written
DICT_ELEMS_PER_BASIS = 5.0


def run_dictionary(inst, params, steps, warmup, profile_iters, graph=True):
    """The paper's spatial dictionary (Dirac + Db1..Db8, n_s = 9) on the same
    cube: voxel-iterations/s and the kernels of a pass."""
    import torch
    from paper_1504_06847_amd import PAPER_DICTIONARY, Solver
    kw = dict(mu_eps=params.mu_eps, mu_s=params.mu_s, mu_nu=params.mu_nu, rho_P=params.rho_P,
              rho_T=params.rho_T, rho_V=params.rho_V, rho_S=params.rho_S)
    s = Solver(inst.psf, inst.dirty, graph=graph, spatial=PAPER_DICTIONARY, **kw)
    schedule = s.autotune(reps=3)
    s.iterate(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    s.iterate(steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    prof = s.profile(profile_iters) if profile_iters > 0 else {}
    s.close()
    L, ny, nx = inst.psf.shape
    V = L * ny * nx
    n_w = len(PAPER_DICTIONARY) - 1
    out = {"bases": "Dirac + Db1..Db8", "n_s": len(PAPER_DICTIONARY), "shape": [L, ny, nx],
           "value": V * steps / (ms / 1e3), "unit": "voxel-iterations/s",
           "ms_per_step": round(ms / steps, 4), "steps": steps, "schedule": list(schedule),
           "kernels_ms": {k: round(v, 5) for k, v in prof.items()}}
    if "dictionary" in prof:
        nbytes = DICT_ELEMS_PER_BASIS * n_w * 4 * V
        out["dictionary_alg_bytes"] = int(nbytes)
        out["dictionary_GBps"] = round(nbytes / (prof["dictionary"] * 1e-3) / 1e9, 1)
        # the least any schedule moves: X read once, each z_b read and
        # written once, B_rest read and written once
        min_bytes = (3 + 2 * n_w) * 4 * V
        out["dictionary_min_bytes"] = int(min_bytes)
        out["dictionary_min_bytes_frac"] = round(min_bytes / (prof["dictionary"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
    return out


def run_large(steps, warmup, profile_iters, graph=True):
    """The large workload: 2048 x 2048 x 256 bands FP32 (curved spectra, 200
    antennas, 500 points + 100 Gaussians), its own 200 passes timed after a
    warm-up, each kernel of a pass timed with events, the spectral pass (the
    largest) against the HBM peak."""
    import torch
    from paper_1504_06847_amd import Solver
    from synth import get_config
    cfg = get_config("large2048")
    t0 = time.perf_counter()
    inst = cfg.make()
    t_gen = time.perf_counter() - t0
    p = cfg.params
    t0 = time.perf_counter()
    s = Solver(inst.psf, inst.dirty, graph=graph, mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=p.rho_P)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    del inst
    schedule = s.autotune(reps=2)
    s.iterate(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    s.iterate(steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    prof = s.profile(profile_iters) if profile_iters > 0 else {}
    rep = s.step_report()
    ws_gib = s._ws_bytes / 2**30
    s.close()
    V = cfg.voxels
    kernels = {}
    for name, kms in prof.items():
        nbytes = KERNEL_ELEMS.get(name, 0.0) * 4 * V
        kernels[name] = dict(ms=round(kms, 4), alg_bytes=int(nbytes), GBps=round(nbytes / (kms * 1e-3) / 1e9, 1))
    dom = max(prof, key=prof.get) if prof else None
    value = V * steps / (ms / 1e3)
    return {"workload": f"{cfg.name}: {cfg.nx}x{cfg.ny} pixels x {cfg.L} bands, FP32, {cfg.n_ant} antennas, "
                        f"{cfg.n_points} points + {cfg.n_gauss} Gaussians with curved spectra",
            "value": value, "unit": "voxel-iterations/s", "steps": steps, "ms_per_step": round(ms / steps, 4),
            "schedule": list(schedule), "kernels": kernels,
            "roofline": None if dom is None else dict(
                bound="hbm", kernel=dom, achieved=kernels[dom]["GBps"], peak=HBM_PEAK_GBPS, unit="GB/s",
                frac=round(kernels[dom]["GBps"] / HBM_PEAK_GBPS, 4)),
            "iteration_62B_frac": round(ITER_MIN5_ELEMS * 4 * value / 1e9 / HBM_PEAK_GBPS, 4),
            "workspace_GiB": round(ws_gib, 2), "generate_s": round(t_gen, 1), "setup_s": round(t_setup, 2),
            "report_after": {k: rep[k] for k in ("iters", "r_pri", "r_dual", "E", "objective")}}


def cpu_context(workers_all):
    """The oracle's full runs of the small workloads (64 x 64 x 8, 100
    passes; the paper's 256 x 256 x 15 shape, 350 passes; 256 x 256 x 32,
    300 passes), on every host core, and the first with one thread too."""
    import oracle as O
    from synth import get_config
    out = {}
    for name, workers in (("plain64", 1), ("plain64", workers_all), ("paper256", workers_all),
                          ("fp32_256", workers_all)):
        c = get_config(name)
        inst = c.make()
        O.set_workers(workers)
        prob = O.Problem(inst.psf, inst.dirty, c.params)
        t0 = time.perf_counter()
        O.run(prob, c.iters)
        dt = time.perf_counter() - t0
        out[f"{name}_w{workers}"] = {"passes": c.iters, "shape": [c.L, c.ny, c.nx], "workers": workers,
                                     "seconds": round(dt, 2), "value": c.voxels * c.iters / dt,
                                     "unit": "voxel-iterations/s"}
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def run_vis(steps, warmup, n_cg=10):
    """The visibility-domain model (step I by n_cg CG iterations per band) at
    the paper's run shape, 256 x 256 x 15, FP32, graph replay: the 20-antenna
    track's 190 baselines x 60 samples = 11,400 visibilities per band."""
    import torch
    from paper_1504_06847_amd import VisSolver
    from synth import get_config
    from synth.visibilities import make_vis_instance
    p = get_config("paper256").params
    inst = make_vis_instance(256, 256, 15, n_points=20, n_gauss=5, n_ant=20, noise_sigma=0.01, seed=6, n_time=60)
    kw = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho_P=p.rho_P, rho_T=p.rho_T, rho_V=p.rho_V,
              rho_S=p.rho_S)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = VisSolver(inst.uv, inst.vis, inst.shape, n_cg=n_cg, graph=True, **kw)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    s.iterate(warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    s.iterate(steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    s.close()
    V = 15 * 256 * 256
    return {"shape": [15, 256, 256], "n_vis_per_band": int(inst.vis[0].size), "n_cg": n_cg, "steps": steps,
            "value": V * steps / (ms / 1e3), "unit": "voxel-iterations/s", "ms_per_step": round(ms / steps, 4),
            "setup_s": round(t_setup, 3),
            "paper_350_iterations_s": round(350 * ms / steps / 1e3, 3)}


def run_batch(steps, warmup):
    """voxel-iterations/s of the batch: each cube iterated on its own (one
    cube after another, the plain per-cube launches), then grouped launches,
    then grouped launches replayed from a graph, then the same after the
    schedule autotuner."""
    import torch
    from paper_1504_06847_amd import Batch, Solver
    from synth.configs import batch_instances
    cubes, p = batch_instances()
    kw = dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho_P=p.rho_P, rho_T=p.rho_T,
              rho_V=p.rho_V, rho_S=p.rho_S)
    V = sum(int(np.prod(c[0].shape)) for c in cubes)

    def timed(fn):
        fn(warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn(steps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    solvers = [Solver(a, b, **kw) for a, b in cubes]

    def seq(k):
        for s in solvers:
            s.iterate(k)
    ms_seq = timed(seq)
    for s in solvers:
        s.close()
    del solvers
    b = Batch(cubes, params=kw)
    ms_grp = timed(lambda k: b.iterate(k))
    b.set_graph(True)
    ms_graph = timed(lambda k: b.iterate(k))
    b.autotune(reps=5)
    ms_tuned = timed(lambda k: b.iterate(k))
    launches = b.launches
    b.close()
    rate = lambda ms: V * steps / (ms / 1e3)
    return {"cubes": len(cubes), "voxels": V, "steps": steps,
            "shapes": [list(c[0].shape) for c in cubes],
            "per_cube_sequential": rate(ms_seq), "grouped": rate(ms_grp),
            "grouped_graph": rate(ms_graph), "grouped_graph_autotuned": rate(ms_tuned),
            "grouped_launches_per_pass": launches,
            "speedup_vs_sequential": round(ms_seq / min(ms_grp, ms_graph, ms_tuned), 3),
            "unit": "voxel-iterations/s"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="cube1024")
    ap.add_argument("--profile-iters", type=int, default=20)
    ap.add_argument("--fp64-steps", type=int, default=20)
    ap.add_argument("--cpu-iters", type=int, default=5)
    ap.add_argument("--grad-K", type=int, default=20,
                    help="passes unrolled in the timed reverse sweep (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="launch each pass's kernels one by one instead of replaying a HIP graph")
    ap.add_argument("--no-batch", action="store_true", help="skip the 16-cube batch measurement")
    ap.add_argument("--batch-steps", type=int, default=50)
    ap.add_argument("--vis-steps", type=int, default=20,
                    help="timed passes of the visibility-domain model at 256x256x15 (0: skip)")
    ap.add_argument("--dict-steps", type=int, default=10,
                    help="timed passes with the paper's spatial dictionary (0: skip)")
    ap.add_argument("--large-steps", type=int, default=200,
                    help="timed passes of the 2048 x 2048 x 256 workload (0: skip)")
    ap.add_argument("--no-cpu-context", action="store_true",
                    help="skip the oracle's full runs of the small workloads")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a device copy (counter calibration)")
    ap.add_argument("--probe-mib", type=int, default=256, help="size of the copy or read probe")
    ap.add_argument("--read-probe", action="store_true",
                    help="only run a read-only sum over a device array (counter calibration)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU "
              "band-sharded layout is a design, not built", file=sys.stderr)
        sys.exit(2)
    import torch
    from synth import get_config
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if a.copy_probe:
        copy_probe(a.probe_mib)
        return
    if a.read_probe:
        read_probe(a.probe_mib)
        return
    cfg = get_config(a.config)
    _log(f"bench: generating {cfg.name} {cfg.nx}x{cfg.ny}x{cfg.L}")
    inst = cfg.make()
    V = cfg.voxels
    _log(f"bench: FP32 {a.warmup} warmup + {a.steps} timed passes")
    ms32, prof32, sched32 = run_gpu(inst, cfg.params, torch.float32, a.steps, a.warmup, a.profile_iters,
                                    graph=a.graph)
    value = V * a.steps / (ms32 / 1e3)
    fused_forms = prof32.pop("_fused_forms_ms", None)
    kernels = {}
    for name, kms in prof32.items():
        nbytes = KERNEL_ELEMS.get(name, 0.0) * 4 * V
        kernels[name] = dict(ms=round(kms, 5), alg_bytes=int(nbytes),
                             GBps=round(nbytes / (kms * 1e-3) / 1e9, 1))
    dom = max(prof32, key=prof32.get) if prof32 else None
    roof = None
    if dom:
        ach = kernels[dom]["GBps"]
        tr = measured_traffic(dom, cfg.name)
        roof = dict(bound="hbm", kernel=dom, achieved=ach, peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBPS, 4),
                    traffic=None if tr is None else int(tr),
                    alg_bytes_per_launch=kernels[dom]["alg_bytes"])
    fp64 = None
    if a.fp64_steps > 0:
        _log(f"bench: FP64 {a.fp64_steps} timed passes")
        ms64, prof64, sched64 = run_gpu(inst, cfg.params, torch.float64, a.fp64_steps, 2, 5, graph=a.graph)
        prof64.pop("_fused_forms_ms", None)
        fp64 = dict(value=V * a.fp64_steps / (ms64 / 1e3), ms_per_step=round(ms64 / a.fp64_steps, 4),
                    kernels_ms={k: round(v, 5) for k, v in prof64.items()}, schedule=list(sched64))
    grad = None
    if a.grad_K > 0:
        _log(f"bench: reverse sweep of {a.grad_K} passes")
        grad = run_grad(inst, cfg.params, a.grad_K)
    dictionary = None
    if a.dict_steps > 0:
        _log(f"bench: spatial dictionary, {a.dict_steps} timed passes")
        dictionary = run_dictionary(inst, cfg.params, a.dict_steps, 2, 3, graph=a.graph)
        pcfg = get_config("paper256")
        dictionary["paper_shape"] = run_dictionary(pcfg.make(), pcfg.params, 5 * a.dict_steps, 3, 3,
                                                   graph=a.graph)
    vis = None
    if a.vis_steps > 0:
        _log(f"bench: visibility-domain model, {a.vis_steps} timed passes")
        vis = run_vis(a.vis_steps, 3)
    batch = None
    if not a.no_batch:
        _log(f"bench: 16-cube batch, {a.batch_steps} passes per form")
        batch = run_batch(a.batch_steps, 3)
    large = None
    if a.large_steps > 0:
        _log(f"bench: 2048 x 2048 x 256, {a.large_steps} timed passes")
        large = run_large(a.large_steps, 3, 5, graph=a.graph)
    cpu = None
    workers_all = os.cpu_count() or 1
    if not a.no_cpu_baseline:
        _log(f"bench: CPU oracle, {a.cpu_iters} passes")
        cpu = cpu_baseline(inst, cfg.params, a.cpu_iters, workers_all)
        cpu["one_thread"] = cpu_baseline(inst, cfg.params, 1, 1)
        if not a.no_cpu_context:
            _log("bench: CPU oracle, full runs of the small workloads")
            cpu["full_runs"] = cpu_context(workers_all)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms32 / a.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.nx}x{cfg.ny} pixels x {cfg.L} bands, FP32 ADMM "
                               f"pass (Dirac W_s, DCT-II W_nu), rho=1, mu_s=mu_nu=0.02, mu_eps=1e-3",
                   "nx": cfg.nx, "ny": cfg.ny, "L": cfg.L, "voxels": V,
                   "parallelism": "1 GPU", "graph": bool(a.graph), "schedule": list(sched32)},
        "roofline": roof,
        # one pass at this rate against the HBM peak, counting the minimum
        # bytes of this algorithm (4-array state, 54 B/voxel in FP32) and of
        # a 5-array state (62 B/voxel)
        "iteration_min_bytes_frac": round(ITER_MIN_ELEMS * 4 * value / 1e9 / HBM_PEAK_GBPS, 4),
        "iteration_62B_frac": round(ITER_MIN5_ELEMS * 4 * value / 1e9 / HBM_PEAK_GBPS, 4),
        "kernels": kernels,
        "fused_forms_ms": fused_forms,
        "fp64": fp64,
        "grad": grad,
        "dictionary": dictionary,
        "visibility": vis,
        "batched": batch,
        "large": large,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
