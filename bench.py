#!/usr/bin/env python3
"""Benchmark of the LOD diffusion-decay step on one MI355X.

Workload (default): the tumour-scale single-GPU share, 1000^3 voxels x 4
substrates in FP64 (32 GB field), D log-uniform in [1e3, 1e5] um^2/min,
lambda in [0.01, 0.1] /min, dt = 0.01 min, 1e6 source/sink voxels; the
paper's "8% liver" cube (Table 1) at 10 um resolution.  One step = Src,
Dir x4 (none in this workload), x, y and z Thomas sweeps.

--workload endtoend: the paper's end-to-end run (5 mm cube, 500^3 x 1, 500
sources + 500 sinks, 500 steps): resize, Gaussian profile, initial save,
agents, simulation, final save, each stage timed (fields saved as .npy).

--workload liver12 / liver16: the larger Table 1 cubes on one GPU, 1500^3 x 8
in FP64 (216 GB) and 2000^3 x 8 in FP32 (256 GB), fields written on the device
(5 timed steps by default); their long lines run in two parts per block (plan
kind 5), or with --one-part-plans as one-part plans (kinds 1 and 3, as few
segments as cover the line: blocks of 768-1024 threads, one per CU) for
comparison.
--workload liver4: Table 1's one-node case, 500^3 x 2
in FP64 (50 timed steps), with the oracle on a bounded sample beside it.

--workload adjoint: the differentiation workload, 128^3 x 2 substrates, 50
steps with a checkpoint every 10, loss = sum of squared differences to a
seeded target: the reverse (adjoint) step timed alone and the whole
forward + backward pass through torch.autograd, FP64 and FP32 storage.

--workload batch: 96 independent domains (each axis uniform in 24..192
voxels, 1..8 substrates, FP32 or FP64 storage by a seeded coin, 1% of the
voxels as sources), autotuned, stepped together by one graph replay per step
(100 steps), plus the reverse step of domains 0..31.

--workload ceiling: the device's streaming ceilings (write only, read only,
in-place read+write, copy) on a 32 GB buffer.

--workload xslab: one process's share of the distributed x sweep (Sec. 3.2)
at the paper's 8-node split of the 1000^3 x 4 cube: a 125-voxel x-slab (4
GB, FP64), its forward and backward shares over 16 blocks of lines (blocks
= 2 x 8 processes, Eq. 5), against the same slab swept as a whole grid; and
all 8 slabs of the cube chained on one GPU, one stream per slab with the
block hand-offs as events, against the whole-line x sweep of the cube.

Fields are placed by the library (bfvm_field_alloc): the sweeps' rate depends
on where a field's allocation lands in device memory, so --placement-candidates
allocations (default 8; the library takes as many as leave a sixteenth of the
device free) are timed on one sweep set each and the fastest is kept; the
line reports every candidate and the step on a plain allocation.

Prints ONE JSON line: voxel-substrate updates/s per LOD step, the roofline
of the dominant kernel (algorithmic HBM bytes per launch / its mean launch
time from HIP events on the grid's stream, against the 8 TB/s HBM peak),
the same step with FP32 storage (errors against the FP64 run per substrate,
over every element), and the FP64 oracle timed on the host on a bounded
sample of the workload, with the host's CPU and the oracle at one and at all
threads on the three small workloads.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
STAGES = ["source", "dirichlet", "sweep_x", "sweep_y", "sweep_z"]
KERNEL_NAMES = {"sweep_x": "k_sweep_seg_strided<..., AX=0> (x rows as lines)",
                "sweep_y": "k_sweep_seg_strided<..., AX=1>", "sweep_z": "k_sweep_seg_strided<..., AX=2>"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 20; 100 for the batch workload)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="liver",
                    choices=["liver", "cells", "gaussian", "batch", "adjoint", "liver4", "liver12", "liver16", "xslab",
                             "endtoend", "ceiling"])
    ap.add_argument("--adjoint-steps", type=int, default=5,
                    help="batch workload: timed reverse steps of the 32-domain subset")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-storage companion run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=10)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 4 GiB buffer twice (reference for FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--placement-candidates", type=int, default=8,
                    help="allocations the library times to place each field (1: a plain allocation)")
    ap.add_argument("--one-part-plans", action="store_true",
                    help="liver12/liver16: run kind-5 axes as the one-part plan of twice the segments")
    return ap.parse_args()


def calibrate_copy():
    import torch
    n = (4 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    print(json.dumps({"calibration": "copy", "bytes_read_per_copy": 4 << 30, "bytes_written_per_copy": 4 << 30,
                      "copies": 2, "GBps_read_plus_write": round(2 * 2 * (4 << 30) / t / 1e9, 1)}), flush=True)


def workload(name):
    import workloads
    if name == "liver":
        return workloads.config(3)
    if name == "cells":
        return workloads.config(2)
    return workloads.config(1)


def make_grid(p, dtype):
    import paper_2602_05017_amd as bf
    g = bf.Grid(p.nx, p.ny, p.nz, p.S, tuple(p.h), dtype=dtype)
    g.set_params(p.D, p.lam, p.dt)
    if p.src is not None:
        g.set_sources(p.src.voxel, p.src.secretion, p.src.saturation, p.src.uptake)
    if p.dr is not None:
        g.set_dirichlet(p.dr.voxel, p.dr.value, p.dr.active)
    return g


def timed_run(p, dtype, steps, warmup, u_host, candidates=1):
    """Warm up, reload the field, then time `steps` steps; per-stage HIP-event times.
    The field is placed by the library (bfvm_field_alloc) among `candidates`
    allocations; with 1 it is a plain torch allocation."""
    import torch
    g = make_grid(p, dtype)
    placement = None
    if candidates > 1:
        u, cand_ms = g.alloc_field(candidates)
        ok = [m for m in cand_ms if m >= 0]
        placement = {"candidates": len(ok), "candidate_sweep_set_ms": [round(m, 3) for m in ok],
                     "kept": int(np.argmin(ok))}
        log(f"{dtype}: placement among {len(ok)} allocations, x+y+z sweep set "
            f"{', '.join(f'{m:.2f}' for m in ok)} ms; kept #{placement['kept']}")
    else:
        u = torch.empty(p.shape, dtype=g.torch_dtype, device="cuda")
    u.copy_(u_host)
    g.step(u, warmup)
    torch.cuda.synchronize()
    u.copy_(u_host)
    torch.cuda.synchronize()
    g.timing(True)
    g.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.step(u, 1)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    stages = {}
    for i, name in enumerate(STAGES):
        ms, n = g.timing_read(i)
        elems = g.timing_elements(i) if name.startswith("sweep") else 0
        stages[name] = {"total_ms": ms, "launches": n, "avg_ms": ms / n if n else 0.0,
                        "elements_per_launch": elems / n if n else 0}
    g.timing(False)
    return g, u, t, stages, placement


def default_allocation_ms(p, dtype, steps=5):
    """ms per step on a plain torch allocation of the field (for comparison
    with the placed one); the field is written on the device."""
    import torch
    g = make_grid(p, dtype)
    u = torch.empty(p.shape, dtype=g.torch_dtype, device="cuda")
    g.fill_uniform(u, p.seed, 0)
    g.step(u, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(u, steps)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    g.close()
    del u
    torch.cuda.empty_cache()
    return round(1e3 * t, 3)


def fp32_error(u32, u64, slab=50):
    """Per-substrate errors of an FP32-storage field against the FP64 GPU
    field over every element, streamed in z-slabs on the device:
    e_max = max|d| / max|u64| and e_2 = ||d||_2 / ||u64||_2."""
    import torch
    S = u64.shape[-1]
    dmax = torch.zeros(S, dtype=torch.float64, device=u64.device)
    rmax = torch.zeros_like(dmax)
    d2 = torch.zeros_like(dmax)
    r2 = torch.zeros_like(dmax)
    for z0 in range(0, u64.shape[0], slab):
        a = u64[z0:z0 + slab].reshape(-1, S)
        d = u32[z0:z0 + slab].reshape(-1, S).double() - a
        dmax = torch.maximum(dmax, d.abs().amax(0))
        rmax = torch.maximum(rmax, a.abs().amax(0))
        d2 += (d * d).sum(0)
        r2 += (a * a).sum(0)
        del d
    emax = (dmax / rmax).cpu().numpy()
    e2 = (d2.sqrt() / r2.sqrt()).cpu().numpy()
    return {"e_max_per_substrate": [float(f"{x:.4g}") for x in emax],
            "e_2_per_substrate": [float(f"{x:.4g}") for x in e2],
            "e_max": float(f"{emax.max():.4g}"), "e_2": float(f"{e2.max():.4g}"),
            "reference": "FP64 GPU run of the same workload, every element"}


SWEEP_SOURCES = ["sweep.hip", "seg_solver.hpp", "internal.hpp"]


def sweep_source_sha256():
    """Hash of the sources the sweep kernels are compiled from."""
    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2602_05017_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def traffic_record(workload_name, dtype, kernel_stage):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload_name}_{dtype}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("sweep_src_sha256") != sweep_source_sha256():
        return None
    k = rec.get("kernels", {}).get(kernel_stage)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def host_info():
    """CPU model, hardware threads and memory of the host the oracle runs on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = round(int(line.split()[1]) / (1 << 20), 1)
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "threads_available": len(os.sched_getaffinity(0)),
            "ram_GiB": ram}


def oracle_thread_runs():
    """The oracle on the three small workloads at one thread and at every
    host thread it is allowed (bounded samples: the whole 64^3 x 1 run, one
    step of the 256^3 x 8 workload with its sources and Dirichlet voxels,
    five steps of the 128^3 x 2 workload)."""
    import oracle
    import workloads
    full = oracle.threads()
    cases = [("gaussian-64^3x1-f64 (10 steps)", workloads.config(1), 10),
             ("cells-256^3x8-f64 (1 of 100 steps)", workloads.config(2), 1),
             ("adjoint-128^3x2 forward (5 of 50 steps)", workloads.config(4), 5)]
    out = {}
    for name, p, n in cases:
        src = dr = None
        if p.src is not None:
            src = oracle.Sources(p.src.voxel, p.src.secretion, p.src.saturation, p.src.uptake)
        if p.dr is not None:
            dr = oracle.Dirichlet(p.dr.voxel, p.dr.value, p.dr.active)
        rec = {}
        for th in (1, full):
            oracle.set_threads(th)
            u = np.array(p.u0, copy=True)
            t0 = time.perf_counter()
            oracle.step(u, p.h, p.D, p.lam, p.dt, src, dr, n)
            t = time.perf_counter() - t0
            rec[f"{th}_thread{'s' if th > 1 else ''}"] = {"updates_per_s": p.V * p.S * n / t,
                                                          "ms_per_step": round(1e3 * t / n, 2)}
        out[name] = rec
    oracle.set_threads(full)
    return out


def cpu_baseline(p, sample_steps):
    """The FP64 oracle on a bounded sample of the workload: `sample_steps`
    step(s) of substrate 0 over the full grid (substrates do not couple)."""
    import oracle
    s = 0
    u = np.ascontiguousarray(p.u0[..., s:s + 1])
    src = None
    if p.src is not None:
        src = oracle.Sources(p.src.voxel, p.src.secretion[:, s:s + 1], p.src.saturation[:, s:s + 1],
                             p.src.uptake[:, s:s + 1])
    dr = None
    if p.dr is not None:
        dr = oracle.Dirichlet(p.dr.voxel, p.dr.value[:, s:s + 1], p.dr.active[:, s:s + 1])
    t0 = time.perf_counter()
    oracle.step(u, p.h, p.D[s:s + 1], p.lam[s:s + 1], p.dt, src, dr, sample_steps)
    t = time.perf_counter() - t0
    upd = p.V * sample_steps
    return {"value": upd / t, "unit": "voxel-substrate updates/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{sample_steps} LOD step(s) of substrate 0 of the {p.nx}x{p.ny}x{p.nz} grid "
                      f"({upd:.3g} voxel-substrate updates, {t:.2f} s)"}


def run_batch(args):
    """The batched form: every domain's step in one graph replay."""
    import torch
    import workloads
    import paper_2602_05017_amd as bf
    steps = 100 if args.steps is None else args.steps
    probs = workloads.batch_config()
    nsub = sum(p.S for p in probs)
    upd = sum(p.V * p.S for p in probs)
    alg = sum(p.V * p.S * (3 * 2 * (8 if p.dtype == "f64" else 4)) for p in probs)
    n64 = sum(p.dtype == "f64" for p in probs)
    log(f"batch: {len(probs)} domains ({n64} f64, {len(probs) - n64} f32), {upd:.4g} voxel-substrates, "
        f"{alg / 1e9:.2f} GB algorithmic traffic per step")
    grids = [make_grid(p, p.dtype) for p in probs]
    hosts = [torch.from_numpy(p.u0) for p in probs]
    fields = [torch.empty(p.shape, dtype=g.torch_dtype, device="cuda") for p, g in zip(probs, grids)]

    def reload():
        for f, h in zip(fields, hosts):
            f.copy_(h)
        torch.cuda.synchronize()

    reload()
    b = bf.Batch(grids, fields)
    t0 = time.perf_counter()
    tuned_ms = b.autotune(None)
    log(f"autotuned in {time.perf_counter() - t0:.1f} s: {tuned_ms:.3f} ms/step (eager launches)")
    info = b.info()
    reload()
    b.step(args.warmup)
    reload()
    t0 = time.perf_counter()
    b.step(steps)
    t = time.perf_counter() - t0
    ms = 1e3 * t / steps
    value = upd * steps / t
    step_gbps = alg / (ms * 1e-3) / 1e9
    log(f"batch: {ms:.3f} ms/step, {value:.4g} updates/s, {step_gbps:.0f} GB/s algorithmic")
    # reverse steps of domains 0..31 (state = current fields, seeded gradients)
    subset = list(range(32))
    rng = np.random.default_rng(1005)
    grads = [torch.from_numpy(rng.random(p.shape) - 0.5).to(device="cuda", dtype=g.torch_dtype)
             if i in subset else None for i, (p, g) in enumerate(zip(probs, grids))]
    b.set_grads(grads)
    b.step_adjoint(subset)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.adjoint_steps):
        b.step_adjoint(subset)
    ta = (time.perf_counter() - t0) / args.adjoint_steps
    sub_upd = sum(probs[i].V * probs[i].S for i in subset)
    log(f"adjoint (32 domains): {1e3 * ta:.3f} ms per reverse step")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # bounded sample: one step of the first 12 domains
        sample = probs[:12]
        t0 = time.perf_counter()
        for p in sample:
            u = np.array(p.u0, copy=True)
            src = None if p.src is None else oracle.Sources(p.src.voxel, p.src.secretion, p.src.saturation,
                                                            p.src.uptake)
            oracle.step(u, p.h, p.D, p.lam, p.dt, src, None, 1)
        tc = time.perf_counter() - t0
        su = sum(p.V * p.S for p in sample)
        cpu = {"value": su / tc, "unit": "voxel-substrate updates/s", "cores": oracle.threads(), "kind": "oracle",
               "sample": f"1 LOD step of domains 0..11 ({su:.3g} voxel-substrate updates, {tc:.2f} s)"}
    b.close()
    line = {
        "metric": "voxel-substrate updates/s per LOD step (batched domains)",
        "value": value, "unit": "voxel-substrate updates/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 and f32 storage (per domain)",
        "data": "synthetic (seeded SplitMix64 inputs)",
        "config": {"workload": "96 uneven domains, axes 24..192, 1..8 substrates, mixed f32/f64, 1% sources",
                   "domains": len(probs), "f64_domains": n64, "substrate_fields": nsub,
                   "voxel_substrates": upd, "launches_per_step": info["launches"],
                   "items_per_step": info["items"], "chunk_elems": info["chunk_elems"]},
        "roofline": {"bound": "hbm", "achieved": round(step_gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(step_gbps / HBM_PEAK_GBPS, 4), "traffic": None,
                     "scope": "whole step: algorithmic bytes of all launches / step time",
                     "algorithmic_bytes_per_step": alg},
        "adjoint": {"domains": 32, "ms_per_reverse_step": round(1e3 * ta, 4),
                    "voxel_substrates": sub_upd, "updates_per_s": sub_upd / ta},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


# algorithmic bytes per element of one reverse step without sources and
# Dirichlet entries, z lines of at most 512 voxels, in units of the element
# size: the recomputed x and y sweeps (4, the first reading the state
# itself), the fused z pass (3: it reads the y output and the gradient and
# writes the gradient; the z output lives in registers) and the x and y
# transposed sweeps that also read the recomputed output for the parameter
# sums (6)
ADJOINT_ELEMS_MOVED = 13


def run_adjoint(args):
    """The differentiation form on the 128^3 x 2 workload."""
    import torch
    import workloads
    from paper_2602_05017_amd.autograd import simulate
    p = workloads.config(4)
    target = workloads.target_field(p)
    reps = 10 if args.steps is None else args.steps
    upd = p.V * p.S
    out = {}
    for dtype in ("f64", "f32"):
        g = make_grid(p, dtype)
        e = 8 if dtype == "f64" else 4
        u = torch.from_numpy(p.u0).to(device="cuda", dtype=g.torch_dtype)
        grad = torch.from_numpy(target - p.u0).to(device="cuda", dtype=g.torch_dtype)
        for _ in range(args.warmup):
            g.step_adjoint(u, grad.clone())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.step_adjoint(u, grad)
        torch.cuda.synchronize()
        t_rev = (time.perf_counter() - t0) / reps
        # the whole differentiation run: 50 forward steps (checkpoints every 10) + backward,
        # after an untimed 2-step pass that loads torch's own kernels for the loss
        tt = torch.from_numpy(target).to(device="cuda", dtype=g.torch_dtype)
        for nsteps in (2, p.nsteps):
            u0 = torch.from_numpy(p.u0).to(device="cuda", dtype=g.torch_dtype).requires_grad_(True)
            Dt = torch.tensor(p.D, dtype=torch.float64, requires_grad=True)
            Lt = torch.tensor(p.lam, dtype=torch.float64, requires_grad=True)
            if nsteps == 2:
                uw = simulate(g, u0, Dt, Lt, p.dt, nsteps, checkpoint_every=10)
                ((uw.double() - tt.double()) ** 2).sum().backward()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        uN = simulate(g, u0, Dt, Lt, p.dt, p.nsteps, checkpoint_every=10)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        loss = ((uN.double() - tt.double()) ** 2).sum()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t_bwd = time.perf_counter() - t0
        alg = ADJOINT_ELEMS_MOVED * e * upd
        out[dtype] = {"ms_per_reverse_step": round(1e3 * t_rev, 4), "reverse_updates_per_s": upd / t_rev,
                      "reverse_step_alg_GBps": round(alg / t_rev / 1e9, 1),
                      "forward_50_steps_ms": round(1e3 * t_fwd, 2), "backward_50_steps_ms": round(1e3 * t_bwd, 2)}
        log(f"adjoint {dtype}: reverse step {1e3 * t_rev:.3f} ms ({alg / t_rev / 1e9:.0f} GB/s algorithmic), "
            f"50-step forward {1e3 * t_fwd:.1f} ms, backward {1e3 * t_bwd:.1f} ms")
        g.close()
    # the reverse step where it is bound by HBM: 512^3 x 4 in FP64 (4.3 GB per
    # field; state, gradient and the three recomputed sweep outputs resident)
    q = workloads.config(4, n=512, nsub=4, with_field=False)
    gq = make_grid(q, "f64")
    uq = torch.empty(q.shape, dtype=torch.float64, device="cuda")
    gradq = torch.empty_like(uq)
    gq.fill_uniform(uq, q.seed, 0)
    gq.fill_uniform(gradq, q.seed, 4, -0.5, 0.5)
    gq.step_adjoint(uq, gradq)
    torch.cuda.synchronize()
    reps_q = 5
    t0 = time.perf_counter()
    for _ in range(reps_q):
        gq.step_adjoint(uq, gradq)
    torch.cuda.synchronize()
    tq = (time.perf_counter() - t0) / reps_q
    upd_q = q.V * q.S
    alg_q = ADJOINT_ELEMS_MOVED * 8 * upd_q
    hbm_bound = {"grid": [q.nx, q.ny, q.nz], "substrates": q.S, "dtype": "f64",
                 "ms_per_reverse_step": round(1e3 * tq, 3), "reverse_updates_per_s": upd_q / tq,
                 "algorithmic_bytes": alg_q, "alg_GBps": round(alg_q / tq / 1e9, 1),
                 "frac": round(alg_q / tq / 1e9 / HBM_PEAK_GBPS, 4)}
    log(f"reverse step on 512^3 x 4 FP64: {1e3 * tq:.2f} ms, {alg_q / tq / 1e9:.0f} GB/s algorithmic "
        f"({ADJOINT_ELEMS_MOVED} element moves per voxel-substrate)")
    gq.close()
    del uq, gradq
    torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        gin = target - p.u0
        reps_cpu = 5
        t0 = time.perf_counter()
        for _ in range(reps_cpu):
            gg = gin.copy()
            oracle.adjoint_step(np.array(p.u0), gg, np.zeros(p.S), np.zeros(p.S), p.h, p.D, p.lam, p.dt, None, None)
        tc = (time.perf_counter() - t0) / reps_cpu
        cpu = {"value": upd / tc, "unit": "voxel-substrate updates/s", "cores": oracle.threads(), "kind": "oracle",
               "sample": f"{reps_cpu} reverse steps of the 128^3 x 2 grid ({tc:.3f} s each)"}
        log(f"oracle reverse step: {tc:.3f} s on {cpu['cores']} threads")
    r64 = out["f64"]
    line = {
        "metric": "voxel-substrate updates/s per reverse (adjoint) LOD step (FP64)",
        "value": r64["reverse_updates_per_s"], "unit": "voxel-substrate updates/s", "n_gpus": 1, "steps": reps,
        "warmup": args.warmup, "ms_per_step": r64["ms_per_reverse_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded SplitMix64 inputs)",
        "config": {"workload": "differentiation, 128^3 x 2 substrates, 50 steps, checkpoints every 10",
                   "grid": [p.nx, p.ny, p.nz], "substrates": p.S},
        "roofline": {"bound": "hbm", "achieved": r64["reverse_step_alg_GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(r64["reverse_step_alg_GBps"] / HBM_PEAK_GBPS, 4), "traffic": None,
                     "scope": f"whole reverse step: {ADJOINT_ELEMS_MOVED} element moves per voxel-substrate / "
                              "step time; the 34 MB field fits the 256 MB memory-side cache, so this can exceed "
                              "HBM bandwidth",
                     "algorithmic_bytes_per_step": ADJOINT_ELEMS_MOVED * 8 * upd},
        "adjoint": out,
        "reverse_step_hbm_bound": hbm_bound,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


# The paper's own step times for these cubes (Table 1, BioFVM-B, FP64 with
# AVX256D on MareNostrum 5 nodes of 2 x Xeon Platinum 8480+): context for the
# line, not a target of this measurement.
PAPER_TABLE2_8PCT = {"case": "8% liver, 1000^3 x 4 (the paper's second table)", "BioFVM-B_ms_per_step": 270,
                     "BioFVM-X_ms_per_step": 2390, "nodes": 8,
                     "hardware": "MareNostrum 5 nodes of 2 x Xeon Platinum 8480+ (112 cores), FP64 with AVX256D, "
                                 "one MPI rank and 112 OpenMP threads per node"}

PAPER_TABLE1 = {
    "liver4": {"BioFVM-B_ms_per_step": 107.5, "nodes": 1, "BioFVM_ms": 241.4, "BioFVM-X_ms": 469},
    "liver12": {"BioFVM-B_ms_per_step": 356.1, "nodes": 48},
    "liver16": {"BioFVM-B_ms_per_step": 453.4, "nodes": 96, "note": "FP64 in the paper"},
}


def run_large(args):
    """A Table 1 cube that only fits on the device: the field is written there."""
    import torch
    import workloads
    p = workloads.large_config(args.workload)
    small = p.V * p.S <= 300_000_000          # fits the host: the oracle runs beside it
    steps = (50 if small else 5) if args.steps is None else args.steps
    upd = p.V * p.S
    e = 8 if p.dtype == "f64" else 4
    log(f"workload {p.name}: {upd:.4g} voxel-substrates, field {upd * e / 1e9:.0f} GB, sources {len(p.src)}")
    g = make_grid(p, p.dtype)
    if args.one_part_plans:
        # as few segments as cover the line, whole waves of 64 / lpw segments
        for a in range(3):
            kind, m, w, lpw = g.get_plan(a)
            if kind == 5:
                spw = 64 // lpw
                K = -(-(-(-p.shape[2 - a] // m)) // spw) * spw
                g.set_plan(a, 3 if a == 0 else 1, m, K * lpw // 64, lpw)
    # the library places the field among as many candidate allocations as
    # fit beside it (one for the 216 GB and 256 GB cubes)
    u, cand_ms = g.alloc_field(args.placement_candidates)
    ok = [m for m in cand_ms if m >= 0]
    placement = {"candidates": max(1, len(ok)), "candidate_sweep_set_ms": [round(m, 3) for m in ok]}
    t0 = time.perf_counter()
    g.fill_uniform(u, p.seed, 0)
    torch.cuda.synchronize()
    t_fill = time.perf_counter() - t0
    g.step(u, args.warmup)
    g.fill_uniform(u, p.seed, 0)
    torch.cuda.synchronize()
    g.timing(True)
    g.timing_reset()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.step(u, 1)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    stages = {}
    for i, name in enumerate(STAGES):
        ms, n = g.timing_read(i)
        elems = g.timing_elements(i) if name.startswith("sweep") else 0
        stages[name] = {"total_ms": ms, "launches": n, "avg_ms": ms / n if n else 0.0,
                        "elements_per_launch": elems / n if n else 0}
    g.timing(False)
    plans = [g.get_plan(a) for a in range(3)]
    lib_bytes = g.device_bytes()
    g.close()
    ms_step = 1e3 * t / steps
    value = upd * steps / t
    sweeps = {k: v for k, v in stages.items() if k.startswith("sweep")}
    dom = max(sweeps, key=lambda k: sweeps[k]["total_ms"])
    alg = int(2 * e * sweeps[dom]["elements_per_launch"])
    ach = alg / (sweeps[dom]["avg_ms"] * 1e-3) / 1e9
    log(f"{p.dtype}: {ms_step:.2f} ms/step, {value:.4g} updates/s (fill {t_fill:.2f} s)")
    line = {
        "metric": f"voxel-substrate updates/s per LOD step ({p.dtype.upper()})",
        "value": value, "unit": "voxel-substrate updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": p.dtype, "data": "synthetic (seeded SplitMix64 field written on the device)",
        "config": {"workload": p.name, "grid": [p.nx, p.ny, p.nz], "substrates": p.S, "sources": len(p.src),
                   "field_GB": round(upd * e / 1e9, 1), "plans": plans},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBPS, 4), "traffic": None, "kernel": KERNEL_NAMES.get(dom, dom),
                     "algorithmic_bytes_per_launch": alg, "avg_launch_ms": round(sweeps[dom]["avg_ms"], 4),
                     "step_alg_GBps": round(3 * 2 * e * upd / (ms_step * 1e-3) / 1e9, 1),
                     "stages_ms_per_step": {k: round(v["total_ms"] / steps, 3) for k, v in stages.items()}},
        "memory": {"field_bytes": upd * e, "library_bytes": lib_bytes,
                   "bytes_per_voxel_substrate": round((upd * e + lib_bytes) / upd, 3)},
        "placement": placement,
        "cpu_baseline": None,
    }
    if args.workload in PAPER_TABLE1:
        line["paper_context"] = PAPER_TABLE1[args.workload]
    if small and not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        p.field()
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_sample_steps * 8)
        log(f"oracle: {line['cpu_baseline']['value']:.4g} updates/s on {line['cpu_baseline']['cores']} threads")
    print(json.dumps(line), flush=True)


def run_endtoend(args):
    """The paper's end-to-end use case, stage by stage (Sec. 5.3)."""
    import shutil
    import tempfile
    import torch
    import workloads
    import paper_2602_05017_amd as bf
    p = workloads.endtoend_config(with_field=False)
    steps = p.nsteps if args.steps is None else args.steps
    tmp = tempfile.mkdtemp(prefix="bfvm_e2e_")

    def pipeline(nsteps, out):
        # each pass writes new files into its own folder: truncating the
        # previous pass's files would add the file system's truncate cost
        os.makedirs(out)
        T = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = bf.Grid(p.nx, p.ny, p.nz, p.S, tuple(p.h), dtype="f64")       # (1) resize
        g.set_params(p.D, p.lam, p.dt)
        u = torch.empty(p.shape, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        T["resize"] = time.perf_counter() - t0
        t0 = time.perf_counter()                                             # (2) Gaussian profile
        g.fill_gaussian(u, (p.nx / 2.0, p.ny / 2.0, p.nz / 2.0), p.gauss_sigma, peak=1.0, noise=p.gauss_noise,
                        seed=p.seed)
        torch.cuda.synchronize()
        T["gaussian_profile"] = time.perf_counter() - t0
        t0 = time.perf_counter()                                             # (3) initial save
        g.save_npy(u, os.path.join(out, "initial.npy"))
        T["initial_save"] = time.perf_counter() - t0
        t0 = time.perf_counter()                                             # (4) agents
        g.set_sources(p.src.voxel, p.src.secretion, p.src.saturation, p.src.uptake)
        torch.cuda.synchronize()
        T["agents"] = time.perf_counter() - t0
        t0 = time.perf_counter()                                             # (5) simulate
        g.step(u, nsteps)
        torch.cuda.synchronize()
        T["simulate"] = time.perf_counter() - t0
        t0 = time.perf_counter()                                             # (6) final save
        g.save_npy(u, os.path.join(out, "final.npy"))
        T["final_save"] = time.perf_counter() - t0
        g.close()
        del u
        torch.cuda.empty_cache()
        return T

    try:
        pipeline(2, os.path.join(tmp, "warmup"))     # warm-up: library, kernels, file system
        T = pipeline(steps, os.path.join(tmp, "run"))
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    total = sum(T.values())
    upd = p.V * p.S * steps
    log("end-to-end: " + ", ".join(f"{k} {v:.3f} s" for k, v in T.items()) + f"; total {total:.3f} s")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        q = workloads.endtoend_config(nsteps=10)
        src = oracle.Sources(q.src.voxel, q.src.secretion, q.src.saturation, q.src.uptake)
        u = np.array(q.u0, copy=True)
        t0 = time.perf_counter()
        oracle.step(u, q.h, q.D, q.lam, q.dt, src, None, q.nsteps)
        tc = time.perf_counter() - t0
        cpu = {"value": q.V * q.nsteps / tc, "unit": "voxel-substrate updates/s", "cores": oracle.threads(),
               "kind": "oracle", "sample": f"the simulate stage for 10 of the 500 steps ({tc:.2f} s); "
                                           f"500 steps would take about {tc * 50:.0f} s"}
    line = {
        "metric": "end-to-end time to solution (5 mm cube, 500 steps)", "value": total, "unit": "s",
        "n_gpus": 1, "steps": steps, "warmup": 2, "ms_per_step": round(1e3 * T["simulate"] / steps, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded agent voxels, Gaussian profile written on the device)",
        "config": {"workload": p.name, "grid": [p.nx, p.ny, p.nz], "substrates": p.S, "agents": len(p.src),
                   "stages_s": {k: round(v, 4) for k, v in T.items()},
                   "simulate_updates_per_s": upd / T["simulate"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def rmw_ceiling(u, reps: int = 3):
    """Practical HBM ceiling of a read+write pass: an in-place streaming
    multiply by 1.0 (values unchanged) over the whole field, timed with events
    on the current stream.  Every sweep reads and writes each element once, so
    this bounds a sweep's algorithmic rate on this device."""
    import torch
    u.mul_(1.0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        u.mul_(1.0)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * u.numel() * u.element_size()
    return {"GBps": round(nbytes / (ms * 1e-3) / 1e9, 1), "kind": "in-place u *= 1.0 over the field (torch)",
            "bytes": nbytes}


def run_xslab(args):
    """One x-slab's share of the distributed x sweep at the paper's 8-node
    split of the tumour-scale cube (1000^3 x 4 FP64), and the 8 slabs chained
    on one GPU.  The carries entering a slab are seeded values for the slab
    measured alone (any finite values exercise the same work)."""
    import torch
    import workloads
    import paper_2602_05017_amd as bf
    reps = 5 if args.steps is None else args.steps
    p = workloads.config(3, with_field=False)
    P, NB = 8, 16
    n, S = p.nx, p.S
    xb = [n * r // P for r in range(P + 1)]
    nl = p.ny * p.nz * S
    lb = [nl * b // NB for b in range(NB + 1)]
    g = bf.Grid(n, p.ny, p.nz, S, tuple(p.h), dtype="f64")
    g.set_params(p.D, p.lam, p.dt)
    # ---- one slab (a middle process), forward then backward over the blocks
    x0, x1 = xb[P // 2], xb[P // 2 + 1]
    m = x1 - x0
    gen = torch.Generator(device="cuda").manual_seed(p.seed)
    slab = torch.empty((p.nz, p.ny, m, S), dtype=torch.float64, device="cuda").uniform_(0.0, 1.0, generator=gen)
    cin = torch.empty(nl, dtype=torch.float64, device="cuda").uniform_(0.0, 1.0, generator=gen)
    cout = torch.empty(nl, dtype=torch.float64, device="cuda")

    def one_slab():
        for b in range(NB):
            g.xslab_forward(slab, x0, x1, lb[b], lb[b + 1], cin[lb[b]:], cout[lb[b]:])
        for b in range(NB):
            g.xslab_backward(slab, x0, x1, lb[b], lb[b + 1], cin[lb[b]:], cout[lb[b]:])

    one_slab()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        one_slab()
    e1.record()
    torch.cuda.synchronize()
    t_slab = e0.elapsed_time(e1) / reps
    elems = m * nl
    alg = 4 * 8 * elems                      # read + write in each direction
    # the same slab swept as a grid of its own (whole lines of 125, 2 moves)
    gs = bf.Grid(m, p.ny, p.nz, S, tuple(p.h), dtype="f64")
    gs.set_params(p.D, p.lam, p.dt)
    gs.sweep(slab, 0)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        gs.sweep(slab, 0)
    e1.record()
    torch.cuda.synchronize()
    t_whole_slab = e0.elapsed_time(e1) / reps
    gs.close()
    del slab, cin, cout
    torch.cuda.empty_cache()
    log(f"x-slab {m}x{p.ny}x{p.nz}x{S}: forward + backward over {NB} blocks {t_slab:.3f} ms "
        f"({alg / (t_slab * 1e-3) / 1e9:.0f} GB/s at 4 moves); as a grid of its own {t_whole_slab:.3f} ms")
    # ---- the 8 slabs chained on one GPU: one stream per slab, events for the
    # block hand-offs (forward slab r after slab r-1, backward after slab r+1)
    from paper_2602_05017_amd.slabs import chained_x_sweep
    u = torch.empty(p.shape, dtype=torch.float64, device="cuda")
    g.fill_uniform(u, p.seed, 0)
    slabs = [u[:, :, xb[r]:xb[r + 1], :].clone(memory_format=torch.contiguous_format) for r in range(P)]
    streams = [torch.cuda.Stream() for _ in range(P)]

    def chained():
        chained_x_sweep(g, slabs, xb, lb, streams)

    chained()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        chained()
    torch.cuda.synchronize()
    t_chain = (time.perf_counter() - t0) * 1e3 / reps
    # the whole-line x sweep of the cube for comparison
    g.sweep(u, 0)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        g.sweep(u, 0)
    e1.record()
    torch.cuda.synchronize()
    t_whole = e0.elapsed_time(e1) / reps
    g.close()
    upd = p.V * S
    log(f"8 slabs chained: {t_chain:.3f} ms per x sweep; whole-line x sweep {t_whole:.3f} ms")
    line = {
        "metric": "voxel-substrate updates/s of one x-slab's share of the distributed x sweep (FP64)",
        "value": elems / (t_slab * 1e-3), "unit": "voxel-substrate updates/s", "n_gpus": 1, "steps": reps,
        "warmup": 1, "ms_per_step": round(t_slab, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded uniform slab and carries)",
        "config": {"workload": f"xslab-{m}x{p.ny}x{p.nz}x{S}-of-1000^3x4-f64", "processes": P, "blocks": NB,
                   "slab": [x0, x1]},
        "roofline": {"bound": "hbm", "achieved": round(alg / (t_slab * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(alg / (t_slab * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4), "traffic": None,
                     "kernel": "k_xslab (forward + backward over the blocks)",
                     "algorithmic_bytes_per_step": alg},
        "slab_as_a_grid_ms": round(t_whole_slab, 4),
        "chained_8_slabs": {"ms_per_x_sweep": round(t_chain, 3), "updates_per_s": upd / (t_chain * 1e-3),
                            "whole_line_x_sweep_ms": round(t_whole, 3), "streams": P, "blocks": NB},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def run_ceiling(args):
    """Streaming ceilings of the device on a buffer the size of the
    1000^3 x 4 FP64 field (32 GB), with torch's vectorised kernels: write
    only (fill), read only (sum), in-place read+write (multiply by 1.0) and
    copy between two halves.  Each is timed with events over `steps` passes
    after one untimed pass.  A sweep reads and writes every element once,
    so the in-place read+write rate bounds what a sweep can reach."""
    import torch
    reps = 5 if args.steps is None else args.steps
    n = 1000 ** 3 * 4
    u = torch.empty(n, dtype=torch.float64, device="cuda")
    u.fill_(0.5)
    half = n // 2
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    nb = n * 8
    for name, fn, moved in (("write_only", lambda: u.fill_(0.5), nb), ("read_only", lambda: u.sum(), nb),
                            ("in_place_read_write", lambda: u.mul_(1.0), 2 * nb),
                            ("copy", lambda: u[half:].copy_(u[:half]), nb)):
        ms = timed(fn)
        gbps = moved / (ms * 1e-3) / 1e9
        out[name] = {"GBps": round(gbps, 1), "frac_of_peak": round(gbps / HBM_PEAK_GBPS, 4), "ms": round(ms, 3),
                     "bytes": moved}
        log(f"{name}: {gbps:.0f} GB/s ({gbps / HBM_PEAK_GBPS:.1%} of peak)")
    best = out["in_place_read_write"]["GBps"]
    line = {"metric": "HBM streaming ceiling (read+write in place)", "value": best, "unit": "GB/s", "n_gpus": 1,
            "steps": reps, "warmup": 1, "ms_per_step": out["in_place_read_write"]["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic (constant buffer)",
            "config": {"workload": "streaming ceilings on a 32 GB buffer (the 1000^3 x 4 FP64 field size)"},
            "roofline": {"bound": "hbm", "achieved": best, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": round(best / HBM_PEAK_GBPS, 4), "traffic": None},
            "patterns": out, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                                   "(no collectives, no sharding)"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "adjoint":
        run_adjoint(args)
        return
    if args.workload in ("liver4", "liver12", "liver16"):
        run_large(args)
        return
    if args.workload == "endtoend":
        run_endtoend(args)
        return
    if args.workload == "ceiling":
        run_ceiling(args)
        return
    if args.workload == "xslab":
        run_xslab(args)
        return
    if args.steps is None:
        args.steps = 20
    p = workload(args.workload)
    log(f"workload {p.name}: grid {p.nx}x{p.ny}x{p.nz}, S={p.S}, sources "
        f"{0 if p.src is None else len(p.src)}")
    u_host = torch.from_numpy(p.u0)
    upd_per_step = p.V * p.S

    g, u, t, stages, placement = timed_run(p, "f64", args.steps, args.warmup, u_host, args.placement_candidates)
    ms_per_step = 1e3 * t / args.steps
    value = upd_per_step * args.steps / t
    log(f"f64: {ms_per_step:.3f} ms/step, {value:.4g} updates/s")
    sweeps = {k: v for k, v in stages.items() if k.startswith("sweep")}
    # dominant kernel: the sweep with the largest share of the step
    dom = max(sweeps, key=lambda k: sweeps[k]["total_ms"])
    alg_bytes = int(2 * 8 * sweeps[dom]["elements_per_launch"])   # one read + one write per element
    achieved = alg_bytes / (sweeps[dom]["avg_ms"] * 1e-3) / 1e9
    traffic = traffic_record(args.workload, "f64", dom)
    sched = g.get_schedule()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": KERNEL_NAMES[dom], "algorithmic_bytes_per_launch": alg_bytes,
                "avg_launch_ms": round(sweeps[dom]["avg_ms"], 5),
                "launches_per_step": sweeps[dom]["launches"] // args.steps,
                "step_alg_GBps": round(3 * 2 * 8 * upd_per_step / (ms_per_step * 1e-3) / 1e9, 1),
                "step_frac": round(3 * 2 * 8 * upd_per_step / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                "schedule": {"fused_yz_slabs": sched[0] == 1, "slab_width": sched[1]},
                "stages_ms_per_step": {k: round(v["total_ms"] / args.steps, 4) for k, v in stages.items()}}
    roofline["practical_ceiling"] = rmw_ceiling(u)
    roofline["frac_of_practical_ceiling"] = round(roofline["step_alg_GBps"] / roofline["practical_ceiling"]["GBps"], 4)
    log(f"in-place read+write ceiling on the same field: {roofline['practical_ceiling']['GBps']:.0f} GB/s; "
        f"the step runs at {roofline['frac_of_practical_ceiling']:.1%} of it")
    lib_bytes = g.device_bytes()
    memory = {"field_bytes": upd_per_step * 8, "library_bytes": lib_bytes,
              "bytes_per_voxel_substrate": round((upd_per_step * 8 + lib_bytes) / upd_per_step, 3)}
    g.close()
    if placement is not None:
        placement["default_allocation_ms_per_step"] = default_allocation_ms(p, "f64")
        log(f"the same step on a plain allocation: {placement['default_allocation_ms_per_step']} ms")

    fp32 = None
    if not args.no_fp32:
        # the FP64 field stays resident: the FP32 runs are compared with it element by element
        for dtype in ("f32", "f32fast"):
            g32, u32, t32, st32, pl32 = timed_run(p, dtype, args.steps, args.warmup, u_host,
                                                  args.placement_candidates)
            v32 = upd_per_step * args.steps / t32
            s32 = {k: v for k, v in st32.items() if k.startswith("sweep")}
            d32 = max(s32, key=lambda k: s32[k]["total_ms"])
            ach32 = 2 * 4 * s32[d32]["elements_per_launch"] / (s32[d32]["avg_ms"] * 1e-3) / 1e9
            err = fp32_error(u32, u)
            rec = {"value": v32, "ms_per_step": round(1e3 * t32 / args.steps, 3),
                   "dtype": "f32 storage, f64 arithmetic" if dtype == "f32" else
                            "f32 storage, f32 arithmetic, f64-precomputed constants",
                   "dominant_kernel": KERNEL_NAMES[d32], "dominant_kernel_GBps": round(ach32, 1),
                   "frac": round(ach32 / HBM_PEAK_GBPS, 4),
                   "step_alg_GBps": round(3 * 2 * 4 * upd_per_step / (t32 / args.steps) / 1e9, 1),
                   "error_vs_f64": err, "placement": pl32,
                   "stages_ms_per_step": {k: round(v["total_ms"] / args.steps, 4) for k, v in st32.items()}}
            log(f"{dtype}: {rec['ms_per_step']} ms/step, {v32:.4g} updates/s, vs f64 e_max {err['e_max']:.2e} "
                f"e_2 {err['e_2']:.2e} (per substrate {err['e_max_per_substrate']})")
            g32.close()
            del u32
            torch.cuda.empty_cache()
            if dtype == "f32":
                fp32 = rec
            else:
                fp32["fp32_arithmetic"] = rec
    del u
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(p, args.cpu_sample_steps)
        log(f"oracle: {cpu['value']:.4g} updates/s on {cpu['cores']} threads")
        cpu["host"] = host_info()
        cpu["small_workloads"] = oracle_thread_runs()
        log(f"host {cpu['host']}; oracle on the small workloads: {json.dumps(cpu['small_workloads'])}")

    line = {
        "metric": "voxel-substrate updates/s per LOD step (FP64)",
        "value": value,
        "unit": "voxel-substrate updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded SplitMix64 inputs)",
        "config": {"workload": p.name, "grid": [p.nx, p.ny, p.nz], "substrates": p.S,
                   "sources": 0 if p.src is None else len(p.src),
                   "dirichlet": 0 if p.dr is None else len(p.dr), "dt_min": p.dt,
                   "h_um": list(map(float, p.h))},
        "roofline": roofline,
        "placement": placement,
        "fp32": fp32,
        "memory": memory,
        "cpu_baseline": cpu,
    }
    if args.workload == "liver":
        line["paper_context"] = PAPER_TABLE2_8PCT
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
