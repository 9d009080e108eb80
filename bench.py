#!/usr/bin/env python3
"""Benchmark of the LOD diffusion-decay step on one MI355X.

Workload (default): the tumour-scale single-GPU share, 1000^3 voxels x 4
substrates in FP64 (32 GB field), D log-uniform in [1e3, 1e5] um^2/min,
lambda in [0.01, 0.1] /min, dt = 0.01 min, 1e6 source/sink voxels; the
paper's "8% liver" cube (Table 1) at 10 um resolution.  One step = Src,
Dir x4 (none in this workload), x, y and z Thomas sweeps.

Prints ONE JSON line: voxel-substrate updates/s per LOD step, the roofline
of the dominant kernel (algorithmic HBM bytes per launch / its mean launch
time from HIP events on the grid's stream, against the 8 TB/s HBM peak),
the same step with FP32 storage, and the FP64 oracle timed on the host on a
bounded sample of the workload.
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="liver", choices=["liver", "cells", "gaussian"])
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-storage companion run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=1)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 4 GiB buffer twice (reference for FETCH_SIZE / WRITE_SIZE counters)")
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


def timed_run(p, dtype, steps, warmup, u_host):
    """Warm up, reload the field, then time `steps` steps; per-stage HIP-event times."""
    import torch
    g = make_grid(p, dtype)
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
    return g, u, t, stages


def traffic_record(workload_name, dtype, kernel_stage):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload_name}_{dtype}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2602_05017_amd", "csrc", "sweep.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("sweep_src_sha256") != sha:
        return None
    k = rec.get("kernels", {}).get(kernel_stage)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


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


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(no collectives, no sharding)"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    p = workload(args.workload)
    log(f"workload {p.name}: grid {p.nx}x{p.ny}x{p.nz}, S={p.S}, sources "
        f"{0 if p.src is None else len(p.src)}")
    u_host = torch.from_numpy(p.u0)
    upd_per_step = p.V * p.S

    g, u, t, stages = timed_run(p, "f64", args.steps, args.warmup, u_host)
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
                "schedule": {"fused_yz_slabs": sched[0] == 1, "slab_width": sched[1]},
                "stages_ms_per_step": {k: round(v["total_ms"] / args.steps, 4) for k, v in stages.items()}}
    fp64_ref = u[..., 0].flatten()[:: 997].double().cpu() if not args.no_fp32 else None
    g.close()
    del u
    torch.cuda.empty_cache()

    fp32 = None
    if not args.no_fp32:
        g32, u32, t32, st32 = timed_run(p, "f32", args.steps, args.warmup, u_host)
        v32 = upd_per_step * args.steps / t32
        s32 = {k: v for k, v in st32.items() if k.startswith("sweep")}
        d32 = max(s32, key=lambda k: s32[k]["total_ms"])
        ach32 = 2 * 4 * s32[d32]["elements_per_launch"] / (s32[d32]["avg_ms"] * 1e-3) / 1e9
        samp = u32[..., 0].flatten()[:: 997].double().cpu()
        err = float((samp - fp64_ref).abs().max() / fp64_ref.abs().max())
        fp32 = {"value": v32, "ms_per_step": round(1e3 * t32 / args.steps, 3),
                "dtype": "f32 storage, f64 arithmetic",
                "dominant_kernel_GBps": round(ach32, 1), "frac": round(ach32 / HBM_PEAK_GBPS, 4),
                "max_rel_diff_vs_f64_sampled": err}
        log(f"f32: {fp32['ms_per_step']} ms/step, {v32:.4g} updates/s, sampled diff vs f64 {err:.2e}")
        g32.close()
        del u32
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(p, args.cpu_sample_steps)
        log(f"oracle: {cpu['value']:.4g} updates/s on {cpu['cores']} threads")

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
        "fp32": fp32,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
