#!/usr/bin/env python3
"""Benchmark of the ALI ray march on one MI355X.

Workload (default): the 128^3 turbulent cloud (lognormal density sigma_ln = 1,
mean 1e3 cm^-3, solenoidal k^-4 velocity, rms 1 km/s, 15 K), 10-level linear
rotor (9 transitions), 48 HEALPix directions with one ray per surface cell,
256 channels over +-4 km/s.  One step = one full ALI iteration (prepare ->
ray march of all transitions -> FP64 equilibrium solve -> convergence test);
the timed region is K steps followed by the final +z spectral map of the
J=1-0 line, with every input already resident on the device.

Prints one JSON line.  ``value`` = nominal ray-cell-channel updates per second
of the whole timed region (every channel counted, including those outside
each step's profile window).  ``roofline`` describes the dominant kernel (the
3D march) from its HIP-event durations; ``cpu_baseline`` is the FP64 oracle
timed on this host's cores on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per ray-cell step of one transition: read the cell's
# {kappa, eta} (8 B) and {u/dv, dv/b} (16 B), read-modify-write the FP64
# {J, Lambda} accumulator pair (16 B, counted once).
BYTES_PER_STEP = 40.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "march3d_regular_128_traffic.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "miloc_internal.h"):
        with open(os.path.join(ROOT, "paper_2009_12609_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(src_hash):
    """HBM bytes per march launch from the committed rocprofv3 counter runs,
    only if they were taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != src_hash:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(w, budget_s=15.0):
    """Oracle (FP64, all channels) on the same cube, one transition (J=1-0),
    directions added one at a time until ~budget_s of wall time."""
    import numpy as np

    import oracle
    m = w.model
    N = int(m.n0[0])
    prob = oracle._Problem(w.mol, m.n_H2, m.T_kin, m.b_turb, m.abundance, w.spec, w.T_bg)
    x0 = oracle.lte_populations(w.mol, prob.T)
    kap, eta = oracle.prepare(w.mol, x0, prob.n_mol)
    vx, vy, vz = (np.asarray(a, dtype=np.float64) for a in (m.vx, m.vy, m.vz))
    dirs = oracle.healpix_nside2()
    t_total = 0.0
    updates = 0.0
    used = 0
    for q in range(dirs.shape[0]):
        cells, _, _ = oracle.walk_3d(N, dirs[q], 0, 0)
        t0 = time.perf_counter()
        oracle.march_3d(N, m.root_cell_cm, vx, vy, vz, prob.bD, kap[0], eta[0], dirs[q:q + 1],
                        w.spec, prob.I_bg[0])
        t_total += time.perf_counter() - t0
        updates += float(len(cells)) * N * N * w.spec.n_channels
        used += 1
        if t_total >= budget_s:
            break
    return {"value": updates / t_total, "unit": "ray-cell-channel updates/s",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"FP64 oracle march of transition J=1-0 along {used} of 48 directions of the "
                      f"full {N}^3 cube, all {w.spec.n_channels} channels ({t_total:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=128, help="grid size (128 = the benchmark workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy kernel (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = 1 << 28                      # 2^28 float32 = 1 GiB read + 1 GiB written
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}))
        return
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU; --gpus must be 1 "
              "(the multi-GPU sharding is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)

    import paper_2009_12609_amd as miloc
    import synth

    w = synth.workload_3d_regular(N=args.N)
    m = w.model
    N = int(m.n0[0])
    ctx = miloc.Context(0)
    ctx.load_molecule(w.mol)
    ctx.load_model_3d(m)
    ctx.set_spectral(w.spec.n_channels, w.spec.v_min, w.spec.dv)
    ctx.set_background(w.T_bg)
    ctx.init_lte()
    if args.warmup > 0:
        ctx.run(args.warmup)
        ctx.spectra(0, n_los=N * N)
    ctx.init_lte()
    ctx.reset_counters()

    t0 = time.perf_counter()
    ctx.run(args.steps)                 # returns after the stream has drained
    ctx.spectra(0, n_los=N * N)         # final LOS map, copied to the host
    elapsed = time.perf_counter() - t0

    cnt = ctx.counters()
    updates = cnt["channel_updates"]
    launches = max(1, cnt["march_launches"])
    march_ms = cnt["march_ms"] / launches
    steps_per_launch = cnt["ray_steps"] / launches
    bytes_per_launch = steps_per_launch * BYTES_PER_STEP
    achieved = bytes_per_launch / (march_ms * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    traffic = measured_traffic(src_hash)

    out = {
        "metric": "ray-cell-channel updates/s (3D)",
        "value": updates / elapsed,
        "unit": "ray-cell-channel updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"3d-regular-{N}^3-rotor10-48dir-256ch",
            "n_cells": N ** 3,
            "n_directions": 48,
            "n_transitions": int(w.mol.n_trans),
            "n_channels": int(w.spec.n_channels),
            "ray_cell_steps_per_iteration": cnt["ray_steps"] / max(1, cnt["iterations"]),
            "march": "FP32 intensities, FP64 accumulation, FP64 equilibrium solve",
            "march_ms_per_launch": march_ms,
            "prepare_ms_per_step": cnt["prepare_ms"] / max(1, cnt["iterations"]),
            "solve_ms_per_step": cnt["solve_ms"] / max(1, cnt["iterations"]),
            "march_updates_per_s": updates / (cnt["march_ms"] * 1e-3),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "march3d_kernel<float,32,true>",
            "bytes_per_step": BYTES_PER_STEP,
            "kernel_source_hash": src_hash,
        },
    }
    if not args.no_cpu_baseline and N == 128:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
