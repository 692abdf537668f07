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
timed on this host's cores on a bounded sample of the same workload.  Three
more objects by default: ``hyperfine`` (the same cube with a three-component
multiplet on every transition, 2 timed iterations), ``octree`` (64^3 root
refined four levels, 2 timed ALI iterations, same per-step measures) and
``serving`` (a 5000-request 1D stream: model solves/s with all requests queued
at once, p50/p99 latency under Poisson arrivals at 0.5x and 0.8x of that rate,
and the first 1024 of the same requests solved one at a time through a
single-model context).
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
FP32_PEAK_TFLOPS = 157.3
# The same vector units without packed FP32 (two FP32 lanes per instruction),
# which the library's kernels do not use: 256 CUs x 4 SIMDs x 16 lanes x 2
# (FMA) x 2.4 GHz.
FP32_UNPACKED_TFLOPS = 78.6
# The paper's GPU-vs-one-CPU-core speed-ups, with the hardware it states.
PAPER_SPEEDUPS = {
    "1d": "about 20x (abstract) to 23x (App. A.1, 2048 rays, 256 channels): NVIDIA GTX 1080 Ti "
          "against one core of an Intel i7-8700K",
    "3d_cartesian": "about 12.9x (App. A.2): AMD Radeon VII (external, Thunderbolt) against one "
                    "i7-8700K core; 6.0x for the 6-core CPU run",
    "3d_octree": "up to about 10x (abstract), hardware as above",
}
# Algorithmic bytes per ray-cell step of one transition: read the cell's
# {kappa, eta} (8 B) and {u/dv, dv/b} (16 B), read-modify-write the FP64
# {J, Lambda} accumulator pair (16 B, counted once).
BYTES_PER_STEP = 40.0
# Algorithmic FP32 operations per in-window channel update: profile argument
# (FMA, 2), its square (1), the exponential (1), tau (1), the escape series
# (3 FMA + 1, 7), e_c beta (FMA, 2), the two absorbed-count sums (2 FMA, 4),
# the intensity update (2 FMA, 4).
FLOPS_PER_CHANNEL = 22.0
WINDOW_K = 5.0                # Doppler widths on each side (FP32 march)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "march3d_regular_128_traffic.json")
OCT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "march_oct_64root_L4_traffic.json")


def off32_tables(w) -> bool:
    """Whether the FP32 regular-grid march addresses the cube's tables with
    32-bit offsets (the launch's own test: fewer than 2^24 cells, tables
    below 4 GB, MILOC_WIDE_OFFSETS unset)."""
    nc = int(w.model.n_cells)
    return (nc < 2 ** 24 and nc * 16 < 2 ** 32 and nc * int(w.mol.n_trans) * 8 < 2 ** 32
            and "MILOC_WIDE_OFFSETS" not in os.environ)


def mean_window_channels(w) -> float:
    """Mean number of channels in a step's window: 2 K b / dv per cell,
    clipped to the band (every cell is crossed about equally often)."""
    import numpy as np
    m = w.model
    AMU, KB = 1.66053906660e-24, 1.380649e-16
    b = np.sqrt(2 * KB * m.T_kin.astype(float) / (w.mol.mass_amu * AMU) + m.b_turb.astype(float) ** 2)
    return float(np.mean(np.minimum(w.spec.n_channels, 2 * WINDOW_K * b / w.spec.dv)))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "miloc_internal.h"):
        with open(os.path.join(ROOT, "paper_2009_12609_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_counters(src_hash, path=TRAFFIC_FILE):
    """From the committed rocprofv3 counter runs of a march kernel, only if
    they were taken on the current kernel source: (HBM bytes per launch,
    VALU-busy fraction of the launch), else (None, None)."""
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None, None
    if d.get("kernel_source_hash") != src_hash:
        return None, None
    return d.get("bytes_per_launch"), d.get("valu_busy")


def host_cpu() -> dict:
    """The host the oracle ran on: CPU model (from /proc/cpuinfo), hardware
    threads the OS reports, and those this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"cpu_model": model, "os_threads": os.cpu_count(), "usable_threads": usable}


def cpu_baseline(w, budget_s=8.0, gpu_value=None):
    """Oracle (FP64, all channels) on the same cube, one transition (J=1-0):
    on all host threads, directions added one at a time until ~budget_s of
    wall time; on one thread, one direction (the paper's speed-ups are against
    one CPU core)."""
    import numpy as np

    import oracle
    m = w.model
    N = int(m.n0[0])
    prob = oracle._Problem(w.mol, m.n_H2, m.T_kin, m.b_turb, m.abundance, w.spec, w.T_bg)
    x0 = oracle.lte_populations(w.mol, prob.T)
    kap, eta = oracle.prepare(w.mol, x0, prob.n_mol)
    vx, vy, vz = (np.asarray(a, dtype=np.float64) for a in (m.vx, m.vy, m.vz))
    dirs = oracle.healpix_nside2()

    def run(threads, max_dirs, budget):
        t_total, updates, used = 0.0, 0.0, 0
        for q in range(min(max_dirs, dirs.shape[0])):
            cells, _, _ = oracle.walk_3d(N, dirs[q], 0, 0)
            t0 = time.perf_counter()
            oracle.march_3d(N, m.root_cell_cm, vx, vy, vz, prob.bD, kap[0], eta[0], dirs[q:q + 1],
                            w.spec, prob.I_bg[0], n_threads=threads)
            t_total += time.perf_counter() - t0
            updates += float(len(cells)) * N * N * w.spec.n_channels
            used += 1
            if t_total >= budget:
                break
        return updates / t_total, used, t_total

    v_all, used_all, t_all = run(0, 48, budget_s)
    v_one, used_one, t_one = run(1, 1, 0.0)
    out = {"value": v_all, "unit": "ray-cell-channel updates/s",
           "cores": oracle.max_threads(), "kind": "oracle",
           "sample": f"FP64 oracle march of transition J=1-0 along {used_all} of 48 directions of the "
                     f"full {N}^3 cube, all {w.spec.n_channels} channels ({t_all:.1f} s)",
           "one_thread": {"value": v_one, "cores": 1,
                          "sample": f"as above on one thread, {used_one} direction ({t_one:.1f} s)"},
           "paper_gpu_vs_one_core": PAPER_SPEEDUPS,
           "host": host_cpu()}
    if gpu_value:
        out["gpu_vs_one_thread"] = gpu_value / v_one
        out["gpu_vs_all_threads"] = gpu_value / v_all
    return out


OCT_BYTES_PER_STEP = 48.0     # the regular step's 40 B plus the 8 B step record


def alu_view(tflops, valu_busy, nwin, flops_per_channel=FLOPS_PER_CHANNEL):
    """The same launch as useful FP32 vector work against the packed and the
    unpacked FP32 peaks, with the measured VALU-busy fraction."""
    return {"achieved": tflops, "unit": "TFLOP/s", "peak_unpacked": FP32_UNPACKED_TFLOPS,
            "frac_unpacked": tflops / FP32_UNPACKED_TFLOPS, "peak_packed": FP32_PEAK_TFLOPS,
            "frac_packed": tflops / FP32_PEAK_TFLOPS, "valu_busy": valu_busy,
            "flops_per_channel_update": flops_per_channel, "window_channels_mean": nwin}


def octree_bench(steps=2, warmup=1):
    """Octree leg: 64^3 root, four refinement levels (about 2e7 leaves), 10-level
    rotor, 48 directions, 256 channels; ALI iterations with the inputs resident
    and the ray schedules built (outside the timed region)."""
    import paper_2009_12609_amd as miloc
    import synth

    t0 = time.perf_counter()
    w = synth.workload_octree()
    t_gen = time.perf_counter() - t0
    ctx = miloc.Context(0)
    ctx.load_molecule(w.mol)
    ctx.load_model_3d(w.model)
    ctx.set_spectral(w.spec.n_channels, w.spec.v_min, w.spec.dv)
    ctx.set_background(w.T_bg)
    t0 = time.perf_counter()
    ctx.init_lte()
    ctx.run(max(1, warmup))              # builds the ray schedules, then warm-up iterations
    t_setup = time.perf_counter() - t0
    ctx.init_lte()
    ctx.reset_counters()
    t0 = time.perf_counter()
    ctx.run(steps)
    elapsed = time.perf_counter() - t0
    cnt = ctx.counters()
    ctx.close()
    launches = max(1, cnt["march_launches"])
    march_ms = cnt["march_ms"] / launches
    steps_per_launch = cnt["ray_steps"] / launches
    hbm_gbs = steps_per_launch * OCT_BYTES_PER_STEP / (march_ms * 1e-3) / 1e9
    nwin = mean_window_channels(w)
    traffic, valu_busy = measured_counters(kernel_source_hash(), OCT_TRAFFIC_FILE)
    alu_tflops = steps_per_launch * nwin * FLOPS_PER_CHANNEL / (march_ms * 1e-3) / 1e12
    return {
        "metric": "ray-cell-channel updates/s (3D octree)",
        "value": cnt["channel_updates"] / elapsed,
        "unit": "ray-cell-channel updates/s",
        "steps": steps,
        "ms_per_step": elapsed * 1e3 / steps,
        "workload": w.name,
        "n_cells_per_level": list(map(int, w.model.n_cells_per_level)),
        "ray_cell_steps_per_iteration": cnt["ray_steps"] / max(1, cnt["iterations"]),
        "march_ms_per_launch": march_ms,
        "solve_ms_per_step": cnt["solve_ms"] / max(1, cnt["iterations"]),
        "setup_s": t_setup,
        "generate_s": t_gen,
        "roofline": {"bound": "hbm", "achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": hbm_gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"march_oct_kernel<float,{cnt['march_lanes']},true,false>",
                     "bytes_per_step": OCT_BYTES_PER_STEP, "steps_per_launch": steps_per_launch,
                     "alu_view": alu_view(alu_tflops, valu_busy, nwin)},
    }


# Synthetic hyperfine multiplet (LTE between the components): offsets and
# relative strengths, the same on every transition of the hyperfine leg.
HF_OFFSETS_KMS = (-0.62, 0.0, 0.37)
HF_STRENGTHS = (1.0, 5.0, 3.0)
# Per in-window channel with K components: the single line's 22 operations
# less its profile (argument FMA, square, exponential: 4) plus, per component,
# the shifted argument (FMA, 2), its square (1), the exponential (1) and the
# weighted sum (FMA, 2).
def hf_flops_per_channel(k):
    return FLOPS_PER_CHANNEL - 4.0 + 6.0 * k


def hyperfine_bench(w, steps=2, warmup=1):
    """Hyperfine leg: the headline cube and species with a three-component
    multiplet on every transition (each channel's profile is the sum of three
    shifted Gaussians, windows widened by the offset range)."""
    import numpy as np

    import paper_2009_12609_amd as miloc
    m = w.model
    ctx = miloc.Context(0)
    ctx.load_molecule(w.mol)
    ctx.load_model_3d(m)
    ctx.set_spectral(w.spec.n_channels, w.spec.v_min, w.spec.dv)
    ctx.set_background(w.T_bg)
    off = np.array(HF_OFFSETS_KMS) * 1e5
    for t in range(int(w.mol.n_trans)):
        ctx.set_hyperfine(t, off, np.array(HF_STRENGTHS))
    ctx.init_lte()
    ctx.run(max(1, warmup))
    ctx.init_lte()
    ctx.reset_counters()
    t0 = time.perf_counter()
    ctx.run(steps)
    elapsed = time.perf_counter() - t0
    cnt = ctx.counters()
    ctx.close()
    launches = max(1, cnt["march_launches"])
    march_ms = cnt["march_ms"] / launches
    steps_per_launch = cnt["ray_steps"] / launches
    k = len(HF_OFFSETS_KMS)
    nwin = mean_window_channels(w) + (max(HF_OFFSETS_KMS) - min(HF_OFFSETS_KMS)) * 1e5 / w.spec.dv
    fpc = hf_flops_per_channel(k)
    alu_tflops = steps_per_launch * nwin * fpc / (march_ms * 1e-3) / 1e12
    hbm_gbs = steps_per_launch * BYTES_PER_STEP / (march_ms * 1e-3) / 1e9
    return {
        "metric": "ray-cell-channel updates/s (3D, hyperfine multiplets)",
        "value": cnt["channel_updates"] / elapsed,
        "unit": "ray-cell-channel updates/s",
        "steps": steps,
        "ms_per_step": elapsed * 1e3 / steps,
        "workload": f"{w.name} with a {k}-component multiplet on every transition",
        "components_kms": list(HF_OFFSETS_KMS),
        "strengths": list(HF_STRENGTHS),
        "march_ms_per_launch": march_ms,
        "solve_ms_per_step": cnt["solve_ms"] / max(1, cnt["iterations"]),
        "roofline": {"bound": "hbm", "achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": hbm_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"march3d_kernel<float,{cnt['march_lanes']},true,true>",
                     "bytes_per_step": BYTES_PER_STEP, "steps_per_launch": steps_per_launch,
                     "alu_view": alu_view(alu_tflops, None, nwin, fpc)},
    }


def lattice_bench(steps=2, warmup=1, n_refine=2):
    """Octree rays compared on a shallow tree: the same 64^3-root cloud refined
    n_refine levels, marched with the scheme's created and ended rays and with
    the brute-force lattice of 4^n_refine straight lines per root element."""
    import paper_2009_12609_amd as miloc
    import synth

    w = synth.workload_octree(n_refine=n_refine)
    out = {"workload": w.name, "n_cells_per_level": list(map(int, w.model.n_cells_per_level)), "steps": steps}
    for name, lattice in (("scheme", False), ("lattice", True)):
        ctx = miloc.Context(0)
        ctx.load_molecule(w.mol)
        ctx.load_model_3d(w.model)
        ctx.set_spectral(w.spec.n_channels, w.spec.v_min, w.spec.dv)
        ctx.set_background(w.T_bg)
        ctx.set_octree_rays(lattice)
        ctx.init_lte()
        ctx.run(max(1, warmup))
        ctx.init_lte()
        ctx.reset_counters()
        t0 = time.perf_counter()
        ctx.run(steps)
        elapsed = time.perf_counter() - t0
        cnt = ctx.counters()
        ctx.close()
        launches = max(1, cnt["march_launches"])
        out[name] = {"ms_per_step": elapsed * 1e3 / steps,
                     "march_ms_per_launch": cnt["march_ms"] / launches,
                     "gather_ms_per_step": cnt["accumulate_ms"] / max(1, cnt["iterations"]),
                     "ray_cell_steps_per_iteration": cnt["ray_steps"] / max(1, cnt["iterations"]),
                     "updates_per_s": cnt["channel_updates"] / elapsed}
    return out


def subiter_bench(n_sub=3, tau_min=0.1, tol=1e-6, max_iter=500):
    """Core sub-iterations on the thick variant of the 1000-shell Plummer
    cloud (abundance 1e-6, line-centre depth ~60 through the centre): wall
    time and iterations to a maximum relative change of tol, plain ALI and
    with n_sub sub-iterations per iteration in the core whose radial depth to
    the surface reaches tau_min."""
    import paper_2009_12609_amd as miloc
    import synth

    w = synth.workload_1d_plummer(n_shells=1000, abundance=1.0e-6)
    out = {"workload": f"{w.name} with abundance 1e-6 (thick), to {tol:g}", "n_sub": n_sub, "tau_min": tau_min}
    for name, ns in (("plain", 0), ("one_subiteration", 1), ("subiterations", n_sub)):
        ctx = miloc.Context(0)
        ctx.load_molecule(w.mol)
        ctx.load_model_1d(w.model)
        ctx.set_spectral(w.spec.n_channels, w.spec.v_min, w.spec.dv)
        ctx.set_background(w.T_bg)
        ctx.set_subiterations(ns, tau_min)
        ctx.run(1)                      # geometry and buffers, outside the timing
        ctx.init_lte()
        ctx.reset_counters()
        t0 = time.perf_counter()
        it, d = ctx.run(max_iter, tol=tol)
        el = time.perf_counter() - t0
        cnt = ctx.counters()
        ctx.close()
        out[name] = {"iterations": it, "last_delta": d, "wall_s": el,
                     "ray_cell_steps": cnt["ray_steps"], "march_ms": cnt["march_ms"]}
    out["speedup"] = out["plain"]["wall_s"] / out["subiterations"]["wall_s"]
    out["speedup_one"] = out["plain"]["wall_s"] / out["one_subiteration"]["wall_s"]
    return out


def batching_bench(steps=5):
    """1D march layouts on the 1000-shell Plummer cloud (10-level rotor, 256
    channels, FP32): every (ray, transition) pair on its own, and all
    transitions of a ray in one pass sharing its steps and line profile."""
    import paper_2009_12609_amd as miloc
    import synth

    w = synth.workload_1d_plummer(n_shells=1000)
    out = {"workload": w.name, "steps": steps}
    for name, on in (("per_transition", False), ("all_transitions", True)):
        ctx = miloc.Context(0)
        ctx.load_molecule(w.mol)
        ctx.load_model_1d(w.model)
        ctx.set_spectral(w.spec.n_channels, w.spec.v_min, w.spec.dv)
        ctx.set_background(w.T_bg)
        ctx.set_transition_batching(on)
        ctx.run(1)
        ctx.init_lte()
        ctx.reset_counters()
        t0 = time.perf_counter()
        ctx.run(steps)
        el = time.perf_counter() - t0
        cnt = ctx.counters()
        ctx.close()
        out[name] = {"ms_per_iteration": el * 1e3 / steps, "march_ms_per_iteration": cnt["march_ms"] / steps,
                     "march_updates_per_s": cnt["channel_updates"] / (cnt["march_ms"] * 1e-3)}
    out["march_speedup"] = (out["per_transition"]["march_ms_per_iteration"] /
                            out["all_transitions"]["march_ms_per_iteration"])
    return out


def _pct(a, q):
    import numpy as np
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def serve_bench(n_req=5000, seed=5001, tol=1e-6, max_iter=500, alone_sample=1024):
    """1D request stream (50-2000 shells, 2/5/10/20 levels, 64/128/256
    channels): model solves/s with every request queued at once (arrival rate
    far above capacity), p50/p99 latency at 0.5x and 0.8x of that capacity
    with Poisson arrivals, and the first `alone_sample` requests of the same
    stream solved one at a time through a single-model context."""
    import numpy as np

    import paper_2009_12609_amd as miloc
    import synth

    reqs = synth.serving_stream(n_req, seed=seed)
    srv = miloc.Server(0, hbm_budget_bytes=8 << 30, max_slots=256)
    # warm-up: one small request through the whole loop
    w0 = synth.serving_stream(1, seed=seed + 99, shells=(50, 50))[0]
    t_w = srv.submit(w0.mol, w0.model, w0.spec, w0.T_bg, tol, max_iter)
    if not srv.wait(t_w, 120.0):
        raise RuntimeError("serving warm-up request did not finish")
    srv.take(t_w)

    def run_stream(rate):
        t_start = time.perf_counter()
        tickets = []
        gaps = np.diff([0.0] + [r.arrival_s for r in reqs]) if rate else None
        t_next = t_start
        for i, r in enumerate(reqs):
            if rate:
                t_next += gaps[i] * (100.0 / rate)        # stream drawn at 100/s, rescaled
                dt = t_next - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            tickets.append(srv.submit(r.mol, r.model, r.spec, r.T_bg, tol, max_iter))
        lat, iters, bad = [], [], 0
        for t in tickets:
            if not srv.wait(t, 600.0):
                raise RuntimeError("serving request did not finish")
            _, _, info, rc = srv.take(t)
            bad += rc != miloc.OK
            lat.append(info["latency_s"])
            iters.append(info["iterations"])
        return time.perf_counter() - t_start, lat, iters, bad

    st0 = srv.stats()
    el_sat, lat_sat, iters, bad = run_stream(None)
    cap = n_req / el_sat
    st = srv.stats()
    ticks_sat = st["ticks"] - st0["ticks"]
    busy_sat = st["busy_s"] - st0["busy_s"]
    lat_runs = {}
    for f in (0.5, 0.8):
        el, lat, _, b = run_stream(f * cap)
        bad += b
        lat_runs[f"{f:g}x"] = {"rate_per_s": f * cap, "p50_s": _pct(lat, 50), "p99_s": _pct(lat, 99)}
    srv.close()

    # one model at a time on the same GPU, same requests, one reused context
    ctx = miloc.Context(0)
    ctx.load_molecule(w0.mol)
    ctx.load_model_1d(w0.model)
    ctx.set_spectral(w0.spec.n_channels, w0.spec.v_min, w0.spec.dv)
    ctx.run(max_iter, tol=tol)
    t0 = time.perf_counter()
    lat1 = []
    n_alone = min(n_req, alone_sample)
    for r in reqs[:n_alone]:
        ts = time.perf_counter()
        ctx.load_molecule(r.mol)
        ctx.load_model_1d(r.model)
        ctx.set_spectral(r.spec.n_channels, r.spec.v_min, r.spec.dv)
        ctx.set_background(r.T_bg)
        ctx.run(max_iter, tol=tol)
        for t in range(r.mol.n_trans):
            ctx.spectra(t, impact=np.array([0.0]))
        ctx.populations()
        lat1.append(time.perf_counter() - ts)
    el1 = time.perf_counter() - t0
    ctx.close()
    return {
        "metric": "model solves/s (1D batched, to 1e-6)",
        "value": cap,
        "unit": "solves/s",
        "requests": n_req,
        "failed": int(bad),
        "mean_iterations": float(np.mean(iters)),
        "saturation_s": el_sat,
        "saturation_ticks": int(ticks_sat),
        "saturation_tick_s": busy_sat,
        "peak_resident": int(st["peak_active"]),
        "latency": lat_runs,
        "one_at_a_time": {"value": n_alone / el1, "p50_service_s": _pct(lat1, 50),
                          "requests": n_alone, "sample": f"the first {n_alone} requests of the stream"},
        "speedup": cap / (n_alone / el1),
        "stream": f"seed {seed}: shells U[50,2000], levels {{2,5,10,20}}, channels {{64,128,256}}, +-2 km/s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=128, help="grid size (128 = the benchmark workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", type=int, default=5000, metavar="N_REQ",
                    help="run the 1D request stream with N_REQ requests ('serving' object; 0 = skip)")
    ap.add_argument("--octree", type=int, default=2, metavar="STEPS",
                    help="time STEPS iterations of the octree workload ('octree' object; 0 = skip)")
    ap.add_argument("--hyperfine", type=int, default=2, metavar="STEPS",
                    help="time STEPS iterations of the headline cube with hyperfine multiplets "
                         "('hyperfine' object; 0 = skip)")
    ap.add_argument("--lattice", type=int, default=0, metavar="STEPS",
                    help="time STEPS iterations of a two-level octree with the scheme's rays and with the "
                         "brute-force lattice ('lattice' object; 0 = skip, the default)")
    ap.add_argument("--subiter", type=int, default=3, metavar="N_SUB",
                    help="thick 1000-shell cloud to 1e-6 with and without N_SUB core sub-iterations "
                         "('subiterations' object; 0 = skip)")
    ap.add_argument("--batching", type=int, default=5, metavar="STEPS",
                    help="1000-shell cloud, STEPS iterations per 1D march layout ('batching' object; 0 = skip)")
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
        print("bench.py: the library runs on exactly one GPU; --gpus must be 1 "
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
    hbm_gbs = bytes_per_launch / (march_ms * 1e-3) / 1e9
    nwin = mean_window_channels(w)
    flops_per_launch = steps_per_launch * nwin * FLOPS_PER_CHANNEL
    alu_tflops = flops_per_launch / (march_ms * 1e-3) / 1e12
    src_hash = kernel_source_hash()
    traffic, valu_busy = measured_counters(src_hash)

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
            "gather_ms_per_step": cnt["accumulate_ms"] / max(1, cnt["iterations"]),
            "solve_ms_per_step": cnt["solve_ms"] / max(1, cnt["iterations"]),
            "march_updates_per_s": updates / (cnt["march_ms"] * 1e-3),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": hbm_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": hbm_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": f"march3d_f32_kernel<{cnt['march_lanes']},true,{str(off32_tables(w)).lower()}>",
            "bytes_per_step": BYTES_PER_STEP,
            "steps_per_launch": steps_per_launch,
            "march_ms_per_launch": march_ms,
            "alu_view": alu_view(alu_tflops, valu_busy, nwin),
            "kernel_source_hash": src_hash,
        },
    }
    ctx.close()
    if args.hyperfine > 0:
        out["hyperfine"] = hyperfine_bench(w, args.hyperfine)
    if args.octree > 0:
        out["octree"] = octree_bench(args.octree)
    if args.lattice > 0:
        out["lattice"] = lattice_bench(args.lattice)
    if args.subiter > 0:
        out["subiterations"] = subiter_bench(args.subiter)
    if args.batching > 0:
        out["batching"] = batching_bench(args.batching)
    if args.serve > 0:
        out["serving"] = serve_bench(args.serve)
    if not args.no_cpu_baseline and N == 128:
        out["cpu_baseline"] = cpu_baseline(w, gpu_value=out["config"]["march_updates_per_s"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
