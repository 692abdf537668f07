"""Convergence on the GPU against the oracle (Sect. 2: the radiation field and
the level populations are iterated until the populations stop changing).

* the maximum relative population change the device reduces after every
  iteration (FP64, over entries >= 1e-10) against the oracle's, iteration by
  iteration, and the number of iterations each needs to reach a tolerance;
* runs to convergence at 1e-6 of the 1000-shell Plummer cloud and of a 32^3
  copy of the turbulent cube (the full-size cube is compared for a few
  iterations in test_gpu_parity).
Bars as in test_gpu_parity.
"""
import numpy as np
import pytest

import oracle
import synth

miloc = pytest.importorskip("paper_2009_12609_amd")

from test_gpu_parity import assert_pops, make_ctx, workload_1d_plummer, workload_3d  # noqa: E402

pytestmark = pytest.mark.gpu


def _deltas(ctx, n):
    out = []
    for _ in range(n):
        it, d = ctx.run(1)
        assert it == 1
        out.append(d)
    return np.array(out)


def _thick_small_1d():
    w = synth.workload_1d_small()
    w.model.abundance[:] = 1.0e-6            # line-centre depth ~6.6 through the cloud
    return w


def test_delta_per_iteration_1d_fp64():
    """Thick 100-shell cloud, FP64 march: every iteration's maximum relative
    change equals the oracle's, and one call with tol = 1e-6 stops after the
    oracle's iteration count."""
    w = _thick_small_1d()
    print("[case] delta per iteration, 1D thick, fp64", flush=True)
    ref = oracle.run_1d(w.mol, w.model, w.spec, w.T_bg, 300, tol=1e-6)
    d_ref = np.array([h["delta"] for h in ref.history])
    assert ref.iters >= 6 and d_ref[-1] < 1e-6 <= d_ref[-2]
    ctx = make_ctx(w, fp64=True)
    d = _deltas(ctx, ref.iters)
    err = np.abs(d - d_ref)
    print(f"[parity] 1D thick fp64 delta: {ref.iters} iterations, max |d - d_ref| / d_ref "
          f"{np.max(err / d_ref):.3e}", flush=True)
    assert np.all(err <= 1e-6 * d_ref + 1e-9)
    ctx.init_lte()
    it, last = ctx.run(500, tol=1e-6, allow_notconv=False)
    assert it == ref.iters
    assert abs(last - d_ref[-1]) <= 1e-6 * d_ref[-1] + 1e-9
    ctx.close()


def test_delta_per_iteration_3d_fp64():
    """Thick 9^3 turbulent cube, 48 directions, FP64 march: the device's
    maximum relative change per iteration against the oracle's."""
    w = workload_3d(9, seed=109, abundance=3e-7, box_pc=0.075, n_levels=5, nch=128)
    n = 6
    print("[case] delta per iteration, 3D 9^3 thick, fp64", flush=True)
    ref = oracle.run_3d(w.mol, w.model, w.spec, w.T_bg, n)
    d_ref = np.array([h["delta"] for h in ref.history])
    ctx = make_ctx(w, fp64=True)
    d = _deltas(ctx, n)
    print(f"[parity] 3D thick fp64 delta: max |d - d_ref| / d_ref {np.max(np.abs(d - d_ref) / d_ref):.3e}",
          flush=True)
    assert np.all(np.abs(d - d_ref) <= 1e-6 * d_ref + 1e-9)
    ctx.close()


def test_delta_per_iteration_1d_fp32():
    """FP32 march on the thick Plummer cloud: the maximum relative change
    follows the oracle's within the FP32 populations' own error, and the
    iterations to 1e-4 differ by at most one."""
    w = workload_1d_plummer(61, abundance=1e-6)
    print("[case] delta per iteration, 1D Plummer thick, fp32", flush=True)
    ref = oracle.run_1d(w.mol, w.model, w.spec, w.T_bg, 200, tol=1e-4)
    d_ref = np.array([h["delta"] for h in ref.history])
    ctx = make_ctx(w)
    d = _deltas(ctx, ref.iters)
    print(f"[parity] 1D thick fp32 delta: {ref.iters} iterations, max |d - d_ref| "
          f"{np.max(np.abs(d - d_ref)):.3e}", flush=True)
    assert np.all(np.abs(d - d_ref) <= 1e-3 * d_ref + 1e-6)
    ctx.init_lte()
    it, _ = ctx.run(500, tol=1e-4, allow_notconv=False)
    assert abs(it - ref.iters) <= 1
    ctx.close()


def test_plummer_full_size_to_convergence():
    """The 1000-shell Plummer cloud (10-level rotor, 256 channels, FP32 march)
    run to a maximum relative change of 1e-6, like the oracle."""
    w = workload_1d_plummer(1000)
    print("[case] 1d-plummer-1000 to 1e-6", flush=True)
    ref = oracle.run_1d(w.mol, w.model, w.spec, w.T_bg, 100, tol=1e-6, record=False)
    ctx = make_ctx(w)
    it, last = ctx.run(100, tol=1e-6, allow_notconv=False)
    print(f"[parity] 1d-plummer-1000 converged: gpu {it} iterations (delta {last:.2e}), oracle {ref.iters}",
          flush=True)
    assert abs(it - ref.iters) <= 1
    assert_pops(ctx.populations(), ref.x, 1e-5, "1d-plummer-1000 converged")
    ctx.close()


def test_cube_32_to_convergence():
    """A 32^3 copy of the turbulent cube (same generators, seed 3001, 1 pc *
    32/128 box so that cells keep their size), 48 directions, 256 channels,
    10-level rotor, FP32 march: populations at convergence (1e-6)."""
    w = workload_3d(32, seed=3001, box_pc=0.25)
    print("[case] 3d 32^3 to 1e-6", flush=True)
    ref = oracle.run_3d(w.mol, w.model, w.spec, w.T_bg, 60, tol=1e-6, record=False)
    ctx = make_ctx(w)
    it, last = ctx.run(60, tol=1e-6, allow_notconv=False)
    print(f"[parity] 3d-32 converged: gpu {it} iterations (delta {last:.2e}), oracle {ref.iters}", flush=True)
    assert abs(it - ref.iters) <= 1
    assert_pops(ctx.populations(), ref.x, 1e-5, "3d-32 converged")
    ctx.close()
