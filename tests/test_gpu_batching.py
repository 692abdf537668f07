"""All transitions of a 1D ray in one pass (miloc_set_transition_batching):
the same results as the per-transition march and the oracle.  Bars as in
test_gpu_parity."""
import numpy as np
import pytest

import oracle
import synth

miloc = pytest.importorskip("paper_2009_12609_amd")

from test_gpu_parity import assert_pops, make_ctx, workload_1d_plummer  # noqa: E402

pytestmark = pytest.mark.gpu


def test_batched_fp64_iteration_by_iteration():
    """100 log shells with a 6-level rotor (5 transitions: two wavefront
    groups, the second with one live transition), FP64."""
    w = synth.workload_1d_small()
    w.mol = synth.rotor_molecule(6)
    w.model.abundance[:] = 1e-7
    ref = oracle.run_1d(w.mol, w.model, w.spec, w.T_bg, 5)
    ctx = make_ctx(w, fp64=True)
    ctx.set_transition_batching(True)
    for it in range(5):
        ctx.run(1)
        assert_pops(ctx.populations(), ref.history[it]["x"], 1e-10, f"batched fp64 it {it}")
    J, Lam = ctx.radiation()
    assert np.allclose(J, ref.history[-1]["J"], rtol=1e-10, atol=0)
    assert np.allclose(Lam, ref.history[-1]["Lam"], rtol=1e-9, atol=1e-20)
    ctx.close()


@pytest.mark.parametrize("n_shells,abundance,n_iter", [(157, 1e-9, 10), (61, 1e-6, 8)])
def test_batched_fp32_plummer(n_shells, abundance, n_iter):
    w = workload_1d_plummer(n_shells, abundance)
    ref = oracle.run_1d(w.mol, w.model, w.spec, w.T_bg, n_iter)
    ctx = make_ctx(w)
    ctx.set_transition_batching(True)
    ctx.run(n_iter)
    assert_pops(ctx.populations(), ref.x, 1e-5, f"batched fp32 plummer-{n_shells}")
    J, Lam = ctx.radiation()
    h = ref.history[-1]
    assert np.allclose(J, h["J"], rtol=2e-5, atol=0)
    assert np.allclose(Lam, h["Lam"], rtol=2e-5, atol=1e-9)
    plain = make_ctx(w)
    plain.run(n_iter)
    assert_pops(ctx.populations(), plain.populations(), 1e-6, "batched vs per-transition")
    ctx.close()
    plain.close()


def test_batched_full_size_two_iterations():
    """The 1000-shell, 10-level, 256-channel cloud: two iterations batched
    against the oracle, and the march times of both layouts."""
    w = workload_1d_plummer(1000)
    ref = oracle.run_1d(w.mol, w.model, w.spec, w.T_bg, 2)
    times = {}
    for on in (False, True):
        ctx = make_ctx(w)
        ctx.set_transition_batching(on)
        ctx.run(2)
        times[on] = ctx.counters()["march_ms"] / 2
        assert_pops(ctx.populations(), ref.x, 1e-5, f"plummer-1000 batched={on}")
        ctx.close()
    print(f"[batching] 1000 shells: march {times[False]:.3f} ms per iteration per transition layout, "
          f"{times[True]:.3f} ms all transitions per pass", flush=True)
