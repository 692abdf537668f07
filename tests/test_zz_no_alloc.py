"""miloc_solve_1d_noalloc (the allocation-free 1D solve, all device memory in
the library's static scratch) against the context entry points that allocate:
two calls in a row, the second on a smaller model, each equal to the context
result; a model larger than the scratch is refused with MILOC_ENOMEM."""
import numpy as np
import pytest

import synth

miloc = pytest.importorskip("paper_2009_12609_amd")

pytestmark = pytest.mark.gpu


def context_solve(w, max_iter, tol):
    ctx = miloc.Context()
    ctx.load_molecule(w.mol)
    ctx.load_model_1d(w.model)
    ctx.set_spectral(w.spec.n_channels, w.spec.v_min, w.spec.dv)
    ctx.set_background(w.T_bg)
    it, d = ctx.run(max_iter, tol=tol)
    x = ctx.populations()
    ctx.close()
    return x, it, d


def test_noalloc_equals_context_on_two_calls():
    big = synth.workload_1d_plummer(n_shells=300)          # 10 levels, 256 channels
    small = synth.workload_1d_small()                      # 100 shells, 2 levels, 128 channels
    for w in (big, small):
        print(f"[case] noalloc solve, {w.model.n_shells} shells, {w.mol.n_levels} levels, "
              f"{w.spec.n_channels} channels", flush=True)
        xr, itr, dr = context_solve(w, 60, 1e-6)
        x, it, d, rc = miloc.solve_1d_noalloc(w.mol, w.model, w.spec, w.T_bg, 60, 1e-6)
        assert rc == miloc.OK and it == itr
        assert x.shape == xr.shape
        big_x = xr >= 1e-12
        rel = float(np.max(np.abs(x[big_x] - xr[big_x]) / xr[big_x]))
        print(f"[parity] noalloc vs context: {it} iterations, max rel {rel:.3e}, delta {d:.3e} / {dr:.3e}",
              flush=True)
        assert rel <= 1e-10
        assert np.all(np.abs(x[~big_x] - xr[~big_x]) <= 1e-17)
        assert abs(d - dr) <= 1e-8 * dr


def test_noalloc_refuses_a_model_beyond_the_scratch():
    s = synth.workload_1d_small()
    big = synth.cloud_1d_log(n_shells=4000)                # ~1.2e7 ray steps: ~100 MB of step records
    print("[case] noalloc solve beyond the scratch", flush=True)
    with pytest.raises(miloc.MilocError) as e:
        miloc.solve_1d_noalloc(s.mol, big, s.spec, s.T_bg, 2, 0.0)
    assert e.value.code == miloc.ENOMEM
    # and the scratch still serves a model that fits afterwards
    x, it, _, rc = miloc.solve_1d_noalloc(s.mol, s.model, s.spec, s.T_bg, 3, 0.0)
    xr, _, _ = context_solve(s, 3, 0.0)
    assert rc == miloc.OK and it == 3
    assert np.allclose(x, xr, rtol=1e-10, atol=1e-17)
