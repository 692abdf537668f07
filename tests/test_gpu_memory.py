"""Device-memory admission of 3D models: a model whose arrays, ray tables and
one transition's per-step sums exceed the usable device memory is refused
with MILOC_ENOMEM before its static arrays are allocated; with room for only
some transitions' sums, an iteration's transitions are marched in several
launches and the results do not change.  The usable memory is capped for the
test through MILOC_DEVICE_BUDGET_GB."""
import numpy as np
import pytest

import synth

miloc = pytest.importorskip("paper_2009_12609_amd")

from test_gpu_parity import make_ctx, workload_3d  # noqa: E402

pytestmark = pytest.mark.gpu


def test_model_beyond_the_budget_is_refused(monkeypatch):
    w = workload_3d(12, seed=112, n_levels=5, nch=128)
    fixed, sums = miloc.model_footprint(w.model, 5, 4, 128)
    monkeypatch.setenv("MILOC_DEVICE_BUDGET_GB", str(0.5 * (fixed + sums) * 1e-9))
    ctx = make_ctx(w)
    with pytest.raises(miloc.MilocError) as e:
        ctx.run(1)
    assert e.value.code == miloc.ENOMEM
    assert "needs" in str(e.value)
    ctx.close()


def test_partial_room_splits_the_launches(monkeypatch):
    w = workload_3d(12, seed=112, n_levels=10, nch=256)
    ref = make_ctx(w)
    ref.run(2)
    x_ref = ref.populations()
    n_ref = ref.counters()["march_launches"]
    ref.close()
    fixed, sums = miloc.model_footprint(w.model, 10, 9, 256)
    # room for the arrays and two transitions' per-step sums (plus what the
    # first context's allocator may still hold back)
    monkeypatch.setenv("MILOC_DEVICE_BUDGET_GB", str((fixed + 2.5 * sums) * 1e-9))
    ctx = make_ctx(w)
    ctx.run(2)
    n = ctx.counters()["march_launches"]
    print(f"[memory] launches per 2 iterations: {n} with room for two transitions, {n_ref} without a cap",
          flush=True)
    assert n_ref == 2 and n == 10
    assert np.array_equal(ctx.populations(), x_ref)
    ctx.close()
