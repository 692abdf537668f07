"""The 1D request loop: each result is the same alone and in the mix,
admission by footprint, rejection and cancellation without disturbing others."""
import numpy as np
import pytest

import oracle
import synth

miloc = pytest.importorskip("paper_2009_12609_amd")

pytestmark = pytest.mark.gpu


def small_stream(n=6, seed=11):
    reqs = synth.serving_stream(n, seed=seed, shells=(40, 150))
    # make sure every level count and channel count shows up
    for r, L, nch in zip(reqs, (2, 5, 10, 20, 5, 10), (64, 128, 256, 128, 64, 256)):
        r.mol = synth.rotor_molecule(L)
        r.spec = synth.Spectral.symmetric(nch, 2.0)
    return reqs


def alone(req, iters):
    ctx = miloc.Context()
    ctx.load_molecule(req.mol)
    ctx.load_model_1d(req.model)
    ctx.set_spectral(req.spec.n_channels, req.spec.v_min, req.spec.dv)
    ctx.set_background(req.T_bg)
    ctx.run(iters)
    x = ctx.populations()
    sp = np.stack([ctx.spectra(t, impact=np.array([0.0]))[0] for t in range(req.mol.n_trans)])
    ctx.close()
    return x, sp


def rel(a, b):
    big = b >= 1e-12
    return float(np.max(np.abs(a[big] - b[big]) / b[big]))


def test_alone_equals_mix_and_oracle():
    reqs = small_stream()
    srv = miloc.Server(hbm_budget_bytes=1 << 30, max_slots=8)
    tickets = [srv.submit(r.mol, r.model, r.spec, r.T_bg, tol=1e-6, max_iter=200) for r in reqs]
    for t in tickets:
        assert srv.wait(t, 120.0)
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["peak_active"] >= 2
    for i, (r, t) in enumerate(zip(reqs, tickets)):
        x, sp, info, rc = srv.take(t)
        assert rc == miloc.OK and info["status"] == miloc.OK, info
        assert info["last_delta"] < 1e-6
        xa, spa = alone(r, info["iterations"])
        e = rel(x, xa)
        print(f"[serve] req {i}: L={r.mol.n_levels} nch={r.spec.n_channels} shells={r.model.n_shells} "
              f"iters={info['iterations']} mix-vs-alone {e:.2e}", flush=True)
        assert e < 1e-5, e
        scale = np.max(np.abs(spa), axis=1, keepdims=True)
        assert np.all(np.abs(sp - spa) <= 1e-5 * scale + 1e-40)
        if i < 2:
            ref = oracle.run_1d(r.mol, r.model, r.spec, r.T_bg, info["iterations"])
            eo = rel(x, ref.x)
            print(f"[serve] req {i}: vs oracle {eo:.2e}", flush=True)
            assert eo < 1e-5
    srv.close()


def test_budget_admits_one_at_a_time():
    reqs = synth.serving_stream(4, seed=12, shells=(1200, 2000), levels=(20,))
    srv0 = miloc.Server(hbm_budget_bytes=1 << 30, max_slots=8)
    sizes = [srv0.footprint(r.mol, r.model, r.spec, r.T_bg) for r in reqs]
    srv0.close()
    # a budget that holds the largest request but no two of them
    big = sorted(sizes)
    assert big[0] + big[1] > big[-1] >= 1 << 20
    srv = miloc.Server(hbm_budget_bytes=big[-1], max_slots=8)
    tickets = [srv.submit(r.mol, r.model, r.spec, r.T_bg, tol=0.0, max_iter=10) for r in reqs]
    for t in tickets:
        assert srv.wait(t, 120.0)
    st = srv.stats()
    assert st["completed"] == 4
    assert st["peak_active"] == 1
    assert st["arena_used"] == 0
    for t in tickets:
        _, _, info, rc = srv.take(t)
        assert rc == miloc.OK and info["iterations"] == 10
    srv.close()


def test_bad_requests_are_isolated_and_cancel_works():
    reqs = small_stream(3, seed=13)
    srv = miloc.Server(hbm_budget_bytes=1 << 30, max_slots=1)
    bad = synth.serving_stream(1, seed=14, shells=(40, 60))[0]
    bad.model.T_kin[5] = float("nan")
    with pytest.raises(miloc.MilocError) as e:
        srv.submit(bad.mol, bad.model, bad.spec)
    assert e.value.code == miloc.EINVAL
    huge = synth.serving_stream(1, seed=15, shells=(3000, 3000))[0]
    with pytest.raises(miloc.MilocError) as e:
        srv.submit(huge.mol, huge.model, huge.spec)
    assert e.value.code == miloc.EINVAL
    tickets = [srv.submit(r.mol, r.model, r.spec, r.T_bg, tol=1e-6, max_iter=200) for r in reqs]
    srv.cancel(tickets[2])            # queued behind the single slot
    for t in tickets[:2]:
        assert srv.wait(t, 120.0)
    assert srv.wait(tickets[2], 10.0)
    for t in tickets[:2]:
        _, _, info, rc = srv.take(t)
        assert rc == miloc.OK
    _, _, info, rc = srv.take(tickets[2])
    assert rc == miloc.ESTATE
    st = srv.stats()
    assert st["cancelled"] == 1 and st["completed"] == 2
    srv.close()


def test_cancel_while_resident():
    """A request cancelled while it is on the device leaves at the next tick;
    the slot is reused by the next request, whose result is unaffected."""
    import time
    reqs = small_stream(2, seed=16)
    srv = miloc.Server(hbm_budget_bytes=1 << 30, max_slots=1)
    t_long = srv.submit(reqs[0].mol, reqs[0].model, reqs[0].spec, reqs[0].T_bg, tol=1e-300, max_iter=100000)
    for _ in range(2000):
        if srv.stats()["active"] == 1:
            break
        time.sleep(0.005)
    assert srv.stats()["active"] == 1
    srv.cancel(t_long)
    assert srv.wait(t_long, 60.0)
    _, _, info, rc = srv.take(t_long)
    assert rc == miloc.ESTATE
    t2 = srv.submit(reqs[1].mol, reqs[1].model, reqs[1].spec, reqs[1].T_bg, tol=1e-6, max_iter=200)
    assert srv.wait(t2, 60.0)
    x, _, info, rc = srv.take(t2)
    assert rc == miloc.OK
    xa, _ = alone(reqs[1], info["iterations"])
    assert rel(x, xa) < 1e-5
    st = srv.stats()
    assert st["cancelled"] == 1 and st["completed"] == 1 and st["arena_used"] == 0
    srv.close()


def _request(shells, levels, nch, seed):
    r = synth.serving_stream(1, seed=seed, shells=(shells, shells), levels=(levels,))[0]
    r.spec = synth.Spectral.symmetric(nch, 2.0)
    return r


def test_large_models_alone_mix_and_oracle():
    """Models that need the larger LDS tiers of the tick's march kernel (FP64
    per-shell accumulators of up to 2048 shells beside sixteen channel vectors
    of up to 512 channels): 1000 shells x 256 channels, 1600 x 256 and
    1300 x 512 (the three largest of the six tiers), served together with two
    small models; each result equals the model solved alone, and two equal
    the oracle's run to the same tolerance."""
    big = [_request(1000, 10, 256, 31), _request(1600, 5, 256, 32), _request(1300, 2, 512, 33)]
    reqs = big + small_stream(2, seed=34)
    srv = miloc.Server(hbm_budget_bytes=2 << 30, max_slots=8)
    tickets = [srv.submit(r.mol, r.model, r.spec, r.T_bg, tol=1e-6, max_iter=200) for r in reqs]
    for t in tickets:
        assert srv.wait(t, 300.0)
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["peak_active"] >= 3
    for i, (r, t) in enumerate(zip(reqs, tickets)):
        x, sp, info, rc = srv.take(t)
        assert rc == miloc.OK and info["status"] == miloc.OK, info
        xa, spa = alone(r, info["iterations"])
        e = rel(x, xa)
        print(f"[serve] large req {i}: L={r.mol.n_levels} nch={r.spec.n_channels} shells={r.model.n_shells} "
              f"iters={info['iterations']} mix-vs-alone {e:.2e}", flush=True)
        assert e < 1e-5, e
        scale = np.max(np.abs(spa), axis=1, keepdims=True)
        assert np.all(np.abs(sp - spa) <= 1e-5 * scale + 1e-40)
        if i in (0, 2):
            ref = oracle.run_1d(r.mol, r.model, r.spec, r.T_bg, 200, tol=1e-6, record=False)
            eo = rel(x, ref.x)
            print(f"[serve] large req {i}: vs oracle {eo:.2e} (oracle {ref.iters} iterations)", flush=True)
            assert abs(ref.iters - info["iterations"]) <= 1
            assert eo < 1e-5
    srv.close()
