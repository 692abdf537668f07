"""Pins of the oracle's sub-iterations in an optically thick core (the
paper's Sect. 4 suggestion: update populations more often where the lines are
thick), independent of the HIP path:

* the core pieces of the rays, started from the intensity each ray carries
  into the core, reproduce the full march's absorbed counts and diagonal
  operator in every core shell (the bookkeeping of the re-march);
* a core that is the whole model turns every iteration into 1 + n_sub plain
  ALI iterations (the entry intensity is then the background at R_out);
* no core leaves plain ALI unchanged;
* the fixed point is plain ALI's (to 1e-9 at tol 1e-12), reached in fewer
  global iterations on a thick cloud.
"""
import numpy as np

import oracle
import synth


def _thick_plummer(n=60, X=1e-6):
    w = synth.workload_1d_plummer(n_shells=n, abundance=X)
    w.mol = synth.rotor_molecule(6)
    w.spec = synth.Spectral.symmetric(128, 4.0)
    return w


def _geometry(w):
    m = w.model
    prob = oracle._Problem(w.mol, m.n_H2, m.T_kin, m.b_turb, m.abundance, w.spec, w.T_bg)
    R = np.asarray(m.r_out, dtype=np.float64)
    impact = oracle.equidistant_impacts(R[-1], m.n_rays)
    area = oracle.ray_areas_1d(R[-1], impact)
    return prob, R, impact, area


def test_core_march_reproduces_the_full_march_in_the_core():
    w = _thick_plummer()
    m = w.model
    prob, R, impact, area = _geometry(w)
    x = oracle.lte_populations(w.mol, prob.T)
    kap, eta = oracle.prepare(w.mol, x, prob.n_mol)
    for K in (0, 7, 30, m.n_shells - 1):
        for t in (0, 3):
            full = oracle.march_1d(R, m.v_r, prob.bD, kap[t], eta[t], impact, area, w.spec, prob.I_bg[t])
            Ie = oracle.core_entry_1d(R, m.v_r, prob.bD, kap[t], eta[t], impact, K, w.spec, prob.I_bg[t])
            jr, lr = oracle.march_core_1d(R, m.v_r, prob.bD, kap[t], eta[t], impact, area, K, w.spec, Ie)
            c = slice(0, K + 1)
            assert np.allclose(jr[c], full.Jraw[c], rtol=1e-12, atol=0)
            assert np.allclose(lr[c], full.Lraw[c], rtol=1e-12, atol=1e-300)
            assert np.all(jr[K + 1:] == 0) and np.all(lr[K + 1:] == 0)
            # rays that never reach the core carry nothing into it
            miss = impact >= R[K]
            assert np.all(Ie[miss] == 0)


def test_whole_model_core_equals_repeated_ali():
    w = _thick_plummer(n=40)
    n_sub = 2
    sub = oracle.run_1d_sub(w.mol, w.model, w.spec, w.T_bg, 3, n_sub, 0.0, core=w.model.n_shells - 1)
    ali = oracle.run_1d(w.mol, w.model, w.spec, w.T_bg, 3 * (n_sub + 1))
    for i, h in enumerate(sub.history):
        ref = ali.history[(n_sub + 1) * i + n_sub]["x"]
        big = ref > 1e-12
        assert np.max(np.abs(h["x"][big] / ref[big] - 1)) < 1e-12
        assert abs(h["delta"] - ali.history[(n_sub + 1) * i]["delta"]) <= 1e-9 * ali.history[(n_sub + 1) * i]["delta"]


def test_no_core_is_plain_ali():
    w = _thick_plummer(n=40)
    sub = oracle.run_1d_sub(w.mol, w.model, w.spec, w.T_bg, 4, 3, 1.0e30)
    ali = oracle.run_1d(w.mol, w.model, w.spec, w.T_bg, 4)
    assert all(h["K"] == -1 for h in sub.history)
    for a, b in zip(sub.history, ali.history):
        assert np.array_equal(a["x"], b["x"])


def test_fixed_point_and_fewer_iterations_on_a_thick_cloud():
    w = _thick_plummer()
    ali = oracle.run_1d(w.mol, w.model, w.spec, w.T_bg, 500, tol=1e-12, record=False)
    sub = oracle.run_1d_sub(w.mol, w.model, w.spec, w.T_bg, 500, 3, 0.1, tol=1e-12, record=False)
    big = ali.x > 1e-10
    assert np.max(np.abs(sub.x[big] / ali.x[big] - 1)) < 1e-9
    K = [h["K"] for h in sub.history]
    assert min(K) > 0 and max(K) < w.model.n_shells - 1      # a genuine core, not the whole cloud
    assert sub.iters < 0.75 * ali.iters
