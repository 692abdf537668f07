"""Population inversion (negative opacity): the transfer equations hold as
written for a moderately inverted line, so the GPU spectra equal the oracle's
on the same populations; a step whose line-centre optical depth falls below
-40 is refused with MILOC_ENUMERIC (by the spectra call and by an iteration,
which then leaves the populations as they were)."""
import numpy as np
import pytest

import oracle
import synth

miloc = pytest.importorskip("paper_2009_12609_amd")

from test_gpu_parity import assert_spectra  # noqa: E402

pytestmark = pytest.mark.gpu

KMS = 1.0e5
PC = synth.PC_CM


def _inverted(nc):
    x = np.empty((nc, 2))
    x[:, 0] = 0.2          # x_l g_u/g_l - x_u = 0.6 - 0.8 < 0
    x[:, 1] = 0.8
    return x


def _ctx(mol, model, spec, T_bg, fp64):
    ctx = miloc.Context()
    ctx.load_molecule(mol)
    if isinstance(model, synth.Model1D):
        ctx.load_model_1d(model)
    else:
        ctx.load_model_3d(model)
    ctx.set_spectral(spec.n_channels, spec.v_min, spec.dv)
    ctx.set_background(T_bg)
    ctx.set_march_precision(fp64)
    return ctx


def _centre_tau(mol, model, spec, x, length):
    prob = oracle._Problem(mol, model.n_H2, model.T_kin, model.b_turb, model.abundance, spec, 2.73)
    kap, _ = oracle.prepare(mol, x, prob.n_mol)
    return float(np.min(kap[0] * length / (prob.bD * np.sqrt(np.pi))))


@pytest.mark.parametrize("fp64,tol", [(False, 1e-4), (True, 1e-9)])
def test_moderate_maser_1d_spectra(fp64, tol):
    mol = synth.two_level_molecule()
    m = synth.uniform_sphere_1d(20, 0.05 * PC, 1.0e4, 10.0, 0.2 * KMS, 3.0e-6, 20)
    spec = synth.Spectral.symmetric(128, 1.5)
    x = _inverted(m.n_shells)
    tau = _centre_tau(mol, m, spec, x[:1], 2.0 * m.r_out[-1])
    print(f"[case] 1D maser, centre line-centre tau {tau:.2f}, fp64={fp64}", flush=True)
    assert -6.0 < tau < -1.0
    ctx = _ctx(mol, m, spec, 2.73, fp64)
    ctx.set_populations(x)
    sp = ctx.spectra(0, n_los=m.n_rays)
    ref = oracle.spectra_1d(mol, m, spec, 2.73, x, 0)
    assert ref.max() > 10.0 * oracle.planck(mol.nu[0], 2.73)     # amplified background
    assert_spectra(sp, ref, tol, f"1D maser fp64={fp64}")
    ctx.close()


@pytest.mark.parametrize("fp64,tol", [(False, 1e-4), (True, 1e-9)])
def test_moderate_maser_3d_spectra(fp64, tol):
    mol = synth.two_level_molecule()
    N = 6
    box = 0.05 * PC
    cube = synth.uniform_cube(N, box, 1.0e4, 10.0, 0.2 * KMS, 3.0e-6)
    spec = synth.Spectral.symmetric(128, 1.5)
    x = _inverted(N ** 3)
    tau = _centre_tau(mol, cube, spec, x[:1], box)
    print(f"[case] 3D maser, column line-centre tau {tau:.2f}, fp64={fp64}", flush=True)
    assert -6.0 < tau < -0.5
    ctx = _ctx(mol, cube, spec, 2.73, fp64)
    ctx.set_populations(x)
    sp = ctx.spectra(0, n_los=N * N)
    ref = oracle.spectra_3d(mol, cube, spec, 2.73, x, 0)
    assert_spectra(sp, ref, tol, f"3D maser fp64={fp64}")
    ctx.close()


@pytest.mark.parametrize("kind", ["1d", "3d", "octree"])
def test_maser_beyond_bound_is_refused(kind):
    mol = synth.two_level_molecule()
    spec = synth.Spectral.symmetric(128, 1.5)
    if kind == "1d":
        model = synth.uniform_sphere_1d(20, 0.05 * PC, 1.0e4, 10.0, 0.2 * KMS, 5.0e-3, 20)
    elif kind == "3d":
        model = synth.uniform_cube(6, 0.05 * PC, 1.0e4, 10.0, 0.2 * KMS, 5.0e-3)
    else:
        model = synth.octree_cloud(N_root=4, n_refine=2, frac=0.35, grf_N=16, box_pc=0.05, abundance=5.0e-3)
        model.T_kin[:] = 10.0
        model.b_turb[:] = 0.2 * KMS
        for v in (model.vx, model.vy, model.vz):
            v[:] = 0.0
    nc = model.n_shells if kind == "1d" else model.n_cells
    x = _inverted(nc)
    print(f"[case] maser beyond the bound, {kind}", flush=True)
    ctx = _ctx(mol, model, spec, 2.73, False)
    ctx.set_populations(x)
    n_los = model.n_rays if kind == "1d" else model.n0[0] ** 2
    with pytest.raises(miloc.MilocError) as e:
        ctx.spectra(0, n_los=n_los)
    assert e.value.code == miloc.ENUMERIC
    with pytest.raises(miloc.MilocError) as e:
        ctx.run(1)
    assert e.value.code == miloc.ENUMERIC
    assert np.array_equal(ctx.populations(), x)
    # a physical (LTE) start runs normally afterwards
    ctx.init_lte()
    ctx.run(1)
    ctx.close()
