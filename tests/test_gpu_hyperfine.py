"""Hyperfine multiplets with LTE between the components (Sect. 1): the HIP
path through the C ABI against the FP64 oracle, bars as in test_gpu_parity.
The components are synthetic (three lines at -0.62, 0 and +0.37 km/s with
strengths 1 : 5 : 3); one transition of a species carries the multiplet, the
others keep single Gaussians, as in the paper's HCN case."""
import numpy as np
import pytest

import oracle
import synth

miloc = pytest.importorskip("paper_2009_12609_amd")

from test_gpu_parity import KMS, assert_pops, assert_spectra, make_ctx, workload_3d  # noqa: E402
from test_gpu_octree import leaf_rows, oct_workload  # noqa: E402

pytestmark = pytest.mark.gpu

HF_V = np.array([-0.62, 0.0, 0.37]) * KMS
HF_W = np.array([1.0, 5.0, 3.0])


def hf_ctx(w, hfs, fp64=False):
    ctx = make_ctx(w, fp64=fp64)
    for t, (v, s) in hfs.items():
        ctx.set_hyperfine(t, v, s)
    return ctx


def test_1d_hyperfine_fp64_iteration_by_iteration():
    """Two-level species on the small shell cloud, thick enough (X = 3e-8) for
    the multiplet to shape the excitation; FP64 march, every iteration."""
    w = synth.workload_1d_small()
    w.model = synth.cloud_1d_log(abundance=3e-8)
    w.spec = synth.Spectral.symmetric(192, 3.0)
    hfs = {0: (HF_V, HF_W)}
    print("[case] 1d hyperfine fp64", flush=True)
    ref = oracle.run_1d(w.mol, w.model, w.spec, w.T_bg, 6, hyperfine=hfs)
    plain = oracle.run_1d(w.mol, w.model, w.spec, w.T_bg, 6)
    ctx = hf_ctx(w, hfs, fp64=True)
    for it in range(6):
        ctx.run(1)
        assert_pops(ctx.populations(), ref.history[it]["x"], 1e-10, f"1d hf fp64 it {it}")
    # the multiplet matters at this optical depth
    assert np.max(np.abs(ref.x - plain.x) / plain.x) > 1e-3
    sp = ctx.spectra(0, n_los=w.model.n_rays)
    ref_sp = oracle.spectra_1d(w.mol, w.model, w.spec, w.T_bg, ref.x, 0, shape=hfs[0])
    assert_spectra(sp, ref_sp, 1e-9, "1d hf fp64")
    ctx.close()


def test_1d_hyperfine_fp32_rotor():
    """Plummer infall cloud, 10-level rotor, multiplets on transitions 0 and 2
    (different offsets), FP32 march."""
    w = synth.workload_1d_plummer(n_shells=61, abundance=1e-8)
    hfs = {0: (HF_V, HF_W), 2: (np.array([-0.3, 0.25]) * KMS, np.array([2.0, 1.0]))}
    print("[case] 1d hyperfine fp32 rotor", flush=True)
    ref = oracle.run_1d(w.mol, w.model, w.spec, w.T_bg, 8, hyperfine=hfs)
    ctx = hf_ctx(w, hfs)
    ctx.run(8)
    x = ctx.populations()
    assert_pops(x, ref.x, 1e-5, "1d hf fp32 rotor")
    J, Lam = ctx.radiation()
    assert np.allclose(J, ref.history[-1]["J"], rtol=2e-5, atol=0)
    for t in (0, 1, 2):
        imp = w.model.r_out[-1] * (np.arange(16) + 0.5) / 16
        sp = ctx.spectra(t, impact=imp)
        ref_sp = oracle.spectra_1d(w.mol, w.model, w.spec, w.T_bg, x, t, impact=imp, shape=hfs.get(t))
        assert_spectra(sp, ref_sp, 1e-4, f"1d hf fp32 spectra t={t}")
    ctx.close()


@pytest.mark.parametrize("fp64", [False, True])
def test_3d_hyperfine(fp64):
    """Turbulent 9^3 cube, 48 directions, thick (X = 1e-7), multiplet on the
    first transition of a 5-level rotor; spectra of the multiplet."""
    w = workload_3d(9, seed=109, abundance=1e-7, n_levels=5, box_pc=0.075, half=5.0)
    hfs = {0: (HF_V, HF_W)}
    print(f"[case] 3d hyperfine fp64={fp64}", flush=True)
    ref = oracle.run_3d(w.mol, w.model, w.spec, w.T_bg, 3, hyperfine=hfs)
    ctx = hf_ctx(w, hfs, fp64=fp64)
    ctx.run(3)
    tol = 1e-10 if fp64 else 1e-5
    assert_pops(ctx.populations(), ref.x, tol, f"3d hf fp64={fp64}")
    J, Lam = ctx.radiation()
    h = ref.history[-1]
    assert np.allclose(J, h["J"], rtol=1e-9 if fp64 else 2e-5, atol=0)
    assert np.allclose(Lam, h["Lam"], rtol=1e-9 if fp64 else 2e-5, atol=1e-9)
    sp = ctx.spectra(0, n_los=81)
    ref_sp = oracle.spectra_3d(w.mol, w.model, w.spec, w.T_bg, ref.x, 0, shape=hfs[0])
    assert_spectra(sp, ref_sp, 1e-9 if fp64 else 1e-4, f"3d hf spectra fp64={fp64}")
    ctx.close()


@pytest.mark.parametrize("fp64,lattice", [(False, False), (True, False), (False, True)])
def test_octree_hyperfine(fp64, lattice):
    """Octree (root 4^3, three refinement levels; two with the brute-force
    lattice) with the multiplet on the first transition: every iteration's
    leaf populations, and the +z map."""
    w = oct_workload(half=5.0, n_refine=2 if lattice else 3)
    hfs = {0: (HF_V, HF_W)}
    lf = leaf_rows(w)
    print(f"[case] octree hyperfine fp64={fp64} lattice={lattice}", flush=True)
    ref = oracle.run_oct(w.mol, w.model, w.spec, w.T_bg, 2, hyperfine=hfs, brute=lattice)
    ctx = hf_ctx(w, hfs, fp64=fp64)
    ctx.set_octree_rays(lattice)
    tol = 1e-10 if fp64 else 1e-5
    for it in range(2):
        ctx.run(1)
        assert_pops(ctx.populations()[lf], ref.history[it]["x"][lf], tol, f"octree hf it {it}")
    sp = ctx.spectra(0, n_los=w.model.n0[0] ** 2)
    sref = oracle.spectra_oct(w.mol, w.model, w.spec, w.T_bg, ref.x, 0, shape=hfs[0])
    assert_spectra(sp, sref, 1e-9 if fp64 else 1e-4, "octree hf +z map")
    ctx.close()


@pytest.mark.parametrize("n_comp,fp64", [(2, False), (4, False), (5, False), (12, False), (20, False),
                                          (6, True), (12, True)])
def test_1d_hyperfine_component_counts(n_comp, fp64):
    """Every unrolled form of the multiplet sum: exactly 2 or 4 components,
    8 or 16 register components with zero-strength padding, and (20 in FP32,
    12 in FP64) the components past the register set read from memory."""
    rng = np.random.default_rng(100 + n_comp)
    v = rng.uniform(-0.6, 0.6, n_comp) * KMS
    s = rng.uniform(0.5, 2.0, n_comp)
    w = synth.workload_1d_small()
    w.model = synth.cloud_1d_log(abundance=3e-8)
    w.spec = synth.Spectral.symmetric(192, 3.0)
    hfs = {0: (v, s)}
    print(f"[case] 1d hyperfine {n_comp} components fp64={fp64}", flush=True)
    ref = oracle.run_1d(w.mol, w.model, w.spec, w.T_bg, 4, hyperfine=hfs)
    ctx = hf_ctx(w, hfs, fp64=fp64)
    ctx.run(4)
    assert_pops(ctx.populations(), ref.x, 1e-10 if fp64 else 1e-5, f"1d hf n={n_comp}")
    sp = ctx.spectra(0, n_los=w.model.n_rays)
    ref_sp = oracle.spectra_1d(w.mol, w.model, w.spec, w.T_bg, ref.x, 0, shape=hfs[0])
    assert_spectra(sp, ref_sp, 1e-9 if fp64 else 1e-4, f"1d hf n={n_comp}")
    ctx.close()


def test_hyperfine_single_component_and_reset():
    """One component at offset 0 runs the multiplet kernels with the plain
    line; clearing the multiplet returns the single-Gaussian kernels."""
    w = workload_3d(8, seed=7, abundance=1e-7, n_levels=4, box_pc=0.05, nch=128)
    print("[case] hyperfine single component / reset", flush=True)
    base = make_ctx(w)
    base.run(2)
    x0 = base.populations()
    base.close()
    one = hf_ctx(w, {0: (np.array([0.0]), np.array([4.0]))})
    one.run(2)
    assert_pops(one.populations(), x0, 1e-6, "single component")
    one.close()
    cleared = hf_ctx(w, {1: (HF_V, HF_W)})
    cleared.set_hyperfine(1, [], [])
    cleared.run(2)
    assert np.array_equal(cleared.populations(), x0)
    cleared.close()


def test_hyperfine_argument_errors():
    ctx = miloc.Context()
    with pytest.raises(miloc.MilocError) as e:
        ctx.set_hyperfine(0, HF_V, HF_W)          # no molecule yet
    assert e.value.code == miloc.ESTATE
    w = synth.workload_1d_small()
    ctx.load_molecule(w.mol)
    ctx.load_model_1d(w.model)
    ctx.set_spectral(w.spec.n_channels, w.spec.v_min, w.spec.dv)
    for args in [(1, HF_V, HF_W),                               # one transition only
                 (-1, HF_V, HF_W),
                 (0, np.zeros(33), np.ones(33)),                # too many components
                 (0, HF_V, np.array([1.0, 0.0, 2.0])),          # strength not > 0
                 (0, np.array([0.0, np.nan, 1.0]), HF_W)]:
        with pytest.raises(miloc.MilocError) as e:
            ctx.set_hyperfine(*args)
        assert e.value.code == miloc.EINVAL
    # offsets that push the line out of the +-2 km/s band
    ctx.set_hyperfine(0, np.array([-1.9, 0.0]) * KMS, np.array([1.0, 1.0]))
    with pytest.raises(miloc.MilocError) as e:
        ctx.run(1)
    assert e.value.code == miloc.EINVAL
    ctx.set_hyperfine(0, HF_V, HF_W)
    it, _ = ctx.run(1)
    assert it == 1
    ctx.close()
