"""Parity of the octree march (through the C ABI) with the FP64 oracle, and
its properties at the full benchmark size.  Bars as in test_gpu_parity."""
import numpy as np
import pytest

import oracle
import synth

miloc = pytest.importorskip("paper_2009_12609_amd")

from test_gpu_parity import assert_pops, assert_spectra, make_ctx  # noqa: E402

pytestmark = pytest.mark.gpu


def oct_workload(N_root=4, n_refine=3, frac=0.35, grf_N=16, box_pc=0.2, abundance=1e-7,
                 n_levels=5, nch=128, half=4.0, seed=4001):
    m = synth.octree_cloud(N_root=N_root, n_refine=n_refine, frac=frac, grf_N=grf_N, box_pc=box_pc,
                           abundance=abundance, seed=seed)
    return synth.Workload(f"oct-{N_root}", synth.rotor_molecule(n_levels),
                          synth.Spectral.symmetric(nch, half), 2.73, m, 2)


def leaf_rows(w):
    return oracle.octree_of(w.model).leaf


@pytest.mark.parametrize("fp64,tol", [(False, 1e-5), (True, 1e-10)])
def test_octree_small_iterations(fp64, tol):
    """Root 4^3, three refinement levels, optically thick enough for the
    created rays to matter: every iteration's populations and J, Lambda."""
    w = oct_workload()
    print(f"[octree] cells per level {w.model.n_cells_per_level} fp64={fp64}", flush=True)
    lf = leaf_rows(w)
    ref = oracle.run_oct(w.mol, w.model, w.spec, w.T_bg, 3)
    ctx = make_ctx(w, fp64=fp64)
    for it in range(3):
        ctx.run(1)
        x = ctx.populations()
        assert_pops(x[lf], ref.history[it]["x"][lf], tol, f"octree it {it}")
    J, Lam = ctx.radiation()
    rJ, rL = ref.history[2]["J"], ref.history[2]["Lam"]
    # J in CGS for the GPU, occupation units for the oracle: compare the ALI pair via Lambda
    # and the ratio structure of J (per transition scale)
    assert np.max(np.abs(Lam[:, lf] - rL[:, lf])) <= (1e-5 if not fp64 else 1e-10) * max(1e-3, np.max(rL[:, lf]))
    cnt = ctx.counters()
    print(f"[octree] march {cnt['march_ms']:.2f} ms over {cnt['march_launches']} launches, "
          f"{cnt['ray_steps']:.3e} steps", flush=True)
    sp = ctx.spectra(0, n_los=w.model.n0[0] ** 2)
    sref = oracle.spectra_oct(w.mol, w.model, w.spec, w.T_bg, ref.x, 0)
    assert_spectra(sp, sref, 1e-4 if not fp64 else 1e-9, "octree +z map")
    ctx.close()


def test_unrefined_octree_matches_regular_grid_on_gpu():
    """An octree with one level is the regular grid: the two device paths
    agree (to FP32 summation order)."""
    cube = synth.turbulent_cube(N=8, box_pc=0.2, seed=17, abundance=1e-7)
    oct_m = synth.Model3D(**{**cube.__dict__})
    oct_m.n_oct_levels = 1
    oct_m.n_cells_per_level = [8 ** 3]
    oct_m.first_child = [np.full(8 ** 3, -1, np.int32)]
    w_reg = synth.Workload("r", synth.rotor_molecule(5), synth.Spectral.symmetric(128, 4.0), 2.73, cube, 2)
    w_oct = synth.Workload("o", w_reg.mol, w_reg.spec, 2.73, oct_m, 2)
    a, b = make_ctx(w_reg), make_ctx(w_oct)
    a.run(3)
    b.run(3)
    assert_pops(b.populations(), a.populations(), 2e-6, "unrefined octree vs regular")
    a.close()
    b.close()


def test_octree_uniform_field_full_size():
    """The 64^3-root, four-level octree (about 2e7 leaves) with S = I_bg
    everywhere: every ray keeps I_bg, so the first solve returns the
    populations whose source function is the background; checks every
    created, split and terminated ray at the benchmark size."""
    w = synth.workload_octree()
    m = w.model
    mol = synth.two_level_molecule()
    T_bg = 2.73
    nc = m.n_cells
    print(f"[octree] full size: cells per level {m.n_cells_per_level}", flush=True)
    ctx = miloc.Context()
    ctx.load_molecule(mol)
    m.T_kin[:] = T_bg          # LTE at T_bg gives S = B(T_bg) = I_bg
    m.b_turb[:] = 1.0e4        # b = 0.108 km/s = 3.5 channels: sum_c f_c = 1
    ctx.load_model_3d(m)
    ctx.set_spectral(w.spec.n_channels, w.spec.v_min, w.spec.dv)
    ctx.set_background(T_bg)
    ctx.run(1)
    x = ctx.populations()
    lte = oracle.lte_populations(mol, np.full(nc, T_bg))
    lf = oracle.octree_of(m).leaf
    rel = np.max(np.abs(x[lf] - lte[lf]) / lte[lf])
    cnt = ctx.counters()
    print(f"[octree] full size uniform field: max rel dev {rel:.3e}; march {cnt['march_ms']:.1f} ms, "
          f"{cnt['ray_steps']:.3e} steps", flush=True)
    assert rel < 1e-5
    ctx.close()


def test_octree_sixteen_lane_groups(monkeypatch):
    """The 16-lane instance of the octree march (MILOC_LANES=16) agrees with
    the oracle like the default 8-lane one."""
    monkeypatch.setenv("MILOC_LANES", "16")
    w = oct_workload()
    lf = leaf_rows(w)
    ref = oracle.run_oct(w.mol, w.model, w.spec, w.T_bg, 2)
    ctx = make_ctx(w)
    ctx.run(2)
    assert ctx.counters()["march_lanes"] == 16
    assert_pops(ctx.populations()[lf], ref.x[lf], 1e-5, "octree 16 lanes")
    ctx.close()


@pytest.mark.parametrize("fp64,tol", [(False, 1e-5), (True, 1e-10)])
def test_octree_lattice_iterations(fp64, tol):
    """The brute-force lattice (miloc_set_octree_rays): 4^2 straight lines per
    root element of a two-level tree, every iteration against the oracle's
    lattice march; the scheme's rays are restored by switching back."""
    w = oct_workload(n_refine=2)
    lf = leaf_rows(w)
    print(f"[octree lattice] cells per level {w.model.n_cells_per_level} fp64={fp64}", flush=True)
    ref = oracle.run_oct(w.mol, w.model, w.spec, w.T_bg, 3, brute=True)
    ctx = make_ctx(w, fp64=fp64)
    ctx.set_octree_rays(True)
    for it in range(3):
        ctx.run(1)
        assert_pops(ctx.populations()[lf], ref.history[it]["x"][lf], tol, f"octree lattice it {it}")
    ctx.set_octree_rays(False)
    ctx.init_lte()
    ctx.run(2)
    ref_s = oracle.run_oct(w.mol, w.model, w.spec, w.T_bg, 2)
    assert_pops(ctx.populations()[lf], ref_s.x[lf], tol, "octree scheme after the lattice")
    ctx.close()
