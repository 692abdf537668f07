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


def assert_radiation(J, Lam, rJ, rL, fp64, label):
    """J relative per entry; Lambda relative where it is not negligible
    against 1 - Lambda (there its absolute error is what the solve sees)."""
    rtol = 1e-9 if fp64 else 2e-5
    eJ = float(np.max(np.abs(J - rJ) / np.abs(rJ)))
    eL = float(np.max(np.abs(Lam - rL) / (np.abs(rL) + 1e-9)))
    print(f"[parity] {label} J max rel {eJ:.3e}, Lambda max rel {eL:.3e}", flush=True)
    assert eJ <= rtol, (label, eJ)
    assert eL <= rtol, (label, eL)


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
    # both in CGS intensity units: J of the external field and the diagonal
    # operator per leaf and transition
    assert_radiation(J[:, lf], Lam[:, lf], rJ[:, lf], rL[:, lf], fp64, "octree it 2")
    cnt = ctx.counters()
    print(f"[octree] march {cnt['march_ms']:.2f} ms over {cnt['march_launches']} launches, "
          f"{cnt['ray_steps']:.3e} steps", flush=True)
    sp = ctx.spectra(0, n_los=w.model.n0[0] ** 2)
    sref = oracle.spectra_oct(w.mol, w.model, w.spec, w.T_bg, ref.x, 0)
    assert_spectra(sp, sref, 1e-4 if not fp64 else 1e-9, "octree +z map")
    ctx.close()


@pytest.mark.parametrize("fp64,nch,tol", [(True, 256, 1e-10), (False, 600, 1e-5)])
def test_octree_wide_vectors(fp64, nch, tol):
    """Channel vectors whose workgroup needs more than 64 KB of LDS (FP64 at
    256 channels, FP32 at 600): populations, J and Lambda per leaf against
    the oracle over two iterations."""
    w = oct_workload(nch=nch, n_refine=2)
    print(f"[octree] wide vectors fp64={fp64} nch={nch} cells {w.model.n_cells_per_level}", flush=True)
    lf = leaf_rows(w)
    ref = oracle.run_oct(w.mol, w.model, w.spec, w.T_bg, 2)
    ctx = make_ctx(w, fp64=fp64)
    for it in range(2):
        ctx.run(1)
        assert_pops(ctx.populations()[lf], ref.history[it]["x"][lf], tol, f"octree wide it {it}")
    J, Lam = ctx.radiation()
    assert_radiation(J[:, lf], Lam[:, lf], ref.history[1]["J"][:, lf], ref.history[1]["Lam"][:, lf], fp64,
                     "octree wide it 1")
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


def refined_once(cube):
    """The octree whose N^3 root cells (cell size 2h) are all split once into
    the cells of the (2N)^3 grid `cube` (cell size h): fields per fine cell
    moved to the children, the roots carry their children's means."""
    M = cube.n0[0]
    N = M // 2
    ii = np.arange(N)
    z, y, x = np.meshgrid(ii, ii, ii, indexing="ij")
    roots = ((z * N + y) * N + x).ravel()            # level-0 order
    fine = []
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                fine.append((((2 * z + cz) * M + (2 * y + cy)) * M + (2 * x + cx)).ravel())
    fine = np.stack(fine, axis=1)                    # [root][child cx + 2 cy + 4 cz]
    order = fine[roots].ravel()                      # level-1 cells, children of root i at 8 i ...

    def field(a):
        a = np.asarray(a, np.float32)
        return np.concatenate([a[fine].mean(axis=1).astype(np.float32), a[order]])

    m = synth.Model3D(n0=(N, N, N), root_cell_cm=2.0 * cube.root_cell_cm,
                      n_H2=field(cube.n_H2), T_kin=field(cube.T_kin), b_turb=field(cube.b_turb),
                      vx=field(cube.vx), vy=field(cube.vy), vz=field(cube.vz),
                      abundance=field(cube.abundance), n_oct_levels=2,
                      n_cells_per_level=[N ** 3, 8 * N ** 3],
                      first_child=[(8 * np.arange(N ** 3)).astype(np.int32),
                                   np.full(8 * N ** 3, -1, np.int32)])
    return m, order


@pytest.mark.parametrize("fp64,tol", [(False, 2e-6), (True, 1e-9)])
def test_refined_once_octree_equals_fine_grid_on_gpu(fp64, tol):
    """Every root cell split once: the octree scheme's rays are the (2N)^3
    grid's rays (the splits happen on the model boundary, where every ray
    still carries the background), so the library's two independent device
    paths -- the regular grid's crossing patterns and march, and the octree's
    host ray schedule and march -- give the same populations, J and Lambda on
    every fine cell (Sect. 2.2; equivalence P9b of the oracle, here without
    the oracle)."""
    cube = synth.turbulent_cube(N=8, box_pc=0.1, seed=23, abundance=2e-7)
    octm, order = refined_once(cube)
    mol = synth.rotor_molecule(5)
    spec = synth.Spectral.symmetric(128, 4.0)
    w_reg = synth.Workload("r", mol, spec, 2.73, cube, 2)
    w_oct = synth.Workload("o", mol, spec, 2.73, octm, 2)
    print(f"[case] refined-once octree vs 8^3 grid fp64={fp64}", flush=True)
    a, b = make_ctx(w_reg, fp64=fp64), make_ctx(w_oct, fp64=fp64)
    a.run(3)
    b.run(3)
    nroot = 4 ** 3
    xr = a.populations()[order]
    xo = b.populations()[nroot:]
    assert_pops(xo, xr, tol, f"refined-once octree vs grid fp64={fp64}")
    Jr, Lr = a.radiation()
    Jo, Lo = b.radiation()
    assert np.allclose(Jo[:, nroot:], Jr[:, order], rtol=tol, atol=0)
    assert np.allclose(Lo[:, nroot:], Lr[:, order], rtol=10 * tol, atol=1e-12)
    a.close()
    b.close()


def test_octree_full_size_sampled_direction():
    """The 64^3-root, four-level cloud (2.25e7 cells) marched along one
    HEALPix direction from LTE: J and Lambda of every leaf for two of the
    nine transitions against the oracle's march of the same direction."""
    w = synth.workload_octree()
    m = w.model
    q = 13
    d = oracle.healpix_nside2()[q:q + 1]
    print(f"[case] octree full size, direction {q}, cells per level {m.n_cells_per_level}", flush=True)
    ctx = make_ctx(w, dirs=d)
    ctx.run(1)
    J, Lam = ctx.radiation()
    ctx.close()
    tree = oracle.octree_of(m)
    lf = tree.leaf
    prob = oracle._Problem(w.mol, m.n_H2, m.T_kin, m.b_turb, m.abundance, w.spec, w.T_bg)
    x0 = oracle.lte_populations(w.mol, prob.T)
    kap, eta = oracle.prepare(w.mol, x0, prob.n_mol)
    for t in (0, 4):
        res, _ = oracle.march_oct(tree, float(m.root_cell_cm), m.vx, m.vy, m.vz, prob.bD, kap[t], eta[t],
                                  d, w.spec, prob.I_bg[t])
        W = res.W[lf]
        assert np.all(W > 0)
        assert_radiation(J[t, lf], Lam[t, lf], res.Jraw[lf] / W, res.Lraw[lf] / W, False,
                         f"octree full size direction {q} t={t}")


def test_octree_reduced_copy_to_convergence():
    """An 8^3-root copy of the octree cloud (four levels, densest 34% refined
    per level, the same generators; box scaled so that root cells keep their
    size), 48 directions, FP32 march: populations of every leaf at
    convergence (1e-6) against the oracle run to the same tolerance."""
    m = synth.octree_cloud(N_root=8, n_refine=4, frac=0.34, grf_N=32, box_pc=0.25, abundance=1e-9, seed=4001)
    w = synth.Workload("oct-8", synth.rotor_molecule(10), synth.Spectral.symmetric(256, 4.0), 2.73, m, 40)
    lf = leaf_rows(w)
    print(f"[case] octree 8^3 root to 1e-6, cells per level {m.n_cells_per_level}", flush=True)
    ref = oracle.run_oct(w.mol, m, w.spec, w.T_bg, 40, tol=1e-6, record=False)
    ctx = make_ctx(w)
    it, last = ctx.run(40, tol=1e-6, allow_notconv=False)
    print(f"[parity] octree-8 converged: gpu {it} iterations (delta {last:.2e}), oracle {ref.iters}", flush=True)
    assert abs(it - ref.iters) <= 1
    assert_pops(ctx.populations()[lf], ref.x[lf], 1e-5, "octree-8 converged")
    ctx.close()
