"""Device-memory footprint of a model (miloc_model_footprint), host only: the
terms it must contain, counted independently here (window table, population,
opacity and sum arrays; the per-step sums of one transition from the oracle's
own count of crossing steps; the 1D ray steps from the oracle's ray
geometry)."""
import numpy as np
import pytest

import oracle
import synth

miloc = pytest.importorskip("paper_2009_12609_amd")


def test_regular_grid_footprint_terms():
    N, L, T, nch = 32, 10, 9, 256
    cube = synth.turbulent_cube(N=N, seed=3001, box_pc=0.25)
    fixed, sums = miloc.model_footprint(cube, L, T, nch)
    dirs = oracle.healpix_nside2()
    nc = N ** 3
    # one representative ray per direction: its step count times N^2 rays,
    # an FP32 pair per step
    steps = sum(len(oracle.walk_3d(N, d, 0, 0)[0]) for d in dirs)
    assert sums == steps * N * N * 8
    core = 48 * nc * 16 + 2 * nc * L * 8 + T * nc * 8 + T * nc * 16
    assert core <= fixed <= 1.1 * core
    f64, s64 = miloc.model_footprint(cube, L, T, nch, fp64=True)
    assert s64 == 2 * sums and f64 > fixed
    big, bsum = miloc.model_footprint(synth.uniform_cube(64, 1e18, 1e3, 15.0, 0.0, 1e-9), L, T, nch)
    assert 7.5 < big / fixed < 8.5 and 7.5 < bsum / sums < 8.5      # both scale as N^3


def test_shell_model_footprint_counts_the_ray_steps():
    w = synth.workload_1d_plummer(n_shells=300)
    fixed, sums = miloc.model_footprint(w.model, 10, 9, 256)
    assert sums == 0
    R = w.model.r_out
    b = oracle.equidistant_impacts(R[-1], w.model.n_rays)
    steps = sum(len(oracle.ray_steps_1d(R, bj)[0]) for bj in b)
    assert fixed >= steps * 8 + 2 * 300 * 10 * 8
    assert fixed <= steps * 8 + 300 * 1000 + 300 * 200


def test_octree_footprint_uses_the_schedule():
    m = synth.octree_cloud(N_root=4, n_refine=2, frac=0.35, grf_N=16, box_pc=0.1, abundance=1e-8)
    dirs = oracle.healpix_nside2()
    steps, trees, _ = miloc.octree_schedule(m, dirs)
    fixed, sums = miloc.model_footprint(m, 5, 4, 128, oct_steps=steps.shape[0])
    assert sums == steps.shape[0] * 2 * 4 * 2          # FP32 rows of two transitions
    assert fixed >= (2 << 30) + steps.shape[0] * 12 + 48 * m.n_cells * 16


def test_footprint_argument_errors():
    cube = synth.uniform_cube(4, 1e18, 1e3, 15.0, 0.0, 1e-9)
    for bad in [dict(n_levels=1), dict(n_trans=0), dict(n_channels=0)]:
        args = dict(n_levels=5, n_trans=4, n_channels=64)
        args.update(bad)
        with pytest.raises(miloc.MilocError):
            miloc.model_footprint(cube, **args)
