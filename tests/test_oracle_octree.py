"""Pins of the oracle's octree march (Sect. 2.2) against what the geometry and
the transfer equation fix independently: the per-leaf path-length invariant,
the equivalence with regular grids, uniform-field invariance, photon
conservation, the slab solution along lines of sight, and detailed balance."""
import math

import numpy as np
import pytest

import oracle
import synth

KMS = 1.0e5

SPECIAL = [(0, 0, 1), (1, 0, 0), (-1, 0, 0), (0, -1, 0), (1, 1, 1), (-1, 1, -1), (1, 1, 0),
           (1, -1, 0), (0, 1, 1), (2, 1, 0), (1, 2, 2), (3, 1, 1)]


def _dirs_all():
    rng = np.random.default_rng(0)
    extra = [np.asarray(d, float) / np.linalg.norm(d) for d in SPECIAL]
    extra += [v / np.linalg.norm(v) for v in rng.normal(size=(8, 3))]
    return np.concatenate([oracle.healpix_nside2(), np.array(extra)])


@pytest.mark.parametrize("N,nref,frac,seed", [(4, 0, 0.0, 1), (4, 2, 0.3, 2), (3, 3, 0.35, 3),
                                              (2, 4, 0.6, 5), (5, 2, 0.5, 7)])
def test_p8_octree_path_per_leaf(N, nref, frac, seed):
    """Per direction, every leaf of level L is crossed by a total path of
    h_L/|d_m| with ray weight h_L^2 |d_m|: W = volume, exactly; refined cells
    are never stepped through.  Any missing or doubled ray (split, side ray,
    termination, wrap) shows up as an error of order one."""
    m = synth.octree_random(N, nref, frac, seed, 1.0 * N, 1e3, 10.0, 0.0, 1e-9)
    tree = oracle.octree_of(m)
    V = (0.5 ** tree.level) ** 3
    for d in _dirs_all():
        res, st = oracle.march_oct(tree, 1.0, *([None] * 6), d[None, :], None, 0.0)
        err = np.abs(res.W - np.where(tree.leaf, V, 0.0)) / V
        assert np.max(err) < 1e-12, (d, np.max(err))
        assert st["root"] == N * N
        if nref == 0:
            assert st["split"] == st["side"] == st["terminated"] == 0


def test_octree_ray_bookkeeping_counts():
    """Rays created = rays ended: every ray ends once, by termination or by
    leaving through the downstream face, and one line of the finest lattice
    leaves per finest downstream element whose leaf admits it."""
    m = synth.octree_random(3, 3, 0.4, 9, 3.0, 1e3, 10.0, 0.0, 1e-9)
    tree = oracle.octree_of(m)
    for d in oracle.healpix_nside2()[[0, 7, 22, 40]]:
        res, st = oracle.march_oct(tree, 1.0, *([None] * 6), d[None, :], None, 0.0)
        started = st["root"] + st["split"] + st["side"]
        assert st["split"] % 3 == 0
        assert started - st["terminated"] >= tree.N ** 2


def _tree_fields(tree, seed, vmax_kms=0.5):
    rng = np.random.default_rng(seed)
    nc = tree.child.shape[0]
    v = rng.normal(scale=vmax_kms * KMS, size=(3, nc))
    b = rng.uniform(0.15, 0.3, nc) * KMS
    kap = rng.uniform(0.5, 2.0, nc) * 3e-13
    eta = rng.uniform(0.5, 2.0, nc) * 1e-27
    return v, b, kap, eta


def test_p9_unrefined_octree_equals_regular_grid():
    N, delta = 5, 1.0e16
    spec = synth.Spectral.symmetric(48, 3.0)
    m = synth.octree_random(N, 0, 0.0, 1, N * delta, 1e3, 10.0, 0.0, 1e-9)
    tree = oracle.octree_of(m)
    v, b, kap, eta = _tree_fields(tree, 3)
    dirs = oracle.healpix_nside2()
    o, _ = oracle.march_oct(tree, delta, v[0], v[1], v[2], b, kap, eta, dirs, spec, 1.5e-15)
    r = oracle.march_3d(N, delta, v[0], v[1], v[2], b, kap, eta, dirs, spec, 1.5e-15)
    for a, c in ((o.Jraw, r.Jraw), (o.Lraw, r.Lraw), (o.W, r.W), (o.E, r.E)):
        assert np.allclose(a, c, rtol=1e-12, atol=0)


def test_p9_uniformly_refined_octree_equals_fine_grid():
    """Every root cell split once: the rays split only on the model boundary,
    where all carry the background, so the march equals the (2N)^3 grid."""
    N, delta = 3, 2.0e16
    spec = synth.Spectral.symmetric(48, 3.0)
    coords, fc = synth.octree_structure(N, 1, 1.0, lambda l, x, y, z: np.zeros(x.shape[0]))
    assert len(fc) == 2 and (fc[0] >= 0).all()
    tree = oracle.octree_of(synth.Model3D(n0=(N,) * 3, root_cell_cm=delta, n_H2=None, T_kin=None,
                                          b_turb=None, vx=None, vy=None, vz=None, abundance=None,
                                          n_oct_levels=2, n_cells_per_level=[N ** 3, 8 * N ** 3],
                                          first_child=fc))
    v, b, kap, eta = _tree_fields(tree, 4)
    dirs = oracle.healpix_nside2()
    o, st = oracle.march_oct(tree, delta, v[0], v[1], v[2], b, kap, eta, dirs, spec, 1.5e-15)
    assert st["side"] == 0 and st["terminated"] == 0
    N2 = 2 * N
    kx, ky, kz = coords[1]
    reg = (kz * N2 + ky) * N2 + kx                  # regular index of each level-1 cell
    leaves = np.arange(N ** 3, N ** 3 + 8 * N ** 3)
    F = lambda a: np.zeros(N2 ** 3) + np.bincount(reg, weights=a[leaves], minlength=N2 ** 3)
    r = oracle.march_3d(N2, delta / 2, F(v[0]), F(v[1]), F(v[2]), F(b), F(kap), F(eta), dirs, spec,
                        1.5e-15)
    for a, c in ((o.Jraw, r.Jraw), (o.Lraw, r.Lraw), (o.W, r.W)):
        assert np.allclose(a[leaves], c[reg], rtol=1e-12, atol=0)
        assert np.all(a[:N ** 3] == 0)


def _source_pops(mol, T):
    return oracle.lte_populations(mol, np.array([T]))[0]


def test_p2_uniform_field_octree_with_velocity():
    """S = I_bg everywhere: every ray, split and side ray included, carries
    I_bg unchanged, so J_LI = I_bg sum_c f_c on every leaf."""
    mol = synth.two_level_molecule()
    spec = synth.Spectral.symmetric(64, 4.0)
    m = synth.octree_cloud(N_root=4, n_refine=3, frac=0.35, grf_N=16, box_pc=0.1,
                           abundance=1e-6, T_kin=10.0, b_turb_kms=0.2, seed=77)
    tree = oracle.octree_of(m)
    T_bg = 2.73
    x = np.tile(_source_pops(mol, T_bg), (tree.child.shape[0], 1))
    prob = oracle._Problem(mol, m.n_H2, m.T_kin, m.b_turb, m.abundance, spec, T_bg)
    kap, eta = oracle.prepare(mol, x, prob.n_mol)
    I_bg = float(prob.I_bg[0])
    r, st = oracle.march_oct(tree, m.root_cell_cm, m.vx.astype(float), m.vy.astype(float),
                             m.vz.astype(float), prob.bD, kap[0], eta[0], oracle.healpix_nside2(),
                             spec, I_bg)
    assert st["split"] > 0 and st["side"] > 0
    lf = tree.leaf
    JLI = r.Jraw + (eta[0] / kap[0]) * r.Lraw
    assert np.allclose(JLI[lf], I_bg * r.E[lf], rtol=1e-12)
    assert np.max(r.Lraw[lf] / r.W[lf]) > 1e-3


def test_p6_conservation_octree():
    """Per step I_in + eta p s = I_out + absorbed: summed over every step of
    every ray (weights change with the level), the identity
    sum a dv (I_in - I_out) + sum eta E = sum W (kappa J + eta Lambda) holds."""
    mol = synth.rotor_molecule(4)
    spec = synth.Spectral.symmetric(64, 4.0)
    m = synth.octree_cloud(N_root=4, n_refine=2, frac=0.4, grf_N=16, box_pc=0.05,
                           abundance=1e-5, T_kin=12.0, b_turb_kms=0.15, seed=21)
    tree = oracle.octree_of(m)
    prob = oracle._Problem(mol, m.n_H2, m.T_kin, m.b_turb, m.abundance, spec, 2.73)
    x = oracle.lte_populations(mol, np.full(tree.child.shape[0], 8.0))
    kap, eta = oracle.prepare(mol, x, prob.n_mol)
    for t in range(mol.n_trans):
        r, _ = oracle.march_oct(tree, m.root_cell_cm, m.vx.astype(float), m.vy.astype(float),
                                m.vz.astype(float), prob.bD, kap[t], eta[t],
                                oracle.healpix_nside2(), spec, prob.I_bg[t])
        lf = tree.leaf
        lhs = r.cons + np.sum(eta[t][lf] * r.E[lf])
        rhs = np.sum(kap[t][lf] * r.Jraw[lf] + eta[t][lf] * r.Lraw[lf])
        assert math.isclose(lhs, rhs, rel_tol=1e-11), (t, lhs, rhs)


def test_p1_octree_line_of_sight_slab():
    """A uniform static octree seen along +z: each line of sight is a slab of
    depth N root cells whatever the refinement it crosses."""
    N, delta = 4, 1.0e16
    spec = synth.Spectral.symmetric(32, 1.5)
    b = 0.2 * KMS
    mol = synth.two_level_molecule()
    m = synth.octree_random(N, 2, 0.4, 3, N * delta, 1e4, 10.0, b, 5e-5)
    tree = oracle.octree_of(m)
    nc = tree.child.shape[0]
    x = np.tile(_source_pops(mol, 25.0), (nc, 1))
    sp = oracle.spectra_oct(mol, m, spec, 2.73, x, 0)
    prob = oracle._Problem(mol, m.n_H2, m.T_kin, m.b_turb, m.abundance, spec, 2.73)
    kap, eta = oracle.prepare(mol, x, prob.n_mol)
    v = spec.v_min + (np.arange(spec.n_channels) + 0.5) * spec.dv
    bD = prob.bD[0]
    p = np.exp(-(v / bD) ** 2) / (bD * math.sqrt(math.pi))
    tau = kap[0][0] * p * N * delta
    S = eta[0][0] / kap[0][0]
    I_bg = prob.I_bg[0]
    expect = S * (1 - np.exp(-tau)) + I_bg * np.exp(-tau) - I_bg
    assert np.max(tau) > 1.0
    assert np.allclose(sp, expect[None, :], rtol=1e-12, atol=1e-12 * np.max(np.abs(expect)))


def test_p5_detailed_balance_octree():
    """Uniform T and T_bg = T_kin: Boltzmann populations are the fixed point on
    every leaf, also after the splits, side rays and terminations."""
    mol = synth.rotor_molecule(4)
    T = 11.0
    m = synth.octree_cloud(N_root=4, n_refine=2, frac=0.35, grf_N=16, box_pc=0.1, T_kin=T,
                           abundance=2e-6, b_turb_kms=0.1, seed=55)
    spec = synth.Spectral.symmetric(160, 3.0)          # dv = b/3.4: sum_c f_c = 1
    lte = oracle.lte_populations(mol, m.T_kin.astype(float))
    run = oracle.run_oct(mol, m, spec, T, 1)
    lf = oracle.octree_of(m).leaf
    assert np.allclose(run.x[lf], lte[lf], rtol=1e-10, atol=1e-16)
    J = run.history[0]["J"]
    assert np.max(run.history[0]["Lam"][:, lf]) > 1e-2       # not transparent
    assert np.all(np.isfinite(J))


# ---------------------------------------------------------------------------
# Brute-force lattice (Sect. 2.2: 4^Lmax straight lines per root element)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N,nref,frac,seed", [(4, 2, 0.3, 2), (3, 3, 0.35, 3), (2, 4, 0.6, 5)])
def test_brute_path_per_leaf(N, nref, frac, seed):
    """Every finest-lattice line, weight h_Lmax^2 |d_m|: each leaf again
    carries W = its volume exactly, with no created or terminated rays."""
    m = synth.octree_random(N, nref, frac, seed, 1.0 * N, 1e3, 10.0, 0.0, 1e-9)
    tree = oracle.octree_of(m)
    V = (0.5 ** tree.level) ** 3
    for d in _dirs_all()[::3]:
        res, st = oracle.march_oct(tree, 1.0, *([None] * 6), d[None, :], None, 0.0, brute=True)
        err = np.abs(res.W - np.where(tree.leaf, V, 0.0)) / V
        assert np.max(err) < 1e-12, (d, np.max(err))
        assert st["root"] == (N << tree.Lmax) ** 2
        assert st["split"] == st["side"] == st["terminated"] == 0


def test_brute_equals_fine_grid_for_root_constant_fields():
    """Fields constant within each root cell: a straight line crossing a leaf
    in one step sees the same medium as the finest regular grid crossing it in
    several, so the lattice march equals the (N 2^Lmax)^3 grid march in the
    path-averaged intensity J + S Lambda and in W, leaf by leaf."""
    N, delta = 3, 2.0e16
    spec = synth.Spectral.symmetric(48, 3.0)
    m = synth.octree_random(N, 2, 0.4, 11, N * delta, 1e3, 10.0, 0.0, 1e-9)
    tree = oracle.octree_of(m)
    L = tree.Lmax
    rng = np.random.default_rng(12)
    nroot = N ** 3
    v = rng.normal(scale=0.3 * KMS, size=(3, nroot))
    b = rng.uniform(0.15, 0.3, nroot) * KMS
    kap = rng.uniform(0.5, 2.0, nroot) * 3e-13
    eta = rng.uniform(0.5, 2.0, nroot) * 1e-27
    # root ancestor of every cell and the leaf of every finest cell
    nc = tree.child.shape[0]
    root_of = np.arange(nc)
    for lev in range(1, L + 1):
        for g in range(int(tree.offsets[lev - 1]), int(tree.offsets[lev])):
            c = tree.child[g]
            if c >= 0:
                root_of[c:c + 8] = root_of[g]
    cx, cy, cz = synth.octree_centres(N, _coords_of(tree))
    F = lambda a: a[root_of]
    dirs = oracle.healpix_nside2()[::2]
    o, st = oracle.march_oct(tree, delta, F(v[0]), F(v[1]), F(v[2]), F(b), F(kap), F(eta), dirs, spec,
                             1.5e-15, brute=True)
    Nf = N << L
    fx, fy, fz = np.meshgrid(np.arange(Nf), np.arange(Nf), np.arange(Nf), indexing="ij")
    fx, fy, fz = fx.ravel(), fy.ravel(), fz.ravel()
    freg = (fz * Nf + fy) * Nf + fx
    froot = ((fz >> L) * N + (fy >> L)) * N + (fx >> L)
    G = lambda a: np.zeros(Nf ** 3) + np.bincount(freg, weights=a[froot], minlength=Nf ** 3)
    r = oracle.march_3d(Nf, delta / (1 << L), G(v[0]), G(v[1]), G(v[2]), G(b), G(kap), G(eta), dirs, spec,
                        1.5e-15)
    # leaf of each finest cell
    leaf_of = np.full(Nf ** 3, -1, np.int64)
    for g in np.flatnonzero(tree.leaf):
        s = 1 << (L - tree.level[g])
        x0 = int(round(cx[g] * Nf - 0.5 * s))
        y0 = int(round(cy[g] * Nf - 0.5 * s))
        z0 = int(round(cz[g] * Nf - 0.5 * s))
        xs, ys, zs = np.meshgrid(np.arange(x0, x0 + s), np.arange(y0, y0 + s), np.arange(z0, z0 + s), indexing="ij")
        leaf_of[((zs * Nf + ys) * Nf + xs).ravel()] = g
    assert (leaf_of >= 0).all()
    S = eta / kap
    JLI_f = r.Jraw + G(S) * r.Lraw
    sum_leaf = lambda a: np.bincount(leaf_of, weights=a, minlength=nc)
    lf = tree.leaf
    JLI_o = o.Jraw + F(S) * o.Lraw
    assert np.allclose(JLI_o[lf], sum_leaf(JLI_f)[lf], rtol=1e-11, atol=0)
    assert np.allclose(o.W[lf], sum_leaf(r.W)[lf], rtol=1e-12, atol=0)


def _coords_of(tree):
    """Integer coordinates per level of every cell (from the child links)."""
    N, L = tree.N, tree.Lmax
    coords = []
    iz, iy, ix = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    cur = (ix.ravel().astype(np.int64), iy.ravel().astype(np.int64), iz.ravel().astype(np.int64))
    coords.append(cur)
    for lev in range(1, L + 1):
        n = int(tree.offsets[lev + 1] - tree.offsets[lev])
        x = np.zeros(n, np.int64); y = np.zeros(n, np.int64); z = np.zeros(n, np.int64)
        base = int(tree.offsets[lev - 1])
        for k in range(int(tree.offsets[lev] - base)):
            c = tree.child[base + k]
            if c < 0:
                continue
            j = c - int(tree.offsets[lev])
            for o in range(8):
                x[j + o] = 2 * coords[lev - 1][0][k] + (o & 1)
                y[j + o] = 2 * coords[lev - 1][1][k] + ((o >> 1) & 1)
                z[j + o] = 2 * coords[lev - 1][2][k] + ((o >> 2) & 1)
        coords.append((x, y, z))
    return coords


def test_brute_uniform_field_invariance():
    """S = I_bg everywhere: J + S Lambda = I_bg sum_c f_c on every leaf also
    for the straight-line lattice."""
    mol = synth.two_level_molecule()
    spec = synth.Spectral.symmetric(64, 4.0)
    m = synth.octree_cloud(N_root=3, n_refine=2, frac=0.35, grf_N=12, box_pc=0.1,
                           abundance=1e-6, T_kin=10.0, b_turb_kms=0.2, seed=78)
    tree = oracle.octree_of(m)
    x = np.tile(_source_pops(mol, 2.73), (tree.child.shape[0], 1))
    prob = oracle._Problem(mol, m.n_H2, m.T_kin, m.b_turb, m.abundance, spec, 2.73)
    kap, eta = oracle.prepare(mol, x, prob.n_mol)
    I_bg = float(prob.I_bg[0])
    r, _ = oracle.march_oct(tree, m.root_cell_cm, m.vx.astype(float), m.vy.astype(float),
                            m.vz.astype(float), prob.bD, kap[0], eta[0], oracle.healpix_nside2()[::4],
                            spec, I_bg, brute=True)
    lf = tree.leaf
    JLI = r.Jraw + (eta[0] / kap[0]) * r.Lraw
    assert np.allclose(JLI[lf], I_bg * r.E[lf], rtol=1e-10, atol=0)


def test_scheme_and_lattice_agree_physically():
    """Two discretisations of the same octree cloud (root 4^3, two refinement
    levels, thick lines): the created and ended rays of the octree scheme and
    the brute-force lattice give populations within a few percent (the side
    rays' copied intensities are the scheme's approximation), 1e-3 on
    average."""
    m = synth.octree_cloud(N_root=4, n_refine=2, frac=0.35, grf_N=16, box_pc=0.2, abundance=1e-7, seed=4001)
    w = synth.Workload("oct-4", synth.rotor_molecule(5), synth.Spectral.symmetric(128, 4.0), 2.73, m, 6)
    lf = oracle.octree_of(w.model).leaf
    b = oracle.run_oct(w.mol, w.model, w.spec, w.T_bg, 6, brute=True, record=False)
    s = oracle.run_oct(w.mol, w.model, w.spec, w.T_bg, 6, record=False)
    xb, xs = b.x[lf], s.x[lf]
    big = xs > 1e-4
    rel = np.abs(xb[big] - xs[big]) / xs[big]
    print(f"[lattice vs scheme] max {rel.max():.3e} mean {rel.mean():.3e}")
    assert rel.max() < 0.08 and rel.mean() < 2e-3
    assert rel.max() > 1e-4          # not the same rays
