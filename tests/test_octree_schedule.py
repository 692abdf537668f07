"""Host logic of the octree march: the ray schedule the library builds on
the host (no device needed) against the oracle's octree march.  The replay
below follows the record format of miloc_octree_schedule; it is the
semantics the device kernel implements."""
import math

import numpy as np
import pytest

import oracle
import synth

miloc = pytest.importorskip("paper_2009_12609_amd")

CELL = 0x0FFFFFFF


def _model(N, nref, frac, seed):
    return synth.octree_random(N, nref, frac, seed, 1.0 * N, 1e3, 10.0, 0.0, 1e-9)


def _dirs():
    extra = [(0, 0, 1), (1, 1, 1), (-1, 1, -1), (1, -1, 0), (2, 1, 0)]
    return np.concatenate([oracle.healpix_nside2(),
                           np.array([np.asarray(d, float) / np.linalg.norm(d) for d in extra])])


@pytest.mark.parametrize("N,nref,frac,seed", [(4, 0, 0.0, 1), (3, 2, 0.35, 2), (2, 3, 0.5, 3)])
def test_schedule_paths_match_oracle(N, nref, frac, seed):
    """Per direction and leaf: the same number of steps as the oracle's rays
    and the same total path (each leaf of level L: 2^-L/|d_m|)."""
    m = _model(N, nref, frac, seed)
    tree = oracle.octree_of(m)
    nc = tree.child.shape[0]
    for d in _dirs():
        steps, trees, depth = miloc.octree_schedule(m, d[None, :])
        cell = (steps[:, 0] & CELL).astype(np.int64)
        ln = steps[:, 1].view(np.float32).astype(np.float64)
        assert cell.max() < nc and np.all(tree.child[cell] < 0)       # leaves only
        path = np.bincount(cell, weights=ln, minlength=nc)
        dm = np.max(np.abs(d))
        expect = np.where(tree.leaf, 0.5 ** tree.level / dm, 0.0)
        assert np.allclose(path, expect, rtol=2e-6, atol=0)
        res, st = oracle.march_oct(tree, 1.0, *([None] * 6), d[None, :], None, 0.0)
        assert st["steps"] == steps.shape[0]
        # trees cover the records exactly once, largest first
        assert trees.shape[0] == N * N
        assert np.all(np.diff(trees[:, 1]) <= 0)
        cover = np.zeros(steps.shape[0], int)
        for off, n, q, r in trees:
            cover[off:off + n] += 1
        assert np.all(cover == 1)


@pytest.mark.parametrize("N,nref,frac,seed", [(3, 2, 0.35, 2), (2, 3, 0.5, 3)])
def test_lattice_schedule_matches_oracle(N, nref, frac, seed):
    """The brute-force lattice: per direction and leaf of level L the lines
    cross it along h_L^3 / (h_Lmax^2 |d_m|) in all, with the oracle's step
    count; every line starts from the background and nothing is saved."""
    m = _model(N, nref, frac, seed)
    tree = oracle.octree_of(m)
    nc = tree.child.shape[0]
    hmax = 0.5 ** tree.Lmax
    for d in _dirs()[::2]:
        steps, trees, depth = miloc.octree_schedule(m, d[None, :], lattice=True)
        assert depth == 0
        cell = (steps[:, 0] & CELL).astype(np.int64)
        ln = steps[:, 1].view(np.float32).astype(np.float64)
        assert np.all(tree.child[cell] < 0)
        assert not np.any(steps[:, 0] & (1 << 28))                     # no saved vectors
        assert np.all((steps[:, 0] >> 29) <= 1)                        # continue or background only
        path = np.bincount(cell, weights=ln, minlength=nc)
        dm = np.max(np.abs(d))
        expect = np.where(tree.leaf, (0.5 ** tree.level) ** 3 / (hmax ** 2 * dm), 0.0)
        assert np.allclose(path, expect, rtol=2e-6, atol=0)
        res, st = oracle.march_oct(tree, 1.0, *([None] * 6), d[None, :], None, 0.0, brute=True)
        assert st["steps"] == steps.shape[0]
        starts = int(np.sum((steps[:, 0] >> 29) == 1))
        assert starts == st["root"] + st["wrapped"]
        assert trees.shape[0] == N * N


def _replay(steps, trees, dirs, tree, root_cm, v, bD, kap, eta, spec, I_bg):
    """FP64 replay of a schedule: per tree, records in order; intensity start
    modes and the saved-vector stack as documented for the records."""
    nc = tree.child.shape[0]
    J = np.zeros(nc)
    Lm = np.zeros(nc)
    vc = spec.v_min + (np.arange(spec.n_channels) + 0.5) * spec.dv
    for off, n, q, r in trees:
        d = dirs[q]
        aw = np.max(np.abs(d))
        stack = []
        I = np.full(spec.n_channels, I_bg)
        for s in range(off, off + n):
            w0 = int(steps[s, 0])
            k = w0 & CELL
            mode = w0 >> 29
            if mode == 1:
                I = np.full(spec.n_channels, I_bg)
            elif mode >= 2:
                I = stack[-1].copy()
                if mode == 3:
                    stack.pop()
            if w0 & (1 << 28):
                stack.append(I.copy())
            hl = 0.5 ** tree.level[k]
            s_cm = float(steps[s, 1:2].view(np.float32)[0]) * root_cm
            a = (hl * root_cm) ** 2 * aw
            w = v[0][k] * d[0] + v[1][k] * d[1] + v[2][k] * d[2]
            p = np.exp(-((vc + w) / bD[k]) ** 2) / (bD[k] * math.sqrt(math.pi))
            f = p * spec.dv
            tau = kap[k] * p * s_cm
            beta = np.where(np.abs(tau) < 1e-8, 1.0 - tau / 2, -np.expm1(-tau) / np.where(tau == 0, 1, tau))
            J[k] += a * s_cm * np.sum(f * I * beta)
            Lm[k] += a * s_cm * np.sum(f * (1 - beta))
            I = I * np.exp(-tau) + eta[k] * p * s_cm * beta
        assert not stack
    return J, Lm


def test_schedule_replay_equals_oracle_march():
    """Replaying the schedule (splits, side rays, terminations, saved vectors)
    gives the oracle's absorbed counts and Lambda sums."""
    N, root_cm = 2, 1.0e16
    m = _model(N, 2, 0.5, 8)
    tree = oracle.octree_of(m)
    nc = tree.child.shape[0]
    rng = np.random.default_rng(5)
    v = rng.normal(scale=0.3e5, size=(3, nc))
    bD = rng.uniform(0.15, 0.3, nc) * 1e5
    kap = rng.uniform(0.5, 2.0, nc) * 1e-12
    eta = rng.uniform(0.5, 2.0, nc) * 1e-27
    spec = synth.Spectral.symmetric(24, 1.5)
    dirs = oracle.healpix_nside2()[[0, 9, 17, 30, 45]]
    steps, trees, depth = miloc.octree_schedule(m, dirs)
    assert depth >= 1
    J, Lm = _replay(steps, trees, dirs, tree, root_cm, v, bD, kap, eta, spec, 2e-15)
    ref, st = oracle.march_oct(tree, root_cm, v[0], v[1], v[2], bD, kap, eta, dirs, spec, 2e-15)
    assert st["split"] > 0 and st["side"] > 0 and st["terminated"] > 0
    lf = tree.leaf
    assert np.allclose(J[lf], ref.Jraw[lf], rtol=2e-6, atol=0)
    assert np.allclose(Lm[lf], ref.Lraw[lf], rtol=2e-6, atol=1e-40)


def test_schedule_rejects_bad_trees():
    m = _model(2, 1, 0.5, 1)
    bad = synth.Model3D(**{**m.__dict__})
    fc = [t.copy() for t in m.first_child]
    fc[0][np.argmax(fc[0] >= 0)] = 3            # not a multiple of 8
    bad.first_child = fc
    with pytest.raises(miloc.MilocError):
        miloc.octree_schedule(bad, np.array([[0, 0, 1.0]]))


def test_lattice_refuses_oversize_schedules():
    """A deep tree's brute-force lattice is refused before it is built (the
    bound: (N 2^Lmax)^2 lines per direction of at most 3 N 2^Lmax steps),
    while the octree scheme's schedule of the same tree is built."""
    m = synth.octree_random(16, 4, 0.02, 13, 16.0, 1e3, 10.0, 0.0, 1e-9)
    rng = np.random.default_rng(1)
    d = rng.normal(size=(100, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    with pytest.raises(miloc.MilocError) as e:
        miloc.octree_schedule(m, d, lattice=True)
    assert e.value.code == miloc.EINVAL
    steps, trees, _ = miloc.octree_schedule(m, d[:2])
    assert steps.shape[0] > 0 and trees.shape[0] == 2 * 16 * 16
