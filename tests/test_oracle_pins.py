"""Pins of the FP64 oracle against closed forms, limits and invariants.

None of these re-types the oracle's own formulas: each compares it with a
result the mathematics fixes independently (closed-form transfer solutions,
the Boltzmann limits, conservation laws, geometric invariants, brute force on
tiny inputs, or LAPACK on the same matrices), chosen so that a dropped term,
a wrong sign or a transposed index in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import synth

KMS = 1.0e5


def _spec(nch=64, half=2.0):
    return synth.Spectral.symmetric(nch, half)


def _thin_two_level():
    return synth.two_level_molecule()


# ---------------------------------------------------------------------------
# HEALPix directions and main axis (Sect. 2.2)
# ---------------------------------------------------------------------------

def test_healpix_nside2_structure():
    d = oracle.healpix_nside2()
    assert d.shape == (48, 3)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    # 7 rings of 4, 8, 8, 8, 8, 8, 4 pixels
    zs, counts = np.unique(np.round(d[:, 2], 12), return_counts=True)
    assert list(counts) == [4, 8, 8, 8, 8, 8, 4]
    # equal-area pixels: the equatorial ring centres are equally spaced in z
    # (Lambert cylindrical property) by 2/(3 N_side) = 1/3
    assert np.allclose(np.diff(zs[1:-1]), 1.0 / 3.0, atol=1e-12)
    # the polar cap z > 2/3 holds exactly 8 pixel areas: area 2 pi (1 - 2/3)
    assert math.isclose(2 * math.pi * (1 - 2.0 / 3.0), 8 * 4 * math.pi / 48, rel_tol=1e-14)
    # antipodal symmetry and invariance under a quarter turn about z
    for v in d:
        assert np.min(np.linalg.norm(d + v, axis=1)) < 1e-12
        rot = np.array([-v[1], v[0], v[2]])
        assert np.min(np.linalg.norm(d - rot, axis=1)) < 1e-12
    assert np.allclose(d.sum(axis=0), 0.0, atol=1e-13)


def test_main_axis_tie_break():
    d = oracle.healpix_nside2()
    ax = np.array([oracle.main_axis(v) for v in d])
    absd = np.abs(d)
    for v, a in zip(absd, ax):
        assert v[a] >= v.max() * (1 - 1e-12)
    ties = [i for i, v in enumerate(absd) if abs(v[0] - v[1]) < 1e-12 and v[0] >= v.max() - 1e-12]
    assert len(ties) == 8
    assert all(ax[i] == 0 for i in ties)


# ---------------------------------------------------------------------------
# P8: path-length invariants
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N", [3, 5, 8])
def test_regular_grid_path_sum_per_cell(N):
    """Per direction, every cell is crossed by the same total length 1/|d_m|."""
    d = oracle.healpix_nside2()
    ps = oracle.path_sums_3d(N, d)
    for q in range(48):
        m = oracle.main_axis(d[q])
        assert np.allclose(ps[q], 1.0 / abs(d[q][m]), rtol=1e-12, atol=0)


def test_regular_walk_total_length_and_wraps():
    """Each ray crosses exactly N layers: total length N/|d_m|; restarts happen
    exactly where the transverse coordinate crosses a multiple of N."""
    N = 6
    for v in oracle.healpix_nside2():
        m = oracle.main_axis(v)
        axes = [a for a in range(3) if a != m]
        for i in range(N):
            for j in range(N):
                cells, ln, rs = oracle.walk_3d(N, v, i, j)
                assert math.isclose(ln.sum(), N / abs(v[m]), rel_tol=1e-12)
                # independent count of boundary crossings of the transverse axes
                T = N / abs(v[m])
                times = []
                for a, p0 in zip(axes, (i + 0.5, j + 0.5)):
                    if v[a] == 0:
                        continue
                    for k in range(-3, 5):
                        t = (k * N - p0) / v[a]
                        if 1e-9 < t < T - 1e-9:
                            times.append(t)
                # a corner crossed by both axes at once is one re-entry
                distinct = len(np.unique(np.round(np.array(times), 9)))
                assert rs.sum() - 1 == distinct


def test_1d_shell_volume_sampling():
    """W_k = sum_j a_j s_jk -> V_k as the number of rays grows (error ~ N^-1.5)."""
    R = np.array([1.0, 2.0, 3.5])
    V = 4.0 / 3.0 * np.pi * (R ** 3 - np.concatenate([[0.0], R[:-1]]) ** 3)
    errs = []
    for n in (1000, 10000):
        b = oracle.equidistant_impacts(R[-1], n)
        a = oracle.ray_areas_1d(R[-1], b)
        W = np.zeros(3)
        for bj, aj in zip(b, a):
            sh, s, mu = oracle.ray_steps_1d(R, bj)
            np.add.at(W, sh, aj * s)
        errs.append(np.max(np.abs(W / V - 1)))
    assert errs[1] < 3e-5
    assert errs[1] < errs[0] / 10.0


def test_1d_power_law_ray_weights():
    """Ray weights of any impact spacing tile the disc (sum = pi R^2, each one
    the annulus between the mid-points of its neighbours) and still sample
    the shell volumes: b_j = R ((j + 1/2)/N)^2."""
    R = np.array([1.0, 2.0, 3.5])
    V = 4.0 / 3.0 * np.pi * (R ** 3 - np.concatenate([[0.0], R[:-1]]) ** 3)
    n = 4000
    b = R[-1] * ((np.arange(n) + 0.5) / n) ** 2
    a = oracle.ray_areas_1d(R[-1], b)
    assert math.isclose(a.sum(), math.pi * R[-1] ** 2, rel_tol=1e-12)
    edges = np.concatenate([[0.0], 0.5 * (b[1:] + b[:-1]), [R[-1]]])
    assert np.allclose(a, np.pi * (edges[1:] ** 2 - edges[:-1] ** 2), rtol=1e-12, atol=0)
    W = np.zeros(3)
    for bj, aj in zip(b, a):
        sh, s, mu = oracle.ray_steps_1d(R, bj)
        np.add.at(W, sh, aj * s)
    assert np.max(np.abs(W / V - 1)) < 2e-3


def test_1d_ray_steps_geometry():
    """Chord pieces add up to 2 sqrt(R^2 - b^2); cosines at step starts."""
    R = np.array([1.0, 2.0, 4.0])
    for b in (0.3, 1.5, 3.9):
        sh, s, mu = oracle.ray_steps_1d(R, b)
        assert math.isclose(s.sum(), 2 * math.sqrt(R[-1] ** 2 - b ** 2), rel_tol=1e-14)
        kmin = int(np.argmax(R > b))
        assert list(sh) == list(range(2, kmin, -1)) + [kmin, kmin] + list(range(kmin + 1, 3))
        # first step starts on the outer surface moving inwards
        assert math.isclose(mu[0], -math.sqrt(1 - (b / R[-1]) ** 2), rel_tol=1e-14)
        # the second tangent half starts at the tangent point, perpendicular
        nin = len(sh) // 2
        assert mu[nin] == 0.0
        assert np.all(mu[:nin] < 0) and np.all(mu[nin + 1:] > 0)


# ---------------------------------------------------------------------------
# P1: homogeneous medium closed form
# ---------------------------------------------------------------------------

def _uniform_kappa_eta(ncell, kappa, eta):
    return np.full(ncell, kappa), np.full(ncell, eta)


def test_p1_homogeneous_sphere_closed_form():
    spec = _spec(48, 1.5)
    nsh, Rtot = 7, 3.0e17
    R = Rtot * (np.arange(nsh) + 1.0) / nsh
    b = np.full(nsh, 0.25 * KMS)
    kap, eta = _uniform_kappa_eta(nsh, 4.0e-13, 3.0e-27)
    impact = np.array([0.1, 0.37, 0.8, 0.99]) * Rtot
    area = np.ones(4)
    I_bg = 1.7e-15
    res = oracle.march_1d(R, np.zeros(nsh), b, kap, eta, impact, area, spec, I_bg, want_I=True)
    v = spec.v_min + (np.arange(spec.n_channels) + 0.5) * spec.dv
    p = np.exp(-(v / b[0]) ** 2) / (b[0] * math.sqrt(math.pi))
    S = eta[0] / kap[0]
    for j, bj in enumerate(impact):
        tau = kap[0] * p * 2 * math.sqrt(Rtot ** 2 - bj ** 2)
        expect = S * (1 - np.exp(-tau)) + I_bg * np.exp(-tau)
        assert np.allclose(res.I_out[j], expect, rtol=1e-12, atol=0)
    assert np.max(kap[0] * p * 2 * Rtot) > 3.0   # optically thick at line centre


def test_p1_homogeneous_cube_closed_form():
    """3D: the intensity leaving a uniform static cube is the slab solution over
    the path since the ray's last (re)entry."""
    N, delta = 5, 1.0e16
    spec = _spec(32, 1.5)
    nc = N ** 3
    b = 0.2 * KMS
    kap, eta = 4.0e-13, 2.0e-27
    dirs = oracle.healpix_nside2()[[0, 5, 13, 20]]
    I_bg = 2.0e-15
    res = oracle.march_3d(N, delta, np.zeros(nc), np.zeros(nc), np.zeros(nc), np.full(nc, b),
                          np.full(nc, kap), np.full(nc, eta), dirs, spec, I_bg, want_I=True)
    v = spec.v_min + (np.arange(spec.n_channels) + 0.5) * spec.dv
    p = np.exp(-(v / b) ** 2) / (b * math.sqrt(math.pi))
    S = eta / kap
    for q, d in enumerate(dirs):
        m = int(np.argmax(np.abs(d)))
        axes = [a for a in range(3) if a != m]
        T = N / abs(d[m])
        for j in range(N):
            for i in range(N):
                # last transverse boundary crossing along the ray (cell units)
                t_last = 0.0
                for a, p0 in zip(axes, (i + 0.5, j + 0.5)):
                    if d[a] == 0:
                        continue
                    for k in range(-3, 5):
                        t = (k * N - p0) / d[a]
                        if 0 < t < T:
                            t_last = max(t_last, t)
                L = (T - t_last) * delta
                tau = kap * p * L
                expect = S * (1 - np.exp(-tau)) + I_bg * np.exp(-tau)
                assert np.allclose(res.I_out[q, j * N + i], expect, rtol=1e-12, atol=0)


# ---------------------------------------------------------------------------
# P2: uniform field invariance (S = I_bg everywhere)
# ---------------------------------------------------------------------------

def _pops_with_source(mol, T):
    """Two-level populations whose source function is B_nu(T)."""
    x = oracle.lte_populations(mol, np.array([T]))
    return x[0]


def test_p2_uniform_field_1d_with_velocity():
    mol = _thin_two_level()
    spec = _spec(96, 3.0)
    model = synth.cloud_1d_plummer(n_shells=30, r_out_pc=0.2, infall_kms=0.1,
                                   abundance=1e-6, b_turb_kms=0.2)
    T_bg = 2.73
    x = np.tile(_pops_with_source(mol, T_bg), (30, 1))
    prob = oracle._Problem(mol, model.n_H2, model.T_kin, model.b_turb, model.abundance, spec, T_bg)
    kap, eta = oracle.prepare(mol, x, prob.n_mol)
    I_bg = float(prob.I_bg[0])
    assert np.allclose(eta[0] / kap[0], I_bg, rtol=1e-13)
    R = model.r_out
    imp = oracle.equidistant_impacts(R[-1], 40)
    area = oracle.ray_areas_1d(R[-1], imp)
    res = oracle.march_1d(R, model.v_r, prob.bD, kap[0], eta[0], imp, area, spec, I_bg, want_I=True)
    assert np.allclose(res.I_out, I_bg, rtol=1e-13, atol=0)
    JLI = res.Jraw + (eta[0] / kap[0]) * res.Lraw
    assert np.allclose(JLI, I_bg * res.E, rtol=1e-12)
    assert np.max(res.Lraw / res.W) > 1e-2   # the medium is not transparent


def test_p2_uniform_field_3d_with_velocity():
    mol = _thin_two_level()
    spec = _spec(64, 4.0)
    N = 6
    cube = synth.turbulent_cube(N=N, box_pc=0.1, seed=11, abundance=1e-6, T_kin=10.0,
                                b_turb_kms=0.2)
    T_bg = 2.73
    x = np.tile(_pops_with_source(mol, T_bg), (N ** 3, 1))
    prob = oracle._Problem(mol, cube.n_H2, cube.T_kin, cube.b_turb, cube.abundance, spec, T_bg)
    kap, eta = oracle.prepare(mol, x, prob.n_mol)
    I_bg = float(prob.I_bg[0])
    res = oracle.march_3d(N, cube.root_cell_cm, cube.vx.astype(float), cube.vy.astype(float),
                          cube.vz.astype(float), prob.bD, kap[0], eta[0],
                          oracle.healpix_nside2(), spec, I_bg, want_I=True)
    assert np.allclose(res.I_out, I_bg, rtol=1e-13, atol=0)
    JLI = res.Jraw + (eta[0] / kap[0]) * res.Lraw
    assert np.allclose(JLI, I_bg * res.E, rtol=1e-12)


# ---------------------------------------------------------------------------
# P6: photon conservation (emitted + entering = absorbed + escaping)
# ---------------------------------------------------------------------------

def test_p6_conservation_1d():
    mol = synth.rotor_molecule(5)
    w = synth.workload_1d_plummer(n_shells=40, abundance=1e-7)
    spec = _spec(128, 4.0)
    m = w.model
    prob = oracle._Problem(mol, m.n_H2, m.T_kin, m.b_turb, m.abundance, spec, 2.73)
    x = oracle.lte_populations(mol, m.T_kin * 0.7)
    kap, eta = oracle.prepare(mol, x, prob.n_mol)
    imp = oracle.equidistant_impacts(m.r_out[-1], 50)
    area = oracle.ray_areas_1d(m.r_out[-1], imp)
    for t in range(mol.n_trans):
        r = oracle.march_1d(m.r_out, m.v_r, prob.bD, kap[t], eta[t], imp, area, spec,
                            prob.I_bg[t])
        lhs = r.cons + np.sum(eta[t] * r.E)
        rhs = np.sum(kap[t] * r.Jraw + eta[t] * r.Lraw)
        assert math.isclose(lhs, rhs, rel_tol=1e-11), (t, lhs, rhs)


def test_p6_conservation_3d():
    mol = synth.rotor_molecule(4)
    spec = _spec(64, 4.0)
    N = 5
    cube = synth.turbulent_cube(N=N, box_pc=0.05, seed=21, abundance=1e-5, T_kin=12.0,
                                b_turb_kms=0.15)
    prob = oracle._Problem(mol, cube.n_H2, cube.T_kin, cube.b_turb, cube.abundance, spec, 2.73)
    x = oracle.lte_populations(mol, np.full(N ** 3, 8.0))
    kap, eta = oracle.prepare(mol, x, prob.n_mol)
    for t in range(mol.n_trans):
        r = oracle.march_3d(N, cube.root_cell_cm, cube.vx.astype(float), cube.vy.astype(float),
                            cube.vz.astype(float), prob.bD, kap[t], eta[t],
                            oracle.healpix_nside2(), spec, prob.I_bg[t])
        lhs = r.cons + np.sum(eta[t] * r.E)
        rhs = np.sum(kap[t] * r.Jraw + eta[t] * r.Lraw)
        assert math.isclose(lhs, rhs, rel_tol=1e-11), (t, lhs, rhs)
        assert np.max(r.Lraw / r.W) > 1e-3


# ---------------------------------------------------------------------------
# R5: channel sampling of the profile
# ---------------------------------------------------------------------------

def test_channel_fractions_sum_to_one():
    """sum_c f_c = 1 to rounding when b/dv >= 1.5 and the band covers the line."""
    mol = _thin_two_level()
    m = synth.cloud_1d_log(n_shells=12)
    spec = synth.Spectral.symmetric(128, 2.0)
    prob = oracle._Problem(mol, m.n_H2, m.T_kin, m.b_turb, m.abundance, spec, 2.73)
    imp = oracle.equidistant_impacts(m.r_out[-1], 20)
    r = oracle.march_1d(m.r_out, m.v_r, prob.bD, np.zeros(12), np.zeros(12), imp,
                        oracle.ray_areas_1d(m.r_out[-1], imp), spec, 1.0)
    assert np.allclose(r.E / r.W, 1.0, atol=1e-13)


# ---------------------------------------------------------------------------
# P11: escape probability of a uniform sphere
# ---------------------------------------------------------------------------

def beta_half_chord(tau):
    """Volume- and channel-free mean of (1 - e^-t)/t over the two half chords of
    a uniform sphere of radial optical depth tau crossed by parallel rays:
    (3/(2 tau)) [1 - 2/tau^2 + (2/tau + 2/tau^2) e^-tau]."""
    tau = np.asarray(tau, dtype=np.float64)
    out = np.empty_like(tau)
    big = tau > 0.5
    t = tau[big]
    out[big] = 1.5 / t * (1 - 2 / t ** 2 + (2 / t + 2 / t ** 2) * np.exp(-t))
    # power series of the same expression, 1.5 sum_{k>=1} c_k tau^(k-1) with
    # c_k = -2 (-1)^k (k+1)/(k+2)!  (= 1 - 3 tau/8 + tau^2/10 - ...)
    t = tau[~big]
    acc = np.zeros_like(t)
    for k in range(18, 0, -1):
        ck = -2.0 * (-1) ** k * (k + 1) / math.factorial(k + 2)
        acc = acc * t + ck
    out[~big] = 1.5 * acc
    return out


def test_p11_uniform_sphere_escape_probability():
    spec = _spec(40, 1.2)
    Rs = 1.0e17
    b = 0.2 * KMS
    kap = 5.0e-12
    n = 10000
    imp = oracle.equidistant_impacts(Rs, n)
    area = oracle.ray_areas_1d(Rs, imp)
    r = oracle.march_1d(np.array([Rs]), np.zeros(1), np.array([b]), np.array([kap]),
                        np.array([1e-27]), imp, area, spec, 0.0)
    v = spec.v_min + (np.arange(spec.n_channels) + 0.5) * spec.dv
    p = np.exp(-(v / b) ** 2) / (b * math.sqrt(math.pi))
    f = p * spec.dv
    tau = kap * p * Rs
    assert tau.max() > 10
    expect = np.sum(f * beta_half_chord(tau))
    got = 1.0 - r.Lraw[0] / r.W[0]
    assert math.isclose(got, expect, rel_tol=2e-5), (got, expect)
    # the full-chord (one step) textbook value would be visibly different
    full = np.sum(f * 0.75 / tau * (1 - 1 / (2 * tau ** 2) + (1 / tau + 1 / (2 * tau ** 2)) * np.exp(-2 * tau)))
    assert abs(full - expect) > 1e-2 * expect


# ---------------------------------------------------------------------------
# P12: brute force on tiny inputs
# ---------------------------------------------------------------------------

def test_p12_one_shell_one_ray_by_hand():
    spec = synth.Spectral(3, -1.5e4, 1.0e4)
    R, bimp, b = 2.0e16, 1.2e16, 1.0e4
    kap, eta, vr, I_bg = 3.0e-12, 4.0e-26, 0.0, 1.0e-14
    r = oracle.march_1d(np.array([R]), np.array([vr]), np.array([b]), np.array([kap]),
                        np.array([eta]), np.array([bimp]), np.array([2.0]), spec, I_bg,
                        want_I=True)
    z = math.sqrt(R * R - bimp * bimp)
    I = np.full(3, I_bg)
    J = Lm = E = 0.0
    for _half in range(2):
        for c in range(3):
            vc = -1.5e4 + (c + 0.5) * 1.0e4
            p = math.exp(-(vc / b) ** 2) / (b * math.sqrt(math.pi))
            tau = kap * p * z
            bet = (1 - math.exp(-tau)) / tau
            J += 2.0 * z * p * 1.0e4 * I[c] * bet
            Lm += 2.0 * z * p * 1.0e4 * (1 - bet)
            E += 2.0 * z * p * 1.0e4
            I[c] = I[c] * math.exp(-tau) + (eta / kap) * (1 - math.exp(-tau))
    assert np.allclose(r.I_out[0], I, rtol=1e-13)
    assert math.isclose(r.Jraw[0], J, rel_tol=1e-13)
    assert math.isclose(r.Lraw[0], Lm, rel_tol=1e-12)
    assert math.isclose(r.E[0], E, rel_tol=1e-13)
    assert math.isclose(r.W[0], 2.0 * 2 * z, rel_tol=1e-14)


def test_p12_two_cubed_axis_direction_by_hand():
    """2^3 grid, one direction +z: four rays, each through two cells."""
    N, delta = 2, 1.0e16
    spec = synth.Spectral(4, -2.0e4, 1.0e4)
    rng = np.random.default_rng(5)
    kap = rng.uniform(1e-13, 1e-12, 8)
    eta = rng.uniform(1e-27, 1e-26, 8)
    vz = rng.uniform(-1e4, 1e4, 8)
    b = rng.uniform(0.8e4, 1.5e4, 8)
    zeros = np.zeros(8)
    I_bg = 3.0e-15
    r = oracle.march_3d(N, delta, zeros, zeros, vz, b, kap, eta, np.array([[0.0, 0.0, 1.0]]),
                        spec, I_bg, want_I=True)
    J = np.zeros(8)
    Lm = np.zeros(8)
    a = delta * delta
    for y in range(2):
        for x in range(2):
            I = np.full(4, I_bg)
            for z in range(2):
                k = (z * 2 + y) * 2 + x
                for c in range(4):
                    vc = -2.0e4 + (c + 0.5) * 1.0e4
                    p = math.exp(-((vc + vz[k]) / b[k]) ** 2) / (b[k] * math.sqrt(math.pi))
                    tau = kap[k] * p * delta
                    bet = (1 - math.exp(-tau)) / tau
                    J[k] += a * delta * p * 1.0e4 * I[c] * bet
                    Lm[k] += a * delta * p * 1.0e4 * (1 - bet)
                    I[c] = I[c] * math.exp(-tau) + eta[k] * p * delta * bet
            assert np.allclose(r.I_out[0, y * 2 + x], I, rtol=1e-13)
    assert np.allclose(r.Jraw, J, rtol=1e-13)
    assert np.allclose(r.Lraw, Lm, rtol=1e-11)
    assert np.allclose(r.W, a * delta, rtol=1e-14)


# ---------------------------------------------------------------------------
# Statistical equilibrium: P3, P4, P5, P7 and the balance residual
# ---------------------------------------------------------------------------

def test_se_balance_residual_and_normalisation():
    mol = synth.rotor_molecule(10)
    rng = np.random.default_rng(3)
    nc = 50
    n = 10 ** rng.uniform(1, 7, nc)
    T = rng.uniform(5, 30, nc)
    J = 10 ** rng.uniform(-16, -12, (mol.n_trans, nc))
    Lam = rng.uniform(0, 0.9, (mol.n_trans, nc))
    R = oracle.rate_matrix(mol, n, T, J, Lam, True)
    x = oracle.se_solve(R, oracle.lte_populations(mol, T))
    assert np.allclose(x.sum(axis=1), 1.0, atol=1e-14)
    assert np.all(x > -1e-18)
    inflow = np.einsum("kj,kji->ki", x, R)
    outflow = x * R.sum(axis=2)
    scale = np.maximum(inflow, outflow).max(axis=1, keepdims=True)
    assert np.max(np.abs(inflow - outflow) / scale) < 1e-12


def test_p3_optically_thin_two_level_closed_form():
    mol = _thin_two_level()
    m = synth.cloud_1d_log(n_shells=20, abundance=1e-20)
    spec = synth.Spectral.symmetric(128, 2.0)
    run = oracle.run_1d(mol, m, spec, 2.73, 1)
    h = run.history[0]
    I_bg = float(oracle.planck(mol.nu[0], 2.73))
    assert np.allclose(h["J"][0], I_bg, rtol=1e-10)
    assert np.max(np.abs(h["Lam"][0])) < 1e-9
    Bul, Blu = oracle.einstein_B(mol)
    Cul = m.n_H2 * 2e-11
    Clu = Cul * 3.0 * np.exp(-mol.E_K[1] / m.T_kin)
    ratio = (Clu + Blu[0] * I_bg) / (mol.A[0] + Cul + Bul[0] * I_bg)
    got = run.x[:, 1] / run.x[:, 0]
    assert np.allclose(got, ratio, rtol=1e-9)


def test_p4_lte_limit_high_density():
    mol = synth.rotor_molecule(10)
    m = synth.cloud_1d_plummer(n_shells=6, n0=1e14, r_flat_pc=10.0, abundance=1e-12,
                               infall_kms=0.0)
    spec = synth.Spectral.symmetric(128, 2.0)
    run = oracle.run_1d(mol, m, spec, 2.73, 2)
    lte = oracle.lte_populations(mol, m.T_kin)
    big = lte > 1e-10
    assert np.max(np.abs(run.x[big] / lte[big] - 1)) < 1e-6


# ---------------------------------------------------------------------------
# Absolute scales: the Doppler width and the opacity / emissivity of
# ``prepare`` (Sect. 2, Eqs. (1)-(3)), and the convergence measure (Sect. 2:
# iterate until the populations stop changing)
# ---------------------------------------------------------------------------

# Textbook constants typed here, not taken from the oracle: CODATA-2018 exact
# k_B, h, c and the 2018 atomic mass constant.
K_B_CGS = 1.380649e-16
H_CGS = 6.62607015e-27
C_CGS = 2.99792458e10
AMU_G = 1.66053906660e-24


def _thin_sphere(T, b_turb, abundance, n_H2=1.0e3, radius_pc=0.01, n_shells=4, n_rays=4):
    return synth.uniform_sphere_1d(n_shells=n_shells, radius_cm=radius_pc * synth.PC_CM,
                                   n_H2=n_H2, T_kin=T, b_turb=b_turb, abundance=abundance,
                                   n_rays=n_rays)


@pytest.mark.parametrize("T,b_turb_kms", [(10.0, 0.0), (40.0, 0.15)])
def test_doppler_width_from_thin_line_moments(T, b_turb_kms):
    """An optically thin, static, uniform sphere with no background emits the
    profile itself: the velocity variance of the emergent line is the 1D
    Maxwell variance k T / m plus the turbulent part b_turb^2 / 2 (a Gaussian
    exp(-v^2/b^2) has variance b^2/2).  Pins the thermal width: a k T / m for
    2 k T / m, a wrong atomic mass unit or a turbulent term added linearly
    each change the variance at O(1)."""
    mol = _thin_two_level()
    m = _thin_sphere(T, b_turb_kms * KMS, abundance=1e-17)
    var_ref = K_B_CGS * T / (mol.mass_amu * AMU_G) + 0.5 * (b_turb_kms * KMS) ** 2
    half = 10.0 * math.sqrt(2.0 * var_ref) / KMS          # +-10 Doppler widths
    spec = synth.Spectral.symmetric(1024, half)           # ~50 channels per width
    x = oracle.lte_populations(mol, m.T_kin)
    sp = oracle.spectra_1d(mol, m, spec, 0.0, x, 0)
    v = spec.v_min + (np.arange(spec.n_channels) + 0.5) * spec.dv
    for row in sp:
        assert row.min() >= 0.0 and row.max() > 0.0
        mean = float(np.sum(v * row) / np.sum(row))
        var = float(np.sum((v - mean) ** 2 * row) / np.sum(row))
        assert abs(mean) < 1e-9 * math.sqrt(var_ref)
        assert var == pytest.approx(var_ref, rel=1e-9)


def test_absolute_emissivity_thin_column():
    """Optically thin line without a background: the integrated line
    temperature W = sum_c T_R dv (T_R = c^2 dI / (2 k nu^2)) and the column of
    upper-level molecules along the line of sight obey the radio relation
    N_u = 8 pi k nu^2 W / (h c^3 A_ul).  The column is counted here from the
    model (n_mol = X n_H2, the ray's chord through the uniform sphere), so the
    absolute scale of the emissivity (h c / 4 pi) A n_mol x_u is pinned, not
    only its ratio to the opacity."""
    mol = _thin_two_level()
    X = 3.0e-17
    m = _thin_sphere(15.0, 0.1 * KMS, abundance=X, n_shells=3, n_rays=5)
    spec = synth.Spectral.symmetric(512, 1.5)
    x = oracle.lte_populations(mol, m.T_kin)
    sp = oracle.spectra_1d(mol, m, spec, 0.0, x, 0)
    nu, A = float(mol.nu[0]), float(mol.A[0])
    R = float(m.r_out[-1])
    b = (np.arange(m.n_rays) + 0.5) * R / m.n_rays
    chord = 2.0 * np.sqrt(R ** 2 - b ** 2)
    N_u = m.n_H2[0] * X * x[0, 1] * chord
    W = np.sum(C_CGS ** 2 * sp / (2.0 * K_B_CGS * nu ** 2), axis=1) * spec.dv
    N_u_radio = 8.0 * math.pi * K_B_CGS * nu ** 2 * W / (H_CGS * C_CGS ** 3 * A)
    assert np.allclose(N_u_radio, N_u, rtol=1e-8)


def test_absolute_opacity_ground_state_absorption():
    """All molecules in the lower level (no emission): the sphere only
    absorbs the background, dI = I_bg (e^-tau - 1), and the velocity-integrated
    optical depth of the line equals the textbook
    sum_c tau_c dv = (c^3 / (8 pi nu^3)) A_ul (g_u/g_l) N_l with N_l = X n_H2
    times the chord.  The Doppler width drops out of the integral, so this pins
    the absolute opacity scale independently of the width."""
    mol = _thin_two_level()
    X = 2.0e-6
    m = _thin_sphere(12.0, 0.12 * KMS, abundance=X, n_shells=3, n_rays=5)
    spec = synth.Spectral.symmetric(400, 2.0)
    x = np.zeros((m.n_shells, 2))
    x[:, 0] = 1.0
    T_bg = 8.0
    sp = oracle.spectra_1d(mol, m, spec, T_bg, x, 0)
    I_bg = 2.0 * H_CGS * mol.nu[0] ** 3 / C_CGS ** 2 / math.expm1(H_CGS * mol.nu[0] / (K_B_CGS * T_bg))
    tau = -np.log1p(sp / I_bg)
    nu, A = float(mol.nu[0]), float(mol.A[0])
    g_ratio = float(mol.g[1] / mol.g[0])
    R = float(m.r_out[-1])
    b = (np.arange(m.n_rays) + 0.5) * R / m.n_rays
    N_l = m.n_H2[0] * X * 2.0 * np.sqrt(R ** 2 - b ** 2)
    ref = C_CGS ** 3 / (8.0 * math.pi * nu ** 3) * A * g_ratio * N_l
    got = np.sum(tau, axis=1) * spec.dv
    assert tau.max() > 0.3          # a real absorption line, not the thin limit
    assert np.allclose(got, ref, rtol=1e-9)


def test_max_rel_change_worked_example():
    """The convergence measure on populations worked out by hand: relative to
    the new value, entries below 1e-10 ignored, zero when nothing is left."""
    x_old = np.array([[0.5, 0.5], [0.8, 0.2], [1.0 - 5e-11, 5e-11], [1.0 - 1e-10, 1e-10]])
    x_new = np.array([[0.4, 0.6], [0.8, 0.2], [1.0 - 9e-11, 9e-11], [1.0 - 2e-10, 2e-10]])
    # rows: 0.1/0.4 = 0.25 and 0.1/0.6; 0; 4e-11/(1-9e-11) (9e-11 is below the
    # floor); 1e-10/(1-2e-10) and 1e-10/2e-10 = 0.5 (2e-10 is above it)
    assert oracle.max_rel_change(x_new, x_old) == pytest.approx(0.5, rel=1e-6)
    assert oracle.max_rel_change(x_new[:3], x_old[:3]) == pytest.approx(0.25, rel=1e-12)
    assert oracle.max_rel_change(x_new[1:3], x_old[1:3]) == pytest.approx(4e-11, rel=1e-6)
    tiny = np.array([[5e-11, 6e-11]])
    assert oracle.max_rel_change(tiny, 2 * tiny) == 0.0


@pytest.mark.parametrize("abund", [1e-9, 1e-6])
def test_p5_detailed_balance_fixed_point(abund):
    """T_bg = T_kin everywhere: Boltzmann populations are the exact fixed point
    at any density and optical depth, and are reached from another start."""
    mol = synth.rotor_molecule(5)
    T = 12.0
    m = synth.cloud_1d_plummer(n_shells=15, r_out_pc=0.1, T_in=T, T_out=T, n0=1e5,
                               infall_kms=0.05, abundance=abund)
    spec = synth.Spectral.symmetric(128, 2.5)
    lte = oracle.lte_populations(mol, m.T_kin)
    run = oracle.run_1d(mol, m, spec, T, 1)
    assert np.allclose(run.x, lte, rtol=1e-10, atol=1e-16)
    x0 = oracle.lte_populations(mol, m.T_kin * 0.5)
    run2 = oracle.run_1d(mol, m, spec, T, 200, x0=x0, tol=1e-12)
    assert np.allclose(run2.x, lte, rtol=1e-8, atol=1e-16)


def test_p7_ali_and_li_share_the_fixed_point():
    mol = synth.rotor_molecule(4)
    m = synth.cloud_1d_plummer(n_shells=12, r_out_pc=0.1, n0=1e5, abundance=2e-6,
                               infall_kms=0.05)
    spec = synth.Spectral.symmetric(96, 3.0)
    ali = oracle.run_1d(mol, m, spec, 2.73, 400, use_ali=True, tol=1e-13, record=False)
    li = oracle.run_1d(mol, m, spec, 2.73, 4000, use_ali=False, tol=1e-13, record=False)
    assert ali.iters < li.iters          # ALI converges faster in thick gas
    big = li.x > 1e-10
    assert np.max(np.abs(ali.x[big] / li.x[big] - 1)) < 1e-9
    # and the model is optically thick (otherwise the test says nothing)
    prob = oracle._Problem(mol, m.n_H2, m.T_kin, m.b_turb, m.abundance, spec, 2.73)
    kap, _ = oracle.prepare(mol, li.x, prob.n_mol)
    dr = np.diff(np.concatenate([[0], m.r_out]))
    tau_c = np.max(np.sum(kap * dr / (prob.bD * math.sqrt(math.pi)), axis=1))
    assert tau_c > 5


# ---------------------------------------------------------------------------
# P10: symmetry
# ---------------------------------------------------------------------------

def test_p10_static_spectra_symmetric():
    mol = synth.rotor_molecule(4)
    m = synth.cloud_1d_plummer(n_shells=20, r_out_pc=0.1, infall_kms=0.0, abundance=1e-7)
    m.v_r[:] = 0.0
    spec = synth.Spectral.symmetric(64, 2.0)
    run = oracle.run_1d(mol, m, spec, 2.73, 3)
    sp = oracle.spectra_1d(mol, m, spec, 2.73, run.x, 0)
    assert np.allclose(sp, sp[:, ::-1], rtol=1e-12, atol=1e-30)
    assert sp.max() > 0


def test_p10_infall_gives_blue_asymmetry():
    """Infall with an optically thick line: the centre spectrum's blue peak
    is the stronger one (radio convention)."""
    mol = synth.rotor_molecule(4)
    m = synth.cloud_1d_plummer(n_shells=40, r_out_pc=0.1, infall_kms=0.1, abundance=1e-7,
                               n0=1e6, T_in=20.0, T_out=8.0)
    spec = synth.Spectral.symmetric(128, 2.0)
    run = oracle.run_1d(mol, m, spec, 2.73, 10)
    sp = oracle.spectra_1d(mol, m, spec, 2.73, run.x, 0, impact=np.array([1e-4 * m.r_out[-1]]))
    half = spec.n_channels // 2
    assert sp[0, :half].max() > sp[0, half:].max()


# ---------------------------------------------------------------------------
# Hyperfine multiplets with LTE between the components (Sect. 1)
# ---------------------------------------------------------------------------

HF_V = np.array([-0.62, 0.0, 0.37]) * KMS      # asymmetric, so a sign error shows
HF_W = np.array([1.0, 5.0, 3.0])


def _hf_profile(v, b):
    """sum_k (w_k / sum w) exp(-((v - v_k)/b)^2) / (b sqrt(pi)) written out."""
    p = np.zeros_like(v)
    for vk, wk in zip(HF_V, HF_W / HF_W.sum()):
        p += wk * np.exp(-((v - vk) / b) ** 2)
    return p / (b * math.sqrt(math.pi))


def test_hf_homogeneous_sphere_closed_form():
    """Uniform static sphere, three components: the emergent spectrum is the
    slab solution with tau_c = kappa L sum_k w_k p_k(c)."""
    spec = _spec(96, 1.5)
    nsh, Rtot = 6, 3.0e17
    R = Rtot * (np.arange(nsh) + 1.0) / nsh
    b = np.full(nsh, 0.12 * KMS)
    kap, eta = _uniform_kappa_eta(nsh, 5.0e-13, 3.0e-27)
    impact = np.array([0.05, 0.5, 0.93]) * Rtot
    I_bg = 1.1e-15
    res = oracle.march_1d(R, np.zeros(nsh), b, kap, eta, impact, np.ones(3), spec, I_bg,
                          want_I=True, shape=(HF_V, HF_W))
    v = spec.v_min + (np.arange(spec.n_channels) + 0.5) * spec.dv
    p = _hf_profile(v, b[0])
    S = eta[0] / kap[0]
    for j, bj in enumerate(impact):
        tau = kap[0] * p * 2 * math.sqrt(Rtot ** 2 - bj ** 2)
        expect = S * (1 - np.exp(-tau)) + I_bg * np.exp(-tau)
        assert np.allclose(res.I_out[j], expect, rtol=1e-12, atol=0)
    # the three components are resolved: the spectrum has three local maxima
    sp = res.I_out[0] - I_bg
    peaks = np.flatnonzero((sp[1:-1] > sp[:-2]) & (sp[1:-1] > sp[2:]))
    assert len(peaks) == 3


def test_hf_moving_cube_closed_form():
    """Uniform cube moving at u along +z, line of sight +z: the components
    appear at channel velocity v_k - u (the sign convention of the shift)."""
    N, delta = 4, 1.0e16
    spec = _spec(96, 1.5)
    nc = N ** 3
    b, u = 0.1 * KMS, 0.21 * KMS
    kap, eta = 3.0e-13, 2.0e-27
    I_bg = 2.0e-15
    res = oracle.march_3d(N, delta, np.zeros(nc), np.zeros(nc), np.full(nc, u), np.full(nc, b),
                          np.full(nc, kap), np.full(nc, eta), np.array([[0.0, 0.0, 1.0]]), spec,
                          I_bg, want_I=True, shape=(HF_V, HF_W))
    v = spec.v_min + (np.arange(spec.n_channels) + 0.5) * spec.dv
    tau = kap * _hf_profile(v + u, b) * N * delta
    expect = eta / kap * (1 - np.exp(-tau)) + I_bg * np.exp(-tau)
    for r in range(N * N):
        assert np.allclose(res.I_out[0, r], expect, rtol=1e-12, atol=0)


def test_hf_single_and_split_components():
    """One component of any strength at offset 0 is the plain Gaussian; one
    component at offset v0 is the plain line of gas moving at -v0 along the
    line of sight; a component split into two at the same offset is unchanged."""
    N, delta = 3, 2.0e16
    spec = _spec(64, 1.5)
    nc = N ** 3
    rng = np.random.default_rng(7)
    b = rng.uniform(0.1, 0.2, nc) * KMS
    kap = rng.uniform(1e-13, 6e-13, nc)
    eta = kap * rng.uniform(1e-15, 3e-15, nc)
    uz = rng.uniform(-0.2, 0.2, nc) * KMS
    z = np.zeros(nc)
    d = np.array([[0.0, 0.0, 1.0]])
    args = (N, delta, z, z, uz, b, kap, eta, d, spec, 1.5e-15)
    plain = oracle.march_3d(*args, want_I=True)
    one = oracle.march_3d(*args, want_I=True, shape=([0.0], [2.5]))
    for f in ("Jraw", "Lraw", "W", "E", "I_out"):
        assert np.allclose(getattr(plain, f), getattr(one, f), rtol=1e-14, atol=0)
    v0 = 0.07 * KMS
    shifted = oracle.march_3d(*args, want_I=True, shape=([v0], [1.0]))
    moved = oracle.march_3d(N, delta, z, z, uz - v0, b, kap, eta, d, spec, 1.5e-15, want_I=True)
    assert np.allclose(shifted.I_out, moved.I_out, rtol=1e-12, atol=0)
    assert np.allclose(shifted.Jraw, moved.Jraw, rtol=1e-12, atol=0)
    split = oracle.march_3d(*args, want_I=True, shape=([v0, v0], [0.25, 0.75]))
    assert np.allclose(split.I_out, shifted.I_out, rtol=1e-13, atol=0)
    assert np.allclose(split.Lraw, shifted.Lraw, rtol=1e-13, atol=0)


def test_hf_channel_fractions_sum_to_one():
    """The multiplet's channel fractions still sum to one (sum_k w_k = 1 after
    normalisation) when the band covers every component."""
    mol = _thin_two_level()
    m = synth.cloud_1d_log(n_shells=12)
    spec = synth.Spectral.symmetric(256, 2.0)
    prob = oracle._Problem(mol, m.n_H2, m.T_kin, m.b_turb, m.abundance, spec, 2.73)
    imp = oracle.equidistant_impacts(m.r_out[-1], 20)
    r = oracle.march_1d(m.r_out, m.v_r, prob.bD, np.zeros(12), np.zeros(12), imp,
                        oracle.ray_areas_1d(m.r_out[-1], imp), spec, 1.0, shape=(HF_V, HF_W))
    assert np.allclose(r.E / r.W, 1.0, atol=1e-12)
