"""FP64 CPU oracle of the LOC accelerated-lambda-iteration ray march.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The HIP library
never calls it and shares no code, table or constant with it.

The heavy loops (ray geometry and the per-channel radiative update) live in
``loc_oracle.c`` (plain C, FP64, all channels, no windowing); this module
adds the per-cell algebra in numpy:

* ``prepare``: opacity and emissivity coefficients of each transition from
  the level populations (Sect. 2, Eqs. (2)-(3) in intensity form);
* ``se_solve``: the statistical-equilibrium equations with the absorbed
  counts in place of B_lu I (Sect. 2), ALI form with A_ul scaled by the
  escape probability (Sect. 2, diagonal operator), solved by LAPACK;
* ``run_1d`` / ``run_3d``: Lambda iteration starting from LTE at T_kin
  (Sect. 3.3.2), all transitions marched from the same populations, then
  all cells solved.

Readings of points the paper leaves open are listed in the design notes;
each function names the one it follows.  Every function is pinned by tests
against closed forms, limits and invariants (tests/test_oracle_*.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "loc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# Physical constants, CGS (CODATA-2018 exact h, k_B, c); the oracle's own copy.
H = 6.62607015e-27
KB = 1.380649e-16
C = 2.99792458e10
AMU = 1.66053906660e-24
SQRT_PI = np.sqrt(np.pi)


def build(force: bool = True) -> str:
    """Compile loc_oracle.c into liboracle.so with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        L.orc1d_ray_steps.restype = ctypes.c_int
        L.orc1d_ray_steps.argtypes = [ctypes.c_int, dp, ctypes.c_double, ip, dp, dp]
        L.orc1d_march.restype = None
        L.orc1d_march.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_int, dp, dp,
                                  ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, dp, dp, dp, dp, dp, dp,
                                  ctypes.c_int, dp, dp]
        L.orc1d_core_entry.restype = None
        L.orc1d_core_entry.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_int, dp, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc1d_march_core.restype = None
        L.orc1d_march_core.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_int, dp, dp, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.orc3d_main_axis.restype = ctypes.c_int
        L.orc3d_main_axis.argtypes = [dp]
        L.orc3d_walk.restype = ctypes.c_int
        L.orc3d_walk.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ip, dp, ctypes.POINTER(ctypes.c_ubyte), ctypes.c_int]
        L.orc3d_path_sums.restype = None
        L.orc3d_path_sums.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc3d_march.restype = None
        L.orc3d_march.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp, dp, dp, dp,
                                  ctypes.c_int, dp, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                  dp, dp, dp, dp, dp, dp, ctypes.c_int, dp, dp]
        llp = ctypes.POINTER(ctypes.c_longlong)
        L.orcoct_march.restype = None
        L.orcoct_march.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, ip, ctypes.c_double,
                                   dp, dp, dp, dp, dp, dp, ctypes.c_int, dp, ctypes.c_int,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   dp, dp, dp, dp, dp, llp, ctypes.c_int, dp, dp]
        L.orcoct_march_brute.restype = None
        L.orcoct_march_brute.argtypes = L.orcoct_march.argtypes
        L.orcoct_map_z.restype = None
        L.orcoct_map_z.argtypes = [ctypes.c_int, ctypes.c_int, ip, ctypes.c_double, dp, dp, dp, dp,
                                   dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int, dp, ctypes.c_int, dp, dp]
        _lib = L
    return _lib


def max_threads() -> int:
    """Threads the oracle's marches use with n_threads = 0."""
    return int(lib().orc_max_threads())


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------------------
# Per-cell physics (numpy)
# ---------------------------------------------------------------------------

def planck(nu, T):
    """B_nu(T) = (2 h nu^3 / c^2) / (exp(h nu / k T) - 1); 0 at T = 0."""
    nu = np.asarray(nu, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return (2.0 * H * nu ** 3 / C ** 2) / np.expm1(H * nu / (KB * T))


def doppler_b(T_kin, b_turb, mass_amu):
    """Doppler parameter b = sqrt(2 k T / m + b_turb^2) (turbulence given as a b value)."""
    T_kin = np.asarray(T_kin, dtype=np.float64)
    b_turb = np.asarray(b_turb, dtype=np.float64)
    return np.sqrt(2.0 * KB * T_kin / (mass_amu * AMU) + b_turb ** 2)


def lte_populations(mol, T_kin):
    """Boltzmann populations x_i = g_i exp(-E_i/T) / sum (shape [ncell, L])."""
    T = np.atleast_1d(np.asarray(T_kin, dtype=np.float64))
    E = np.asarray(mol.E_K, dtype=np.float64)
    w = np.asarray(mol.g, dtype=np.float64)[None, :] * np.exp(-(E[None, :] - E.min()) / T[:, None])
    return w / w.sum(axis=1, keepdims=True)


def einstein_B(mol):
    """B_ul = A c^2 / (2 h nu^3), B_lu = (g_u/g_l) B_ul (intensity convention)."""
    A = np.asarray(mol.A, dtype=np.float64)
    nu = np.asarray(mol.nu, dtype=np.float64)
    Bul = A * C ** 2 / (2.0 * H * nu ** 3)
    g = np.asarray(mol.g, dtype=np.float64)
    Blu = Bul * g[mol.up] / g[mol.lo]
    return Bul, Blu


def prepare(mol, x, n_mol):
    """Line opacity and emissivity coefficients per transition and cell.

    kappa = (c^3 / (8 pi nu^3)) A n_mol (x_l g_u/g_l - x_u)   [s^-1],
    eta   = (h c / (4 pi)) A n_mol x_u,
    so that over a step of length s with profile density p (s/cm)
    tau = kappa p s and the emitted intensity is eta p s (source S = eta/kappa).
    Returns arrays [n_trans, ncell].
    """
    x = np.asarray(x, dtype=np.float64)
    n_mol = np.asarray(n_mol, dtype=np.float64)
    g = np.asarray(mol.g, dtype=np.float64)
    out_k, out_e = [], []
    for t in range(mol.n_trans):
        u, l = int(mol.up[t]), int(mol.lo[t])
        A, nu = float(mol.A[t]), float(mol.nu[t])
        xu, xl = x[:, u], x[:, l]
        out_k.append((C ** 3 / (8.0 * np.pi * nu ** 3)) * A * n_mol * (xl * g[u] / g[l] - xu))
        out_e.append((H * C / (4.0 * np.pi)) * A * n_mol * xu)
    return np.array(out_k), np.array(out_e)


def collision_matrix(mol, n_H2, T_kin):
    """C[k, i, j] = collisional rate i -> j (s^-1) for every pair of levels:
    downward C_ul = n_H2 gamma_ul, upward by detailed balance
    C_lu = C_ul (g_u/g_l) exp(-(E_u - E_l)/T_kin)."""
    n = np.atleast_1d(np.asarray(n_H2, dtype=np.float64))
    T = np.atleast_1d(np.asarray(T_kin, dtype=np.float64))
    L = mol.n_levels
    g = np.asarray(mol.g, dtype=np.float64)
    E = np.asarray(mol.E_K, dtype=np.float64)
    Cm = np.zeros((n.shape[0], L, L))
    for u in range(L):
        for l in range(u):
            gam = float(mol.gamma_down[u, l])
            if gam == 0.0:
                continue
            down = n * gam
            Cm[:, u, l] = down
            Cm[:, l, u] = down * (g[u] / g[l]) * np.exp(-(E[u] - E[l]) / T)
    return Cm


def rate_matrix(mol, n_H2, T_kin, J, Lam, use_ali):
    """R[k, i, j] = total rate i -> j.

    Radiative (per transition t = (u,l)): R_ul += A (1 - Lam) + B_ul J,
    R_lu += B_lu J when ``use_ali`` (J is then the external field only);
    plain Lambda iteration uses A and the full J."""
    R = collision_matrix(mol, n_H2, T_kin)
    Bul, Blu = einstein_B(mol)
    for t in range(mol.n_trans):
        u, l = int(mol.up[t]), int(mol.lo[t])
        esc = (1.0 - Lam[t]) if use_ali else 1.0
        R[:, u, l] += mol.A[t] * esc + Bul[t] * J[t]
        R[:, l, u] += Blu[t] * J[t]
    return R


def se_solve(R, x_old):
    """Solve sum_j x_j R_ji - x_i sum_j R_ij = 0 with sum_i x_i = 1.

    The conservation row replaces the equation of the level with the largest
    current population (ties -> lowest index).  numpy.linalg.solve (LAPACK
    LU with partial pivoting) does the elimination.  Returns x [ncell, L]."""
    nc, L, _ = R.shape
    M = np.transpose(R, (0, 2, 1)).copy()          # M[i, j] = R[j, i]
    out = R.sum(axis=2)                            # sum_j R_ij
    idx = np.arange(L)
    M[:, idx, idx] -= out
    r = np.argmax(x_old, axis=1)
    rhs = np.zeros((nc, L))
    M[np.arange(nc), r, :] = 1.0
    rhs[np.arange(nc), r] = 1.0
    return np.linalg.solve(M, rhs[..., None])[..., 0]


def max_rel_change(x_new, x_old, floor=1.0e-10):
    """delta = max |x_new - x_old| / x_new over entries with x_new >= floor."""
    m = x_new >= floor
    if not np.any(m):
        return 0.0
    return float(np.max(np.abs(x_new[m] - x_old[m]) / x_new[m]))


# ---------------------------------------------------------------------------
# Geometry helpers
# ---------------------------------------------------------------------------

def ray_areas_1d(R_out, impact):
    """Ray weights: the annulus between the mid-points of neighbouring impact
    parameters (0 and R_out at the ends).  For equidistant rays this is
    2 pi b_j db."""
    b = np.asarray(impact, dtype=np.float64)
    edges = np.concatenate([[0.0], 0.5 * (b[1:] + b[:-1]), [float(R_out)]])
    return np.pi * (edges[1:] ** 2 - edges[:-1] ** 2)


def equidistant_impacts(R_out, n_rays):
    return (np.arange(n_rays) + 0.5) * float(R_out) / n_rays


def ray_steps_1d(R, b):
    R = _f64(R)
    n = R.shape[0]
    sh = np.zeros(2 * n, np.int32)
    s = np.zeros(2 * n)
    mu = np.zeros(2 * n)
    ns = lib().orc1d_ray_steps(n, _dp(R), float(b), sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                               _dp(s), _dp(mu))
    return sh[:ns], s[:ns], mu[:ns]


def healpix_nside2():
    """The 48 HEALPix N_side = 2 RING pixel centres (Gorski et al. 2005):
    polar rings z = +-(1 - i^2/12) with 4i pixels at phi = pi (j - 1/2)/(2i);
    equatorial rings i = 2..6 with z = 4/3 - i/3 and 8 pixels at
    phi = pi (j - s/2)/4, s = (i - 1) mod 2.  Returns [48, 3] (FP64)."""
    ns = 2
    dirs = []
    for i in range(1, 4 * ns):
        if i < ns:
            z = 1.0 - i * i / (3.0 * ns * ns)
            npix = 4 * i
            phis = [np.pi * (j - 0.5) / (2 * i) for j in range(1, npix + 1)]
        elif i <= 3 * ns:
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * ns)
            s = (i - ns + 1) % 2
            phis = [np.pi * (j - s / 2.0) / (2 * ns) for j in range(1, 4 * ns + 1)]
        else:
            ii = 4 * ns - i
            z = -(1.0 - ii * ii / (3.0 * ns * ns))
            npix = 4 * ii
            phis = [np.pi * (j - 0.5) / (2 * ii) for j in range(1, npix + 1)]
        st = np.sqrt(max(0.0, 1.0 - z * z))
        for ph in phis:
            dirs.append((st * np.cos(ph), st * np.sin(ph), z))
    return np.array(dirs, dtype=np.float64)


def main_axis(d):
    return int(lib().orc3d_main_axis(_dp(_f64(d))))


def walk_3d(N, d, i, j, off=0.5):
    cap = 8 * N + 16
    cell = np.zeros(cap, np.int32)
    ln = np.zeros(cap)
    rs = np.zeros(cap, np.uint8)
    ns = lib().orc3d_walk(int(N), _dp(_f64(d)), int(i), int(j), float(off),
                          cell.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(ln),
                          rs.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), cap)
    assert ns >= 0
    return cell[:ns], ln[:ns], rs[:ns].astype(bool)


def path_sums_3d(N, dirs):
    dirs = _f64(dirs)
    out = np.zeros((dirs.shape[0], N ** 3))
    lib().orc3d_path_sums(int(N), dirs.shape[0], _dp(dirs), _dp(out))
    return out


# ---------------------------------------------------------------------------
# Marches (one transition)
# ---------------------------------------------------------------------------

@dataclass
class MarchResult:
    Jraw: np.ndarray
    Lraw: np.ndarray
    W: np.ndarray
    E: np.ndarray
    I_out: Optional[np.ndarray]
    cons: float


def _shape_call(shape):
    """C arguments (n, v, w) of a line shape plus the arrays that must stay
    alive during the call.  None is the single Gaussian; otherwise (v_k [cm/s],
    w_k) of the hyperfine components (Sect. 1: LTE between the components),
    the strengths relative (the C side divides by their sum)."""
    if shape is None:
        return [0, None, None], None
    v, w = _f64(shape[0]).ravel(), _f64(shape[1]).ravel()
    assert v.shape == w.shape and v.size > 0 and np.all(w > 0)
    return [int(v.size), _dp(v), _dp(w)], (v, w)


def march_1d(R, vr, bD, kappa, eta, impact, area, spec, I_bg, n_threads=0, want_I=False,
             shape=None):
    R, vr, bD, kappa, eta = map(_f64, (R, vr, bD, kappa, eta))
    impact, area = _f64(impact), _f64(area)
    n, nr, nch = R.shape[0], impact.shape[0], spec.n_channels
    J, Lm, W, E = (np.zeros(n) for _ in range(4))
    I_out = np.zeros(nr * nch) if want_I else None
    cons = np.zeros(1)
    hf, _keep = _shape_call(shape)
    lib().orc1d_march(n, _dp(R), _dp(vr), _dp(bD), _dp(kappa), _dp(eta), nr, _dp(impact),
                      _dp(area), nch, float(spec.v_min), float(spec.dv), float(I_bg),
                      int(n_threads), _dp(J), _dp(Lm), _dp(W), _dp(E), _dp(I_out), _dp(cons), *hf)
    return MarchResult(J, Lm, W, E, None if I_out is None else I_out.reshape(nr, nch), float(cons[0]))


def march_3d(N, delta, vx, vy, vz, bD, kappa, eta, dirs, spec, I_bg, n_threads=0, want_I=False,
             shape=None):
    vx, vy, vz, bD, kappa, eta = map(_f64, (vx, vy, vz, bD, kappa, eta))
    dirs = _f64(dirs)
    nc, nd, nch = N ** 3, dirs.shape[0], spec.n_channels
    J, Lm, W, E = (np.zeros(nc) for _ in range(4))
    I_out = np.zeros(nd * N * N * nch) if want_I else None
    cons = np.zeros(1)
    hf, _keep = _shape_call(shape)
    lib().orc3d_march(int(N), float(delta), _dp(vx), _dp(vy), _dp(vz), _dp(bD), _dp(kappa),
                      _dp(eta), nd, _dp(dirs), nch, float(spec.v_min), float(spec.dv),
                      float(I_bg), int(n_threads), _dp(J), _dp(Lm), _dp(W), _dp(E),
                      _dp(I_out), _dp(cons), *hf)
    return MarchResult(J, Lm, W, E, None if I_out is None else I_out.reshape(nd, N * N, nch),
                       float(cons[0]))


# ---------------------------------------------------------------------------
# Iteration drivers
# ---------------------------------------------------------------------------

@dataclass
class RunResult:
    x: np.ndarray            # final populations [ncell, L]
    history: list            # per iteration: dict(x, J, Lam, delta)
    W: np.ndarray
    iters: int


class _Problem:
    """Geometry-independent part of an oracle run."""

    def __init__(self, mol, n_H2, T_kin, b_turb, abundance, spec, T_bg):
        self.mol = mol
        self.n_H2 = _f64(n_H2)
        self.T = _f64(T_kin)
        self.bD = doppler_b(self.T, _f64(b_turb), mol.mass_amu)
        self.n_mol = self.n_H2 * _f64(abundance)
        self.spec = spec
        self.I_bg = planck(np.asarray(mol.nu, dtype=np.float64), T_bg)


def _iterate(prob, march, n_iter, use_ali, x0, tol, record, solve_mask=None):
    mol = prob.mol
    x = lte_populations(mol, prob.T) if x0 is None else _f64(x0).copy()
    hist = []
    W = None
    it_done = 0
    for it in range(n_iter):
        kap, eta = prepare(mol, x, prob.n_mol)
        J = np.zeros((mol.n_trans, x.shape[0]))
        Lam = np.zeros_like(J)
        for t in range(mol.n_trans):
            res = march(t, kap[t], eta[t])
            W = res.W
            Wsafe = np.where(W > 0, W, 1.0)
            J[t] = res.Jraw / Wsafe
            Lam[t] = res.Lraw / Wsafe
            if not use_ali:
                S = np.where(kap[t] != 0, eta[t] / np.where(kap[t] != 0, kap[t], 1.0), 0.0)
                J[t] = J[t] + S * Lam[t]
        if solve_mask is None:
            R = rate_matrix(mol, prob.n_H2, prob.T, J, Lam, use_ali)
            x_new = se_solve(R, x)
        else:
            sel = solve_mask
            R = rate_matrix(mol, prob.n_H2[sel], prob.T[sel], J[:, sel], Lam[:, sel], use_ali)
            x_new = x.copy()
            x_new[sel] = se_solve(R, x[sel])
        delta = max_rel_change(x_new, x)
        if record:
            hist.append(dict(x=x_new.copy(), J=J, Lam=Lam, delta=delta))
        else:
            hist.append(dict(delta=delta))
        x = x_new
        it_done = it + 1
        if tol is not None and delta < tol:
            break
    return RunResult(x=x, history=hist, W=W, iters=it_done)


def run_1d(mol, model, spec, T_bg, n_iter, use_ali=True, x0=None, tol=None,
           n_threads=0, record=True, hyperfine=None):
    """Lambda / ALI iteration on a 1D shell model from LTE (or x0).
    hyperfine: {transition: (v_k [cm/s], w_k)} line shapes (others Gaussian)."""
    hfs = hyperfine or {}
    prob = _Problem(mol, model.n_H2, model.T_kin, model.b_turb, model.abundance, spec, T_bg)
    R = _f64(model.r_out)
    impact = equidistant_impacts(R[-1], model.n_rays) if model.impact is None else _f64(model.impact)
    area = ray_areas_1d(R[-1], impact)
    vr = _f64(model.v_r)

    def march(t, kap, eta):
        return march_1d(R, vr, prob.bD, kap, eta, impact, area, spec, prob.I_bg[t], n_threads,
                        shape=hfs.get(t))

    return _iterate(prob, march, n_iter, use_ali, x0, tol, record)


def core_entry_1d(R, vr, bD, kappa, eta, impact, K, spec, I_bg):
    """Intensity [n_rays, n_ch] each ray carries when it reaches the core
    boundary R[K] on its way in (rows of rays that do not reach it are 0)."""
    R, vr, bD, kappa, eta, impact = map(_f64, (R, vr, bD, kappa, eta, impact))
    out = np.zeros(impact.shape[0] * spec.n_channels)
    lib().orc1d_core_entry(R.shape[0], _dp(R), _dp(vr), _dp(bD), _dp(kappa), _dp(eta), impact.shape[0],
                           _dp(impact), int(K), spec.n_channels, float(spec.v_min), float(spec.dv),
                           float(I_bg), _dp(out))
    return out.reshape(impact.shape[0], spec.n_channels)


def march_core_1d(R, vr, bD, kappa, eta, impact, area, K, spec, I_enter):
    """Raw sums (Jraw, Lraw) of the core pieces of the rays (shells 0..K),
    each ray starting from its row of I_enter at the core boundary."""
    R, vr, bD, kappa, eta, impact, area = map(_f64, (R, vr, bD, kappa, eta, impact, area))
    I_enter = _f64(I_enter)
    J, Lm = np.zeros(R.shape[0]), np.zeros(R.shape[0])
    lib().orc1d_march_core(R.shape[0], _dp(R), _dp(vr), _dp(bD), _dp(kappa), _dp(eta), impact.shape[0],
                           _dp(impact), _dp(area), int(K), spec.n_channels, float(spec.v_min),
                           float(spec.dv), _dp(I_enter), _dp(J), _dp(Lm))
    return J, Lm


def core_extent(mol, model, spec, x, n_mol, bD, tau_min):
    """Outermost shell of the optically thick core: the largest k whose
    line-centre optical depth to the model's surface along the radius,
    tau_k = sum_{k' >= k} kappa_k' (R_k' - R_k'-1) / (b_k' sqrt(pi)) (static
    gas), reaches tau_min in some transition; -1 when none does."""
    kap, _ = prepare(mol, x, n_mol)
    R = _f64(model.r_out)
    dr = np.diff(np.concatenate([[0.0], R]))
    tau_shell = kap * dr / (_f64(bD) * SQRT_PI)
    tau_out = np.cumsum(tau_shell[:, ::-1], axis=1)[:, ::-1]
    hit = np.nonzero(np.max(tau_out, axis=0) >= tau_min)[0]
    return int(hit[-1]) if hit.size else -1


def run_1d_sub(mol, model, spec, T_bg, n_iter, n_sub, tau_min, x0=None, tol=None, record=True,
               core=None):
    """ALI iteration of a 1D model with sub-iterations in its optically thick
    core (the paper's Sect. 4: populations updated more frequently where the
    lines are thick; equilibrium and ALI form of Sect. 2).

    Each iteration: (1) every transition is marched along every ray with the
    current populations and every shell is solved, exactly as run_1d does
    (delta is this solve's maximum relative change); (2) the core is the
    shells 0..K, K = core_extent(the new populations, tau_min) (or the fixed
    ``core``); with the envelope's new populations held, n_sub times: the
    core's opacities and emissivities from its current populations, the core
    pieces of the rays (each from the intensity it enters the core with,
    computed once per iteration from the envelope), the core shells' solve
    with those absorbed counts and diagonal operator (normalised by the full
    ray set's W).  history[i]: x (after the sub-iterations), delta, K."""
    prob = _Problem(mol, model.n_H2, model.T_kin, model.b_turb, model.abundance, spec, T_bg)
    R = _f64(model.r_out)
    impact = equidistant_impacts(R[-1], model.n_rays) if model.impact is None else _f64(model.impact)
    area = ray_areas_1d(R[-1], impact)
    vr = _f64(model.v_r)
    x = lte_populations(mol, prob.T) if x0 is None else _f64(x0).copy()
    hist = []
    it_done = 0
    W = None
    for it in range(n_iter):
        kap, eta = prepare(mol, x, prob.n_mol)
        J = np.zeros((mol.n_trans, x.shape[0]))
        Lam = np.zeros_like(J)
        for t in range(mol.n_trans):
            res = march_1d(R, vr, prob.bD, kap[t], eta[t], impact, area, spec, prob.I_bg[t])
            W = res.W
            Wsafe = np.where(W > 0, W, 1.0)
            J[t] = res.Jraw / Wsafe
            Lam[t] = res.Lraw / Wsafe
        Rm = rate_matrix(mol, prob.n_H2, prob.T, J, Lam, True)
        x_new = se_solve(Rm, x)
        delta = max_rel_change(x_new, x)
        if core is None:
            K = core_extent(mol, model, spec, x_new, prob.n_mol, prob.bD, tau_min)
        else:
            K = int(core)
        if K >= 0 and n_sub > 0:
            c = slice(0, K + 1)
            kap_n, eta_n = prepare(mol, x_new, prob.n_mol)
            I_enter = [core_entry_1d(R, vr, prob.bD, kap_n[t], eta_n[t], impact, K, spec, prob.I_bg[t])
                       for t in range(mol.n_trans)]
            Wsafe = np.where(W > 0, W, 1.0)
            for _ in range(n_sub):
                kap_c, eta_c = prepare(mol, x_new, prob.n_mol)
                Jc = np.zeros((mol.n_trans, K + 1))
                Lc = np.zeros_like(Jc)
                for t in range(mol.n_trans):
                    jr, lr = march_core_1d(R, vr, prob.bD, kap_c[t], eta_c[t], impact, area, K, spec,
                                           I_enter[t])
                    Jc[t] = (jr / Wsafe)[c]
                    Lc[t] = (lr / Wsafe)[c]
                Rc = rate_matrix(mol, prob.n_H2[c], prob.T[c], Jc, Lc, True)
                x_new[c] = se_solve(Rc, x_new[c])
        if record:
            hist.append(dict(x=x_new.copy(), delta=delta, K=K, J=J, Lam=Lam))
        else:
            hist.append(dict(delta=delta, K=K))
        x = x_new
        it_done = it + 1
        if tol is not None and delta < tol:
            break
    return RunResult(x=x, history=hist, W=W, iters=it_done)


def run_3d(mol, model, spec, T_bg, n_iter, dirs=None, use_ali=True, x0=None, tol=None,
           n_threads=0, record=True, hyperfine=None):
    """Lambda / ALI iteration on a regular N^3 model (FP32 fields promoted to
    FP64); hyperfine as in run_1d."""
    hfs = hyperfine or {}
    N = int(model.n0[0])
    assert model.n0 == (N, N, N) and model.n_oct_levels == 0
    prob = _Problem(mol, model.n_H2, model.T_kin, model.b_turb, model.abundance, spec, T_bg)
    dirs = healpix_nside2() if dirs is None else _f64(dirs)
    vx, vy, vz = _f64(model.vx), _f64(model.vy), _f64(model.vz)

    def march(t, kap, eta):
        return march_3d(N, float(model.root_cell_cm), vx, vy, vz, prob.bD, kap, eta, dirs,
                        spec, prob.I_bg[t], n_threads, shape=hfs.get(t))

    return _iterate(prob, march, n_iter, use_ali, x0, tol, record)


# ---------------------------------------------------------------------------
# Octrees (Sect. 2.2)
# ---------------------------------------------------------------------------

@dataclass
class OctTree:
    """Global numbering of an octree model: cells level by level; child[g] is
    the global index of the first of the 8 children of cell g (-1: leaf)."""
    N: int
    Lmax: int
    child: np.ndarray        # int32 [n_cells]
    level: np.ndarray        # int32 [n_cells]
    offsets: np.ndarray      # first global index of each level

    @property
    def leaf(self) -> np.ndarray:
        return self.child < 0


def octree_of(model) -> OctTree:
    counts = [int(c) for c in model.n_cells_per_level]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    child = np.full(int(offs[-1]), -1, np.int32)
    level = np.zeros(int(offs[-1]), np.int32)
    for lev, fc in enumerate(model.first_child):
        fc = np.asarray(fc, dtype=np.int64)
        g = slice(int(offs[lev]), int(offs[lev + 1]))
        level[g] = lev
        if lev + 1 < len(counts):
            child[g] = np.where(fc >= 0, fc + offs[lev + 1], -1)
    return OctTree(N=int(model.n0[0]), Lmax=len(counts) - 1, child=child, level=level, offsets=offs)


OCT_STATS = ("root", "split", "side", "terminated", "wrapped", "steps")


def march_oct(tree: OctTree, root_cm, vx, vy, vz, bD, kappa, eta, dirs, spec, I_bg, n_threads=0,
              shape=None, brute=False):
    """One transition through an octree for the given directions; also returns
    the ray statistics (dict over OCT_STATS).  kappa None: geometry only.
    brute: the brute-force lattice of 4^Lmax straight lines per root surface
    element instead of the created and terminated rays (Sect. 2.2)."""
    nc = tree.child.shape[0]
    dirs = _f64(dirs)
    geo = kappa is None
    args = [None] * 6 if geo else list(map(_f64, (vx, vy, vz, bD, kappa, eta)))
    nch = 0 if geo else spec.n_channels
    J, Lm, W, E = (np.zeros(nc) for _ in range(4))
    cons = np.zeros(1)
    st = np.zeros(len(OCT_STATS), np.int64)
    child = np.ascontiguousarray(tree.child, dtype=np.int32)
    hf, _keep = _shape_call(shape)
    fn = lib().orcoct_march_brute if brute else lib().orcoct_march
    fn(tree.N, tree.Lmax, nc, child.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                       float(root_cm), *[_dp(a) for a in args], dirs.shape[0], _dp(dirs), nch,
                       0.0 if geo else float(spec.v_min), 1.0 if geo else float(spec.dv),
                       0.0 if geo else float(I_bg), int(n_threads), _dp(J), _dp(Lm), _dp(W),
                       _dp(E), _dp(cons), st.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), *hf)
    return MarchResult(J, Lm, W, E, None, float(cons[0])), dict(zip(OCT_STATS, map(int, st)))


def run_oct(mol, model, spec, T_bg, n_iter, dirs=None, use_ali=True, x0=None, tol=None,
            n_threads=0, record=True, hyperfine=None, brute=False):
    """Lambda / ALI iteration on an octree model.  Every cell of every level
    carries populations; only leaves are marched and solved, refined cells
    keep their starting values.  hyperfine as in run_1d; brute as in
    march_oct."""
    hfs = hyperfine or {}
    tree = octree_of(model)
    leaf = tree.leaf
    prob = _Problem(mol, model.n_H2, model.T_kin, model.b_turb, model.abundance, spec, T_bg)
    dirs = healpix_nside2() if dirs is None else _f64(dirs)
    vx, vy, vz = _f64(model.vx), _f64(model.vy), _f64(model.vz)

    def march(t, kap, eta):
        return march_oct(tree, float(model.root_cell_cm), vx, vy, vz, prob.bD, kap, eta, dirs,
                         spec, prob.I_bg[t], n_threads, shape=hfs.get(t), brute=brute)[0]

    res = _iterate(prob, march, n_iter, use_ali, x0, tol, record, solve_mask=leaf)
    return res


def spectra_oct(mol, model, spec, T_bg, x, trans, n_threads=0, shape=None):
    """+z map of an octree: one line of sight per root surface element on the
    level-0 ray lattice, Delta I [N*N (index y*N + x), n_ch]; shape: the
    transition's hyperfine components (v_k, w_k) or None."""
    tree = octree_of(model)
    N = tree.N
    prob = _Problem(mol, model.n_H2, model.T_kin, model.b_turb, model.abundance, spec, T_bg)
    kap, eta = prepare(mol, _f64(x), prob.n_mol)
    out = np.zeros(N * N * spec.n_channels)
    child = np.ascontiguousarray(tree.child, dtype=np.int32)
    hf, _keep = _shape_call(shape)
    lib().orcoct_map_z(N, tree.Lmax, child.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                       float(model.root_cell_cm), _dp(_f64(model.vx)), _dp(_f64(model.vy)),
                       _dp(_f64(model.vz)), _dp(prob.bD), _dp(_f64(kap[trans])), _dp(_f64(eta[trans])),
                       spec.n_channels, float(spec.v_min), float(spec.dv), float(prob.I_bg[trans]),
                       int(n_threads), _dp(out), *hf)
    return out.reshape(N * N, spec.n_channels) - prob.I_bg[trans]


def spectra_1d(mol, model, spec, T_bg, x, trans, impact=None, n_threads=0, shape=None):
    """Emergent Delta I = I - I_bg [n_los, n_ch] of transition ``trans`` for
    rays with the given impact parameters (default: the model's ray set);
    shape as in spectra_oct."""
    prob = _Problem(mol, model.n_H2, model.T_kin, model.b_turb, model.abundance, spec, T_bg)
    R = _f64(model.r_out)
    if impact is None:
        impact = equidistant_impacts(R[-1], model.n_rays) if model.impact is None else model.impact
    impact = _f64(impact)
    kap, eta = prepare(mol, _f64(x), prob.n_mol)
    area = np.ones_like(impact)
    res = march_1d(R, _f64(model.v_r), prob.bD, kap[trans], eta[trans], impact, area, spec,
                   prob.I_bg[trans], n_threads, want_I=True, shape=shape)
    return res.I_out - prob.I_bg[trans]


def spectra_3d(mol, model, spec, T_bg, x, trans, n_threads=0, shape=None):
    """+z map: one line of sight per surface cell (x, y) through the cell
    centres, Delta I [N*N (index y*N + x), n_ch]; shape as in spectra_oct."""
    N = int(model.n0[0])
    prob = _Problem(mol, model.n_H2, model.T_kin, model.b_turb, model.abundance, spec, T_bg)
    kap, eta = prepare(mol, _f64(x), prob.n_mol)
    res = march_3d(N, float(model.root_cell_cm), _f64(model.vx), _f64(model.vy), _f64(model.vz),
                   prob.bD, kap[trans], eta[trans], np.array([[0.0, 0.0, 1.0]]), spec,
                   prob.I_bg[trans], n_threads, want_I=True, shape=shape)
    return res.I_out[0] - prob.I_bg[trans]
