"""Seeded synthetic inputs for the ALI line ray march.

This module only *generates inputs*: molecule tables, 1D shell models, 3D
density/velocity cubes and the serving request stream.  It holds none of the
method's arithmetic (no profiles, optical depths, rates or solves), so both
the HIP path and the FP64 oracle may consume what it produces.

Everything is deterministic for a given seed (numpy PCG64 via
``numpy.random.default_rng``).

Units are CGS and Kelvin throughout.  The shapes follow the paper's
workloads: 1D clouds of nested shells with infall (Sect. 3.1, App. A.1),
a turbulent N^3 Cartesian cloud with a 10-level linear rotor and a few
hundred channels (Sect. 3.3, App. A.2), and an octree built on top of the
same fields (App. A.3).
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

# CODATA-2018 exact values (SI redefinition), CGS.  Used here only to express
# the synthetic level energies in Kelvin and the inputs in CGS units.
H_PLANCK = 6.62607015e-27      # erg s
K_BOLTZ = 1.380649e-16         # erg / K
C_LIGHT = 2.99792458e10        # cm / s
PC_CM = 3.0856775814913673e18  # cm
KMS = 1.0e5                    # cm/s per km/s


@dataclass
class Molecule:
    """Level and transition tables of a synthetic species.

    ``gamma_down[u, l]`` (u > l) is the downward collision rate coefficient
    (cm^3 s^-1, temperature independent); all other entries are zero.
    Radiative transitions are (up[t], lo[t]) with Einstein A[t] and rest
    frequency nu[t].
    """
    E_K: np.ndarray
    g: np.ndarray
    up: np.ndarray
    lo: np.ndarray
    A: np.ndarray
    nu: np.ndarray
    gamma_down: np.ndarray
    mass_amu: float
    name: str = ""

    @property
    def n_levels(self) -> int:
        return int(self.E_K.shape[0])

    @property
    def n_trans(self) -> int:
        return int(self.up.shape[0])


def two_level_molecule(nu_hz: float = 110.0e9, A: float = 6.0e-8,
                       g_l: float = 1.0, g_u: float = 3.0,
                       gamma: float = 2.0e-11, mass_amu: float = 29.0) -> Molecule:
    """Synthetic two-level species: E_u - E_l = h nu, g_u/g_l = 3."""
    E = np.array([0.0, H_PLANCK * nu_hz / K_BOLTZ])
    gd = np.zeros((2, 2))
    gd[1, 0] = gamma
    return Molecule(E_K=E, g=np.array([g_l, g_u]), up=np.array([1], np.int32),
                    lo=np.array([0], np.int32), A=np.array([A]),
                    nu=np.array([nu_hz]), gamma_down=gd, mass_amu=mass_amu,
                    name="two-level")


def rotor_molecule(n_levels: int = 10, B_hz: float = 55.0e9, A10: float = 7.0e-8,
                   gamma: float = 1.0e-11, mass_amu: float = 29.0) -> Molecule:
    """Synthetic linear rotor with ``n_levels`` levels J = 0..n_levels-1.

    E_J = h B J(J+1), g_J = 2J+1, radiative only for J -> J-1 with
    nu = 2 B J and A_J = A10 * J^3 (A_{1->0} = A10); every pair u > l
    collides with the same downward rate coefficient ``gamma``.
    """
    J = np.arange(n_levels, dtype=np.float64)
    E = H_PLANCK * B_hz * J * (J + 1.0) / K_BOLTZ
    g = 2.0 * J + 1.0
    up = np.arange(1, n_levels, dtype=np.int32)
    lo = up - 1
    Ju = up.astype(np.float64)
    A = A10 * Ju ** 3
    nu = 2.0 * B_hz * Ju
    gd = np.zeros((n_levels, n_levels))
    for u in range(n_levels):
        for l in range(u):
            gd[u, l] = gamma
    return Molecule(E_K=E, g=g, up=up, lo=lo, A=A, nu=nu, gamma_down=gd,
                    mass_amu=mass_amu, name=f"rotor{n_levels}")


@dataclass
class Spectral:
    """Channel grid: centres v_c = v_min + (c + 1/2) dv, c = 0..n_channels-1."""
    n_channels: int
    v_min: float
    dv: float

    @staticmethod
    def symmetric(n_channels: int, half_width_kms: float) -> "Spectral":
        vmin = -half_width_kms * KMS
        return Spectral(n_channels, vmin, 2.0 * half_width_kms * KMS / n_channels)


@dataclass
class Model1D:
    """Spherical cloud of nested shells; values refer to shell k = (R_{k-1}, R_k]."""
    r_out: np.ndarray
    n_H2: np.ndarray
    T_kin: np.ndarray
    b_turb: np.ndarray
    v_r: np.ndarray
    abundance: np.ndarray
    n_rays: int
    impact: Optional[np.ndarray] = None

    @property
    def n_shells(self) -> int:
        return int(self.r_out.shape[0])


@dataclass
class Model3D:
    """Regular N^3 grid (cell (x,y,z) stored at index (z*N + y)*N + x) or an
    octree (see ``octree`` module docs).  Fields are float32 per leaf."""
    n0: tuple
    root_cell_cm: float
    n_H2: np.ndarray
    T_kin: np.ndarray
    b_turb: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    abundance: np.ndarray
    n_oct_levels: int = 0
    n_cells_per_level: Optional[List[int]] = None
    first_child: Optional[List[np.ndarray]] = None

    @property
    def n_cells(self) -> int:
        return int(self.n_H2.shape[0])


@dataclass
class Workload:
    name: str
    mol: Molecule
    spec: Spectral
    T_bg: float
    model: object
    n_iter: int
    extra: Dict = field(default_factory=dict)


# ---------------------------------------------------------------------------
# 1D clouds
# ---------------------------------------------------------------------------

def cloud_1d_log(n_shells: int = 100, r_in_pc: float = 0.01, r_out_pc: float = 0.1,
                 n_out: float = 1.0e3, T_kin: float = 10.0, b_turb_kms: float = 0.2,
                 abundance: float = 1.0e-9, n_rays: Optional[int] = None,
                 infall_kms_at_005pc: float = 0.0) -> Model1D:
    """Log-spaced shells R_k = r_out (r_in/r_out)^{(N-1-k)/(N-1)}, n = n_out (R/r_out)^-2.

    With the defaults: 100 shells between 0.01 and 0.1 pc and n from 1e5 to
    1e3 cm^-3.  Values are sampled at the outer radius of each shell.  An
    optional infall v_r = -A (R/0.05 pc)^-1/2 can be added.
    """
    k = np.arange(n_shells, dtype=np.float64)
    ratio = r_in_pc / r_out_pc
    R_pc = r_out_pc * ratio ** ((n_shells - 1 - k) / (n_shells - 1))
    R = R_pc * PC_CM
    n = n_out * (R_pc / r_out_pc) ** (-2.0)
    vr = np.zeros(n_shells)
    if infall_kms_at_005pc != 0.0:
        vr = -infall_kms_at_005pc * KMS * (R_pc / 0.05) ** (-0.5)
    return Model1D(r_out=R, n_H2=n, T_kin=np.full(n_shells, T_kin),
                   b_turb=np.full(n_shells, b_turb_kms * KMS), v_r=vr,
                   abundance=np.full(n_shells, abundance),
                   n_rays=n_rays if n_rays is not None else n_shells)


def cloud_1d_plummer(n_shells: int = 1000, r_out_pc: float = 0.5, n0: float = 1.0e6,
                     r_flat_pc: float = 0.02, T_in: float = 8.0, T_out: float = 20.0,
                     infall_kms: float = 0.3, b_turb_kms: float = 0.15,
                     abundance: float = 1.0e-9, n_rays: Optional[int] = None) -> Model1D:
    """Linear shells R_k = r_out (k+1)/N with a Plummer profile
    n = n0 (1 + (r/r_flat)^2)^-5/2, T linear from T_in (centre) to T_out (edge),
    infall v = -infall (r/0.05 pc)^-1/2, all sampled at the shell's outer radius.
    """
    k = np.arange(n_shells, dtype=np.float64)
    R_pc = r_out_pc * (k + 1.0) / n_shells
    n = n0 * (1.0 + (R_pc / r_flat_pc) ** 2) ** (-2.5)
    T = T_in + (T_out - T_in) * R_pc / r_out_pc
    vr = -infall_kms * KMS * (R_pc / 0.05) ** (-0.5)
    return Model1D(r_out=R_pc * PC_CM, n_H2=n, T_kin=T,
                   b_turb=np.full(n_shells, b_turb_kms * KMS), v_r=vr,
                   abundance=np.full(n_shells, abundance),
                   n_rays=n_rays if n_rays is not None else n_shells)


def uniform_sphere_1d(n_shells: int, radius_cm: float, n_H2: float, T_kin: float,
                      b_turb: float, abundance: float, n_rays: int,
                      v_r: float = 0.0) -> Model1D:
    """Homogeneous sphere split into equal-width shells (for closed-form checks)."""
    R = radius_cm * (np.arange(n_shells) + 1.0) / n_shells
    return Model1D(r_out=R, n_H2=np.full(n_shells, n_H2), T_kin=np.full(n_shells, T_kin),
                   b_turb=np.full(n_shells, b_turb), v_r=np.full(n_shells, v_r),
                   abundance=np.full(n_shells, abundance), n_rays=n_rays)


# ---------------------------------------------------------------------------
# 3D fields
# ---------------------------------------------------------------------------

def _kgrid(N: int):
    kx = np.fft.fftfreq(N, d=1.0 / N)
    kz = np.fft.rfftfreq(N, d=1.0 / N)
    KX, KY, KZ = np.meshgrid(kx, kx, kz, indexing="ij")
    return KX, KY, KZ


def grf_k4(N: int, seed: int) -> np.ndarray:
    """Gaussian random field with power ~ k^-4 (amplitude |k|^-2), zero mean,
    unit variance.  Axis order of the returned array is (x, y, z)."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((N, N, N))
    F = np.fft.rfftn(white)
    KX, KY, KZ = _kgrid(N)
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = 1.0 / k2[nz]
    g = np.fft.irfftn(F * amp, s=(N, N, N), axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    return g


def solenoidal_k4(N: int, seed: int, rms_cms: float) -> np.ndarray:
    """Divergence-free random velocity field (3, N, N, N) with a k^-4 spectrum,
    scaled so that sqrt(<|u|^2>) = rms_cms.  Components use seeds seed+1..+3."""
    KX, KY, KZ = _kgrid(N)
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = 1.0 / k2[nz]
    comps = []
    for i in range(3):
        rng = np.random.default_rng(seed + 1 + i)
        comps.append(np.fft.rfftn(rng.standard_normal((N, N, N))) * amp)
    kinv = np.zeros_like(k2)
    kinv[nz] = 1.0 / np.sqrt(k2[nz])
    khat = [KX * kinv, KY * kinv, KZ * kinv]
    dot = comps[0] * khat[0] + comps[1] * khat[1] + comps[2] * khat[2]
    comps = [comps[i] - khat[i] * dot for i in range(3)]
    u = np.stack([np.fft.irfftn(c, s=(N, N, N), axes=(0, 1, 2)) for c in comps])
    u *= rms_cms / math.sqrt(np.mean(np.sum(u ** 2, axis=0)))
    return u


def _to_cell_order(a_xyz: np.ndarray) -> np.ndarray:
    """(x,y,z)-indexed cube -> flat array with index (z*N + y)*N + x."""
    return np.ascontiguousarray(np.transpose(a_xyz, (2, 1, 0))).reshape(-1)


def turbulent_cube(N: int = 128, box_pc: float = 1.0, sigma_ln: float = 1.0,
                   mean_n: float = 1.0e3, v_rms_kms: float = 1.0, T_kin: float = 15.0,
                   b_turb_kms: float = 0.0, abundance: float = 1.0e-9,
                   seed: int = 3001) -> Model3D:
    """Lognormal density (k^-4 GRF, exact sample mean ``mean_n``) and a
    solenoidal k^-4 velocity field on a regular N^3 grid (float32 fields)."""
    g = grf_k4(N, seed)
    rho = np.exp(sigma_ln * g)
    rho *= mean_n / rho.mean()
    u = solenoidal_k4(N, seed, v_rms_kms * KMS)
    f32 = lambda a: _to_cell_order(a).astype(np.float32)
    nc = N ** 3
    return Model3D(n0=(N, N, N), root_cell_cm=box_pc * PC_CM / N,
                   n_H2=f32(rho), T_kin=np.full(nc, T_kin, np.float32),
                   b_turb=np.full(nc, b_turb_kms * KMS, np.float32),
                   vx=f32(u[0]), vy=f32(u[1]), vz=f32(u[2]),
                   abundance=np.full(nc, abundance, np.float32))


def uniform_cube(N: int, box_cm: float, n_H2: float, T_kin: float, b_turb: float,
                 abundance: float, velocity=(0.0, 0.0, 0.0)) -> Model3D:
    nc = N ** 3
    full = lambda v: np.full(nc, v, np.float32)
    return Model3D(n0=(N, N, N), root_cell_cm=box_cm / N, n_H2=full(n_H2),
                   T_kin=full(T_kin), b_turb=full(b_turb), vx=full(velocity[0]),
                   vy=full(velocity[1]), vz=full(velocity[2]), abundance=full(abundance))


# ---------------------------------------------------------------------------
# Octrees
# ---------------------------------------------------------------------------
# Layout: level 0 is the N^3 root grid in cell order (z*N + y)*N + x; the
# children of a refined level-l cell are 8 consecutive level-(l+1) cells,
# child offset cx + 2 cy + 4 cz, and the refined cells of a level hand out
# their children in index order.  first_child[l][i] is the level-(l+1) index
# of the first child of cell i of level l, -1 for a leaf.  Field arrays hold
# every cell of every level, level by level (values of refined cells are
# samples at their centres and carry no meaning).


def _morton3(x, y, z, bits):
    m = np.zeros(x.shape, np.int64)
    for b in range(bits):
        m |= ((x >> b) & 1).astype(np.int64) << (3 * b)
        m |= ((y >> b) & 1).astype(np.int64) << (3 * b + 1)
        m |= ((z >> b) & 1).astype(np.int64) << (3 * b + 2)
    return m


def octree_structure(N_root: int, n_refine: int, frac: float, score):
    """Refine, level by level, the fraction ``frac`` of cells with the highest
    ``score(level, ix, iy, iz)`` (ties: lower Morton index first).  Returns
    (coords per level [(ix, iy, iz) int64 arrays], first_child per level)."""
    iz, iy, ix = np.meshgrid(np.arange(N_root), np.arange(N_root), np.arange(N_root), indexing="ij")
    coords = [(ix.reshape(-1).astype(np.int64), iy.reshape(-1).astype(np.int64),
               iz.reshape(-1).astype(np.int64))]
    first_child = []
    for lev in range(n_refine):
        cx, cy, cz = coords[lev]
        n = cx.shape[0]
        n_ref = int(round(frac * n))
        fc = np.full(n, -1, np.int32)
        if n_ref > 0:
            sc = np.asarray(score(lev, cx, cy, cz), dtype=np.float64)
            bits = int(math.ceil(math.log2(N_root))) + lev + 1
            order = np.lexsort((_morton3(cx, cy, cz, bits), -sc))
            chosen = np.sort(order[:n_ref])
            fc[chosen] = 8 * np.arange(n_ref, dtype=np.int32)
            off = np.arange(8)
            kx = (2 * cx[chosen][:, None] + (off & 1)).reshape(-1)
            ky = (2 * cy[chosen][:, None] + ((off >> 1) & 1)).reshape(-1)
            kz = (2 * cz[chosen][:, None] + ((off >> 2) & 1)).reshape(-1)
            coords.append((kx, ky, kz))
        else:
            coords.append((np.zeros(0, np.int64),) * 3)
        first_child.append(fc)
        if n_ref == 0:
            break
    first_child.append(np.full(coords[-1][0].shape[0], -1, np.int32))
    return coords, first_child


def _trilinear(grids, px, py, pz):
    """Periodic trilinear interpolation of cell-centred (x, y, z) grids at
    positions in box units [0, 1); one output per grid."""
    G = grids[0].shape[0]
    outs = [np.zeros(px.shape, np.float64) for _ in grids]
    q = [p * G - 0.5 for p in (px, py, pz)]
    i0 = [np.floor(v).astype(np.int64) for v in q]
    fr = [v - i for v, i in zip(q, i0)]
    for dx in (0, 1):
        wx = fr[0] if dx else 1.0 - fr[0]
        ix = (i0[0] + dx) % G
        for dy in (0, 1):
            wxy = wx * (fr[1] if dy else 1.0 - fr[1])
            iy = (i0[1] + dy) % G
            for dz in (0, 1):
                w = wxy * (fr[2] if dz else 1.0 - fr[2])
                flat = (ix * G + iy) * G + (i0[2] + dz) % G
                for g, o in zip(grids, outs):
                    o += w * g.reshape(-1)[flat]
    return outs


def octree_centres(N_root, coords):
    """Cell centres (box units) of every cell, level by level."""
    pts = []
    for lev, (cx, cy, cz) in enumerate(coords):
        n_l = N_root << lev
        pts.append(((cx + 0.5) / n_l, (cy + 0.5) / n_l, (cz + 0.5) / n_l))
    return [np.concatenate([p[k] for p in pts]) for k in range(3)]


def octree_cloud(N_root: int = 64, n_refine: int = 4, frac: float = 0.34, grf_N: int = 256,
                 box_pc: float = 2.0, sigma_ln: float = 1.0, mean_n: float = 1.0e3,
                 v_rms_kms: float = 1.0, T_kin: float = 15.0, b_turb_kms: float = 0.0,
                 abundance: float = 1.0e-9, seed: int = 4001) -> Model3D:
    """Turbulent cloud on an octree: the lognormal k^-4 density and solenoidal
    k^-4 velocity of ``turbulent_cube`` generated on a grf_N^3 grid and sampled
    trilinearly (periodic) at every cell centre; each level refines its
    densest fraction ``frac`` of cells."""
    g = grf_k4(grf_N, seed)
    rho = np.exp(sigma_ln * g)
    rho *= mean_n / rho.mean()
    u = solenoidal_k4(grf_N, seed, v_rms_kms * KMS)

    def score(lev, cx, cy, cz):
        n_l = N_root << lev
        return _trilinear([rho], (cx + 0.5) / n_l, (cy + 0.5) / n_l, (cz + 0.5) / n_l)[0]

    coords, fc = octree_structure(N_root, n_refine, frac, score)
    px, py, pz = octree_centres(N_root, coords)
    nc = px.shape[0]
    n_s, ux, uy, uz = _trilinear([rho, u[0], u[1], u[2]], px, py, pz)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Model3D(n0=(N_root,) * 3, root_cell_cm=box_pc * PC_CM / N_root,
                   n_H2=f32(n_s), T_kin=f32(np.full(nc, T_kin)),
                   b_turb=f32(np.full(nc, b_turb_kms * KMS)),
                   vx=f32(ux), vy=f32(uy), vz=f32(uz), abundance=f32(np.full(nc, abundance)),
                   n_oct_levels=len(fc), n_cells_per_level=[int(c[0].shape[0]) for c in coords],
                   first_child=fc)


def octree_random(N_root: int, n_refine: int, frac: float, seed: int, box_cm: float,
                  n_H2: float, T_kin: float, b_turb: float, abundance: float,
                  velocity=(0.0, 0.0, 0.0)) -> Model3D:
    """Octree with uniform fields whose refined cells are drawn at random
    (seeded): the geometry-only cases of the tests."""
    rng = np.random.default_rng(seed)
    coords, fc = octree_structure(N_root, n_refine, frac, lambda lev, cx, cy, cz: rng.random(cx.shape[0]))
    nc = sum(int(c[0].shape[0]) for c in coords)
    full = lambda v: np.full(nc, v, np.float32)
    return Model3D(n0=(N_root,) * 3, root_cell_cm=box_cm / N_root, n_H2=full(n_H2), T_kin=full(T_kin),
                   b_turb=full(b_turb), vx=full(velocity[0]), vy=full(velocity[1]), vz=full(velocity[2]),
                   abundance=full(abundance), n_oct_levels=len(fc),
                   n_cells_per_level=[int(c[0].shape[0]) for c in coords], first_child=fc)

# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def workload_1d_small() -> Workload:
    """100 log shells 0.01-0.1 pc, n ~ r^-2 from 1e5 to 1e3 cm^-3, T = 10 K,
    b_turb = 0.2 km/s, static, X = 1e-9; two-level species; 128 channels
    over +-2 km/s; 100 equidistant rays; 20 ALI iterations in FP64."""
    return Workload("1d-100shell-2level", two_level_molecule(),
                    Spectral.symmetric(128, 2.0), 2.73, cloud_1d_log(), 20)


def workload_1d_plummer(n_shells: int = 1000, abundance: float = 1.0e-9) -> Workload:
    """1000 linear shells to 0.5 pc, Plummer n0 = 1e6, r_flat = 0.02 pc,
    T 8-20 K, infall -0.3 (r/0.05 pc)^-1/2 km/s, b_turb = 0.15 km/s,
    10-level rotor, 256 channels over +-4 km/s, FP32 march."""
    return Workload(f"1d-{n_shells}shell-plummer-rotor10", rotor_molecule(10),
                    Spectral.symmetric(256, 4.0), 2.73,
                    cloud_1d_plummer(n_shells=n_shells, abundance=abundance), 20)


def workload_3d_regular(N: int = 128, seed: int = 3001) -> Workload:
    """N^3 turbulent cloud, 1 pc box, lognormal sigma_ln = 1 (mean 1e3 cm^-3),
    solenoidal velocity rms 1 km/s, T = 15 K, 10-level rotor, 48 HEALPix
    directions, 256 channels over +-4 km/s."""
    return Workload(f"3d-regular-{N}^3-rotor10", rotor_molecule(10),
                    Spectral.symmetric(256, 4.0), 2.73,
                    turbulent_cube(N=N, seed=seed), 2, extra={"nside": 2})


def workload_octree(N_root: int = 64, n_refine: int = 4, seed: int = 4001) -> Workload:
    """Octree turbulent cloud: 64^3 root grid, 2 pc box, four refinement levels
    each refining the densest 34% of its cells (about 2e7 leaves), fields
    from a 256^3 lognormal / solenoidal k^-4 realisation sampled at the cell
    centres, T = 15 K, 10-level rotor, 256 channels over +-4 km/s."""
    m = octree_cloud(N_root=N_root, n_refine=n_refine, frac=0.34, grf_N=256, box_pc=2.0, seed=seed)
    return Workload(f"octree-{N_root}^3-L{n_refine}-rotor10", rotor_molecule(10),
                    Spectral.symmetric(256, 4.0), 2.73, m, 1, extra={"nside": 2})


def array_digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


# ---------------------------------------------------------------------------
# 1D request stream (parameter-search style)
# ---------------------------------------------------------------------------

@dataclass
class ServeRequest:
    mol: Molecule
    model: Model1D
    spec: Spectral
    arrival_s: float
    T_bg: float = 2.73


def serving_stream(n: int, seed: int = 5001, rate_per_s: float = 100.0,
                   shells=(50, 2000), levels=(2, 5, 10, 20), channels=(64, 128, 256)):
    """Requests with Poisson arrivals: shells uniform in [shells], level count
    and channel count uniform over the given sets, the log-shell geometry of
    the small 1D cloud (0.01-0.1 pc, n ~ r^-2) with the density scaled by a
    log-uniform factor in [0.1, 10], T_kin log-uniform in [5, 20] K, infall
    amplitude log-uniform in [0.01, 0.3] km/s at 0.05 pc with an r^-1/2 law,
    X = 1e-9, b_turb = 0.2 km/s, +-2 km/s band, one ray per shell."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n):
        t += rng.exponential(1.0 / rate_per_s)
        ns = int(rng.integers(shells[0], shells[1] + 1))
        L = int(rng.choice(levels))
        nch = int(rng.choice(channels))
        dens = float(10 ** rng.uniform(-1, 1))
        T = float(10 ** rng.uniform(np.log10(5.0), np.log10(20.0)))
        inf = float(10 ** rng.uniform(np.log10(0.01), np.log10(0.3)))
        m = cloud_1d_log(n_shells=ns, n_out=1.0e3 * dens, T_kin=T, b_turb_kms=0.2,
                         abundance=1.0e-9, infall_kms_at_005pc=inf)
        out.append(ServeRequest(rotor_molecule(L), m, Spectral.symmetric(nch, 2.0), t))
    return out
