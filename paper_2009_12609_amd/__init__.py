"""miloc: MI355X-native ALI line radiative transfer (Python binding).

A thin ctypes binding of ``libmiloc.so`` (C ABI declared in
``include/miloc.h``).  It only marshals arguments: every step of the
computation runs in the library's HIP kernels.  There is no fallback: if the
library is missing or no gfx950 GPU is present the calls raise.

Example::

    import paper_2009_12609_amd as miloc
    ctx = miloc.Context()
    ctx.load_molecule(mol)            # any object with E_K, g, up, lo, A, nu, gamma_down, mass_amu
    ctx.load_model_1d(model)          # r_out, n_H2, T_kin, b_turb, v_r, abundance, n_rays[, impact]
    ctx.set_spectral(128, -2e5, 3125.0)
    iters, delta = ctx.run(20, tol=0.0)
    x = ctx.populations()
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmiloc.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENOTCONV, ENUMERIC, EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
MARCH_FP32, MARCH_FP64 = 0, 1
_NAMES = {0: "MILOC_OK", -1: "MILOC_EINVAL", -2: "MILOC_ENOMEM", -3: "MILOC_EDEVICE",
          -4: "MILOC_ESTATE", -5: "MILOC_ENOTCONV", -6: "MILOC_ENUMERIC", -7: "MILOC_EBUSY"}

# Every function declared in include/miloc.h, with its ctypes signature.
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_ip = ctypes.POINTER(ctypes.c_int)
_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p


class MolStruct(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("E_K", _dp), ("g", _dp), ("n_trans", ctypes.c_int),
                ("up", _ip), ("lo", _ip), ("A", _dp), ("nu_Hz", _dp), ("gamma_down", _dp),
                ("mass_amu", ctypes.c_double)]


class Model1DStruct(ctypes.Structure):
    _fields_ = [("n_shells", ctypes.c_int), ("r_out_cm", _dp), ("n_H2", _dp), ("T_kin", _dp),
                ("b_turb_cms", _dp), ("v_r_cms", _dp), ("abundance", _dp),
                ("n_rays", ctypes.c_int), ("impact_cm", _dp)]


class Model3DStruct(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int * 3), ("n_oct_levels", ctypes.c_int),
                ("root_cell_cm", ctypes.c_double), ("n_cells_per_level", _i64p),
                ("first_child", ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))),
                ("n_H2", _fp), ("T_kin", _fp), ("b_turb_cms", _fp), ("vx", _fp), ("vy", _fp),
                ("vz", _fp), ("abundance", _fp)]


class Counters(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("march_launches", ctypes.c_int64),
                ("march_ms", ctypes.c_double), ("accumulate_ms", ctypes.c_double),
                ("prepare_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("ray_steps", ctypes.c_double),
                ("channel_updates", ctypes.c_double), ("march_lanes", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ResultInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("last_delta", ctypes.c_double),
                ("latency_s", ctypes.c_double), ("queue_s", ctypes.c_double), ("status", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("cancelled", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("active", ctypes.c_int64), ("peak_active", ctypes.c_int64),
                ("ticks", ctypes.c_int64), ("busy_s", ctypes.c_double),
                ("arena_used", ctypes.c_int64)]


_u64p = ctypes.POINTER(ctypes.c_uint64)

SIGNATURES = {
    "miloc_version": (ctypes.c_char_p, []),
    "miloc_create": (ctypes.c_int, [ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "miloc_destroy": (None, [_vp]),
    "miloc_last_error": (ctypes.c_char_p, [_vp]),
    "miloc_load_molecule": (ctypes.c_int, [_vp, ctypes.POINTER(MolStruct)]),
    "miloc_load_model_1d": (ctypes.c_int, [_vp, ctypes.POINTER(Model1DStruct)]),
    "miloc_load_model_3d": (ctypes.c_int, [_vp, ctypes.POINTER(Model3DStruct)]),
    "miloc_octree_schedule": (ctypes.c_int, [ctypes.POINTER(Model3DStruct), ctypes.c_int, _dp, ctypes.c_int,
                                             _i64p, _i64p, _ip, ctypes.POINTER(ctypes.c_uint32), _i64p]),
    "miloc_model_footprint": (ctypes.c_int, [ctypes.POINTER(Model1DStruct), ctypes.POINTER(Model3DStruct),
                                             ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                                             ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t),
                                             ctypes.POINTER(ctypes.c_size_t)]),
    "miloc_set_spectral": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_double]),
    "miloc_set_background": (ctypes.c_int, [_vp, ctypes.c_double]),
    "miloc_set_hyperfine": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _dp, _dp]),
    "miloc_set_octree_rays": (ctypes.c_int, [_vp, ctypes.c_int]),
    "miloc_set_directions_healpix": (ctypes.c_int, [_vp, ctypes.c_int]),
    "miloc_set_directions": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "miloc_set_march_precision": (ctypes.c_int, [_vp, ctypes.c_int]),
    "miloc_set_subiterations": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double]),
    "miloc_set_transition_batching": (ctypes.c_int, [_vp, ctypes.c_int]),
    "miloc_init_lte": (ctypes.c_int, [_vp]),
    "miloc_set_populations": (ctypes.c_int, [_vp, _dp]),
    "miloc_run": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _ip, _dp]),
    "miloc_get_sizes": (ctypes.c_int, [_vp, _i64p, _ip, _ip, _ip]),
    "miloc_get_populations": (ctypes.c_int, [_vp, _dp]),
    "miloc_get_radiation": (ctypes.c_int, [_vp, _dp, _dp]),
    "miloc_get_spectra": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _dp, _dp]),
    "miloc_get_counters": (ctypes.c_int, [_vp, ctypes.POINTER(Counters)]),
    "miloc_reset_counters": (ctypes.c_int, [_vp]),
    "miloc_server_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_vp)]),
    "miloc_server_destroy": (None, [_vp]),
    "miloc_server_last_error": (ctypes.c_char_p, [_vp]),
    "miloc_server_submit": (ctypes.c_int, [_vp, ctypes.POINTER(MolStruct), ctypes.POINTER(Model1DStruct),
                                           ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int, _u64p]),
    "miloc_server_footprint": (ctypes.c_int, [_vp, ctypes.POINTER(MolStruct), ctypes.POINTER(Model1DStruct),
                                              ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                              ctypes.POINTER(ctypes.c_size_t)]),
    "miloc_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, _ip]),
    "miloc_server_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_double, _ip]),
    "miloc_server_result_sizes": (ctypes.c_int, [_vp, ctypes.c_uint64, _ip, _ip, _ip, _ip]),
    "miloc_server_take": (ctypes.c_int, [_vp, ctypes.c_uint64, _dp, _dp, ctypes.POINTER(ResultInfo)]),
    "miloc_server_cancel": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "miloc_server_get_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ServerStats)]),
    "miloc_solve_1d_noalloc": (ctypes.c_int, [ctypes.c_int, _vp, ctypes.POINTER(MolStruct),
                                              ctypes.POINTER(Model1DStruct), ctypes.c_int, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                              _ip, _dp, _dp]),
}

_lib = None


def load_library(path: Optional[str] = None):
    """Load libmiloc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError(f"{p} is missing: build it with python paper_2009_12609_amd/build.py")
        L = ctypes.CDLL(p)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class MilocError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct)) if a is not None else ctypes.POINTER(ct)()


def _mol_struct(mol, keep):
    E, g = _f64(mol.E_K), _f64(mol.g)
    up = np.ascontiguousarray(np.asarray(mol.up, dtype=np.int32))
    lo = np.ascontiguousarray(np.asarray(mol.lo, dtype=np.int32))
    A, nu, gd = _f64(mol.A), _f64(mol.nu), _f64(mol.gamma_down)
    keep.extend([E, g, up, lo, A, nu, gd])
    return MolStruct(int(E.shape[0]), _ptr(E, ctypes.c_double), _ptr(g, ctypes.c_double),
                     int(up.shape[0]), _ptr(up, ctypes.c_int), _ptr(lo, ctypes.c_int),
                     _ptr(A, ctypes.c_double), _ptr(nu, ctypes.c_double), _ptr(gd, ctypes.c_double),
                     float(mol.mass_amu))


def _model1d_struct(m, keep):
    arrs = [_f64(a) for a in (m.r_out, m.n_H2, m.T_kin, m.b_turb, m.v_r, m.abundance)]
    imp = None if getattr(m, "impact", None) is None else _f64(m.impact)
    keep.extend(arrs + [imp])
    return Model1DStruct(int(arrs[0].shape[0]), *[_ptr(a, ctypes.c_double) for a in arrs],
                         int(m.n_rays), _ptr(imp, ctypes.c_double))


def _model3d_struct(m, keep):
    """Model3DStruct of a regular grid or an octree; arrays kept alive in keep."""
    arrs = [_f32(a) for a in (m.n_H2, m.T_kin, m.b_turb, m.vx, m.vy, m.vz, m.abundance)]
    keep.extend(arrs)
    n0 = (ctypes.c_int * 3)(*[int(v) for v in m.n0])
    nl = int(getattr(m, "n_oct_levels", 0) or 0)
    counts = _i64p()
    fc = ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))()
    if nl > 0:
        cnt = np.ascontiguousarray(np.asarray(m.n_cells_per_level, dtype=np.int64))
        tabs = [np.ascontiguousarray(np.asarray(t, dtype=np.int32)) for t in m.first_child]
        ptrs = (ctypes.POINTER(ctypes.c_int32) * len(tabs))(*[_ptr(t, ctypes.c_int32) for t in tabs])
        keep.extend([cnt, tabs, ptrs])
        counts = _ptr(cnt, ctypes.c_int64)
        fc = ctypes.cast(ptrs, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)))
    return Model3DStruct(n0, nl, float(m.root_cell_cm), counts, fc,
                         *[_ptr(a, ctypes.c_float) for a in arrs])


def model_footprint(model, n_levels, n_trans, n_channels, dirs=None, fp64=False, oct_steps=0):
    """Device bytes a context holds for a model (miloc_model_footprint):
    (fixed, sums of one launch's transition)."""
    L = load_library()
    keep = []
    m1 = m3 = None
    if hasattr(model, "r_out"):
        m1 = _model1d_struct(model, keep)
    else:
        m3 = _model3d_struct(model, keep)
    d = None if dirs is None else _f64(dirs).reshape(-1, 3)
    fixed, sums = ctypes.c_size_t(0), ctypes.c_size_t(0)
    rc = L.miloc_model_footprint(ctypes.byref(m1) if m1 else None, ctypes.byref(m3) if m3 else None,
                                 int(n_levels), int(n_trans), int(n_channels), 0 if d is None else int(d.shape[0]),
                                 _ptr(d, ctypes.c_double), 1 if fp64 else 0, int(oct_steps),
                                 ctypes.byref(fixed), ctypes.byref(sums))
    if rc != OK:
        raise MilocError(rc, "miloc_model_footprint failed")
    return fixed.value, sums.value


def octree_schedule(model, dirs, plain=False, lattice=False):
    """Host-built ray schedule of an octree model (miloc_octree_schedule):
    (steps uint32 [n_steps, 2], trees int64 [n_trees, 4], max_depth).
    plain: root lines only, traced straight; lattice: the brute-force lattice
    of 4^Lmax straight lines per root element."""
    L = load_library()
    keep = []
    s = _model3d_struct(model, keep)
    d = _f64(dirs).reshape(-1, 3)
    ns, nt, md = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int(0)
    mode = 2 if lattice else (1 if plain else 0)
    rc = L.miloc_octree_schedule(ctypes.byref(s), int(d.shape[0]), _ptr(d, ctypes.c_double), mode,
                                 ctypes.byref(ns), ctypes.byref(nt), ctypes.byref(md), None, None)
    if rc != OK:
        raise MilocError(rc, "miloc_octree_schedule failed")
    steps = np.zeros((ns.value, 2), np.uint32)
    trees = np.zeros((nt.value, 4), np.int64)
    rc = L.miloc_octree_schedule(ctypes.byref(s), int(d.shape[0]), _ptr(d, ctypes.c_double), mode,
                                 ctypes.byref(ns), ctypes.byref(nt), ctypes.byref(md),
                                 _ptr(steps, ctypes.c_uint32), _ptr(trees, ctypes.c_int64))
    if rc != OK:
        raise MilocError(rc, "miloc_octree_schedule failed")
    return steps, trees, md.value


def solve_1d_noalloc(mol, model, spec, T_bg: float = 2.73, max_iter: int = 100, tol: float = 0.0,
                     device: int = 0, stream: Optional[int] = None):
    """miloc_solve_1d_noalloc: one 1D ALI solve whose device memory is the
    library's static scratch (no device allocation).  Returns (x [n_shells,
    n_levels], iterations, last_delta, status) with status MILOC_OK or
    MILOC_ENOTCONV; other statuses raise."""
    L = load_library()
    keep = []
    ms = _mol_struct(mol, keep)
    m1 = _model1d_struct(model, keep)
    x = np.empty((int(np.asarray(model.r_out).shape[0]), int(np.asarray(mol.E_K).shape[0])))
    it, d = ctypes.c_int(0), ctypes.c_double(0.0)
    rc = L.miloc_solve_1d_noalloc(int(device), _vp(stream) if stream else None, ctypes.byref(ms), ctypes.byref(m1),
                                  int(spec.n_channels), float(spec.v_min), float(spec.dv), float(T_bg),
                                  int(max_iter), float(tol), ctypes.byref(it), ctypes.byref(d),
                                  _ptr(x, ctypes.c_double))
    if rc not in (OK, ENOTCONV):
        raise MilocError(rc, "miloc_solve_1d_noalloc failed")
    return x, it.value, d.value, rc


class Server:
    """1D request loop with continuous batching (miloc_server_*)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 4 << 30, max_slots: int = 256):
        self._lib = load_library()
        h = _vp()
        rc = self._lib.miloc_server_create(int(device), int(hbm_budget_bytes), int(max_slots), ctypes.byref(h))
        if rc != OK:
            raise MilocError(rc, "miloc_server_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.miloc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != OK and rc not in allow:
            msg = self._lib.miloc_server_last_error(self._h)
            raise MilocError(rc, msg.decode() if msg else "")
        return rc

    def submit(self, mol, model, spec, T_bg=2.73, tol=1e-6, max_iter=500) -> int:
        keep = []
        ms = _mol_struct(mol, keep)
        md = _model1d_struct(model, keep)
        t = ctypes.c_uint64(0)
        self._check(self._lib.miloc_server_submit(self._h, ctypes.byref(ms), ctypes.byref(md),
                                                  int(spec.n_channels), float(spec.v_min), float(spec.dv),
                                                  float(T_bg), float(tol), int(max_iter), ctypes.byref(t)))
        return int(t.value)

    def footprint(self, mol, model, spec, T_bg=2.73) -> int:
        """Arena bytes the request would hold while resident."""
        keep = []
        ms = _mol_struct(mol, keep)
        md = _model1d_struct(model, keep)
        b = ctypes.c_size_t(0)
        self._check(self._lib.miloc_server_footprint(self._h, ctypes.byref(ms), ctypes.byref(md),
                                                     int(spec.n_channels), float(spec.v_min), float(spec.dv),
                                                     float(T_bg), ctypes.byref(b)))
        return int(b.value)

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int(0)
        self._check(self._lib.miloc_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int, timeout_s: float = 60.0) -> bool:
        d = ctypes.c_int(0)
        self._check(self._lib.miloc_server_wait(self._h, ctypes.c_uint64(ticket), float(timeout_s),
                                                ctypes.byref(d)))
        return bool(d.value)

    def take(self, ticket: int):
        """(x [n_shells, n_levels], centre spectra [n_trans, n_channels], info dict, status)."""
        n, L, T, nch = (ctypes.c_int(0) for _ in range(4))
        self._check(self._lib.miloc_server_result_sizes(self._h, ctypes.c_uint64(ticket), ctypes.byref(n),
                                                        ctypes.byref(L), ctypes.byref(T), ctypes.byref(nch)))
        x = np.zeros((n.value, L.value))
        sp = np.zeros((T.value, nch.value))
        info = ResultInfo()
        rc = self._lib.miloc_server_take(self._h, ctypes.c_uint64(ticket), _ptr(x, ctypes.c_double),
                                         _ptr(sp, ctypes.c_double), ctypes.byref(info))
        return x, sp, {k: getattr(info, k) for k, _ in ResultInfo._fields_}, rc

    def cancel(self, ticket: int):
        self._check(self._lib.miloc_server_cancel(self._h, ctypes.c_uint64(ticket)))

    def stats(self) -> dict:
        st = ServerStats()
        self._check(self._lib.miloc_server_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}


class Context:
    """One library context (one HIP device and stream)."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        self._lib = load_library()
        h = _vp()
        rc = self._lib.miloc_create(int(device), _vp(stream) if stream else None, ctypes.byref(h))
        if rc != OK:
            raise MilocError(rc, "miloc_create failed (no gfx950 device?)")
        self._h = h
        self._keep = []

    def close(self):
        if getattr(self, "_h", None):
            self._lib.miloc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != OK and rc not in allow:
            msg = self._lib.miloc_last_error(self._h)
            raise MilocError(rc, msg.decode() if msg else "")
        return rc

    # -- inputs ---------------------------------------------------------
    def load_molecule(self, mol):
        E, g = _f64(mol.E_K), _f64(mol.g)
        up = np.ascontiguousarray(np.asarray(mol.up, dtype=np.int32))
        lo = np.ascontiguousarray(np.asarray(mol.lo, dtype=np.int32))
        A, nu, gd = _f64(mol.A), _f64(mol.nu), _f64(mol.gamma_down)
        s = MolStruct(int(E.shape[0]), _ptr(E, ctypes.c_double), _ptr(g, ctypes.c_double),
                      int(up.shape[0]), _ptr(up, ctypes.c_int), _ptr(lo, ctypes.c_int),
                      _ptr(A, ctypes.c_double), _ptr(nu, ctypes.c_double), _ptr(gd, ctypes.c_double),
                      float(mol.mass_amu))
        self._check(self._lib.miloc_load_molecule(self._h, ctypes.byref(s)))

    def load_model_1d(self, m):
        arrs = [_f64(a) for a in (m.r_out, m.n_H2, m.T_kin, m.b_turb, m.v_r, m.abundance)]
        imp = None if getattr(m, "impact", None) is None else _f64(m.impact)
        s = Model1DStruct(int(arrs[0].shape[0]), *[_ptr(a, ctypes.c_double) for a in arrs],
                          int(m.n_rays), _ptr(imp, ctypes.c_double))
        self._check(self._lib.miloc_load_model_1d(self._h, ctypes.byref(s)))

    def load_model_3d(self, m):
        keep = []
        s = _model3d_struct(m, keep)
        self._check(self._lib.miloc_load_model_3d(self._h, ctypes.byref(s)))

    def set_spectral(self, n_channels: int, v_min: float, dv: float):
        self._check(self._lib.miloc_set_spectral(self._h, int(n_channels), float(v_min), float(dv)))

    def set_background(self, T_bg: float):
        self._check(self._lib.miloc_set_background(self._h, float(T_bg)))

    def set_hyperfine(self, trans: int, dv_cms, strength):
        """Hyperfine components of one transition (LTE between them): velocity
        offsets [cm/s] and relative strengths; empty arrays restore the single
        Gaussian."""
        v = _f64(dv_cms).ravel()
        w = _f64(strength).ravel()
        if v.shape != w.shape:
            raise ValueError("dv_cms and strength differ in length")
        self._check(self._lib.miloc_set_hyperfine(self._h, int(trans), int(v.size),
                                                  _ptr(v, ctypes.c_double), _ptr(w, ctypes.c_double)))

    def set_octree_rays(self, lattice: bool):
        """Octree rays: the scheme's created and ended rays (False, default) or
        the brute-force lattice of 4^Lmax straight lines per root element."""
        self._check(self._lib.miloc_set_octree_rays(self._h, 1 if lattice else 0))

    def set_directions_healpix(self, nside: int):
        self._check(self._lib.miloc_set_directions_healpix(self._h, int(nside)))

    def set_directions(self, dirs):
        d = _f64(dirs).reshape(-1, 3)
        self._check(self._lib.miloc_set_directions(self._h, int(d.shape[0]), _ptr(d, ctypes.c_double)))

    def set_subiterations(self, n_sub: int, tau_min: float = 0.1):
        self._check(self._lib.miloc_set_subiterations(self._h, int(n_sub), float(tau_min)))

    def set_transition_batching(self, on: bool):
        self._check(self._lib.miloc_set_transition_batching(self._h, 1 if on else 0))

    def set_march_precision(self, fp64: bool):
        self._check(self._lib.miloc_set_march_precision(self._h, MARCH_FP64 if fp64 else MARCH_FP32))

    # -- iteration --------------------------------------------------------
    def init_lte(self):
        self._check(self._lib.miloc_init_lte(self._h))

    def set_populations(self, x):
        x = _f64(x)
        self._check(self._lib.miloc_set_populations(self._h, _ptr(x, ctypes.c_double)))

    def run(self, max_iter: int, tol: float = 0.0, use_ali: bool = True,
            allow_notconv: bool = True) -> Tuple[int, float]:
        it = ctypes.c_int(0)
        d = ctypes.c_double(0.0)
        allow = (ENOTCONV,) if allow_notconv else ()
        self._check(self._lib.miloc_run(self._h, int(max_iter), float(tol), 1 if use_ali else 0,
                                        ctypes.byref(it), ctypes.byref(d)), allow)
        return it.value, d.value

    # -- outputs ------------------------------------------------------------
    def sizes(self):
        nc = ctypes.c_int64(0)
        L, T, nch = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        self._check(self._lib.miloc_get_sizes(self._h, ctypes.byref(nc), ctypes.byref(L),
                                              ctypes.byref(T), ctypes.byref(nch)))
        return nc.value, L.value, T.value, nch.value

    def populations(self) -> np.ndarray:
        nc, L, _, _ = self.sizes()
        x = np.empty((nc, L))
        self._check(self._lib.miloc_get_populations(self._h, _ptr(x, ctypes.c_double)))
        return x

    def radiation(self):
        nc, _, T, _ = self.sizes()
        J = np.empty((T, nc))
        Lam = np.empty((T, nc))
        self._check(self._lib.miloc_get_radiation(self._h, _ptr(J, ctypes.c_double),
                                                  _ptr(Lam, ctypes.c_double)))
        return J, Lam

    def spectra(self, trans: int, impact=None, n_los: Optional[int] = None) -> np.ndarray:
        _, _, _, nch = self.sizes()
        imp = None if impact is None else _f64(impact)
        if n_los is None:
            if imp is None:
                raise ValueError("n_los is required without impact parameters")
            n_los = imp.shape[0]
        out = np.empty((int(n_los), nch))
        self._check(self._lib.miloc_get_spectra(self._h, int(trans), int(n_los),
                                                _ptr(imp, ctypes.c_double), _ptr(out, ctypes.c_double)))
        return out

    def counters(self) -> dict:
        c = Counters()
        self._check(self._lib.miloc_get_counters(self._h, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in Counters._fields_}

    def reset_counters(self):
        self._check(self._lib.miloc_reset_counters(self._h))


def version() -> str:
    return load_library().miloc_version().decode()
