"""ctypes binding of the CPU oracle (TEST INFRASTRUCTURE ONLY).

The oracle is plain double-precision C (``oracle.c``) written from the paper.  Only
the test-suite, the smoke check and the benchmark's CPU-baseline leg may import this
package; the product path never does.  Nothing here is shared with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-Wno-unknown-pragmas",
          "-fPIC", "-shared"]
# the CPU-baseline builds: the same source for the host it runs on, serial and with
# OpenMP over target bodies (per-target sums in a fixed order: identical results)
CFLAGS_FAST = ["-O3", "-march=native", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-Wno-unknown-pragmas", "-fPIC", "-shared"]

OR_OK, OR_EINVAL, OR_ENOMEM, OR_ENOCONV, OR_EBS = 0, -1, -2, -4, -5


def build_lib(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no FMA contraction).  Without
    force, rebuilds only when the library is missing or older than its sources."""
    stale = (not os.path.exists(_LIB_PATH) or
             os.path.getmtime(_LIB_PATH) < max(os.path.getmtime(_SRC),
                                               os.path.getmtime(os.path.join(_HERE, "oracle.h"))))
    if force or stale:
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(C.Structure):
    _fields_ = [("G", C.c_double), ("m0", C.c_double), ("dt", C.c_double),
                ("rcrit_hill", C.c_double), ("bs_tol", C.c_double),
                ("n_big", C.c_int32), ("n_small", C.c_int32), ("gas_on", C.c_int32),
                ("pad", C.c_int32),
                ("sigma1", C.c_double), ("gamma", C.c_double), ("r_c", C.c_double),
                ("r_in", C.c_double), ("h_over_r", C.c_double), ("eta", C.c_double),
                ("kdrag_exp", C.c_double), ("rho_unit", C.c_double), ("au_cm", C.c_double),
                ("mfp_coef", C.c_double),
                ("temp_1au", C.c_double), ("temp_beta", C.c_double), ("cs2_per_k", C.c_double),
                ("eta_mode", C.c_int32), ("dg_mode", C.c_int32)]


class Planet(C.Structure):
    """Time-dependent physics of one massive body (or_planet)."""
    _fields_ = [(f, C.c_double) for f in
                ("M0", "Mc", "tau_c", "Mf", "tau_g", "R_I", "da1", "tau1", "da2", "tau2", "gap_C")]


def make_planets(rows):
    """rows: sequence of dicts with the Planet fields (missing ones 0)."""
    arr = (Planet * len(rows))()
    for k, r in enumerate(rows):
        for f, _ in Planet._fields_:
            setattr(arr[k], f, float(r.get(f, 0.0)))
    return arr


def make_params(p: dict) -> _Params:
    q = _Params()
    for name, _ in _Params._fields_:
        if name == "pad":
            continue
        setattr(q, name, p.get(name, 0))
    return q


def build_variant(path: str, openmp: bool) -> str:
    """Compile oracle.c with CFLAGS_FAST (plus -fopenmp) into path; for timing the
    oracle on the host that runs it."""
    flags = CFLAGS_FAST + (["-fopenmp"] if openmp else [])
    subprocess.check_call(["gcc", *flags, "-o", path, _SRC, "-lm"])
    return path


_lib = None
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)


def load(path: str):
    """Load an oracle library and declare its functions."""
    L = C.CDLL(path)
    _declare(L)
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib()
        _lib = load(_LIB_PATH)
    return _lib


def _declare(L):
    L.or_create.restype = C.c_void_p
    L.or_create.argtypes = [C.POINTER(_Params), _D, _D, _D, _D, _D, _D, C.POINTER(C.c_int)]
    L.or_destroy.argtypes = [C.c_void_p]
    L.or_step.argtypes = [C.c_void_p, C.c_int]
    L.or_energy.argtypes = [C.c_void_p, _D, _D]
    L.or_encounters.argtypes = [C.c_void_p, _I32, C.c_int]
    L.or_get_state.argtypes = [C.c_void_p, _D, _D]
    L.or_get_dh.argtypes = [C.c_void_p, _D, _D]
    L.or_set_dh.argtypes = [C.c_void_p, _D, _D, C.c_long]
    L.or_get_accel.argtypes = [C.c_void_p, _D]
    L.or_get_mu.argtypes = [C.c_void_p, _D, _D]
    L.or_set_rcrit.argtypes = [C.c_void_p, _D]
    L.or_step_index.restype = C.c_long
    L.or_step_index.argtypes = [C.c_void_p]
    L.or_changeover.restype = C.c_double
    L.or_changeover.argtypes = [C.c_double, C.c_double]
    L.or_gravity.argtypes = [C.c_int, C.c_int, _D, _D, _D, _D]
    L.or_drag.argtypes = [C.POINTER(_Params), C.c_int, C.c_int, _D, _D, _D, _D, _D, _D]
    L.or_drag_cd.restype = C.c_double
    L.or_drag_cd.argtypes = [C.c_double, C.c_double, C.c_double]
    L.or_drift.argtypes = [C.c_double, _D, _D, C.c_double, _D, _D]
    L.or_pair_dmin2.restype = C.c_double
    L.or_pair_dmin2.argtypes = [_D, _D, _D, _D, C.c_double]
    L.or_flag.argtypes = [C.c_int, C.c_int, _D, _D, _D, _D, _D, C.c_double, _I32, C.c_int,
                          C.POINTER(C.c_int)]
    L.or_bs.argtypes = [C.c_int, _D, _D, C.c_int, _I32, C.c_double, C.c_double, C.c_double,
                        _D, _D]
    L.or_x2el.argtypes = [C.c_double, _D, _D, _D]
    L.or_dg_series.restype = C.c_double
    L.or_dg_series.argtypes = [C.c_double]
    L.or_disk_gravity.restype = C.c_double
    L.or_disk_gravity.argtypes = [C.POINTER(_Params), C.c_double]
    L.or_gas_sigma.restype = C.c_double
    L.or_gas_sigma.argtypes = [C.POINTER(_Params), C.c_double]
    L.or_last_pair_dmin2.restype = C.c_double
    L.or_last_pair_dmin2.argtypes = [C.c_void_p, C.c_int, C.c_int, _D]
    L.or_set_physics.argtypes = [C.c_void_p, C.POINTER(Planet), C.c_double, C.c_double]
    L.or_get_radii.argtypes = [C.c_void_p, _D]
    L.or_time.restype = C.c_double
    L.or_time.argtypes = [C.c_void_p]
    L.or_step_size.restype = C.c_double
    L.or_step_size.argtypes = [C.c_void_p]
    L.or_set_xu.argtypes = [C.c_void_p, _D, _D]
    L.or_get_gaps.argtypes = [C.c_void_p, _D]
    L.or_check_removal.restype = C.c_int
    L.or_check_removal.argtypes = [C.c_void_p, C.c_double]
    L.or_compact.restype = C.c_int
    L.or_compact.argtypes = [C.c_void_p, _I32]
    L.or_get_status.argtypes = [C.c_void_p, _I32]
    L.or_n_bodies.restype = C.c_int
    L.or_n_bodies.argtypes = [C.c_void_p]
    L.or_clone.restype = C.c_void_p
    L.or_clone.argtypes = [C.c_void_p]
    L.or_drag_gaps.argtypes = [C.POINTER(_Params), C.c_int, C.c_int, _D, _D, _D, _D, _D, _D,
                               C.POINTER(C.c_int), _D]
    L.or_threads.restype = C.c_int
    L.or_threads.argtypes = []


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(_D) if a is not None else None


class OracleSystem:
    """Whole-system oracle: create / step / energy / encounters / state."""

    def __init__(self, params: dict, x, v, m_big, r_p=None, rho_p=None, growth=None,
                 library=None):
        self._L = library if library is not None else lib()
        self.params = dict(params)
        self.n = int(params["n_big"]) + int(params["n_small"])
        self.nb = int(params["n_big"])
        x, v, m = _d(x), _d(v), _d(m_big)
        assert x.shape == (3, self.n) and v.shape == (3, self.n) and m.shape == (self.nb,)
        rp = _d(r_p) if r_p is not None else None
        rh = _d(rho_p) if rho_p is not None else None
        gr = _d(growth) if growth is not None else None
        st = C.c_int(0)
        self._pp = make_params(params)
        self._h = self._L.or_create(C.byref(self._pp), _p(x), _p(v), _p(m), _p(rp), _p(rh), _p(gr),
                                  C.byref(st))
        if not self._h:
            raise ValueError(f"oracle create failed: {st.value}")

    @classmethod
    def from_workload(cls, w):
        return cls(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, w.growth)

    def close(self):
        if getattr(self, "_h", None):
            self._L.or_destroy(self._h)
            self._h = None

    __del__ = close

    def step(self, n=1):
        st = self._L.or_step(self._h, int(n))
        if st != OR_OK:
            raise RuntimeError(f"oracle step failed: {st}")

    def energy(self):
        E = C.c_double(0)
        L = np.zeros(3)
        self._L.or_energy(self._h, C.byref(E), _p(L))
        return E.value, L

    def encounters(self):
        cap = 1 << 20
        buf = np.zeros(2 * cap, dtype=np.int32)
        k = self._L.or_encounters(self._h, buf.ctypes.data_as(_I32), cap)
        return buf[: 2 * min(k, cap)].reshape(-1, 2).copy()

    def get_state(self):
        x = np.zeros((3, self.n)); v = np.zeros((3, self.n))
        self._L.or_get_state(self._h, _p(x), _p(v))
        return x, v

    def get_dh(self):
        x = np.zeros((3, self.n)); u = np.zeros((3, self.n))
        self._L.or_get_dh(self._h, _p(x), _p(u))
        return x, u

    def set_dh(self, x, u, step_index=0):
        x, u = _d(x), _d(u)
        self._L.or_set_dh(self._h, _p(x), _p(u), int(step_index))

    def accel(self):
        a = np.zeros((3, self.n))
        self._L.or_get_accel(self._h, _p(a))
        return a

    def mu(self):
        mu = np.zeros(max(self.nb, 1)); rc = np.zeros(max(self.nb, 1))
        self._L.or_get_mu(self._h, _p(mu), _p(rc))
        return mu[: self.nb], rc[: self.nb]

    def step_index(self):
        return self._L.or_step_index(self._h)

    def last_pair_dmin2(self, i, j):
        """(d_min^2, rc^2) of the last step's encounter test for the pair (i, j)."""
        rc2 = C.c_double(0)
        d = self._L.or_last_pair_dmin2(self._h, int(i), int(j), C.byref(rc2))
        return d, rc2.value

    def set_physics(self, planets, a_switch=0.0, a_min=0.0):
        """Growth, radius, migration and gap of every massive body (list of dicts
        with the Planet fields) and the step switch."""
        self._planets = make_planets(planets)
        st = self._L.or_set_physics(self._h, self._planets, float(a_switch), float(a_min))
        if st != OR_OK:
            raise ValueError(f"oracle set_physics failed: {st}")

    def radii(self):
        r = np.zeros(max(self.nb, 1))
        self._L.or_get_radii(self._h, _p(r))
        return r[: self.nb]

    def time(self):
        return self._L.or_time(self._h)

    def step_size(self):
        return self._L.or_step_size(self._h)

    def check_removal(self, r_cen=0.0):
        """Ejection (e >= 1) and central-body encounter flags; returns ejcount."""
        k = self._L.or_check_removal(self._h, float(r_cen))
        if k < 0:
            raise RuntimeError(f"oracle check_removal failed: {k}")
        return k

    def status(self):
        st = np.zeros(self.n, dtype=np.int32)
        self._L.or_get_status(self._h, st.ctypes.data_as(_I32))
        return st

    def compact(self):
        """Remove the flagged massless bodies; returns (number removed, index map)."""
        mp = np.zeros(self.n, dtype=np.int32)
        k = self._L.or_compact(self._h, mp.ctypes.data_as(_I32))
        self.n = self._L.or_n_bodies(self._h)
        self.params["n_small"] = self.n - self.nb
        return k, mp

    def clone(self):
        """A deep copy (state, masses, clock, physics state)."""
        c = OracleSystem.__new__(OracleSystem)
        c._L, c.params, c.n, c.nb = self._L, dict(self.params), self.n, self.nb
        c._pp = self._pp
        c._planets = getattr(self, "_planets", None)
        c._h = self._L.or_clone(self._h)
        if not c._h:
            raise MemoryError("oracle clone failed")
        return c

    def gaps(self):
        """[nb, 4]: centre R, half width, density factor, open (1/0) of each gap."""
        g = np.zeros(4 * max(self.nb, 1))
        self._L.or_get_gaps(self._h, _p(g))
        return g[: 4 * self.nb].reshape(-1, 4)

    def set_xu(self, x, u):
        """Replace positions and velocities only (time and physics state kept)."""
        x, u = _d(x), _d(u)
        self._L.or_set_xu(self._h, _p(x), _p(u))

    def set_rcrit(self, rcrit):
        """Hold the changeover radii at the given values (FSAL force refreshed)."""
        rc = _d(rcrit)
        assert rc.shape == (self.nb,)
        self._L.or_set_rcrit(self._h, _p(rc))


# ------------------------------------------------------------ components
def changeover(s, rc):
    return lib().or_changeover(float(s), float(rc))


def gravity(x, mu, rcrit, nb):
    x = _d(x); mu = _d(mu); rc = _d(rcrit)
    n = x.shape[1]
    a = np.zeros((3, n))
    lib().or_gravity(n, nb, _p(x), _p(mu), _p(rc), _p(a))
    return a


def drag(params, x, u, mu, r_p, rho_p_internal, nb):
    """rho_p_internal in Msun/AU^3 (already converted)."""
    x = _d(x); u = _d(u); mu = _d(mu); rp = _d(r_p); rh = _d(rho_p_internal)
    n = x.shape[1]
    a = np.zeros((3, n))
    pp = make_params(params)
    lib().or_drag(C.byref(pp), n, nb, _p(x), _p(u), _p(mu), _p(rp), _p(rh), _p(a))
    return a


def gas_sigma(params, R):
    """Eq. 1 surface density in g cm^-2 at cylindrical radius R [AU]."""
    pp = make_params(params)
    return lib().or_gas_sigma(C.byref(pp), float(R))


def dg_series(gamma):
    """S(gamma) of the disk-gravity series (Eq. 10)."""
    return lib().or_dg_series(float(gamma))


def disk_gravity(params, R):
    """Signed radial disk-gravity acceleration at R (positive away from the star)."""
    pp = make_params(params)
    return lib().or_disk_gravity(C.byref(pp), float(R))


def drag_gaps(params, x, u, mu, r_p, rho_p_internal, nb, gaps, gap_on):
    """Gas acceleration with the density factors of open gaps (gaps [nb, 3]: centre R,
    half width, factor; gap_on [nb])."""
    x = _d(x); u = _d(u); mu = _d(mu); rp = _d(r_p); rh = _d(rho_p_internal)
    g = _d(gaps); on = np.ascontiguousarray(gap_on, dtype=np.int32)
    n = x.shape[1]
    a = np.zeros((3, n))
    pp = make_params(params)
    lib().or_drag_gaps(C.byref(pp), n, nb, _p(x), _p(u), _p(mu), _p(rp), _p(rh), _p(g),
                       on.ctypes.data_as(C.POINTER(C.c_int)), _p(a))
    return a


def drag_cd(re, ma, kexp=-2.0):
    return lib().or_drag_cd(float(re), float(ma), float(kexp))


def drift(mu0, x0, v0, h):
    x0 = _d(x0); v0 = _d(v0)
    x1 = np.zeros(3); v1 = np.zeros(3)
    st = lib().or_drift(float(mu0), _p(x0), _p(v0), float(h), _p(x1), _p(v1))
    if st != OR_OK:
        raise RuntimeError(f"oracle drift failed: {st}")
    return x1, v1


def pair_dmin2(r0, w0, r1, w1, h):
    return lib().or_pair_dmin2(_p(_d(r0)), _p(_d(w0)), _p(_d(r1)), _p(_d(w1)), float(h))


def flag(nb, rcrit, x0, u0, x1, u1, h, cap=1 << 20):
    x0, u0, x1, u1 = _d(x0), _d(u0), _d(x1), _d(u1)
    rc = _d(rcrit)
    n = x0.shape[1]
    buf = np.zeros(2 * cap, dtype=np.int32)
    npairs = C.c_int(0)
    lib().or_flag(n, nb, _p(rc), _p(x0), _p(u0), _p(x1), _p(u1), float(h),
                  buf.ctypes.data_as(_I32), cap, C.byref(npairs))
    return buf[: 2 * min(npairs.value, cap)].reshape(-1, 2).copy()


def bs(mu_m, rc_m, pairs, mu0, h, tol, xs, vs):
    """xs, vs: [m, 3]; pairs: [np, 2] local indices. Returns (status, xs, vs)."""
    mu_m = _d(mu_m); rc_m = _d(rc_m)
    xs = _d(xs).copy(); vs = _d(vs).copy()
    pl = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1))
    m = xs.shape[0]
    st = lib().or_bs(m, _p(mu_m), _p(rc_m), len(pl) // 2, pl.ctypes.data_as(_I32), float(mu0),
                     float(h), float(tol), _p(xs), _p(vs))
    return st, xs, vs


def x2el(gm, x, v):
    el = np.zeros(6)
    lib().or_x2el(float(gm), _p(_d(x)), _p(_d(v)), _p(el))
    return el
