"""ctypes marshalling for libmx.so: argument conversion only, no arithmetic of the method."""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmx.so")

MX_OK = 0
_CODES = {0: "MX_OK", -1: "MX_EINVAL", -2: "MX_ENOMEM", -3: "MX_EHIP", -4: "MX_ENOCONV",
          -5: "MX_EBS", -6: "MX_ENONFINITE", -7: "MX_ECAPACITY"}


class MxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
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
    """mx_planet: time-dependent physics of one massive body."""
    _fields_ = [(f, C.c_double) for f in
                ("M0", "Mc", "tau_c", "Mf", "tau_g", "R_I", "da1", "tau1", "da2", "tau2", "gap_C")]


# fields a parameter dict may leave out (the disk physics beyond the plain drag is off)
_OPTIONAL = {"temp_1au": 0.0, "temp_beta": 0.0, "cs2_per_k": 0.0, "eta_mode": 0, "dg_mode": 0}


def make_params(p: dict) -> Params:
    q = Params()
    for name, _ in Params._fields_:
        if name != "pad":
            setattr(q, name, p[name] if name in p else _OPTIONAL[name])
    return q


_lib = None
_P = C.c_void_p
_D = C.c_void_p


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Load libmx.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"HIP library not built: {_LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(_LIB_PATH)
        st = C.c_int
        L.mx_last_error.restype = C.c_char_p
        L.mx_init_system.restype = st
        L.mx_init_system.argtypes = [C.POINTER(Params), _D, _D, _D, _D, _D, _D, C.c_int, _P,
                                     C.POINTER(C.c_void_p)]
        L.mx_step.restype = st
        L.mx_step.argtypes = [_P, C.c_int32]
        L.mx_step_profiled.restype = st
        L.mx_step_profiled.argtypes = [_P, C.c_int32, C.POINTER(C.c_double)]
        L.mx_set_launch_mode.restype = st
        L.mx_set_launch_mode.argtypes = [_P, C.c_int32]
        L.mx_step_timed.restype = st
        L.mx_step_timed.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32,
                                    C.POINTER(C.c_float), C.POINTER(C.c_int32)]
        L.mx_get_counters.restype = st
        L.mx_get_counters.argtypes = [_P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.mx_sync.restype = st
        L.mx_sync.argtypes = [_P]
        L.mx_energy.restype = st
        L.mx_energy.argtypes = [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.mx_encounters.restype = st
        L.mx_encounters.argtypes = [_P, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]
        for name in ("mx_get_state", "mx_get_state_dh"):
            f = getattr(L, name)
            f.restype = st
            f.argtypes = [_P, _D, _D, C.c_int]
        for name in ("mx_set_state", "mx_set_state_dh"):
            f = getattr(L, name)
            f.restype = st
            f.argtypes = [_P, _D, _D, C.c_int, C.c_int64]
        L.mx_get_accel.restype = st
        L.mx_get_accel.argtypes = [_P, _D, C.c_int]
        L.mx_get_masses.restype = st
        L.mx_get_masses.argtypes = [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.mx_get_step_index.restype = st
        L.mx_get_step_index.argtypes = [_P, C.POINTER(C.c_int64)]
        L.mx_destroy.restype = None
        L.mx_destroy.argtypes = [_P]
        L.mx_gravity.restype = st
        L.mx_gravity.argtypes = [C.c_int32, C.c_int32, _D, _D, _D, _D, _P]
        L.mx_gas_drag.restype = st
        L.mx_gas_drag.argtypes = [C.POINTER(Params), C.c_int32, C.c_int32, _D, _D, _D, _D, _D, _D,
                                  _P]
        L.mx_kepler_drift.restype = st
        L.mx_kepler_drift.argtypes = [C.c_int32, C.c_double, C.c_double, _D, _D, _D, _D, _P]
        L.mx_init_batch.restype = st
        L.mx_init_batch.argtypes = [C.c_int32, C.POINTER(Params), C.POINTER(C.c_int64), _D, _D,
                                    _D, _D, _D, C.c_int, _P, C.POINTER(C.c_void_p)]
        L.mx_step_batch.restype = st
        L.mx_step_batch.argtypes = [_P, C.c_int32]
        L.mx_batch_set_launch_mode.restype = st
        L.mx_batch_set_launch_mode.argtypes = [_P, C.c_int32, C.c_int32]
        L.mx_batch_set_config.restype = st
        L.mx_batch_set_config.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32]
        L.mx_batch_get_config.restype = st
        L.mx_batch_get_config.argtypes = [_P, C.POINTER(C.c_int32)]
        L.mx_batch_autotune.restype = st
        L.mx_batch_autotune.argtypes = [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_float)]
        L.mx_batch_sync.restype = st
        L.mx_batch_sync.argtypes = [_P]
        L.mx_batch_system.restype = st
        L.mx_batch_system.argtypes = [_P, C.c_int32, C.POINTER(C.c_void_p)]
        L.mx_destroy_batch.argtypes = [_P]
        L.mx_adjoint_create.restype = st
        L.mx_adjoint_create.argtypes = [C.POINTER(Params), _D, _D, _D, _D, _D, _D, C.c_int32,
                                        C.c_int32, C.c_int, _P, C.POINTER(C.c_void_p)]
        L.mx_adjoint_forward.restype = st
        L.mx_adjoint_forward.argtypes = [_P, _D, _D, C.c_int]
        L.mx_adjoint_backward.restype = st
        L.mx_adjoint_backward.argtypes = [_P, _D, _D, _D, _D, _D, C.c_int]
        L.mx_adjoint_system.restype = st
        L.mx_adjoint_system.argtypes = [_P, C.POINTER(C.c_void_p)]
        L.mx_destroy_adjoint.argtypes = [_P]
        L.mx_set_planet_physics.restype = st
        L.mx_set_planet_physics.argtypes = [_P, C.POINTER(Planet), C.c_double, C.c_double]
        L.mx_get_planet_radii.restype = st
        L.mx_get_planet_radii.argtypes = [_P, _D]
        L.mx_get_time.restype = st
        L.mx_get_time.argtypes = [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.mx_check_removal.restype = st
        L.mx_check_removal.argtypes = [_P, C.c_double, C.POINTER(C.c_int32)]
        L.mx_compact.restype = st
        L.mx_compact.argtypes = [_P, C.POINTER(C.c_int32), _D]
        L.mx_get_status.restype = st
        L.mx_get_status.argtypes = [_P, _D]
        L.mx_get_counts.restype = st
        L.mx_get_counts.argtypes = [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.mx_flag_pairs.restype = st
        L.mx_flag_pairs.argtypes = [C.c_int32, C.c_int32, _D, _D, _D, _D, _D, C.c_double, _D,
                                    C.c_int32, C.POINTER(C.c_int32), _P]
        L.mx_flag_pairs_noalloc.restype = st
        L.mx_flag_pairs_noalloc.argtypes = [C.c_int32, C.c_int32, _D, _D, _D, _D, _D, C.c_double,
                                            _D, C.c_int32, C.POINTER(C.c_int32), _P]
        _lib = L
    return _lib


def _check(code: int):
    if code != MX_OK:
        raise MxError(code, lib().mx_last_error().decode())


def _torch():
    import torch
    return torch


def _dev(a, device="cuda"):
    """float64 contiguous device tensor (copy of a numpy array or tensor)."""
    torch = _torch()
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.detach().to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class System:
    """One planetary system on the GPU (owns an mx_system and a dedicated stream)."""

    def __init__(self, params: dict, x, v, m_big, r_p=None, rho_p=None, growth=None,
                 device="cuda"):
        torch = _torch()
        self.params = dict(params)
        self.n = int(params["n_big"]) + int(params["n_small"])
        self.nb = int(params["n_big"])
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        tx, tv, tm = _dev(x, device), _dev(v, device), _dev(m_big, device)
        if tm is None or tm.numel() == 0:
            tm = torch.zeros(1, dtype=torch.float64, device=device)
        trp, trh, tg = _dev(r_p, device), _dev(rho_p, device), _dev(growth, device)
        torch.cuda.current_stream(self.device).synchronize()
        self._pp = make_params(params)
        h = C.c_void_p()
        _check(lib().mx_init_system(C.byref(self._pp), _ptr(tx), _ptr(tv), _ptr(tm), _ptr(trp),
                                    _ptr(trh), _ptr(tg), 1, C.c_void_p(self.stream.cuda_stream),
                                    C.byref(h)))
        self._h = h

    @classmethod
    def from_workload(cls, w, device="cuda"):
        return cls(w.params, w.x, w.v, w.m_big, w.r_p, w.rho_p, w.growth, device=device)

    @classmethod
    def _view(cls, handle, params, device, stream, owner):
        """A system owned by a batch (closing the view does not free it)."""
        torch = _torch()
        obj = cls.__new__(cls)
        obj.params = dict(params)
        obj.n = int(params["n_big"]) + int(params["n_small"])
        obj.nb = int(params["n_big"])
        obj.device = torch.device(device)
        obj.stream = stream
        obj._h = handle
        obj._owner = owner  # keeps the batch alive while the view exists
        return obj

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self, "_owner", None) is None:
                lib().mx_destroy(self._h)
            self._h = None  # a view only lets go of the batch member

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1, sync=False):
        _check(lib().mx_step(self._h, int(n)))
        if sync:
            self.sync()

    KERNELS = ("growth", "kick_jump_drift", "flag", "plan", "bs", "jump_pack", "force_kick")

    def step_profiled(self, n=1):
        """Eager steps with HIP events around each kernel group; returns {name: ms total}."""
        ms = (C.c_double * len(self.KERNELS))()
        _check(lib().mx_step_profiled(self._h, int(n), ms))
        return dict(zip(self.KERNELS, ms[:]))

    def set_launch_mode(self, mode):
        """'eager' (default) or 'graph' (one captured HIP graph per step)."""
        _check(lib().mx_set_launch_mode(self._h, {"eager": 0, "graph": 1}[mode]))

    def step_timed(self, n, group, stride=1):
        """n eager steps; HIP events bound to the kernels of `group` (a name of
        KERNELS, "step_joined": the launch joining two steps, or "step_joint":
        the launch integrating one step's encounters beside the closing of that
        step and the opening of the next) in every `stride`-th step.  Returns
        (per-step group milliseconds as a list, 0 for untimed steps; timed steps
        where the group launched)."""
        extra = {"step_joined": len(self.KERNELS), "step_joint": len(self.KERNELS) + 1}
        g = extra[group] if group in extra else self.KERNELS.index(group)
        ms = (C.c_float * max(int(n), 1))()
        nl = C.c_int32(0)
        _check(lib().mx_step_timed(self._h, int(n), g, int(stride), ms, C.byref(nl)))
        return list(ms[: int(n)]), nl.value

    def counters(self):
        """(model FP64 ops of the encounter integrator, flagged pairs), cumulative."""
        a = C.c_uint64(0)
        b = C.c_uint64(0)
        _check(lib().mx_get_counters(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def sync(self):
        _check(lib().mx_sync(self._h))

    def energy(self):
        E = C.c_double(0)
        L = (C.c_double * 3)()
        _check(lib().mx_energy(self._h, C.byref(E), L))
        return E.value, np.array(L[:])

    def encounters(self, cap=1 << 16):
        buf = (C.c_int32 * (2 * cap))()
        n = C.c_int32(0)
        _check(lib().mx_encounters(self._h, buf, cap, C.byref(n)))
        k = min(n.value, cap)
        return np.frombuffer(buf, dtype=np.int32, count=2 * k).reshape(-1, 2).copy()

    def _pair_out(self, fn):
        torch = _torch()
        a = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        b = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        _check(fn(self._h, _ptr(a), _ptr(b), 1))
        return a, b

    def get_state(self, numpy=True):
        a, b = self._pair_out(lib().mx_get_state)
        return (a.cpu().numpy(), b.cpu().numpy()) if numpy else (a, b)

    def get_dh(self, numpy=True):
        a, b = self._pair_out(lib().mx_get_state_dh)
        return (a.cpu().numpy(), b.cpu().numpy()) if numpy else (a, b)

    def _set(self, fn, x, u, step_index):
        torch = _torch()
        tx, tu = _dev(x, self.device), _dev(u, self.device)
        torch.cuda.current_stream(self.device).synchronize()
        _check(fn(self._h, _ptr(tx), _ptr(tu), 1, int(step_index)))

    def set_state(self, x, v, step_index=0):
        self._set(lib().mx_set_state, x, v, step_index)

    def set_dh(self, x, u, step_index=0):
        self._set(lib().mx_set_state_dh, x, u, step_index)

    def accel(self, numpy=True):
        torch = _torch()
        a = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        _check(lib().mx_get_accel(self._h, _ptr(a), 1))
        return a.cpu().numpy() if numpy else a

    def masses(self):
        k = max(self.nb, 1)
        mu = (C.c_double * k)()
        rc = (C.c_double * k)()
        _check(lib().mx_get_masses(self._h, mu, rc))
        return np.array(mu[: self.nb]), np.array(rc[: self.nb])

    def set_planet_physics(self, planets, a_switch=0.0, a_min=0.0):
        """planets: one dict per massive body with the Planet fields (missing = 0)."""
        arr = (Planet * len(planets))()
        for k, r in enumerate(planets):
            for f, _ in Planet._fields_:
                setattr(arr[k], f, float(r.get(f, 0.0)))
        _check(lib().mx_set_planet_physics(self._h, arr, float(a_switch), float(a_min)))

    def check_removal(self, r_cen=0.0):
        """Ejection and central-body flags (statuses -3, -2); returns ejcount."""
        k = C.c_int32(0)
        _check(lib().mx_check_removal(self._h, float(r_cen), C.byref(k)))
        return k.value

    def status(self):
        st = np.zeros(self.n, dtype=np.int32)
        _check(lib().mx_get_status(self._h, st.ctypes.data_as(C.c_void_p)))
        return st

    def compact(self):
        """Remove the flagged massless bodies; returns (number removed, index map)."""
        mp = np.zeros(self.n, dtype=np.int32)
        k = C.c_int32(0)
        _check(lib().mx_compact(self._h, C.byref(k), mp.ctypes.data_as(C.c_void_p)))
        nb, ns = C.c_int32(0), C.c_int32(0)
        _check(lib().mx_get_counts(self._h, C.byref(nb), C.byref(ns)))
        self.n = nb.value + ns.value
        self.params["n_small"] = ns.value
        return k.value, mp

    def radii(self):
        k = max(self.nb, 1)
        r = (C.c_double * k)()
        _check(lib().mx_get_planet_radii(self._h, r))
        return np.array(r[: self.nb])

    def time(self):
        """(time at the start of the next step, current step size)."""
        t, h = C.c_double(0), C.c_double(0)
        _check(lib().mx_get_time(self._h, C.byref(t), C.byref(h)))
        return t.value, h.value

    def step_index(self):
        v = C.c_int64(0)
        _check(lib().mx_get_step_index(self._h, C.byref(v)))
        return v.value


class Batch:
    """Independent systems stepped together (every system needs n_big <= 64)."""

    def __init__(self, params_list, xs, vs, m_bigs, r_ps=None, rho_ps=None, device="cuda"):
        torch = _torch()
        k = len(params_list)
        self.params = [dict(p) for p in params_list]
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        sizes = [int(p["n_big"]) + int(p["n_small"]) for p in self.params]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        tx = _dev(np.hstack([np.asarray(x, dtype=np.float64) for x in xs]), device)
        tv = _dev(np.hstack([np.asarray(v, dtype=np.float64) for v in vs]), device)
        mb = [np.asarray(m, dtype=np.float64).reshape(-1) for m in m_bigs]
        tm = _dev(np.concatenate(mb) if sum(len(m) for m in mb) else np.zeros(1), device)
        trp = trh = None
        if r_ps is not None and any(r is not None for r in r_ps):
            rp = [np.asarray(r if r is not None else np.zeros(int(p["n_small"])), dtype=np.float64)
                  for r, p in zip(r_ps, self.params)]
            rh = [np.asarray(r if r is not None else np.ones(int(p["n_small"])), dtype=np.float64)
                  for r, p in zip(rho_ps, self.params)]
            trp, trh = _dev(np.concatenate(rp), device), _dev(np.concatenate(rh), device)
        torch.cuda.current_stream(self.device).synchronize()
        self._pp = (Params * k)(*[make_params(p) for p in self.params])
        offs = (C.c_int64 * (k + 1))(*[int(o) for o in self.offsets])
        h = C.c_void_p()
        _check(lib().mx_init_batch(k, self._pp, offs, _ptr(tx), _ptr(tv), _ptr(tm), _ptr(trp),
                                   _ptr(trh), 1, C.c_void_p(self.stream.cuda_stream),
                                   C.byref(h)))
        self._h = h
        self.n_sys = k
        self._views = weakref.WeakSet()

    @classmethod
    def from_workloads(cls, ws, device="cuda"):
        return cls([w.params for w in ws], [w.x for w in ws], [w.v for w in ws],
                   [w.m_big for w in ws], [w.r_p for w in ws], [w.rho_p for w in ws],
                   device=device)

    def close(self):
        if getattr(self, "_h", None):
            for v in list(self._views):
                v._h = None  # views of destroyed members become unusable
            lib().mx_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1, sync=False):
        _check(lib().mx_step_batch(self._h, int(n)))
        if sync:
            self.sync()

    def sync(self):
        _check(lib().mx_batch_sync(self._h))

    def set_launch_mode(self, mode, steps_per_graph=1):
        _check(lib().mx_batch_set_launch_mode(self._h, {"eager": 0, "graph": 1}[mode],
                                              int(steps_per_graph)))

    def set_config(self, blk, tiles_per_block, bs_blocks):
        _check(lib().mx_batch_set_config(self._h, int(blk), int(tiles_per_block), int(bs_blocks)))

    def config(self):
        cfg = (C.c_int32 * 3)()
        _check(lib().mx_batch_get_config(self._h, cfg))
        return tuple(cfg[:])

    def autotune(self, steps_per_candidate=3):
        """Returns (steps taken, (blk, tiles_per_block, bs_blocks), best ms per step)."""
        taken = C.c_int32(0)
        cfg = (C.c_int32 * 3)()
        ms = C.c_float(0)
        _check(lib().mx_batch_autotune(self._h, int(steps_per_candidate), C.byref(taken), cfg,
                                       C.byref(ms)))
        return taken.value, tuple(cfg[:]), ms.value

    def system(self, k):
        h = C.c_void_p()
        _check(lib().mx_batch_system(self._h, int(k), C.byref(h)))
        v = System._view(h, self.params[k], self.device, self.stream, self)
        self._views.add(v)
        return v


class Adjoint:
    """n_steps hybrid steps of one system (n_big <= 64) with checkpoints every
    `checkpoint_every` steps, and the reverse-mode adjoint of the run: gradients
    of a function of the final heliocentric state with respect to the masses and
    the initial heliocentric state.  The changeover radii are held fixed (given,
    or from the Hill rule at the initial state)."""

    def __init__(self, params, x, v, m_big, r_p=None, rho_p=None, n_steps=1,
                 checkpoint_every=50, rcrit=None, device="cuda"):
        torch = _torch()
        self.params = dict(params)
        self.nb = int(params["n_big"])
        self.n = self.nb + int(params["n_small"])
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        tx, tv, tm = _dev(x, device), _dev(v, device), _dev(m_big, device)
        if tm is None or tm.numel() == 0:
            tm = torch.zeros(1, dtype=torch.float64, device=device)
        trp, trh, trc = _dev(r_p, device), _dev(rho_p, device), _dev(rcrit, device)
        torch.cuda.current_stream(self.device).synchronize()
        self._pp = make_params(params)
        h = C.c_void_p()
        _check(lib().mx_adjoint_create(C.byref(self._pp), _ptr(tx), _ptr(tv), _ptr(tm), _ptr(trp),
                                       _ptr(trh), _ptr(trc), int(n_steps), int(checkpoint_every),
                                       1, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().mx_destroy_adjoint(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self):
        """Final heliocentric (x, v), device tensors [3, n]."""
        torch = _torch()
        x = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        v = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().mx_adjoint_forward(self._h, _ptr(x), _ptr(v), 1))
        return x, v

    def backward(self, gx, gv):
        """(dL/dm [n_big], dL/dx0 [3, n], dL/dv0 [3, n]) from dL/dx, dL/dv of the
        final heliocentric state."""
        torch = _torch()
        tgx, tgv = _dev(gx, self.device), _dev(gv, self.device)
        gm = torch.zeros(max(self.nb, 1), dtype=torch.float64, device=self.device)
        g_x = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        g_v = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().mx_adjoint_backward(self._h, _ptr(tgx), _ptr(tgv), _ptr(gm), _ptr(g_x),
                                         _ptr(g_v), 1))
        return gm[: self.nb], g_x, g_v

    def rcrit(self):
        h = C.c_void_p()
        _check(lib().mx_adjoint_system(self._h, C.byref(h)))
        k = max(self.nb, 1)
        mu = (C.c_double * k)()
        rc = (C.c_double * k)()
        _check(lib().mx_get_masses(h, mu, rc))
        return np.array(rc[: self.nb])


def _hybrid_function():
    torch = _torch()

    class HybridRun(torch.autograd.Function):
        """(m_big, x_big, v_big) -> final heliocentric (x, v) of every body after the
        spec's n_steps hybrid steps; backward runs the adjoint of the library."""

        @staticmethod
        def forward(ctx, m_big, x_big, v_big, spec):
            nb = int(spec["params"]["n_big"])
            x = torch.as_tensor(np.asarray(spec["x"], dtype=np.float64)).clone()
            v = torch.as_tensor(np.asarray(spec["v"], dtype=np.float64)).clone()
            x[:, :nb] = x_big.detach().cpu()
            v[:, :nb] = v_big.detach().cpu()
            rcrit = spec.get("rcrit")
            if rcrit is None:
                # the changeover radii are constants of the differentiated map: taken
                # from the undifferentiated base state, never from the inputs
                if "m_big" not in spec:
                    raise ValueError("spec needs 'rcrit' (changeover radii [n_big]) or "
                                     "'m_big' (the base masses they are computed from with "
                                     "the base state spec['x'], spec['v'])")
                base = Adjoint(spec["params"], spec["x"], spec["v"], spec["m_big"],
                               spec.get("r_p"), spec.get("rho_p"), 1, 1, device=m_big.device)
                rcrit = base.rcrit()
                base.close()
            adj = Adjoint(spec["params"], x, v, m_big.detach(), spec.get("r_p"),
                          spec.get("rho_p"), spec["n_steps"], spec.get("checkpoint_every", 50),
                          rcrit, device=m_big.device)
            xf, vf = adj.forward()
            ctx.adj = adj
            ctx.nb = nb
            return xf, vf

        @staticmethod
        def backward(ctx, gx, gv):
            gm, g_x, g_v = ctx.adj.backward(gx.contiguous(), gv.contiguous())
            ctx.adj.close()
            nb = ctx.nb
            return gm, g_x[:, :nb].contiguous(), g_v[:, :nb].contiguous(), None

    return HybridRun


_HYBRID = None


def hybrid_run(m_big, x_big, v_big, spec):
    """Differentiable run: m_big [n_big], x_big, v_big [3, n_big] torch tensors (float64,
    device); spec: dict(params, x, v (all bodies, heliocentric), r_p, rho_p, n_steps,
    checkpoint_every, and rcrit or m_big).  The changeover radii are held fixed: spec's
    rcrit, else the Hill-rule radii of the base state (spec's x, v and m_big), never
    radii of the differentiated inputs.  Returns the final heliocentric (x, v) [3, n]."""
    global _HYBRID
    if _HYBRID is None:
        _HYBRID = _hybrid_function()
    return _HYBRID.apply(m_big, x_big, v_big, spec)


# ------------------------------------------------------------ single kernels
def _stream():
    torch = _torch()
    return torch.cuda.current_stream().cuda_stream


def gravity(x, mu, rcrit, nb):
    """Changeover-weighted gravity of every body from the nb massive ones."""
    torch = _torch()
    tx = _dev(x)
    n = tx.shape[1]
    tmu = _dev(mu) if nb > 0 else torch.zeros(1, dtype=torch.float64, device="cuda")
    trc = _dev(rcrit) if nb > 0 else torch.zeros(1, dtype=torch.float64, device="cuda")
    a = torch.empty((3, n), dtype=torch.float64, device="cuda")
    _check(lib().mx_gravity(n, nb, _ptr(tx), _ptr(tmu), _ptr(trc), _ptr(a), C.c_void_p(_stream())))
    torch.cuda.synchronize()
    return a


def gas_drag(params, x, u, mu, r_p, rho_p_internal, nb):
    """Gas drag of the massless bodies; rho_p_internal in Msun/AU^3."""
    torch = _torch()
    tx, tu = _dev(x), _dev(u)
    n = tx.shape[1]
    tmu = _dev(mu) if nb > 0 else torch.zeros(1, dtype=torch.float64, device="cuda")
    trp, trh = _dev(r_p), _dev(rho_p_internal)
    a = torch.empty((3, n), dtype=torch.float64, device="cuda")
    pp = make_params(params)
    _check(lib().mx_gas_drag(C.byref(pp), n, nb, _ptr(tx), _ptr(tu), _ptr(tmu), _ptr(trp),
                             _ptr(trh), _ptr(a), C.c_void_p(_stream())))
    torch.cuda.synchronize()
    return a


def kepler_drift(mu0, x0, u0, h):
    torch = _torch()
    tx, tu = _dev(x0), _dev(u0)
    n = tx.shape[1]
    x1 = torch.empty_like(tx)
    u1 = torch.empty_like(tu)
    _check(lib().mx_kepler_drift(n, float(mu0), float(h), _ptr(tx), _ptr(tu), _ptr(x1), _ptr(u1),
                                 C.c_void_p(_stream())))
    return x1, u1


def flag_pairs(nb, rcrit, x0, u0, x1, u1, h, cap=1 << 16, noalloc=False):
    """Encounter flagging of the pairs (i < nb, j > i); noalloc selects the entry point
    that takes its scratch from the library's fixed device array."""
    torch = _torch()
    tx0, tu0, tx1, tu1 = _dev(x0), _dev(u0), _dev(x1), _dev(u1)
    n = tx0.shape[1]
    trc = _dev(rcrit) if nb > 0 else torch.zeros(1, dtype=torch.float64, device="cuda")
    pairs = torch.empty(2 * cap, dtype=torch.int32, device="cuda")
    nout = C.c_int32(0)
    fn = lib().mx_flag_pairs_noalloc if noalloc else lib().mx_flag_pairs
    _check(fn(n, nb, _ptr(trc), _ptr(tx0), _ptr(tu0), _ptr(tx1), _ptr(tu1), float(h),
              _ptr(pairs), cap, C.byref(nout), C.c_void_p(_stream())))
    k = min(nout.value, cap)
    return pairs[: 2 * k].view(-1, 2).cpu().numpy()
