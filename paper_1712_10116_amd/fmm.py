"""Python binding of libfmm355 (the C ABI in include/fmm355.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every step of the solve runs in the library's kernels.  Loading fails
loudly if the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm355.so")

FMM_OK, FMM_EINVAL, FMM_ENOMEM, FMM_EDEVICE, FMM_ENONFINITE, FMM_ESTALE, FMM_EOVERFLOW = range(7)
WENDLAND, PLUMMER = 0, 1
FP64, MIXED = 0, 1

EXPORTED = (
    "fmm_create", "fmm_destroy", "fmm_last_error", "fmm_build", "fmm_evaluate", "fmm_forces",
    "fmm_tree_info", "fmm_export_tree", "fmm_invariants", "hhs_init", "hhs_step",
    "fmm_profile_enable", "fmm_profile_read", "fmm_build_batched", "fmm_evaluate_batched",
    "fmm_forces_batched", "hhs_run_bytes", "hhs_run_create", "hhs_run_destroy",
    "hhs_init_batched", "hhs_step_batched", "serve_footprint", "serve_create", "serve_destroy",
    "serve_submit", "serve_step", "serve_poll", "serve_cancel", "serve_info",
    "fmm_set_small_path", "fmm_set_level_prediction", "trad_step", "fmm_forces_grad",
    "fmm_cosmo_create", "fmm_cosmo_factors", "fmm_cosmo_destroy", "fmm_invariants_noalloc",
    "fmm_evaluate_dipole", "chin_work_bytes", "chin_init", "chin_step",
)
PHASES = ("sort", "tree", "walk", "upward", "m2l", "p2p", "downward")


class FMMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fmm status {status}: {msg}")
        self.status = status


class ServeParams(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int),
                ("dt_max", ctypes.c_double)]


class ServeRequest(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("vel", ctypes.c_void_p), ("mass", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("t_end", ctypes.c_double), ("pos_out", ctypes.c_void_p),
                ("vel_out", ctypes.c_void_p)]


class ServeResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("n", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("force_calls", ctypes.c_int64), ("force_particles", ctypes.c_int64),
                ("dt_top", ctypes.c_double), ("t_end", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("p_max", ctypes.c_int), ("leaf_size", ctypes.c_int), ("kernel", ctypes.c_int),
                ("precision", ctypes.c_int)]


class Request(ctypes.Structure):
    """One independent system of a batched solve (fmm_request)."""
    _fields_ = [("pos", ctypes.c_void_p), ("n_total", ctypes.c_int64), ("active", ctypes.c_void_p),
                ("n_active", ctypes.c_int64), ("mass", ctypes.c_void_p), ("acc", ctypes.c_void_p),
                ("pot", ctypes.c_void_p), ("sinks", ctypes.c_void_p)]


class HHSState(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("vel", ctypes.c_void_p), ("mass", ctypes.c_void_p),
                ("a_old", ctypes.c_void_p), ("a_cur", ctypes.c_void_p), ("rung", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("t", ctypes.c_double), ("a_tot", ctypes.c_void_p)]


class ChinState(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("vel", ctypes.c_void_p), ("mass", ctypes.c_void_p),
                ("acc", ctypes.c_void_p), ("work", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("t", ctypes.c_double)]


class CosmoParams(ctypes.Structure):
    _fields_ = [("omega_m", ctypes.c_double), ("omega_l", ctypes.c_double),
                ("h0", ctypes.c_double), ("a_min", ctypes.c_double), ("a_max", ctypes.c_double),
                ("n", ctypes.c_int)]


class Cosmology:
    """Lookup table of the comoving drift and kick factors (fmm_cosmo_*)."""

    def __init__(self, *, omega_m, omega_l, h0, a_min, a_max, n=1024):
        self.params = CosmoParams(float(omega_m), float(omega_l), float(h0), float(a_min),
                                  float(a_max), int(n))
        h = ctypes.c_void_p()
        st = lib().fmm_cosmo_create(ctypes.byref(self.params), ctypes.byref(h))
        if st != FMM_OK:
            raise FMMError(st, "cosmology table rejected its parameters")
        self._h = h

    def factors(self, a0, a1):
        """(integral of dt/a^2, integral of dt/a) from a0 to a1."""
        d, k = ctypes.c_double(), ctypes.c_double()
        st = lib().fmm_cosmo_factors(self._h, float(a0), float(a1), ctypes.byref(d),
                                     ctypes.byref(k))
        if st != FMM_OK:
            raise FMMError(st, "scale factor outside the table")
        return d.value, k.value

    def close(self):
        if self._h:
            lib().fmm_cosmo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HHSParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("theta", ctypes.c_double), ("p", ctypes.c_int),
                ("eta", ctypes.c_double), ("max_levels", ctypes.c_int),
                ("freeze_rungs", ctypes.c_int), ("eta1", ctypes.c_double),
                ("cosmo", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libfmm355.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        L.fmm_create.argtypes = [ctypes.POINTER(_Params), i64, vp, ctypes.POINTER(vp)]
        L.fmm_destroy.argtypes = [vp]
        L.fmm_last_error.argtypes = [vp]
        L.fmm_last_error.restype = ctypes.c_char_p
        L.fmm_build.argtypes = [vp, vp, i64, vp, i64, dbl, dbl]
        L.fmm_evaluate.argtypes = [vp, vp, vp, i64, vp, i64, ci, vp, vp]
        L.fmm_forces.argtypes = [vp, vp, vp, i64, vp, i64, dbl, dbl, ci, vp, vp]
        L.fmm_forces_grad.argtypes = [vp, vp, vp, i64, vp, i64, dbl, dbl, ci, vp, vp, vp]
        L.fmm_cosmo_create.argtypes = [ctypes.POINTER(CosmoParams), ctypes.POINTER(vp)]
        L.fmm_cosmo_factors.argtypes = [vp, dbl, dbl, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
        L.fmm_cosmo_destroy.argtypes = [vp]
        L.fmm_tree_info.argtypes = [vp, vp]
        L.fmm_export_tree.argtypes = [vp] + [vp] * 11
        L.fmm_invariants.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp]
        L.fmm_invariants_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp]
        L.fmm_evaluate_dipole.argtypes = [vp, vp, vp, i64, vp, i64, ci, vp, vp, vp]
        L.chin_work_bytes.argtypes = [i64]
        L.chin_init.argtypes = [vp, ctypes.POINTER(ChinState), dbl, dbl, ci]
        L.chin_step.argtypes = [vp, ctypes.POINTER(ChinState), dbl, dbl, ci, dbl, vp]
        L.hhs_init.argtypes = [vp, ctypes.POINTER(HHSState), ctypes.POINTER(HHSParams)]
        L.hhs_step.argtypes = [vp, ctypes.POINTER(HHSState), ctypes.POINTER(HHSParams), dbl, vp]
        L.trad_step.argtypes = [vp, ctypes.POINTER(HHSState), ctypes.POINTER(HHSParams), dbl, vp]
        L.fmm_build_batched.argtypes = [vp, ci, ctypes.POINTER(Request), dbl, dbl]
        L.fmm_evaluate_batched.argtypes = [vp, ci, ctypes.POINTER(Request), ci]
        L.fmm_forces_batched.argtypes = [vp, ci, ctypes.POINTER(Request), dbl, dbl, ci]
        L.fmm_set_small_path.argtypes = [vp, ci]
        L.fmm_set_level_prediction.argtypes = [vp, ci]
        L.fmm_profile_enable.argtypes = [vp, ci]
        L.fmm_profile_read.argtypes = [vp, vp, vp]
        L.hhs_run_bytes.argtypes = [i64, ci]
        L.hhs_run_create.argtypes = [vp, i64, ci, ctypes.POINTER(vp)]
        L.hhs_run_destroy.argtypes = [vp]
        L.hhs_init_batched.argtypes = [vp, ci, ctypes.POINTER(vp),
                                       ctypes.POINTER(ctypes.POINTER(HHSState)),
                                       ctypes.POINTER(HHSParams)]
        L.hhs_step_batched.argtypes = [vp, ci, ctypes.POINTER(vp),
                                       ctypes.POINTER(ctypes.POINTER(HHSState)),
                                       ctypes.POINTER(HHSParams), vp, vp]
        L.serve_footprint.argtypes = [i64, ci]
        L.serve_create.argtypes = [vp, ctypes.POINTER(HHSParams), ctypes.POINTER(ServeParams),
                                   ctypes.POINTER(vp)]
        L.serve_destroy.argtypes = [vp]
        L.serve_submit.argtypes = [vp, ctypes.POINTER(ServeRequest), ctypes.POINTER(i64)]
        L.serve_step.argtypes = [vp, ctypes.POINTER(ci), ctypes.POINTER(ci)]
        L.serve_poll.argtypes = [vp, ctypes.POINTER(ServeResult), ci, ctypes.POINTER(ci)]
        L.serve_cancel.argtypes = [vp, i64]
        L.serve_info.argtypes = [vp, vp]
        for name in EXPORTED:
            if name not in ("fmm_last_error", "hhs_run_bytes", "serve_footprint",
                            "chin_work_bytes"):
                getattr(L, name).restype = ctypes.c_int
        L.hhs_run_bytes.restype = i64
        L.chin_work_bytes.restype = i64
        L.serve_footprint.restype = i64
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _check_dev(t, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Solver:
    """One solver context (workspace for up to max_n active particles)."""

    def __init__(self, max_n, *, p_max=6, leaf_size=16, kernel=WENDLAND, precision=FP64,
                 stream=None):
        self._h = None
        self.max_n = int(max_n)
        self.precision = precision
        self.kernel = kernel
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        prm = _Params(int(p_max), int(leaf_size), int(kernel), int(precision))
        h = ctypes.c_void_p()
        st = lib().fmm_create(ctypes.byref(prm), self.max_n, ctypes.c_void_p(self.stream.cuda_stream),
                              ctypes.byref(h))
        if st != FMM_OK:
            raise FMMError(st, "fmm_create failed")
        self._h = h

    def close(self):
        if self._h:
            lib().fmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st):
        if st != FMM_OK:
            raise FMMError(st, lib().fmm_last_error(self._h).decode())

    def build(self, pos, active=None, *, eps, theta):
        n_total = pos.shape[1]
        _check_dev(pos, torch.float64, (3, n_total), "pos")
        n = n_total if active is None else active.shape[0]
        if active is not None:
            _check_dev(active, torch.int32, None, "active")
        self._raise(lib().fmm_build(self._h, _ptr(pos), n_total, _ptr(active), n, float(eps),
                                    float(theta)))

    def evaluate(self, pos, mass, active=None, *, p, acc=None, pot=None):
        n_total = pos.shape[1]
        n = n_total if active is None else active.shape[0]
        _check_dev(mass, torch.float64, (n_total,), "mass")
        if acc is None:
            acc = torch.empty((3, n), dtype=torch.float64, device=pos.device)
        if pot is None:
            pot = torch.empty((n,), dtype=torch.float64, device=pos.device)
        _check_dev(acc, torch.float64, (3, n), "acc")
        _check_dev(pot, torch.float64, (n,), "pot")
        self._raise(lib().fmm_evaluate(self._h, _ptr(pos), _ptr(mass), n_total, _ptr(active), n,
                                       int(p), _ptr(acc), _ptr(pot)))
        return acc, pot

    def forces(self, pos, mass, active=None, *, eps, theta, p, acc=None, pot=None, sinks=None):
        """Build and evaluate in one call (fmm_forces).  sinks: optional uint8
        flags over the active set; then only flagged particles get acc/pot."""
        if sinks is not None:
            d = dict(pos=pos, mass=mass, sinks=sinks, acc=acc, pot=pot)
            if active is not None:
                d["active"] = active
            arr, outs = self._requests([d], True)
            self._raise(lib().fmm_forces_batched(self._h, 1, arr, float(eps), float(theta),
                                                 int(p)))
            return outs[0]
        n_total = pos.shape[1]
        _check_dev(pos, torch.float64, (3, n_total), "pos")
        n = n_total if active is None else active.shape[0]
        if active is not None:
            _check_dev(active, torch.int32, None, "active")
        _check_dev(mass, torch.float64, (n_total,), "mass")
        if acc is None:
            acc = torch.empty((3, n), dtype=torch.float64, device=pos.device)
        if pot is None:
            pot = torch.empty((n,), dtype=torch.float64, device=pos.device)
        _check_dev(acc, torch.float64, (3, n), "acc")
        _check_dev(pot, torch.float64, (n,), "pot")
        self._raise(lib().fmm_forces(self._h, _ptr(pos), _ptr(mass), n_total, _ptr(active), n,
                                     float(eps), float(theta), int(p), _ptr(acc), _ptr(pot)))
        return acc, pot

    def forces_grad(self, pos, mass, active=None, *, eps, theta, p):
        """forces() plus the force gradient d a_i/d x_i (fmm_forces_grad):
        (acc (3,n), pot (n), grad (6,n): xx, yy, zz, xy, xz, yz)."""
        n_total = pos.shape[1]
        _check_dev(pos, torch.float64, (3, n_total), "pos")
        n = n_total if active is None else active.shape[0]
        if active is not None:
            _check_dev(active, torch.int32, None, "active")
        _check_dev(mass, torch.float64, (n_total,), "mass")
        acc = torch.empty((3, n), dtype=torch.float64, device=pos.device)
        pot = torch.empty((n,), dtype=torch.float64, device=pos.device)
        grad = torch.empty((6, n), dtype=torch.float64, device=pos.device)
        self._raise(lib().fmm_forces_grad(self._h, _ptr(pos), _ptr(mass), n_total, _ptr(active),
                                          n, float(eps), float(theta), int(p), _ptr(acc),
                                          _ptr(pot), _ptr(grad)))
        return acc, pot, grad

    def evaluate_dipole(self, pos, mass, vec, active=None, *, p):
        """fmm_evaluate_dipole on the last tree: (u (3,n), phi (n)) of the
        vector sources m_j vec_j (vec (3,n) in active order)."""
        n_total = pos.shape[1]
        n = n_total if active is None else active.shape[0]
        _check_dev(mass, torch.float64, (n_total,), "mass")
        _check_dev(vec, torch.float64, (3, n), "vec")
        u = torch.empty((3, n), dtype=torch.float64, device=pos.device)
        phi = torch.empty((n,), dtype=torch.float64, device=pos.device)
        self._raise(lib().fmm_evaluate_dipole(self._h, _ptr(pos), _ptr(mass), n_total,
                                              _ptr(active), n, int(p), _ptr(vec), _ptr(u),
                                              _ptr(phi)))
        return u, phi

    def _requests(self, systems, with_outputs):
        arr = (Request * len(systems))()
        outs = []
        for k, sysd in enumerate(systems):
            pos = sysd["pos"]
            n_total = pos.shape[1]
            _check_dev(pos, torch.float64, (3, n_total), "pos")
            active = sysd.get("active")
            n = n_total if active is None else active.shape[0]
            q = arr[k]
            q.pos, q.n_total, q.active, q.n_active = pos.data_ptr(), n_total, (
                None if active is None else active.data_ptr()), n
            if with_outputs:
                mass = sysd["mass"]
                _check_dev(mass, torch.float64, (n_total,), "mass")
                acc = sysd.get("acc")
                pot = sysd.get("pot")
                if acc is None:
                    acc = torch.empty((3, n), dtype=torch.float64, device=pos.device)
                if pot is None:
                    pot = torch.empty((n,), dtype=torch.float64, device=pos.device)
                _check_dev(acc, torch.float64, (3, n), "acc")
                _check_dev(pot, torch.float64, (n,), "pot")
                q.mass, q.acc, q.pot = mass.data_ptr(), acc.data_ptr(), pot.data_ptr()
                sinks = sysd.get("sinks")
                if sinks is not None:
                    _check_dev(sinks, torch.uint8, (n,), "sinks")
                    q.sinks = sinks.data_ptr()
                outs.append((acc, pot))
        return arr, outs

    def build_batched(self, systems, *, eps, theta):
        """systems: list of dicts with 'pos' (3 x n_total) and optional 'active'."""
        arr, _ = self._requests(systems, False)
        self._raise(lib().fmm_build_batched(self._h, len(systems), arr, float(eps), float(theta)))

    def evaluate_batched(self, systems, *, p):
        """systems as for build_batched plus 'mass' (and optional 'acc', 'pot');
        returns [(acc, pot), ...]."""
        arr, outs = self._requests(systems, True)
        self._raise(lib().fmm_evaluate_batched(self._h, len(systems), arr, int(p)))
        return outs

    def forces_batched(self, systems, *, eps, theta, p):
        self.build_batched(systems, eps=eps, theta=theta)
        return self.evaluate_batched(systems, p=p)

    def set_small_path(self, enable):
        """Single-workgroup build and walk for small batches: True (default)
        up to 1024 particles, 2 up to 8192 (the most those launches hold),
        False never; same trees, lists and results either way."""
        mode = 2 if enable == 2 else int(bool(enable))
        self._raise(lib().fmm_set_small_path(self._h, mode))

    def set_level_prediction(self, enable):
        """Queue tree and walk (and in forces() the evaluation) for the split
        depth of recent builds, one header readback (off by default: the split
        depth is read first).  Same trees, lists and results either way."""
        self._raise(lib().fmm_set_level_prediction(self._h, int(bool(enable))))

    def tree_info(self):
        import numpy as np
        info = np.zeros(9, dtype=np.int64)
        self._raise(lib().fmm_tree_info(self._h, _hptr(info)))
        keys = ("n", "nodes", "m2l", "p2p", "depth", "leaves", "m2l_directed", "p2p_directed",
                "p2p_interactions")
        return dict(zip(keys, (int(x) for x in info)))

    def export_tree(self):
        import numpy as np
        info = self.tree_info()
        nn, n = info["nodes"], info["n"]
        out = dict(
            perm=np.zeros(n, dtype=np.int64), level=np.zeros(nn, dtype=np.int32),
            prefix=np.zeros(nn, dtype=np.uint64), begin=np.zeros(nn, dtype=np.int64),
            end=np.zeros(nn, dtype=np.int64), is_leaf=np.zeros(nn, dtype=np.int32),
            centre=np.zeros((nn, 3)), half=np.zeros(nn),
            m2l=np.zeros((info["m2l"], 2), dtype=np.int64),
            p2p=np.zeros((info["p2p"], 2), dtype=np.int64), box=np.zeros(5))
        self._raise(lib().fmm_export_tree(self._h, *[_hptr(out[k]) for k in (
            "perm", "level", "prefix", "begin", "end", "is_leaf", "centre", "half", "m2l", "p2p",
            "box")]))
        return out

    def profile(self, enable=True, kernels_only=False):
        """Start (clearing totals) or stop per-phase HIP-event timing; with
        kernels_only only the M2L and P2P kernels are timed."""
        mode = (2 if kernels_only else 1) if enable else 0
        self._raise(lib().fmm_profile_enable(self._h, mode))

    def profile_read(self):
        """{phase: (milliseconds, timed launch groups)} since profile(True)."""
        import numpy as np
        ms = np.zeros(7)
        calls = np.zeros(7, dtype=np.int64)
        self._raise(lib().fmm_profile_read(self._h, _hptr(ms), _hptr(calls)))
        return {k: (float(ms[i]), int(calls[i])) for i, k in enumerate(PHASES)}

    def invariants(self, pos=None, vel=None, mass=None, acc=None, pot=None, n=None):
        import numpy as np
        if n is None:
            for t in (pos, vel, acc, pot, mass):
                if t is not None:
                    n = t.shape[-1]
                    break
        out = np.zeros(12)
        self._raise(lib().fmm_invariants(self._h, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(acc),
                                         _ptr(pot), int(n), _hptr(out)))
        keys = ("F", "P", "L")
        res = {k: out[3 * i:3 * i + 3].copy() for i, k in enumerate(keys)}
        res.update(T=out[9], W=out[10], Fabs=out[11])
        return res


def invariants_noalloc(out, pos=None, vel=None, mass=None, acc=None, pot=None, n=None,
                       stream=None):
    """fmm_invariants_noalloc: the twelve sums of Solver.invariants written to
    the device tensor ``out`` (12 float64) on ``stream`` (default: torch's
    current stream), with no allocation and no synchronisation."""
    if n is None:
        for t in (pos, vel, acc, pot, mass):
            if t is not None:
                n = t.shape[-1]
                break
    _check_dev(out, torch.float64, (12,), "out")
    s = stream if stream is not None else torch.cuda.current_stream()
    st = lib().fmm_invariants_noalloc(ctypes.c_void_p(s.cuda_stream), _ptr(pos), _ptr(vel),
                                      _ptr(mass), _ptr(acc), _ptr(pot), int(n), _ptr(out))
    if st != FMM_OK:
        raise FMMError(st, "fmm_invariants_noalloc failed")
    return out


class HHSRun:
    """Device scratch of one system's integration (hhs_run_create)."""

    def __init__(self, solver, n, max_levels):
        self.solver = solver
        h = ctypes.c_void_p()
        solver._raise(lib().hhs_run_create(solver._h, int(n), int(max_levels), ctypes.byref(h)))
        self._h = h

    @staticmethod
    def nbytes(n, max_levels):
        return int(lib().hhs_run_bytes(int(n), int(max_levels)))

    def close(self):
        if self._h:
            lib().hhs_run_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HHS:
    """Device-resident HHS integrator state driven by hhs_init / hhs_step.

    With ``run`` (an HHSRun of at least n particles) the system can take part
    in hhs_init_batched / hhs_step_batched with other systems."""

    def __init__(self, solver, pos, vel, mass, *, eps, theta, p, eta, max_levels,
                 freeze_rungs=False, run=None, eta1=0.0, cosmo=None, t=0.0):
        self.solver = solver
        self.run = run
        n = pos.shape[1]
        for arr, nm, shp in ((pos, "pos", (3, n)), (vel, "vel", (3, n)), (mass, "mass", (n,))):
            _check_dev(arr, torch.float64, shp, nm)
        self.pos, self.vel, self.mass = pos, vel, mass
        dev = pos.device
        self.a_old = torch.zeros(n, dtype=torch.float64, device=dev)
        self.a_cur = torch.zeros(n, dtype=torch.float64, device=dev)
        self.rung = torch.zeros(n, dtype=torch.int32, device=dev)
        self.a_tot = torch.zeros(n, dtype=torch.float64, device=dev)
        self.state = HHSState(pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), self.a_old.data_ptr(),
                              self.a_cur.data_ptr(), self.rung.data_ptr(), n, float(t),
                              self.a_tot.data_ptr())
        # cosmo: a Cosmology table for the comoving form (t and dt_top in ln a)
        self.cosmo = cosmo
        self.params = HHSParams(float(eps), float(theta), int(p), float(eta), int(max_levels),
                                int(bool(freeze_rungs)), float(eta1),
                                None if cosmo is None else cosmo._h.value)

    @property
    def t(self):
        return self.state.t

    def init(self):
        self.solver._raise(lib().hhs_init(self.solver._h, ctypes.byref(self.state),
                                          ctypes.byref(self.params)))

    def step(self, dt_top):
        import numpy as np
        stats = np.zeros(3, dtype=np.int64)
        self.solver._raise(lib().hhs_step(self.solver._h, ctypes.byref(self.state),
                                          ctypes.byref(self.params), float(dt_top), _hptr(stats)))
        return dict(force_calls=int(stats[0]), force_particles=int(stats[1]), builds=int(stats[2]))

    def trad_step(self, dt_top):
        """One top step of the individual-timestep comparison integrator
        (trad_step) on this state; needs no init()."""
        import numpy as np
        stats = np.zeros(3, dtype=np.int64)
        self.solver._raise(lib().trad_step(self.solver._h, ctypes.byref(self.state),
                                           ctypes.byref(self.params), float(dt_top),
                                           _hptr(stats)))
        return dict(force_calls=int(stats[0]), force_particles=int(stats[1]), builds=int(stats[2]))


class Chin:
    """Device state of the fourth-order integrator (chin_init / chin_step):
    positions and velocities are updated in place; ``acc`` holds the
    acceleration at the current positions."""

    def __init__(self, solver, pos, vel, mass, *, eps, theta, p, t=0.0):
        n = pos.shape[1]
        for arr, nm, shp in ((pos, "pos", (3, n)), (vel, "vel", (3, n)), (mass, "mass", (n,))):
            _check_dev(arr, torch.float64, shp, nm)
        self.solver = solver
        self.pos, self.vel, self.mass = pos, vel, mass
        self.acc = torch.zeros((3, n), dtype=torch.float64, device=pos.device)
        nb = int(lib().chin_work_bytes(n))
        self.work = torch.empty((nb // 8,), dtype=torch.float64, device=pos.device)
        self.state = ChinState(pos.data_ptr(), vel.data_ptr(), mass.data_ptr(),
                               self.acc.data_ptr(), self.work.data_ptr(), n, float(t))
        self.eps, self.theta, self.p = float(eps), float(theta), int(p)

    @property
    def t(self):
        return self.state.t

    def init(self):
        self.solver._raise(lib().chin_init(self.solver._h, ctypes.byref(self.state), self.eps,
                                           self.theta, self.p))

    def step(self, h):
        import numpy as np
        stats = np.zeros(3, dtype=np.int64)
        self.solver._raise(lib().chin_step(self.solver._h, ctypes.byref(self.state), self.eps,
                                           self.theta, self.p, float(h), _hptr(stats)))
        return dict(evaluations=int(stats[0]), particles=int(stats[1]), builds=int(stats[2]))


def _batch_args(systems):
    n = len(systems)
    runs = (ctypes.c_void_p * n)(*[s.run._h.value for s in systems])
    sts = (ctypes.POINTER(HHSState) * n)(*[ctypes.pointer(s.state) for s in systems])
    return n, runs, sts


def hhs_init_batched(solver, systems):
    """hhs_init of several HHS systems (each with its own ``run``) at once."""
    n, runs, sts = _batch_args(systems)
    solver._raise(lib().hhs_init_batched(solver._h, n, runs, sts, ctypes.byref(systems[0].params)))


def hhs_step_batched(solver, systems, dt_top):
    """One top-level step of each system (dt_top: one value or one per system);
    every system ends as after an hhs_step of it alone."""
    import numpy as np
    n, runs, sts = _batch_args(systems)
    dts = np.broadcast_to(np.asarray(dt_top, dtype=np.float64), (n,)).copy()
    stats = np.zeros(3, dtype=np.int64)
    solver._raise(lib().hhs_step_batched(solver._h, n, runs, sts, ctypes.byref(systems[0].params),
                                         _hptr(dts), _hptr(stats)))
    return dict(force_calls=int(stats[0]), force_particles=int(stats[1]), builds=int(stats[2]))


class Server:
    """Request server for ensembles of HHS simulations (serve_* in the C ABI).

    ``submit`` takes host float64 arrays (pos and vel 3 x n, mass n) and keeps
    them, with the output arrays, alive until the request's result is polled."""

    def __init__(self, solver, *, eps, theta, p, eta, max_levels, arena_bytes, max_slots,
                 dt_max=1.0 / 16, eta1=0.0):
        self.solver = solver
        self.params = HHSParams(float(eps), float(theta), int(p), float(eta), int(max_levels), 0,
                                float(eta1))
        sp = ServeParams(int(arena_bytes), int(max_slots), float(dt_max))
        h = ctypes.c_void_p()
        solver._raise(lib().serve_create(solver._h, ctypes.byref(self.params), ctypes.byref(sp),
                                         ctypes.byref(h)))
        self._h = h
        self._live = {}

    @staticmethod
    def footprint(n, max_levels):
        return int(lib().serve_footprint(int(n), int(max_levels)))

    def submit(self, pos, vel, mass, t_end):
        import numpy as np
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        n = mass.size
        if pos.shape != (3, n) or vel.shape != (3, n):
            raise ValueError("pos and vel must be 3 x n")
        out_p = np.empty((3, n))
        out_v = np.empty((3, n))
        rq = ServeRequest(pos.ctypes.data, vel.ctypes.data, mass.ctypes.data, n, float(t_end),
                          out_p.ctypes.data, out_v.ctypes.data)
        rid = ctypes.c_int64()
        self.solver._raise(lib().serve_submit(self._h, ctypes.byref(rq), ctypes.byref(rid)))
        self._live[rid.value] = (pos, vel, mass, out_p, out_v)
        return rid.value

    def step(self):
        nr, nq = ctypes.c_int(), ctypes.c_int()
        self.solver._raise(lib().serve_step(self._h, ctypes.byref(nr), ctypes.byref(nq)))
        return nr.value, nq.value

    def poll(self, max_out=64):
        """Finished requests: list of dicts with the result fields and the
        final ``pos`` and ``vel``."""
        buf = (ServeResult * max_out)()
        k = ctypes.c_int()
        out = []
        while True:
            self.solver._raise(lib().serve_poll(self._h, buf, max_out, ctypes.byref(k)))
            for i in range(k.value):
                r = buf[i]
                d = {f: getattr(r, f) for f, _ in ServeResult._fields_}
                keep = self._live.pop(r.id)
                d["pos"], d["vel"] = keep[3], keep[4]
                out.append(d)
            if k.value < max_out:
                return out

    def cancel(self, rid):
        self.solver._raise(lib().serve_cancel(self._h, int(rid)))
        self._live.pop(rid, None)

    def info(self):
        import numpy as np
        v = np.zeros(6, dtype=np.int64)
        self.solver._raise(lib().serve_info(self._h, _hptr(v)))
        return dict(resident=int(v[0]), queued=int(v[1]), finished=int(v[2]),
                    arena_used=int(v[3]), arena_bytes=int(v[4]), steps=int(v[5]))

    def close(self):
        if self._h:
            lib().serve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
