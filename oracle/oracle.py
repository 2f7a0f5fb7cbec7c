"""Python face of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Wraps ``liboracle.so`` (plain C, built from ``fmm_oracle.c``) and adds the
hierarchical Hamiltonian splitting (HHS) integrator of the paper (Sec. 2.2,
Algorithms 1-3), the paper's comparison integrator with individual
timesteps (Sec. 2.3) and the fourth-order integrator it proposes (Sec. 4.1)
in plain numpy on top of the oracle's force solve, and the comoving drift and
kick factors of Sec. 3.5 by adaptive quadrature.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It imports nothing from the GPU package, and the GPU
package imports nothing from here.

Conventions (shared with the GPU path only through their documented meaning):
positions are SoA float64 arrays of shape (3, n); accelerations are per unit
mass, a_i = -grad_i Phi; potentials Phi_i = sum_{j != i} m_j psi(r_ij) with
G = 1 and psi < 0.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

WENDLAND = 0
PLUMMER = 1


def build_oracle() -> str:
    """Compile the C oracle (gcc, FP64, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           _SRC, "-o", _LIB, "-lm"]
    subprocess.check_call(cmd)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L.orc_fmm.restype = ctypes.c_int
        L.orc_tree_build.restype = ctypes.c_void_p
        L.orc_tree_build.argtypes = [dp, i64, ctypes.c_void_p, i64, ctypes.c_void_p]
        L.orc_tree_free.argtypes = [ctypes.c_void_p]
        L.orc_tree_info.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_tree_export.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 11
        L.orc_tree_eval_ex.argtypes = [ctypes.c_void_p, dp, i64, ctypes.c_void_p, dp, dp,
                                       ctypes.c_void_p, ctypes.c_void_p]
        L.orc_tree_eval_grad.argtypes = [ctypes.c_void_p, dp, i64, ctypes.c_void_p, dp, dp, dp]
        L.orc_tree_eval_dipole.argtypes = [ctypes.c_void_p, dp, i64, ctypes.c_void_p, dp, dp,
                                           dp]
        L.orc_tree_eval_par.argtypes = [ctypes.c_void_p, dp, i64, ctypes.c_void_p, dp, dp]
        L.orc_threads.argtypes = [ctypes.c_int]
        L.orc_threads.restype = ctypes.c_int
        L.orc_tree_eval_sinks.argtypes = [ctypes.c_void_p, dp, ctypes.c_void_p, ctypes.c_void_p,
                                          i64, dp, dp]
        L.orc_tree_eval_sinks_grad.argtypes = [ctypes.c_void_p, dp, ctypes.c_void_p,
                                               ctypes.c_void_p, i64, dp, dp, dp]
        L.orc_direct.argtypes = [dp, dp, i64, ctypes.c_void_p, i64, ctypes.c_int,
                                 ctypes.c_double, dp, dp]
        L.orc_derivs_export.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp,
                                        ctypes.POINTER(ctypes.c_int)]
        for name in ("orc_wendland_phi", "orc_wendland_g", "orc_plummer_phi", "orc_plummer_g"):
            f = getattr(L, name)
            f.restype = ctypes.c_double
            f.argtypes = [ctypes.c_double, ctypes.c_double]
        _lib = L
    return _lib


class _Params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("theta", ctypes.c_double), ("eps", ctypes.c_double),
                ("leaf_size", ctypes.c_int), ("kernel", ctypes.c_int)]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vp(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _pos(pos):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    assert pos.ndim == 2 and pos.shape[0] == 3
    return pos


def _active(active):
    if active is None:
        return None
    return np.ascontiguousarray(active, dtype=np.int32)


def kernel_phi(kernel, r, eps):
    f = lib().orc_plummer_phi if kernel == PLUMMER else lib().orc_wendland_phi
    return f(float(r), float(eps))


def kernel_g(kernel, r, eps):
    f = lib().orc_plummer_g if kernel == PLUMMER else lib().orc_wendland_g
    return f(float(r), float(eps))


def coeff_count(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


def derivs(p, R, e2=0.0):
    """D^k psi(R) for |k| <= p by power-series composition; returns (D, k)."""
    K = coeff_count(p)
    D = np.zeros(K)
    k = np.zeros(3 * K, dtype=np.int32)
    R = np.ascontiguousarray(R, dtype=np.float64)
    rc = lib().orc_derivs_export(p, _dp(R), float(e2), _dp(D),
                                 k.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    assert rc == 0
    return D, k.reshape(K, 3)


def direct(pos, mass, kernel, eps, sinks=None):
    """O(N^2) direct summation: (acc (3, n_sinks), pot (n_sinks))."""
    pos = _pos(pos)
    n = pos.shape[1]
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
    ns = n if s is None else len(s)
    acc = np.zeros((3, ns))
    pot = np.zeros(ns)
    rc = lib().orc_direct(_dp(pos), _dp(mass), n, _vp(s), ns, int(kernel), float(eps),
                          _dp(acc), _dp(pot))
    assert rc == 0
    return acc, pot


class Tree:
    """Oracle tree + interaction lists over the active set, canonical export."""

    def __init__(self, pos, active=None, *, p, theta, eps, leaf_size, kernel):
        self.pos = _pos(pos)
        self.n_total = self.pos.shape[1]
        self.active = _active(active)
        self.n = self.n_total if self.active is None else len(self.active)
        self.prm = _Params(int(p), float(theta), float(eps), int(leaf_size), int(kernel))
        self.p = int(p)
        self._h = lib().orc_tree_build(_dp(self.pos), self.n_total, _vp(self.active), self.n,
                                       ctypes.byref(self.prm))
        if not self._h:
            raise ValueError("oracle tree build rejected its arguments")
        info = np.zeros(6, dtype=np.int64)
        lib().orc_tree_info(self._h, _vp(info))
        self.n_nodes, self.n_m2l, self.n_p2p, self.depth, self.n_leaves = (
            int(info[1]), int(info[2]), int(info[3]), int(info[4]), int(info[5]))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_tree_free(h)
            self._h = None

    def export(self):
        nn = self.n_nodes
        out = dict(
            perm=np.zeros(self.n, dtype=np.int64),
            level=np.zeros(nn, dtype=np.int32),
            prefix=np.zeros(nn, dtype=np.uint64),
            begin=np.zeros(nn, dtype=np.int64),
            end=np.zeros(nn, dtype=np.int64),
            is_leaf=np.zeros(nn, dtype=np.int32),
            centre=np.zeros((nn, 3)),
            half=np.zeros(nn),
            m2l=np.zeros((self.n_m2l, 2), dtype=np.int64),
            p2p=np.zeros((self.n_p2p, 2), dtype=np.int64),
            box=np.zeros(5),
        )
        lib().orc_tree_export(self._h, *[_vp(out[k]) for k in (
            "perm", "level", "prefix", "begin", "end", "is_leaf", "centre", "half", "m2l",
            "p2p", "box")])
        return out

    def evaluate(self, mass, want_expansions=False):
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        acc = np.zeros((3, self.n))
        pot = np.zeros(self.n)
        M = L = None
        if want_expansions:
            K = coeff_count(self.p)
            M = np.zeros((self.n_nodes, K))
            L = np.zeros((self.n_nodes, K))
        rc = lib().orc_tree_eval_ex(self._h, _dp(mass), self.n_total, _vp(self.active),
                                    _dp(acc), _dp(pot), _vp(M), _vp(L))
        assert rc == 0
        if want_expansions:
            return acc, pot, M, L
        return acc, pot


    def evaluate_parallel(self, mass):
        """evaluate() spread over OpenMP threads (orc_threads), each sum formed
        in evaluate()'s order: the same (acc, pot) bit for bit."""
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        acc = np.zeros((3, self.n))
        pot = np.zeros(self.n)
        rc = lib().orc_tree_eval_par(self._h, _dp(mass), self.n_total, _vp(self.active),
                                     _dp(acc), _dp(pot))
        assert rc == 0
        return acc, pot

    def evaluate_grad(self, mass):
        """acc (3,n), pot (n) and the force gradient d a_i / d x_i of every
        sink, SoA (6,n) in the order xx, yy, zz, xy, xz, yz (Sec. 4.1)."""
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        acc = np.zeros((3, self.n))
        pot = np.zeros(self.n)
        grad = np.zeros((6, self.n))
        rc = lib().orc_tree_eval_grad(self._h, _dp(mass), self.n_total, _vp(self.active),
                                      _dp(acc), _dp(pot), _dp(grad))
        assert rc == 0
        return acc, pot, grad

    def evaluate_dipole(self, mass, vec):
        """Field of the vector sources m_j v_j on this tree: u (3,n) with
        u_i = sum_j m_j H(x_i - x_j) v_j (H the pair Hessian of psi), i.e. the
        derivative of a_i along a displacement of every particle j by v_j, and
        phi (n) = sum_j m_j v_j . grad psi(x_i - x_j).  vec: (3,n) in active
        order.  With vec = the accelerations this is the cross term of the
        force-gradient kick of Chin's fourth-order integrator (Sec. 4.1)."""
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        vec = np.ascontiguousarray(vec, dtype=np.float64)
        assert vec.shape == (3, self.n)
        u = np.zeros((3, self.n))
        phi = np.zeros(self.n)
        rc = lib().orc_tree_eval_dipole(self._h, _dp(mass), self.n_total, _vp(self.active),
                                        _dp(vec), _dp(u), _dp(phi))
        assert rc == 0
        return u, phi

    def evaluate_sinks(self, mass, sinks):
        """FMM acceleration/potential of the given active slots only."""
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        sinks = np.ascontiguousarray(sinks, dtype=np.int64)
        acc = np.zeros((3, len(sinks)))
        pot = np.zeros(len(sinks))
        rc = lib().orc_tree_eval_sinks(self._h, _dp(mass), _vp(self.active), _vp(sinks),
                                       len(sinks), _dp(acc), _dp(pot))
        assert rc == 0
        return acc, pot

    def evaluate_sinks_grad(self, mass, sinks):
        """evaluate_sinks plus the force gradient of those sinks, SoA (6, n)
        as evaluate_grad orders it (Sec. 4.1)."""
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        sinks = np.ascontiguousarray(sinks, dtype=np.int64)
        acc = np.zeros((3, len(sinks)))
        pot = np.zeros(len(sinks))
        grad = np.zeros((6, len(sinks)))
        rc = lib().orc_tree_eval_sinks_grad(self._h, _dp(mass), _vp(self.active), _vp(sinks),
                                            len(sinks), _dp(acc), _dp(pot), _dp(grad))
        assert rc == 0
        return acc, pot, grad


def threads(n=0):
    """Threads of Tree.evaluate_parallel: sets them when n > 0; returns the
    number in use."""
    return int(lib().orc_threads(int(n)))


def fmm(pos, mass, active=None, *, p, theta, eps, leaf_size, kernel):
    """One oracle FMM force evaluation on the active set: (acc (3,n), pot (n))."""
    t = Tree(pos, active, p=p, theta=theta, eps=eps, leaf_size=leaf_size, kernel=kernel)
    return t.evaluate(mass)


# --------------------------------------------------------------------------
# HHS integrator, Sec. 2.2, Algorithms 1-3, in plain numpy
# --------------------------------------------------------------------------
class HHSState:
    """Particle state of the HHS integrator (float64, SoA)."""

    def __init__(self, pos, vel, mass):
        self.pos = np.array(pos, dtype=np.float64, copy=True)
        self.vel = np.array(vel, dtype=np.float64, copy=True)
        self.mass = np.array(mass, dtype=np.float64, copy=True)
        n = self.mass.shape[0]
        self.a_old = np.zeros(n)   # |a| from the latest second kickS2F
        self.a_cur = np.zeros(n)   # |a| from the latest second kickFS2S
        self.a_tot = np.zeros(n)   # |a| of the latest all-particle kickFS2S (Eq. 9)
        self.rung = np.zeros(n, dtype=np.int32)
        self.t = 0.0
        self.force_calls = 0
        self.force_particles = 0


class HHSOracle:
    """The hierarchical Hamiltonian splitting of Sec. 2.2 (Algorithms 1-3)
    with the oracle FMM: each level's kick-drift-kick is a table of operations
    (LEVEL_OPS), the nesting of levels a list of open time intervals (step).

    Readings where the paper is silent: a particle's timestep is
    sqrt(eta*eps/|a|) (Sec. 2.2) with |a| = |a_old| + |a_cur|; its rung is the
    smallest r >= 0 with dt_top*2^-r <= dt_i (clamped to max_levels-1), decided
    as (dt_r*dt_r)*|a| <= eta*eps so no square root enters the decision;
    at rung k the slow set is {rung <= k}, the fast set {rung > k}; rungs of the
    system are recomputed on entry when calc_timestep is set; a_old is refreshed
    at second kickS2F kicks and a_cur at second kickFS2S kicks (Algorithm 3).

    With eta1 > 0 the timestep is also bounded by sqrt(eta1*eps/|a|_tot)
    (Eq. 9, Sec. 3.4): a rung must satisfy both (dt_r*dt_r)*(|a_old|+|a_cur|)
    <= eta*eps and (dt_r*dt_r)*|a|_tot <= eta1*eps.  |a|_tot is the magnitude
    of the acceleration due to all the mass, taken where the solver sees every
    particle: the full solve of init_forces, then the second kickFS2S of each
    top-level (rung 0) KDK, whose joint set is the whole system; a top-level
    KDK with no slow particle skips that kick and leaves |a|_tot as it was.
    """

    def __init__(self, *, p, theta, eps, leaf_size, kernel, eta, max_levels, freeze_rungs=False,
                 eta1=0.0, cosmo=None):
        self.kw = dict(p=p, theta=theta, eps=eps, leaf_size=leaf_size, kernel=kernel)
        self.eps = float(eps)
        self.eta = float(eta)
        self.eta1 = float(eta1)
        # comoving form (Sec. 3.5): cosmo = dict(omega_m, omega_l, h0); the time
        # variable is then ln a, velocities are canonical momenta per unit
        # mass, a kick over [x0, x1] uses the integral of dt/a and a drift the
        # integral of dt/a^2 between a = e^x0 and e^x1 (Eqs. 10-11), and a
        # rung's step is compared in physical time, d(ln a) / H(a) at the start
        # of the subsystem's step
        self.cosmo = cosmo
        self.max_levels = int(max_levels)
        self.freeze_rungs = bool(freeze_rungs)

    def forces(self, st, active, mass):
        st.force_calls += 1
        st.force_particles += len(active)
        return fmm(st.pos, mass, active.astype(np.int32), **self.kw)

    def init_forces(self, st):
        idx = np.arange(st.mass.shape[0], dtype=np.int32)
        acc, pot = self.forces(st, idx, st.mass)
        st.a_cur = np.sqrt((acc * acc).sum(axis=0))
        st.a_old = np.zeros_like(st.a_cur)
        st.a_tot = st.a_cur.copy()
        return acc, pot

    def hubble(self, a):
        c = self.cosmo
        ok = 1.0 - c["omega_m"] - c["omega_l"]
        return c["h0"] * np.sqrt(c["omega_m"] / (a * a * a) + ok / (a * a) + c["omega_l"])

    def factors(self, x0, x1):
        """(drift, kick) factors of a step from ln a = x0 to x1."""
        c = self.cosmo
        return cosmo_factors(np.exp(x0), np.exp(x1), omega_m=c["omega_m"],
                             omega_l=c["omega_l"], h0=c["h0"])

    def rungs(self, st, idx, dt_top, t0=0.0):
        a = st.a_old[idx] + st.a_cur[idx]
        rhs = self.eta * self.eps
        H = None
        if self.cosmo is not None:
            H = self.hubble(np.exp(t0))
            rhs = rhs * (H * H)
        r = np.full(len(idx), self.max_levels - 1, dtype=np.int32)
        for k in range(self.max_levels - 1, -1, -1):
            dtk = np.ldexp(dt_top, -k)
            ok = (dtk * dtk) * a <= rhs
            if self.eta1 > 0:
                rhs1 = self.eta1 * self.eps
                if self.cosmo is not None:
                    rhs1 = rhs1 * (H * H)
                ok &= (dtk * dtk) * st.a_tot[idx] <= rhs1
            r = np.where(ok, k, r)
        return r

    def kick(self, st, sys1, joint, dt, kick_s2f, second, top=False, t0=0.0):
        mass = st.mass.copy()
        if kick_s2f:
            mass[sys1] = 0.0
        acc, _ = self.forces(st, joint, mass)
        if top and second and not kick_s2f:   # every particle is a sink here (Eq. 9)
            st.a_tot[joint] = np.sqrt((acc * acc).sum(axis=0))
        pos_in_joint = np.searchsorted(joint, sys1)
        a1 = acc[:, pos_in_joint]
        if self.cosmo is not None:
            dt = self.factors(t0, t0 + dt)[1]
        st.vel[:, sys1] += a1 * dt
        if second:
            mag = np.sqrt((a1 * a1).sum(axis=0))
            if kick_s2f:
                st.a_old[sys1] = mag
            else:
                st.a_cur[sys1] = mag

    # One level's kick-drift-kick (Sec. 2.2) as data, in time order: the
    # operation, the particles it moves, the sources of a kick ("slow": the
    # masses of the fast set zeroed, kickS2F; "all": kickFS2S), which half of
    # the level's interval a kick covers, and the |a| slot a kick over the
    # second half refreshes.  The drift moves the slow set over the whole
    # interval.  A kick whose moved set is empty, or a kickS2F with no slow
    # particle (every force zero), is skipped: this is what gives a two-rung
    # system 2 + 2 + 2^(k+1) solver calls.
    LEVEL_OPS = (("kick", "fast", "slow", 0, None),
                 ("kick", "slow", "all", 0, None),
                 ("drift", "slow", None, None, None),
                 ("kick", "slow", "all", 1, "a_cur"),
                 ("kick", "fast", "slow", 1, "a_old"))

    def level_kdk(self, st, level, slow, fast, members, t0, dt):
        sets = {"slow": slow, "fast": fast, "all": members}
        for op, moved, sources, half, slot in self.LEVEL_OPS:
            who = sets[moved]
            if op == "drift":
                length = dt if self.cosmo is None else self.factors(t0, t0 + dt)[0]
                st.pos[:, who] += st.vel[:, who] * length
                continue
            if len(who) == 0 or (sources == "slow" and len(slow) == 0):
                continue
            self.kick(st, who, members, dt / 2, sources == "slow", slot is not None,
                      top=(level == 0), t0=t0 + half * (dt / 2))

    def step(self, st, dt_top):
        """Advance every particle by dt_top (one top-level step); in the
        comoving form st.t is ln a and dt_top a step in ln a.

        A level's interval [t0, t0 + dt] for the particles handed to it
        (rung >= level) is: the faster particles (rung > level) advanced over
        the first half at the next level, this level's kick-drift-kick, the
        faster ones over the second half (their rungs set anew first).  The
        nesting is walked with an explicit list of open intervals."""
        everyone = np.arange(st.mass.shape[0], dtype=np.int32)

        class Span:
            def __init__(self, level, members, t0, dt, refresh):
                self.level, self.members, self.t0, self.dt = level, members, t0, dt
                self.refresh = refresh
                self.stage = 0
                self.slow = self.fast = None

        todo = [Span(0, everyone, st.t, dt_top, True)]
        while todo:
            sp = todo[-1]
            if sp.stage == 0:            # set rungs (when asked), split, first half
                if sp.refresh and not self.freeze_rungs:
                    st.rung[sp.members] = self.rungs(st, sp.members, dt_top, sp.t0)
                r = st.rung[sp.members]
                sp.slow, sp.fast = sp.members[r <= sp.level], sp.members[r > sp.level]
                sp.stage = 1
                if len(sp.fast):
                    todo.append(Span(sp.level + 1, sp.fast, sp.t0, sp.dt / 2, False))
            elif sp.stage == 1:          # this level's kick-drift-kick, second half
                self.level_kdk(st, sp.level, sp.slow, sp.fast, sp.members, sp.t0, sp.dt)
                sp.stage = 2
                if len(sp.fast):
                    todo.append(Span(sp.level + 1, sp.fast, sp.t0 + sp.dt / 2, sp.dt / 2, True))
            else:
                todo.pop()
        st.t += dt_top


# --------------------------------------------------------------------------
# The comparison integrator of Sec. 2.3: individual (block) timesteps with the
# same FMM, forces on the active particles from all the mass in the system
# --------------------------------------------------------------------------
class TradOracle:
    """Individual-timestep KDK with FMM forces (Sec. 2.3), in plain numpy.

    Readings where the paper is silent: the timestep of particle i is
    sqrt(eta*eps/|a_i|) (the function of Sec. 2.2 with |a| the magnitude of
    the particle's acceleration from an all-particle solve at the start of
    the top step), rounded to a rung exactly as in HHSOracle.rungs; rungs are
    fixed within a top step of length dt_top, which is split into 2^R ticks,
    R the largest rung present.  At the start every particle takes the
    opening half kick of its first step.  At the end of tick j the particles
    whose step ends there (rung >= R - ctz(j+1)) drift over their own step,
    are given the acceleration due to all the mass at the stored positions
    (a particle that is not active sits where its last step ended: positions
    are not synchronised), and take the closing half kick and, unless the top
    step ends, the opening half kick of their next step, as two separate
    additions.  a_cur holds |a| of each particle's latest force evaluation.
    """

    def __init__(self, *, p, theta, eps, leaf_size, kernel, eta, max_levels):
        self.kw = dict(p=p, theta=theta, eps=eps, leaf_size=leaf_size, kernel=kernel)
        self.H = HHSOracle(p=p, theta=theta, eps=eps, leaf_size=leaf_size, kernel=kernel,
                           eta=eta, max_levels=max_levels)

    def forces(self, st):
        """Acceleration of every particle due to all the mass (one solve)."""
        st.force_calls += 1
        acc, _ = fmm(st.pos, st.mass, None, **self.kw)
        return acc

    def step(self, st, dt_top):
        n = st.mass.shape[0]
        everyone = np.arange(n, dtype=np.int32)
        acc = self.forces(st)
        st.force_particles += n
        st.a_cur = np.sqrt((acc * acc).sum(axis=0))
        st.a_old = np.zeros(n)
        st.rung = self.H.rungs(st, everyone, dt_top)
        R = int(st.rung.max())
        half = np.ldexp(dt_top, -st.rung) * 0.5      # half step of each particle
        st.vel += acc * half
        for j in range(1 << R):
            tz = ((j + 1) & -(j + 1)).bit_length() - 1  # trailing zeros of j + 1
            ending = st.rung >= R - tz
            full = np.ldexp(dt_top, -st.rung[ending])
            st.pos[:, ending] += st.vel[:, ending] * full
            acc = self.forces(st)
            st.force_particles += int(ending.sum())
            a = acc[:, ending]
            st.vel[:, ending] += a * half[ending]
            if j + 1 < (1 << R):
                st.vel[:, ending] += a * half[ending]
            st.a_cur[ending] = np.sqrt((a * a).sum(axis=0))
        st.t += dt_top


# --------------------------------------------------------------------------
# The fourth-order integrator proposed in Sec. 4.1 (Chin & Chen 2005)
# --------------------------------------------------------------------------
class ChinState:
    """Particle state of the fourth-order integrator (float64, SoA); acc is
    the acceleration at pos."""

    def __init__(self, pos, vel, mass):
        self.pos = np.array(pos, dtype=np.float64, copy=True)
        self.vel = np.array(vel, dtype=np.float64, copy=True)
        self.mass = np.array(mass, dtype=np.float64, copy=True)
        self.acc = np.zeros_like(self.pos)
        self.t = 0.0
        self.evaluations = 0


def tensor_apply(grad, v):
    """T v for the symmetric tensors of Tree.evaluate_grad (rows xx, yy, zz,
    xy, xz, yz) and vectors v (3, n)."""
    xx, yy, zz, xy, xz, yz = grad
    return np.stack([xx * v[0] + xy * v[1] + xz * v[2],
                     xy * v[0] + yy * v[1] + yz * v[2],
                     xz * v[0] + yz * v[1] + zz * v[2]])


class ChinOracle:
    """Forward fourth-order symplectic integrator of Chin & Chen (2005),
    their algorithm 4A, with one shared timestep h and the oracle FMM.

    The flow exp(h (T + V)) is approximated by kicks and drifts with positive
    coefficients only: kick h/6 with the acceleration, drift h/2, kick 2h/3
    with the acceleration of the modified potential V + (h^2/48)[V,[T,V]],
    drift h/2, kick h/6.  For gravity that modified acceleration is
        a~_i = a_i + (h^2/24) sum_j (d a_i / d x_j) a_j,
    the sum being the derivative of a_i along a displacement of every
    particle by its own acceleration.  It splits into the force gradient of
    particle i applied to a_i (Tree.evaluate_grad) and the field of the
    vector sources m_j a_j (Tree.evaluate_dipole), both on the tree of the
    middle positions.  The paper names the scheme (Sec. 4.1) without its
    details: the coefficients and the form of the modified force are the
    published algorithm's, the sign of the correction pinned by its order.
    """

    def __init__(self, *, p, theta, eps, leaf_size, kernel):
        self.kw = dict(p=p, theta=theta, eps=eps, leaf_size=leaf_size, kernel=kernel)

    def accelerations(self, st):
        st.evaluations += 1
        acc, _ = fmm(st.pos, st.mass, None, **self.kw)
        return acc

    def init(self, st):
        st.acc = self.accelerations(st)

    def modified_acceleration(self, st, h):
        """a~ at the current positions, and the plain acceleration there."""
        t = Tree(st.pos, None, **self.kw)
        acc, _, grad = t.evaluate_grad(st.mass)
        u, _ = t.evaluate_dipole(st.mass, acc)
        st.evaluations += 2
        return acc + h * h / 24 * (tensor_apply(grad, acc) + u), acc

    def step(self, st, h):
        st.vel += h / 6 * st.acc
        st.pos += h / 2 * st.vel
        amod, _ = self.modified_acceleration(st, h)
        st.vel += 2 * h / 3 * amod
        st.pos += h / 2 * st.vel
        st.acc = self.accelerations(st)
        st.vel += h / 6 * st.acc
        st.t += h


# --------------------------------------------------------------------------
# Comoving integration factors of Sec. 3.5 (Eqs. 10-11)
# --------------------------------------------------------------------------
def cosmo_factors(a0, a1, *, omega_m, omega_l, h0):
    """(integral of dt/a^2, integral of dt/a) from scale factor a0 to a1, by
    adaptive quadrature over a with dt = da / (a H(a)),
    H = h0 sqrt(omega_m a^-3 + (1 - omega_m - omega_l) a^-2 + omega_l)."""
    from scipy.integrate import quad
    ok = 1.0 - omega_m - omega_l

    def hub(a):
        return h0 * np.sqrt(omega_m / a**3 + ok / a**2 + omega_l)

    kw = dict(epsabs=0.0, epsrel=1e-13, limit=200)
    drift = quad(lambda a: 1.0 / (a**3 * hub(a)), a0, a1, **kw)[0]
    kick = quad(lambda a: 1.0 / (a**2 * hub(a)), a0, a1, **kw)[0]
    return drift, kick


def invariants(pos, vel, mass, acc=None, pot=None):
    """Sec. 3.2's accuracy monitors as plain numpy sums: total momentum P,
    angular momentum L = sum m x cross v, kinetic energy T, and, when given,
    the potential energy W = 1/2 sum m Phi, the total force sum m a and the
    scale sum m |a|."""
    P = (mass * vel).sum(axis=1)
    Lm = (mass * np.cross(pos.T, vel.T).T).sum(axis=1)
    T = 0.5 * (mass * (vel * vel).sum(axis=0)).sum()
    out = dict(P=P, L=Lm, T=T)
    if pot is not None:
        out["W"] = 0.5 * (mass * pot).sum()
    if acc is not None:
        out["F"] = (mass * acc).sum(axis=1)
        out["Fabs"] = (mass * np.sqrt((acc * acc).sum(axis=0))).sum()
    return out
