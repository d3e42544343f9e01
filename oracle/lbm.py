"""ctypes wrapper around the C oracle (``lbm_oracle.c``) plus whole-run helpers.

TEST INFRASTRUCTURE (see the package docstring).

Arrays follow the C layout: populations ``f[2][9][ny][nx]``, densities
``rho[2][ny][nx]``, mask ``[ny][nx]`` (uint8, 1 = fluid).  Species 0 is oil,
species 1 is water.  All floating point is float64.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("periodic_y", ctypes.c_int32),
        ("reg_order", ctypes.c_int32),
        ("tau", ctypes.c_double * 2),
        ("G", ctypes.c_double),
        ("rho_s", ctypes.c_double * 2),
        ("g", ctypes.c_double * 2),
        ("wall_interp", ctypes.c_int32),
        ("reserved2", ctypes.c_int32),
        ("wall_yc", ctypes.c_double),
        ("wall_h0", ctypes.c_double),
        ("wall_a", ctypes.c_double),
        ("wall_lam", ctypes.c_double),
    ]


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        pp = ctypes.POINTER(OrcParams)
        lib.orc_equilibrium.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        lib.orc_regularize.argtypes = [dp, dp, dp, dp]
        lib.orc_regularize3.argtypes = [dp, dp, dp, dp]
        lib.orc_wall_fraction.argtypes = [pp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.orc_wall_fraction.restype = ctypes.c_double
        lib.orc_densities.argtypes = [pp, u8p, dp, dp]
        lib.orc_interaction_sum.argtypes = [pp, u8p, dp, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, dp, dp]
        lib.orc_tau_mix.argtypes = [pp, ctypes.c_double, ctypes.c_double]
        lib.orc_tau_mix.restype = ctypes.c_double
        lib.orc_step.argtypes = [pp, u8p, dp, dp, dp]
        lib.orc_step.restype = ctypes.c_int
        lib.orc_run.argtypes = [pp, u8p, dp, dp, ctypes.c_int64]
        lib.orc_run.restype = ctypes.c_int64
        lib.orc_init.argtypes = [pp, u8p, dp, dp]
        lib.orc_moments.argtypes = [pp, u8p, dp, dp, dp, dp, dp, dp]
        lib.orc_lattice.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                    dp, ctypes.POINTER(ctypes.c_int)]
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_get_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8(a):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def lattice():
    """Return (cx, cy, w, opp) of the oracle's D2Q9 velocity set."""
    cx = (ctypes.c_int * 9)()
    cy = (ctypes.c_int * 9)()
    w = (ctypes.c_double * 9)()
    opp = (ctypes.c_int * 9)()
    _lib().orc_lattice(cx, cy, w, opp)
    return (np.array(cx[:]), np.array(cy[:]), np.array(w[:]), np.array(opp[:]))


def equilibrium(rho, ux, uy):
    """Eq. 7 at one node; returns the 9 equilibrium populations."""
    out = np.zeros(9)
    _lib().orc_equilibrium(float(rho), float(ux), float(uy), _dp(out))
    return out


def regularize(f, feq):
    """Eq. 6: returns (f' [9], Pi^neq [xx, xy, yy])."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    feq = np.ascontiguousarray(feq, dtype=np.float64)
    out = np.zeros(9)
    pi = np.zeros(3)
    _lib().orc_regularize(_dp(f), _dp(feq), _dp(out), _dp(pi))
    return out, pi


def regularize3(f, feq):
    """Eq. 6 with the third-order Hermite terms: returns (f' [9], a3 [2,2,2])."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    feq = np.ascontiguousarray(feq, dtype=np.float64)
    out = np.zeros(9)
    a3 = np.zeros(8)
    _lib().orc_regularize3(_dp(f), _dp(feq), _dp(out), _dp(a3))
    return out, a3.reshape(2, 2, 2)


class Params:
    """Physical and lattice parameters of one oracle lattice (reg_order: Hermite
    order of the regularization, 2 or 3)."""

    def __init__(self, nx, ny, tau=(1.0, 1.0), G=0.0, rho_s=(0.0, 0.0), g=(0.0, 0.0),
                 periodic_y=False, reg_order=2, wall=None):
        """wall: None (half-way bounce-back) or (yc, h0, a, lam) of the channel
        walls, placed at their sub-lattice positions by interpolated
        bounce-back."""
        self.c = OrcParams()
        self.c.nx, self.c.ny = int(nx), int(ny)
        self.c.periodic_y = 1 if periodic_y else 0
        self.c.reg_order = int(reg_order)
        if wall is not None:
            self.c.wall_interp = 1
            self.c.wall_yc, self.c.wall_h0, self.c.wall_a, self.c.wall_lam = (float(v) for v in wall)
        self.c.tau[0], self.c.tau[1] = float(tau[0]), float(tau[1])
        self.c.G = float(G)
        self.c.rho_s[0], self.c.rho_s[1] = float(rho_s[0]), float(rho_s[1])
        self.c.g[0], self.c.g[1] = float(g[0]), float(g[1])

    @property
    def nx(self):
        return self.c.nx

    @property
    def ny(self):
        return self.c.ny

    def ref(self):
        return ctypes.byref(self.c)


def wall_fraction(params, x, y, i):
    """Fraction of the link from (x, y) along c_i at which it meets the wall."""
    return _lib().orc_wall_fraction(params.ref(), int(x), int(y), int(i))


def tau_mix(params, rho_o, rho_w):
    return _lib().orc_tau_mix(params.ref(), float(rho_o), float(rho_w))


def interaction_sum(params, mask, rho, beta, x, y):
    """sum_i w_i c_i rho~^beta(x + c_i) at node (x, y) (Eq. 8 without G rho^alpha)."""
    sx = ctypes.c_double()
    sy = ctypes.c_double()
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    _lib().orc_interaction_sum(params.ref(), _u8(mask), _dp(rho), int(beta), int(x), int(y),
                               ctypes.byref(sx), ctypes.byref(sy))
    return sx.value, sy.value


class Lattice:
    """A two-species oracle lattice: parameters, fluid mask and state."""

    def __init__(self, params, mask, rho0):
        self.p = params
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        assert self.mask.shape == (params.ny, params.nx)
        n = params.nx * params.ny
        self.f = np.zeros((2, 9, params.ny, params.nx))
        self.work = np.zeros(2 * 9 * n + 2 * n)
        self.t = 0
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        assert rho0.shape == (2, params.ny, params.nx)
        _lib().orc_init(params.ref(), _u8(self.mask), _dp(rho0), _dp(self.f))

    def step(self, nsteps=1):
        """Advance nsteps; raises FloatingPointError on a non-physical state."""
        bad = _lib().orc_run(self.p.ref(), _u8(self.mask), _dp(self.f), _dp(self.work),
                             int(nsteps))
        if bad >= 0:
            self.t += int(bad) + 1
            raise FloatingPointError("oracle state became non-physical at step %d" % self.t)
        self.t += int(nsteps)

    def set_body_force(self, gx, gy=0.0):
        self.p.c.g[0], self.p.c.g[1] = float(gx), float(gy)

    def moments(self):
        """Return dict with rho [2,ny,nx], u [2,ny,nx] (physical), p [ny,nx], mon [8]."""
        ny, nx = self.p.ny, self.p.nx
        rho = np.zeros((2, ny, nx))
        u = np.zeros((2, ny, nx))
        pr = np.zeros((ny, nx))
        mon = np.zeros(8)
        rw = np.zeros(2 * nx * ny)
        _lib().orc_moments(self.p.ref(), _u8(self.mask), _dp(self.f), _dp(rw), _dp(rho),
                           _dp(u), _dp(pr), _dp(mon))
        return {"rho": rho, "u": u, "p": pr, "mon": mon}

    def copy_state(self):
        return self.f.copy(), self.t

    def restore_state(self, state):
        self.f[...] = state[0]
        self.t = state[1]


def step_once(params, mask, f):
    """One step of an explicit population array; returns (f_new, bad_count)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    rho = np.zeros((2, params.ny, params.nx))
    bad = _lib().orc_step(params.ref(), _u8(np.ascontiguousarray(mask, dtype=np.uint8)),
                          _dp(f), _dp(out), _dp(rho))
    return out, bad


def threads_used():
    """OpenMP threads the oracle's step loops will use."""
    return int(_lib().orc_get_threads())


def set_threads(n):
    """Threads of the oracle's OpenMP step loops (D2Q9 and D3Q19; timing only,
    results do not depend on it)."""
    _lib().orc_set_threads(int(n))
