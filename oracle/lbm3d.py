"""ctypes wrapper around the D3Q19 C oracle (``lbm3d_oracle.c``).

TEST INFRASTRUCTURE (see the package docstring).

Arrays follow the C layout: populations ``f[2][19][nz][ny][nx]``, densities
``rho[2][nz][ny][nx]``, mask ``[nz][ny][nx]`` (uint8, 1 = fluid).  Species 0 is
oil, species 1 water.  All floating point is float64.
"""
import ctypes

import numpy as np

from . import lbm as _lbm2

Q3 = 19


class Orc3Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("periodic_yz", ctypes.c_int32), ("tau", ctypes.c_double * 2),
                ("G", ctypes.c_double), ("rho_s", ctypes.c_double * 2),
                ("g", ctypes.c_double * 3), ("wall_interp", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("wall_yc", ctypes.c_double),
                ("wall_zc", ctypes.c_double), ("wall_r0", ctypes.c_double),
                ("wall_a", ctypes.c_double), ("wall_lam", ctypes.c_double)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        lib = _lbm2._lib()  # the same shared object holds both lattices
        dp = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        pp = ctypes.POINTER(Orc3Params)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc3_lattice.argtypes = [ip, ip, ip, dp, ip]
        lib.orc3_equilibrium.argtypes = [ctypes.c_double] * 4 + [dp]
        lib.orc3_regularize.argtypes = [dp, dp, dp]
        lib.orc3_densities.argtypes = [pp, u8p, dp, dp]
        lib.orc3_step.argtypes = [pp, u8p, dp, dp, dp]
        lib.orc3_step.restype = ctypes.c_int
        lib.orc3_run.argtypes = [pp, u8p, dp, dp, ctypes.c_int64]
        lib.orc3_run.restype = ctypes.c_int64
        lib.orc3_init.argtypes = [pp, u8p, dp, dp]
        lib.orc3_moments.argtypes = [pp, u8p, dp, dp, dp, dp, dp, dp]
        lib.orc3_wall_fraction.argtypes = [pp] + [ctypes.c_int] * 4
        lib.orc3_wall_fraction.restype = ctypes.c_double
        _LIB = lib
    return _LIB


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8(a):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def lattice():
    """(cx, cy, cz, w, opp) of the oracle's D3Q19 velocity set."""
    a = [(ctypes.c_int * Q3)() for _ in range(3)]
    w = (ctypes.c_double * Q3)()
    opp = (ctypes.c_int * Q3)()
    _lib().orc3_lattice(a[0], a[1], a[2], w, opp)
    return tuple(np.array(v[:]) for v in a) + (np.array(w[:]), np.array(opp[:]))


def equilibrium(rho, ux, uy, uz):
    out = np.zeros(Q3)
    _lib().orc3_equilibrium(float(rho), float(ux), float(uy), float(uz), _dp(out))
    return out


def regularize(f, feq):
    out = np.zeros(Q3)
    _lib().orc3_regularize(_dp(np.ascontiguousarray(f, dtype=np.float64)),
                           _dp(np.ascontiguousarray(feq, dtype=np.float64)), _dp(out))
    return out


class Params3:
    def __init__(self, nx, ny, nz, tau=(1.0, 1.0), G=0.0, rho_s=(0.0, 0.0),
                 g=(0.0, 0.0, 0.0), periodic_yz=False, wall=None):
        """wall = (y_c, z_c, r0, a, lambda): interpolated walls on the tube
        (y - y_c)^2 + (z - z_c)^2 = (r0 + a cos(2 pi x / lambda))^2; None:
        half-way bounce-back at the mask's solid nodes."""
        self.c = Orc3Params()
        self.c.nx, self.c.ny, self.c.nz = int(nx), int(ny), int(nz)
        self.c.periodic_yz = 1 if periodic_yz else 0
        self.c.tau[0], self.c.tau[1] = float(tau[0]), float(tau[1])
        self.c.G = float(G)
        self.c.rho_s[0], self.c.rho_s[1] = float(rho_s[0]), float(rho_s[1])
        for a in range(3):
            self.c.g[a] = float(g[a])
        if wall is not None:
            self.c.wall_interp = 1
            (self.c.wall_yc, self.c.wall_zc, self.c.wall_r0, self.c.wall_a,
             self.c.wall_lam) = (float(v) for v in wall)

    @property
    def shape(self):
        return (self.c.nz, self.c.ny, self.c.nx)

    def ref(self):
        return ctypes.byref(self.c)


def wall_fraction(params, x, y, z, i):
    """Fraction of the link from fluid node (x, y, z) along c_i at which it
    leaves the tube of params' interpolated walls."""
    return _lib().orc3_wall_fraction(params.ref(), int(x), int(y), int(z), int(i))


def step_once(params, mask, f):
    """One step of an explicit population array; returns (f_new, bad_count)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    rho = np.zeros((2,) + params.shape)
    bad = _lib().orc3_step(params.ref(), _u8(np.ascontiguousarray(mask, dtype=np.uint8)),
                           _dp(f), _dp(out), _dp(rho))
    return out, bad


class Lattice3:
    """A two-species D3Q19 oracle lattice: parameters, fluid mask and state."""

    def __init__(self, params, mask, rho0):
        self.p = params
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        assert self.mask.shape == params.shape
        n = self.mask.size
        self.f = np.zeros((2, Q3) + params.shape)
        self.work = np.zeros(2 * Q3 * n + 2 * n)
        self.t = 0
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        assert rho0.shape == (2,) + params.shape
        _lib().orc3_init(params.ref(), _u8(self.mask), _dp(rho0), _dp(self.f))

    def step(self, nsteps=1):
        bad = _lib().orc3_run(self.p.ref(), _u8(self.mask), _dp(self.f), _dp(self.work),
                              int(nsteps))
        if bad >= 0:
            self.t += int(bad) + 1
            raise FloatingPointError("oracle state became non-physical at step %d" % self.t)
        self.t += int(nsteps)

    def set_body_force(self, gx, gy=0.0, gz=0.0):
        self.p.c.g[0], self.p.c.g[1], self.p.c.g[2] = float(gx), float(gy), float(gz)

    def moments(self):
        """dict rho [2,nz,ny,nx], u [3,nz,ny,nx] (physical), p [nz,ny,nx], mon [8]."""
        sh = self.p.shape
        rho = np.zeros((2,) + sh)
        u = np.zeros((3,) + sh)
        pr = np.zeros(sh)
        mon = np.zeros(8)
        rw = np.zeros((2,) + sh)
        _lib().orc3_moments(self.p.ref(), _u8(self.mask), _dp(self.f), _dp(rw), _dp(rho),
                            _dp(u), _dp(pr), _dp(mon))
        return {"rho": rho, "u": u, "p": pr, "mon": mon}

    def copy_state(self):
        return self.f.copy(), self.t

    def restore_state(self, state):
        self.f[...] = state[0]
        self.t = state[1]
