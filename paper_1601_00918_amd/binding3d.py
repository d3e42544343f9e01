"""Thin Python binding over the D3Q19 C ABI (include/lbm3d.h).

Argument marshalling only; torch provides the device workspace and the HIP
stream.  Function names follow the ABI."""
import ctypes

import numpy as np

from . import _lib
from .binding import workspace_on
from ._lib import (GEOM3_BOX, GEOM3_MASK, GEOM3_TUBE, INIT3_DROPLET, INIT3_SLUG, INIT3_UNIFORM,
                   OPT_SNAPSHOT, STORE_BF16, STORE_F16, STORE_F32, Lbm3dCpProblem, Lbm3dFluid,
                   Lbm3dGeom, Lbm3dInitFields, LbmCpOptions, LbmCpResult, LbmMonitor, check)

_GEOM_KINDS = {"box3d": GEOM3_BOX, "box": GEOM3_BOX, "tube": GEOM3_TUBE, "mask": GEOM3_MASK}
_INIT_KINDS = {"uniform": INIT3_UNIFORM, "droplet": INIT3_DROPLET, "slug": INIT3_SLUG}
_STORAGE = {"f32": STORE_F32, "f16": STORE_F16, "bf16": STORE_BF16}


def geom3_struct(kind, nx, ny, nz, lam=0.0, r0=0.0, a=0.0, mask=None, _keep=None,
                 wall_interp=False):
    g = Lbm3dGeom()
    g.kind = _GEOM_KINDS[kind] if isinstance(kind, str) else int(kind)
    g.nx, g.ny, g.nz = int(nx), int(ny), int(nz)
    g.lam, g.r0, g.a = float(lam), float(r0), float(a)
    g.wall_interp = 1 if wall_interp else 0
    if mask is not None:
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        assert m.shape == (nz, ny, nx)
        if _keep is not None:
            _keep.append(m)
        g.mask = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    return g


def fluid3_struct(tau, G, rho_s=(0.0, 0.0), g=(0.0, 0.0, 0.0)):
    f = Lbm3dFluid()
    f.tau[0], f.tau[1] = float(tau[0]), float(tau[1])
    f.G = float(G)
    f.rho_s[0], f.rho_s[1] = float(rho_s[0]), float(rho_s[1])
    for a in range(3):
        f.g[a] = float(g[a])
    return f


def init3_struct(kind, rho_hi=1.0, rho_lo=0.03, cx=0.0, cy=0.0, cz=0.0, r=0.0, x0=0.0,
                 length=0.0, slugs=None, width=0.0, _keep=None):
    """slugs: optional list of (x0, length) pairs (several slugs in series);
    width: tanh width of the slug interfaces (0: a step)."""
    s = Lbm3dInitFields()
    s.kind = _INIT_KINDS[kind] if isinstance(kind, str) else int(kind)
    s.rho_hi, s.rho_lo = float(rho_hi), float(rho_lo)
    s.cx, s.cy, s.cz, s.r = float(cx), float(cy), float(cz), float(r)
    s.x0, s.length = float(x0), float(length)
    s.width = float(width)
    if slugs is not None:
        a = np.ascontiguousarray(slugs, dtype=np.float64).reshape(-1, 2)
        s.n_slugs = a.shape[0]
        s.slugs = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s._slugs = a
        if _keep is not None:
            _keep.append(a)
    return s


def structs3_from_config(cfg, keep=None, rho_hi=None, rho_lo=None):
    """(geom, fluid, init) structs from a 3-D workload dict (box3d, tube or mask)."""
    kind = cfg["kind"]
    geom = geom3_struct(kind, cfg["nx"], cfg["ny"], cfg["nz"], cfg.get("lam", 0.0),
                        cfg.get("r0", 0.0), cfg.get("a", 0.0), cfg.get("mask"), keep,
                        wall_interp=cfg.get("wall_interp", False))
    fluid = fluid3_struct(cfg["tau"], cfg["G"], cfg.get("rho_s", (0, 0)),
                          cfg.get("g", (0, 0, 0)))
    ini = dict(cfg["init"])
    ikind = ini.pop("kind")
    if rho_hi is not None:
        ini["rho_hi"] = rho_hi
    if rho_lo is not None:
        ini["rho_lo"] = rho_lo
    init = init3_struct(ikind, _keep=keep, **ini)
    return geom, fluid, init


def _storage_code(storage, snapshot=False):
    return _STORAGE[storage] | (OPT_SNAPSHOT if snapshot else 0)


def lbm3d_required_bytes(geom, storage="f32", snapshot=False):
    n = ctypes.c_size_t()
    check(_lib.load().lbm3d_required_bytes(ctypes.byref(geom), _storage_code(storage, snapshot),
                                           ctypes.byref(n)), "lbm3d_required_bytes")
    return n.value


def lbm3d_init(geom, fluid, init, storage, workspace_ptr, workspace_bytes, stream_ptr,
               snapshot=False):
    ctx = ctypes.c_void_p()
    check(_lib.load().lbm3d_init(ctypes.byref(geom), ctypes.byref(fluid), ctypes.byref(init),
                                 _storage_code(storage, snapshot), ctypes.c_void_p(workspace_ptr),
                                 workspace_bytes, ctypes.c_void_p(stream_ptr),
                                 ctypes.byref(ctx)), "lbm3d_init")
    return ctx


def lbm3d_step(ctx, nsteps):
    check(_lib.load().lbm3d_step(ctx, int(nsteps)), "lbm3d_step")


def lbm3d_time(ctx):
    return _lib.load().lbm3d_time(ctx)


def lbm3d_set_fluid(ctx, fluid):
    check(_lib.load().lbm3d_set_fluid(ctx, ctypes.byref(fluid)), "lbm3d_set_fluid")


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _monitor_dict(m):
    return {"mass": (m.mass[0], m.mass[1]), "momentum": (m.momentum[0], m.momentum[1]),
            "oil_flux": m.oil_flux, "oil_cos": m.oil_cos, "oil_sin": m.oil_sin,
            "bad_nodes": m.bad_nodes}


def lbm3d_moments(ctx, nx, ny, nz):
    rho = np.zeros((2, nz, ny, nx))
    u = np.zeros((3, nz, ny, nx))
    p = np.zeros((nz, ny, nx))
    mon = LbmMonitor()
    check(_lib.load().lbm3d_moments(ctx, _dp(rho), _dp(u), _dp(p), ctypes.byref(mon)),
          "lbm3d_moments")
    return {"rho": rho, "u": u, "p": p, "mon": _monitor_dict(mon)}


def lbm3d_monitors(ctx):
    mon = LbmMonitor()
    check(_lib.load().lbm3d_monitors(ctx, ctypes.byref(mon)), "lbm3d_monitors")
    return _monitor_dict(mon)


def lbm3d_get_populations(ctx, nx, ny, nz):
    f = np.zeros((2, 19, nz, ny, nx))
    check(_lib.load().lbm3d_get_populations(ctx, _dp(f)), "lbm3d_get_populations")
    return f


def lbm3d_fluid_mask(ctx, nx, ny, nz):
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    check(_lib.load().lbm3d_fluid_mask(ctx, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))),
          "lbm3d_fluid_mask")
    return m


def lbm3d_set_tiling(ctx, bx, by, strip_planes):
    check(_lib.load().lbm3d_set_tiling(ctx, int(bx), int(by), int(strip_planes)),
          "lbm3d_set_tiling")


def lbm3d_get_tiling(ctx):
    v = [ctypes.c_int32() for _ in range(4)]
    check(_lib.load().lbm3d_get_tiling(ctx, *[ctypes.byref(x) for x in v]), "lbm3d_get_tiling")
    return tuple(x.value for x in v)


def lbm3d_snapshot_save(ctx):
    check(_lib.load().lbm3d_snapshot_save(ctx), "lbm3d_snapshot_save")


def lbm3d_snapshot_restore(ctx):
    check(_lib.load().lbm3d_snapshot_restore(ctx), "lbm3d_snapshot_restore")


def lbm3d_destroy(ctx):
    _lib.load().lbm3d_destroy(ctx)


def cp3_problem(cfg, g_lo, g_hi, sigma, rho_bar, equil_steps, max_steps, min_steps=0):
    """Tube critical-pressure problem from a tube workload dict."""
    keep = []  # host arrays the structs point to, alive as long as the problem
    g, f, i = structs3_from_config(cfg, keep)
    p = Lbm3dCpProblem()
    p.geom, p.fluid, p.init = g, f, i
    p._keep = keep
    p.sigma, p.rho_bar = float(sigma), float(rho_bar)
    p.g_lo, p.g_hi = float(g_lo), float(g_hi)
    p.equil_steps, p.max_steps = int(equil_steps), int(max_steps)
    p.min_steps = int(min_steps)
    return p


def lbm3d_cp_required_bytes(problems, storage="f32"):
    n = ctypes.c_size_t()
    arr = (Lbm3dCpProblem * len(problems))(*problems)
    check(_lib.load().lbm3d_cp_required_bytes(arr, len(problems), _STORAGE[storage],
                                              ctypes.byref(n)), "lbm3d_cp_required_bytes")
    return n.value


def lbm3d_critical_pressure(problems, opts=None, device="cuda", stream=None):
    """Solve tube problems on the GPU; returns a list of result dicts."""
    import torch  # device memory and streams only

    from .binding import _result_dict, cp_options
    o = opts if opts is not None else cp_options()
    storage = {STORE_F32: "f32", STORE_F16: "f16", STORE_BF16: "bf16"}[o.storage]
    nbytes = lbm3d_cp_required_bytes(problems, storage)
    st = stream if stream is not None else torch.cuda.Stream(torch.device(device))
    ws = workspace_on(st, nbytes, device)
    res = (LbmCpResult * len(problems))()
    arr = (Lbm3dCpProblem * len(problems))(*problems)
    check(_lib.load().lbm3d_critical_pressure(arr, len(problems), ctypes.byref(o),
                                              ctypes.c_void_p(ws.data_ptr()), nbytes,
                                              ctypes.c_void_p(st.cuda_stream), res),
          "lbm3d_critical_pressure")
    del ws
    return [_result_dict(r) for r in res]


# D3Q19 velocities in the library's numbering (include/lbm3d.h).
C3 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
               [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
               [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])


class Simulation3D:
    """A D3Q19 context plus the torch device workspace that backs it.

    cfg: a 3-D workload dict (keys kind = box3d / tube / mask, nx, ny, nz, lam,
    r0, a, mask, tau, G, rho_s, g, init)."""

    def __init__(self, cfg, storage="f32", device="cuda", snapshot=False, stream=None):
        import torch  # device memory and streams only

        _lib.load()
        self.cfg = dict(cfg)
        keep = []
        geom, fluid, init = structs3_from_config(self.cfg, keep)
        self.fluid = fluid
        self.shape = (int(cfg["nz"]), int(cfg["ny"]), int(cfg["nx"]))
        nbytes = lbm3d_required_bytes(geom, storage, snapshot)
        self.workspace = workspace_on(stream, nbytes, device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(
            self.workspace.device)
        self.ctx = lbm3d_init(geom, fluid, init, storage, self.workspace.data_ptr(), nbytes,
                              self.stream.cuda_stream, snapshot)
        self.workspace_bytes = nbytes
        del keep

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx and _lib is not None and _lib._LIB is not None:
            _lib._LIB.lbm3d_destroy(ctx)
        self.ctx = None

    @property
    def t(self):
        return lbm3d_time(self.ctx)

    def step(self, nsteps=1):
        lbm3d_step(self.ctx, nsteps)

    def set_body_force(self, gx, gy=0.0, gz=0.0):
        self.fluid.g[0], self.fluid.g[1], self.fluid.g[2] = float(gx), float(gy), float(gz)
        lbm3d_set_fluid(self.ctx, self.fluid)

    def moments(self):
        nz, ny, nx = self.shape
        return lbm3d_moments(self.ctx, nx, ny, nz)

    def monitors(self):
        return lbm3d_monitors(self.ctx)

    def populations(self):
        nz, ny, nx = self.shape
        return lbm3d_get_populations(self.ctx, nx, ny, nz)

    def fluid_mask(self):
        nz, ny, nx = self.shape
        return lbm3d_fluid_mask(self.ctx, nx, ny, nz)

    def set_tiling(self, bx, by, strip_planes):
        lbm3d_set_tiling(self.ctx, bx, by, strip_planes)

    def tiling(self):
        return lbm3d_get_tiling(self.ctx)

    def snapshot_save(self):
        lbm3d_snapshot_save(self.ctx)

    def snapshot_restore(self):
        lbm3d_snapshot_restore(self.ctx)
