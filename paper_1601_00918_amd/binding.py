"""Thin Python binding over the C ABI (include/lbm.h).

Argument marshalling only: numpy arrays are passed as host pointers, torch
provides the device workspace (``torch.empty(..., dtype=torch.uint8)``) and the
HIP stream (``torch.cuda.current_stream().cuda_stream``).
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import (CP_ADVANCE, CP_BEGIN, CP_MONITORS, CP_RAMP, CP_SET_FORCING, GEOM_BOX, GEOM_CHANNEL, GEOM_MASK,
                   INIT_DROPLET, INIT_LAYERS, INIT_SLUG, INIT_UNIFORM, OPT_SNAPSHOT,
                   STORE_BF16, STORE_F16, STORE_F32, LbmCpEngine, LbmCpOptions, LbmCpProblem,
                   LbmCpResult, LbmFluid, LbmGeom, LbmInitFields, LbmMonitor, LbmTuneReport,
                   check)

_GEOM_KINDS = {"box": GEOM_BOX, "channel": GEOM_CHANNEL, "mask": GEOM_MASK}
_INIT_KINDS = {"uniform": INIT_UNIFORM, "droplet": INIT_DROPLET, "layers": INIT_LAYERS,
               "slug": INIT_SLUG}
_STORAGE = {"f32": STORE_F32, "f16": STORE_F16, "bf16": STORE_BF16}


def lbm_version():
    return _lib.load().lbm_version().decode()


# ------------------------------------------------------------- structs -------
def geom_struct(kind, nx, ny, lam=0.0, h0=0.0, a=0.0, mask=None, _keep=None, wall_interp=0,
                y_offset=0.0, island=(0.0, 0.0)):
    g = LbmGeom()
    g.kind = _GEOM_KINDS[kind] if isinstance(kind, str) else int(kind)
    g.nx, g.ny = int(nx), int(ny)
    g.lam, g.h0, g.a = float(lam), float(h0), float(a)
    g.wall_interp, g.y_offset = int(wall_interp), float(y_offset)
    g.island_h, g.island_len = float(island[0]), float(island[1])
    if mask is not None:
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        assert m.shape == (ny, nx)
        if _keep is not None:
            _keep.append(m)
        g.mask = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    return g


def fluid_struct(tau, G, rho_s=(0.0, 0.0), g=(0.0, 0.0), reg_order=2):
    f = LbmFluid()
    f.tau[0], f.tau[1] = float(tau[0]), float(tau[1])
    f.G = float(G)
    f.rho_s[0], f.rho_s[1] = float(rho_s[0]), float(rho_s[1])
    f.g[0], f.g[1] = float(g[0]), float(g[1])
    f.reg_order = int(reg_order)
    return f


def init_struct(kind, rho_hi=1.0, rho_lo=0.03, cx=0.0, cy=0.0, r=0.0, wall_rows=0,
                core_species=0, x0=0.0, length=0.0, slugs=None, width=0.0, _keep=None):
    """slugs: optional list of (x0, length) pairs (several slugs in series);
    width: tanh width of the slug interfaces (0: a step)."""
    s = LbmInitFields()
    s.kind = _INIT_KINDS[kind] if isinstance(kind, str) else int(kind)
    s.rho_hi, s.rho_lo = float(rho_hi), float(rho_lo)
    s.cx, s.cy, s.r = float(cx), float(cy), float(r)
    s.wall_rows, s.core_species = int(wall_rows), int(core_species)
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


def structs_from_config(cfg, keep=None):
    """(geom, fluid, init) structs from a workload dict."""
    geom = geom_struct(cfg["kind"], cfg["nx"], cfg["ny"], cfg.get("lam", 0.0),
                       cfg.get("h0", 0.0), cfg.get("a", 0.0), cfg.get("mask"), keep,
                       cfg.get("wall_interp", 0), cfg.get("y_offset", 0.0),
                       cfg.get("island", (0.0, 0.0)))
    fluid = fluid_struct(cfg["tau"], cfg["G"], cfg.get("rho_s", (0, 0)), cfg.get("g", (0, 0)),
                         cfg.get("reg_order", 2))
    ini = dict(cfg["init"])
    kind = ini.pop("kind")
    init = init_struct(kind, _keep=keep, **ini)
    return geom, fluid, init


# ------------------------------------------------------------- ABI calls -----
def _arr(structs, typ):
    a = (typ * len(structs))()
    for k, s in enumerate(structs):
        a[k] = s
    return a


def _storage_code(storage, snapshot=False):
    return _STORAGE[storage] | (OPT_SNAPSHOT if snapshot else 0)


def lbm_required_bytes(geoms, storage="f32", snapshot=False):
    n = ctypes.c_size_t()
    ga = _arr(geoms, LbmGeom)
    check(_lib.load().lbm_required_bytes(ga, len(geoms), _storage_code(storage, snapshot),
                                         ctypes.byref(n)), "lbm_required_bytes")
    return n.value


def lbm_init(geoms, fluids, inits, storage, workspace_ptr, workspace_bytes, stream_ptr,
             snapshot=False):
    ctx = ctypes.c_void_p()
    check(_lib.load().lbm_init(_arr(geoms, LbmGeom), _arr(fluids, LbmFluid),
                               _arr(inits, LbmInitFields), len(geoms),
                               _storage_code(storage, snapshot),
                               ctypes.c_void_p(workspace_ptr), workspace_bytes,
                               ctypes.c_void_p(stream_ptr), ctypes.byref(ctx)), "lbm_init")
    return ctx


def lbm_step(ctx, nsteps):
    check(_lib.load().lbm_step(ctx, int(nsteps)), "lbm_step")


def lbm_time(ctx):
    return _lib.load().lbm_time(ctx)


def lbm_set_fluid(ctx, inst, fluid):
    check(_lib.load().lbm_set_fluid(ctx, int(inst), ctypes.byref(fluid)), "lbm_set_fluid")


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _monitor_dict(m):
    return {"mass": (m.mass[0], m.mass[1]), "momentum": (m.momentum[0], m.momentum[1]),
            "oil_flux": m.oil_flux, "oil_cos": m.oil_cos, "oil_sin": m.oil_sin,
            "bad_nodes": m.bad_nodes}


def lbm_moments(ctx, inst, nx, ny):
    rho = np.zeros((2, ny, nx))
    u = np.zeros((2, ny, nx))
    p = np.zeros((ny, nx))
    mon = LbmMonitor()
    check(_lib.load().lbm_moments(ctx, int(inst), _dp(rho), _dp(u), _dp(p), ctypes.byref(mon)),
          "lbm_moments")
    return {"rho": rho, "u": u, "p": p, "mon": _monitor_dict(mon)}


def lbm_monitors(ctx, n_inst):
    arr = (LbmMonitor * n_inst)()
    check(_lib.load().lbm_monitors(ctx, arr), "lbm_monitors")
    return [_monitor_dict(m) for m in arr]


def lbm_get_populations(ctx, inst, nx, ny):
    f = np.zeros((2, 9, ny, nx))
    check(_lib.load().lbm_get_populations(ctx, int(inst), _dp(f)), "lbm_get_populations")
    return f


def lbm_fluid_mask(ctx, inst, nx, ny):
    m = np.zeros((ny, nx), dtype=np.uint8)
    check(_lib.load().lbm_fluid_mask(ctx, int(inst),
                                     m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))),
          "lbm_fluid_mask")
    return m


def lbm_set_tiling(ctx, bx, strip_rows):
    check(_lib.load().lbm_set_tiling(ctx, int(bx), int(strip_rows)), "lbm_set_tiling")


def lbm_get_tiling(ctx):
    bx, st, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(_lib.load().lbm_get_tiling(ctx, ctypes.byref(bx), ctypes.byref(st), ctypes.byref(n)),
          "lbm_get_tiling")
    return bx.value, st.value, n.value


def lbm_set_instance_tiling(ctx, inst, bx, strip_rows):
    check(_lib.load().lbm_set_instance_tiling(ctx, int(inst), int(bx), int(strip_rows)),
          "lbm_set_instance_tiling")


def lbm_get_instance_tiling(ctx, inst):
    bx, st = ctypes.c_int32(), ctypes.c_int32()
    check(_lib.load().lbm_get_instance_tiling(ctx, int(inst), ctypes.byref(bx), ctypes.byref(st)),
          "lbm_get_instance_tiling")
    return bx.value, st.value


def lbm_autotune(ctx, steps_per_trial=32):
    r = LbmTuneReport()
    check(_lib.load().lbm_autotune(ctx, int(steps_per_trial), ctypes.byref(r)), "lbm_autotune")
    return {"buckets": r.buckets, "trials": r.trials, "steps": r.steps,
            "ms_before": r.ms_before, "ms_after": r.ms_after}


def lbm_set_active(ctx, active):
    a = (ctypes.c_uint8 * len(active))(*[1 if v else 0 for v in active])
    check(_lib.load().lbm_set_active(ctx, a), "lbm_set_active")


def lbm_snapshot_save(ctx):
    check(_lib.load().lbm_snapshot_save(ctx), "lbm_snapshot_save")


def lbm_snapshot_restore(ctx, inst=-1):
    check(_lib.load().lbm_snapshot_restore(ctx, int(inst)), "lbm_snapshot_restore")


def lbm_destroy(ctx):
    _lib.load().lbm_destroy(ctx)


# ---------------------------------------------------------- critical pressure --
def cp_options(**overrides):
    """Default critical-pressure options (include/lbm.h) with overrides."""
    o = LbmCpOptions()
    _lib.load().lbm_cp_default_options(ctypes.byref(o))
    for k, v in overrides.items():
        if k == "storage" and isinstance(v, str):
            v = _STORAGE[v]
        if k == "protocol" and isinstance(v, str):
            v = {"bisect": 0, "ramp": CP_RAMP}[v]
        setattr(o, k, v)
    return o


def cp_problem(cfg, g_lo, g_hi, sigma, rho_bar, equil_steps, max_steps, keep=None,
               min_steps=0):
    """Critical-pressure problem from a channel workload dict (min_steps 0:
    the options' value)."""
    keep = [] if keep is None else keep  # host arrays the structs point to
    g, f, i = structs_from_config(cfg, keep)
    p = LbmCpProblem()
    p.geom, p.fluid, p.init = g, f, i
    p._keep = keep
    p.sigma, p.rho_bar = float(sigma), float(rho_bar)
    p.g_lo, p.g_hi = float(g_lo), float(g_hi)
    p.equil_steps, p.max_steps = int(equil_steps), int(max_steps)
    p.min_steps = int(min_steps)
    return p


def _result_dict(r):
    return {"g_lo": r.g_lo, "g_hi": r.g_hi, "g_crit": r.g_crit, "bo_crit": r.bo_crit,
            "probes": r.probes, "flags": r.flags, "steps": r.steps}


def lbm_cp_required_bytes(problems):
    n = ctypes.c_size_t()
    check(_lib.load().lbm_cp_required_bytes(_arr(problems, LbmCpProblem), len(problems),
                                            ctypes.byref(n)), "lbm_cp_required_bytes")
    return n.value


def lbm_critical_pressure(problems, opts=None, device="cuda", stream=None):
    """Solve the problems together on the GPU; returns a list of result dicts."""
    import torch  # device memory and streams only

    _lib.load()
    nbytes = lbm_cp_required_bytes(problems)
    st = stream if stream is not None else torch.cuda.Stream(torch.device(device))
    ws = workspace_on(st, nbytes, device)
    res = (LbmCpResult * len(problems))()
    o = opts if opts is not None else cp_options()
    check(_lib.load().lbm_critical_pressure(_arr(problems, LbmCpProblem), len(problems),
                                            ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()),
                                            nbytes, ctypes.c_void_p(st.cuda_stream), res),
          "lbm_critical_pressure")
    del ws
    return [_result_dict(r) for r in res]


def lbm_cp_drive(engine, problems, opts=None):
    """Run the library's driver on a Python engine object with methods
    begin_probe(k, g), advance(active_list, steps), monitors() -> list of
    monitor dicts (keys as returned by lbm_monitors), and, for the ramp
    protocol, set_forcing(k, g)."""
    n = len(problems)

    def _begin(user, k, g):
        try:
            engine.begin_probe(int(k), float(g))
            return 0
        except Exception:  # reported as an engine failure by the driver
            return 1

    def _advance(user, active, steps):
        try:
            engine.advance([active[k] for k in range(n)], int(steps))
            return 0
        except Exception:
            return 1

    def _monitors(user, out):
        try:
            for k, m in enumerate(engine.monitors()):
                out[k].mass[0], out[k].mass[1] = m["mass"]
                out[k].momentum[0], out[k].momentum[1] = m["momentum"]
                out[k].oil_flux, out[k].oil_cos = m["oil_flux"], m["oil_cos"]
                out[k].oil_sin, out[k].bad_nodes = m["oil_sin"], m["bad_nodes"]
            return 0
        except Exception:
            return 1

    def _set_forcing(user, k, g):
        try:
            engine.set_forcing(int(k), float(g))
            return 0
        except Exception:
            return 1

    sf = CP_SET_FORCING(_set_forcing) if hasattr(engine, "set_forcing") else CP_SET_FORCING()
    cb = LbmCpEngine(CP_BEGIN(_begin), CP_ADVANCE(_advance), CP_MONITORS(_monitors), None, sf)
    res = (LbmCpResult * n)()
    o = opts if opts is not None else cp_options()
    check(_lib.load().lbm_cp_drive(ctypes.byref(cb), _arr(problems, LbmCpProblem), n,
                                   ctypes.byref(o), res), "lbm_cp_drive")
    return [_result_dict(r) for r in res]


# ------------------------------------------------------------- convenience ---
def workspace_on(stream, nbytes, device):
    """A torch byte buffer allocated on the stream the library will use it on
    (torch's current stream if None), so the caching allocator orders its
    reuse after that stream's work: a block freed by other streams' pending
    kernels is never handed to it, and once freed it is handed out again only
    behind the library's queued work."""
    import torch  # device memory and streams only
    if stream is None:
        return torch.empty(nbytes, dtype=torch.uint8, device=device)
    with torch.cuda.stream(stream):
        return torch.empty(nbytes, dtype=torch.uint8, device=device)


class Simulation:
    """A context plus the torch device workspace that backs it.

    configs: list of workload dicts (keys nx, ny, kind, lam, h0, a, tau, G,
    rho_s, g, init; the initial state is the config's preset)."""

    def __init__(self, configs, storage="f32", device="cuda", snapshot=False, stream=None):
        import torch  # device memory and streams only

        _lib.load()
        self.configs = list(configs)
        keep = []
        geoms, fluids, inits = [], [], []
        for k, cfg in enumerate(self.configs):
            g, f, i = structs_from_config(cfg, keep)
            geoms.append(g)
            fluids.append(f)
            inits.append(i)
        self.fluids = fluids
        nbytes = lbm_required_bytes(geoms, storage, snapshot)
        self.workspace = workspace_on(stream, nbytes, device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(
            self.workspace.device)
        self.ctx = lbm_init(geoms, fluids, inits, storage, self.workspace.data_ptr(), nbytes,
                            self.stream.cuda_stream, snapshot)
        self.workspace_bytes = nbytes
        del keep

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx and _lib is not None and _lib._LIB is not None:
            _lib._LIB.lbm_destroy(ctx)
        self.ctx = None

    @property
    def n_inst(self):
        return len(self.configs)

    @property
    def t(self):
        return lbm_time(self.ctx)

    def step(self, nsteps=1):
        lbm_step(self.ctx, nsteps)

    def set_body_force(self, inst, gx, gy=0.0):
        f = self.fluids[inst]
        f.g[0], f.g[1] = float(gx), float(gy)
        lbm_set_fluid(self.ctx, inst, f)

    def moments(self, inst=0):
        c = self.configs[inst]
        return lbm_moments(self.ctx, inst, c["nx"], c["ny"])

    def monitors(self):
        return lbm_monitors(self.ctx, self.n_inst)

    def populations(self, inst=0):
        c = self.configs[inst]
        return lbm_get_populations(self.ctx, inst, c["nx"], c["ny"])

    def set_active(self, active):
        lbm_set_active(self.ctx, active)

    def snapshot_save(self):
        lbm_snapshot_save(self.ctx)

    def snapshot_restore(self, inst=-1):
        lbm_snapshot_restore(self.ctx, inst)

    def set_tiling(self, bx, strip_rows):
        lbm_set_tiling(self.ctx, bx, strip_rows)

    def tiling(self):
        return lbm_get_tiling(self.ctx)

    def set_instance_tiling(self, inst, bx, strip_rows):
        lbm_set_instance_tiling(self.ctx, inst, bx, strip_rows)

    def instance_tiling(self, inst):
        return lbm_get_instance_tiling(self.ctx, inst)

    def autotune(self, steps_per_trial=32):
        """Tune the tiling per width class; advances the run by the steps timed."""
        return lbm_autotune(self.ctx, steps_per_trial)

    def fluid_mask(self, inst=0):
        c = self.configs[inst]
        return lbm_fluid_mask(self.ctx, inst, c["nx"], c["ny"])
