"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds no lattice-Boltzmann arithmetic: only geometry voxelisation
(which nodes are fluid), initial density fields and the parameter sets of the
workloads.  Both sides of every parity test take their inputs from here.

Geometry conventions (cell centres at integer coordinates):
  * x is periodic with period nx.
  * sinusoidal channel: walls at y = y_c +- h(x), h(x) = h0 + a cos(2 pi x / lam),
    y_c = (ny - 1) / 2; a node is fluid iff |y - y_c| < h(x) (strict; equality
    is solid).  ny = 2 (h0 + a) + 2 leaves one solid row at each side.
  * flat channel: the a = 0 case; with ny = 66 and h0 = 32 the fluid rows are
    1..64, i.e. the wall planes sit half-way between nodes at y = 0.5, 64.5.
  * box: every node fluid, periodic in x and y.
Species 0 is oil (the "A" component), species 1 water ("B").
"""
import math

import numpy as np

RHO_HI = 1.0   # majority density of a component inside its own phase
RHO_LO = 0.03  # minority density of the same component in the other phase

# Interaction strength in the paper's sign convention (repulsion: G < 0).  The
# mean-field coexistence condition ln(rho_hi / rho_lo) = G_c (rho_hi - rho_lo)
# for 1.0 / 0.03 gives G_c = 3.615.  The workloads use G = -2.7 (past the
# spinodal G_c rho_tot = 2): it separates the species to about 1.12 / 0.003-0.026
# and keeps the viscosity-ratio-20 pairs tau = (0.55, 1.5) and (1.5, 0.55)
# stable from a sharp 1.0 / 0.03 start.
G_DEFAULT = -2.7


# ---------------------------------------------------------------- geometry ---
def channel_half_width(x, lam, h0, a):
    return h0 + a * np.cos(2.0 * np.pi * np.asarray(x, dtype=np.float64) / lam)


def channel_mask(nx, ny, lam, h0, a, y_offset=0.0, island=(0.0, 0.0)):
    """uint8 [ny, nx] fluid mask of a sinusoidal (a > 0) or flat (a = 0) channel
    whose centre line is y_c = (ny - 1) / 2 + y_offset.  island = (half-height
    s, length l): the nodes with |y - y_c| < s in the columns whose distance to
    the nearest multiple of lam is below l / 2 are solid, which splits the
    channel there into two branches (a bypass)."""
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    yc = 0.5 * (ny - 1) + y_offset
    h = channel_half_width(x, lam, h0, a)
    fluid = np.abs(y - yc) < h
    s, ln = island
    if s > 0 and ln > 0:
        r = np.mod(x, lam)
        fluid &= ~((np.minimum(r, lam - r) < 0.5 * ln) & (np.abs(y - yc) < s))
    return fluid.astype(np.uint8)


def box_mask(nx, ny):
    return np.ones((ny, nx), dtype=np.uint8)


# ---------------------------------------------------------- initial fields ---
def droplet_field(nx, ny, cx, cy, r, hi=RHO_HI, lo=RHO_LO):
    """rho0 [2, ny, nx]: species 0 = hi inside the disc (dist < r), lo outside;
    species 1 mirrored.  Distances use the periodic image nearest the centre."""
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    dx = np.abs(x - cx)
    dx = np.minimum(dx, nx - dx)
    dy = np.abs(y - cy)
    dy = np.minimum(dy, ny - dy)
    inside = (dx * dx + dy * dy) < r * r
    rho = np.empty((2, ny, nx))
    rho[0] = np.where(inside, hi, lo)
    rho[1] = np.where(inside, lo, hi)
    return rho


def layers_field(nx, ny, wall_rows, mask, core_species=0, hi=RHO_HI, lo=RHO_LO):
    """Two-layer channel: the 'wall_rows' fluid rows next to each wall belong to
    species 1 - core_species, the rest of the fluid to core_species."""
    rows = np.nonzero(mask.any(axis=1))[0]
    first, last = rows.min(), rows.max()
    y = np.arange(ny)[:, None] * np.ones((1, nx), dtype=np.int64)
    wall_layer = (y < first + wall_rows) | (y > last - wall_rows)
    core = ~wall_layer
    rho = np.empty((2, ny, nx))
    a, b = core_species, 1 - core_species
    rho[a] = np.where(core, hi, lo)
    rho[b] = np.where(core, lo, hi)
    rho *= mask[None, :, :]
    return rho


def slug_fraction(nx, x0, length, slugs=None, width=0.0):
    """Oil fraction phi(x) [nx] of slugs along x: 1 on [x0, x0 + length)
    (periodic), 0 elsewhere; with width > 0 the interfaces at x0 - 1/2 and
    x0 + length - 1/2 (and their images at +-nx) are hyperbolic tangents of
    that width, phi clipped to [0, 1]."""
    x = np.arange(nx, dtype=np.float64)
    phi = np.zeros(nx)
    for s0, sl in (slugs if slugs is not None else [(x0, length)]):
        if width > 0:
            a = np.mod(float(s0), nx)
            for img in (-1, 0, 1):
                xx = x + img * nx
                phi += 0.5 * (np.tanh((xx - a + 0.5) / width) -
                              np.tanh((xx - a - sl + 0.5) / width))
        else:
            phi = np.maximum(phi, (np.mod(x - s0, nx) < sl).astype(np.float64))
    return np.clip(phi, 0.0, 1.0)


def slug_field(nx, ny, x0, length, mask, hi=RHO_HI, lo=RHO_LO, slugs=None, width=0.0):
    """Oil slug: fluid nodes with x in [x0, x0 + length) (periodic) are oil;
    with slugs (a list of (x0, length) pairs) every listed slug is oil; with
    width > 0 the oil fraction follows slug_fraction's tanh interfaces."""
    phi = slug_fraction(nx, x0, length, slugs, width)[None, :] * np.ones((ny, 1))
    rho = np.empty((2, ny, nx))
    if width > 0:
        rho[0] = lo + (hi - lo) * phi
        rho[1] = hi - (hi - lo) * phi
    else:  # exactly hi / lo
        rho[0] = np.where(phi > 0, hi, lo)
        rho[1] = np.where(phi > 0, lo, hi)
    rho *= mask[None, :, :]
    return rho


def random_field(nx, ny, mask, seed, mean=(0.5, 0.5), amp=0.05):
    """Smoothly random densities (for tiny brute-force cross-checks)."""
    rng = np.random.default_rng(seed)
    rho = np.empty((2, ny, nx))
    for s in range(2):
        rho[s] = mean[s] * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(ny, nx)))
    return rho * mask[None, :, :]


def random_populations(nx, ny, mask, seed, amp=0.02):
    """Random non-equilibrium populations: w_i * rho0 * (1 + noise) per node.
    Returns f [2, 9, ny, nx] (float64); solid nodes are 0."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    rng = np.random.default_rng(seed)
    base = 0.2 + 0.8 * rng.uniform(size=(2, 1, ny, nx))
    f = w[None, :, None, None] * base * (1.0 + amp * rng.uniform(-1, 1, size=(2, 9, ny, nx)))
    return f * mask[None, None, :, :]


# -------------------------------------------------------------- wettability ---
WALL_SCALE = 0.5


def wall_potentials_for_angle(theta_deg, hi=RHO_HI, lo=RHO_LO, scale=WALL_SCALE):
    """First-guess wall potentials (rho_s^o, rho_s^w) for a contact angle theta
    measured through water.  The wall is made to look like a scaled mixture of
    the two bulk phases with oil fraction phi = (1 - cos theta) / 2:
        rho_s^o = scale ((1 - phi) lo + phi hi),  rho_s^w = scale (phi lo + (1 - phi) hi),
    so rho_s^w - rho_s^o = scale (hi - lo) cos theta, both potentials are
    positive, and theta = 90 deg gives equal potentials.  This is a starting
    map, not a calibration."""
    phi = 0.5 * (1.0 - math.cos(math.radians(theta_deg)))
    return (scale * ((1.0 - phi) * lo + phi * hi), scale * (phi * lo + (1.0 - phi) * hi))


# ------------------------------------------------------------------ configs ---
def config_droplet(n=128, r=20.0, tau=(1.0, 1.0), G=G_DEFAULT):
    """Free droplet on a periodic n x n box."""
    return dict(name="droplet", nx=n, ny=n, kind="box", lam=0.0, h0=0.0, a=0.0,
                tau=tau, G=G, rho_s=(0.0, 0.0), g=(0.0, 0.0),
                init=dict(kind="droplet", cx=n / 2, cy=n / 2, r=r))


def config_uniform(n=64, tau=(1.0, 1.0), G=G_DEFAULT):
    """Periodic n x n box of uniform oil (RHO_HI) with dissolved water (RHO_LO)."""
    return dict(name="uniform", nx=n, ny=n, kind="box", lam=0.0, h0=0.0, a=0.0,
                tau=tau, G=G, rho_s=(0.0, 0.0), g=(0.0, 0.0), init=dict(kind="uniform"))


def config_poiseuille(nx=256, width=64, tau=(0.6, 1.5), g=1e-6, wall_rows=16,
                      core_species=0, G=G_DEFAULT):
    """Two-layer Poiseuille: flat channel of `width` fluid rows, species
    1 - core_species in `wall_rows` rows next to each wall."""
    ny = width + 2
    return dict(name="poiseuille", nx=nx, ny=ny, kind="channel", lam=float(nx),
                h0=width / 2.0, a=0.0, tau=tau, G=G, rho_s=(0.0, 0.0), g=(g, 0.0),
                init=dict(kind="layers", wall_rows=wall_rows, core_species=core_species))


def config_channel(lam=256, theta=90.0, tau=(1.0, 1.0), g=0.0, G=G_DEFAULT, slug_len=None,
                   slug_x0=None, h0=None, a=None):
    """Sinusoidal channel of four wavelengths with an oil slug."""
    h0 = lam // 8 if h0 is None else h0
    a = lam // 16 if a is None else a
    nx = 4 * lam
    ny = 2 * (h0 + a) + 2
    slug_len = int(1.5 * lam) if slug_len is None else slug_len
    slug_x0 = lam // 4 if slug_x0 is None else slug_x0
    return dict(name="channel", nx=nx, ny=ny, kind="channel", lam=float(lam), h0=float(h0),
                a=float(a), tau=tau, G=G, rho_s=wall_potentials_for_angle(theta),
                g=(g, 0.0), theta=theta,
                init=dict(kind="slug", x0=slug_x0, length=slug_len))


def config_bypass(lam=64, theta=120.0, tau=(1.0, 1.0), g=0.0, G=G_DEFAULT, island_h=None,
                  island_len=None, slug_len=None, slug_x0=None):
    """Sinusoidal channel of the batch family (h0 = lam/8, a = lam/16) whose
    wide part holds a solid island of half-height lam/32 over lam/2 columns:
    there the channel splits into two branches, a bypass around the
    island.  The oil slug (1.5 lam from lam/4 by default) fills both branches
    where it crosses the islands."""
    cfg = config_channel(lam=lam, theta=theta, tau=tau, g=g, G=G, slug_len=slug_len,
                         slug_x0=slug_x0)
    cfg["island"] = (float(lam // 32 if island_h is None else island_h),
                     float(lam // 2 if island_len is None else island_len))
    cfg["name"] = "bypass"
    return cfg


def config_plates(H=32, theta=90.0, tau=(1.0, 1.0), G=G_DEFAULT, nx=None, rho_s=None,
                  offset=0.0):
    """An oil slug at rest between flat plates H nodes apart (a = 0 channel,
    walls half-way between the outermost fluid rows and the solid rows):
    nx = 4 H, slug of length nx / 2 from x = nx / 4.  rho_s overrides the
    wall-potential map.  offset (0 <= offset < 1) shifts both walls by that
    fraction of a lattice spacing relative to the lattice (with interpolated
    walls, wall_interp = 1; one more row of nodes is allotted)."""
    nx = 4 * H if nx is None else nx
    cfg = config_channel(lam=nx, theta=theta, tau=tau, G=G, h0=H // 2, a=0,
                         slug_len=nx // 2, slug_x0=nx // 4)
    cfg["nx"] = nx
    cfg["name"] = "plates"
    if offset:
        cfg["ny"] += 1
        cfg["y_offset"] = float(offset) - 0.5
        cfg["wall_interp"] = 1
    if rho_s is not None:
        cfg["rho_s"] = tuple(rho_s)
    return cfg


def config_batch(n_inst=256, seed=1601, lams=(64, 128, 256, 512), G=G_DEFAULT,
                 sigma=0.05, rho_bar=1.03):
    """The batch of uneven channels: lam ~ U{lams}, h0 = lam/8, a = lam/16,
    theta ~ U(30, 150) deg, viscosity ratio M = nu_o / nu_w ~ logU(0.1, 10)
    split symmetrically between the two relaxation times, Bond number
    ~ logU(10^-1.5, 10^1.5) converted to a body acceleration with the given
    surface-tension scale sigma: g = Bo sigma / (rho_bar * 4 lam * (h0 - a))."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_inst):
        lam = int(rng.choice(lams))
        theta = float(rng.uniform(30.0, 150.0))
        m = float(10.0 ** rng.uniform(-1.0, 1.0))
        bo = float(10.0 ** rng.uniform(-1.5, 1.5))
        tau = (0.5 + 0.5 * math.sqrt(m), 0.5 + 0.5 / math.sqrt(m))
        h0, a = lam // 8, lam // 16
        g = bo * sigma / (rho_bar * 4 * lam * (h0 - a))
        cfg = config_channel(lam=lam, theta=theta, tau=tau, g=g, G=G)
        cfg["M"] = m
        cfg["Bo"] = bo
        out.append(cfg)
    return out


def mask_of(cfg):
    if cfg["kind"] == "box":
        return box_mask(cfg["nx"], cfg["ny"])
    return channel_mask(cfg["nx"], cfg["ny"], cfg["lam"], cfg["h0"], cfg["a"],
                        cfg.get("y_offset", 0.0), cfg.get("island", (0.0, 0.0)))


def rho0_of(cfg, mask=None):
    mask = mask_of(cfg) if mask is None else mask
    ini = cfg["init"]
    nx, ny = cfg["nx"], cfg["ny"]
    if ini["kind"] == "droplet":
        return droplet_field(nx, ny, ini["cx"], ini["cy"], ini["r"])
    if ini["kind"] == "layers":
        return layers_field(nx, ny, ini["wall_rows"], mask, ini.get("core_species", 0))
    if ini["kind"] == "slug":
        return slug_field(nx, ny, ini.get("x0", 0.0), ini.get("length", 0.0), mask,
                          slugs=ini.get("slugs"), width=ini.get("width", 0.0))
    if ini["kind"] == "uniform":
        return np.stack([np.full((ny, nx), RHO_HI), np.full((ny, nx), RHO_LO)])
    raise ValueError(ini["kind"])


def mlp_init(seed=918, sizes=(6, 128, 128, 128, 1)):
    """Initial parameters of the surrogate network as one flat float32 vector
    (layout W1, b1, W2, b2, W3, b3, W4, b4, weights one row per output unit):
    weights uniform in +-1/sqrt(fan_in), biases zero, from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(sizes) - 1):
        k, n = sizes[i], sizes[i + 1]
        bound = 1.0 / math.sqrt(k)
        parts.append(rng.uniform(-bound, bound, size=n * k))
        parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)


def mlp_batch(n, seed=7, sizes=(6, 128, 128, 128, 1)):
    """Random standardised inputs [n, 6] and targets [n] (float32) for the
    network's parity tests."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, sizes[0])).astype(np.float32)
    t = rng.standard_normal(n).astype(np.float32)
    return X, t


def config_cp_set(n, seed, lams=(64,), theta=(30.0, 150.0), log10_m=(-1.0, 1.0)):
    """Critical-pressure problems: channels of the batch family (h0 = lam/8,
    a = lam/16, slug 1.5 lam), lam ~ U{lams}, theta ~ U(theta), viscosity
    ratio M = nu_o / nu_w ~ logU split symmetrically between the relaxation
    times (tau_o = 1/2 + sqrt(M)/2, tau_w = 1/2 + 1/(2 sqrt(M))), unforced."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        lam = int(rng.choice(lams))
        th = float(rng.uniform(*theta))
        m = float(10.0 ** rng.uniform(*log10_m))
        tau = (0.5 + 0.5 * math.sqrt(m), 0.5 + 0.5 / math.sqrt(m))
        cfg = config_channel(lam=lam, theta=th, tau=tau)
        cfg["M"] = m
        out.append(cfg)
    return out


# ---------------------------------------------------------------- 3-D (D3Q19) --
# Tube conventions (cell centres at integer coordinates): x periodic with
# period nx, axis at y_c = (ny - 1) / 2, z_c = (nz - 1) / 2, radius
# r(x) = r0 + a cos(2 pi x / lam); a node is fluid iff its squared distance to
# the axis is < r(x)^2.  3-D arrays are [nz][ny][nx] (x fastest).
def tube_mask(nx, ny, nz, lam, r0, a):
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    r = r0 + a * np.cos(2.0 * np.pi * x / lam)
    d2 = (y - 0.5 * (ny - 1)) ** 2 + (z - 0.5 * (nz - 1)) ** 2
    return (d2 < r * r).astype(np.uint8)


def config_tube(lam=64, r0=10.0, a=4.0, nx=None, ny=None, nz=None, theta=90.0,
                tau=(1.0, 1.0), g=0.0, G=G_DEFAULT, slug_len=None, slug_x0=None,
                wall_interp=False):
    """Sinusoidal tube (three wavelengths unless nx is given) with an oil slug;
    wall_interp: walls at their analytic position (interpolated bounce-back)."""
    nx = 3 * lam if nx is None else nx
    side = int(2 * (r0 + a) + 2)
    ny = side if ny is None else ny
    nz = side if nz is None else nz
    slug_len = int(1.5 * lam) if slug_len is None else slug_len
    slug_x0 = lam // 4 if slug_x0 is None else slug_x0
    return dict(name="tube", nx=nx, ny=ny, nz=nz, kind="tube", lam=float(lam), r0=float(r0),
                a=float(a), tau=tau, G=G, rho_s=wall_potentials_for_angle(theta),
                g=(g, 0.0, 0.0), theta=theta, init=dict(kind="slug", x0=slug_x0, length=slug_len),
                wall_interp=bool(wall_interp))


def config_box3d(n=32, r=8.0, tau=(1.0, 1.0), G=G_DEFAULT, kind="droplet"):
    """Periodic n^3 box: an oil sphere of radius r at the centre, or uniform."""
    init = dict(kind="droplet", cx=n / 2, cy=n / 2, cz=n / 2, r=r) if kind == "droplet" \
        else dict(kind="uniform")
    return dict(name="box3d", nx=n, ny=n, nz=n, kind="box3d", tau=tau, G=G,
                rho_s=(0.0, 0.0), g=(0.0, 0.0, 0.0), init=init)


def mask3_of(cfg):
    if cfg["kind"] == "box3d":
        return np.ones((cfg["nz"], cfg["ny"], cfg["nx"]), dtype=np.uint8)
    return tube_mask(cfg["nx"], cfg["ny"], cfg["nz"], cfg["lam"], cfg["r0"], cfg["a"])


def rho03_of(cfg, mask=None):
    """Initial densities [2][nz][ny][nx]: sphere (periodic distance), slug
    (fluid nodes with x in [x0, x0 + length), periodic) or uniform."""
    mask = mask3_of(cfg) if mask is None else mask
    nz, ny, nx = mask.shape
    ini = cfg["init"]
    if ini["kind"] == "uniform":
        oil = np.ones(mask.shape, dtype=bool)
    elif ini["kind"] == "droplet":
        x = np.arange(nx, dtype=np.float64)[None, None, :]
        y = np.arange(ny, dtype=np.float64)[None, :, None]
        z = np.arange(nz, dtype=np.float64)[:, None, None]

        def pd(v, c, n):
            d = np.abs(v - c)
            return np.minimum(d, n - d)
        oil = (pd(x, ini["cx"], nx) ** 2 + pd(y, ini["cy"], ny) ** 2 +
               pd(z, ini["cz"], nz) ** 2) < ini["r"] ** 2
    elif ini["kind"] == "slug":
        width = ini.get("width", 0.0)
        phi = slug_fraction(nx, ini.get("x0", 0.0), ini.get("length", 0.0), ini.get("slugs"),
                            width)
        phi = phi[None, None, :] * np.ones(mask.shape)
        if width <= 0:
            oil = phi > 0
        else:
            rho = np.empty((2,) + mask.shape)
            rho[0] = RHO_LO + (RHO_HI - RHO_LO) * phi
            rho[1] = RHO_HI - (RHO_HI - RHO_LO) * phi
            return rho * mask[None]
    else:
        raise ValueError(ini["kind"])
    rho = np.empty((2,) + mask.shape)
    rho[0] = np.where(oil, RHO_HI, RHO_LO)
    rho[1] = np.where(oil, RHO_LO, RHO_HI)
    return rho * mask[None]
