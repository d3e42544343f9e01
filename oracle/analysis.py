"""Measurement procedures of Sec. 3 applied to density / pressure fields.

TEST INFRASTRUCTURE (see the package docstring).  Fields may come from the
oracle or from the HIP library; these functions only post-process them.
"""
import math

import numpy as np
from scipy.optimize import curve_fit


def bond_number(rho, g, L, D, sigma):
    """Eq. 15: ratio of the driving to the capillary force, rho g L D / sigma."""
    return rho * g * L * D / sigma


def tanh_profile(x, c1, c2, c3, c4):
    """Eq. 12: rho(x) = C1 tanh(C2 (x - C3)) + C4."""
    return c1 * np.tanh(c2 * (x - c3)) + c4


def fit_interface(x, rho, guess_pos):
    """Fit Eq. 12 to a density profile crossing one interface near guess_pos;
    returns (C1, C2, C3, C4) with C3 the interface position."""
    x = np.asarray(x, dtype=float)
    rho = np.asarray(rho, dtype=float)
    c1 = 0.5 * (rho.max() - rho.min())
    c4 = 0.5 * (rho.max() + rho.min())
    left = rho[np.argmin(np.abs(x - (guess_pos - 3)))]
    sign = -1.0 if left > c4 else 1.0
    p, _ = curve_fit(tanh_profile, x, rho, p0=(c1, sign * 0.5, guess_pos, c4), maxfev=20000)
    return p


def droplet_radius_from_mass(rho_o, rho_hi, rho_lo):
    """Radius of a 2-D droplet from its oil mass: the area whose density is
    rho_hi instead of rho_lo, A = (sum rho_o - rho_lo N) / (rho_hi - rho_lo)."""
    area = (rho_o.sum() - rho_lo * rho_o.size) / (rho_hi - rho_lo)
    return math.sqrt(area / math.pi)


def laplace_fit(inv_r, dp):
    """Least-squares line dP = sigma / R + b (Eq. 11); returns (sigma, b, R^2)."""
    inv_r = np.asarray(inv_r, dtype=float)
    dp = np.asarray(dp, dtype=float)
    A = np.stack([inv_r, np.ones_like(inv_r)], axis=1)
    (s, b), *_ = np.linalg.lstsq(A, dp, rcond=None)
    pred = A @ np.array([s, b])
    ss_res = float(((dp - pred) ** 2).sum())
    ss_tot = float(((dp - dp.mean()) ** 2).sum())
    return float(s), float(b), 1.0 - ss_res / ss_tot


def two_layer_poiseuille(eta, h, b, g, nu_core, nu_wall):
    """Steady velocity of two immiscible layers of equal density between plates
    at eta = +-h, interface at |eta| = b, body acceleration g: the wall layer
    u = g (h^2 - eta^2) / (2 nu_wall), the core
    u = g (b^2 - eta^2) / (2 nu_core) + g (h^2 - b^2) / (2 nu_wall)."""
    eta = np.abs(np.asarray(eta, dtype=float))
    wall = g * (h * h - eta * eta) / (2.0 * nu_wall)
    core = g * (b * b - eta * eta) / (2.0 * nu_core) + g * (h * h - b * b) / (2.0 * nu_wall)
    return np.where(eta >= b, wall, core)


def variable_viscosity_profile(eta, rho, nu, g, h, n_fine=20001):
    """Steady unidirectional flow between no-slip plates at eta = +-h for a
    fluid whose density rho(eta) and kinematic viscosity nu(eta) vary across
    the channel (given at the nodes eta, linearly interpolated): integrating
    d/deta (rho nu du/deta) = -rho g with du/deta = 0 at eta = 0 and u = 0 at
    the walls gives u(eta) = int_|eta|^h S(e) / (rho nu)(e) de with
    S(e) = int_0^e rho g.  Returns u at the nodes."""
    eta = np.asarray(eta, dtype=float)
    order = np.argsort(eta)
    eta_s = eta[order]
    e = np.linspace(0.0, h, n_fine)
    # symmetrise about the centre line
    r = 0.5 * (np.interp(e, eta_s, np.asarray(rho, float)[order])
               + np.interp(-e, eta_s, np.asarray(rho, float)[order]))
    v = 0.5 * (np.interp(e, eta_s, np.asarray(nu, float)[order])
               + np.interp(-e, eta_s, np.asarray(nu, float)[order]))
    de = e[1] - e[0]
    S = np.concatenate([[0.0], np.cumsum(0.5 * (r[1:] + r[:-1]) * g * de)])
    integrand = S / (r * v)
    tail = np.concatenate([np.cumsum((0.5 * (integrand[1:] + integrand[:-1]) * de)[::-1])[::-1],
                           [0.0]])
    return np.interp(np.abs(eta), e, tail)


def circle_fit(x, y):
    """Algebraic least-squares circle through points; returns (xc, yc, R)."""
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    A = np.stack([x, y, np.ones_like(x)], axis=1)
    rhs = x * x + y * y
    (a, b, c), *_ = np.linalg.lstsq(A, rhs, rcond=None)
    xc, yc = a / 2.0, b / 2.0
    return xc, yc, math.sqrt(c + xc * xc + yc * yc)


def contact_angle(R, y0, centre_on_oil_side):
    """Eq. 14 at the contact point of an arc of radius R spanning a channel of
    half width y0: the tangent makes acos(y0 / R) with the wall (the arctan
    form of Eq. 14 is the same angle).  The angle through water is that value
    when the arc's centre lies on the oil side, else its supplement."""
    a = math.degrees(math.acos(min(1.0, y0 / R)))
    return a if centre_on_oil_side else 180.0 - a


def meniscus_contact_angle(frac, mask, x_guess, oil_left, window=8, walls=None):
    """Sec. 3.3 contact-angle detection on a slug between flat plates.

    frac: oil fraction rho^o / (rho^o + rho^w), [ny][nx]; mask: fluid mask;
    x_guess: approximate meniscus position; oil_left: True when oil is on the
    meniscus's -x side.  Interfacial points: for every fluid row except the two
    next to the walls, Eq. 12 fitted along x within x_guess +- window.  A circle
    is fitted to the points and Eq. 14 applied with y0 the half width of the
    channel (the walls sit half-way between the last fluid row and the solid
    row beyond it; walls = (y_c, y0) gives the centre line and half width of
    walls placed off the lattice instead).  Returns (theta through water in
    degrees, R, points)."""
    frac = np.asarray(frac, dtype=float)
    rows = np.nonzero(np.asarray(mask, dtype=bool).any(axis=1))[0]
    lo, hi = rows.min(), rows.max()
    y0 = 0.5 * (hi - lo + 1)
    yc = 0.5 * (lo + hi)
    if walls is not None:
        yc, y0 = float(walls[0]), float(walls[1])
    xs, ys = [], []
    nx = frac.shape[1]
    x = np.arange(int(round(x_guess)) - window, int(round(x_guess)) + window + 1)
    for yy in range(lo + 1, hi):
        prof = frac[yy, np.mod(x, nx)]
        c = fit_interface(x, prof, x_guess)
        xs.append(c[2])
        ys.append(yy - yc)
    xc, ycc, R = circle_fit(xs, ys)
    mean_x = float(np.mean(xs))
    centre_on_oil = (xc < mean_x) if oil_left else (xc > mean_x)
    return contact_angle(R, y0, centre_on_oil), R, (np.array(xs), np.array(ys))


def tube_meniscus_contact_angle(frac, mask, x_guess, oil_left, window=8, axis=None):
    """Sec. 3.3 contact-angle detection carried to a slug in a straight tube
    (the axisymmetric counterpart of meniscus_contact_angle).

    frac: oil fraction [nz][ny][nx]; mask: fluid mask [nz][ny][nx] of a tube
    along x with the same cross-section at every x; axis = (y_c, z_c), default
    the box centre.  Eq. 12 is fitted along x on every fluid line of the
    cross-section whose four in-plane neighbours are fluid (the ring next to
    the wall is left out, as the rows next to the walls are in the planar
    case), a sphere centred on the axis is fitted to the interface points in
    the meridian plane, (x - x_c)^2 + r^2 = R^2, and Eq. 14 is applied with
    the tube radius r_w = sqrt(A / pi), A the number of fluid nodes in the
    cross-section (the area the half-way walls enclose).  Returns (theta
    through water in degrees, R, (x points, r points))."""
    frac = np.asarray(frac, dtype=float)
    sec = np.asarray(mask, dtype=bool)[:, :, 0]
    nz, ny, nx = frac.shape
    if axis is None:
        axis = (0.5 * (ny - 1), 0.5 * (nz - 1))
    r_w = math.sqrt(float(sec.sum()) / math.pi)
    inner = sec.copy()
    inner[1:, :] &= sec[:-1, :]
    inner[:-1, :] &= sec[1:, :]
    inner[:, 1:] &= sec[:, :-1]
    inner[:, :-1] &= sec[:, 1:]
    inner[0, :] = inner[-1, :] = False
    inner[:, 0] = inner[:, -1] = False
    x = np.arange(int(round(x_guess)) - window, int(round(x_guess)) + window + 1)
    xs, rs = [], []
    for z, y in zip(*np.nonzero(inner)):
        prof = frac[z, y, np.mod(x, nx)]
        c = fit_interface(x, prof, x_guess)
        xs.append(c[2])
        rs.append(math.hypot(y - axis[0], z - axis[1]))
    xs, rs = np.array(xs), np.array(rs)
    A = np.stack([2.0 * xs, np.ones_like(xs)], axis=1)
    (xc, c), *_ = np.linalg.lstsq(A, xs * xs + rs * rs, rcond=None)
    R = math.sqrt(c + xc * xc)
    mean_x = float(np.mean(xs))
    centre_on_oil = (xc < mean_x) if oil_left else (xc > mean_x)
    return contact_angle(R, r_w, centre_on_oil), R, (xs, rs)
