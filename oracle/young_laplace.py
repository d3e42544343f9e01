"""Quasi-static Young-Laplace critical pressure of a slug in a periodically
constricted channel or tube (the analytic comparison of Sec. 3.4, Eq. 16).

TEST INFRASTRUCTURE (see the package docstring).

The paper takes its analytic critical Bond numbers from Oh and Slattery's
curvature formulas, which are not reproduced in it.  This module derives the
same quantity from the Young-Laplace law (Eq. 11) and the contact angle
(Eq. 14) directly:

* The slug (oil) occupies x_r < x < x_f of a channel with half-width h(x)
  (planar) or a tube of radius r(x) (axisymmetric); water is on both sides and
  the driving force pushes in +x.  theta is measured through water.
* Each meniscus is a circular arc (planar) or spherical cap (axisymmetric)
  meeting the wall, whose slope angle is phi = atan(h'(x)), at the contact
  angle.  Working the tangent condition through gives the oil-minus-water
  capillary pressure
      front (oil on its -x side):  P_f = k sigma cos(theta - phi_f) / h_f
      rear  (oil on its +x side):  P_r = k sigma cos(theta + phi_r) / h_r
  with k = 1 (planar) or 2 (axisymmetric, h -> r).
* Static balance around the periodic domain: the body-force pressure rise
  rho g L equals the net capillary jump, Delta P = P_f - P_r.
* For each rear position x_r the front x_f follows from the fixed slug volume
  (wall-bounded volume between the contact lines plus the two signed caps).
  The critical Delta P is the maximum of Delta P(x_r) over one period, and
  Bo_crit = Delta P_crit D / sigma (Eq. 15, D the neck half-width / radius).
* Contact-angle variation (Sec. 3.4.2, Table 3's fifth column): the front and
  rear menisci may meet the wall at different angles theta_f, theta_r; with
  the angle known only to lie in a range [theta_lo, theta_hi] (Table 1's
  spread over wall offsets), the highest critical pressure over the pairs of
  angles in the range is the one compared with.
"""
import math

import numpy as np
from scipy.optimize import brentq, minimize_scalar


class Channel:
    """Wall profile h(x) = h0 + a cos(2 pi x / lam)."""

    def __init__(self, h0, a, lam, axisymmetric):
        self.h0, self.a, self.lam = float(h0), float(a), float(lam)
        self.axi = bool(axisymmetric)

    def h(self, x):
        return self.h0 + self.a * np.cos(2.0 * np.pi * x / self.lam)

    def slope_angle(self, x):
        return np.arctan(-self.a * 2.0 * np.pi / self.lam * np.sin(2.0 * np.pi * x / self.lam))

    def section(self, x):
        """Cross-section area (axisymmetric) or width (planar) at x."""
        h = self.h(x)
        return np.pi * h * h if self.axi else 2.0 * h

    def body_volume(self, x0, x1):
        """Wall-bounded volume (area) between x0 and x1, in closed form."""
        k = 2.0 * np.pi / self.lam
        h0, a = self.h0, self.a
        if self.axi:
            # integral of pi (h0 + a cos kx)^2
            def prim(x):
                return np.pi * (h0 * h0 * x + 2 * h0 * a * np.sin(k * x) / k
                                + a * a * (x / 2 + np.sin(2 * k * x) / (4 * k)))
        else:
            def prim(x):
                return 2.0 * (h0 * x + a * np.sin(k * x) / k)
        return prim(x1) - prim(x0)

    @property
    def neck(self):
        return self.h0 - abs(self.a)


def meniscus(channel, x, theta, front):
    """(capillary pressure / sigma, signed cap volume) of a meniscus at x."""
    h = float(channel.h(x))
    phi = float(channel.slope_angle(x))
    beta = theta - phi if front else theta + phi
    c = math.cos(beta)
    k = 2.0 if channel.axi else 1.0
    p = k * c / h
    if abs(c) < 1e-14:
        return p, 0.0
    R = h / abs(c)  # arc / sphere radius
    if channel.axi:
        s = R - math.sqrt(max(R * R - h * h, 0.0))
        vol = math.pi * s * s * (3.0 * R - s) / 3.0
    else:
        vol = R * R * math.asin(min(h / R, 1.0)) - h * math.sqrt(max(R * R - h * h, 0.0))
    return p, math.copysign(vol, c)


def slug_volume(channel, xr, xf, theta, theta_rear=None):
    """Wall-bounded volume between the contact lines plus the two signed caps
    (front meniscus at theta, rear at theta_rear, default theta)."""
    tr = theta if theta_rear is None else theta_rear
    _, vf = meniscus(channel, xf, theta, True)
    _, vr = meniscus(channel, xr, tr, False)
    return channel.body_volume(xr, xf) + vf + vr


def front_position(channel, xr, theta, volume, theta_rear=None):
    """x_f > x_r with slug_volume = volume (volume grows monotonically with x_f
    over the bracket searched)."""
    lo = xr + 1e-9
    hi = xr + 1e-3
    while slug_volume(channel, xr, hi, theta, theta_rear) < volume:
        hi += 0.25 * channel.lam
        if hi - xr > 20 * channel.lam:
            raise ValueError("slug volume not reachable")
    return brentq(lambda xf: slug_volume(channel, xr, xf, theta, theta_rear) - volume, lo, hi,
                  xtol=1e-12, rtol=1e-14)


def pressure_drop(channel, xr, theta, volume, theta_rear=None):
    """Delta P / sigma = (P_f - P_r) / sigma for the slug with rear at x_r
    (front angle theta, rear angle theta_rear, default theta; radians)."""
    tr = theta if theta_rear is None else theta_rear
    xf = front_position(channel, xr, theta, volume, theta_rear)
    pf, _ = meniscus(channel, xf, theta, True)
    pr, _ = meniscus(channel, xr, tr, False)
    return pf - pr


def critical_pressure(channel, theta_deg, volume, n_scan=241, theta_rear_deg=None):
    """max over rear positions of Delta P / sigma (the static slug gives way
    once the driving pressure exceeds it), front meniscus at theta_deg and rear
    at theta_rear_deg (default the same).  Returns (dP/sigma, x_r at max)."""
    th = math.radians(theta_deg)
    tr = None if theta_rear_deg is None else math.radians(theta_rear_deg)
    xs = np.linspace(0.0, channel.lam, n_scan, endpoint=False)
    vals = np.array([pressure_drop(channel, x, th, volume, tr) for x in xs])
    k = int(np.argmax(vals))
    step = channel.lam / n_scan
    res = minimize_scalar(lambda x: -pressure_drop(channel, x, th, volume, tr),
                          bounds=(xs[k] - step, xs[k] + step), method="bounded",
                          options={"xatol": 1e-9})
    best = max(vals[k], -res.fun)
    return best, (res.x if -res.fun >= vals[k] else xs[k])


def critical_pressure_range(channel, theta_lo_deg, theta_hi_deg, volume, n_scan=241):
    """Highest critical Delta P / sigma over front and rear angles in
    [theta_lo, theta_hi].  Each meniscus pressure is monotonic in its own
    angle (cos(theta -+ phi) over (0, pi)), so the highest value is taken at
    the ends of the range: all four pairs are evaluated.  Returns
    (dP/sigma, (theta_front, theta_rear) in degrees)."""
    best, arg = -np.inf, None
    for tf in (theta_lo_deg, theta_hi_deg):
        for tr in (theta_lo_deg, theta_hi_deg):
            dp, _ = critical_pressure(channel, tf, volume, n_scan, theta_rear_deg=tr)
            if dp > best:
                best, arg = dp, (tf, tr)
    return best, arg


def paper_tube(D=1.0):
    """The paper's sinusoidal tube in units of the neck radius D: three periods
    over L = 18 D, so lam = 6 D; radius D at the neck and 2.5 D at the widest
    section (neck / maximum = 0.4): r(x) = D (1.75 + 0.75 cos(2 pi x / lam))."""
    return Channel(1.75 * D, 0.75 * D, 6.0 * D, axisymmetric=True)


def bond_critical_tube(theta_deg, volume_over_D3):
    """Analytic critical Bond number Bo = Delta P D / sigma of the paper's tube
    for a slug of volume V0 / D^3 (Eq. 15-16)."""
    dp, _ = critical_pressure(paper_tube(1.0), theta_deg, volume_over_D3)
    return dp * 1.0


def bond_critical_tube_range(theta_lo_deg, theta_hi_deg, volume_over_D3):
    """Analytic critical Bond number of the paper's tube when the contact
    angle is known only to lie in [theta_lo, theta_hi] (the highest over the
    front and rear angles in the range)."""
    dp, _ = critical_pressure_range(paper_tube(1.0), theta_lo_deg, theta_hi_deg,
                                    volume_over_D3)
    return dp


def bond_critical_channel(lam, h0, a, theta_deg, area):
    """Planar analogue: channel walls y = +-(h0 + a cos(2 pi x / lam)), slug area
    `area` (lattice units).  Returns (Delta P_crit / sigma, Bo = dP D / sigma)
    with D = h0 - a."""
    ch = Channel(h0, a, lam, axisymmetric=False)
    dp, _ = critical_pressure(ch, theta_deg, area)
    return dp, dp * ch.neck
