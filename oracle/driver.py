"""Critical-pressure search on the oracle (Sec. 3.4): the smallest body
acceleration that mobilises the slug, by bisection in log g over probes that
restart from an equilibrated state.

TEST INFRASTRUCTURE (see the package docstring).  This is an independent
implementation of the probe rules the library documents (moving once the
slug's centre of oil mass has advanced by move_frac * lambda; static once
min_steps have run, the mean oil velocity has stayed below still_frac * U_ref
for still_chunks consecutive checks and the slug has advanced less than
creep_frac * lambda, U_ref = g h0^2 / (3 nu_w); at the step budget, static (it
did not advance move_frac * lambda); a non-physical state counts as moving;
stop when
(g_hi - g_lo) / g_lo <= rel_tol).  It shares no code with the library.

Bracket checks (verify_bracket): 0 trusts the given bracket; 1 probes g_lo
and then g_hi before bisecting, widening by sqrt(10) past an end that fails;
2 ("lazy") bisects first and probes an end of the given bracket only if the
converged bracket still has it as an end (it was never probed), widening by
sqrt(10) and bisecting on when it fails.
"""
import math

import numpy as np

UNDECIDED, UNSTABLE, WIDENED, NOT_CONVERGED = 1, 2, 4, 8

DEFAULT_RULES = dict(rel_tol=0.005, move_frac=0.5, creep_frac=0.25, still_frac=1e-3,
                     chunk_steps=1000, still_chunks=3, max_probes=60, verify_bracket=0,
                     min_steps=20000)


def _centre(mon, nx):
    """Periodic centre of oil mass (x) from the first circular moments."""
    return math.atan2(mon["oil_sin"], mon["oil_cos"]) / (2.0 * math.pi) * nx


def _wrap(d, nx):
    while d > 0.5 * nx:
        d -= nx
    while d <= -0.5 * nx:
        d += nx
    return d


def solve(engine, problems, **rules):
    """problems: list of dicts with nx, lam, h0, a, tau_w, g_lo, g_hi, max_steps,
    sigma, rho_bar (optional min_steps overriding the rule's).  engine: begin_probe(k, g), advance(active, steps),
    monitors() -> list of dicts (mass, oil_flux, oil_cos, oil_sin, bad_nodes).
    Returns a list of result dicts and, per problem, the probed g values."""
    R = dict(DEFAULT_RULES)
    R.update(rules)
    n = len(problems)
    mon = engine.monitors()
    x_start = [_centre(mon[k], problems[k]["nx"]) for k in range(n)]
    st = []
    for k, p in enumerate(problems):
        eager = R["verify_bracket"] == 1
        s = dict(lo=p["g_lo"], hi=p["g_hi"], widen=0, probes=0, flags=0, history=[],
                 phase="verify_lo" if eager else "bisect",
                 lo_ok=R["verify_bracket"] != 2, hi_ok=R["verify_bracket"] != 2)
        s["g"] = s["lo"] if eager else math.sqrt(s["lo"] * s["hi"])
        st.append(s)

    def begin(k):
        s = st[k]
        s.update(t=0, X=0.0, prev=x_start[k], still=0)
        s["history"].append(s["g"])
        engine.begin_probe(k, s["g"])

    for k in range(n):
        begin(k)
    active = [True] * n
    while any(active):
        engine.advance(list(active), R["chunk_steps"])
        mon = engine.monitors()
        for k in range(n):
            if not active[k]:
                continue
            p, s, m = problems[k], st[k], mon[k]
            s["t"] += R["chunk_steps"]
            outcome = None
            if m["bad_nodes"] > 0 or not np.isfinite(m["oil_cos"] + m["oil_sin"] + m["oil_flux"]):
                s["flags"] |= UNSTABLE
                outcome = "moving"
            else:
                x = _centre(m, p["nx"])
                s["X"] += _wrap(x - s["prev"], p["nx"])
                s["prev"] = x
                if s["X"] >= R["move_frac"] * p["lam"]:
                    outcome = "moving"
                else:
                    nu_w = (p["tau_w"] - 0.5) / 3.0
                    u_ref = s["g"] * p["h0"] ** 2 / (3.0 * nu_w)
                    U = m["oil_flux"] / m["mass"][0] if m["mass"][0] > 0 else 0.0
                    min_steps = p.get("min_steps") or R["min_steps"]
                    if s["t"] >= min_steps and abs(U) < R["still_frac"] * u_ref:
                        s["still"] += 1
                    else:
                        s["still"] = 0
                    if s["still"] >= R["still_chunks"] and s["X"] < R["creep_frac"] * p["lam"]:
                        outcome = "static"
                    elif s["t"] >= p["max_steps"]:
                        s["flags"] |= UNDECIDED
                        outcome = "static"
            if outcome is None:
                continue
            s["probes"] += 1
            moving = outcome == "moving"
            if s["phase"] == "verify_lo":
                if moving and s["widen"] < 8:
                    s["widen"] += 1
                    s["flags"] |= WIDENED
                    s["hi"] = s["lo"]
                    s["lo"] /= math.sqrt(10.0)
                    s["g"] = s["lo"]
                else:
                    s["phase"] = "verify_hi"
                    s["g"] = s["hi"]
            elif s["phase"] == "verify_hi":
                if not moving and s["widen"] < 8:
                    s["widen"] += 1
                    s["flags"] |= WIDENED
                    s["lo"] = s["hi"]
                    s["hi"] *= math.sqrt(10.0)
                    s["g"] = s["hi"]
                else:
                    s["phase"] = "bisect"
                    s["g"] = math.sqrt(s["lo"] * s["hi"])
            elif s["phase"] == "check_lo":
                if not moving:
                    s["lo_ok"] = True
                elif s["widen"] < 8:
                    s["widen"] += 1
                    s["flags"] |= WIDENED
                    s["hi"], s["hi_ok"] = s["lo"], True
                    s["lo"] /= math.sqrt(10.0)
                else:
                    s["flags"] |= NOT_CONVERGED
                    s["phase"] = "done"
            elif s["phase"] == "check_hi":
                if moving:
                    s["hi_ok"] = True
                elif s["widen"] < 8:
                    s["widen"] += 1
                    s["flags"] |= WIDENED
                    s["lo"], s["lo_ok"] = s["hi"], True
                    s["hi"] *= math.sqrt(10.0)
                else:
                    s["flags"] |= NOT_CONVERGED
                    s["phase"] = "done"
            else:
                if moving:
                    s["hi"], s["hi_ok"] = s["g"], True
                else:
                    s["lo"], s["lo_ok"] = s["g"], True
            if s["phase"] in ("bisect", "check_lo", "check_hi"):
                # next probe: bisect while wide, then the unprobed ends
                if (s["hi"] - s["lo"]) / s["lo"] > R["rel_tol"]:
                    s["phase"], s["g"] = "bisect", math.sqrt(s["lo"] * s["hi"])
                elif not s["lo_ok"]:
                    s["phase"], s["g"] = "check_lo", s["lo"]
                elif not s["hi_ok"]:
                    s["phase"], s["g"] = "check_hi", s["hi"]
                else:
                    s["phase"] = "done"
            if s["phase"] != "done" and s["probes"] >= R["max_probes"]:
                s["flags"] |= NOT_CONVERGED
                s["phase"] = "done"
            if s["phase"] == "done":
                active[k] = False
            else:
                begin(k)
    out = []
    for k, p in enumerate(problems):
        s = st[k]
        g = math.sqrt(s["lo"] * s["hi"])
        out.append(dict(g_lo=s["lo"], g_hi=s["hi"], g_crit=g, probes=s["probes"],
                        flags=s["flags"], history=s["history"],
                        bo_crit=p["rho_bar"] * g * p["nx"] * (p["h0"] - p["a"]) / p["sigma"]))
    return out


def ramp(engine, problems, ramp_dg, ramp_steps=40000, **rules):
    """Continuation search (Sec. 3.4: the forcing is switched on after the
    unforced equilibration and raised by a fixed increment at fixed intervals
    while the slug's centre of oil mass is tracked).  One continuous run per
    problem: level k has g_k = g_lo + k * ramp_dg for ramp_steps steps.  The
    displacement X is counted from the start of a level at which the slug is
    still (|U| < still_frac * U_ref with the level's g, measured at the end of
    the previous level); when it is not still the count continues across the
    level change.  Mobilised at level k once X >= move_frac * lam, or when the
    state turns non-physical (UNSTABLE).  Result: g_hi = g_crit = g_k and
    g_lo = g_{k-1} (0 and NOT_CONVERGED if k = 0); without mobilisation up to
    g_hi or within max_probes levels: g_lo = the last level, g_crit = g_hi =
    the problem's g_hi, UNDECIDED | NOT_CONVERGED.  probes counts the levels.
    engine additionally needs set_forcing(k, g)."""
    R = dict(DEFAULT_RULES)
    R.update(rules)
    n = len(problems)
    mon = engine.monitors()
    st = []
    for k, p in enumerate(problems):
        st.append(dict(level=0, g=p["g_lo"], t_level=0, X=0.0,
                       prev=_centre(mon[k], p["nx"]), U=0.0, moved=False, flags=0, levels=1))
        engine.begin_probe(k, p["g_lo"])
    active = [True] * n
    while any(active):
        engine.advance(list(active), R["chunk_steps"])
        mon = engine.monitors()
        for k in range(n):
            if not active[k]:
                continue
            p, s, m = problems[k], st[k], mon[k]
            s["t_level"] += R["chunk_steps"]
            finished = False
            if m["bad_nodes"] > 0 or not np.isfinite(m["oil_cos"] + m["oil_sin"] + m["oil_flux"]):
                s["flags"] |= UNSTABLE
                s["moved"] = finished = True
            else:
                x = _centre(m, p["nx"])
                s["X"] += _wrap(x - s["prev"], p["nx"])
                s["prev"] = x
                s["U"] = m["oil_flux"] / m["mass"][0] if m["mass"][0] > 0 else 0.0
                if s["X"] >= R["move_frac"] * p["lam"]:
                    s["moved"] = finished = True
            if not finished and s["t_level"] >= ramp_steps:
                nu_w = (p["tau_w"] - 0.5) / 3.0
                if abs(s["U"]) < R["still_frac"] * s["g"] * p["h0"] ** 2 / (3.0 * nu_w):
                    s["X"] = 0.0
                g_next = p["g_lo"] + (s["level"] + 1) * ramp_dg
                if g_next > p["g_hi"] * (1.0 + 1e-12) or s["levels"] >= R["max_probes"]:
                    finished = True
                else:
                    s["level"] += 1
                    s["levels"] += 1
                    s["g"] = g_next
                    s["t_level"] = 0
                    engine.set_forcing(k, g_next)
            if finished:
                active[k] = False
    out = []
    for k, p in enumerate(problems):
        s = st[k]
        flags = s["flags"]
        if s["moved"]:
            hi = s["g"]
            lo = p["g_lo"] + (s["level"] - 1) * ramp_dg if s["level"] > 0 else 0.0
            if s["level"] == 0:
                flags |= NOT_CONVERGED
        else:
            lo, hi = s["g"], p["g_hi"]
            flags |= UNDECIDED | NOT_CONVERGED
        out.append(dict(g_lo=lo, g_hi=hi, g_crit=hi, probes=s["levels"], flags=flags,
                        bo_crit=p["rho_bar"] * hi * p["nx"] * (p["h0"] - p["a"]) / p["sigma"]))
    return out


class OracleEngine:
    """Oracle lattices as a critical-pressure engine: equilibrate without
    forcing, keep that state, and restart every probe from it."""

    def __init__(self, lattices, equil_steps):
        self.lat = lattices
        for L in self.lat:
            L.set_body_force(0.0)
            L.step(equil_steps)
        self.snap = [L.copy_state() for L in self.lat]

    def begin_probe(self, k, g):
        self.lat[k].restore_state(self.snap[k])
        self.lat[k].set_body_force(g)

    def set_forcing(self, k, g):
        self.lat[k].set_body_force(g)

    def advance(self, active, steps):
        for k, L in enumerate(self.lat):
            if active[k]:
                try:
                    L.step(steps)
                except FloatingPointError:
                    pass  # reported through bad_nodes by the next monitors() call

    def monitors(self):
        out = []
        for L in self.lat:
            m = L.moments()["mon"]
            out.append({"mass": (m[0], m[1]), "momentum": (m[2], m[3]), "oil_flux": m[4],
                        "oil_cos": m[5], "oil_sin": m[6], "bad_nodes": m[7]})
        return out
