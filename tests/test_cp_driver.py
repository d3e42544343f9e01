"""The library's critical-pressure driver (lbm_cp_drive) against a synthetic
engine whose critical forcing is known, and against the oracle's independent
implementation of the same probe rules.  CPU only."""
import math

import pytest

import synth
from oracle import driver as odrv
from paper_1601_00918_amd import binding


class FakeEngine:
    """Slugs that move at speed 2e-3 + c (g - g*) / g* once g exceeds g*, and
    otherwise creep with a decaying speed that stops well short of the
    creep threshold.  Optionally becomes non-physical above g_bad, or creeps
    forever (never settles) for problems listed in `creepers`."""

    def __init__(self, problems, g_star, g_bad=None, creepers=()):
        self.p = problems
        self.g_star = g_star
        self.g_bad = g_bad or [math.inf] * len(problems)
        self.creepers = set(creepers)
        self.x0 = [0.37 * p["nx"] for p in problems]
        self.state = [dict(g=0.0, t=0, X=0.0, U=0.0) for _ in problems]

    def begin_probe(self, k, g):
        self.state[k] = dict(g=g, t=0, X=0.0, U=0.0)

    def advance(self, active, steps):
        for k, a in enumerate(active):
            if not a:
                continue
            s, gs = self.state[k], self.g_star[k]
            t0, t1 = s["t"], s["t"] + steps
            if s["g"] > gs:
                s["U"] = 0.02 * (s["g"] - gs) / gs + 2e-3
                s["X"] += s["U"] * steps
            elif k in self.creepers:
                s["U"] = 1e-4
                s["X"] += s["U"] * steps
            else:
                U0, T = 1e-4, 3000.0
                s["X"] += U0 * T * (math.exp(-t0 / T) - math.exp(-t1 / T))
                s["U"] = U0 * math.exp(-t1 / T)
            s["t"] = t1

    def monitors(self):
        out = []
        for k, s in enumerate(self.state):
            nx = self.p[k]["nx"]
            x = self.x0[k] + s["X"]
            M = 1000.0
            bad = 1.0 if s["g"] > self.g_bad[k] else 0.0
            out.append({"mass": (M, 5000.0), "momentum": (0.0, 0.0), "oil_flux": M * s["U"],
                        "oil_cos": M * math.cos(2 * math.pi * x / nx),
                        "oil_sin": M * math.sin(2 * math.pi * x / nx), "bad_nodes": bad})
        return out


def _problems(g_stars, span=30.0, max_steps=200000):
    cfgs, plain = [], []
    for k, gs in enumerate(g_stars):
        cfg = synth.config_channel(lam=64 * (1 + k % 3), theta=90.0)
        cfgs.append(binding.cp_problem(cfg, gs / span, gs * span, sigma=0.161, rho_bar=1.03,
                                       equil_steps=0, max_steps=max_steps))
        plain.append(dict(nx=cfg["nx"], lam=cfg["lam"], h0=cfg["h0"], a=cfg["a"],
                          tau_w=cfg["tau"][1], g_lo=gs / span, g_hi=gs * span,
                          max_steps=max_steps, sigma=0.161, rho_bar=1.03))
    return cfgs, plain


def test_bisection_brackets_the_known_threshold():
    g_stars = [3.3e-5, 1.1e-6, 7.7e-4, 2.0e-5]
    probs, plain = _problems(g_stars)
    res = binding.lbm_cp_drive(FakeEngine(plain, g_stars), probs, binding.cp_options())
    for r, gs in zip(res, g_stars):
        assert r["g_lo"] <= gs <= r["g_hi"]
        assert (r["g_hi"] - r["g_lo"]) / r["g_lo"] <= 0.005
        assert abs(r["g_crit"] / gs - 1) < 0.005
        assert r["flags"] == 0
        # log2(ln(900) / 0.005) ~ 10.4 halvings of the log-bracket
        assert 10 <= r["probes"] <= 12
    assert res[0]["bo_crit"] == pytest.approx(1.03 * res[0]["g_crit"] * 256 * (8 - 4) / 0.161)


def test_library_driver_matches_the_oracle_driver():
    """Same engine, same rules: both drivers probe the same g sequence."""
    g_stars = [3.3e-5, 1.1e-6, 7.7e-4]
    probs, plain = _problems(g_stars)
    history = [[] for _ in g_stars]

    class Recording(FakeEngine):
        def begin_probe(self, k, g):
            history[k].append(g)
            super().begin_probe(k, g)

    lib = binding.lbm_cp_drive(Recording(plain, g_stars), probs, binding.cp_options())
    ref = odrv.solve(FakeEngine(plain, g_stars), plain)
    for k in range(len(g_stars)):
        assert len(history[k]) == len(ref[k]["history"])
        for a, b in zip(history[k], ref[k]["history"]):
            assert a == pytest.approx(b, rel=1e-12)
        assert lib[k]["g_crit"] == pytest.approx(ref[k]["g_crit"], rel=1e-12)
        assert lib[k]["probes"] == ref[k]["probes"] and lib[k]["flags"] == ref[k]["flags"]


def test_bracket_verification_widens_a_wrong_bracket():
    g_stars = [5e-5, 5e-5]
    probs, plain = _problems(g_stars, span=1.0)
    probs[0].g_lo, probs[0].g_hi = 2e-4, 4e-4     # threshold below the bracket
    probs[1].g_lo, probs[1].g_hi = 1e-6, 2e-6     # threshold above the bracket
    plain[0].update(g_lo=2e-4, g_hi=4e-4)
    plain[1].update(g_lo=1e-6, g_hi=2e-6)
    opts = binding.cp_options(verify_bracket=1)
    res = binding.lbm_cp_drive(FakeEngine(plain, g_stars), probs, opts)
    ref = odrv.solve(FakeEngine(plain, g_stars), plain, verify_bracket=1)
    for r, o in zip(res, ref):
        assert r["flags"] & binding._lib.CP_WIDENED
        assert r["g_lo"] <= 5e-5 <= r["g_hi"]
        assert r["g_crit"] == pytest.approx(o["g_crit"], rel=1e-12)


def test_unstable_and_undecided_probes_are_flagged():
    g_stars = [2e-5, 2e-5]
    probs, plain = _problems(g_stars, max_steps=60000)
    eng = FakeEngine(plain, g_stars, g_bad=[1e-4, math.inf], creepers=[1])
    res = binding.lbm_cp_drive(eng, probs, binding.cp_options())
    assert res[0]["flags"] & binding._lib.CP_UNSTABLE
    assert res[0]["g_lo"] <= 2e-5 <= res[0]["g_hi"]
    assert res[1]["flags"] & binding._lib.CP_UNDECIDED


def test_driver_rejects_bad_problems():
    probs, plain = _problems([1e-5])
    probs[0].g_lo = 0.0
    with pytest.raises(binding._lib.LbmError):
        binding.lbm_cp_drive(FakeEngine(plain, [1e-5]), probs, binding.cp_options())


def test_lazy_bracket_check_matches_the_oracle_and_recovers_wrong_brackets():
    """verify_bracket = 2: a bracket around the threshold costs no end probes;
    a bracket that misses it is widened after convergence; both drivers
    probe the same g sequence."""
    g_stars = [5e-5, 5e-5, 5e-5, 5e-5]
    probs, plain = _problems(g_stars, span=1.0)
    brackets = [(4e-5, 6e-5), (2e-4, 4e-4), (1e-6, 2e-6), (4.99e-5, 5.2e-5)]
    for p, q, (lo, hi) in zip(probs, plain, brackets):
        p.g_lo, p.g_hi = lo, hi
        q.update(g_lo=lo, g_hi=hi)
    history = [[] for _ in g_stars]

    class Recording(FakeEngine):
        def begin_probe(self, k, g):
            history[k].append(g)
            super().begin_probe(k, g)

    opts = binding.cp_options(verify_bracket=2)
    lib = binding.lbm_cp_drive(Recording(plain, g_stars), probs, opts)
    ref = odrv.solve(FakeEngine(plain, g_stars), plain, verify_bracket=2)
    for k, (r, o) in enumerate(zip(lib, ref)):
        assert len(history[k]) == len(o["history"])
        for a, b in zip(history[k], o["history"]):
            assert a == pytest.approx(b, rel=1e-12)
        assert r["g_crit"] == pytest.approx(o["g_crit"], rel=1e-12) and r["flags"] == o["flags"]
        assert r["g_lo"] <= 5e-5 <= r["g_hi"] and (r["g_hi"] - r["g_lo"]) / r["g_lo"] <= 0.005
    # inside bracket: plain bisection, no end probes, no widening
    assert lib[0]["flags"] == 0 and lib[0]["probes"] == math.ceil(math.log2(math.log(1.5) / 0.005))
    assert lib[1]["flags"] & binding._lib.CP_WIDENED and lib[2]["flags"] & binding._lib.CP_WIDENED


class RampEngine(FakeEngine):
    """FakeEngine with in-place forcing changes (the slug keeps its state)."""

    def set_forcing(self, k, g):
        self.state[k]["g"] = g


def _ramp_problems(g_stars, levels=12):
    cfgs, plain = [], []
    for k, gs in enumerate(g_stars):
        cfg = synth.config_channel(lam=64, theta=90.0)
        lo, hi = 0.8 * gs, 0.8 * gs + levels * 0.04 * gs
        cfgs.append(binding.cp_problem(cfg, lo, hi, sigma=0.161, rho_bar=1.03, equil_steps=0,
                                       max_steps=200000))
        plain.append(dict(nx=cfg["nx"], lam=cfg["lam"], h0=cfg["h0"], a=cfg["a"],
                          tau_w=cfg["tau"][1], g_lo=lo, g_hi=hi, max_steps=200000,
                          sigma=0.161, rho_bar=1.03))
    return cfgs, plain


def test_ramp_finds_the_first_level_above_the_threshold():
    """Levels g_k = 0.8 g* + k 0.04 g*: the first level strictly above g* is
    k = 6 (1.04 g*); the slug moves within that level, so the library reports
    g_crit = g_6 and g_lo = g_5, and the oracle's implementation agrees."""
    g_stars = [3.3e-5, 1.1e-6]
    probs, plain = _ramp_problems(g_stars)
    rules = dict(chunk_steps=1000)
    for k, gs in enumerate(g_stars):
        dg = 0.04 * gs
        opts = binding.cp_options(protocol="ramp", ramp_dg=dg, ramp_steps=40000, **rules)
        res = binding.lbm_cp_drive(RampEngine([plain[k]], [gs]), [probs[k]], opts)[0]
        ref = odrv.ramp(RampEngine([plain[k]], [gs]), [plain[k]], dg, 40000, **rules)[0]
        print(res, ref)
        assert res["g_crit"] == pytest.approx(0.8 * gs + 6 * dg, rel=1e-12)
        assert res["g_lo"] == pytest.approx(0.8 * gs + 5 * dg, rel=1e-12)
        assert res["probes"] == 7 and res["flags"] == 0
        for key in ("g_lo", "g_hi", "g_crit", "probes", "flags"):
            assert res[key] == pytest.approx(ref[key], rel=1e-12), key


def test_ramp_without_mobilisation_and_bad_options():
    """A threshold above the ramp's top level: undecided, g_crit = g_hi.  The
    ramp needs set_forcing, ramp_dg > 0 and ramp_steps a multiple of the chunk."""
    g_stars = [3.3e-5]
    probs, plain = _ramp_problems(g_stars, levels=3)
    opts = binding.cp_options(protocol="ramp", ramp_dg=0.04 * g_stars[0], ramp_steps=20000)
    res = binding.lbm_cp_drive(RampEngine(plain, g_stars), probs, opts)[0]
    ref = odrv.ramp(RampEngine(plain, g_stars), plain, 0.04 * g_stars[0], 20000)[0]
    assert res["flags"] == ref["flags"] == 1 | 8
    assert res["g_crit"] == pytest.approx(plain[0]["g_hi"], rel=1e-12)
    assert res["probes"] == ref["probes"] == 4
    with pytest.raises(binding._lib.LbmError):
        binding.lbm_cp_drive(FakeEngine(plain, g_stars), probs, opts)   # no set_forcing
    with pytest.raises(binding._lib.LbmError):
        binding.lbm_cp_drive(RampEngine(plain, g_stars), probs,
                             binding.cp_options(protocol="ramp", ramp_dg=0.0))
    with pytest.raises(binding._lib.LbmError):
        binding.lbm_cp_drive(RampEngine(plain, g_stars), probs,
                             binding.cp_options(protocol="ramp", ramp_dg=1e-6, ramp_steps=1500))


def test_ramp_carries_the_displacement_of_a_moving_slug():
    """A slug still creeping (never settles) at the end of a level keeps its
    displacement across the level change; a settled one starts afresh."""
    g_stars = [1e-4]
    probs, plain = _ramp_problems(g_stars, levels=12)
    dg = 0.04 * g_stars[0]
    opts = binding.cp_options(protocol="ramp", ramp_dg=dg, ramp_steps=40000)
    # creeper: U = 1e-4 below g*, 4 nodes per level; lambda / 2 = 32 nodes takes 8 levels
    res = binding.lbm_cp_drive(RampEngine(plain, g_stars, creepers=[0]), probs, opts)[0]
    ref = odrv.ramp(RampEngine(plain, g_stars, creepers=[0]), plain, dg, 40000)[0]
    assert res["probes"] == ref["probes"] and res["g_crit"] == pytest.approx(ref["g_crit"])
    assert res["g_crit"] <= 0.8 * g_stars[0] + 6 * dg + 1e-18


def test_slugs_without_a_first_fourier_mode_are_rejected():
    """Identical slugs spaced evenly around the domain cancel the first Fourier
    mode of the oil density that the probes track: both protocols refuse
    them instead of following noise."""
    probs, plain = _problems([1e-5])

    class Even(RampEngine):
        def monitors(self):
            out = super().monitors()
            for m in out:
                m["oil_cos"], m["oil_sin"] = 1e-9, -2e-9
            return out
    for proto in ("bisect", "ramp"):
        opts = binding.cp_options(protocol=proto, ramp_dg=1e-6, ramp_steps=1000,
                                  chunk_steps=500)
        with pytest.raises(binding._lib.LbmError) as e:
            binding.lbm_cp_drive(Even(plain, [1e-5]), probs, opts)
        assert e.value.status == 6 and "Fourier" in str(e.value)


def test_non_finite_states_are_flagged_not_refused():
    """A state that is already non-physical when the probes start is reported
    as unstable (as a probe that turns non-physical is), not refused as an
    untrackable slug."""
    probs, plain = _problems([1e-5])

    class Broken(FakeEngine):
        def monitors(self):
            out = super().monitors()
            for m in out:
                m["oil_cos"], m["oil_sin"], m["bad_nodes"] = float("nan"), float("nan"), 7.0
            return out
    r = binding.lbm_cp_drive(Broken(plain, [1e-5]), probs, binding.cp_options())[0]
    assert r["flags"] & binding._lib.CP_UNSTABLE


def test_verbose_logs_every_classified_probe(capfd):
    """verbose = 1: one stderr line per classified probe (bisection) or ramp
    level, naming the problem, the probe count and the forcing; nothing
    without it."""
    g_stars = [3.3e-5, 1.1e-6]
    probs, plain = _problems(g_stars)
    res = binding.lbm_cp_drive(FakeEngine(plain, g_stars), probs, binding.cp_options())
    assert "lbm_cp:" not in capfd.readouterr().err
    res_v = binding.lbm_cp_drive(FakeEngine(plain, g_stars), probs,
                                 binding.cp_options(verbose=1))
    lines = [ln for ln in capfd.readouterr().err.splitlines() if ln.startswith("lbm_cp:")]
    assert [r["g_crit"] for r in res_v] == [r["g_crit"] for r in res]
    assert len(lines) == sum(r["probes"] for r in res_v)
    for k, r in enumerate(res_v):
        mine = [ln for ln in lines if ln.startswith("lbm_cp: problem %d probe" % k)]
        assert len(mine) == r["probes"]
        assert mine[-1].startswith("lbm_cp: problem %d probe %d g " % (k, r["probes"]))
        assert all(("moving" in ln) != ("static" in ln) for ln in mine)
    rp, rplain = _ramp_problems(g_stars[:1])
    opts = binding.cp_options(protocol="ramp", ramp_dg=0.04 * g_stars[0], ramp_steps=40000,
                              chunk_steps=1000, verbose=1)
    r = binding.lbm_cp_drive(RampEngine(rplain, g_stars[:1]), rp, opts)[0]
    levels = [ln for ln in capfd.readouterr().err.splitlines() if "ramp level" in ln]
    assert len(levels) == r["probes"] - 1   # the first level is not a step up
