// Critical-pressure driver (Sec. 3.4): bisection in log g over probes that
// restart from an equilibrated state, with the motion / rest classification
// documented in include/lbm.h.  The same state machine runs on the HIP engine
// (lbm_critical_pressure: every problem in one batched launch per step,
// finished probes restarted at once, finished problems dropped from the
// launch), on D3Q19 tube contexts (lbm3d_critical_pressure) and on caller
// callbacks (lbm_cp_drive).
#include "lbm3d.h"
#include "lbm_ctx.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

using namespace lbm;

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kMaxWiden = 8;

struct CpEngine {
    virtual ~CpEngine() {}
    virtual lbm_status begin_probe(int k, double g) = 0;
    virtual lbm_status set_forcing(int k, double g) = 0;
    virtual lbm_status advance(const std::vector<uint8_t>& active, int64_t steps) = 0;
    virtual lbm_status monitors(std::vector<lbm_monitor>& mon) = 0;
};

enum Outcome { kNone, kStatic, kMoving };
enum Phase { kVerifyLo, kVerifyHi, kBisect, kCheckLo, kCheckHi, kDone };

struct ProbeState {
    Phase phase = kBisect;
    double g_lo = 0, g_hi = 0, g = 0;
    bool lo_ok = true, hi_ok = true;  // the end has been probed (or is trusted)
    int widen = 0;
    // current probe
    int64_t probe_steps = 0;
    double X = 0.0, xc_prev = 0.0;
    int still = 0;
};

double centroid(const lbm_monitor& m, double nx)
{
    return std::atan2(m.oil_sin, m.oil_cos) / kTwoPi * nx;
}

double wrap_half(double d, double nx)
{
    while (d > 0.5 * nx)
        d -= nx;
    while (d <= -0.5 * nx)
        d += nx;
    return d;
}

// Probes follow the periodic centre of oil mass through the first Fourier
// mode of the oil density along x.  Identical slugs spaced evenly around the
// domain cancel that mode, and their motion cannot be followed.
lbm_status check_trackable(const std::vector<lbm_monitor>& mon)
{
    for (size_t k = 0; k < mon.size(); ++k) {
        const double amp = std::hypot(mon[k].oil_cos, mon[k].oil_sin);
        if (mon[k].bad_nodes > 0.0 || !std::isfinite(amp + mon[k].mass[0]))
            continue;  // a non-physical state: the probes flag it as unstable
        if (!(amp > 0.01 * mon[k].mass[0]))
            return fail(LBM_ERR_UNSUPPORTED,
                        "problem %d: the oil density has no first Fourier mode along x "
                        "(slugs spaced evenly around the domain?), so the slug cannot be "
                        "tracked",
                        (int)k);
    }
    return LBM_OK;
}

lbm_status check_problem(const lbm_cp_problem& p, int k)
{
    if (p.geom.kind != LBM_GEOM_CHANNEL)
        return fail(LBM_ERR_INVALID, "problem %d: critical pressure needs a channel geometry", k);
    if (!(p.g_lo > 0.0) || !(p.g_hi > p.g_lo) || !std::isfinite(p.g_hi))
        return fail(LBM_ERR_INVALID, "problem %d: bracket must satisfy 0 < g_lo < g_hi", k);
    if (!(p.sigma > 0.0) || !(p.rho_bar > 0.0))
        return fail(LBM_ERR_INVALID, "problem %d: sigma and rho_bar must be > 0", k);
    if (p.max_steps <= 0 || p.equil_steps < 0 || p.min_steps < 0)
        return fail(LBM_ERR_INVALID, "problem %d: bad step counts", k);
    if (!(p.fluid.tau[1] > 0.5))
        return fail(LBM_ERR_INVALID, "problem %d: tau_w must be > 1/2", k);
    return LBM_OK;
}

lbm_status check_options(const lbm_cp_options& o)
{
    if (!(o.rel_tol > 0.0) || !(o.move_frac > 0.0) || !(o.creep_frac > 0.0) ||
        !(o.still_frac > 0.0) || o.chunk_steps < 2 || (o.chunk_steps & 1) || o.still_chunks < 1 ||
        o.max_probes < 1 || o.min_steps < 0 || o.verify_bracket < 0 || o.verify_bracket > 2 ||
        o.storage < LBM_STORE_F32 ||
        o.storage > LBM_STORE_BF16 || o.verbose < 0 || o.verbose > 1)
        return fail(LBM_ERR_INVALID, "invalid critical-pressure options");
    if (o.protocol != LBM_CP_BISECT && o.protocol != LBM_CP_RAMP)
        return fail(LBM_ERR_INVALID, "unknown critical-pressure protocol %d", o.protocol);
    if (o.protocol == LBM_CP_RAMP &&
        (!(o.ramp_dg > 0.0) || !std::isfinite(o.ramp_dg) || o.ramp_steps < o.chunk_steps ||
         o.ramp_steps % o.chunk_steps != 0))
        return fail(LBM_ERR_INVALID, "ramp needs ramp_dg > 0 and ramp_steps a positive "
                                     "multiple of chunk_steps");
    return LBM_OK;
}

// Classify the running probe of problem k from its monitors.
Outcome classify(const lbm_cp_problem& p, const lbm_cp_options& o, ProbeState& s,
                 const lbm_monitor& m, int32_t& flags)
{
    const double nx = p.geom.nx;
    const double lam = p.geom.lambda;
    if (m.bad_nodes > 0.0 || !std::isfinite(m.oil_cos + m.oil_sin + m.oil_flux)) {
        flags |= LBM_CP_UNSTABLE;
        return kMoving;
    }
    const double xc = centroid(m, nx);
    s.X += wrap_half(xc - s.xc_prev, nx);
    s.xc_prev = xc;
    if (s.X >= o.move_frac * lam)
        return kMoving;
    const double nu_w = (p.fluid.tau[1] - 0.5) / 3.0;
    const double u_ref = s.g * p.geom.h0 * p.geom.h0 / (3.0 * nu_w);
    const double U = m.mass[0] > 0.0 ? m.oil_flux / m.mass[0] : 0.0;
    const int64_t min_steps = p.min_steps > 0 ? p.min_steps : o.min_steps;
    if (s.probe_steps >= min_steps && std::fabs(U) < o.still_frac * u_ref)
        ++s.still;
    else
        s.still = 0;
    if (s.still >= o.still_chunks && s.X < o.creep_frac * lam)
        return kStatic;
    if (s.probe_steps >= p.max_steps) {
        flags |= LBM_CP_UNDECIDED;
        return kStatic;  // did not advance move_frac * lambda within the budget
    }
    return kNone;
}

lbm_status cp_run(CpEngine& eng, const lbm_cp_problem* probs, int n, const lbm_cp_options& o,
                  lbm_cp_result* res, const std::vector<int64_t>& steps0)
{
    std::vector<ProbeState> st(n);
    std::vector<lbm_monitor> mon(n);
    lbm_status e = eng.monitors(mon);
    if (e != LBM_OK)
        return e;
    if ((e = check_trackable(mon)) != LBM_OK)
        return e;
    std::vector<double> xc0(n);
    for (int k = 0; k < n; ++k) {
        const lbm_cp_problem& p = probs[k];
        xc0[k] = centroid(mon[k], p.geom.nx);
        ProbeState& s = st[k];
        s.g_lo = p.g_lo;
        s.g_hi = p.g_hi;
        const bool eager = o.verify_bracket == 1;
        s.phase = eager ? kVerifyLo : kBisect;
        s.g = eager ? s.g_lo : std::sqrt(s.g_lo * s.g_hi);
        s.lo_ok = s.hi_ok = o.verify_bracket != 2;
        std::memset(&res[k], 0, sizeof(lbm_cp_result));
        res[k].steps = steps0[k];
    }
    auto start = [&](int k) -> lbm_status {
        ProbeState& s = st[k];
        s.probe_steps = 0;
        s.X = 0.0;
        s.xc_prev = xc0[k];
        s.still = 0;
        return eng.begin_probe(k, s.g);
    };
    for (int k = 0; k < n; ++k)
        if ((e = start(k)) != LBM_OK)
            return e;

    std::vector<uint8_t> active(n, 1);
    int remaining = n;
    while (remaining > 0) {
        if ((e = eng.advance(active, o.chunk_steps)) != LBM_OK)
            return e;
        if ((e = eng.monitors(mon)) != LBM_OK)
            return e;
        for (int k = 0; k < n; ++k) {
            if (!active[k])
                continue;
            const lbm_cp_problem& p = probs[k];
            ProbeState& s = st[k];
            lbm_cp_result& r = res[k];
            s.probe_steps += o.chunk_steps;
            r.steps += o.chunk_steps;
            const Outcome out = classify(p, o, s, mon[k], r.flags);
            if (out == kNone)
                continue;
            ++r.probes;
            const bool moving = out == kMoving;
            if (o.verbose)
                std::fprintf(stderr, "lbm_cp: problem %d probe %d g %.6e %s after %lld steps\n",
                             k, r.probes, s.g, moving ? "moving" : "static",
                             (long long)s.probe_steps);
            switch (s.phase) {
            case kVerifyLo:
                if (moving && s.widen < kMaxWiden) {
                    ++s.widen;
                    r.flags |= LBM_CP_WIDENED;
                    s.g_hi = s.g_lo;
                    s.g_lo /= std::sqrt(10.0);
                    s.g = s.g_lo;
                } else {
                    s.phase = kVerifyHi;
                    s.g = s.g_hi;
                }
                break;
            case kVerifyHi:
                if (!moving && s.widen < kMaxWiden) {
                    ++s.widen;
                    r.flags |= LBM_CP_WIDENED;
                    s.g_lo = s.g_hi;
                    s.g_hi *= std::sqrt(10.0);
                    s.g = s.g_hi;
                } else {
                    s.phase = kBisect;
                    s.g = std::sqrt(s.g_lo * s.g_hi);
                }
                break;
            case kCheckLo:
                if (!moving) {
                    s.lo_ok = true;
                } else if (s.widen < kMaxWiden) {
                    ++s.widen;
                    r.flags |= LBM_CP_WIDENED;
                    s.g_hi = s.g_lo;
                    s.hi_ok = true;
                    s.g_lo /= std::sqrt(10.0);
                } else {
                    r.flags |= LBM_CP_NOT_CONVERGED;
                    s.phase = kDone;
                }
                break;
            case kCheckHi:
                if (moving) {
                    s.hi_ok = true;
                } else if (s.widen < kMaxWiden) {
                    ++s.widen;
                    r.flags |= LBM_CP_WIDENED;
                    s.g_lo = s.g_hi;
                    s.lo_ok = true;
                    s.g_hi *= std::sqrt(10.0);
                } else {
                    r.flags |= LBM_CP_NOT_CONVERGED;
                    s.phase = kDone;
                }
                break;
            default:
                if (moving) {
                    s.g_hi = s.g;
                    s.hi_ok = true;
                } else {
                    s.g_lo = s.g;
                    s.lo_ok = true;
                }
                break;
            }
            if (s.phase == kBisect || s.phase == kCheckLo || s.phase == kCheckHi) {
                // next probe: bisect while wide, then the ends never probed
                if ((s.g_hi - s.g_lo) / s.g_lo > o.rel_tol) {
                    s.phase = kBisect;
                    s.g = std::sqrt(s.g_lo * s.g_hi);
                } else if (!s.lo_ok) {
                    s.phase = kCheckLo;
                    s.g = s.g_lo;
                } else if (!s.hi_ok) {
                    s.phase = kCheckHi;
                    s.g = s.g_hi;
                } else {
                    s.phase = kDone;
                }
            }
            if (s.phase != kDone && r.probes >= o.max_probes) {
                r.flags |= LBM_CP_NOT_CONVERGED;
                s.phase = kDone;
            }
            if (s.phase == kDone) {
                active[k] = 0;
                --remaining;
            } else if ((e = start(k)) != LBM_OK) {
                return e;
            }
        }
    }
    for (int k = 0; k < n; ++k) {
        const lbm_cp_problem& p = probs[k];
        lbm_cp_result& r = res[k];
        r.g_lo = st[k].g_lo;
        r.g_hi = st[k].g_hi;
        r.g_crit = std::sqrt(r.g_lo * r.g_hi);
        const double D = p.geom.h0 - p.geom.a;
        r.bo_crit = p.rho_bar * r.g_crit * (double)p.geom.nx * D / p.sigma;
    }
    return LBM_OK;
}

// Continuation (LBM_CP_RAMP): one run per problem, the forcing raised level
// by level until the slug is mobilised (rules in include/lbm.h).
lbm_status ramp_run(CpEngine& eng, const lbm_cp_problem* probs, int n, const lbm_cp_options& o,
                    lbm_cp_result* res, const std::vector<int64_t>& steps0)
{
    struct Ramp {
        int level = 0;
        double g = 0.0;
        int64_t level_steps = 0;
        double X = 0.0, xc_prev = 0.0, U = 0.0;
        bool moved = false;
    };
    std::vector<Ramp> st(n);
    std::vector<lbm_monitor> mon(n);
    lbm_status e = eng.monitors(mon);
    if (e != LBM_OK)
        return e;
    if ((e = check_trackable(mon)) != LBM_OK)
        return e;
    for (int k = 0; k < n; ++k) {
        std::memset(&res[k], 0, sizeof(lbm_cp_result));
        res[k].steps = steps0[k];
        res[k].probes = 1;
        st[k].g = probs[k].g_lo;
        st[k].xc_prev = centroid(mon[k], probs[k].geom.nx);
        if ((e = eng.begin_probe(k, st[k].g)) != LBM_OK)
            return e;
    }
    std::vector<uint8_t> active(n, 1);
    int remaining = n;
    while (remaining > 0) {
        if ((e = eng.advance(active, o.chunk_steps)) != LBM_OK)
            return e;
        if ((e = eng.monitors(mon)) != LBM_OK)
            return e;
        for (int k = 0; k < n; ++k) {
            if (!active[k])
                continue;
            const lbm_cp_problem& p = probs[k];
            Ramp& s = st[k];
            lbm_cp_result& r = res[k];
            s.level_steps += o.chunk_steps;
            r.steps += o.chunk_steps;
            const lbm_monitor& m = mon[k];
            bool done = false;
            if (m.bad_nodes > 0.0 || !std::isfinite(m.oil_cos + m.oil_sin + m.oil_flux)) {
                r.flags |= LBM_CP_UNSTABLE;
                s.moved = done = true;
            } else {
                const double nx = p.geom.nx;
                const double xc = centroid(m, nx);
                s.X += wrap_half(xc - s.xc_prev, nx);
                s.xc_prev = xc;
                s.U = m.mass[0] > 0.0 ? m.oil_flux / m.mass[0] : 0.0;
                if (s.X >= o.move_frac * p.geom.lambda)
                    s.moved = done = true;
            }
            if (!done && s.level_steps >= o.ramp_steps) {
                const double nu_w = (p.fluid.tau[1] - 0.5) / 3.0;
                const double u_ref = s.g * p.geom.h0 * p.geom.h0 / (3.0 * nu_w);
                if (std::fabs(s.U) < o.still_frac * u_ref)
                    s.X = 0.0;  // settled: count the next level's displacement afresh
                const double g_next = p.g_lo + (double)(s.level + 1) * o.ramp_dg;
                if (g_next > p.g_hi * (1.0 + 1e-12) || r.probes >= o.max_probes) {
                    done = true;
                } else {
                    ++s.level;
                    ++r.probes;
                    if (o.verbose)
                        std::fprintf(stderr, "lbm_cp: problem %d ramp level %d g %.6e\n", k,
                                     s.level, g_next);
                    s.g = g_next;
                    s.level_steps = 0;
                    if ((e = eng.set_forcing(k, s.g)) != LBM_OK)
                        return e;
                }
            }
            if (done) {
                active[k] = 0;
                --remaining;
            }
        }
    }
    for (int k = 0; k < n; ++k) {
        const lbm_cp_problem& p = probs[k];
        const Ramp& s = st[k];
        lbm_cp_result& r = res[k];
        if (s.moved) {
            r.g_hi = s.g;
            r.g_lo = s.level > 0 ? p.g_lo + (double)(s.level - 1) * o.ramp_dg : 0.0;
            if (s.level == 0)
                r.flags |= LBM_CP_NOT_CONVERGED;
        } else {
            r.g_lo = s.g;
            r.g_hi = p.g_hi;
            r.flags |= LBM_CP_UNDECIDED | LBM_CP_NOT_CONVERGED;
        }
        r.g_crit = r.g_hi;
        const double D = p.geom.h0 - p.geom.a;
        r.bo_crit = p.rho_bar * r.g_crit * (double)p.geom.nx * D / p.sigma;
    }
    return LBM_OK;
}

lbm_status run_protocol(CpEngine& eng, const lbm_cp_problem* probs, int n,
                        const lbm_cp_options& o, lbm_cp_result* res,
                        const std::vector<int64_t>& steps0)
{
    return o.protocol == LBM_CP_RAMP ? ramp_run(eng, probs, n, o, res, steps0)
                                     : cp_run(eng, probs, n, o, res, steps0);
}

// ---- engine over the library's own context -----------------------------------
struct HipEngine : CpEngine {
    lbm_ctx* ctx = nullptr;
    std::vector<lbm_fluid> fluids;
    std::vector<uint8_t> cur_active;

    lbm_status begin_probe(int k, double g) override
    {
        lbm_status e = lbm_snapshot_restore(ctx, k);
        if (e != LBM_OK)
            return e;
        fluids[k].g[0] = g;
        fluids[k].g[1] = 0.0;
        return lbm_set_fluid(ctx, k, &fluids[k]);
    }
    lbm_status set_forcing(int k, double g) override
    {
        fluids[k].g[0] = g;
        fluids[k].g[1] = 0.0;
        return lbm_set_fluid(ctx, k, &fluids[k]);
    }
    lbm_status advance(const std::vector<uint8_t>& active, int64_t steps) override
    {
        if (active != cur_active) {
            lbm_status e = lbm_set_active(ctx, active.data());
            if (e != LBM_OK)
                return e;
            cur_active = active;
        }
        return lbm_step(ctx, steps);
    }
    lbm_status monitors(std::vector<lbm_monitor>& mon) override
    {
        return lbm_monitors(ctx, mon.data());
    }
};

// ---- engine over D3Q19 tube contexts (one per problem) -------------------------
struct TubeEngine : CpEngine {
    std::vector<lbm3d_ctx*> ctx;
    std::vector<lbm3d_fluid> fluids;
    ~TubeEngine() override
    {
        for (lbm3d_ctx* c : ctx)
            lbm3d_destroy(c);
    }
    lbm_status begin_probe(int k, double g) override
    {
        lbm_status e = lbm3d_snapshot_restore(ctx[k]);
        if (e != LBM_OK)
            return e;
        fluids[k].g[0] = g;
        fluids[k].g[1] = fluids[k].g[2] = 0.0;
        return lbm3d_set_fluid(ctx[k], &fluids[k]);
    }
    lbm_status set_forcing(int k, double g) override
    {
        fluids[k].g[0] = g;
        fluids[k].g[1] = fluids[k].g[2] = 0.0;
        return lbm3d_set_fluid(ctx[k], &fluids[k]);
    }
    lbm_status advance(const std::vector<uint8_t>& active, int64_t steps) override
    {
        for (size_t k = 0; k < ctx.size(); ++k)
            if (active[k]) {
                lbm_status e = lbm3d_step(ctx[k], steps);
                if (e != LBM_OK)
                    return e;
            }
        return LBM_OK;
    }
    lbm_status monitors(std::vector<lbm_monitor>& mon) override
    {
        for (size_t k = 0; k < ctx.size(); ++k) {
            lbm_status e = lbm3d_monitors(ctx[k], &mon[k]);
            if (e != LBM_OK)
                return e;
        }
        return LBM_OK;
    }
};

// The classification parameters of a tube problem in the planar problem's
// terms: lambda, r0 as h0, a, nx; tau_w, sigma, rho_bar, bracket, budgets.
lbm_cp_problem as_channel_problem(const lbm3d_cp_problem& q)
{
    lbm_cp_problem p{};
    p.geom.kind = LBM_GEOM_CHANNEL;
    p.geom.nx = q.geom.nx;
    p.geom.ny = q.geom.ny;
    p.geom.lambda = q.geom.lambda;
    p.geom.h0 = q.geom.r0;
    p.geom.a = q.geom.a;
    p.fluid.tau[0] = q.fluid.tau[0];
    p.fluid.tau[1] = q.fluid.tau[1];
    p.fluid.G = q.fluid.G;
    p.sigma = q.sigma;
    p.rho_bar = q.rho_bar;
    p.g_lo = q.g_lo;
    p.g_hi = q.g_hi;
    p.equil_steps = q.equil_steps;
    p.max_steps = q.max_steps;
    p.min_steps = q.min_steps;
    return p;
}

constexpr size_t kTubeAlign = 256;

// ---- engine over caller callbacks --------------------------------------------
struct CallbackEngine : CpEngine {
    const lbm_cp_engine* cb = nullptr;
    lbm_status begin_probe(int k, double g) override
    {
        return cb->begin_probe(cb->user, k, g) == 0
                   ? LBM_OK
                   : fail(LBM_ERR_INVALID, "engine begin_probe(%d) failed", k);
    }
    lbm_status set_forcing(int k, double g) override
    {
        if (!cb->set_forcing)
            return fail(LBM_ERR_INVALID, "the ramp protocol needs the engine's set_forcing");
        return cb->set_forcing(cb->user, k, g) == 0
                   ? LBM_OK
                   : fail(LBM_ERR_INVALID, "engine set_forcing(%d) failed", k);
    }
    lbm_status advance(const std::vector<uint8_t>& active, int64_t steps) override
    {
        return cb->advance(cb->user, active.data(), steps) == 0
                   ? LBM_OK
                   : fail(LBM_ERR_INVALID, "engine advance failed");
    }
    lbm_status monitors(std::vector<lbm_monitor>& mon) override
    {
        return cb->monitors(cb->user, mon.data()) == 0
                   ? LBM_OK
                   : fail(LBM_ERR_INVALID, "engine monitors failed");
    }
};

}  // namespace

extern "C" {

void lbm_cp_default_options(lbm_cp_options* o)
{
    if (!o)
        return;
    std::memset(o, 0, sizeof *o);
    o->rel_tol = 0.005;
    o->move_frac = 0.5;
    o->creep_frac = 0.25;
    o->still_frac = 1e-3;
    o->chunk_steps = 1000;
    o->still_chunks = 3;
    o->max_probes = 60;
    o->verify_bracket = 0;
    o->min_steps = 20000;
    o->protocol = LBM_CP_BISECT;
    o->ramp_dg = 0.0;
    o->ramp_steps = 40000;
}

lbm_status lbm_cp_required_bytes(const lbm_cp_problem* probs, int32_t n, size_t* bytes)
{
    if (!probs || n < 1 || !bytes)
        return fail(LBM_ERR_INVALID, "lbm_cp_required_bytes: bad argument");
    std::vector<lbm_geom> geoms(n);
    for (int k = 0; k < n; ++k)
        geoms[k] = probs[k].geom;
    return lbm_required_bytes(geoms.data(), n, LBM_STORE_F32 | LBM_OPT_SNAPSHOT, bytes);
}

lbm_status lbm_critical_pressure(const lbm_cp_problem* probs, int32_t n,
                                 const lbm_cp_options* opts, void* device_workspace,
                                 size_t workspace_bytes, void* hip_stream,
                                 lbm_cp_result* results)
{
    if (!probs || n < 1 || !results)
        return fail(LBM_ERR_INVALID, "lbm_critical_pressure: bad argument");
    lbm_cp_options o;
    if (opts)
        o = *opts;
    else
        lbm_cp_default_options(&o);
    lbm_status e = check_options(o);
    if (e != LBM_OK)
        return e;
    std::vector<lbm_geom> geoms(n);
    std::vector<lbm_fluid> fluids(n);
    std::vector<lbm_init_fields> inits(n);
    for (int k = 0; k < n; ++k) {
        if ((e = check_problem(probs[k], k)) != LBM_OK)
            return e;
        geoms[k] = probs[k].geom;
        fluids[k] = probs[k].fluid;
        fluids[k].g[0] = fluids[k].g[1] = 0.0;
        inits[k] = probs[k].init;
    }
    HipEngine eng;
    e = lbm_init(geoms.data(), fluids.data(), inits.data(), n, o.storage | LBM_OPT_SNAPSHOT,
                 device_workspace, workspace_bytes, hip_stream, &eng.ctx);
    if (e != LBM_OK)
        return e;
    eng.fluids = fluids;
    eng.cur_active.assign(n, 1);
    // Unforced equilibration, each problem for its own number of steps; the
    // autotuner's timed steps are its first steps when every problem has room.
    std::vector<int64_t> steps0(n, 0);
    int64_t done = 0;
    if (o.autotune) {
        constexpr int kTrial = 32;
        std::vector<int> widths;
        int64_t min_equil = probs[0].equil_steps;
        for (int k = 0; k < n; ++k) {
            min_equil = std::min(min_equil, probs[k].equil_steps);
            if (std::find(widths.begin(), widths.end(), probs[k].geom.nx) == widths.end())
                widths.push_back(probs[k].geom.nx);
        }
        // at most 3 + 11 trials per width class (lbm_autotune)
        const int64_t bound = (int64_t)kTrial * (3 + 11 * (int64_t)widths.size());
        if (min_equil >= bound) {
            lbm_tune_report rep{};
            if ((e = lbm_autotune(eng.ctx, kTrial, &rep)) != LBM_OK) {
                lbm_destroy(eng.ctx);
                return e;
            }
            done = rep.steps;
            for (int k = 0; k < n; ++k)
                steps0[k] = rep.steps;
        }
    }
    for (;;) {
        std::vector<uint8_t> act(n, 0);
        int64_t next = -1;
        for (int k = 0; k < n; ++k)
            if (probs[k].equil_steps > done) {
                act[k] = 1;
                next = next < 0 ? probs[k].equil_steps : std::min(next, probs[k].equil_steps);
            }
        if (next < 0)
            break;
        if ((e = eng.advance(act, next - done)) != LBM_OK)
            break;
        for (int k = 0; k < n; ++k)
            if (act[k])
                steps0[k] += next - done;
        done = next;
    }
    if (e == LBM_OK)
        e = lbm_snapshot_save(eng.ctx);
    if (e == LBM_OK)
        e = run_protocol(eng, probs, n, o, results, steps0);
    lbm_destroy(eng.ctx);
    return e;
}

lbm_status lbm3d_cp_required_bytes(const lbm3d_cp_problem* probs, int32_t n, int32_t storage,
                                   size_t* bytes)
{
    if (!probs || n < 1 || !bytes)
        return fail(LBM_ERR_INVALID, "lbm3d_cp_required_bytes: bad argument");
    size_t total = 0;
    for (int k = 0; k < n; ++k) {
        size_t b = 0;
        lbm_status e = lbm3d_required_bytes(&probs[k].geom, storage | LBM_OPT_SNAPSHOT, &b);
        if (e != LBM_OK)
            return e;
        total += (b + kTubeAlign - 1) / kTubeAlign * kTubeAlign;
    }
    *bytes = total;
    return LBM_OK;
}

lbm_status lbm3d_critical_pressure(const lbm3d_cp_problem* probs, int32_t n,
                                   const lbm_cp_options* opts, void* device_workspace,
                                   size_t workspace_bytes, void* hip_stream,
                                   lbm_cp_result* results)
{
    if (!probs || n < 1 || !results || !device_workspace)
        return fail(LBM_ERR_INVALID, "lbm3d_critical_pressure: bad argument");
    lbm_cp_options o;
    if (opts)
        o = *opts;
    else
        lbm_cp_default_options(&o);
    lbm_status e = check_options(o);
    if (e != LBM_OK)
        return e;
    std::vector<lbm_cp_problem> shadow(n);
    for (int k = 0; k < n; ++k) {
        if (probs[k].geom.kind != LBM3D_GEOM_TUBE)
            return fail(LBM_ERR_INVALID, "problem %d: critical pressure needs a tube geometry", k);
        shadow[k] = as_channel_problem(probs[k]);
        if ((e = check_problem(shadow[k], k)) != LBM_OK)
            return e;
    }
    size_t need = 0;
    if ((e = lbm3d_cp_required_bytes(probs, n, o.storage, &need)) != LBM_OK)
        return e;
    if (workspace_bytes < need)
        return fail(LBM_ERR_OOM, "lbm3d_critical_pressure: workspace of %zu bytes, %zu needed",
                    workspace_bytes, need);
    TubeEngine eng;
    char* ws = (char*)device_workspace;
    for (int k = 0; k < n; ++k) {
        size_t b = 0;
        lbm3d_required_bytes(&probs[k].geom, o.storage | LBM_OPT_SNAPSHOT, &b);
        lbm3d_fluid f = probs[k].fluid;
        f.g[0] = f.g[1] = f.g[2] = 0.0;
        lbm3d_ctx* c = nullptr;
        if ((e = lbm3d_init(&probs[k].geom, &f, &probs[k].init, o.storage | LBM_OPT_SNAPSHOT, ws,
                            b, hip_stream, &c)) != LBM_OK)
            return e;
        eng.ctx.push_back(c);
        eng.fluids.push_back(f);
        ws += (b + kTubeAlign - 1) / kTubeAlign * kTubeAlign;
    }
    // Unforced equilibration, then the state every probe restarts from.
    std::vector<int64_t> steps0(n, 0);
    for (int k = 0; k < n; ++k) {
        if ((e = lbm3d_step(eng.ctx[k], probs[k].equil_steps)) != LBM_OK)
            return e;
        if ((e = lbm3d_snapshot_save(eng.ctx[k])) != LBM_OK)
            return e;
        steps0[k] = probs[k].equil_steps;
    }
    return run_protocol(eng, shadow.data(), n, o, results, steps0);
}

lbm_status lbm_cp_drive(const lbm_cp_engine* engine, const lbm_cp_problem* probs, int32_t n,
                        const lbm_cp_options* opts, lbm_cp_result* results)
{
    if (!engine || !engine->begin_probe || !engine->advance || !engine->monitors || !probs ||
        n < 1 || !results)
        return fail(LBM_ERR_INVALID, "lbm_cp_drive: bad argument");
    lbm_cp_options o;
    if (opts)
        o = *opts;
    else
        lbm_cp_default_options(&o);
    lbm_status e = check_options(o);
    if (e != LBM_OK)
        return e;
    for (int k = 0; k < n; ++k)
        if ((e = check_problem(probs[k], k)) != LBM_OK)
            return e;
    CallbackEngine eng;
    eng.cb = engine;
    if (o.protocol == LBM_CP_RAMP && !engine->set_forcing)
        return fail(LBM_ERR_INVALID, "lbm_cp_drive: the ramp protocol needs set_forcing");
    return run_protocol(eng, probs, n, o, results, std::vector<int64_t>(n, 0));
}

}  // extern "C"
