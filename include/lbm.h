/*
 * lbm.h - C ABI of the MI355X two-component lattice Boltzmann library.
 *
 * The library advances the two-component (oil / water) lattice Boltzmann model
 * of Otomo et al., "Simulation of residual oil displacement in a sinusoidal
 * channel with the lattice Boltzmann method" (arXiv 1601.00918), on a D2Q9
 * lattice, for one or many independent lattices ("instances") at once:
 *
 *   - per-species regularized collision toward the third-order equilibrium
 *     with a density-weighted mixed relaxation time (Sec. 2, Eqs. 3-7);
 *   - the inter-species interaction force from neighbour densities (Eq. 8),
 *     with wall potentials replacing solid neighbours (Sec. 2, last paragraph);
 *   - a homogeneous body force (Sec. 3.4, Eq. 15);
 *   - the force applied as a shift of the equilibrium velocity (Eqs. 9-10);
 *   - streaming with half-way bounce-back on voxelised walls (Eq. 1).
 *
 * Conventions
 *   Species 0 is oil ("o"), species 1 water ("w").  Lattice units throughout.
 *   D2Q9 numbering: c_0 = (0,0), c_1..c_4 = (1,0), (0,1), (-1,0), (0,-1),
 *   c_5..c_8 = (1,1), (-1,1), (-1,-1), (1,-1).
 *   Node arrays exchanged with the host are row-major [ny][nx], x fastest.
 *   x is always periodic.
 *
 * Memory and streams
 *   The library never allocates device memory: every call that needs device
 *   memory takes a caller-owned workspace (size from the matching *_bytes
 *   call) and a caller-owned HIP stream (hipStream_t passed as void*; NULL is
 *   the null stream).  The caller keeps both alive until lbm_destroy.  Host
 *   pointers are read or written during the call only and never retained.
 *
 * Errors
 *   Every entry point returns an lbm_status; on failure lbm_last_error()
 *   returns a message for the calling thread.  No C++ exception crosses the
 *   ABI.  One context must not be used from two threads at once.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_ERR_INVALID = 1,     /* bad argument or parameter */
    LBM_ERR_DEVICE = 2,      /* a HIP call failed */
    LBM_ERR_OOM = 3,         /* workspace smaller than required */
    LBM_ERR_UNSTABLE = 4,    /* a density became non-finite or non-positive */
    LBM_ERR_BUDGET = 5,      /* step budget exhausted without a decision */
    LBM_ERR_UNSUPPORTED = 6  /* valid request the library does not support */
} lbm_status;

/* Geometry of one instance. */
typedef enum {
    LBM_GEOM_BOX = 0,     /* every node fluid, periodic in x and y */
    LBM_GEOM_CHANNEL = 1, /* walls at y = y_c +- (h0 + a cos(2 pi x / lambda)),
                             y_c = (ny - 1) / 2 + y_offset; node fluid iff |y - y_c| < h(x)
                             (a = 0: flat plates), except inside the optional island
                             (island_h, island_len below).  Rows outside 0..ny-1 are
                             solid. */
    LBM_GEOM_MASK = 2     /* host mask [ny][nx], 1 = fluid; the fluid nodes of every
                             column must form at most two contiguous runs of rows
                             (two runs: a bypass, two flow paths side by side), and
                             rows outside 0..ny-1 are solid */
} lbm_geom_kind;

typedef struct {
    int32_t kind;          /* lbm_geom_kind */
    int32_t nx, ny;        /* bounding box in nodes; 1 <= nx, ny <= 32768 */
    int32_t wall_interp;   /* LBM_GEOM_CHANNEL, any storage: 1 places the walls at
                              their sub-lattice positions by linear interpolated
                              bounce-back (Bouzidi, Firdaouss and Lallemand 2001):
                              a population leaving a fluid node towards a wall met
                              at the fraction q of the link returns as
                              2q f*_i(x) + (1 - 2q) f*_i(x - c_i) for q < 1/2 and
                              f*_i(x) / (2q) + (1 - 1/(2q)) f*_opp(i)(x) otherwise,
                              and the node's rest population gives back what that
                              adds to the half-way value, so each species' mass is
                              conserved (to rounding).  q is computed in FP64 at
                              lbm_init (32 floats of workspace per column).  Walls
                              steeper than one row per column are rejected
                              (LBM_ERR_UNSUPPORTED).  0: half-way bounce-back */
    double lambda, h0, a;  /* LBM_GEOM_CHANNEL only */
    const uint8_t* mask;   /* LBM_GEOM_MASK only, [ny][nx], copied */
    double y_offset;       /* LBM_GEOM_CHANNEL: centre line at y_c = (ny - 1) / 2 +
                              y_offset (|y_offset| <= 1), to place walls off the
                              lattice */
    double island_h;       /* LBM_GEOM_CHANNEL bypass (the paper's closing section
                              names bypass channels as further work): a solid island
                              |y - y_c| < island_h over the columns whose distance
                              to the nearest multiple of lambda is below
                              island_len / 2 (the wide part of every period), which
                              splits the channel there into two parallel branches.
                              0 (or island_len 0): no island.  Not with wall_interp
                              (LBM_ERR_UNSUPPORTED). */
    double island_len;
} lbm_geom;

/* Fluid parameters of one instance. */
typedef struct {
    double tau[2];   /* single-species relaxation times (> 1/2); the node's
                        relaxation time mixes them by density (Eqs. 4-5) */
    double G;        /* interaction strength of Eq. 8 in the paper's sign:
                        repulsion (immiscible species) needs G < 0 */
    double rho_s[2]; /* wall potentials: the densities a solid neighbour
                        contributes to Eq. 8 for species o and w */
    double g[2];     /* homogeneous body acceleration (x, y); the force on
                        species a is rho^a g */
    int32_t reg_order; /* Hermite order of the regularized non-equilibrium part
                          (Eq. 6): 2 (or 0) projects f - f^eq on the second-order
                          polynomials only; 3 adds the third-order projection
                          (on D2Q9 its xxy and xyy coefficients), the
                          higher-order variant of the schemes the paper cites */
    int32_t reserved;
} lbm_fluid;

/* Initial densities; populations start at rest equilibrium f_i = w_i rho0. */
#define LBM_MAX_SLUGS 8 /* slugs of one SLUG initial state */

typedef enum {
    LBM_INIT_UNIFORM = 0, /* rho0 = (rho_hi, rho_lo) everywhere */
    LBM_INIT_DROPLET = 1, /* oil rho_hi inside the disc of radius r around (cx, cy)
                             (periodic distance, strict <), rho_lo outside; water mirrored */
    LBM_INIT_LAYERS = 2,  /* the first and last `wall_rows` fluid rows of the box hold
                             species 1 - core_species at rho_hi, the rest species
                             core_species at rho_hi; the other species rho_lo */
    LBM_INIT_SLUG = 3,    /* oil rho_hi at fluid nodes with (x - x0) mod nx < length,
                             water elsewhere; the other species rho_lo.  With
                             n_slugs >= 1: oil in every slug (x0_k, length_k) of
                             `slugs` (several slugs in series) */
} lbm_init_kind;

typedef struct {
    int32_t kind;        /* lbm_init_kind */
    int32_t wall_rows;   /* LAYERS */
    int32_t core_species;/* LAYERS */
    int32_t n_slugs;     /* SLUG: 0 = the slug (x0, length); 1..LBM_MAX_SLUGS = that
                            many slugs, given in `slugs` */
    double rho_hi, rho_lo;
    double cx, cy, r;    /* DROPLET */
    double x0, length;   /* SLUG */
    const double* slugs; /* SLUG with n_slugs >= 1: host [n_slugs][2] pairs
                            (x0, length), length >= 0, read during lbm_init;
                            LBM_ERR_INVALID if null or out of range */
    double width;        /* SLUG: width w of the initial oil/water interfaces along x.
                            0: a step at each slug end.  w > 0: the hyperbolic-tangent
                            profile the paper fits to interfaces (Sec. 3.1, Eq. 12):
                            phi(x) = sum over slugs and their periodic images at
                            +-nx of (tanh((x - x0 + 1/2) / w) - tanh((x - x0 - length
                            + 1/2) / w)) / 2, clipped to [0, 1]; oil rho_lo +
                            (rho_hi - rho_lo) phi, water rho_hi - (rho_hi - rho_lo) phi.
                            Finite, >= 0, else LBM_ERR_INVALID. */
} lbm_init_fields;

/* Population storage format in HBM (arithmetic is always FP32).  The storage
 * argument of lbm_required_bytes / lbm_init may be OR-ed with LBM_OPT_SNAPSHOT
 * to reserve a snapshot buffer (lbm_snapshot_save / lbm_snapshot_restore).
 *
 * The 16-bit formats store, per node and species, the deviations
 * d_i = f_i / w_i - R of the populations from the lattice weights times a
 * reference density R of that node, plus R itself as binary16: 20 two-byte
 * values per node and buffer, 80 bytes read and written per node update
 * against 144 in FP32.  d_1..d_8 are rounded to nearest even; d_0 carries the
 * remainder that keeps the node's stored mass equal to its density, rounded
 * stochastically with a counter-based generator keyed by node and step, so
 * results are deterministic and independent of tiling and batching.
 * Accuracy (against the FP64 reference, after 1000 steps): densities to a few
 * 1e-4 (binary16) or 1e-3 (bfloat16) relative, velocities on two-phase
 * interfaces to about 5e-5 absolute (binary16), total mass to 1e-5.  Critical
 * forcings agree with FP32 storage to 1 % (binary16) and 2 % (bfloat16). */
typedef enum {
    LBM_STORE_F32 = 0,   /* f_i in binary32 */
    LBM_STORE_F16 = 1,   /* deviations in binary16 */
    LBM_STORE_BF16 = 2,  /* deviations in bfloat16 (reference density in binary16) */
    LBM_OPT_SNAPSHOT = 0x100
} lbm_storage;

/* Per-instance monitor values, accumulated in FP64 over fluid nodes at the
 * current time t (the state the next step starts from). */
typedef struct {
    double mass[2];      /* sum of rho^o, sum of rho^w */
    double momentum[2];  /* sum of (j^o + j^w + (F^o + F^w) / 2), x and y */
    double oil_flux;     /* sum of rho^o u_x, u the physical mixture velocity */
    double oil_cos;      /* sum of rho^o cos(2 pi x / nx) */
    double oil_sin;      /* sum of rho^o sin(2 pi x / nx); atan2(sin, cos) is the
                            periodic centre of oil mass (Sec. 3.4 slug tracking) */
    double bad_nodes;    /* fluid nodes with a non-finite or non-positive density */
} lbm_monitor;

typedef struct lbm_ctx lbm_ctx;

/* Thread-local message describing the last failing call on this thread. */
const char* lbm_last_error(void);

/* Library version string. */
const char* lbm_version(void);

/*
 * Streaming copy of `bytes` bytes from device src to device dst (a
 * measurement aid, not part of the method): each workgroup of 256 lanes
 * copies one contiguous chunk of chunk_bytes with 16-byte nontemporal loads
 * and stores, four vectors per lane in flight.  It moves data the way the
 * step kernels do (every byte read once and written once) and nothing else,
 * so its rate is the bandwidth ceiling the step's HBM fraction is read
 * against.  src and dst 16-byte aligned and not overlapping, bytes a multiple
 * of 4, chunk_bytes a positive multiple of 16384 (256 KiB measured best);
 * otherwise LBM_ERR_INVALID (lbm_last_error is not set).  Enqueues on
 * hip_stream and returns.
 */
lbm_status lbm_stream_copy(const void* src, void* dst, size_t bytes, size_t chunk_bytes,
                           void* hip_stream);

/* Workspace bytes lbm_init needs for these instances. */
lbm_status lbm_required_bytes(const lbm_geom* geoms, int32_t n_inst, int32_t storage,
                              size_t* bytes);

/*
 * Create a context over n_inst instances (arrays of length n_inst) and set the
 * initial state (time t = 0).  device_workspace must hold at least
 * lbm_required_bytes() bytes; it is carved into the population buffers, the
 * geometry and parameter tables, monitor and staging areas.  Enqueues on
 * hip_stream and synchronises it before returning.
 */
lbm_status lbm_init(const lbm_geom* geoms, const lbm_fluid* fluids,
                    const lbm_init_fields* inits, int32_t n_inst, int32_t storage,
                    void* device_workspace, size_t workspace_bytes, void* hip_stream,
                    lbm_ctx** out);

/* Advance every active instance by nsteps time steps (Eq. 1).  Enqueues work
 * and returns without synchronising.  On a non-null stream, runs of 64 steps are
 * replayed from a captured HIP graph (same kernels, same results). */
lbm_status lbm_step(lbm_ctx* ctx, int64_t nsteps);

/* Choose which instances lbm_step advances: active[n_inst], nonzero = advance.
 * Inactive instances keep their state; monitors and exports still cover them.
 * Synchronises the stream. */
lbm_status lbm_set_active(lbm_ctx* ctx, const uint8_t* active);

/* Copy the whole current state into the snapshot buffer (needs
 * LBM_OPT_SNAPSHOT at init), or copy instance inst (all instances if inst < 0)
 * back from it.  Stream-ordered; no synchronisation. */
lbm_status lbm_snapshot_save(lbm_ctx* ctx);
lbm_status lbm_snapshot_restore(lbm_ctx* ctx, int32_t inst);

/* Current time step count. */
int64_t lbm_time(const lbm_ctx* ctx);

/* Replace the fluid parameters of instance inst (takes effect at the next step). */
lbm_status lbm_set_fluid(lbm_ctx* ctx, int32_t inst, const lbm_fluid* fluid);

/*
 * Macroscopic fields of instance inst at the current time, into caller-owned
 * host arrays (any may be NULL):
 *   rho [2][ny][nx]  species densities,
 *   u   [2][ny][nx]  physical mixture velocity u_mix + (F^o + F^w) / (2 rho) (x then y),
 *   p   [ny][nx]     bulk pressure T0 (rho^o + rho^w) - G T0 rho^o rho^w, T0 = 1/3,
 *   mon              monitor sums of this instance.
 * Solid nodes are 0.  Synchronises the stream.
 */
lbm_status lbm_moments(lbm_ctx* ctx, int32_t inst, double* rho, double* u, double* p,
                       lbm_monitor* mon);

/* Monitors of all instances at the current time into mon[n_inst].  Synchronises. */
lbm_status lbm_monitors(lbm_ctx* ctx, lbm_monitor* mon);

/* Populations f_i of instance inst at the current time (after streaming),
 * as host FP64 [2][9][ny][nx]; solid nodes 0.  Synchronises. */
lbm_status lbm_get_populations(lbm_ctx* ctx, int32_t inst, double* f);

/* Fluid mask the library uses for instance inst, host [ny][nx] (1 = fluid). */
lbm_status lbm_fluid_mask(lbm_ctx* ctx, int32_t inst, uint8_t* mask);

/*
 * Tiling of the step kernel: every instance is cut into work items of bx
 * consecutive columns (bx in {64, 128, 256}) by strip_rows rows (>= 4); one
 * workgroup of bx threads advances one item.  Instances of different bx run
 * as separate launches within a step.  Results do not depend on the tiling
 * (bit for bit).  These calls synchronise the stream.
 * lbm_set_tiling sets every instance; lbm_get_tiling returns the values last
 * set for every instance and the total number of work items.  Defaults after
 * lbm_init: FP32 bx = 256 (narrower if every instance is narrower), 8 rows;
 * 16-bit formats bx = 64, 16 rows.
 */
lbm_status lbm_set_tiling(lbm_ctx* ctx, int32_t bx, int32_t strip_rows);
lbm_status lbm_get_tiling(const lbm_ctx* ctx, int32_t* bx, int32_t* strip_rows,
                          int32_t* n_items);
lbm_status lbm_set_instance_tiling(lbm_ctx* ctx, int32_t inst, int32_t bx, int32_t strip_rows);
lbm_status lbm_get_instance_tiling(const lbm_ctx* ctx, int32_t inst, int32_t* bx,
                                   int32_t* strip_rows);

/* Outcome of lbm_autotune. */
typedef struct {
    int32_t buckets;    /* width classes tuned (active instances of equal nx) */
    int32_t trials;     /* timed trials, warm-up included */
    int64_t steps;      /* real steps advanced by the tuning */
    double ms_before;   /* per-step time with the tiling on entry */
    double ms_after;    /* per-step time with the chosen tiling */
} lbm_tune_report;

/*
 * Autotuner of the tiling, per width class of the active instances (the
 * channels of one wavelength share nx = 4 lambda): for the classes in
 * decreasing order of fluid nodes, try bx in {64, 128, 256} (not wider than
 * the instance) and strip_rows in {4, 8, 16, 32}, keep a candidate when the
 * whole step gets at least 0.3 % faster, then move to the next class.  Each
 * trial times steps_per_trial (>= 2) REAL steps of the run on ctx's stream
 * with HIP events, through lbm_step (so graphs are used on non-null streams);
 * the state advances by report->steps steps exactly as lbm_step would
 * advance it, whatever tiling is chosen.  Call it during a phase whose steps
 * are wanted anyway (an equilibration).  Synchronises; report may be NULL.
 */
lbm_status lbm_autotune(lbm_ctx* ctx, int32_t steps_per_trial, lbm_tune_report* report);

/* Release the context (not the caller's workspace or stream).  Waits for the
 * work the context queued on its stream first, so the workspace may be freed
 * as soon as this returns.  NULL is ignored. */
void lbm_destroy(lbm_ctx* ctx);

/* ------------------------------------------------------------------------
 * Critical pressure (Sec. 3.4): the smallest homogeneous body acceleration g
 * (along +x) that mobilises an oil slug, found by bisection in log g over
 * independent runs ("probes") that each restart from an equilibrated state.
 *
 * A probe at g advances the slug in chunks and watches its periodic centre of
 * oil mass X (unwrapped displacement since the probe started) and mean oil
 * velocity U = sum rho^o u_x / sum rho^o:
 *   moving  once X >= move_frac * lambda;
 *   static  once at least min_steps have run, |U| < still_frac * U_ref for
 *           still_chunks consecutive chunks and X < creep_frac * lambda, with
 *           U_ref = g h0^2 / (3 nu_w) and nu_w = (tau_w - 1/2) / 3;
 *   at the step budget: static (the slug did not advance move_frac * lambda;
 *           LBM_CP_UNDECIDED is set).  A slug released from rest may hop by
 *           about a quarter wavelength to the next pinning site at forcings
 *           well below the critical one and stick there; half a wavelength
 *           within the budget means it passed a constriction, so "critical"
 *           is the smallest g that carries the slug half a wavelength within
 *           max_steps;
 *   a non-finite or non-positive density counts as moving (LBM_CP_UNSTABLE).
 * Moving shrinks the bracket from above, static from below; the solve stops
 * when (g_hi - g_lo) / g_lo <= rel_tol and reports g_crit = sqrt(g_lo g_hi)
 * and Bo = rho_bar g_crit L D / sigma (Eq. 15) with L = nx and D = h0 - a.
 * ---------------------------------------------------------------------- */
typedef struct {
    lbm_geom geom;          /* LBM_GEOM_CHANNEL */
    lbm_fluid fluid;        /* tau, G, rho_s; g is set by the solver */
    lbm_init_fields init;   /* usually LBM_INIT_SLUG */
    double sigma;           /* surface tension used for Bo */
    double rho_bar;         /* density used for Bo */
    double g_lo, g_hi;      /* initial bracket, 0 < g_lo < g_hi */
    int64_t equil_steps;    /* unforced steps before the snapshot */
    int64_t max_steps;      /* step budget of one probe */
    int64_t min_steps;      /* steps before a probe may be called static; 0: the
                               options' min_steps (relaxation scales like lambda^2,
                               so mixed batches set it per problem) */
} lbm_cp_problem;

typedef struct {
    double rel_tol;         /* default 0.005 */
    double move_frac;       /* default 0.5 */
    double creep_frac;      /* default 0.25 */
    double still_frac;      /* default 1e-3 */
    int32_t chunk_steps;    /* steps between monitor checks, default 1000 (even) */
    int32_t still_chunks;   /* default 3 */
    int32_t max_probes;     /* default 60 */
    int32_t verify_bracket; /* 0 (default): trust [g_lo, g_hi].
                               1: probe both ends first and widen the bracket (by a
                               factor 10^0.5 per try) until g_lo is static and g_hi
                               is moving, then bisect.
                               2 (lazy, for predicted brackets): bisect first; once
                               the bracket is within rel_tol, probe each end that was
                               never probed; an end that fails moves the bracket out
                               by 10^0.5 and bisection resumes.  At most 8 widenings
                               (then LBM_CP_NOT_CONVERGED). */
    int64_t min_steps;      /* default 20000 */
    int32_t storage;        /* lbm_storage of the populations, default LBM_STORE_F32 */
    int32_t autotune;       /* 1: run lbm_autotune (32 steps per trial) at the start of
                               the equilibration when every problem's equil_steps covers
                               its steps; default 0 */
    int32_t protocol;       /* LBM_CP_BISECT (default) or LBM_CP_RAMP */
    int32_t verbose;        /* 1: one line on stderr per classified probe or ramp level
                               (problem index, probe count, forcing, outcome, steps);
                               default 0 */
    double ramp_dg;         /* LBM_CP_RAMP: forcing increment per level (> 0) */
    int64_t ramp_steps;     /* LBM_CP_RAMP: steps per level, a multiple of chunk_steps
                               (default 40000) */
} lbm_cp_options;

/*
 * Protocols.
 * LBM_CP_BISECT: the bisection over independent probes described above.
 * LBM_CP_RAMP: the continuation of Sec. 3.4.  After the unforced equilibration
 *   the forcing starts at g_lo and is raised by ramp_dg every ramp_steps steps
 *   (level k: g_k = g_lo + k ramp_dg) in one continuous run.  The slug's
 *   displacement X is counted from the start of a level at which it is still
 *   (|U| < still_frac U_ref at the end of the previous level; otherwise it keeps
 *   counting across the level change); the slug is mobilised at level k when X
 *   reaches move_frac * lambda (or the state becomes non-physical: also
 *   LBM_CP_UNSTABLE).  Result: g_hi = g_crit = g_k, g_lo = g_{k-1} (0 and
 *   LBM_CP_NOT_CONVERGED when the first level already moves the slug),
 *   probes = levels run.  Past g_hi, or after max_probes levels, without
 *   mobilisation: g_lo = the last level, g_crit = g_hi = the problem's g_hi,
 *   flags LBM_CP_UNDECIDED | LBM_CP_NOT_CONVERGED.  The engine must support
 *   set_forcing.
 */
enum { LBM_CP_BISECT = 0, LBM_CP_RAMP = 1 };

enum {
    LBM_CP_UNDECIDED = 1,   /* a probe hit its step budget */
    LBM_CP_UNSTABLE = 2,    /* a probe became non-physical */
    LBM_CP_WIDENED = 4,     /* the initial bracket had to be widened */
    LBM_CP_NOT_CONVERGED = 8 /* max_probes reached before rel_tol */
};

typedef struct {
    double g_lo, g_hi;      /* final bracket */
    double g_crit;          /* sqrt(g_lo g_hi) */
    double bo_crit;         /* Eq. 15 */
    int32_t probes;         /* probes run */
    int32_t flags;          /* LBM_CP_* */
    int64_t steps;          /* lattice steps run (equilibration included) */
} lbm_cp_result;

/* Fill opts with the defaults above. */
void lbm_cp_default_options(lbm_cp_options* opts);

/* Workspace bytes lbm_critical_pressure needs for these problems. */
lbm_status lbm_cp_required_bytes(const lbm_cp_problem* probs, int32_t n, size_t* bytes);

/*
 * Solve n critical-pressure problems together on the GPU: all problems are
 * equilibrated and probed in one batched launch per step; a problem whose
 * probe ends restarts at once from its snapshot with the next g, and finished
 * problems leave the launch.  results[n] is caller-owned.  Synchronises.
 */
lbm_status lbm_critical_pressure(const lbm_cp_problem* probs, int32_t n,
                                 const lbm_cp_options* opts, void* device_workspace,
                                 size_t workspace_bytes, void* hip_stream,
                                 lbm_cp_result* results);

/*
 * The same protocols and classification driven through caller callbacks (for
 * other engines and for testing the driver itself).  The driver calls
 *   begin_probe(user, k, g)        restart problem k from its equilibrated state
 *                                   with body acceleration g;
 *   advance(user, active, steps)   advance the problems with active[k] != 0;
 *   monitors(user, mon)            monitors of all n problems at the current time.
 * Each callback returns 0 on success.  probs supplies geometry (lambda, h0, a,
 * nx), tau_w, sigma, rho_bar, the bracket and the step budget; equil_steps is
 * ignored (the engine starts equilibrated).
 */
typedef struct {
    int (*begin_probe)(void* user, int32_t k, double g);
    int (*advance)(void* user, const uint8_t* active, int64_t steps);
    int (*monitors)(void* user, lbm_monitor* mon);
    void* user;
    int (*set_forcing)(void* user, int32_t k, double g); /* change problem k's body
                                   acceleration in place (LBM_CP_RAMP only; may be NULL
                                   for bisection) */
} lbm_cp_engine;

lbm_status lbm_cp_drive(const lbm_cp_engine* engine, const lbm_cp_problem* probs, int32_t n,
                        const lbm_cp_options* opts, lbm_cp_result* results);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
