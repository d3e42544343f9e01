/*
 * lbm3d.h - C ABI of the D3Q19 (three-dimensional) part of the MI355X
 * two-component lattice Boltzmann library.
 *
 * The same model as include/lbm.h (Otomo et al., arXiv 1601.00918, Sec. 2:
 * regularized collision toward the third-order equilibrium with density-weighted
 * relaxation, Eqs. 3-7; inter-species force from neighbour densities with wall
 * potentials, Eq. 8; body force; force as an equilibrium-velocity shift,
 * Eqs. 9-10; pull streaming with half-way bounce-back, Eq. 1) on the D3Q19
 * lattice the paper's own simulations use, for one lattice per context: the
 * sinusoidal tube of Sec. 3.4 (circular cross-sections whose radius varies
 * sinusoidally along the axis) and periodic boxes.
 *
 * Conventions
 *   Species 0 is oil, species 1 water.  Lattice units.  Node arrays exchanged
 *   with the host are row-major [nz][ny][nx], x fastest; x is always periodic.
 *   D3Q19 numbering used by lbm3d_get_populations:
 *     c_0 = (0,0,0); c_1, c_2 = (+-1,0,0); c_3, c_4 = (0,+-1,0); c_5, c_6 = (0,0,+-1);
 *     c_7, c_8 = +-(1,1,0); c_9, c_10 = +-(1,-1,0); c_11, c_12 = +-(1,0,1);
 *     c_13, c_14 = +-(1,0,-1); c_15, c_16 = +-(0,1,1); c_17, c_18 = +-(0,1,-1)
 *   with weights 1/3 (rest), 1/18 (axes), 1/36 (face diagonals), T0 = 1/3.
 *   Status codes, lbm_last_error() and lbm_monitor are those of lbm.h.
 *
 * Memory and streams: as in lbm.h, the library never allocates device memory;
 * lbm3d_init carves the caller's workspace (size from lbm3d_required_bytes) and
 * enqueues on the caller's HIP stream (hipStream_t passed as void*).  Host
 * pointers are used during the call only.  One context must not be used from
 * two threads at once.
 */
#ifndef LBM3D_H
#define LBM3D_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM3D_GEOM_BOX = 0,  /* every node fluid, periodic in x, y and z; nx, ny, nz >= 3 */
    LBM3D_GEOM_TUBE = 1, /* sinusoidal tube along x: node fluid iff
                            (y - y_c)^2 + (z - z_c)^2 < r(x)^2 with
                            r(x) = r0 + a cos(2 pi x / lambda), y_c = (ny - 1) / 2,
                            z_c = (nz - 1) / 2; nodes outside the box are solid */
    LBM3D_GEOM_MASK = 2  /* host mask [nz][ny][nx], 1 = fluid; the fluid nodes of
                            every (x, y) column must form one contiguous run in z;
                            nodes outside the box are solid */
} lbm3d_geom_kind;

typedef struct {
    int32_t kind;         /* lbm3d_geom_kind */
    int32_t nx, ny, nz;   /* 3 <= nx, ny <= 32768, 3 <= nz <= 32767; one population
                             buffer (nz ny 19 or 20 planes of ceil(nx/64)*64 pairs)
                             must stay below 4 GiB */
    double lambda, r0, a; /* LBM3D_GEOM_TUBE only: lambda > 0, r0 > 0, a >= 0 */
    const uint8_t* mask;  /* LBM3D_GEOM_MASK only, copied during lbm3d_init */
    int32_t wall_interp;  /* LBM3D_GEOM_TUBE: 1 places the wall at its analytic
                             position between the nodes by linear interpolated
                             bounce-back (Bouzidi, Firdaouss and Lallemand 2001),
                             with what the blends add taken from the node's rest
                             population so each species keeps its mass; the link
                             fractions are computed once at init, in FP64, and
                             kept in the workspace.  0: half-way bounce-back on
                             the voxelised tube.  Any storage format. */
} lbm3d_geom;

typedef struct {
    double tau[2];   /* single-species relaxation times (> 1/2), mixed by density (Eqs. 4-5) */
    double G;        /* interaction strength of Eq. 8 (G < 0: immiscible) */
    double rho_s[2]; /* wall potentials (densities a solid neighbour contributes to Eq. 8) */
    double g[3];     /* homogeneous body acceleration; the force on species a is rho^a g */
} lbm3d_fluid;

typedef enum {
    LBM3D_INIT_UNIFORM = 0, /* (rho_hi, rho_lo) everywhere */
    LBM3D_INIT_DROPLET = 1, /* oil rho_hi inside the ball of radius r around (cx, cy, cz)
                               (periodic distance, strict <), rho_lo outside; water mirrored */
    LBM3D_INIT_SLUG = 3     /* oil rho_hi at fluid nodes with (x - x0) mod nx < length,
                               water elsewhere; the other species rho_lo; with
                               n_slugs >= 1 every slug of `slugs` (as in lbm.h) */
} lbm3d_init_kind;

typedef struct {
    int32_t kind;         /* lbm3d_init_kind */
    int32_t n_slugs;      /* SLUG: 0 = (x0, length); 1..LBM_MAX_SLUGS: `slugs` */
    double rho_hi, rho_lo;
    double cx, cy, cz, r; /* DROPLET */
    double x0, length;    /* SLUG */
    const double* slugs;  /* SLUG, n_slugs >= 1: host [n_slugs][2] (x0, length) */
    double width;         /* SLUG: initial interface width along x, as in
                             lbm_init_fields (0: a step) */
} lbm3d_init_fields;

typedef struct lbm3d_ctx lbm3d_ctx;

/* Workspace bytes lbm3d_init needs.  storage: LBM_STORE_F32, LBM_STORE_F16 or
 * LBM_STORE_BF16 (lbm.h; the 16-bit formats store deviations from the node's
 * reference density as in lbm.h, 20 two-byte pairs per node instead of 19
 * four-byte pairs), optionally OR-ed with LBM_OPT_SNAPSHOT. */
lbm_status lbm3d_required_bytes(const lbm3d_geom* geom, int32_t storage, size_t* bytes);

/* Create a context and set the initial state (t = 0): rest equilibrium
 * f_i = w_i rho0 at every fluid node.  Enqueues on hip_stream and synchronises
 * it before returning. */
lbm_status lbm3d_init(const lbm3d_geom* geom, const lbm3d_fluid* fluid,
                      const lbm3d_init_fields* init, int32_t storage, void* device_workspace,
                      size_t workspace_bytes, void* hip_stream, lbm3d_ctx** out);

/* Advance by nsteps time steps (Eq. 1).  Enqueues and returns. */
lbm_status lbm3d_step(lbm3d_ctx* ctx, int64_t nsteps);

/* Current time step count (-1 for NULL). */
int64_t lbm3d_time(const lbm3d_ctx* ctx);

/* Replace the fluid parameters (takes effect at the next step). */
lbm_status lbm3d_set_fluid(lbm3d_ctx* ctx, const lbm3d_fluid* fluid);

/* Macroscopic fields at the current time into caller-owned host arrays (any
 * may be NULL): rho [2][nz][ny][nx]; u [3][nz][ny][nx], the physical mixture
 * velocity u_mix + (F^o + F^w) / (2 rho); p [nz][ny][nx],
 * T0 (rho^o + rho^w) - G T0 rho^o rho^w; mon, the monitor sums (momentum is
 * its x and y components).  Solid nodes are 0.  Synchronises. */
lbm_status lbm3d_moments(lbm3d_ctx* ctx, double* rho, double* u, double* p, lbm_monitor* mon);

/* Monitor sums at the current time (FP64 over fluid nodes).  Synchronises. */
lbm_status lbm3d_monitors(lbm3d_ctx* ctx, lbm_monitor* mon);

/* Populations f_i at the current time (after streaming) as host FP64
 * [2][19][nz][ny][nx] in the numbering above; solid nodes 0.  Synchronises. */
lbm_status lbm3d_get_populations(lbm3d_ctx* ctx, double* f);

/* Fluid mask the library uses, host [nz][ny][nx] (1 = fluid). */
lbm_status lbm3d_fluid_mask(lbm3d_ctx* ctx, uint8_t* mask);

/* Tiling of the step kernel: one workgroup advances a tile of bx x by nodes
 * (x, y) through a strip of strip_planes planes along z.  (bx, by) is one of
 * (16, 12) (default),
 * (32, 16), (64, 8), (32, 8); strip_planes >= 4 (default 8).
 * Results do not depend on the tiling (bit for bit).  Synchronises. */
lbm_status lbm3d_set_tiling(lbm3d_ctx* ctx, int32_t bx, int32_t by, int32_t strip_planes);
lbm_status lbm3d_get_tiling(const lbm3d_ctx* ctx, int32_t* bx, int32_t* by,
                            int32_t* strip_planes, int32_t* n_items);

/* Copy the current state into the snapshot buffer (needs LBM_OPT_SNAPSHOT at
 * init) or back from it (restoring also restores the time).  Stream-ordered. */
lbm_status lbm3d_snapshot_save(lbm3d_ctx* ctx);
lbm_status lbm3d_snapshot_restore(lbm3d_ctx* ctx);

/* Release the context (not the caller's workspace or stream).  Waits for the
 * work the context queued on its stream first, so the workspace may be freed
 * as soon as this returns.  NULL is ignored. */
void lbm3d_destroy(lbm3d_ctx* ctx);

/* ------------------------------------------------------------------------
 * Critical pressure in the tube (Sec. 3.4): the smallest body acceleration g
 * along +x that mobilises the oil slug, by the bisection and the probe
 * classification of lbm_critical_pressure (lbm.h), with the tube's lambda,
 * mean radius r0 (in place of h0: U_ref = g r0^2 / (3 nu_w)), a and nx, and
 * Bo = rho_bar g_crit L D / sigma (Eq. 15) with L = nx and D = r0 - a, the
 * neck radius (the length unit of the paper's tube).  Every problem has its
 * own context; they are equilibrated, snapshotted and probed on the caller's
 * stream, one after another within each chunk of steps.  opts->storage
 * selects the population format; opts->autotune is ignored.
 * ---------------------------------------------------------------------- */
typedef struct {
    lbm3d_geom geom;         /* LBM3D_GEOM_TUBE */
    lbm3d_fluid fluid;       /* tau, G, rho_s; g is set by the solver */
    lbm3d_init_fields init;  /* usually LBM3D_INIT_SLUG */
    double sigma;            /* surface tension used for Bo */
    double rho_bar;          /* density used for Bo */
    double g_lo, g_hi;       /* initial bracket, 0 < g_lo < g_hi */
    int64_t equil_steps;     /* unforced steps before the snapshot */
    int64_t max_steps;       /* step budget of one probe */
    int64_t min_steps;       /* steps before a probe may be called static (0: options) */
} lbm3d_cp_problem;

/* Workspace bytes lbm3d_critical_pressure needs for these problems in this
 * storage format (lbm_storage). */
lbm_status lbm3d_cp_required_bytes(const lbm3d_cp_problem* probs, int32_t n, int32_t storage,
                                   size_t* bytes);

/* Solve n tube problems; results[n] is caller-owned.  Synchronises. */
lbm_status lbm3d_critical_pressure(const lbm3d_cp_problem* probs, int32_t n,
                                   const lbm_cp_options* opts, void* device_workspace,
                                   size_t workspace_bytes, void* hip_stream,
                                   lbm_cp_result* results);

#ifdef __cplusplus
}
#endif

#endif /* LBM3D_H */
