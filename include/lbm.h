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
    LBM_ERR_UNSUPPORTED = 6  /* valid request this build does not support */
} lbm_status;

/* Geometry of one instance. */
typedef enum {
    LBM_GEOM_BOX = 0,     /* every node fluid, periodic in x and y */
    LBM_GEOM_CHANNEL = 1, /* walls at y = y_c +- (h0 + a cos(2 pi x / lambda)),
                             y_c = (ny - 1) / 2; node fluid iff |y - y_c| < h(x)
                             (a = 0: flat plates).  Rows outside 0..ny-1 are solid. */
    LBM_GEOM_MASK = 2     /* host mask [ny][nx], 1 = fluid; the fluid nodes of every
                             column must form one contiguous run of rows, and rows
                             outside 0..ny-1 are solid */
} lbm_geom_kind;

typedef struct {
    int32_t kind;          /* lbm_geom_kind */
    int32_t nx, ny;        /* bounding box in nodes; 1 <= nx, ny <= 32768 */
    int32_t reserved;
    double lambda, h0, a;  /* LBM_GEOM_CHANNEL only */
    const uint8_t* mask;   /* LBM_GEOM_MASK only, [ny][nx], copied */
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
} lbm_fluid;

/* Initial densities; populations start at rest equilibrium f_i = w_i rho0. */
typedef enum {
    LBM_INIT_UNIFORM = 0, /* rho0 = (rho_hi, rho_lo) everywhere */
    LBM_INIT_DROPLET = 1, /* oil rho_hi inside the disc of radius r around (cx, cy)
                             (periodic distance, strict <), rho_lo outside; water mirrored */
    LBM_INIT_LAYERS = 2,  /* the first and last `wall_rows` fluid rows of the box hold
                             species 1 - core_species at rho_hi, the rest species
                             core_species at rho_hi; the other species rho_lo */
    LBM_INIT_SLUG = 3,    /* oil rho_hi at fluid nodes with (x - x0) mod nx < length,
                             water elsewhere; the other species rho_lo */
    LBM_INIT_FIELD = 4    /* explicit host field rho0 [2][ny][nx]: reserved, currently
                             rejected with LBM_ERR_UNSUPPORTED */
} lbm_init_kind;

typedef struct {
    int32_t kind;        /* lbm_init_kind */
    int32_t wall_rows;   /* LAYERS */
    int32_t core_species;/* LAYERS */
    int32_t reserved;
    double rho_hi, rho_lo;
    double cx, cy, r;    /* DROPLET */
    double x0, length;   /* SLUG */
    const double* rho0;  /* FIELD (reserved), [2][ny][nx] */
} lbm_init_fields;

/* Population storage format in HBM (arithmetic is always FP32). */
typedef enum {
    LBM_STORE_F32 = 0,
    LBM_STORE_F16 = 1,   /* reserved: FP16 deviation storage */
    LBM_STORE_BF16 = 2   /* reserved: BF16 deviation storage */
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

/* Advance every instance by nsteps time steps (Eq. 1).  Enqueues work and
 * returns without synchronising. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t nsteps);

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
 * workgroup of bx threads advances one item.  Results do not depend on the
 * tiling (bit for bit).  Synchronises the stream.
 */
lbm_status lbm_set_tiling(lbm_ctx* ctx, int32_t bx, int32_t strip_rows);
lbm_status lbm_get_tiling(const lbm_ctx* ctx, int32_t* bx, int32_t* strip_rows,
                          int32_t* n_items);

/* Release the context (not the caller's workspace or stream). */
void lbm_destroy(lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
