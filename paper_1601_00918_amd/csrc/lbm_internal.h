// Internal definitions shared by the HIP kernels (lbm_kernels.hip) and the
// host runtime (lbm_runtime.cpp).  Not part of the public ABI.
#pragma once

#include "lbm.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// One instance as the kernels see it.  A lattice row y is one contiguous
// block of planes; plane i holds, for every column x, the pair (oil, water)
// of direction i:
//   pair (i, x) of row y at element f_off + y * rstride + 2 * (i * pitch + x),
// in units of one species value (4 bytes in FP32, 2 in the 16-bit formats).
// FP32 has 9 planes (rstride = 18 * pitch).  The 16-bit formats add a tenth
// plane with the node reference densities (rstride = 20 * pitch).
struct InstDev {
    int64_t f_off;      // element offset of the instance in the population buffers
    int32_t nx, ny;
    int32_t pitch;      // elements per population row (>= nx, multiple of 64)
    int32_t rstride;    // species values per lattice row (18 or 20 times pitch)
    int32_t periodic_y; // 1: box geometry, every node fluid, rows wrap
    int32_t col_off;    // offset of this instance's column table entries
    float tau_h[2];     // tau^a - 1/2 (= nu^a / T0, Eqs. 4-5)
    float G36;          // G / 36: the D2Q9 weights of Eq. 8 are multiples of 1/36
    float rho_s[2];     // wall potentials
    float g[2];         // body acceleration
    int32_t reg3;       // 1: third-order Hermite regularization
    int32_t gaps;       // 1: some column holds two fluid runs (a bypass)
    double Gd;          // G in double (pressure export)
    // Interpolated walls (channel, FP32 storage): the wall fraction q of every
    // wall link, [nx][kWallSlots][8] (see wall_slot), or null for half-way
    // bounce-back.
    const float* wq;
};

// Rows of a column whose nodes may have wall links, when neighbouring fluid
// runs differ by at most one row at each end: lo, lo + 1, hi - 1 and hi.  A
// node's slot is y - lo if that is below 2, else 3 - (hi - y) if hi - y is
// below 2, else it has none (-1).  Entry (x, slot, j - 1) of the wall table
// is the fraction of the link from the node along -c_j (pulled direction j)
// at which it meets the wall.
constexpr int kWallSlots = 4;
__host__ __device__ inline int wall_slot(int y, int lo, int hi)
{
    return y - lo < 2 ? y - lo : (hi - y < 2 ? 3 - (hi - y) : -1);
}

// A work item: one workgroup advances the columns x0..x0+BX-1 of instance
// inst over rows y0..y1-1 marching up (y0 < y1), or over rows y0 down to
// y1+1 marching down (y0 > y1).
struct Item {
    int32_t inst, x0, y0, y1;
};

// Column table entry: the fluid rows of a column are lo..hi (empty if lo > hi)
// except the solid gap glo..ghi between two runs (no gap if glo > ghi).
struct Col {
    int32_t lo, hi, glo, ghi;
};

__host__ __device__ inline bool col_fluid(const Col& c, int y)
{
    return (y >= c.lo) & (y <= c.hi) & ((y < c.glo) | (y > c.ghi));
}

// Fluid nodes of a column.
__host__ __device__ inline int col_nodes(const Col& c)
{
    const int run = c.hi >= c.lo ? c.hi - c.lo + 1 : 0;
    const int gap = c.ghi >= c.glo ? c.ghi - c.glo + 1 : 0;
    return run - gap;
}

// Initial-state description for the init kernel (one instance per launch).
struct InitDev {
    int32_t kind;
    int32_t core_species;
    int32_t first_row, last_row;   // LAYERS: first / last fluid row of the box
    int32_t wall_rows;
    int32_t n_slugs;               // SLUG: slugs in x0 / length (>= 1)
    double rho_hi, rho_lo;
    double cx, cy, r;
    double x0[LBM_MAX_SLUGS], length[LBM_MAX_SLUGS];
    double width;                  // SLUG: tanh interface width (0: a step)
};

// Export staging layout (doubles, one instance): [23][ny*nx]
//   0..17  populations f[s*9+i], 18..19 rho, 20..21 u, 22 p
constexpr int kExportFields = 23;

enum Mode : int { kStep = 0, kStepMon = 1, kMonOnly = 2, kExport = 3 };

constexpr int kMonWidth = 8;

// Launchers (lbm_kernels.hip).  All enqueue on `stream` and return the launch
// status.  ext selects the extended step kernels, with the branches of the
// optional features (taken by instances with reg3 set, a wall table or
// two-run columns).
// The rounding sequence of the 16-bit formats is keyed by the step number
// seed + (seed_dev ? *seed_dev : 0) (seed_dev lets a captured graph take the
// step number from device memory; see launch_set_seed).
hipError_t launch_step(int storage, int bx, int mode, bool ext, const void* fin, void* fout,
                       const InstDev* insts, const Item* items, int item_base, int n_items,
                       const Col* cols, double* partial, double* stage, uint32_t seed,
                       const uint32_t* seed_dev, hipStream_t stream);
hipError_t launch_set_seed(uint32_t* seed_dev, uint32_t value, hipStream_t stream);
hipError_t launch_mon_reduce(const double* partial, const int32_t* item_first,
                             const int32_t* item_count, int n_inst, double* mon,
                             hipStream_t stream);
hipError_t launch_init(int storage, void* A, const InstDev* insts, int inst, const Col* cols,
                       int nx, int ny, const InitDev& ini, hipStream_t stream);

}  // namespace lbm
