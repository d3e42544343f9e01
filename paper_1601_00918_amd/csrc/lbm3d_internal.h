// Internal definitions shared by the D3Q19 kernels (lbm3d_kernels.hip) and
// their host runtime (lbm3d_runtime.cpp).  Not part of the public ABI.
#pragma once

#include "lbm.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm3 {

// Interpolated walls, per (x, y) column with fluid run [lo, hi]: the nodes
// a <= z < b have no wall link (every neighbour x - c_i fluid); each other
// node owns a row of link fractions, node z < a at row base + z - lo and
// node z >= b at row base + (a - lo) + (z - b).
struct WallCol {
    uint32_t base;
    uint32_t ab;  // a | b << 16
};

// The lattice as the kernels see it.  Lattice row (y, z) is the contiguous
// block of planes at pair index ((z * ny + y) * rs); plane i holds, for every
// x, the pair (oil, water) of direction i:
//   pair (i, x) of row (y, z) at pair index (z * ny + y) * rs + i * pitch + x.
// FP32 has 19 planes (8-byte pairs); the 16-bit formats add a twentieth plane
// of reference-density pairs (4-byte pairs).
struct Inst3Dev {
    int32_t nx, ny, nz;
    int32_t pitch;     // pairs per plane row (>= nx, multiple of 64)
    int32_t rs;        // pairs per lattice row (19 or 20 times pitch)
    int32_t periodic;  // 1: box, every node fluid, y and z wrap
    float tau_h[2];    // tau^a - 1/2 (= nu^a / T0, Eqs. 4-5)
    float G36;         // G / 36: the D3Q19 weights of Eq. 8 are multiples of 1/36
    float rho_s[2];    // wall potentials
    float g[3];        // body acceleration
    double Gd;         // G in double (pressure export)
    // Interpolated tube walls (null: half-way bounce-back everywhere).
    const WallCol* wcol;  // [ny][nx]
    const float* wq;      // [rows][18]: link fraction of pulled direction i at i - 1
};

// A work item: one workgroup collides the nodes x0 .. x0 + BXI - 1,
// y0 .. y0 + BYI - 1 (clipped to the lattice) of planes z0 .. z1 - 1 marching
// up (z0 < z1), or z0 down to z1 + 1 marching down (z0 > z1).
struct Item3 {
    int32_t x0, y0, z0, z1;
};

// Fluid run of the column (x, y) along z, packed: lo | (hi + 1) << 16; the
// node (x, y, z) is fluid iff lo <= z < hi + 1.  An empty column is 0.
constexpr uint32_t kEmptyRun = 0u;

// Export staging layout (doubles): [44][nz * ny * nx]
//   0..37 populations f[s * 19 + i], 38..39 rho, 40..42 u, 43 p
constexpr int kExport3Fields = 44;

enum Mode3 : int { kStep = 0, kStepMon = 1, kMonOnly = 2, kExport = 3 };
constexpr int kMon3Width = 8;

// Initial state (one launch).
struct Init3Dev {
    int32_t kind;  // 0 uniform, 1 droplet (sphere), 3 slug
    int32_t n_slugs;  // slug: slugs in x0 / length (>= 1)
    double rho_hi, rho_lo;
    double cx, cy, cz, r;
    double x0[LBM_MAX_SLUGS], length[LBM_MAX_SLUGS];
    double width;  // slug: tanh interface width (0: a step)
};

// Supported workgroup tiles (inner nodes per item in x and y).
constexpr int kTiles3 = 4;
constexpr int kTileBx[kTiles3] = {32, 64, 32, 16};
constexpr int kTileBy[kTiles3] = {16, 8, 8, 12};

// Launchers (lbm3d_kernels.hip); all enqueue on `stream` and return the launch
// status.  tile indexes kTileBx / kTileBy.
hipError_t launch3_step(int storage, int tile, int mode, const void* fin, void* fout,
                        const Inst3Dev& inst, const Item3* items, int n_items,
                        const uint32_t* runs, double* partial, double* stage, uint32_t seed,
                        hipStream_t stream);
hipError_t launch3_mon_reduce(const double* partial, int n_items, double* mon,
                              hipStream_t stream);
hipError_t launch3_init(int storage, void* A, const Inst3Dev& inst, const uint32_t* runs,
                        const Init3Dev& ini, hipStream_t stream);

}  // namespace lbm3
