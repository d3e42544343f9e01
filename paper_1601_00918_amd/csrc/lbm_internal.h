// Internal definitions shared by the HIP kernels (lbm_kernels.hip) and the
// host runtime (lbm_runtime.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// One instance as the kernels see it.  The 18 population rows (species s,
// direction i) of lattice row y are stored next to each other:
//   buf[f_off + y * rstride + (s * 9 + i) * pitch + x],  rstride = 18 * pitch,
// so one lattice row of one instance is a single contiguous block.
struct InstDev {
    int64_t f_off;      // element offset of the instance in the population buffers
    int32_t nx, ny;
    int32_t pitch;      // elements per population row (>= nx, multiple of 64)
    int32_t rstride;    // elements per lattice row (18 * pitch)
    int32_t periodic_y; // 1: box geometry, every node fluid, rows wrap
    int32_t col_off;    // offset of this instance's column table entries
    float tau_h[2];     // tau^a - 1/2 (= nu^a / T0, Eqs. 4-5)
    float G36;          // G / 36: the D2Q9 weights of Eq. 8 are multiples of 1/36
    float rho_s[2];     // wall potentials
    float g[2];         // body acceleration
    float pad1;
    double Gd;          // G in double (pressure export)
    double enc_ref[2];  // reserved for deviation storage
};

// A work item: one workgroup advances the columns x0..x0+BX-1 of instance
// inst over rows y0..y1-1 marching up (y0 < y1), or over rows y0 down to
// y1+1 marching down (y0 > y1).
struct Item {
    int32_t inst, x0, y0, y1;
};

// Column table entry: the fluid rows of a column are lo..hi (empty if lo > hi).
struct Col {
    int32_t lo, hi;
};

// Initial-state description for the init kernel (one instance per launch).
struct InitDev {
    int32_t kind;
    int32_t core_species;
    int32_t first_row, last_row;   // LAYERS: first / last fluid row of the box
    int32_t wall_rows;
    int32_t pad;
    double rho_hi, rho_lo;
    double cx, cy, r;
    double x0, length;
};

// Export staging layout (doubles, one instance): [23][ny*nx]
//   0..17  populations f[s*9+i], 18..19 rho, 20..21 u, 22 p
constexpr int kExportFields = 23;

enum Mode : int { kStep = 0, kStepMon = 1, kMonOnly = 2, kExport = 3 };

constexpr int kMonWidth = 8;

// Launchers (lbm_kernels.hip).  All enqueue on `stream` and return the launch
// status.
hipError_t launch_step(int bx, int mode, const float* fin, float* fout, const InstDev* insts,
                       const Item* items, int item_base, int n_items, const Col* cols,
                       double* partial, double* stage, hipStream_t stream);
hipError_t launch_mon_reduce(const double* partial, const int32_t* item_first,
                             const int32_t* item_count, int n_inst, double* mon,
                             hipStream_t stream);
hipError_t launch_init(float* A, const InstDev* insts, int inst, const Col* cols, int nx,
                       int ny, const InitDev& ini, hipStream_t stream);

}  // namespace lbm
