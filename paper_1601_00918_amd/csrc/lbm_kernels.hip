// HIP kernels (gfx950) of the two-component D2Q9 lattice Boltzmann step.
//
// Stored state.  Buffer A holds, for every fluid node x and direction i, the
// post-collision population f*_i(x) of the previous step, not yet streamed.
// A step is then a pure "pull": node x gathers f_i(x, t) = f*_i(x - c_i) (or,
// when x - c_i is solid, the half-way bounce-back value f*_opp(i)(x)), which
// are the populations of Eq. 1's left side at time t, collides them and writes
// its own f*(x, t) to buffer B at its own address.  Reads are coalesced
// (neighbouring lanes read neighbouring addresses, shifted by at most one
// element) and writes are aligned; every population is read once and written
// once per step: 2 species x 9 directions x (4 B read + 4 B write) = 144 B per
// fluid node.
//
// Tiling.  A workgroup of BX threads owns BX consecutive columns of one
// instance and marches up a strip of rows y0..y1-1, one row per iteration.
// The collision of row r needs the densities of rows r-1, r, r+1 at time t
// (Eq. 8), so the march pulls row r+1, reduces it to its 12 moments (the
// regularized collision depends on the populations only through rho, j and
// the momentum flux Pi, per species), publishes its densities in an LDS ring
// of four rows, and after one barrier collides row r from the moments it kept
// in registers.  The two columns left and right of the workgroup are pulled by
// lanes of wave 0 (one population per lane) and reduced in the same order as a
// node's own density, so a density is bitwise the same whichever workgroup
// computes it.  Solid neighbours enter the ring as the wall potentials rho_s.
#include "lbm_internal.h"

#include <hip/hip_runtime.h>

namespace lbm {
namespace {

constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// 36 * w_i: the D2Q9 weights are exact multiples of 1/36.
constexpr float kW36[9] = {16.f, 4.f, 4.f, 4.f, 4.f, 1.f, 1.f, 1.f, 1.f};

__device__ __forceinline__ int wrapi(int a, int n)
{
    return a < 0 ? a + n : (a >= n ? a - n : a);
}

__device__ __forceinline__ bool in_run(Col c, int y)
{
    return y >= c.lo && y <= c.hi;
}

// Direction constants for a lane-varying direction index.
__device__ __forceinline__ int dir_cx(int i)
{
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__device__ __forceinline__ int dir_cy(int i)
{
    return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__device__ __forceinline__ int dir_opp(int i)
{
    return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5);
}

// Density of one species from its 9 populations.  Every density that enters
// the interaction stencil is summed by this one expression.
__device__ __forceinline__ float rho9(const float* f)
{
    const float a13 = f[1] + f[3], a24 = f[2] + f[4];
    const float a57 = f[5] + f[7], a68 = f[6] + f[8];
    return ((f[0] + a13) + a24) + (a57 + a68);
}

struct Mom {
    float rho, jx, jy, pxx, pxy, pyy;
};

// Zeroth, first and second moments of the 9 populations of one species.
__device__ __forceinline__ Mom moments9(const float* f)
{
    Mom m;
    const float a13 = f[1] + f[3], a24 = f[2] + f[4];
    const float a57 = f[5] + f[7], a68 = f[6] + f[8];
    const float diag = a57 + a68;
    m.rho = ((f[0] + a13) + a24) + diag;
    const float d57 = f[5] - f[7], d86 = f[8] - f[6];
    m.jx = (f[1] - f[3]) + (d57 + d86);
    m.jy = (f[2] - f[4]) + (d57 - d86);
    m.pxx = a13 + diag;
    m.pyy = a24 + diag;
    m.pxy = a57 - a68;
    return m;
}

struct ColG {
    Col m, c, p;  // columns x-1, x, x+1
};

// Pull the 18 populations f_i(x, r, t) of a fluid node (Eq. 1 with half-way
// bounce-back).  xm/xp are the wrapped neighbour columns.
__device__ __forceinline__ void pull_node(const float* __restrict__ fin, const InstDev& P,
                                          int xm, int x, int xp, int r, const ColG& g,
                                          float (&f)[2][9])
{
    const float* base = fin + P.f_off;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int sx = kCx[i] == 1 ? xm : (kCx[i] == -1 ? xp : x);
        int sy = r - kCy[i];
        bool src_fluid;
        if (P.periodic_y) {
            sy = wrapi(sy, P.ny);
            src_fluid = true;
        } else {
            const Col cc = kCx[i] == 1 ? g.m : (kCx[i] == -1 ? g.p : g.c);
            src_fluid = in_run(cc, sy);
        }
        const int64_t off = src_fluid ? (int64_t)sy * P.pitch + sx : (int64_t)r * P.pitch + x;
        const int dir = src_fluid ? i : kOpp[i];
#pragma unroll
        for (int s = 0; s < 2; ++s)
            f[s][i] = base[(int64_t)(s * 9 + dir) * P.plane + off];
    }
}

// One population of node (x, r) for a lane-varying direction i.
__device__ __forceinline__ float pull_one(const float* __restrict__ fin, const InstDev& P, int s,
                                          int i, int xm, int x, int xp, int r, const ColG& g)
{
    const int cx = dir_cx(i), cy = dir_cy(i);
    const int sx = cx == 1 ? xm : (cx == -1 ? xp : x);
    int sy = r - cy;
    bool src_fluid;
    if (P.periodic_y) {
        sy = wrapi(sy, P.ny);
        src_fluid = true;
    } else {
        const Col cc = cx == 1 ? g.m : (cx == -1 ? g.p : g.c);
        src_fluid = in_run(cc, sy);
    }
    const int64_t off = src_fluid ? (int64_t)sy * P.pitch + sx : (int64_t)r * P.pitch + x;
    const int dir = src_fluid ? i : dir_opp(i);
    return fin[P.f_off + (int64_t)(s * 9 + dir) * P.plane + off];
}

// Post-collision populations of one species (Eqs. 3, 6, 7, 9) in FP32.
//   m      moments of the pulled populations
//   vx,vy  shifted equilibrium velocity u_mix + F / rho (Eqs. 9-10)
//   om     1 - 1 / tau_mix
// The equilibrium is written as w_i rho (1 + P_i(v)); w_i rho is formed as
// (36 w_i) * (rho / 36) with a correctly rounded division, so the nine rest
// parts sum to the same value for every direction set and carry no bias.
// The regularized non-equilibrium part is the second-order Hermite
// projection w_i / (2 T0^2) H_i : Pi^neq of the species' non-equilibrium
// momentum flux Pi^neq = Pi - rho T0 I - j j / rho, the second moment of
// f - f^eq(rho, j / rho) in closed form (the species' own equilibrium).
__device__ __forceinline__ void collide_species(const Mom& m, float vx, float vy, float om,
                                                float (&out)[9])
{
    const float third = 1.0f / 3.0f;
    const float ax = m.jx / m.rho, ay = m.jy / m.rho;
    const float nxx = m.pxx - (m.rho * third + m.jx * ax);
    const float nyy = m.pyy - (m.rho * third + m.jy * ay);
    const float nxy = m.pxy - m.jx * ay;
    const float tr = nxx + nyy;
    float fneq[9];
    fneq[0] = -(2.0f / 3.0f) * tr;
    fneq[1] = (2.0f * nxx - nyy) * (1.0f / 6.0f);
    fneq[3] = fneq[1];
    fneq[2] = (2.0f * nyy - nxx) * (1.0f / 6.0f);
    fneq[4] = fneq[2];
    fneq[5] = tr * (1.0f / 12.0f) + 0.25f * nxy;
    fneq[7] = fneq[5];
    fneq[6] = tr * (1.0f / 12.0f) - 0.25f * nxy;
    fneq[8] = fneq[6];
    const float r36 = m.rho / 36.0f;
    const float usq15 = 1.5f * (vx * vx + vy * vy);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const float base = kW36[i] * r36;
        const float cu = kCx[i] * vx + kCy[i] * vy;
        const float poly = 3.0f * cu * (1.0f + 1.5f * cu * (1.0f + cu) - usq15) - usq15;
        out[i] = base + (base * poly + om * fneq[i]);
    }
}

__device__ __forceinline__ int remap_xcd(int b, int n)
{
    // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous range of items so neighbouring strips share one L2.
    const int q = n >> 3, rem = n & 7;
    const int xcd = b & 7, slot = b >> 3;
    const int start = xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q;
    return start + slot;
}

template <int BX, int MODE>
__global__ void __launch_bounds__(BX)
step_kernel(const float* __restrict__ fin, float* __restrict__ fout,
            const InstDev* __restrict__ insts, const Item* __restrict__ items, int item_base,
            const Col* __restrict__ cols, double* __restrict__ partial,
            double* __restrict__ stage)
{
    __shared__ float ring[4][2][BX + 2];
    __shared__ double red[BX / 64][kMonWidth];

    const int item_idx = item_base + remap_xcd((int)blockIdx.x, (int)gridDim.x);
    const Item it = items[item_idx];
    const InstDev P = insts[it.inst];
    const int tid = threadIdx.x;
    const int wdt = min(BX, P.nx - it.x0);
    const bool act = tid < wdt;
    const int x = it.x0 + (act ? tid : 0);
    const int xm = wrapi(x - 1, P.nx), xp = wrapi(x + 1, P.nx);
    ColG g;
    if (!P.periodic_y) {
        g.m = cols[P.col_off + xm];
        g.c = cols[P.col_off + x];
        g.p = cols[P.col_off + xp];
    }

    // Halo lanes (wave 0): lane 16 k + j, k = side * 2 + species, j = direction.
    const int hk = (tid >> 4) & 3, hj = tid & 15;
    const int hside = hk >> 1, hs = hk & 1;
    const int hx = hside ? wrapi(it.x0 + wdt, P.nx) : wrapi(it.x0 - 1, P.nx);
    const int hxm = wrapi(hx - 1, P.nx), hxp = wrapi(hx + 1, P.nx);
    ColG hg;
    if (tid < 64 && !P.periodic_y) {
        hg.m = cols[P.col_off + hxm];
        hg.c = cols[P.col_off + hx];
        hg.p = cols[P.col_off + hxp];
    }

    const int64_t n_nodes = (int64_t)P.nx * P.ny;
    double macc[kMonWidth];
#pragma unroll
    for (int j = 0; j < kMonWidth; ++j)
        macc[j] = 0.0;
    double cosx = 0.0, sinx = 0.0;
    if (MODE != kStep)
        sincospi(2.0 * (double)x / (double)P.nx, &sinx, &cosx);

    Mom prev[2], cur[2];
    bool prev_fluid = false;

    for (int r = it.y0 - 1; r <= it.y1; ++r) {
        const int rr = P.periodic_y ? wrapi(r, P.ny) : r;
        // ---- phase 1: pull row r and publish its densities ----------------
        const bool fl = act && (P.periodic_y || in_run(g.c, rr));
        if (fl) {
            float f[2][9];
            pull_node(fin, P, xm, x, xp, rr, g, f);
            cur[0] = moments9(f[0]);
            cur[1] = moments9(f[1]);
            if (MODE == kExport && r >= it.y0 && r < it.y1) {
                const int64_t k = (int64_t)rr * P.nx + x;
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int i = 0; i < 9; ++i)
                        stage[(int64_t)(s * 9 + i) * n_nodes + k] = (double)f[s][i];
            }
        }
        if (act) {
            ring[r & 3][0][tid + 1] = fl ? cur[0].rho : P.rho_s[0];
            ring[r & 3][1][tid + 1] = fl ? cur[1].rho : P.rho_s[1];
        }
        if (tid < 64) {
            const bool hfl = P.periodic_y || in_run(hg.c, rr);
            float v = 0.0f;
            if (hfl && hj < 9)
                v = pull_one(fin, P, hs, hj, hxm, hx, hxp, rr, hg);
            float q[9];
#pragma unroll
            for (int j = 0; j < 9; ++j)
                q[j] = __shfl(v, (tid & ~15) + j, 64);
            const float rh = rho9(q);
            if (hj == 0)
                ring[r & 3][hs][hside ? wdt + 1 : 0] = hfl ? rh : (hs ? P.rho_s[1] : P.rho_s[0]);
        }
        __syncthreads();

        // ---- phase 2: collide row r - 1 ---------------------------------
        if (r - 1 >= it.y0 && prev_fluid) {
            const int rc = r - 1;
            const int rrc = P.periodic_y ? wrapi(rc, P.ny) : rc;
            const int rs = (rc - 1) & 3, rm = rc & 3, rn = r & 3;
            float sx[2], sy[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int b = 1 - s;  // the other species
                const float E = ring[rm][b][tid + 2], W = ring[rm][b][tid];
                const float N = ring[rn][b][tid + 1], S = ring[rs][b][tid + 1];
                const float NE = ring[rn][b][tid + 2], NW = ring[rn][b][tid];
                const float SE = ring[rs][b][tid + 2], SW = ring[rs][b][tid];
                sx[s] = 4.0f * (E - W) + ((NE - SW) + (SE - NW));
                sy[s] = 4.0f * (N - S) + ((NE - SW) + (NW - SE));
            }
            const float ro = prev[0].rho, rw = prev[1].rho;
            const float rho = ro + rw;
            const float inv = 1.0f / rho;
            const float ux = (prev[0].jx + prev[1].jx) * inv;
            const float uy = (prev[0].jy + prev[1].jy) * inv;
            const float taum = 0.5f + (ro * P.tau_h[0] + rw * P.tau_h[1]) * inv;
            const float om = 1.0f - 1.0f / taum;

            if (MODE == kStep || MODE == kStepMon) {
                const int64_t off = (int64_t)rrc * P.pitch + x;
                float* ob = fout + P.f_off;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float vx = ux + P.G36 * sx[s] + P.g[0];
                    const float vy = uy + P.G36 * sy[s] + P.g[1];
                    float out[9];
                    collide_species(prev[s], vx, vy, om, out);
#pragma unroll
                    for (int i = 0; i < 9; ++i)
                        ob[(int64_t)(s * 9 + i) * P.plane + off] = out[i];
                }
            }
            if (MODE != kStep) {
                // Physical quantities of the state at time t, evaluated in FP64
                // from the node's FP32 moments and neighbour densities.
                const double dro = ro, drw = rw, drho = dro + drw;
                const double G36 = P.Gd / 36.0;
                const double fxo = dro * (G36 * (double)sx[0] + (double)P.g[0]);
                const double fyo = dro * (G36 * (double)sy[0] + (double)P.g[1]);
                const double fxw = drw * (G36 * (double)sx[1] + (double)P.g[0]);
                const double fyw = drw * (G36 * (double)sy[1] + (double)P.g[1]);
                const double px = (double)prev[0].jx + (double)prev[1].jx + 0.5 * (fxo + fxw);
                const double py = (double)prev[0].jy + (double)prev[1].jy + 0.5 * (fyo + fyw);
                const double upx = px / drho, upy = py / drho;
                if (MODE == kExport) {
                    const int64_t k = (int64_t)rrc * P.nx + x;
                    stage[18 * n_nodes + k] = dro;
                    stage[19 * n_nodes + k] = drw;
                    stage[20 * n_nodes + k] = upx;
                    stage[21 * n_nodes + k] = upy;
                    stage[22 * n_nodes + k] = (drho - P.Gd * dro * drw) / 3.0;
                } else {
                    macc[0] += dro;
                    macc[1] += drw;
                    macc[2] += px;
                    macc[3] += py;
                    macc[4] += dro * upx;
                    macc[5] += dro * cosx;
                    macc[6] += dro * sinx;
                    const bool bad = !(ro > 0.0f) || !(rw > 0.0f) || !isfinite(upx + upy);
                    macc[7] += bad ? 1.0 : 0.0;
                }
            }
        }
        prev[0] = cur[0];
        prev[1] = cur[1];
        prev_fluid = fl;
    }

    if (MODE == kStepMon || MODE == kMonOnly) {
        const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
        for (int j = 0; j < kMonWidth; ++j) {
            double v = macc[j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1)
                v += __shfl_xor(v, o, 64);
            if (lane == 0)
                red[wave][j] = v;
        }
        __syncthreads();
        if (tid < kMonWidth) {
            double v = 0.0;
            for (int w = 0; w < BX / 64; ++w)
                v += red[w][tid];
            partial[(int64_t)item_idx * kMonWidth + tid] = v;
        }
    }
}

__global__ void mon_reduce_kernel(const double* __restrict__ partial,
                                  const int32_t* __restrict__ item_first,
                                  const int32_t* __restrict__ item_count,
                                  double* __restrict__ mon)
{
    const int inst = blockIdx.x;
    const int j = threadIdx.x;
    if (j >= kMonWidth)
        return;
    const int first = item_first[inst], cnt = item_count[inst];
    double v = 0.0;
    for (int k = 0; k < cnt; ++k)
        v += partial[(int64_t)(first + k) * kMonWidth + j];
    mon[(int64_t)inst * kMonWidth + j] = v;
}

// Initial density of species s at node (x, y) for the preset kinds 0-3.
__device__ double init_density(const InitDev& ini, const InstDev& P, int s, int x, int y)
{
    double oil;  // 1: the node belongs to the oil phase
    switch (ini.kind) {
    case 0:  // uniform
        return s == 0 ? ini.rho_hi : ini.rho_lo;
    case 1: {  // droplet of oil, periodic distance
        double dx = fabs((double)x - ini.cx);
        dx = fmin(dx, (double)P.nx - dx);
        double dy = fabs((double)y - ini.cy);
        dy = fmin(dy, (double)P.ny - dy);
        oil = (dx * dx + dy * dy) < ini.r * ini.r ? 1.0 : 0.0;
        break;
    }
    case 2: {  // layers
        const bool wall_layer =
            (y < ini.first_row + ini.wall_rows) || (y > ini.last_row - ini.wall_rows);
        const bool core = !wall_layer;
        const bool in_core_species = (s == ini.core_species);
        return (core == in_core_species) ? ini.rho_hi : ini.rho_lo;
    }
    default: {  // slug
        double rel = fmod((double)x - ini.x0, (double)P.nx);
        if (rel < 0.0)
            rel += (double)P.nx;
        oil = rel < ini.length ? 1.0 : 0.0;
        break;
    }
    }
    const bool is_hi = (s == 0) ? (oil != 0.0) : (oil == 0.0);
    return is_hi ? ini.rho_hi : ini.rho_lo;
}

// Rest equilibrium f_i = w_i rho0, placed where the first pull reads it: the
// slot (x, i) is read by node x + c_i (direction i) when that node is fluid,
// otherwise by node x itself after bounce-back (direction opp(i)).
__global__ void init_kernel(float* __restrict__ A, const InstDev* __restrict__ insts, int inst,
                            const Col* __restrict__ cols, InitDev ini)
{
    const InstDev P = insts[inst];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= P.nx)
        return;
    auto fluid = [&](int xx, int yy) -> bool {
        if (P.periodic_y)
            return true;
        if (yy < 0 || yy >= P.ny)
            return false;
        return in_run(cols[P.col_off + xx], yy);
    };
    if (!fluid(x, y))
        return;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double w = kW36[i] / 36.0;
        int xr = wrapi(x + kCx[i], P.nx);
        int yr = y + kCy[i];
        if (P.periodic_y)
            yr = wrapi(yr, P.ny);
        if (!fluid(xr, yr)) {
            xr = x;
            yr = y;
        }
        for (int s = 0; s < 2; ++s) {
            const double rho0 = init_density(ini, P, s, xr, yr);
            A[P.f_off + (int64_t)(s * 9 + i) * P.plane + (int64_t)y * P.pitch + x] =
                (float)(w * rho0);
        }
    }
}

template <int BX>
hipError_t launch_step_bx(int mode, const float* fin, float* fout, const InstDev* insts,
                          const Item* items, int item_base, int n_items, const Col* cols,
                          double* partial, double* stage, hipStream_t stream)
{
    const dim3 grid(n_items), block(BX);
    switch (mode) {
    case kStep:
        step_kernel<BX, kStep><<<grid, block, 0, stream>>>(fin, fout, insts, items, item_base,
                                                           cols, partial, stage);
        break;
    case kStepMon:
        step_kernel<BX, kStepMon><<<grid, block, 0, stream>>>(fin, fout, insts, items,
                                                              item_base, cols, partial, stage);
        break;
    case kMonOnly:
        step_kernel<BX, kMonOnly><<<grid, block, 0, stream>>>(fin, fout, insts, items,
                                                              item_base, cols, partial, stage);
        break;
    case kExport:
        step_kernel<BX, kExport><<<grid, block, 0, stream>>>(fin, fout, insts, items,
                                                             item_base, cols, partial, stage);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step(int bx, int mode, const float* fin, float* fout, const InstDev* insts,
                       const Item* items, int item_base, int n_items, const Col* cols,
                       double* partial, double* stage, hipStream_t stream)
{
    if (n_items <= 0)
        return hipSuccess;
    switch (bx) {
    case 64:
        return launch_step_bx<64>(mode, fin, fout, insts, items, item_base, n_items, cols,
                                  partial, stage, stream);
    case 128:
        return launch_step_bx<128>(mode, fin, fout, insts, items, item_base, n_items, cols,
                                   partial, stage, stream);
    case 256:
        return launch_step_bx<256>(mode, fin, fout, insts, items, item_base, n_items, cols,
                                   partial, stage, stream);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_mon_reduce(const double* partial, const int32_t* item_first,
                             const int32_t* item_count, int n_inst, double* mon,
                             hipStream_t stream)
{
    if (n_inst <= 0)
        return hipSuccess;
    mon_reduce_kernel<<<dim3(n_inst), dim3(64), 0, stream>>>(partial, item_first, item_count,
                                                            mon);
    return hipGetLastError();
}

hipError_t launch_init(float* A, const InstDev* insts, int inst, const Col* cols, int nx,
                       int ny, const InitDev& ini, hipStream_t stream)
{
    if (ini.kind < 0 || ini.kind > 3)
        return hipErrorInvalidValue;
    const dim3 block(256), grid((nx + 255) / 256, ny);
    init_kernel<<<grid, block, 0, stream>>>(A, insts, inst, cols, ini);
    return hipGetLastError();
}

}  // namespace lbm
