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
// instance and marches along a strip of rows, one row per iteration
// (adjacent strips march in opposite directions, so the two workgroups that
// both need a boundary row reach it at the same time and share it in L2).
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

// Post-collision populations of one species (Eqs. 3, 6, 7, 9) in FP32.
//   m      moments of the pulled populations
//   vx,vy  shifted equilibrium velocity u_mix + F / rho (Eqs. 9-10)
//   om     1 - 1 / tau_mix
// Equilibrium: f_i^eq = w_i rho (1 + P(c_i . v)) with, for T0 = 1/3 and
// cu = c_i . v, P = E + O, E = 4.5 cu^2 - 1.5 v^2 (even in cu) and
// O = cu (3 - 4.5 v^2 + 4.5 cu^2) (odd in cu), so the two directions of a pair
// (c_i, -c_i) share E and take +-O.  The rest parts w_i rho are exact
// multiples (16, 4, 1) of one correctly rounded rho / 36: every direction
// carries the same unbiased relative rounding, so neither the mass nor the
// momentum of the equilibrium drifts (a rounded constant weight such as
// fl(1/9) would scale the momentum by a fixed factor every step).
// Regularized non-equilibrium part (Eq. 6): the second-order Hermite
// projection w_i / (2 T0^2) H_i : Pi^neq of the species' non-equilibrium
// momentum flux Pi^neq = Pi - rho T0 I - j j / rho, the second moment of
// f - f^eq(rho, j / rho) in closed form (the species' own equilibrium); on
// D2Q9 it takes five distinct values (rest, axis x, axis y, two diagonals).
__device__ __forceinline__ void collide_species(const Mom& m, float vx, float vy, float om,
                                                float (&out)[9])
{
    const float rinv = __builtin_amdgcn_rcpf(m.rho);
    const float ax = m.jx * rinv, ay = m.jy * rinv;
    const float nxx = m.pxx - (m.rho * (1.0f / 3.0f) + m.jx * ax);
    const float nyy = m.pyy - (m.rho * (1.0f / 3.0f) + m.jy * ay);
    const float nxy = m.pxy - m.jx * ay;
    const float tr = nxx + nyy;
    const float g0 = om * (-(2.0f / 3.0f) * tr);
    const float g1 = om * ((2.0f * nxx - nyy) * (1.0f / 6.0f));
    const float g2 = om * ((2.0f * nyy - nxx) * (1.0f / 6.0f));
    const float gd = tr * (1.0f / 12.0f);
    const float g5 = om * (gd + 0.25f * nxy);
    const float g6 = om * (gd - 0.25f * nxy);
    const float b5 = m.rho / 36.0f;  // correctly rounded: no bias in w_i rho
    const float b1 = 4.0f * b5;
    const float b0 = 16.0f * b5;
    const float vsq15 = 1.5f * (vx * vx + vy * vy);
    const float t = 3.0f - 3.0f * vsq15;
    out[0] = b0 + (g0 - b0 * vsq15);
    auto pair = [&](float cu, float b, float g, float& plus, float& minus) {
        const float cu2 = cu * cu;
        const float E = 4.5f * cu2 - vsq15;
        const float O = cu * (t + 4.5f * cu2);
        const float C = b + (b * E + g);
        const float BO = b * O;
        plus = C + BO;
        minus = C - BO;
    };
    pair(vx, b1, g1, out[1], out[3]);
    pair(vy, b1, g2, out[2], out[4]);
    pair(vx + vy, b5, g5, out[5], out[7]);
    pair(vy - vx, b5, g6, out[6], out[8]);
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

// Barrier that orders LDS only: global loads of the next row stay in flight.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Byte offsets (relative to the instance's first element) of the 9 pulled
// populations of species 0 at node (x, r); species 1 adds 9 * pitch elements.
// rb[k] is the element offset (row index times rstride) of row r - 1 + k.
// Where x - c_i is solid the half-way bounce-back source f*_opp(i)(x) is used
// instead.  Instances are smaller than 4 GiB, so 32-bit offsets suffice.
template <bool PY>
__device__ __forceinline__ void pull_offsets(const InstDev& P, const int (&rb)[3], int r, int xm,
                                             int x, int xp, const ColG& g, uint32_t (&off)[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int cx = kCx[i], cy = kCy[i];
        const int sx = cx == 1 ? xm : (cx == -1 ? xp : x);
        const int srb = rb[1 - cy];
        bool src_fluid = true;
        if (!PY) {
            const Col cc = cx == 1 ? g.m : (cx == -1 ? g.p : g.c);
            const int sy = r - cy;
            src_fluid = (sy >= cc.lo) & (sy <= cc.hi);
        }
        const uint32_t o_src = 4u * ((uint32_t)(i * P.pitch) + (uint32_t)(srb + sx));
        const uint32_t o_bb = 4u * ((uint32_t)(kOpp[i] * P.pitch) + (uint32_t)(rb[1] + x));
        off[i] = src_fluid ? o_src : o_bb;
    }
}

template <int BX, int MODE, bool PY>
__device__ __forceinline__ void march(const float* __restrict__ fin, float* __restrict__ fout,
                                      const InstDev& P, const Item& it, int item_idx,
                                      const Col* __restrict__ cols, double* __restrict__ partial,
                                      double* __restrict__ stage, float (&ring)[4][2][BX + 2],
                                      double (&red)[BX / 64][kMonWidth])
{
    const int tid = threadIdx.x;
    const int wdt = min(BX, P.nx - it.x0);
    const bool act = tid < wdt;
    const int x = it.x0 + (act ? tid : 0);
    const int xm = wrapi(x - 1, P.nx), xp = wrapi(x + 1, P.nx);
    // Scalar base pointers; every lane adds a 32-bit byte offset.
    const char* __restrict__ base0 = reinterpret_cast<const char*>(fin + P.f_off);
    const char* __restrict__ base1 = base0 + 36 * P.pitch;  // species 1
    char* __restrict__ obase = reinterpret_cast<char*>(fout + P.f_off);
    const uint32_t sp = 36u * (uint32_t)P.pitch;  // species stride in bytes
    ColG g{};
    if (!PY) {
        g.m = cols[P.col_off + xm];
        g.c = cols[P.col_off + x];
        g.p = cols[P.col_off + xp];
    }
    // Halo lanes of wave 0: lane 16 k + j, k = side * 2 + species, j = direction.
    const int hk = (tid >> 4) & 3, hj = tid & 15;
    const int hside = hk >> 1, hs = hk & 1;
    const bool hlane = tid < 64 && hj < 9;
    const int hx = hside ? wrapi(it.x0 + wdt, P.nx) : wrapi(it.x0 - 1, P.nx);
    const int hxm = wrapi(hx - 1, P.nx), hxp = wrapi(hx + 1, P.nx);
    const int hd = hj < 9 ? hj : 0;
    const int hcx = dir_cx(hd), hcy = dir_cy(hd), hopp = dir_opp(hd);
    const int hsx = hcx == 1 ? hxm : (hcx == -1 ? hxp : hx);
    Col hgc{0, 0}, hgs{0, 0};
    if (!PY && tid < 64) {
        hgc = cols[P.col_off + hx];
        hgs = cols[P.col_off + hsx];
    }

    const int64_t n_nodes = (int64_t)P.nx * P.ny;
    double macc[kMonWidth];
#pragma unroll
    for (int j = 0; j < kMonWidth; ++j)
        macc[j] = 0.0;
    double cosx = 0.0, sinx = 0.0;
    if (MODE == kStepMon || MODE == kMonOnly)
        sincospi(2.0 * (double)x / (double)P.nx, &sinx, &cosx);

    auto row_of = [&](int r) -> int { return PY ? wrapi(r, P.ny) : r; };
    auto node_fluid = [&](const Col& c, int rr) -> bool {
        return PY ? true : ((rr >= c.lo) & (rr <= c.hi));
    };

    // Issue the pulls of row r into raw / hraw (loads left in flight).
    float raw[18];
    float hraw = 0.0f;
    bool fl_next = false, hfl_next = false;
    auto issue_row = [&](int r) {
        const int rr = row_of(r);
        int rb[3];
        rb[0] = row_of(r - 1) * P.rstride;
        rb[1] = rr * P.rstride;
        rb[2] = row_of(r + 1) * P.rstride;
        fl_next = act && node_fluid(g.c, rr);
        if (fl_next) {
            uint32_t off[9];
            pull_offsets<PY>(P, rb, rr, xm, x, xp, g, off);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                raw[i] = *reinterpret_cast<const float*>(base0 + off[i]);
                raw[9 + i] = *reinterpret_cast<const float*>(base1 + off[i]);
            }
        }
        hfl_next = node_fluid(hgc, rr);
        if (hlane && hfl_next) {
            const int srb = rb[1 - hcy];
            const bool src_fluid = PY ? true : (((rr - hcy) >= hgs.lo) & ((rr - hcy) <= hgs.hi));
            const uint32_t o = src_fluid ? 4u * ((uint32_t)(hd * P.pitch) + (uint32_t)(srb + hsx))
                                         : 4u * ((uint32_t)(hopp * P.pitch) + (uint32_t)(rb[1] + hx));
            hraw = *reinterpret_cast<const float*>(base0 + o + (hs ? sp : 0u));
        }
    };

    // March direction: y0 < y1 marches up over rows y0 .. y1 - 1; y0 > y1
    // marches down over rows y0 .. y1 + 1.  Row r is pulled in the iteration
    // that collides row r - d.
    const int d = it.y1 > it.y0 ? 1 : -1;
    Mom prev[2], cur[2];
    bool prev_fluid = false;
    issue_row(it.y0 - d);

    for (int r = it.y0 - d; r != it.y1 + d; r += d) {
        const int rr = row_of(r);
        // ---- row r: moments from the pulls issued one iteration earlier ----
        const bool fl = fl_next;
        const bool hfl = hfl_next;
        if (fl) {
            cur[0] = moments9(raw);
            cur[1] = moments9(raw + 9);
            if (MODE == kExport && d * (r - it.y0) >= 0 && d * (it.y1 - r) > 0) {
                const int64_t k = (int64_t)rr * P.nx + x;
#pragma unroll
                for (int i = 0; i < 18; ++i)
                    stage[(int64_t)i * n_nodes + k] = (double)raw[i];
            }
        }
        if (act) {
            ring[r & 3][0][tid + 1] = fl ? cur[0].rho : P.rho_s[0];
            ring[r & 3][1][tid + 1] = fl ? cur[1].rho : P.rho_s[1];
        }
        if (tid < 64) {
            const float v = (hlane && hfl) ? hraw : 0.0f;
            float q[9];
#pragma unroll
            for (int j = 0; j < 9; ++j)
                q[j] = __shfl(v, (tid & ~15) + j, 64);
            const float rh = rho9(q);
            if (hj == 0)
                ring[r & 3][hs][hside ? wdt + 1 : 0] =
                    hfl ? rh : (hs ? P.rho_s[1] : P.rho_s[0]);
        }
        // ---- pulls of row r + d go out before the barrier -----------------
        if (r != it.y1)
            issue_row(r + d);
        lds_barrier();

        // ---- collide row r - d ---------------------------------------------
        if (d * (r - d - it.y0) >= 0 && prev_fluid) {
            const int rc = r - d;
            const int rrc = row_of(rc);
            const int rs = (rc - 1) & 3, rm = rc & 3, rn = (rc + 1) & 3;
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
            const float inv = 1.0f / rho;  // correctly rounded: u_mix carries no bias
            const float ux = (prev[0].jx + prev[1].jx) * inv;
            const float uy = (prev[0].jy + prev[1].jy) * inv;
            const float taum = 0.5f + (ro * P.tau_h[0] + rw * P.tau_h[1]) * inv;
            const float om = 1.0f - __builtin_amdgcn_rcpf(taum);

            if (MODE == kStep || MODE == kStepMon) {
                const uint32_t o = 4u * (uint32_t)(rrc * P.rstride + x);
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float vx = ux + P.G36 * sx[s] + P.g[0];
                    const float vy = uy + P.G36 * sy[s] + P.g[1];
                    float out[9];
                    collide_species(prev[s], vx, vy, om, out);
#pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        // Streaming store: the populations are read back only by
                        // the next step, long after they would have left L2.
                        char* dst = obase + 4 * (s * 9 + i) * P.pitch;
                        __builtin_nontemporal_store(out[i], reinterpret_cast<float*>(dst + o));
                    }
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
    if (P.periodic_y)
        march<BX, MODE, true>(fin, fout, P, it, item_idx, cols, partial, stage, ring, red);
    else
        march<BX, MODE, false>(fin, fout, P, it, item_idx, cols, partial, stage, ring, red);
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
            A[P.f_off + (int64_t)y * P.rstride + (int64_t)(s * 9 + i) * P.pitch + x] =
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
