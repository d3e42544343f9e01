// HIP kernels (gfx950) of the two-component D2Q9 lattice Boltzmann step.
//
// Stored state.  Buffer A holds, for every fluid node x and direction i, the
// post-collision population f*_i(x) of the previous step, not yet streamed.
// A step is then a pure "pull": node x gathers f_i(x, t) = f*_i(x - c_i) (or,
// when x - c_i is solid, the half-way bounce-back value f*_opp(i)(x)), which
// are the populations of Eq. 1's left side at time t, collides them and writes
// its own f*(x, t) to buffer B at its own address.  The two species of one
// (node, direction) are stored as one pair, so a node reads 9 pairs and
// writes 9 pairs.  Reads are coalesced (neighbouring lanes read neighbouring
// addresses, shifted by at most one pair) and writes are aligned; every
// population is read once and written once per step: 2 species x 9
// directions x (4 B read + 4 B write) = 144 B per fluid node in FP32.
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
// lanes of wave 0 (one direction per lane) and reduced in the same order as a
// node's own density, so a density is bitwise the same whichever workgroup
// computes it.  Solid neighbours enter the ring as the wall potentials rho_s.
#include "lbm_internal.h"
#include "lbm_store.h"

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

namespace lbm {
namespace {

using namespace dev;

constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// 36 * w_i: the D2Q9 weights are exact multiples of 1/36.
constexpr float kW36[9] = {16.f, 4.f, 4.f, 4.f, 4.f, 1.f, 1.f, 1.f, 1.f};

// 1 / (36 w_i): exact powers of two.
constexpr float kInvW36[9] = {1.f / 16.f, 0.25f, 0.25f, 0.25f, 0.25f, 1.f, 1.f, 1.f, 1.f};

// Population storage formats.  A lattice row of an instance is one block of
// planes; plane i holds, for every column x, the pair (oil, water) of
// direction i, so one load or store moves both species of one (node,
// direction).  FP32 stores f_i itself (8-byte pairs, 9 planes).  The 16-bit
// formats (binary16, bfloat16; 4-byte pairs) store the deviation
// d_i = f*_i(y) / w_i - R(y) of the post-collision population from the
// lattice weight times a reference density R(y) of the same node and
// species, and R(y) itself, in binary16, in a tenth plane.  A slow creeping
// flow changes a population by far less than one unit in the last place of a
// 16-bit number per step; storing the deviation from the node's own density
// leaves only the velocity and stress part to round, so the step's small
// changes are kept.  The two species have bulk densities about 30 times
// apart and each takes both values somewhere in the domain, which is why the
// reference is per node rather than per species.  The encoder makes the
// node's stored mass exact: d_1..d_8 are rounded to nearest even and d_0 takes
// the remainder of rho - R - sum w_i d_i, rounded stochastically (unbiased,
// independent from step to step), so per-node mass errors do not freeze into
// a drift when the flow is steady.  The kernels work in populations scaled by
// 36 (36 f_i = (36 w_i)(R + d_i)), so the weights are the exact factors 16,
// 4 and 1; the regularized collision is linear in the moments and runs
// unchanged on scaled values; the interaction constant, the wall potentials
// and the FP64 monitors and exports take the scale into account.  The format
// types (Store<float>, Store<F16Tag>, Store<BF16Tag>) live in lbm_store.h.

// Encode the scaled post-collision populations F[s][9] of both species at one
// node (scaled densities rho36[s]) into the 16-bit deviation format and store
// the 9 pairs and the reference pair.  plane: bytes between planes.
template <typename S>
__device__ __forceinline__ void encode_node(const float (&F)[2][9], const float (&rho36)[2],
                                            const uint32_t (&rnd)[2], char* dst, uint32_t plane)
{
    uint32_t rb[2];
    float R[2], msum[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        rb[s] = f2h_rn(rho36[s] * (1.0f / 36.0f));
        R[s] = h2f(rb[s]);
        msum[s] = 0.0f;
    }
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        uint32_t b[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            b[s] = S::rne(F[s][i] * kInvW36[i] - R[s]);
            msum[s] += kW36[i] * S::val(b[s]);
        }
        put32(dst + i * plane, b[0] | (b[1] << 16));
    }
    // 36 R is exact (R has 11 significant bits); rho36 - 36 R is exact
    // whenever the two are within a factor of two.
    uint32_t b0[2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
        b0[s] = S::sr(((rho36[s] - 36.0f * R[s]) - msum[s]) * (1.0f / 16.0f), rnd[s]);
    put32(dst, b0[0] | (b0[1] << 16));
    put32(dst + 9 * plane, rb[0] | (rb[1] << 16));
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
__device__ __forceinline__ float dir_w36(int i) { return i == 0 ? 16.f : (i <= 4 ? 4.f : 1.f); }
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

// Scaled population (36 w_i)(R + d) of a 16-bit deviation d with reference
// density R, w36 = 36 w_i in {1, 4, 16}: one rounding of the exact w36 d +
// w36 R, which for a power of two equals the rounded sum scaled, written as an
// FMA so that the conversion of the binary16 d folds into it.  one is 1.0
// hidden from the compiler (which would otherwise turn the w36 = 1 case into
// a separate conversion and add).
__device__ __forceinline__ float dec16(float d, float w36, float R, float one)
{
    return w36 == 1.0f ? fmaf(d, one, R) : fmaf(d, w36, w36 * R);
}

// Halo lanes: within each group of 16 lanes, direction j sits at lane
// kHaloLane[j] and the other lanes hold zero, so that halo_rho's butterfly
// adds exactly the pairs rho9 adds, in its order: lanes (0, 1) = (f1, f3),
// (2, 3) = (f0, 0), (4, 5) = (f2, f4), (8, 9) = (f5, f7), (10, 11) = (f6, f8).
// Adding a zero is exact, and every lane pair holds equal sums after each
// level, so all 16 lanes end with rho9's value, bit for bit.
constexpr int kHaloLane[9] = {2, 0, 4, 1, 5, 8, 10, 9, 11};
__device__ __forceinline__ int halo_dir(int lane)
{
    return lane == 0 ? 1 : lane == 1 ? 3 : lane == 2 ? 0 : lane == 4 ? 2 : lane == 5 ? 4
         : lane == 8 ? 5 : lane == 9 ? 7 : lane == 10 ? 6 : lane == 11 ? 8 : -1;
}

// v + the value of the partner lane selected by the DPP control CTRL (lanes
// of one row of 16).
template <int CTRL>
__device__ __forceinline__ float dpp_pair_sum(float v)
{
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

// Density of a halo node from its 16 halo lanes (whole wave active): lane
// pairs (i, i ^ 1), then (i, i ^ 2) within quads, then mirrored halves of 8
// and of 16.
__device__ __forceinline__ float halo_rho(float v)
{
    v = dpp_pair_sum<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_pair_sum<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_pair_sum<0x141>(v);  // row_half_mirror
    return dpp_pair_sum<0x140>(v);  // row_mirror
}

// Interpolated walls (instances with a wall table, any storage): the wall
// fraction q of the link from node (x, y) along -c_j comes from the table the
// runtime computes in FP64 (a wall exactly half-way gives q = 1/2, and the
// blend below is then the half-way value itself); the linear interpolated
// bounce-back of Bouzidi, Firdaouss and Lallemand (2001) for the population
// pulled in direction j, given its half-way value f*_opp(j)(x) and
//   q <  1/2: f*_opp(j)(x + c_j) (the half-way value again if that node is solid),
//   q >= 1/2: f*_j(x).
// What the blends add to the half-way values, summed over j = 1..8 in order,
// is taken from the node's rest population, so each species keeps its mass.
// Owner and halo lanes use these same functions and the same summation order,
// so a wall node's density is bitwise the same whichever workgroup computes it.
// In the 16-bit formats the blend works on decoded values: the partner is
// decoded with its own node's reference density.
__device__ __forceinline__ float ibb_q(const InstDev& P, int x, int y, const Col& c, int j)
{
    return P.wq[(x * kWallSlots + wall_slot(y, c.lo, c.hi)) * 8 + (j - 1)];
}

__device__ __forceinline__ float ibb_blend(float q, float half_way, float extra)
{
    return q < 0.5f ? (2.0f * q) * half_way + (1.0f - 2.0f * q) * extra
                    : half_way * (0.5f / q) + (1.0f - 0.5f / q) * extra;
}

struct Mom {
    float rho, jx, jy, pxx, pxy, pyy;
    float mxxy, mxyy;  // third moments sum c_x^2 c_y f, sum c_x c_y^2 f
};

// Zeroth, first and second moments of the 9 populations of one species, and
// the two third moments the third-order regularization needs (unused, and
// removed by the compiler, in the second-order kernels).
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
    m.mxxy = d57 - d86;
    m.mxyy = d57 + d86;
    return m;
}

// Fluid test of row y in column c: the plain kernels serve instances whose
// columns hold one run; the extended kernels also test the gap of two-run
// columns.
template <bool EXT>
__device__ __forceinline__ bool col_in(const Col& c, int y)
{
    if constexpr (EXT)
        return col_fluid(c, y);
    else
        return (y >= c.lo) & (y <= c.hi);
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
template <bool R3, bool FASTDIV>
__device__ __forceinline__ void collide_species(const Mom& m, float vx, float vy, float om,
                                                bool reg3, float (&out)[9])
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
    // correctly rounded (FP32 storage), or within about half a unit (the
    // 16-bit formats, FASTDIV): either way no systematic bias in w_i rho
    const float b5 = FASTDIV ? div36_fast(m.rho) : m.rho / 36.0f;
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
    if constexpr (R3) {
        if (reg3) {
            // Third-order Hermite part: on D2Q9 only the xxy and xyy
            // coefficients of f - f^eq(rho, j / rho) survive,
            //   a_xxy = M_xxy - T0 j_y - j_x^2 j_y / rho^2,
            //   a_xyy = M_xyy - T0 j_x - j_x j_y^2 / rho^2,
            // and w_i / (6 T0^3) H3_i : a3 adds -+a_xyy / 2 on the x axis,
            // -+a_xxy / 2 on the y axis and (s_y a_xxy + s_x a_xyy) / 4 on the
            // diagonal (s_x, s_y); odd in c, so mass, momentum and the second
            // moment are unchanged.
            const float axxy = m.mxxy - (m.jy * (1.0f / 3.0f) + m.jy * ax * ax);
            const float axyy = m.mxyy - (m.jx * (1.0f / 3.0f) + m.jx * ay * ay);
            const float t1 = om * (-0.5f * axyy);
            const float t2 = om * (-0.5f * axxy);
            const float t5 = om * (0.25f * (axxy + axyy));
            const float t6 = om * (0.25f * (axxy - axyy));
            out[1] += t1;
            out[3] -= t1;
            out[2] += t2;
            out[4] -= t2;
            out[5] += t5;
            out[7] -= t5;
            out[6] += t6;
            out[8] -= t6;
        }
    }
}

// Byte offsets (relative to the instance's first byte) of the 9 pulled
// (oil, water) pairs at node (x, r).  rb[k] is the pair offset (row index
// times the row stride in pairs) of row r - 1 + k.  Where x - c_i is solid the
// half-way bounce-back source f*_opp(i)(x) is used instead (bit i of the
// returned mask).  Instances are smaller than 4 GiB, so 32-bit offsets suffice.
template <bool PY, uint32_t PB, bool EXT>
__device__ __forceinline__ uint32_t pull_offsets(const InstDev& P, const int (&rb)[3], int r, int xm,
                                                 int x, int xp, const ColG& g, uint32_t (&off)[9])
{
    uint32_t bb = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int cx = kCx[i], cy = kCy[i];
        const int sx = cx == 1 ? xm : (cx == -1 ? xp : x);
        const int srb = rb[1 - cy];
        bool src_fluid = true;
        if (!PY) {
            const Col cc = cx == 1 ? g.m : (cx == -1 ? g.p : g.c);
            const int sy = r - cy;
            src_fluid = col_in<EXT>(cc, sy);
        }
        const uint32_t o_src = PB * ((uint32_t)(i * P.pitch) + (uint32_t)(srb + sx));
        const uint32_t o_bb = PB * ((uint32_t)(kOpp[i] * P.pitch) + (uint32_t)(rb[1] + x));
        off[i] = src_fluid ? o_src : o_bb;
        bb |= src_fluid ? 0u : (1u << i);
    }
    return bb;
}

template <int BX, int MODE, bool PY, typename T, bool EXT>
__device__ __forceinline__ void march(const void* __restrict__ fin, void* __restrict__ fout,
                                      const InstDev& P, const Item& it, int item_idx,
                                      const Col* __restrict__ cols, double* __restrict__ partial,
                                      double* __restrict__ stage, uint32_t seed,
                                      float (&ring)[4][2][BX + 2], float2* __restrict__ rref,
                                      double (&red)[BX / 64][kMonWidth])
{
    const int tid = threadIdx.x;
    const int wdt = min(BX, P.nx - it.x0);
    const bool act = tid < wdt;
    const int x = it.x0 + (act ? tid : 0);
    const int xm = wrapi(x - 1, P.nx), xp = wrapi(x + 1, P.nx);
    using S = Store<T>;
    using Pair = typename S::Pair;
    constexpr uint32_t PB = S::kPair;
    constexpr float SC = S::kScale;
    constexpr int RW = BX + 4;  // reference ring row: columns x0 - 2 .. x0 + BX + 1
    const int RS = P.rstride >> 1;  // row stride in pairs
    const uint32_t plane = PB * (uint32_t)P.pitch;  // bytes between planes
    const char* __restrict__ base = reinterpret_cast<const char*>(fin) + S::kBytes * P.f_off;
    char* __restrict__ obase = reinterpret_cast<char*>(fout) + S::kBytes * P.f_off;
    const float rs0 = SC * P.rho_s[0], rs1 = SC * P.rho_s[1];  // wall potentials (scaled)
    const float G36 = P.G36 * (1.0f / SC);
    ColG g{};
    if (!PY) {
        g.m = cols[P.col_off + xm];
        g.c = cols[P.col_off + x];
        g.p = cols[P.col_off + xp];
    }
    // Halo lanes of wave 0: lanes 16 side + 0 .. 15 serve the column left
    // (side 0) or right (side 1) of the workgroup; lane 16 side + kHaloLane[j]
    // pulls its direction j (the layout lets a four-level butterfly of
    // lane-pair sums reproduce rho9's summation order, halo_rho).
    const int hj = tid & 15, hside = (tid >> 4) & 1;
    const bool hgrp = tid < 32;
    const int hdir = halo_dir(hj);
    const bool hlane = hgrp && hdir >= 0;
    const int hx = hside ? wrapi(it.x0 + wdt, P.nx) : wrapi(it.x0 - 1, P.nx);
    const int hxm = wrapi(hx - 1, P.nx), hxp = wrapi(hx + 1, P.nx);
    const int hd = hdir >= 0 ? hdir : 0;
    const int hcx = dir_cx(hd), hcy = dir_cy(hd), hopp = dir_opp(hd);
    const int hsx = hcx == 1 ? hxm : (hcx == -1 ? hxp : hx);
    Col hgc{0, 0, 1, 0}, hgs{0, 0, 1, 0}, hge{0, 0, 1, 0};  // halo column, its source, the one beyond
    if (!PY && hgrp) {
        hgc = cols[P.col_off + hx];
        hgs = cols[P.col_off + hsx];
        if (EXT)
            hge = cols[P.col_off + (hcx == 1 ? hxp : (hcx == -1 ? hxm : hx))];
    }
    // Reference-density lanes of wave 0 (16-bit formats): lanes 16 side + 12
    // and + 13 load the reference pairs of the two columns beyond each side
    // that halo pulls reach (ring columns 0, 1 and wdt + 2, wdt + 3).
    const bool rlane = S::kRef && hgrp && (hj == 12 || hj == 13);
    const int rcol = hside ? wdt + 2 + (hj - 12) : hj - 12;
    const int rx = wrapi(it.x0 - 2 + rcol, P.nx);

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
        return PY ? true : col_in<EXT>(c, rr);
    };
    // Reference pair of node (xx, row q); rows outside a channel read as 0.
    auto load_ref = [&](int q, int xx) -> uint32_t {
        const int qq = row_of(q);
        if (!PY && (qq < 0 || qq >= P.ny))
            return 0u;
        return *reinterpret_cast<const uint32_t*>(
            base + PB * ((uint32_t)(qq * RS) + (uint32_t)(9 * P.pitch) + (uint32_t)xx));
    };
    auto put_ref = [&](int q, int col, uint32_t v) {
        rref[(q & 3) * RW + col] = make_float2(h2f(v & 0xffffu), h2f(v >> 16));
    };

    // March direction: y0 < y1 marches up over rows y0 .. y1 - 1; y0 > y1
    // marches down over rows y0 .. y1 + 1.  Row r is pulled in the iteration
    // that collides row r - d; its decoding needs the reference densities of
    // rows r - 1 .. r + 1, which enter the ring two rows ahead of the pulls.
    const int d = it.y1 > it.y0 ? 1 : -1;

    // Issue the pulls of row r (loads left in flight).
    Pair rawp[9];
    Pair hrawp{};
    bool fl_next = false, hfl_next = false, hbb_next = false;
    uint32_t bb_next = 0, rnext = 0, hrnext = 0;
    auto issue_row = [&](int r) {
        const int rr = row_of(r);
        int rb[3];
        rb[0] = row_of(r - 1) * RS;
        rb[1] = rr * RS;
        rb[2] = row_of(r + 1) * RS;
        fl_next = act && node_fluid(g.c, rr);
        if (fl_next) {
            uint32_t off[9];
            bb_next = pull_offsets<PY, PB, EXT>(P, rb, rr, xm, x, xp, g, off);
#pragma unroll
            for (int i = 0; i < 9; ++i)
                rawp[i] = S::load(base + off[i]);
        }
        hfl_next = node_fluid(hgc, rr);
        if (hlane && hfl_next) {
            const int srb = rb[1 - hcy];
            const bool src_fluid = PY ? true : col_in<EXT>(hgs, rr - hcy);
            hbb_next = !src_fluid;
            const uint32_t o = src_fluid ? PB * ((uint32_t)(hd * P.pitch) + (uint32_t)(srb + hsx))
                                         : PB * ((uint32_t)(hopp * P.pitch) + (uint32_t)(rb[1] + hx));
            hrawp = S::load(base + o);
        }
        if (S::kRef) {
            const int q = r + 2 * d;
            const bool need = d * (q - (it.y1 + d)) <= 0;
            rnext = (act && need) ? load_ref(q, x) : 0u;
            hrnext = (rlane && need) ? load_ref(q, rx) : 0u;
        }
    };

    if (S::kRef) {
        // Reference densities of the rows around the first pulled row.
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int q = it.y0 - 2 * d + k * d;
            if (act)
                put_ref(q, tid + 2, load_ref(q, x));
            if (rlane)
                put_ref(q, rcol, load_ref(q, rx));
        }
        lds_barrier();
    }
    const uint32_t seed_h = lowbias32(seed);
    float one = 1.0f;
    __asm__("" : "+s"(one));

    Mom prev[2], cur[2];
    bool prev_fluid = false;
    issue_row(it.y0 - d);

    for (int r = it.y0 - d; r != it.y1 + d; r += d) {
        const int rr = row_of(r);
        // ---- row r: moments from the pulls issued one iteration earlier ----
        const bool fl = fl_next;
        const bool hfl = hfl_next;
        if (fl) {
            float raw[18];
#pragma unroll
            for (int i = 0; i < 9; ++i)
                S::unpack(rawp[i], raw[i], raw[9 + i]);
            // Reference densities (16-bit formats) of the nodes around this one:
            // rrow[1 - c_y][c_x] is node (x + c_x, r + c_y), from one of three
            // ring rows.
            const float2* rrow[3] = {rref + ((r + 1) & 3) * RW + tid + 2,   // row r + 1
                                     rref + (r & 3) * RW + tid + 2,         // row r
                                     rref + ((r - 1) & 3) * RW + tid + 2};  // row r - 1
            if (S::kRef) {
                // Reference density of each pull's source node (x - c_i, r -
                // c_y,i): a constant offset from this column in one of three
                // ring rows; the node's own after bounce-back.
                const uint32_t bbm = bb_next;
                const float2 Rown = rrow[1][0];
                if (__ballot(bbm != 0u) == 0) {  // no bounce-back in the wave
#pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        const float2 Rs = rrow[1 + kCy[i]][-kCx[i]];
                        raw[i] = dec16(raw[i], kW36[i], Rs.x, one);
                        raw[9 + i] = dec16(raw[9 + i], kW36[i], Rs.y, one);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        const float2 Rs = rrow[1 + kCy[i]][-kCx[i]];
                        const bool bb = (bbm >> i) & 1u;
                        const float Ro = bb ? Rown.x : Rs.x, Rw = bb ? Rown.y : Rs.y;
                        raw[i] = dec16(raw[i], kW36[i], Ro, one);
                        raw[9 + i] = dec16(raw[9 + i], kW36[i], Rw, one);
                    }
                }
            }
            if constexpr (EXT && !PY) {
                if (P.wq && bb_next) {
                    float dmo = 0.0f, dmw = 0.0f;  // added beyond half-way bounce-back
#pragma unroll
                    for (int i = 1; i < 9; ++i) {
                        if (!((bb_next >> i) & 1u))
                            continue;
                        const int cx = kCx[i], cy = kCy[i];
                        const float q = ibb_q(P, x, rr, g.c, i);
                        uint32_t o_extra;
                        bool use = true;
                        if (q < 0.5f) {
                            const Col ce = cx == 1 ? g.p : (cx == -1 ? g.m : g.c);
                            const int ye = rr + cy;
                            use = col_fluid(ce, ye);
                            const int xe = cx == 1 ? xp : (cx == -1 ? xm : x);
                            o_extra = PB * ((uint32_t)(kOpp[i] * P.pitch) +
                                            (uint32_t)(ye * RS + xe));
                        } else {
                            o_extra = PB * ((uint32_t)(i * P.pitch) + (uint32_t)(rr * RS + x));
                        }
                        float eo = raw[i], ew = raw[9 + i];
                        if (use) {
                            S::unpack(S::load(base + o_extra), eo, ew);
                            if constexpr (S::kRef) {  // x + c_i, or the node itself
                                const float2 Re = q < 0.5f ? rrow[1 - cy][cx] : rrow[1][0];
                                eo = dec16(eo, kW36[i], Re.x, one);
                                ew = dec16(ew, kW36[i], Re.y, one);
                            }
                        }
                        const float bo = ibb_blend(q, raw[i], eo);
                        const float bw = ibb_blend(q, raw[9 + i], ew);
                        dmo += bo - raw[i];
                        dmw += bw - raw[9 + i];
                        raw[i] = bo;
                        raw[9 + i] = bw;
                    }
                    raw[0] -= dmo;
                    raw[9] -= dmw;
                }
            }
            cur[0] = moments9(raw);
            cur[1] = moments9(raw + 9);
            if (MODE == kExport && d * (r - it.y0) >= 0 && d * (it.y1 - r) > 0) {
                const int64_t k = (int64_t)rr * P.nx + x;
#pragma unroll
                for (int i = 0; i < 18; ++i)
                    stage[(int64_t)i * n_nodes + k] = (double)raw[i] / (double)SC;
            }
        }
        if (act) {
            ring[r & 3][0][tid + 1] = fl ? cur[0].rho : rs0;
            ring[r & 3][1][tid + 1] = fl ? cur[1].rho : rs1;
        }
        if (tid < 64) {
            float v0 = 0.0f, v1 = 0.0f;
            float e0 = 0.0f, e1 = 0.0f;  // interpolated walls: added beyond half-way
            if (hlane && hfl) {
                S::unpack(hrawp, v0, v1);
                if (S::kRef) {
                    const int ch = hside ? wdt + 2 : 1;
                    const int sl = hbb_next ? (r & 3) : ((r - hcy) & 3);
                    const int cl = hbb_next ? ch : ch - hcx;
                    const float2 R = rref[sl * RW + cl];
                    const float w = dir_w36(hd);
                    v0 = fmaf(v0, w, w * R.x);  // = w (R + v0): w is a power of two
                    v1 = fmaf(v1, w, w * R.y);
                }
                if constexpr (EXT && !PY) {
                    if (P.wq && hbb_next) {
                        const float q = ibb_q(P, hx, rr, hgc, hd);
                        uint32_t o_extra;
                        bool use = true;
                        if (q < 0.5f) {
                            const int ye = rr + hcy;
                            use = col_fluid(hge, ye);
                            const int xe = hcx == 1 ? hxp : (hcx == -1 ? hxm : hx);
                            o_extra = PB * ((uint32_t)(hopp * P.pitch) +
                                            (uint32_t)(ye * RS + xe));
                        } else {
                            o_extra = PB * ((uint32_t)(hd * P.pitch) + (uint32_t)(rr * RS + hx));
                        }
                        float eo = v0, ew = v1;
                        if (use) {
                            S::unpack(S::load(base + o_extra), eo, ew);
                            if constexpr (S::kRef) {  // x + c_j, or the node itself
                                const int ch = hside ? wdt + 2 : 1;
                                const int sl = q < 0.5f ? ((r + hcy) & 3) : (r & 3);
                                const int cl = q < 0.5f ? ch + hcx : ch;
                                const float2 Re = rref[sl * RW + cl];
                                const float w = dir_w36(hd);
                                eo = fmaf(eo, w, w * Re.x);
                                ew = fmaf(ew, w, w * Re.y);
                            }
                        }
                        const float b0 = ibb_blend(q, v0, eo);
                        const float b1 = ibb_blend(q, v1, ew);
                        e0 = b0 - v0;
                        e1 = b1 - v1;
                        v0 = b0;
                        v1 = b1;
                    }
                }
            }
            float rh0, rh1;
            if constexpr (EXT && !PY) {
                float q0[9], q1[9];
#pragma unroll
                for (int j = 0; j < 9; ++j) {
                    q0[j] = __shfl(v0, (tid & ~15) + kHaloLane[j], 64);
                    q1[j] = __shfl(v1, (tid & ~15) + kHaloLane[j], 64);
                }
                if (P.wq) {
                    float dm0 = 0.0f, dm1 = 0.0f;
#pragma unroll
                    for (int j = 1; j < 9; ++j) {
                        dm0 += __shfl(e0, (tid & ~15) + kHaloLane[j], 64);
                        dm1 += __shfl(e1, (tid & ~15) + kHaloLane[j], 64);
                    }
                    q0[0] -= dm0;
                    q1[0] -= dm1;
                }
                rh0 = rho9(q0);
                rh1 = rho9(q1);
            } else {
                rh0 = halo_rho(v0);
                rh1 = halo_rho(v1);
            }
            if (hgrp && hj == 0) {
                const int col = hside ? wdt + 1 : 0;
                ring[r & 3][0][col] = hfl ? rh0 : rs0;
                ring[r & 3][1][col] = hfl ? rh1 : rs1;
            }
        }
        if (S::kRef) {
            // Reference row r + 2d (loaded with the pulls of row r).
            if (act)
                put_ref(r + 2 * d, tid + 2, rnext);
            if (rlane)
                put_ref(r + 2 * d, rcol, hrnext);
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
            // correctly rounded (or, 16-bit formats, within about half a unit):
            // u_mix carries no bias
            const float inv = S::kRef ? rcp_fast(rho) : 1.0f / rho;
            const float ux = (prev[0].jx + prev[1].jx) * inv;
            const float uy = (prev[0].jy + prev[1].jy) * inv;
            const float taum = 0.5f + (ro * P.tau_h[0] + rw * P.tau_h[1]) * inv;
            const float om = 1.0f - __builtin_amdgcn_rcpf(taum);

            if (MODE == kStep || MODE == kStepMon) {
                float out[2][9];
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float vx = ux + G36 * sx[s] + P.g[0];
                    const float vy = uy + G36 * sy[s] + P.g[1];
                    collide_species<EXT, S::kRef>(prev[s], vx, vy, om, P.reg3 != 0, out[s]);
                }
                // Streaming stores: the populations are read back only by the
                // next step, long after they would have left L2.
                char* dst = obase + PB * ((uint32_t)(rrc * RS) + (uint32_t)x);
                if constexpr (S::kRef) {
                    uint32_t rnd[2];
                    split_rnd(lowbias32((uint32_t)(rrc * P.nx + x) ^ seed_h), rnd);
                    const float rho36[2] = {ro, rw};
                    encode_node<S>(out, rho36, rnd, dst, plane);
                } else {
#pragma unroll
                    for (int i = 0; i < 9; ++i)
                        S::put(dst + i * plane, out[0][i], out[1][i]);
                }
            }
            if (MODE != kStep) {
                // Physical quantities of the state at time t, evaluated in FP64
                // from the node's FP32 moments and neighbour densities.
                const double isc = 1.0 / (double)SC;
                const double dro = ro * isc, drw = rw * isc, drho = dro + drw;
                const double Gd36 = P.Gd / 36.0 * isc;
                const double fxo = dro * (Gd36 * (double)sx[0] + (double)P.g[0]);
                const double fyo = dro * (Gd36 * (double)sy[0] + (double)P.g[1]);
                const double fxw = drw * (Gd36 * (double)sx[1] + (double)P.g[0]);
                const double fyw = drw * (Gd36 * (double)sy[1] + (double)P.g[1]);
                const double px = ((double)prev[0].jx + (double)prev[1].jx) * isc + 0.5 * (fxo + fxw);
                const double py = ((double)prev[0].jy + (double)prev[1].jy) * isc + 0.5 * (fyo + fyw);
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

template <int BX, int MODE, typename T, bool EXT>
__global__ void __launch_bounds__(BX)
step_kernel(const void* __restrict__ fin, void* __restrict__ fout,
            const InstDev* __restrict__ insts, const Item* __restrict__ items, int item_base,
            const Col* __restrict__ cols, double* __restrict__ partial,
            double* __restrict__ stage, uint32_t seed, const uint32_t* __restrict__ seed_dev)
{
    __shared__ float ring[4][2][BX + 2];
    __shared__ float2 rref[Store<T>::kRef ? 4 * (BX + 4) : 1];
    __shared__ double red[BX / 64][kMonWidth];
    const uint32_t sd = seed + (seed_dev ? seed_dev[0] : 0u);
    const int item_idx = item_base + remap_xcd((int)blockIdx.x, (int)gridDim.x);
    const Item it = items[item_idx];
    const InstDev P = insts[it.inst];
    if (P.periodic_y)
        march<BX, MODE, true, T, EXT>(fin, fout, P, it, item_idx, cols, partial, stage, sd, ring,
                                     rref, red);
    else
        march<BX, MODE, false, T, EXT>(fin, fout, P, it, item_idx, cols, partial, stage, sd, ring,
                                      rref, red);
}

__global__ void set_seed_kernel(uint32_t* seed_dev, uint32_t v)
{
    if (threadIdx.x == 0)
        seed_dev[0] = v;
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
    default: {  // slugs: (x - x0_k) mod nx < length_k for some k
        if (ini.width > 0.0) {
            // tanh interfaces at x0_k - 1/2 and x0_k + length_k - 1/2 (and
            // their periodic images), the oil fraction phi clipped to [0, 1]
            double phi = 0.0;
            for (int k = 0; k < ini.n_slugs; ++k) {
                double a = fmod(ini.x0[k], (double)P.nx);
                if (a < 0.0)
                    a += (double)P.nx;
                for (int img = -1; img <= 1; ++img) {
                    const double xx = (double)x + (double)img * (double)P.nx;
                    phi += 0.5 * (tanh((xx - a + 0.5) / ini.width) -
                                  tanh((xx - a - ini.length[k] + 0.5) / ini.width));
                }
            }
            phi = fmin(fmax(phi, 0.0), 1.0);
            const double span = ini.rho_hi - ini.rho_lo;
            return s == 0 ? ini.rho_lo + span * phi : ini.rho_hi - span * phi;
        }
        oil = 0.0;
        for (int k = 0; k < ini.n_slugs; ++k) {
            double rel = fmod((double)x - ini.x0[k], (double)P.nx);
            if (rel < 0.0)
                rel += (double)P.nx;
            if (rel < ini.length[k])
                oil = 1.0;
        }
        break;
    }
    }
    const bool is_hi = (s == 0) ? (oil != 0.0) : (oil == 0.0);
    return is_hi ? ini.rho_hi : ini.rho_lo;
}

// Rest equilibrium f_i = w_i rho0, placed where the first pull reads it: the
// slot (x, i) is read by node x + c_i (direction i) when that node is fluid,
// otherwise by node x itself after bounce-back (direction opp(i)).  In the
// 16-bit formats the slot holds rho0(reader) - R(x), rounded to nearest even,
// with R(x) the binary16 value of rho0(x).
template <typename T>
__global__ void init_kernel(void* __restrict__ A, const InstDev* __restrict__ insts, int inst,
                            const Col* __restrict__ cols, InitDev ini)
{
    using S = Store<T>;
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
        return col_fluid(cols[P.col_off + xx], yy);
    };
    if (!fluid(x, y))
        return;
    char* node = reinterpret_cast<char*>(A) +
                 S::kBytes * (P.f_off + (int64_t)y * P.rstride) + S::kPair * (int64_t)x;
    const int64_t plane = (int64_t)S::kPair * P.pitch;
    float R[2] = {0.0f, 0.0f};
    if constexpr (S::kRef) {
        uint32_t rpair = 0;
        for (int s = 0; s < 2; ++s) {
            const uint32_t rb = f2h_rn((float)init_density(ini, P, s, x, y));
            R[s] = h2f(rb);
            rpair |= rb << (16 * s);
        }
        *reinterpret_cast<uint32_t*>(node + 9 * plane) = rpair;
    }
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
        double rho_o = init_density(ini, P, 0, xr, yr);
        double rho_w = init_density(ini, P, 1, xr, yr);
        // Interpolated walls: x reads this slot as the half-way value of
        // direction j = opp(i); when the wall is at q >= 1/2 the first
        // pull blends it with slot (x, j), which holds w rho0(x + c_j) for
        // the node x + c_j that pulls it.  Store the value that makes the
        // blend w_i rho0(x), the rest state.  (For q < 1/2 the blend
        // partner already holds w_i rho0(x).)
        if (P.wq && xr == x && yr == y && i > 0) {
            const int j = kOpp[i];
            const float q = ibb_q(P, x, y, cols[P.col_off + x], j);
            const int xo = wrapi(x + kCx[j], P.nx), yo = y + kCy[j];
            if (q >= 0.5f && fluid(xo, yo)) {
                const double two_q = 2.0 * (double)q;
                rho_o = two_q * rho_o - (two_q - 1.0) * init_density(ini, P, 0, xo, yo);
                rho_w = two_q * rho_w - (two_q - 1.0) * init_density(ini, P, 1, xo, yo);
            }
        }
        // The first pull takes from the rest population what those
        // blends add to their half-way slots, (2q - 1) w_j (rho0(x + c_j)
        // - rho0(x)) per link; store it in advance so that the pulled rest
        // population is w_0 rho0(x).
        if (P.wq && i == 0) {
            const double ro = rho_o, rw = rho_w;
            for (int j = 1; j < 9; ++j) {
                if (fluid(wrapi(x - kCx[j], P.nx), y - kCy[j]))
                    continue;
                const float q = ibb_q(P, x, y, cols[P.col_off + x], j);
                const int xo = wrapi(x + kCx[j], P.nx), yo = y + kCy[j];
                if (q >= 0.5f && fluid(xo, yo)) {
                    const double c = (2.0 * (double)q - 1.0) * (kW36[j] / kW36[0]);
                    rho_o += c * (init_density(ini, P, 0, xo, yo) - ro);
                    rho_w += c * (init_density(ini, P, 1, xo, yo) - rw);
                }
            }
        }
        if constexpr (S::kRef)
            *reinterpret_cast<uint32_t*>(node + i * plane) =
                S::rne((float)(rho_o - (double)R[0])) |
                (S::rne((float)(rho_w - (double)R[1])) << 16);
        else
            S::put(node + i * plane, (float)(w * rho_o), (float)(w * rho_w));
    }
}

// ext: the extended kernels, with the branches of the optional features
// (third-order regularization, interpolated walls) that instances with
// those flags take.  Monitors and exports need the extended pull too.
template <int BX, typename T>
hipError_t launch_step_bx(int mode, bool ext, const void* fin, void* fout, const InstDev* insts,
                          const Item* items, int item_base, int n_items, const Col* cols,
                          double* partial, double* stage, uint32_t seed,
                          const uint32_t* seed_dev, hipStream_t stream)
{
    const dim3 grid(n_items), block(BX);
#define LBM_LAUNCH(M)                                                                      \
    do {                                                                                   \
        if (ext)                                                                           \
            step_kernel<BX, M, T, true><<<grid, block, 0, stream>>>(                       \
                fin, fout, insts, items, item_base, cols, partial, stage, seed, seed_dev); \
        else                                                                               \
            step_kernel<BX, M, T, false><<<grid, block, 0, stream>>>(                      \
                fin, fout, insts, items, item_base, cols, partial, stage, seed, seed_dev); \
    } while (0)
    switch (mode) {
    case kStep:
        LBM_LAUNCH(kStep);
        break;
    case kStepMon:
        LBM_LAUNCH(kStepMon);
        break;
    case kMonOnly:
        LBM_LAUNCH(kMonOnly);
        break;
    case kExport:
        LBM_LAUNCH(kExport);
        break;
    default:
        return hipErrorInvalidValue;
    }
#undef LBM_LAUNCH
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step_t(int bx, int mode, bool ext, const void* fin, void* fout, const InstDev* insts,
                         const Item* items, int item_base, int n_items, const Col* cols,
                         double* partial, double* stage, uint32_t seed, const uint32_t* seed_dev,
                         hipStream_t stream)
{
    switch (bx) {
    case 64:
        return launch_step_bx<64, T>(mode, ext, fin, fout, insts, items, item_base, n_items, cols,
                                     partial, stage, seed, seed_dev, stream);
    case 128:
        return launch_step_bx<128, T>(mode, ext, fin, fout, insts, items, item_base, n_items, cols,
                                      partial, stage, seed, seed_dev, stream);
    case 256:
        return launch_step_bx<256, T>(mode, ext, fin, fout, insts, items, item_base, n_items, cols,
                                      partial, stage, seed, seed_dev, stream);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_step(int storage, int bx, int mode, bool ext, const void* fin, void* fout,
                       const InstDev* insts, const Item* items, int item_base, int n_items,
                       const Col* cols, double* partial, double* stage, uint32_t seed,
                       const uint32_t* seed_dev, hipStream_t stream)
{
    if (n_items <= 0)
        return hipSuccess;
    switch (storage) {
    case 0:
        return launch_step_t<float>(bx, mode, ext, fin, fout, insts, items, item_base, n_items, cols,
                                    partial, stage, seed, seed_dev, stream);
    case 1:
        return launch_step_t<F16Tag>(bx, mode, ext, fin, fout, insts, items, item_base, n_items, cols,
                                     partial, stage, seed, seed_dev, stream);
    case 2:
        return launch_step_t<BF16Tag>(bx, mode, ext, fin, fout, insts, items, item_base, n_items,
                                      cols, partial, stage, seed, seed_dev, stream);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_set_seed(uint32_t* seed_dev, uint32_t value, hipStream_t stream)
{
    set_seed_kernel<<<dim3(1), dim3(64), 0, stream>>>(seed_dev, value);
    return hipGetLastError();
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

hipError_t launch_init(int storage, void* A, const InstDev* insts, int inst, const Col* cols,
                       int nx, int ny, const InitDev& ini, hipStream_t stream)
{
    if (ini.kind < 0 || ini.kind > 3)
        return hipErrorInvalidValue;
    const dim3 block(256), grid((nx + 255) / 256, ny);
    switch (storage) {
    case 0:
        init_kernel<float><<<grid, block, 0, stream>>>(A, insts, inst, cols, ini);
        break;
    case 1:
        init_kernel<F16Tag><<<grid, block, 0, stream>>>(A, insts, inst, cols, ini);
        break;
    case 2:
        init_kernel<BF16Tag><<<grid, block, 0, stream>>>(A, insts, inst, cols, ini);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm
