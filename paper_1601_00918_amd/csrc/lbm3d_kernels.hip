// HIP kernels (gfx950) of the two-component lattice Boltzmann step on the
// D3Q19 lattice, the lattice of the paper's 3-D runs (Sec. 2), for the
// sinusoidal tube (Sec. 3.4) and periodic boxes.
//
// Same model and the same stored state as the D2Q9 kernels: buffer A holds
// the post-collision populations f*_i(x) of the previous step, not yet
// streamed, and a step is a pure pull (f_i(x, t) = f*_i(x - c_i), or the
// half-way bounce-back value f*_opp(i)(x) where x - c_i is solid), followed by
// the regularized collision (Eqs. 3-7) with the interaction force of Eq. 8
// folded into the equilibrium velocity (Eqs. 9-10), and a store of the node's
// own f*.  Every population is read once and written once per step:
// 2 species x 19 directions x (4 B + 4 B) = 304 B per fluid node in FP32,
// 152 B in the 16-bit deviation formats (plus 8 B of reference densities).
//
// Tiling.  A workgroup owns an x-y tile of BXI x BYI nodes and marches along
// z through a strip of planes.  Eq. 8 needs the densities of the 18
// neighbours, including those across the tile edge, so the workgroup also
// pulls the one-node frame around its tile: thread (tx, ty) of a
// (BXI + 2) x (BYI + 2) grid handles node (x0 - 1 + tx, y0 - 1 + ty); every
// thread pulls its node and reduces it to its 20 moments (rho, j and the
// momentum flux Pi per species: the regularized collision depends on the
// populations only through them), the densities go to an LDS ring of four
// planes, and after one barrier the inner threads collide the previous plane.
// Frame nodes are pulled and reduced exactly like inner nodes, so a density is
// bitwise the same whichever workgroup computes it.  The frame costs
// 2 (BXI + BYI) + 4 extra pulls per plane, served from L2: neighbouring tiles
// are dispatched to the same XCD and march side by side, and adjacent strips
// march in opposite directions so the planes they share are read back-to-back.
// Solid neighbours enter the ring as the wall potentials rho_s.
//
// Direction numbering (pairs of opposite directions are adjacent):
//   0 rest; 1, 2 = +-x; 3, 4 = +-y; 5, 6 = +-z;
//   7, 8 = +-(1,1,0); 9, 10 = +-(1,-1,0); 11, 12 = +-(1,0,1);
//   13, 14 = +-(1,0,-1); 15, 16 = +-(0,1,1); 17, 18 = +-(0,1,-1).
// Weights 1/3, 1/18, 1/36 are 12, 2 and 1 times 1/36.
#include "lbm3d_internal.h"
#include "lbm_store.h"

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

namespace lbm3 {
namespace {

using namespace lbm::dev;

constexpr int kQ = 19;
constexpr int kCx[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCy[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCz[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int kOpp[kQ] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
// 36 w_i and 1 / (36 w_i) for i >= 1 (exact: 2 and 1; 1/2 and 1).
constexpr float kW36[kQ] = {12.f, 2.f, 2.f, 2.f, 2.f, 2.f, 2.f, 1.f, 1.f, 1.f,
                            1.f,  1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f};
constexpr float kInvW36[kQ] = {1.f / 12.f, 0.5f, 0.5f, 0.5f, 0.5f, 0.5f, 0.5f, 1.f, 1.f, 1.f,
                               1.f,        1.f,  1.f,  1.f,  1.f,  1.f,  1.f,  1.f, 1.f};

template <int BXI, int BYI>
struct Tile {
    static constexpr int TXW = BXI + 2;  // threads per tile row (frame included)
    static constexpr int TYW = BYI + 2;
    static constexpr int NLIVE = TXW * TYW;
    static constexpr int NT = (NLIVE + 63) / 64 * 64;  // workgroup size
    static constexpr int RXW = TXW + 2;  // reference-ring row (16-bit formats)
    static constexpr int REFN = RXW * (TYW + 2);
};

struct Mom3 {
    float rho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz;
};

// Zeroth, first and second moments of the 19 populations of one species.
// Every density that enters the interaction stencil comes from this one
// expression (same summation order everywhere).
__device__ __forceinline__ Mom3 moments19(const float* f)
{
    float a[9], d[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        a[k] = f[2 * k + 1] + f[2 * k + 2];
        d[k] = f[2 * k + 1] - f[2 * k + 2];
    }
    // a[0..2]: axes x, y, z; a[3], a[4]: xy+-, a[5], a[6]: xz+-, a[7], a[8]: yz+-
    Mom3 m;
    const float axy = a[3] + a[4], axz = a[5] + a[6], ayz = a[7] + a[8];
    m.rho = ((f[0] + (a[0] + a[1])) + (a[2] + axy)) + (axz + ayz);
    m.jx = (d[0] + (d[3] + d[4])) + (d[5] + d[6]);
    m.jy = (d[1] + (d[3] - d[4])) + (d[7] + d[8]);
    m.jz = (d[2] + (d[5] - d[6])) + (d[7] - d[8]);
    m.pxx = a[0] + (axy + axz);
    m.pyy = a[1] + (axy + ayz);
    m.pzz = a[2] + (axz + ayz);
    m.pxy = a[3] - a[4];
    m.pxz = a[5] - a[6];
    m.pyz = a[7] - a[8];
    return m;
}

// Post-collision populations of one species (Eqs. 3, 6, 7, 9) in FP32.
//   m         moments of the pulled populations (scaled like the storage)
//   vx,vy,vz  shifted equilibrium velocity u_mix + F / rho (Eqs. 9-10)
//   om        1 - 1 / tau_mix
// Equilibrium: f_i^eq = w_i rho (1 + P(c_i . v)) with P = E + O,
// E = 4.5 cu^2 - 1.5 v^2 and O = cu (3 - 4.5 v^2 + 4.5 cu^2) for T0 = 1/3, so
// the two directions of a pair share E and take +-O.  The rest parts w_i rho
// are 12, 2 and 1 times one correctly rounded rho / 36, so the moving
// directions carry the same relative rounding and the momentum of the
// equilibrium is unbiased.  Regularized part (Eq. 6): the Hermite projection
// w_i / (2 T0^2) H_i : Pi^neq of the species' own non-equilibrium flux
// Pi^neq = Pi - rho T0 I - j j / rho; with w_i = W_i / 36 it is
// W_i / 8 (c_i c_i : Pi^neq - tr Pi^neq / 3).
template <bool FASTDIV>
__device__ __forceinline__ void collide19(const Mom3& m, float vx, float vy, float vz, float om,
                                          float (&out)[kQ])
{
    const float rinv = __builtin_amdgcn_rcpf(m.rho);
    const float ax = m.jx * rinv, ay = m.jy * rinv, az = m.jz * rinv;
    const float r3 = m.rho * (1.0f / 3.0f);
    const float nxx = m.pxx - (r3 + m.jx * ax);
    const float nyy = m.pyy - (r3 + m.jy * ay);
    const float nzz = m.pzz - (r3 + m.jz * az);
    const float nxy = m.pxy - m.jx * ay;
    const float nxz = m.pxz - m.jx * az;
    const float nyz = m.pyz - m.jy * az;
    const float tr3 = (nxx + nyy + nzz) * (1.0f / 3.0f);
    const float g0 = om * (-1.5f * tr3);
    const float gx = om * (0.25f * (nxx - tr3));
    const float gy = om * (0.25f * (nyy - tr3));
    const float gz = om * (0.25f * (nzz - tr3));
    const float sxy = nxx + nyy - tr3, sxz = nxx + nzz - tr3, syz = nyy + nzz - tr3;
    const float gxyp = om * (0.125f * (sxy + 2.0f * nxy));
    const float gxym = om * (0.125f * (sxy - 2.0f * nxy));
    const float gxzp = om * (0.125f * (sxz + 2.0f * nxz));
    const float gxzm = om * (0.125f * (sxz - 2.0f * nxz));
    const float gyzp = om * (0.125f * (syz + 2.0f * nyz));
    const float gyzm = om * (0.125f * (syz - 2.0f * nyz));
    // correctly rounded (FP32), within about half a unit (16-bit formats)
    const float b5 = FASTDIV ? div36_fast(m.rho) : m.rho / 36.0f;
    const float b1 = 2.0f * b5;
    const float b0 = 12.0f * b5;
    const float vsq15 = 1.5f * (vx * vx + vy * vy + vz * vz);
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
    pair(vx, b1, gx, out[1], out[2]);
    pair(vy, b1, gy, out[3], out[4]);
    pair(vz, b1, gz, out[5], out[6]);
    pair(vx + vy, b5, gxyp, out[7], out[8]);
    pair(vx - vy, b5, gxym, out[9], out[10]);
    pair(vx + vz, b5, gxzp, out[11], out[12]);
    pair(vx - vz, b5, gxzm, out[13], out[14]);
    pair(vy + vz, b5, gyzp, out[15], out[16]);
    pair(vy - vz, b5, gyzm, out[17], out[18]);
}

// 16-bit deviation format on D3Q19 (see lbm_store.h for the element formats):
// d_i = f*_i / w_i - R, R = binary16(rho); d_1..d_18 rounded to nearest even,
// d_0 takes the remainder rho - R - sum_{i>0} w_i d_i (over w_0), rounded
// stochastically.  F holds 36-scaled populations, rho36 the scaled densities.
template <typename S>
__device__ __forceinline__ void encode_node19(const float (&F)[2][kQ], const float (&rho36)[2],
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
    for (int i = 1; i < kQ; ++i) {
        uint32_t b[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            b[s] = S::rne(F[s][i] * kInvW36[i] - R[s]);
            msum[s] += kW36[i] * S::val(b[s]);
        }
        put32(dst + i * plane, b[0] | (b[1] << 16));
    }
    // 36 R is exact (11 significant bits times 9 * 4).
    uint32_t b0[2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
        b0[s] = S::sr(((rho36[s] - 36.0f * R[s]) - msum[s]) * (1.0f / 12.0f), rnd[s]);
    put32(dst, b0[0] | (b0[1] << 16));
    put32(dst + kQ * plane, rb[0] | (rb[1] << 16));
}

__device__ __forceinline__ bool in_run(uint32_t run, int z)
{
    const int lo = (int)(run & 0xffffu), hi1 = (int)(run >> 16);
    return (unsigned)(z - lo) < (unsigned)(hi1 - lo);
}

// Interpolated walls: the linear interpolated bounce-back of Bouzidi,
// Firdaouss and Lallemand (2001) for a population pulled in direction i from a
// solid node, given its half-way value f*_opp(i)(x), the wall's fraction q of
// the link from x along -c_i, and
//   q <  1/2: f*_opp(i)(x + c_i) (the half-way value again if that node is solid),
//   q >= 1/2: f*_i(x).
// (q = 1/2 gives the half-way value itself.)
__device__ __forceinline__ float ibb_blend(float q, float half_way, float extra)
{
    return q < 0.5f ? (2.0f * q) * half_way + (1.0f - 2.0f * q) * extra
                    : half_way * (0.5f / q) + (1.0f - 0.5f / q) * extra;
}

template <int BXI, int BYI, int MODE, bool PER, typename T, bool WALL>
__device__ __forceinline__ void march3(const void* __restrict__ fin, void* __restrict__ fout,
                                       const Inst3Dev& P, const Item3& it, int item_idx,
                                       const uint32_t* __restrict__ runs,
                                       double* __restrict__ partial, double* __restrict__ stage,
                                       uint32_t seed, float* __restrict__ ring,
                                       float2* __restrict__ rref, double* __restrict__ red)
{
    using TL = Tile<BXI, BYI>;
    constexpr int TXW = TL::TXW, NLIVE = TL::NLIVE, NT = TL::NT, RXW = TL::RXW;
    using S = Store<T>;
    using Pair = typename S::Pair;
    constexpr uint32_t PB = S::kPair;
    constexpr float SC = S::kScale;

    const int tid = threadIdx.x;
    const bool live = tid < NLIVE;
    const int tx = live ? tid % TXW : 0, ty = live ? tid / TXW : 0;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int wdt = min(BXI, nx - it.x0), hgt = min(BYI, ny - it.y0);
    const bool need = live && tx <= wdt + 1 && ty <= hgt + 1;
    const bool inner = need && tx >= 1 && tx <= wdt && ty >= 1 && ty <= hgt;
    const int x = wrapi(it.x0 - 1 + tx, nx);
    const int yraw = it.y0 - 1 + ty;
    const int y = PER ? wrapi(yraw, ny) : yraw;
    const int xm = wrapi(x - 1, nx), xp = wrapi(x + 1, nx);
    const int ym = PER ? wrapi(y - 1, ny) : y - 1, yp = PER ? wrapi(y + 1, ny) : y + 1;
    const int rs = P.rs;
    const uint32_t plane = PB * (uint32_t)P.pitch;  // bytes between planes
    const char* __restrict__ base = reinterpret_cast<const char*>(fin);
    char* __restrict__ obase = reinterpret_cast<char*>(fout);
    const float rs0 = SC * P.rho_s[0], rs1 = SC * P.rho_s[1];
    const float G36 = P.G36 * (1.0f / SC);

    // Fluid runs of the 3 x 3 columns around the node: run[1 + dy][1 + dx].
    uint32_t run[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            run[a][b] = 0u;
            if (!PER) {
                const int yy = y + a - 1;
                const int xx = b == 0 ? xm : (b == 1 ? x : xp);
                if (need && yy >= 0 && yy < ny)
                    run[a][b] = runs[yy * nx + xx];
            }
        }

    // Interpolated walls: this column's entry of the link-fraction table.
    WallCol wc{0u, 0u};
    int wlo = 0;
    if constexpr (WALL) {
        if (run[1][1] != kEmptyRun) {
            wc = P.wcol[y * nx + x];
            wlo = (int)(run[1][1] & 0xffffu);
        }
    }

    const int64_t n_nodes = (int64_t)nx * ny * nz;
    double macc[kMon3Width];
#pragma unroll
    for (int j = 0; j < kMon3Width; ++j)
        macc[j] = 0.0;
    double cosx = 0.0, sinx = 0.0;
    if (MODE == kStepMon || MODE == kMonOnly)
        sincospi(2.0 * (double)x / (double)nx, &sinx, &cosx);

    const int d = it.z1 > it.z0 ? 1 : -1;
    auto zwrap = [&](int z) -> int { return PER ? wrapi(z, nz) : z; };

    // Reference-ring entries of this thread (16-bit formats): the
    // (TXW + 2) x (TYW + 2) nodes around the pulled grid, so that the decode
    // of any pull (source x - c_i of a frame node included) finds its R.
    constexpr int REFN = TL::REFN;
    auto ref_node = [&](int e, int& xx, int& yy) -> bool {
        const int ex = e % RXW, ey = e / RXW;
        xx = wrapi(it.x0 - 2 + ex, nx);
        const int yr = it.y0 - 2 + ey;
        yy = PER ? wrapi(yr, ny) : yr;
        return PER || (yy >= 0 && yy < ny);
    };
    int rxx[2] = {0, 0}, ryy[2] = {0, 0};
    bool rok[2] = {false, false};
    if (S::kRef) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int e = tid + k * NT;
            if (e < REFN)
                rok[k] = ref_node(e, rxx[k], ryy[k]);
        }
    }
    auto load_ref = [&](int k, int q) -> uint32_t {
        const int qq = zwrap(q);
        if (!rok[k] || (!PER && (qq < 0 || qq >= nz)))
            return 0u;
        return *reinterpret_cast<const uint32_t*>(
            base + PB * ((uint32_t)((qq * ny + ryy[k]) * rs) + (uint32_t)(kQ * P.pitch) +
                         (uint32_t)rxx[k]));
    };
    auto put_ref = [&](int k, int q, uint32_t v) {
        const int e = tid + k * NT;
        if (e < REFN)
            rref[(q & 3) * REFN + e] = make_float2(h2f(v & 0xffffu), h2f(v >> 16));
    };

    // Issue the pulls of plane r (loads left in flight).
    Pair rawp[kQ];
    bool fl_next = false;
    uint32_t bb_next = 0, rnext[2] = {0u, 0u};
    auto issue_plane = [&](int r) {
        const int zr = zwrap(r);
        fl_next = need && (PER || in_run(run[1][1], r));
        if (fl_next) {
            const int zs[3] = {zwrap(r - 1) * ny, zr * ny, zwrap(r + 1) * ny};  // z - 1, z, z + 1
            const int ys[3] = {ym, y, yp};
            const int xs[3] = {xm, x, xp};
            uint32_t bb = 0;
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const int cx = kCx[i], cy = kCy[i], cz = kCz[i];
                // source node x - c_i
                const bool src_fluid = PER || in_run(run[1 - cy][1 - cx], r - cz);
                const uint32_t o_src =
                    PB * ((uint32_t)((zs[1 - cz] + ys[1 - cy]) * rs) +
                          (uint32_t)(i * P.pitch) + (uint32_t)xs[1 - cx]);
                const uint32_t o_bb = PB * ((uint32_t)((zs[1] + y) * rs) +
                                            (uint32_t)(kOpp[i] * P.pitch) + (uint32_t)x);
                rawp[i] = S::load(base + (src_fluid ? o_src : o_bb));
                bb |= src_fluid ? 0u : (1u << i);
            }
            bb_next = bb;
        }
        if (S::kRef) {
            const int q = r + 2 * d;
            const bool want = d * (q - (it.z1 + d)) <= 0;
#pragma unroll
            for (int k = 0; k < 2; ++k)
                rnext[k] = want ? load_ref(k, q) : 0u;
        }
    };

    if (S::kRef) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int q = it.z0 - 2 * d + j * d;
#pragma unroll
            for (int k = 0; k < 2; ++k)
                put_ref(k, q, load_ref(k, q));
        }
        lds_barrier();
    }
    const uint32_t seed_h = lowbias32(seed);

    Mom3 prev[2], cur[2];
    bool prev_fluid = false;
    issue_plane(it.z0 - d);

    for (int r = it.z0 - d; r != it.z1 + d; r += d) {
        // ---- plane r: moments from the pulls issued one iteration earlier ----
        const bool fl = fl_next;
        if (fl) {
            float raw[2 * kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i)
                S::unpack(rawp[i], raw[i], raw[kQ + i]);
            if (S::kRef) {
                const uint32_t bbm = bb_next;
#pragma unroll
                for (int i = 0; i < kQ; ++i) {
                    const bool bb = (bbm >> i) & 1u;
                    const int sl = bb ? (r & 3) : ((r - kCz[i]) & 3);
                    const int cl = bb ? (ty + 1) * RXW + tx + 1
                                      : (ty + 1 - kCy[i]) * RXW + tx + 1 - kCx[i];
                    const float2 R = rref[sl * REFN + cl];
                    raw[i] = kW36[i] * (R.x + raw[i]);
                    raw[kQ + i] = kW36[i] * (R.y + raw[kQ + i]);
                }
            }
            if constexpr (WALL) {
                // Blend every wall link (waves holding a node next to the
                // wall only).  The node's 18 link fractions come in one batch
                // of loads, then the blend partners in two batches of nine
                // directions, branch-free (lanes without that link load their
                // own slot and keep the pulled value), so a wave waits on
                // memory three times per plane.  What the blends add, summed
                // over i = 1..18 in order, is taken from the rest population,
                // so each species keeps its mass.  Frame and inner threads run
                // the same code, so a density is the same whichever workgroup
                // computes it.
                const uint32_t bbm = bb_next;
                if (__ballot(bbm != 0u) != 0) {
                    const int wa = (int)(wc.ab & 0xffffu), wb = (int)(wc.ab >> 16);
                    const int row = (int)wc.base + (r < wa ? r - wlo : (wa - wlo) + (r - wb));
                    float qv[kQ - 1];
                    {
                        const float2* __restrict__ q2 = reinterpret_cast<const float2*>(
                            P.wq + (int64_t)(bbm ? row : 0) * (kQ - 1));
#pragma unroll
                        for (int k = 0; k < (kQ - 1) / 2; ++k) {
                            const float2 t = q2[k];
                            qv[2 * k] = t.x;
                            qv[2 * k + 1] = t.y;
                        }
                    }
                    const int zs[3] = {(r - 1) * ny, r * ny, (r + 1) * ny};
                    const int ys[3] = {ym, y, yp};
                    const int xs[3] = {xm, x, xp};
                    float dm0 = 0.0f, dm1 = 0.0f;
#pragma unroll
                    for (int g0 = 1; g0 < kQ; g0 += 9) {
                        Pair ex[9];
                        bool far[9];
#pragma unroll
                        for (int t = 0; t < 9; ++t) {
                            const int i = g0 + t;
                            const int cx = kCx[i], cy = kCy[i], cz = kCz[i];
                            const bool wall = (bbm >> i) & 1u;
                            // q < 1/2: f*_opp(i) at x + c_i, if that node is fluid
                            far[t] = wall && qv[i - 1] < 0.5f &&
                                     in_run(run[1 + cy][1 + cx], r + cz);
                            const uint32_t o_far =
                                PB * ((uint32_t)((zs[1 + cz] + ys[1 + cy]) * rs) +
                                      (uint32_t)(kOpp[i] * P.pitch) + (uint32_t)xs[1 + cx]);
                            const uint32_t o_own = PB * ((uint32_t)((zs[1] + y) * rs) +
                                                         (uint32_t)(i * P.pitch) + (uint32_t)x);
                            ex[t] = S::load(base + (far[t] ? o_far : o_own));
                        }
#pragma unroll
                        for (int t = 0; t < 9; ++t) {
                            const int i = g0 + t;
                            const int cx = kCx[i], cy = kCy[i], cz = kCz[i];
                            const bool wall = (bbm >> i) & 1u;
                            const float q = qv[i - 1];
                            float eo, ew;
                            S::unpack(ex[t], eo, ew);
                            if (S::kRef) {
                                const int sl = far[t] ? ((r + cz) & 3) : (r & 3);
                                const int cl = far[t] ? (ty + 1 + cy) * RXW + tx + 1 + cx
                                                      : (ty + 1) * RXW + tx + 1;
                                const float2 R = rref[sl * REFN + cl];
                                eo = kW36[i] * (R.x + eo);
                                ew = kW36[i] * (R.y + ew);
                            }
                            // q < 1/2 with a solid partner: the half-way value
                            const bool keep = !far[t] && q < 0.5f;
                            eo = keep ? raw[i] : eo;
                            ew = keep ? raw[kQ + i] : ew;
                            const float bo = wall ? ibb_blend(q, raw[i], eo) : raw[i];
                            const float bw = wall ? ibb_blend(q, raw[kQ + i], ew) : raw[kQ + i];
                            dm0 += bo - raw[i];
                            dm1 += bw - raw[kQ + i];
                            raw[i] = bo;
                            raw[kQ + i] = bw;
                        }
                    }
                    raw[0] -= dm0;
                    raw[kQ] -= dm1;
                }
            }
            cur[0] = moments19(raw);
            cur[1] = moments19(raw + kQ);
            if (MODE == kExport && inner && d * (r - it.z0) >= 0 && d * (it.z1 - r) > 0) {
                const int64_t k = ((int64_t)zwrap(r) * ny + y) * nx + x;
#pragma unroll
                for (int i = 0; i < 2 * kQ; ++i)
                    stage[(int64_t)i * n_nodes + k] = (double)raw[i] / (double)SC;
            }
        }
        if (live) {
            ring[((r & 3) * 2 + 0) * NLIVE + tid] = fl ? cur[0].rho : rs0;
            ring[((r & 3) * 2 + 1) * NLIVE + tid] = fl ? cur[1].rho : rs1;
        }
        if (S::kRef) {
#pragma unroll
            for (int k = 0; k < 2; ++k)
                put_ref(k, r + 2 * d, rnext[k]);
        }
        // ---- pulls of plane r + d go out before the barrier --------------
        if (r != it.z1)
            issue_plane(r + d);
        lds_barrier();

        // ---- collide plane r - d --------------------------------------------
        if (d * (r - d - it.z0) >= 0 && inner && prev_fluid) {
            const int rc = r - d;
            const int zc = zwrap(rc);
            float sx[2], sy[2], sz[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int b = 1 - s;  // the other species
                const float* lo = ring + (((rc - 1) & 3) * 2 + b) * NLIVE + tid;
                const float* mi = ring + ((rc & 3) * 2 + b) * NLIVE + tid;
                const float* hi = ring + (((rc + 1) & 3) * 2 + b) * NLIVE + tid;
                // neighbour (dx, dy) in the node's own plane / the planes below, above
                auto M = [&](int dx, int dy) { return mi[dy * TXW + dx]; };
                const float xp0 = M(1, 0), xm0 = M(-1, 0), yp0 = M(0, 1), ym0 = M(0, -1);
                const float xyp = M(1, 1) - M(-1, -1), xym = M(1, -1) - M(-1, 1);
                const float xzp = hi[1] - lo[-1], xzm = lo[1] - hi[-1];
                const float yzp = hi[TXW] - lo[-TXW], yzm = lo[TXW] - hi[-TXW];
                sx[s] = 2.0f * (xp0 - xm0) + ((xyp + xym) + (xzp + xzm));
                sy[s] = 2.0f * (yp0 - ym0) + ((xyp - xym) + (yzp + yzm));
                sz[s] = 2.0f * (hi[0] - lo[0]) + ((xzp - xzm) + (yzp - yzm));
            }
            const float ro = prev[0].rho, rw = prev[1].rho;
            const float rho = ro + rw;
            // correctly rounded (or, 16-bit formats, within about half a unit):
            // u_mix carries no bias
            const float inv = S::kRef ? rcp_fast(rho) : 1.0f / rho;
            const float ux = (prev[0].jx + prev[1].jx) * inv;
            const float uy = (prev[0].jy + prev[1].jy) * inv;
            const float uz = (prev[0].jz + prev[1].jz) * inv;
            const float taum = 0.5f + (ro * P.tau_h[0] + rw * P.tau_h[1]) * inv;
            const float om = 1.0f - __builtin_amdgcn_rcpf(taum);

            if (MODE == kStep || MODE == kStepMon) {
                float out[2][kQ];
#pragma unroll
                for (int s = 0; s < 2; ++s)
                    collide19<S::kRef>(prev[s], ux + G36 * sx[s] + P.g[0],
                                       uy + G36 * sy[s] + P.g[1], uz + G36 * sz[s] + P.g[2],
                                       om, out[s]);
                // Streaming stores: read back only by the next step.
                char* dst = obase + PB * ((uint32_t)((zc * ny + y) * rs) + (uint32_t)x);
                if constexpr (S::kRef) {
                    uint32_t rnd[2];
                    split_rnd(lowbias32((uint32_t)((zc * ny + y) * nx + x) ^ seed_h), rnd);
                    const float rho36[2] = {ro, rw};
                    encode_node19<S>(out, rho36, rnd, dst, plane);
                } else {
#pragma unroll
                    for (int i = 0; i < kQ; ++i)
                        S::put(dst + i * plane, out[0][i], out[1][i]);
                }
            }
            if (MODE != kStep) {
                // Physical quantities of the state at time t, in FP64 from the
                // node's FP32 moments and neighbour densities.
                const double isc = 1.0 / (double)SC;
                const double dro = ro * isc, drw = rw * isc, drho = dro + drw;
                const double Gd36 = P.Gd / 36.0 * isc;
                double pm[3];
                const float js[3] = {prev[0].jx, prev[0].jy, prev[0].jz};
                const float jw[3] = {prev[1].jx, prev[1].jy, prev[1].jz};
                const float so[3] = {sx[0], sy[0], sz[0]}, sw[3] = {sx[1], sy[1], sz[1]};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double fo = dro * (Gd36 * (double)so[a] + (double)P.g[a]);
                    const double fw = drw * (Gd36 * (double)sw[a] + (double)P.g[a]);
                    pm[a] = ((double)js[a] + (double)jw[a]) * isc + 0.5 * (fo + fw);
                }
                const double upx = pm[0] / drho, upy = pm[1] / drho, upz = pm[2] / drho;
                if (MODE == kExport) {
                    const int64_t k = ((int64_t)zc * ny + y) * nx + x;
                    stage[38 * n_nodes + k] = dro;
                    stage[39 * n_nodes + k] = drw;
                    stage[40 * n_nodes + k] = upx;
                    stage[41 * n_nodes + k] = upy;
                    stage[42 * n_nodes + k] = upz;
                    stage[43 * n_nodes + k] = (drho - P.Gd * dro * drw) / 3.0;
                } else {
                    macc[0] += dro;
                    macc[1] += drw;
                    macc[2] += pm[0];
                    macc[3] += pm[1];
                    macc[4] += dro * upx;
                    macc[5] += dro * cosx;
                    macc[6] += dro * sinx;
                    const bool bad = !(ro > 0.0f) || !(rw > 0.0f) || !isfinite(upx + upy + upz);
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
        for (int j = 0; j < kMon3Width; ++j) {
            double v = macc[j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1)
                v += __shfl_xor(v, o, 64);
            if (lane == 0)
                red[wave * kMon3Width + j] = v;
        }
        __syncthreads();
        if (tid < kMon3Width) {
            double v = 0.0;
            for (int w = 0; w < NT / 64; ++w)
                v += red[w * kMon3Width + tid];
            partial[(int64_t)item_idx * kMon3Width + tid] = v;
        }
    }
}

// Workgroups of at most 256 threads run three per CU (three waves per SIMD:
// at most 168 registers), two with interpolated walls (at most 256).
template <int BXI, int BYI, int MODE, typename T, bool WALL>
__global__ void __launch_bounds__((Tile<BXI, BYI>::NT),
                                  (Tile<BXI, BYI>::NT <= 256 ? (WALL ? 2 : 3) : 1))
step3_kernel(const void* __restrict__ fin, void* __restrict__ fout, const Inst3Dev P,
             const Item3* __restrict__ items, const uint32_t* __restrict__ runs,
             double* __restrict__ partial, double* __restrict__ stage, uint32_t seed)
{
    using TL = Tile<BXI, BYI>;
    __shared__ float ring[4 * 2 * TL::NLIVE];
    __shared__ float2 rref[Store<T>::kRef ? 4 * TL::REFN : 1];
    __shared__ double red[TL::NT / 64 * kMon3Width];
    const int item_idx = remap_xcd((int)blockIdx.x, (int)gridDim.x);
    const Item3 it = items[item_idx];
    if constexpr (WALL)  // a tube: never periodic in y and z
        march3<BXI, BYI, MODE, false, T, true>(fin, fout, P, it, item_idx, runs, partial, stage,
                                               seed, ring, rref, red);
    else if (P.periodic)
        march3<BXI, BYI, MODE, true, T, false>(fin, fout, P, it, item_idx, runs, partial, stage,
                                               seed, ring, rref, red);
    else
        march3<BXI, BYI, MODE, false, T, false>(fin, fout, P, it, item_idx, runs, partial,
                                                stage, seed, ring, rref, red);
}

__global__ void mon3_reduce_kernel(const double* __restrict__ partial, int n_items,
                                   double* __restrict__ mon)
{
    const int j = threadIdx.x;
    if (j >= kMon3Width)
        return;
    double v = 0.0;
    for (int k = 0; k < n_items; ++k)
        v += partial[(int64_t)k * kMon3Width + j];
    mon[j] = v;
}

// Initial density of species s at node (x, y, z).
__device__ double init_density3(const Init3Dev& ini, const Inst3Dev& P, int s, int x, int y,
                                int z)
{
    bool oil;
    switch (ini.kind) {
    case 0:  // uniform
        return s == 0 ? ini.rho_hi : ini.rho_lo;
    case 1: {  // sphere of oil, periodic distance
        auto pd = [](double v, double c, int n) {
            const double dd = fabs(v - c);
            return fmin(dd, (double)n - dd);
        };
        const double dx = pd((double)x, ini.cx, P.nx), dy = pd((double)y, ini.cy, P.ny),
                     dz = pd((double)z, ini.cz, P.nz);
        oil = (dx * dx + dy * dy + dz * dz) < ini.r * ini.r;
        break;
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
        oil = false;
        for (int k = 0; k < ini.n_slugs; ++k) {
            double rel = fmod((double)x - ini.x0[k], (double)P.nx);
            if (rel < 0.0)
                rel += (double)P.nx;
            oil = oil || rel < ini.length[k];
        }
        break;
    }
    }
    const bool is_hi = (s == 0) ? oil : !oil;
    return is_hi ? ini.rho_hi : ini.rho_lo;
}

// Rest equilibrium f_i = w_i rho0, placed where the first pull reads it: the
// slot (x, i) is read by node x + c_i when that node is fluid, otherwise by x
// itself after bounce-back.  16-bit formats: rho0(reader) - R(x) to nearest
// even, R(x) = binary16(rho0(x)).  Interpolated walls: the slots the first
// pull blends are set so that the blends, and the rest population after the
// mass return, give w_i rho0(x) too (below).
template <typename T>
__global__ void init3_kernel(void* __restrict__ A, const Inst3Dev P,
                             const uint32_t* __restrict__ runs, Init3Dev ini)
{
    using S = Store<T>;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= P.nx)
        return;
    auto fluid = [&](int xx, int yy, int zz) -> bool {
        if (P.periodic)
            return true;
        if (yy < 0 || yy >= P.ny || zz < 0 || zz >= P.nz)
            return false;
        return in_run(runs[yy * P.nx + xx], zz);
    };
    if (!fluid(x, y, z))
        return;
    // Link fractions of this node (interpolated walls, nodes with a wall link).
    const float* qrow = nullptr;
    if (P.wq) {
        const uint32_t run = runs[y * P.nx + x];
        const WallCol wc = P.wcol[y * P.nx + x];
        const int lo = (int)(run & 0xffffu);
        const int wa = (int)(wc.ab & 0xffffu), wb = (int)(wc.ab >> 16);
        if (z < wa || z >= wb)
            qrow = P.wq + (int64_t)((int)wc.base + (z < wa ? z - lo : (wa - lo) + (z - wb))) *
                              (kQ - 1);
    }
    char* node = reinterpret_cast<char*>(A) +
                 (int64_t)S::kPair * (((int64_t)z * P.ny + y) * P.rs + x);
    const int64_t plane = (int64_t)S::kPair * P.pitch;
    float R[2] = {0.0f, 0.0f};
    if constexpr (S::kRef) {
        uint32_t rpair = 0;
        for (int s = 0; s < 2; ++s) {
            const uint32_t rb = f2h_rn((float)init_density3(ini, P, s, x, y, z));
            R[s] = h2f(rb);
            rpair |= rb << (16 * s);
        }
        *reinterpret_cast<uint32_t*>(node + kQ * plane) = rpair;
    }
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const double w = kW36[i] / 36.0;
        int xr = wrapi(x + kCx[i], P.nx), yr = y + kCy[i], zr = z + kCz[i];
        if (P.periodic) {
            yr = wrapi(yr, P.ny);
            zr = wrapi(zr, P.nz);
        }
        if (!fluid(xr, yr, zr)) {
            xr = x;
            yr = y;
            zr = z;
        }
        double rho_o = init_density3(ini, P, 0, xr, yr, zr);
        double rho_w = init_density3(ini, P, 1, xr, yr, zr);
        if (qrow && i > 0 && xr == x && yr == y && zr == z) {
            // x reads this slot as the half-way value of j = opp(i); with the
            // wall at q >= 1/2 the first pull blends it with slot (x, j),
            // which holds w rho0(x + c_j) for the node x + c_j that pulls it.
            // Store the value that makes the blend w_i rho0(x).  (For
            // q < 1/2 the partner already holds w_i rho0(x).)
            const int j = kOpp[i];
            const float q = qrow[j - 1];
            const int xo = wrapi(x + kCx[j], P.nx), yo = y + kCy[j], zo = z + kCz[j];
            if (q >= 0.5f && fluid(xo, yo, zo)) {
                const double two_q = 2.0 * (double)q;
                rho_o = two_q * rho_o - (two_q - 1.0) * init_density3(ini, P, 0, xo, yo, zo);
                rho_w = two_q * rho_w - (two_q - 1.0) * init_density3(ini, P, 1, xo, yo, zo);
            }
        }
        if (qrow && i == 0) {
            // The first pull takes from the rest population what those blends
            // add to their half-way values, (2q - 1) w_j (rho0(x + c_j) -
            // rho0(x)) per link: store it in advance, so that the pulled rest
            // population is w_0 rho0(x).
            const double ro = rho_o, rw = rho_w;
            for (int j = 1; j < kQ; ++j) {
                if (fluid(wrapi(x - kCx[j], P.nx), y - kCy[j], z - kCz[j]))
                    continue;
                const float q = qrow[j - 1];
                const int xo = wrapi(x + kCx[j], P.nx), yo = y + kCy[j], zo = z + kCz[j];
                if (q >= 0.5f && fluid(xo, yo, zo)) {
                    const double c = (2.0 * (double)q - 1.0) * (kW36[j] / kW36[0]);
                    rho_o += c * (init_density3(ini, P, 0, xo, yo, zo) - ro);
                    rho_w += c * (init_density3(ini, P, 1, xo, yo, zo) - rw);
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

template <int BXI, int BYI, int MODE, typename T>
void launch_mode(const void* fin, void* fout, const Inst3Dev& P, const Item3* items,
                 int n_items, const uint32_t* runs, double* partial, double* stage,
                 uint32_t seed, hipStream_t stream)
{
    const dim3 grid(n_items), block(Tile<BXI, BYI>::NT);
    if (P.wq)
        step3_kernel<BXI, BYI, MODE, T, true>
            <<<grid, block, 0, stream>>>(fin, fout, P, items, runs, partial, stage, seed);
    else
        step3_kernel<BXI, BYI, MODE, T, false>
            <<<grid, block, 0, stream>>>(fin, fout, P, items, runs, partial, stage, seed);
}

template <int BXI, int BYI, typename T>
hipError_t launch_tile(int mode, const void* fin, void* fout, const Inst3Dev& P,
                       const Item3* items, int n_items, const uint32_t* runs, double* partial,
                       double* stage, uint32_t seed, hipStream_t stream)
{
    switch (mode) {
    case kStep:
        launch_mode<BXI, BYI, kStep, T>(fin, fout, P, items, n_items, runs, partial, stage,
                                        seed, stream);
        break;
    case kStepMon:
        launch_mode<BXI, BYI, kStepMon, T>(fin, fout, P, items, n_items, runs, partial, stage,
                                           seed, stream);
        break;
    case kMonOnly:
        launch_mode<BXI, BYI, kMonOnly, T>(fin, fout, P, items, n_items, runs, partial, stage,
                                           seed, stream);
        break;
    case kExport:
        launch_mode<BXI, BYI, kExport, T>(fin, fout, P, items, n_items, runs, partial, stage,
                                          seed, stream);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_t(int tile, int mode, const void* fin, void* fout, const Inst3Dev& P,
                    const Item3* items, int n_items, const uint32_t* runs, double* partial,
                    double* stage, uint32_t seed, hipStream_t stream)
{
    static_assert(kTileBx[0] == 32 && kTileBy[0] == 16 && kTileBx[1] == 64 && kTileBy[1] == 8 &&
                      kTileBx[2] == 32 && kTileBy[2] == 8 && kTileBx[3] == 16 && kTileBy[3] == 12,
                  "tile table and instantiations disagree");
    switch (tile) {
    case 0:
        return launch_tile<32, 16, T>(mode, fin, fout, P, items, n_items, runs, partial, stage,
                                      seed, stream);
    case 1:
        return launch_tile<64, 8, T>(mode, fin, fout, P, items, n_items, runs, partial, stage,
                                     seed, stream);
    case 2:
        return launch_tile<32, 8, T>(mode, fin, fout, P, items, n_items, runs, partial, stage,
                                     seed, stream);
    case 3:
        return launch_tile<16, 12, T>(mode, fin, fout, P, items, n_items, runs, partial, stage,
                                      seed, stream);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch3_step(int storage, int tile, int mode, const void* fin, void* fout,
                        const Inst3Dev& P, const Item3* items, int n_items,
                        const uint32_t* runs, double* partial, double* stage, uint32_t seed,
                        hipStream_t stream)
{
    if (n_items <= 0)
        return hipSuccess;
    switch (storage) {
    case 0:
        return launch_t<float>(tile, mode, fin, fout, P, items, n_items, runs, partial, stage,
                               seed, stream);
    case 1:
        return launch_t<F16Tag>(tile, mode, fin, fout, P, items, n_items, runs, partial, stage,
                                seed, stream);
    case 2:
        return launch_t<BF16Tag>(tile, mode, fin, fout, P, items, n_items, runs, partial, stage,
                                 seed, stream);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch3_mon_reduce(const double* partial, int n_items, double* mon,
                              hipStream_t stream)
{
    mon3_reduce_kernel<<<dim3(1), dim3(64), 0, stream>>>(partial, n_items, mon);
    return hipGetLastError();
}

hipError_t launch3_init(int storage, void* A, const Inst3Dev& P, const uint32_t* runs,
                        const Init3Dev& ini, hipStream_t stream)
{
    if (ini.kind != 0 && ini.kind != 1 && ini.kind != 3)
        return hipErrorInvalidValue;
    const dim3 block(256), grid((P.nx + 255) / 256, P.ny, P.nz);
    switch (storage) {
    case 0:
        init3_kernel<float><<<grid, block, 0, stream>>>(A, P, runs, ini);
        break;
    case 1:
        init3_kernel<F16Tag><<<grid, block, 0, stream>>>(A, P, runs, ini);
        break;
    case 2:
        init3_kernel<BF16Tag><<<grid, block, 0, stream>>>(A, P, runs, ini);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm3
