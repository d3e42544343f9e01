// Host runtime behind include/lbm3d.h: validation, voxelisation of the tube or
// mask into per-column fluid runs along z, work-item tiling, workspace
// carving, launch sequencing and export to the host.
#include "lbm3d.h"
#include "lbm3d_internal.h"
#include "lbm_ctx.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using lbm::fail;
using namespace lbm3;

namespace {

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(LBM_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kMinStrip = 4;
constexpr int kDefaultStrip = 8;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int pitch_of(int nx) { return (int)align_up((size_t)nx, 64); }
int planes_of(int storage) { return storage == LBM_STORE_F32 ? 19 : 20; }
size_t pair_bytes(int storage) { return storage == LBM_STORE_F32 ? 8 : 4; }

size_t buffer_bytes(const lbm3d_geom& g, int storage)
{
    return (size_t)g.nz * g.ny * planes_of(storage) * pitch_of(g.nx) * pair_bytes(storage);
}

int64_t max_items(const lbm3d_geom& g)
{
    int64_t m = 0;
    for (int k = 0; k < kTiles3; ++k)
        m = std::max<int64_t>(m, (int64_t)((g.nx + kTileBx[k] - 1) / kTileBx[k]) *
                                     ((g.ny + kTileBy[k] - 1) / kTileBy[k]) *
                                     ((g.nz + kMinStrip - 1) / kMinStrip));
    return m;
}

struct Layout3 {
    size_t buf_bytes, off_buf[2], off_snap, off_items, off_runs, off_partial, off_mon,
        off_stage, off_wcol, off_wq, total;
    int64_t n_items_max;
};

Layout3 layout_of(const lbm3d_geom& g, int storage_and_opts, int64_t wall_rows)
{
    const int storage = storage_and_opts & 0xff;
    Layout3 L{};
    const int64_t nodes = (int64_t)g.nx * g.ny * g.nz;
    L.n_items_max = max_items(g);
    L.buf_bytes = align_up(buffer_bytes(g, storage), kAlign);
    size_t o = 0;
    L.off_buf[0] = o;
    o += L.buf_bytes;
    L.off_buf[1] = o;
    o += L.buf_bytes;
    L.off_snap = o;
    if (storage_and_opts & LBM_OPT_SNAPSHOT)
        o += L.buf_bytes;
    L.off_items = o;
    o = align_up(o + sizeof(Item3) * L.n_items_max, kAlign);
    L.off_runs = o;
    o = align_up(o + sizeof(uint32_t) * (size_t)g.nx * g.ny, kAlign);
    L.off_partial = o;
    o = align_up(o + sizeof(double) * kMon3Width * L.n_items_max, kAlign);
    L.off_mon = o;
    o = align_up(o + sizeof(double) * kMon3Width, kAlign);
    L.off_stage = o;
    o = align_up(o + sizeof(double) * kExport3Fields * (size_t)nodes, kAlign);
    L.off_wcol = o;
    L.off_wq = o;
    if (g.wall_interp) {
        o = align_up(o + sizeof(WallCol) * (size_t)g.nx * g.ny, kAlign);
        L.off_wq = o;
        // at least one row: lanes without a wall link read row 0
        o = align_up(o + sizeof(float) * 18 * (size_t)std::max<int64_t>(wall_rows, 1), kAlign);
    }
    L.total = o;
    return L;
}

lbm_status check_geom(const lbm3d_geom* g, int storage)
{
    if (!g)
        return fail(LBM_ERR_INVALID, "lbm3d: geometry is NULL");
    if (g->nx < 3 || g->ny < 3 || g->nz < 3 || g->nx > 32768 || g->ny > 32768 || g->nz > 32767)
        return fail(LBM_ERR_INVALID, "lbm3d: lattice size %d x %d x %d out of range", g->nx,
                    g->ny, g->nz);
    if (storage != LBM_STORE_F32 && storage != LBM_STORE_F16 && storage != LBM_STORE_BF16)
        return fail(LBM_ERR_UNSUPPORTED, "lbm3d: unknown storage format %d", storage);
    // The kernels address a buffer with 32-bit byte offsets.
    if (buffer_bytes(*g, storage) >= ((size_t)1 << 32))
        return fail(LBM_ERR_UNSUPPORTED,
                    "lbm3d: lattice %d x %d x %d too large (a population buffer exceeds 4 GiB)",
                    g->nx, g->ny, g->nz);
    switch (g->kind) {
    case LBM3D_GEOM_BOX:
    case LBM3D_GEOM_MASK:
        if (g->wall_interp != 0)
            return fail(LBM_ERR_UNSUPPORTED,
                        "lbm3d: interpolated walls need the analytic tube geometry");
        break;
    default:
        break;
    }
    switch (g->kind) {
    case LBM3D_GEOM_BOX:
        return LBM_OK;
    case LBM3D_GEOM_TUBE:
        if (!(g->lambda > 0.0) || !(g->r0 > 0.0) || !(g->a >= 0.0) ||
            !std::isfinite(g->lambda + g->r0 + g->a))
            return fail(LBM_ERR_INVALID, "lbm3d: tube needs lambda > 0, r0 > 0, a >= 0");
        if (g->wall_interp != 0 && g->wall_interp != 1)
            return fail(LBM_ERR_INVALID, "lbm3d: wall_interp must be 0 or 1");
        return LBM_OK;
    case LBM3D_GEOM_MASK:
        if (!g->mask)
            return fail(LBM_ERR_INVALID, "lbm3d: mask geometry without a mask");
        return LBM_OK;
    default:
        return fail(LBM_ERR_INVALID, "lbm3d: unknown geometry kind %d", g->kind);
    }
}

lbm_status check_fluid(const lbm3d_fluid* f)
{
    if (!f)
        return fail(LBM_ERR_INVALID, "lbm3d: fluid is NULL");
    for (int s = 0; s < 2; ++s) {
        if (!(f->tau[s] > 0.5) || !std::isfinite(f->tau[s]))
            return fail(LBM_ERR_INVALID, "lbm3d: tau[%d] = %g must be finite and > 1/2", s,
                        f->tau[s]);
        if (!std::isfinite(f->rho_s[s]) || f->rho_s[s] < 0.0)
            return fail(LBM_ERR_INVALID, "lbm3d: rho_s[%d] must be finite and >= 0", s);
    }
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(f->g[a]) || std::fabs(f->g[a]) > 0.1)
            return fail(LBM_ERR_INVALID, "lbm3d: |g[%d]| must be <= 0.1", a);
    if (!std::isfinite(f->G))
        return fail(LBM_ERR_INVALID, "lbm3d: G must be finite");
    return LBM_OK;
}

uint32_t pack_run(int lo, int hi)
{
    return lo <= hi ? ((uint32_t)lo | ((uint32_t)(hi + 1) << 16)) : kEmptyRun;
}

// Fluid runs along z of every (x, y) column, [ny][nx].
lbm_status voxelise(const lbm3d_geom& g, std::vector<uint32_t>& runs)
{
    runs.assign((size_t)g.nx * g.ny, kEmptyRun);
    if (g.kind == LBM3D_GEOM_BOX) {
        for (auto& r : runs)
            r = pack_run(0, g.nz - 1);
        return LBM_OK;
    }
    if (g.kind == LBM3D_GEOM_TUBE) {
        const double yc = 0.5 * (g.ny - 1), zc = 0.5 * (g.nz - 1);
        for (int x = 0; x < g.nx; ++x) {
            const double r = g.r0 + g.a * std::cos(2.0 * M_PI * (double)x / g.lambda);
            for (int y = 0; y < g.ny; ++y) {
                int lo = g.nz, hi = -1;
                const double dy = (double)y - yc;
                for (int z = 0; z < g.nz; ++z) {
                    const double dz = (double)z - zc;
                    if (dy * dy + dz * dz < r * r) {
                        lo = std::min(lo, z);
                        hi = std::max(hi, z);
                    }
                }
                runs[(size_t)y * g.nx + x] = pack_run(lo, hi);
            }
        }
        return LBM_OK;
    }
    for (int y = 0; y < g.ny; ++y)
        for (int x = 0; x < g.nx; ++x) {
            int lo = -1, hi = -1;
            for (int z = 0; z < g.nz; ++z)
                if (g.mask[((size_t)z * g.ny + y) * g.nx + x]) {
                    if (lo < 0)
                        lo = z;
                    else if (hi != z - 1)
                        return fail(LBM_ERR_UNSUPPORTED,
                                    "lbm3d: mask column (x %d, y %d) has more than one run of "
                                    "fluid nodes along z",
                                    x, y);
                    hi = z;
                }
            runs[(size_t)y * g.nx + x] = lo >= 0 ? pack_run(lo, hi) : kEmptyRun;
        }
    return LBM_OK;
}

constexpr int kCx3[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCy3[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCz3[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// Interpolated tube walls: the column table (WallCol) from the fluid runs,
// and, with `wq`, the link fractions of every node that has a wall link.
// Node (x, y, z) pulls direction i from x - c_i; where that node is solid the
// row holds, at i - 1, the fraction q in (0, 1] of the link from the node
// along -c_i at which it leaves the tube (the voxelisation's own expression),
// in FP64 by 60 halvings of the link, keeping the first point found outside.
// Returns the number of rows.
int64_t wall_table(const lbm3d_geom& g, const std::vector<uint32_t>& runs,
                   std::vector<WallCol>* wcol, std::vector<float>* wq)
{
    auto run_at = [&](int x, int y) -> uint32_t {
        if (y < 0 || y >= g.ny)
            return kEmptyRun;
        return runs[(size_t)y * g.nx + (x + g.nx) % g.nx];
    };
    const double yc = 0.5 * (g.ny - 1), zc = 0.5 * (g.nz - 1);
    auto inside = [&](double X, double Y, double Z) {
        const double r = g.r0 + g.a * std::cos(2.0 * M_PI * X / g.lambda);
        const double dy = Y - yc, dz = Z - zc;
        return dy * dy + dz * dz < r * r;
    };
    if (wcol)
        wcol->assign((size_t)g.nx * g.ny, WallCol{0u, 0u});
    if (wq)
        wq->clear();
    int64_t rows = 0;
    for (int y = 0; y < g.ny; ++y)
        for (int x = 0; x < g.nx; ++x) {
            const uint32_t r = runs[(size_t)y * g.nx + x];
            if (r == kEmptyRun)
                continue;
            const int lo = (int)(r & 0xffffu), hi = (int)(r >> 16) - 1;
            int A = lo, B = hi;  // nodes whose every neighbour is fluid
            for (int i = 1; i < 19; ++i) {
                const uint32_t rn = run_at(x - kCx3[i], y - kCy3[i]);
                if (rn == kEmptyRun) {
                    A = hi + 1;
                    break;
                }
                A = std::max(A, (int)(rn & 0xffffu) + kCz3[i]);
                B = std::min(B, (int)(rn >> 16) - 1 + kCz3[i]);
            }
            int a = A, b = B + 1;
            if (A > B)
                a = b = hi + 1;
            if (wcol)
                (*wcol)[(size_t)y * g.nx + x] =
                    WallCol{(uint32_t)rows, (uint32_t)a | ((uint32_t)b << 16)};
            if (wq) {
                for (int z = lo; z <= hi; ++z) {
                    if (z >= a && z < b)
                        continue;
                    for (int i = 1; i < 19; ++i) {
                        const uint32_t rn = run_at(x - kCx3[i], y - kCy3[i]);
                        const int zs = z - kCz3[i];
                        const bool src_fluid = rn != kEmptyRun && zs >= (int)(rn & 0xffffu) &&
                                               zs < (int)(rn >> 16);
                        double q = 1.0;
                        if (!src_fluid) {
                            double tlo = 0.0, thi = 1.0;
                            for (int it = 0; it < 60; ++it) {
                                const double t = 0.5 * (tlo + thi);
                                if (inside(x - t * kCx3[i], y - t * kCy3[i], z - t * kCz3[i]))
                                    tlo = t;
                                else
                                    thi = t;
                            }
                            q = thi;
                        }
                        wq->push_back((float)q);
                    }
                }
            }
            rows += (a - lo) + (hi + 1 - b);
        }
    return rows;
}

// Rows of the link-fraction table (0 without interpolated walls).
int64_t wall_rows_of(const lbm3d_geom& g)
{
    if (!g.wall_interp)
        return 0;
    std::vector<uint32_t> runs;
    if (voxelise(g, runs) != LBM_OK)
        return 0;
    return wall_table(g, runs, nullptr, nullptr);
}

Inst3Dev make_inst(const lbm3d_geom& g, int storage)
{
    Inst3Dev d{};
    d.nx = g.nx;
    d.ny = g.ny;
    d.nz = g.nz;
    d.pitch = pitch_of(g.nx);
    d.rs = planes_of(storage) * d.pitch;
    d.periodic = g.kind == LBM3D_GEOM_BOX ? 1 : 0;
    return d;
}

void fill_fluid(Inst3Dev& d, const lbm3d_fluid& f)
{
    d.tau_h[0] = (float)(f.tau[0] - 0.5);
    d.tau_h[1] = (float)(f.tau[1] - 0.5);
    d.G36 = (float)(f.G / 36.0);
    d.rho_s[0] = (float)f.rho_s[0];
    d.rho_s[1] = (float)f.rho_s[1];
    for (int a = 0; a < 3; ++a)
        d.g[a] = (float)f.g[a];
    d.Gd = f.G;
}

}  // namespace

struct lbm3d_ctx {
    int storage = LBM_STORE_F32;
    lbm3d_geom geom{};
    Inst3Dev P{};
    Layout3 L{};
    std::vector<uint32_t> runs;
    std::vector<Item3> items;
    int tile = 3, strip = kDefaultStrip;
    char* buf[2] = {nullptr, nullptr};
    char* snap = nullptr;
    Item3* items_d = nullptr;
    uint32_t* runs_d = nullptr;
    double* partial_d = nullptr;
    double* mon_d = nullptr;
    double* stage_d = nullptr;
    hipStream_t stream = nullptr;
    int cur = 0;
    int64_t t = 0, snap_t = -1;
};

namespace {

// Cut the lattice into work items: tiles of bx x by nodes over the rows that
// hold fluid, each split into strips of `strip` planes covering the tile's
// fluid planes; strip-major order (all tiles of one band of planes, then the
// next) so tiles that share boundary planes run side by side on one XCD, and
// odd bands march down.
void build_items(lbm3d_ctx* c)
{
    const lbm3d_geom& g = c->geom;
    const int bx = kTileBx[c->tile], by = kTileBy[c->tile];
    const bool per = c->P.periodic != 0;
    int ylo = 0, yhi = g.ny - 1;
    if (!per) {
        ylo = g.ny;
        yhi = -1;
        for (int y = 0; y < g.ny; ++y)
            for (int x = 0; x < g.nx; ++x)
                if (c->runs[(size_t)y * g.nx + x] != kEmptyRun) {
                    ylo = std::min(ylo, y);
                    yhi = std::max(yhi, y);
                }
    }
    c->items.clear();
    if (ylo > yhi)
        return;
    const int ntx = (g.nx + bx - 1) / bx, nty = (yhi - ylo + by) / by;
    std::vector<int> zlo(ntx * nty, g.nz), zhi(ntx * nty, -1);
    int glo = g.nz, ghi = -1;
    for (int ty = 0; ty < nty; ++ty)
        for (int tx = 0; tx < ntx; ++tx) {
            const int k = ty * ntx + tx;
            for (int y = ylo + ty * by; y < std::min(yhi + 1, ylo + (ty + 1) * by); ++y)
                for (int x = tx * bx; x < std::min(g.nx, (tx + 1) * bx); ++x) {
                    const uint32_t r = c->runs[(size_t)y * g.nx + x];
                    if (r == kEmptyRun)
                        continue;
                    zlo[k] = std::min(zlo[k], (int)(r & 0xffffu));
                    zhi[k] = std::max(zhi[k], (int)(r >> 16) - 1);
                }
            glo = std::min(glo, zlo[k]);
            ghi = std::max(ghi, zhi[k]);
        }
    int band = 0;
    for (int z0 = glo; z0 <= ghi; z0 += c->strip, ++band) {
        const int z1 = std::min(ghi + 1, z0 + c->strip);
        for (int ty = 0; ty < nty; ++ty)
            for (int tx = 0; tx < ntx; ++tx) {
                const int k = ty * ntx + tx;
                const int a0 = std::max(z0, zlo[k]), a1 = std::min(z1, zhi[k] + 1);
                if (a0 >= a1)
                    continue;
                const int x0 = tx * bx, y0 = ylo + ty * by;
                if (band & 1)
                    c->items.push_back(Item3{x0, y0, a1 - 1, a0 - 1});
                else
                    c->items.push_back(Item3{x0, y0, a0, a1});
            }
    }
}

lbm_status upload_items(lbm3d_ctx* c)
{
    build_items(c);
    if ((int64_t)c->items.size() > c->L.n_items_max)
        return fail(LBM_ERR_INVALID, "lbm3d: internal error, item table overflow");
    if (!c->items.empty())
        HIP_TRY(hipMemcpyAsync(c->items_d, c->items.data(), sizeof(Item3) * c->items.size(),
                               hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status launch_mode(lbm3d_ctx* c, int mode, void* fout)
{
    HIP_TRY(launch3_step(c->storage, c->tile, mode, c->buf[c->cur], fout, c->P, c->items_d,
                         (int)c->items.size(), c->runs_d, c->partial_d, c->stage_d,
                         (uint32_t)c->t, c->stream));
    return LBM_OK;
}

lbm_status monitors_to_host(lbm3d_ctx* c, lbm_monitor* mon)
{
    lbm_status st = launch_mode(c, kMonOnly, nullptr);
    if (st != LBM_OK)
        return st;
    HIP_TRY(launch3_mon_reduce(c->partial_d, (int)c->items.size(), c->mon_d, c->stream));
    double m[kMon3Width];
    HIP_TRY(hipMemcpyAsync(m, c->mon_d, sizeof m, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->items.empty())
        std::fill(m, m + kMon3Width, 0.0);
    mon->mass[0] = m[0];
    mon->mass[1] = m[1];
    mon->momentum[0] = m[2];
    mon->momentum[1] = m[3];
    mon->oil_flux = m[4];
    mon->oil_cos = m[5];
    mon->oil_sin = m[6];
    mon->bad_nodes = m[7];
    return LBM_OK;
}

lbm_status export_state(lbm3d_ctx* c)
{
    const size_t n = (size_t)c->geom.nx * c->geom.ny * c->geom.nz;
    HIP_TRY(hipMemsetAsync(c->stage_d, 0, sizeof(double) * kExport3Fields * n, c->stream));
    return launch_mode(c, kExport, nullptr);
}

}  // namespace

extern "C" {

lbm_status lbm3d_required_bytes(const lbm3d_geom* geom, int32_t storage, size_t* bytes)
{
    if (!bytes)
        return fail(LBM_ERR_INVALID, "lbm3d_required_bytes: bytes is NULL");
    lbm_status st = check_geom(geom, storage & 0xff);
    if (st != LBM_OK)
        return st;
    if (storage & ~(0xff | LBM_OPT_SNAPSHOT))
        return fail(LBM_ERR_INVALID, "lbm3d_required_bytes: unknown option bits 0x%x", storage);
    *bytes = layout_of(*geom, storage, wall_rows_of(*geom)).total;
    return LBM_OK;
}

lbm_status lbm3d_init(const lbm3d_geom* geom, const lbm3d_fluid* fluid,
                      const lbm3d_init_fields* init, int32_t storage, void* device_workspace,
                      size_t workspace_bytes, void* hip_stream, lbm3d_ctx** out)
{
    if (!out)
        return fail(LBM_ERR_INVALID, "lbm3d_init: out is NULL");
    *out = nullptr;
    const int fmt = storage & 0xff;
    lbm_status st = check_geom(geom, fmt);
    if (st != LBM_OK)
        return st;
    if (storage & ~(0xff | LBM_OPT_SNAPSHOT))
        return fail(LBM_ERR_INVALID, "lbm3d_init: unknown option bits 0x%x", storage);
    st = check_fluid(fluid);
    if (st != LBM_OK)
        return st;
    if (!init)
        return fail(LBM_ERR_INVALID, "lbm3d_init: init is NULL");
    if (init->kind != LBM3D_INIT_UNIFORM && init->kind != LBM3D_INIT_DROPLET &&
        init->kind != LBM3D_INIT_SLUG)
        return fail(LBM_ERR_INVALID, "lbm3d_init: unknown init kind %d", init->kind);
    double slug_x0[LBM_MAX_SLUGS], slug_len[LBM_MAX_SLUGS];
    int32_t n_slugs = 1;
    if (init->kind == LBM3D_INIT_SLUG) {
        std::string err;
        if (!lbm::slug_list(init->n_slugs, init->slugs, init->x0, init->length, slug_x0,
                            slug_len, n_slugs, err))
            return fail(LBM_ERR_INVALID, "lbm3d_init: %s", err.c_str());
        if (!std::isfinite(init->width) || init->width < 0.0)
            return fail(LBM_ERR_INVALID,
                        "lbm3d_init: slug interface width must be finite and >= 0");
    }
    if (!(init->rho_hi > 0.0) || !(init->rho_lo > 0.0) ||
        !std::isfinite(init->rho_hi + init->rho_lo))
        return fail(LBM_ERR_INVALID, "lbm3d_init: densities must be finite and > 0");
    std::vector<uint32_t> runs;
    st = voxelise(*geom, runs);
    if (st != LBM_OK)
        return st;
    std::vector<WallCol> wcol;
    std::vector<float> wq;
    const int64_t wall_rows = geom->wall_interp ? wall_table(*geom, runs, &wcol, &wq) : 0;
    const Layout3 L = layout_of(*geom, storage, wall_rows);
    if (!device_workspace)
        return fail(LBM_ERR_INVALID, "lbm3d_init: workspace is NULL");
    if (workspace_bytes < L.total)
        return fail(LBM_ERR_OOM, "lbm3d_init: workspace of %zu bytes, %zu needed",
                    workspace_bytes, L.total);
    if ((uintptr_t)device_workspace % kAlign)
        return fail(LBM_ERR_INVALID, "lbm3d_init: workspace must be %zu-byte aligned", kAlign);

    lbm3d_ctx* c = new (std::nothrow) lbm3d_ctx();
    if (!c)
        return fail(LBM_ERR_INVALID, "lbm3d_init: out of host memory");
    c->storage = fmt;
    c->geom = *geom;
    c->geom.mask = nullptr;
    c->L = L;
    c->stream = (hipStream_t)hip_stream;
    c->runs = std::move(runs);
    // Default tile, measured on the 512 x 128 x 128 tube in every storage
    // format, with and without interpolated walls: 16 x 12 (four-wave
    // workgroups, three per CU, two with interpolated walls, which hold more
    // live values per node and spill in the 612-thread tiles).
    c->tile = 3;
    c->P = make_inst(*geom, fmt);
    fill_fluid(c->P, *fluid);
    char* ws = (char*)device_workspace;
    c->buf[0] = ws + L.off_buf[0];
    c->buf[1] = ws + L.off_buf[1];
    c->snap = (storage & LBM_OPT_SNAPSHOT) ? ws + L.off_snap : nullptr;
    c->items_d = (Item3*)(ws + L.off_items);
    c->runs_d = (uint32_t*)(ws + L.off_runs);
    c->partial_d = (double*)(ws + L.off_partial);
    c->mon_d = (double*)(ws + L.off_mon);
    c->stage_d = (double*)(ws + L.off_stage);

    auto bail = [&](lbm_status s) {
        delete c;
        return s;
    };
    auto hip_bail = [&](hipError_t e, const char* what) {
        delete c;
        return fail(LBM_ERR_DEVICE, "lbm3d_init: %s failed: %s", what, hipGetErrorString(e));
    };
    hipError_t e = hipMemsetAsync(ws, 0, 2 * L.buf_bytes, c->stream);
    if (e != hipSuccess)
        return hip_bail(e, "hipMemsetAsync");
    e = hipMemcpyAsync(c->runs_d, c->runs.data(), sizeof(uint32_t) * c->runs.size(),
                       hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess)
        return hip_bail(e, "hipMemcpyAsync");
    if (geom->wall_interp) {
        WallCol* wcol_d = (WallCol*)(ws + L.off_wcol);
        float* wq_d = (float*)(ws + L.off_wq);
        e = hipMemcpyAsync(wcol_d, wcol.data(), sizeof(WallCol) * wcol.size(),
                           hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess && !wq.empty())
            e = hipMemcpyAsync(wq_d, wq.data(), sizeof(float) * wq.size(),
                               hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess)
            return hip_bail(e, "hipMemcpyAsync");
        c->P.wcol = wcol_d;
        c->P.wq = wq_d;
    }
    Init3Dev ini{};
    ini.kind = init->kind;
    ini.rho_hi = init->rho_hi;
    ini.rho_lo = init->rho_lo;
    ini.cx = init->cx;
    ini.cy = init->cy;
    ini.cz = init->cz;
    ini.r = init->r;
    ini.n_slugs = n_slugs;
    for (int k = 0; k < n_slugs; ++k) {
        ini.x0[k] = init->kind == LBM3D_INIT_SLUG ? slug_x0[k] : init->x0;
        ini.length[k] = init->kind == LBM3D_INIT_SLUG ? slug_len[k] : init->length;
    }
    ini.width = init->kind == LBM3D_INIT_SLUG ? init->width : 0.0;
    e = launch3_init(fmt, c->buf[0], c->P, c->runs_d, ini, c->stream);
    if (e != hipSuccess)
        return hip_bail(e, "init kernel launch");
    st = upload_items(c);  // synchronises
    if (st != LBM_OK)
        return bail(st);
    *out = c;
    return LBM_OK;
}

lbm_status lbm3d_step(lbm3d_ctx* c, int64_t nsteps)
{
    if (!c || nsteps < 0)
        return fail(LBM_ERR_INVALID, "lbm3d_step: bad argument");
    for (int64_t k = 0; k < nsteps; ++k) {
        lbm_status st = launch_mode(c, kStep, c->buf[1 - c->cur]);
        if (st != LBM_OK)
            return st;
        c->cur = 1 - c->cur;
        ++c->t;
    }
    return LBM_OK;
}

int64_t lbm3d_time(const lbm3d_ctx* c) { return c ? c->t : -1; }

lbm_status lbm3d_set_fluid(lbm3d_ctx* c, const lbm3d_fluid* fluid)
{
    if (!c)
        return fail(LBM_ERR_INVALID, "lbm3d_set_fluid: context is NULL");
    lbm_status st = check_fluid(fluid);
    if (st != LBM_OK)
        return st;
    fill_fluid(c->P, *fluid);
    return LBM_OK;
}

lbm_status lbm3d_monitors(lbm3d_ctx* c, lbm_monitor* mon)
{
    if (!c || !mon)
        return fail(LBM_ERR_INVALID, "lbm3d_monitors: bad argument");
    return monitors_to_host(c, mon);
}

lbm_status lbm3d_moments(lbm3d_ctx* c, double* rho, double* u, double* p, lbm_monitor* mon)
{
    if (!c)
        return fail(LBM_ERR_INVALID, "lbm3d_moments: context is NULL");
    const size_t n = (size_t)c->geom.nx * c->geom.ny * c->geom.nz;
    if (rho || u || p) {
        lbm_status st = export_state(c);
        if (st != LBM_OK)
            return st;
        if (rho)
            HIP_TRY(hipMemcpyAsync(rho, c->stage_d + 38 * n, sizeof(double) * 2 * n,
                                   hipMemcpyDeviceToHost, c->stream));
        if (u)
            HIP_TRY(hipMemcpyAsync(u, c->stage_d + 40 * n, sizeof(double) * 3 * n,
                                   hipMemcpyDeviceToHost, c->stream));
        if (p)
            HIP_TRY(hipMemcpyAsync(p, c->stage_d + 43 * n, sizeof(double) * n,
                                   hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    if (mon)
        return monitors_to_host(c, mon);
    return LBM_OK;
}

lbm_status lbm3d_get_populations(lbm3d_ctx* c, double* f)
{
    if (!c || !f)
        return fail(LBM_ERR_INVALID, "lbm3d_get_populations: bad argument");
    const size_t n = (size_t)c->geom.nx * c->geom.ny * c->geom.nz;
    lbm_status st = export_state(c);
    if (st != LBM_OK)
        return st;
    HIP_TRY(hipMemcpyAsync(f, c->stage_d, sizeof(double) * 38 * n, hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm3d_fluid_mask(lbm3d_ctx* c, uint8_t* mask)
{
    if (!c || !mask)
        return fail(LBM_ERR_INVALID, "lbm3d_fluid_mask: bad argument");
    const lbm3d_geom& g = c->geom;
    for (int z = 0; z < g.nz; ++z)
        for (int y = 0; y < g.ny; ++y)
            for (int x = 0; x < g.nx; ++x) {
                const uint32_t r = c->runs[(size_t)y * g.nx + x];
                const int lo = (int)(r & 0xffffu), hi1 = (int)(r >> 16);
                mask[((size_t)z * g.ny + y) * g.nx + x] = (z >= lo && z < hi1) ? 1 : 0;
            }
    return LBM_OK;
}

lbm_status lbm3d_set_tiling(lbm3d_ctx* c, int32_t bx, int32_t by, int32_t strip_planes)
{
    if (!c)
        return fail(LBM_ERR_INVALID, "lbm3d_set_tiling: context is NULL");
    int tile = -1;
    for (int k = 0; k < kTiles3; ++k)
        if (kTileBx[k] == bx && kTileBy[k] == by)
            tile = k;
    if (tile < 0)
        return fail(LBM_ERR_INVALID, "lbm3d_set_tiling: tile %d x %d not supported", bx, by);
    if (strip_planes < kMinStrip || strip_planes > 32767)
        return fail(LBM_ERR_INVALID, "lbm3d_set_tiling: strip_planes must be >= %d", kMinStrip);
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->tile = tile;
    c->strip = strip_planes;
    return upload_items(c);
}

lbm_status lbm3d_get_tiling(const lbm3d_ctx* c, int32_t* bx, int32_t* by, int32_t* strip_planes,
                            int32_t* n_items)
{
    if (!c)
        return fail(LBM_ERR_INVALID, "lbm3d_get_tiling: context is NULL");
    if (bx)
        *bx = kTileBx[c->tile];
    if (by)
        *by = kTileBy[c->tile];
    if (strip_planes)
        *strip_planes = c->strip;
    if (n_items)
        *n_items = (int32_t)c->items.size();
    return LBM_OK;
}

lbm_status lbm3d_snapshot_save(lbm3d_ctx* c)
{
    if (!c || !c->snap)
        return fail(LBM_ERR_INVALID, "lbm3d_snapshot_save: no snapshot buffer "
                                     "(LBM_OPT_SNAPSHOT at init)");
    HIP_TRY(hipMemcpyAsync(c->snap, c->buf[c->cur], c->L.buf_bytes, hipMemcpyDeviceToDevice,
                           c->stream));
    c->snap_t = c->t;
    return LBM_OK;
}

lbm_status lbm3d_snapshot_restore(lbm3d_ctx* c)
{
    if (!c || !c->snap || c->snap_t < 0)
        return fail(LBM_ERR_INVALID, "lbm3d_snapshot_restore: no snapshot saved");
    HIP_TRY(hipMemcpyAsync(c->buf[c->cur], c->snap, c->L.buf_bytes, hipMemcpyDeviceToDevice,
                           c->stream));
    c->t = c->snap_t;
    return LBM_OK;
}

void lbm3d_destroy(lbm3d_ctx* c)
{
    // Queued steps (graph replays included) still use the caller's workspace:
    // drain them before the caller can free it.
    if (c)
        (void)hipStreamSynchronize(c->stream);
    delete c;
}

}  // extern "C"
