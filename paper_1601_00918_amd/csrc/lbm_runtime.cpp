// Host runtime behind the C ABI of include/lbm.h: parameter validation,
// voxelisation into column runs, work-item tiling, workspace carving, launch
// sequencing and device-to-host export.
#include "lbm_ctx.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <vector>

using namespace lbm;

namespace {

thread_local std::string g_last_error;

}  // namespace

lbm_status lbm::fail(lbm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

namespace {

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(LBM_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kMinBx = 64;
constexpr int kMinStrip = 4;
constexpr int kGraphSteps = 64;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Column entry from a column's fluid predicate over rows 0..ny-1: one run, or
// two runs with the solid gap between them; false if there are more.
template <typename F>
bool column_runs(int ny, F fluid, Col& out)
{
    int starts[2], ends[2], n = 0;
    for (int y = 0; y < ny; ++y) {
        if (!fluid(y))
            continue;
        if (n > 0 && ends[n - 1] == y - 1) {
            ends[n - 1] = y;
            continue;
        }
        if (n == 2)
            return false;
        starts[n] = ends[n] = y;
        ++n;
    }
    if (n == 0)
        out = Col{0, -1, 1, 0};
    else if (n == 1)
        out = Col{starts[0], ends[0], 1, 0};
    else
        out = Col{starts[0], ends[1], ends[0] + 1, starts[1] - 1};
    return true;
}

// Whether column x of a channel lies under its island (the wide part of
// every period, where the distance to the nearest multiple of lambda is
// below island_len / 2).
bool island_column(const lbm_geom& g, int x)
{
    if (!(g.island_h > 0.0) || !(g.island_len > 0.0))
        return false;
    const double r = std::fmod((double)x, g.lambda);
    return std::min(r, g.lambda - r) < 0.5 * g.island_len;
}

// Fluid runs per column for a geometry; returns false with a message on error.
bool voxelise(const lbm_geom& g, std::vector<Col>& cols, std::string& err)
{
    cols.assign(g.nx, Col{0, -1, 1, 0});
    if (g.kind == LBM_GEOM_BOX) {
        for (auto& c : cols)
            c = Col{0, g.ny - 1, 1, 0};
        return true;
    }
    if (g.kind == LBM_GEOM_CHANNEL) {
        const double yc = 0.5 * (g.ny - 1) + g.y_offset;
        for (int x = 0; x < g.nx; ++x) {
            const double h = g.h0 + g.a * std::cos(2.0 * M_PI * (double)x / g.lambda);
            const bool isl = island_column(g, x);
            auto fluid = [&](int y) {
                const double dy = std::fabs((double)y - yc);
                return dy < h && !(isl && dy < g.island_h);
            };
            if (!column_runs(g.ny, fluid, cols[x])) {
                err = "channel column " + std::to_string(x) + " has more than two fluid runs";
                return false;
            }
        }
        return true;
    }
    if (g.kind == LBM_GEOM_MASK) {
        if (!g.mask) {
            err = "LBM_GEOM_MASK needs a mask";
            return false;
        }
        for (int x = 0; x < g.nx; ++x) {
            auto fluid = [&](int y) { return g.mask[(size_t)y * g.nx + x] != 0; };
            if (!column_runs(g.ny, fluid, cols[x])) {
                err = "mask column " + std::to_string(x) + " has more than two runs of fluid rows";
                return false;
            }
        }
        return true;
    }
    err = "unknown geometry kind";
    return false;
}

// Wall table of a channel with interpolated walls ([nx][kWallSlots][8]
// floats, 1 where a slot has no wall link): for every fluid node (x, y) and
// pulled direction j whose source node x - c_j is solid, the fraction q in
// (0, 1] of the link from (x, y) along -c_j at which it leaves the fluid region
// |y - y_c| < h(x), in FP64: in closed form for flat walls, otherwise by 60
// halvings of the link, keeping the first point found outside.  Fails if a
// node outside the wall slots has a wall link (walls steeper than one row per
// column).
bool wall_table(const lbm_geom& g, const std::vector<Col>& cols, std::vector<float>& wq,
                std::string& err)
{
    static const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const double yc = 0.5 * (g.ny - 1) + g.y_offset;
    auto inside = [&](double X, double Y) {  // the expression voxelise classifies by
        return std::fabs(Y - yc) < g.h0 + g.a * std::cos(2.0 * M_PI * X / g.lambda);
    };
    wq.assign((size_t)g.nx * kWallSlots * 8, 1.0f);
    for (int x = 0; x < g.nx; ++x) {
        const Col c = cols[x];
        for (int y = c.lo; y <= c.hi; ++y)
            for (int j = 1; j < 9; ++j) {
                const Col& cs = cols[(x - cx[j] + g.nx) % g.nx];
                const int ys = y - cy[j];
                if (col_fluid(cs, ys))
                    continue;
                const int slot = wall_slot(y, c.lo, c.hi);
                if (slot < 0) {
                    err = "interpolated walls: node (" + std::to_string(x) + ", " +
                          std::to_string(y) +
                          ") two rows inside the wall has a wall link (walls steeper "
                          "than one row per column)";
                    return false;
                }
                double q;
                if (g.a == 0.0) {
                    q = (g.h0 - std::fabs((double)y - yc)) / std::fabs((double)cy[j]);
                } else {
                    double lo = 0.0, hi = 1.0;
                    for (int it = 0; it < 60; ++it) {
                        const double t = 0.5 * (lo + hi);
                        if (inside((double)x - t * cx[j], (double)y - t * cy[j]))
                            lo = t;
                        else
                            hi = t;
                    }
                    q = hi;
                }
                wq[((size_t)x * kWallSlots + slot) * 8 + (j - 1)] = (float)q;
            }
    }
    return true;
}

lbm_status check_geom(const lbm_geom& g)
{
    if (g.wall_interp != 0 && g.wall_interp != 1)
        return fail(LBM_ERR_INVALID, "wall_interp must be 0 or 1");
    if (g.wall_interp && g.kind != LBM_GEOM_CHANNEL)
        return fail(LBM_ERR_UNSUPPORTED, "interpolated walls need the analytic channel geometry");
    if (!std::isfinite(g.island_h) || !std::isfinite(g.island_len) || g.island_h < 0.0 ||
        g.island_len < 0.0)
        return fail(LBM_ERR_INVALID, "island_h and island_len must be finite and >= 0");
    if (g.wall_interp && g.island_h > 0.0 && g.island_len > 0.0)
        return fail(LBM_ERR_UNSUPPORTED, "interpolated walls do not support an island");
    if (g.nx < 1 || g.ny < 1 || g.nx > 32768 || g.ny > 32768)
        return fail(LBM_ERR_INVALID, "geometry size %d x %d out of range", g.nx, g.ny);
    // The kernels address an instance with 32-bit byte offsets.
    if ((int64_t)72 * (int64_t)((g.nx + 63) / 64 * 64) * g.ny >= ((int64_t)1 << 32))
        return fail(LBM_ERR_UNSUPPORTED,
                    "instance %d x %d too large (its populations exceed 4 GiB)", g.nx, g.ny);
    if (g.kind == LBM_GEOM_BOX) {
        if (g.ny < 3 || g.nx < 3)
            return fail(LBM_ERR_INVALID, "box geometry needs nx, ny >= 3");
        return LBM_OK;
    }
    if (g.kind == LBM_GEOM_CHANNEL) {
        if (!(g.lambda > 0.0) || !(g.h0 > 0.0) || !(g.a >= 0.0) || !std::isfinite(g.h0 + g.a))
            return fail(LBM_ERR_INVALID, "channel needs lambda > 0, h0 > 0, a >= 0");
        if (!(std::fabs(g.y_offset) <= 1.0))
            return fail(LBM_ERR_INVALID, "channel y_offset must lie in [-1, 1]");
        if (g.nx < 3)
            return fail(LBM_ERR_INVALID, "channel needs nx >= 3");
        return LBM_OK;
    }
    if (g.kind == LBM_GEOM_MASK) {
        if (!g.mask)
            return fail(LBM_ERR_INVALID, "mask geometry without a mask");
        if (g.nx < 3)
            return fail(LBM_ERR_INVALID, "mask geometry needs nx >= 3");
        return LBM_OK;
    }
    return fail(LBM_ERR_INVALID, "unknown geometry kind %d", g.kind);
}

lbm_status check_fluid(const lbm_fluid& f)
{
    for (int s = 0; s < 2; ++s) {
        if (!(f.tau[s] > 0.5) || !std::isfinite(f.tau[s]))
            return fail(LBM_ERR_INVALID, "tau[%d] = %g must be finite and > 1/2", s, f.tau[s]);
        if (!std::isfinite(f.rho_s[s]) || f.rho_s[s] < 0.0)
            return fail(LBM_ERR_INVALID, "rho_s[%d] must be finite and >= 0", s);
        if (!std::isfinite(f.g[s]) || std::fabs(f.g[s]) > 0.1)
            return fail(LBM_ERR_INVALID, "|g[%d]| must be <= 0.1", s);
    }
    if (!std::isfinite(f.G))
        return fail(LBM_ERR_INVALID, "G must be finite");
    if (f.reg_order != 0 && f.reg_order != 2 && f.reg_order != 3)
        return fail(LBM_ERR_INVALID, "reg_order = %d must be 2 or 3 (0: 2)", f.reg_order);
    return LBM_OK;
}

int pitch_of(int nx) { return (int)align_up((size_t)nx, 64); }

size_t elem_size(int storage) { return storage == LBM_STORE_F32 ? 4 : 2; }

// Elements per lattice row and pitch: 18 population rows, plus (16-bit
// formats) the row of reference-density pairs.
int row_planes(int storage) { return storage == LBM_STORE_F32 ? 18 : 20; }

// Elements of one instance in one population buffer.
int64_t inst_elems(int nx, int ny, int storage)
{
    return (int64_t)row_planes(storage) * pitch_of(nx) * ny;
}

// Upper bound on the number of work items for any supported tiling.
int64_t max_items(const lbm_geom& g)
{
    return (int64_t)((g.nx + kMinBx - 1) / kMinBx) * ((g.ny + kMinStrip - 1) / kMinStrip);
}

Layout layout_of(const lbm_geom* geoms, int n_inst, int storage_and_opts)
{
    const int storage = storage_and_opts & 0xff;
    const bool with_snap = (storage_and_opts & LBM_OPT_SNAPSHOT) != 0;
    Layout L{};
    int64_t elems = 0, ncols = 0, nwq = 0;
    L.n_items_max = 0;
    L.max_nodes = 0;
    for (int k = 0; k < n_inst; ++k) {
        const lbm_geom& g = geoms[k];
        elems += inst_elems(g.nx, g.ny, storage);
        ncols += g.nx;
        if (g.wall_interp)
            nwq += (int64_t)g.nx * kWallSlots * 8;
        L.n_items_max += max_items(g);
        L.max_nodes = std::max<int64_t>(L.max_nodes, (int64_t)g.nx * g.ny);
    }
    L.buf_bytes = align_up((size_t)elems * elem_size(storage), kAlign);
    size_t o = 0;
    L.off_buf[0] = o;
    o += L.buf_bytes;
    L.off_buf[1] = o;
    o += L.buf_bytes;
    L.off_snap = o;
    if (with_snap)
        o += L.buf_bytes;
    L.off_inst = o;
    o = align_up(o + sizeof(InstDev) * n_inst, kAlign);
    L.off_items = o;  // full item list, then the active-instance list
    o = align_up(o + 2 * sizeof(Item) * L.n_items_max, kAlign);
    L.off_cols = o;
    o = align_up(o + sizeof(Col) * ncols, kAlign);
    L.off_partial = o;
    o = align_up(o + 2 * sizeof(double) * kMonWidth * L.n_items_max, kAlign);
    L.off_mon = o;
    o = align_up(o + sizeof(double) * kMonWidth * n_inst, kAlign);
    L.off_first = o;
    o = align_up(o + sizeof(int32_t) * n_inst, kAlign);
    L.off_count = o;
    o = align_up(o + sizeof(int32_t) * n_inst, kAlign);
    L.off_stage = o;
    o = align_up(o + sizeof(double) * kExportFields * L.max_nodes, kAlign);
    L.off_seed = o;
    o = align_up(o + sizeof(uint32_t), kAlign);
    L.off_wq = o;
    o = align_up(o + sizeof(float) * nwq, kAlign);
    L.total = o;
    return L;
}

}  // namespace

lbm_ctx::~lbm_ctx()
{
    if (graph)
        (void)hipGraphExecDestroy(graph);
}

namespace {

void fill_inst_params(InstDev& d, const lbm_fluid& f)
{
    d.tau_h[0] = (float)(f.tau[0] - 0.5);
    d.tau_h[1] = (float)(f.tau[1] - 0.5);
    d.G36 = (float)(f.G / 36.0);
    d.rho_s[0] = (float)f.rho_s[0];
    d.rho_s[1] = (float)f.rho_s[1];
    d.g[0] = (float)f.g[0];
    d.g[1] = (float)f.g[1];
    d.reg3 = f.reg_order == 3 ? 1 : 0;
    d.Gd = f.G;
}

// Whether any instance uses an optional feature (third-order regularization,
// interpolated walls, two-run columns): then the step launches the extended
// kernels.
bool any_ext(const lbm_ctx* c)
{
    for (const InstDev& d : c->idv)
        if (d.reg3 || d.wq || d.gaps)
            return true;
    return false;
}

constexpr int kBxClasses[3] = {256, 128, 64};

// Cut every instance into work items: blocks of bx columns, each split into
// strips of `strip` rows covering the block's fluid rows.  An instance's items
// are ordered strip-major (all column blocks of one band of rows, then the
// next band), so the blocks that share boundary cache lines run side by side
// on one XCD.  Instances are grouped by their workgroup width.
void build_items(lbm_ctx* c)
{
    c->items.clear();
    c->item_first.assign(c->n_inst, 0);
    c->item_count.assign(c->n_inst, 0);
    for (int cl = 0; cl < 3; ++cl) {
        c->cls_first[cl] = (int)c->items.size();
        for (int k = 0; k < c->n_inst; ++k) {
            const int bx = c->ibx[k], strip = c->istrip[k];
            if (bx != kBxClasses[cl])
                continue;
            const InstHost& h = c->ih[k];
            c->item_first[k] = (int32_t)c->items.size();
            const int nblk = (h.nx + bx - 1) / bx;
            std::vector<int> ylo(nblk, h.ny), yhi(nblk, -1);
            int glo = h.ny, ghi = -1;
            for (int b = 0; b < nblk; ++b) {
                for (int x = b * bx; x < std::min(h.nx, (b + 1) * bx); ++x)
                    if (h.cols[x].lo <= h.cols[x].hi) {
                        ylo[b] = std::min(ylo[b], h.cols[x].lo);
                        yhi[b] = std::max(yhi[b], h.cols[x].hi);
                    }
                glo = std::min(glo, ylo[b]);
                ghi = std::max(ghi, yhi[b]);
            }
            int band = 0;
            for (int y0 = glo; y0 <= ghi; y0 += strip, ++band) {
                const int y1 = std::min(ghi + 1, y0 + strip);
                for (int b = 0; b < nblk; ++b) {
                    const int a0 = std::max(y0, ylo[b]), a1 = std::min(y1, yhi[b] + 1);
                    if (a0 >= a1)
                        continue;
                    // odd bands march down: rows a1 - 1 .. a0
                    if (band & 1)
                        c->items.push_back(Item{k, b * bx, a1 - 1, a0 - 1});
                    else
                        c->items.push_back(Item{k, b * bx, a0, a1});
                }
            }
            c->item_count[k] = (int32_t)c->items.size() - c->item_first[k];
        }
        c->cls_count[cl] = (int)c->items.size() - c->cls_first[cl];
    }
}

// Items of the active instances, grouped like the full list.
std::vector<Item> active_items(lbm_ctx* c)
{
    std::vector<Item> v;
    v.reserve(c->items.size());
    for (int cl = 0; cl < 3; ++cl) {
        c->act_first[cl] = (int)v.size();
        for (int k = 0; k < c->n_inst; ++k)
            if (c->active[k] && c->ibx[k] == kBxClasses[cl])
                v.insert(v.end(), c->items.begin() + c->item_first[k],
                         c->items.begin() + c->item_first[k] + c->item_count[k]);
        c->act_count[cl] = (int)v.size() - c->act_first[cl];
    }
    return v;
}

lbm_status upload_tables(lbm_ctx* c)
{
    HIP_TRY(hipMemcpyAsync(c->items_d, c->items.data(), sizeof(Item) * c->items.size(),
                           hipMemcpyHostToDevice, c->stream));
    c->act_items = active_items(c);  // kept: the source of an asynchronous copy
    const std::vector<Item>& act = c->act_items;
    c->n_active_items = (int)act.size();
    if (!act.empty())
        HIP_TRY(hipMemcpyAsync(c->items_d + c->L.n_items_max, act.data(), sizeof(Item) * act.size(),
                               hipMemcpyHostToDevice, c->stream));
    c->graph_dirty = true;
    HIP_TRY(hipMemcpyAsync(c->first_d, c->item_first.data(), sizeof(int32_t) * c->n_inst,
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->count_d, c->item_count.data(), sizeof(int32_t) * c->n_inst,
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// Bring instance k's state into buffer `cur` (it lags behind when it was
// inactive while the buffers swapped an odd number of times).
lbm_status sync_instance(lbm_ctx* c, int k)
{
    if (c->ipar[k] == c->cur)
        return LBM_OK;
    const InstHost& h = c->ih[k];
    HIP_TRY(hipMemcpyAsync(c->buf[c->cur] + c->es * h.f_off, c->buf[c->ipar[k]] + c->es * h.f_off,
                           c->es * h.elems, hipMemcpyDeviceToDevice, c->stream));
    c->ipar[k] = c->cur;
    return LBM_OK;
}

lbm_status sync_all(lbm_ctx* c)
{
    for (int k = 0; k < c->n_inst; ++k) {
        lbm_status st = sync_instance(c, k);
        if (st != LBM_OK)
            return st;
    }
    return LBM_OK;
}

lbm_status run_range(lbm_ctx* c, int bx, int mode, int item_base, int n_items,
                     uint32_t seed = 0, const uint32_t* seed_dev = nullptr)
{
    hipError_t e = launch_step(c->storage, bx, mode, any_ext(c), c->buf[c->cur],
                               c->buf[c->cur ^ 1], c->inst_d, c->items_d, item_base, n_items,
                               c->cols_d,
                               c->partial_d, c->stage_d, seed, seed_dev, c->stream);
    if (e != hipSuccess)
        return fail(LBM_ERR_DEVICE, "step launch failed: %s", hipGetErrorString(e));
    return LBM_OK;
}

// One pass of `mode` over the active items (kStep, kStepMon) or over every
// item (kMonOnly): one launch per workgroup width.
lbm_status run_mode(lbm_ctx* c, int mode, uint32_t seed = 0, const uint32_t* seed_dev = nullptr)
{
    const bool act = mode == kStep || mode == kStepMon;
    const int base = act ? (int)c->L.n_items_max : 0;
    for (int cl = 0; cl < 3; ++cl) {
        const int first = act ? c->act_first[cl] : c->cls_first[cl];
        const int n = act ? c->act_count[cl] : c->cls_count[cl];
        if (n == 0)
            continue;
        lbm_status st = run_range(c, kBxClasses[cl], mode, base + first, n, seed, seed_dev);
        if (st != LBM_OK)
            return st;
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_last_error.c_str(); }

const char* lbm_version(void) { return "mi355x-mclbm 0.1 (gfx950, D2Q9)"; }

lbm_status lbm_required_bytes(const lbm_geom* geoms, int32_t n_inst, int32_t storage,
                              size_t* bytes)
{
    if (!geoms || n_inst < 1 || !bytes)
        return fail(LBM_ERR_INVALID, "lbm_required_bytes: null argument or n_inst < 1");
    if ((storage & 0xff) > LBM_STORE_BF16 || (storage & ~(0xff | LBM_OPT_SNAPSHOT)))
        return fail(LBM_ERR_UNSUPPORTED, "storage %d not supported", storage);
    for (int k = 0; k < n_inst; ++k) {
        lbm_status st = check_geom(geoms[k]);
        if (st != LBM_OK)
            return st;
    }
    *bytes = layout_of(geoms, n_inst, storage).total;
    return LBM_OK;
}

lbm_status lbm_init(const lbm_geom* geoms, const lbm_fluid* fluids,
                    const lbm_init_fields* inits, int32_t n_inst, int32_t storage,
                    void* device_workspace, size_t workspace_bytes, void* hip_stream,
                    lbm_ctx** out)
{
    if (!out)
        return fail(LBM_ERR_INVALID, "lbm_init: out is null");
    *out = nullptr;
    if (!geoms || !fluids || !inits || n_inst < 1 || !device_workspace)
        return fail(LBM_ERR_INVALID, "lbm_init: null argument or n_inst < 1");
    if ((storage & 0xff) > LBM_STORE_BF16 || (storage & ~(0xff | LBM_OPT_SNAPSHOT)))
        return fail(LBM_ERR_UNSUPPORTED, "storage %d not supported", storage);
    if ((uintptr_t)device_workspace % kAlign)
        return fail(LBM_ERR_INVALID, "workspace must be %zu-byte aligned", kAlign);
    for (int k = 0; k < n_inst; ++k) {
        lbm_status st = check_geom(geoms[k]);
        if (st != LBM_OK)
            return st;
        st = check_fluid(fluids[k]);
        if (st != LBM_OK)
            return st;
        const lbm_init_fields& in = inits[k];
        if (in.kind < LBM_INIT_UNIFORM || in.kind > LBM_INIT_SLUG)
            return fail(LBM_ERR_INVALID, "instance %d: unknown init kind %d", k, in.kind);
        if (!(in.rho_hi > 0.0) || !(in.rho_lo > 0.0) || !std::isfinite(in.rho_hi + in.rho_lo))
            return fail(LBM_ERR_INVALID, "instance %d: rho_hi, rho_lo must be > 0", k);
        if (in.kind == LBM_INIT_LAYERS && (in.core_species < 0 || in.core_species > 1))
            return fail(LBM_ERR_INVALID, "instance %d: core_species must be 0 or 1", k);
        if (in.kind == LBM_INIT_SLUG) {
            double xs[LBM_MAX_SLUGS], ls[LBM_MAX_SLUGS];
            int32_t cnt = 0;
            std::string err;
            if (!slug_list(in.n_slugs, in.slugs, in.x0, in.length, xs, ls, cnt, err))
                return fail(LBM_ERR_INVALID, "instance %d: %s", k, err.c_str());
            if (!std::isfinite(in.width) || in.width < 0.0)
                return fail(LBM_ERR_INVALID, "instance %d: slug interface width must be "
                            "finite and >= 0", k);
        }
    }
    const Layout L = layout_of(geoms, n_inst, storage);
    if (workspace_bytes < L.total)
        return fail(LBM_ERR_OOM, "workspace %zu bytes < required %zu", workspace_bytes, L.total);

    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c)
        return fail(LBM_ERR_INVALID, "out of host memory");
    c->n_inst = n_inst;
    c->storage = storage & 0xff;
    if (storage & LBM_OPT_SNAPSHOT)
        c->snap = (char*)device_workspace + L.off_snap;
    c->active.assign(n_inst, 1);
    c->ipar.assign(n_inst, 0);
    c->L = L;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char*)device_workspace;
    c->buf[0] = c->ws + L.off_buf[0];
    c->buf[1] = c->ws + L.off_buf[1];
    c->es = elem_size(storage & 0xff);
    c->inst_d = (InstDev*)(c->ws + L.off_inst);
    c->items_d = (Item*)(c->ws + L.off_items);
    c->cols_d = (Col*)(c->ws + L.off_cols);
    c->partial_d = (double*)(c->ws + L.off_partial);
    c->mon_d = (double*)(c->ws + L.off_mon);
    c->first_d = (int32_t*)(c->ws + L.off_first);
    c->count_d = (int32_t*)(c->ws + L.off_count);
    c->stage_d = (double*)(c->ws + L.off_stage);
    c->seed_d = (uint32_t*)(c->ws + L.off_seed);

    // Instances, column tables.
    c->ih.resize(n_inst);
    c->idv.resize(n_inst);
    std::vector<Col> all_cols;
    std::vector<float> all_wq;
    int64_t f_off = 0;
    int max_nx = 0;
    for (int k = 0; k < n_inst; ++k) {
        const lbm_geom& g = geoms[k];
        InstHost& h = c->ih[k];
        std::string err;
        if (!voxelise(g, h.cols, err)) {
            delete c;
            return fail(LBM_ERR_UNSUPPORTED, "instance %d: %s", k, err.c_str());
        }
        h.kind = g.kind;
        h.nx = g.nx;
        h.ny = g.ny;
        h.pitch = pitch_of(g.nx);
        h.elems = inst_elems(g.nx, g.ny, storage & 0xff);
        h.f_off = f_off;
        f_off += h.elems;
        max_nx = std::max(max_nx, g.nx);
        InstDev& d = c->idv[k];
        std::memset(&d, 0, sizeof d);
        d.f_off = h.f_off;
        d.rstride = row_planes(storage & 0xff) * h.pitch;
        d.nx = g.nx;
        d.ny = g.ny;
        d.pitch = h.pitch;
        d.periodic_y = g.kind == LBM_GEOM_BOX ? 1 : 0;
        d.wq = nullptr;
        if (g.wall_interp) {
            std::vector<float> wq;
            if (!wall_table(g, h.cols, wq, err)) {
                delete c;
                return fail(LBM_ERR_UNSUPPORTED, "instance %d: %s", k, err.c_str());
            }
            d.wq = (const float*)(c->ws + L.off_wq) + all_wq.size();
            all_wq.insert(all_wq.end(), wq.begin(), wq.end());
        }
        d.col_off = (int32_t)all_cols.size();
        fill_inst_params(d, fluids[k]);
        d.gaps = 0;
        for (const Col& cc : h.cols)
            if (cc.glo <= cc.ghi)
                d.gaps = 1;
        all_cols.insert(all_cols.end(), h.cols.begin(), h.cols.end());
    }
    // Default tiling.  FP32: the widest block not wider than the widest
    // instance, short strips (many concurrent items sweeping a narrow band of
    // rows, so halo rows and block-boundary lines are shared in L2).  16-bit
    // formats: one-wave blocks of 64 columns and 16-row strips (their step is
    // bound by issue and latency, not bytes, and runs fastest without the
    // four-wave row barrier; measured on the 256-channel batch: 0.53 ms
    // against 0.64 ms at 256 x 8).
    if ((storage & 0xff) == LBM_STORE_F32) {
        c->bx = max_nx >= 256 ? 256 : (max_nx >= 128 ? 128 : 64);
        c->strip = 8;
    } else {
        c->bx = 64;
        c->strip = 16;
    }
    c->ibx.assign(n_inst, c->bx);
    c->istrip.assign(n_inst, c->strip);
    build_items(c);

    lbm_status st = LBM_OK;
    auto bail = [&](lbm_status s) {
        delete c;
        return s;
    };
    hipError_t e;
    if ((e = hipMemcpyAsync(c->inst_d, c->idv.data(), sizeof(InstDev) * n_inst,
                            hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(c->cols_d, all_cols.data(), sizeof(Col) * all_cols.size(),
                            hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
        (!all_wq.empty() &&
         (e = hipMemcpyAsync(c->ws + L.off_wq, all_wq.data(), sizeof(float) * all_wq.size(),
                             hipMemcpyHostToDevice, c->stream)) != hipSuccess) ||
        (e = hipMemsetAsync(c->ws + L.off_buf[0], 0, 2 * L.buf_bytes, c->stream)) !=
            hipSuccess)
        return bail(fail(LBM_ERR_DEVICE, "lbm_init upload failed: %s", hipGetErrorString(e)));
    if ((st = upload_tables(c)) != LBM_OK)
        return bail(st);

    // Initial state, one instance at a time.
    for (int k = 0; k < n_inst; ++k) {
        const lbm_init_fields& in = inits[k];
        const InstHost& h = c->ih[k];
        InitDev ini{};
        ini.kind = in.kind;
        ini.core_species = in.core_species;
        ini.wall_rows = in.wall_rows;
        ini.rho_hi = in.rho_hi;
        ini.rho_lo = in.rho_lo;
        ini.cx = in.cx;
        ini.cy = in.cy;
        ini.r = in.r;
        {
            std::string err;  // validated above
            (void)slug_list(in.n_slugs, in.slugs, in.x0, in.length, ini.x0, ini.length,
                            ini.n_slugs, err);
        }
        ini.width = in.kind == LBM_INIT_SLUG ? in.width : 0.0;
        int first = h.ny, last = -1;
        for (const Col& cc : h.cols)
            if (cc.lo <= cc.hi) {
                first = std::min(first, cc.lo);
                last = std::max(last, cc.hi);
            }
        ini.first_row = first;
        ini.last_row = last;
        if ((e = launch_init(c->storage, c->buf[0], c->inst_d, k, c->cols_d, h.nx, h.ny, ini,
                             c->stream)) !=
            hipSuccess)
            return bail(fail(LBM_ERR_DEVICE, "init launch failed: %s", hipGetErrorString(e)));
    }
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return bail(fail(LBM_ERR_DEVICE, "init failed: %s", hipGetErrorString(e)));
    c->cur = 0;
    c->t = 0;
    *out = c;
    return LBM_OK;
}

// Enqueue nsteps step launches.  The rounding sequence of the 16-bit formats
// is keyed by the step number: passed as an argument, or, inside a captured
// graph, as the offset k from the value in seed_d that is set before every
// replay.
static lbm_status step_direct(lbm_ctx* c, int64_t nsteps, bool in_graph = false)
{
    for (int64_t k = 0; k < nsteps; ++k) {
        const uint32_t seed = in_graph ? (uint32_t)k : (uint32_t)c->t;
        lbm_status st = run_mode(c, kStep, seed, in_graph ? c->seed_d : nullptr);
        if (st != LBM_OK)
            return st;
        c->cur ^= 1;
        ++c->t;
    }
    return LBM_OK;
}

// Capture kGraphSteps step launches (an even number, so the buffers end where
// they started) into a graph for the current buffer parity and item list.
static lbm_status ensure_graph(lbm_ctx* c)
{
    if (c->graph && !c->graph_dirty && c->graph_cur == c->cur)
        return LBM_OK;
    if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    const int cur0 = c->cur;
    const int64_t t0 = c->t;
    lbm_status st = step_direct(c, kGraphSteps, true);
    c->cur = cur0;
    c->t = t0;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (st != LBM_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess)
        return fail(LBM_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->graph = nullptr;
        return fail(LBM_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    c->graph_cur = c->cur;
    c->graph_dirty = false;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps)
{
    if (!c || nsteps < 0)
        return fail(LBM_ERR_INVALID, "lbm_step: null context or negative step count");
    if (c->n_active_items == 0) {
        c->t += nsteps;
        return LBM_OK;
    }
    int64_t done = 0;
    lbm_status st = LBM_OK;
    if (c->stream != nullptr && nsteps >= kGraphSteps) {
        st = ensure_graph(c);
        if (st != LBM_OK)
            return st;
        for (; done + kGraphSteps <= nsteps; done += kGraphSteps) {
            HIP_TRY(launch_set_seed(c->seed_d, (uint32_t)c->t, c->stream));
            HIP_TRY(hipGraphLaunch(c->graph, c->stream));
            c->t += kGraphSteps;
        }
    }
    st = step_direct(c, nsteps - done);
    for (int k = 0; k < c->n_inst; ++k)
        if (c->active[k])
            c->ipar[k] = c->cur;
    return st;
}

lbm_status lbm_set_active(lbm_ctx* c, const uint8_t* active)
{
    if (!c || !active)
        return fail(LBM_ERR_INVALID, "lbm_set_active: null argument");
    lbm_status st = sync_all(c);
    if (st != LBM_OK)
        return st;
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int k = 0; k < c->n_inst; ++k)
        c->active[k] = active[k] ? 1 : 0;
    return upload_tables(c);
}

lbm_status lbm_snapshot_save(lbm_ctx* c)
{
    if (!c)
        return fail(LBM_ERR_INVALID, "lbm_snapshot_save: null context");
    if (!c->snap)
        return fail(LBM_ERR_INVALID, "lbm_snapshot_save: context created without LBM_OPT_SNAPSHOT");
    lbm_status st = sync_all(c);
    if (st != LBM_OK)
        return st;
    HIP_TRY(hipMemcpyAsync(c->snap, c->buf[c->cur], c->L.buf_bytes, hipMemcpyDeviceToDevice,
                           c->stream));
    c->snap_t = c->t;
    return LBM_OK;
}

lbm_status lbm_snapshot_restore(lbm_ctx* c, int32_t inst)
{
    if (!c || inst >= c->n_inst)
        return fail(LBM_ERR_INVALID, "lbm_snapshot_restore: bad argument");
    if (!c->snap || c->snap_t < 0)
        return fail(LBM_ERR_INVALID, "lbm_snapshot_restore: no snapshot saved");
    if (inst < 0) {
        HIP_TRY(hipMemcpyAsync(c->buf[c->cur], c->snap, c->L.buf_bytes, hipMemcpyDeviceToDevice,
                               c->stream));
        for (int k = 0; k < c->n_inst; ++k)
            c->ipar[k] = c->cur;
        return LBM_OK;
    }
    const InstHost& h = c->ih[inst];
    HIP_TRY(hipMemcpyAsync(c->buf[c->cur] + c->es * h.f_off, c->snap + c->es * h.f_off,
                           c->es * h.elems, hipMemcpyDeviceToDevice, c->stream));
    c->ipar[inst] = c->cur;
    return LBM_OK;
}

int64_t lbm_time(const lbm_ctx* c) { return c ? c->t : -1; }

lbm_status lbm_set_fluid(lbm_ctx* c, int32_t inst, const lbm_fluid* fluid)
{
    if (!c || !fluid || inst < 0 || inst >= c->n_inst)
        return fail(LBM_ERR_INVALID, "lbm_set_fluid: bad argument");
    lbm_status st = check_fluid(*fluid);
    if (st != LBM_OK)
        return st;
    const bool ext_before = any_ext(c);
    fill_inst_params(c->idv[inst], *fluid);
    if (any_ext(c) != ext_before)
        c->graph_dirty = true;  // the captured launches name the other kernels
    HIP_TRY(hipMemcpyAsync(c->inst_d + inst, &c->idv[inst], sizeof(InstDev),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_monitors(lbm_ctx* c, lbm_monitor* mon)
{
    if (!c || !mon)
        return fail(LBM_ERR_INVALID, "lbm_monitors: null argument");
    lbm_status st = sync_all(c);
    if (st != LBM_OK)
        return st;
    st = run_mode(c, kMonOnly);
    if (st != LBM_OK)
        return st;
    hipError_t e = launch_mon_reduce(c->partial_d, c->first_d, c->count_d, c->n_inst, c->mon_d,
                                     c->stream);
    if (e != hipSuccess)
        return fail(LBM_ERR_DEVICE, "monitor reduce failed: %s", hipGetErrorString(e));
    static_assert(sizeof(lbm_monitor) == kMonWidth * sizeof(double), "monitor layout");
    HIP_TRY(hipMemcpyAsync(mon, c->mon_d, sizeof(lbm_monitor) * c->n_inst, hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

static lbm_status export_instance(lbm_ctx* c, int inst)
{
    lbm_status st = sync_instance(c, inst);
    if (st != LBM_OK)
        return st;
    const InstHost& h = c->ih[inst];
    const size_t n = (size_t)h.nx * h.ny;
    HIP_TRY(hipMemsetAsync(c->stage_d, 0, sizeof(double) * kExportFields * n, c->stream));
    return run_range(c, c->ibx[inst], kExport, c->item_first[inst], c->item_count[inst]);
}

lbm_status lbm_moments(lbm_ctx* c, int32_t inst, double* rho, double* u, double* p,
                       lbm_monitor* mon)
{
    if (!c || inst < 0 || inst >= c->n_inst)
        return fail(LBM_ERR_INVALID, "lbm_moments: bad argument");
    const InstHost& h = c->ih[inst];
    const size_t n = (size_t)h.nx * h.ny;
    if (rho || u || p) {
        lbm_status st = export_instance(c, inst);
        if (st != LBM_OK)
            return st;
        if (rho)
            HIP_TRY(hipMemcpyAsync(rho, c->stage_d + 18 * n, sizeof(double) * 2 * n,
                                   hipMemcpyDeviceToHost, c->stream));
        if (u)
            HIP_TRY(hipMemcpyAsync(u, c->stage_d + 20 * n, sizeof(double) * 2 * n,
                                   hipMemcpyDeviceToHost, c->stream));
        if (p)
            HIP_TRY(hipMemcpyAsync(p, c->stage_d + 22 * n, sizeof(double) * n,
                                   hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    if (mon) {
        std::vector<lbm_monitor> all(c->n_inst);
        lbm_status st = lbm_monitors(c, all.data());
        if (st != LBM_OK)
            return st;
        *mon = all[inst];
    }
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_ctx* c, int32_t inst, double* f)
{
    if (!c || !f || inst < 0 || inst >= c->n_inst)
        return fail(LBM_ERR_INVALID, "lbm_get_populations: bad argument");
    const InstHost& h = c->ih[inst];
    const size_t n = (size_t)h.nx * h.ny;
    lbm_status st = export_instance(c, inst);
    if (st != LBM_OK)
        return st;
    HIP_TRY(hipMemcpyAsync(f, c->stage_d, sizeof(double) * 18 * n, hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_fluid_mask(lbm_ctx* c, int32_t inst, uint8_t* mask)
{
    if (!c || !mask || inst < 0 || inst >= c->n_inst)
        return fail(LBM_ERR_INVALID, "lbm_fluid_mask: bad argument");
    const InstHost& h = c->ih[inst];
    for (int y = 0; y < h.ny; ++y)
        for (int x = 0; x < h.nx; ++x)
            mask[(size_t)y * h.nx + x] = col_fluid(h.cols[x], y) ? 1 : 0;
    return LBM_OK;
}

lbm_status lbm_set_tiling(lbm_ctx* c, int32_t bx, int32_t strip_rows)
{
    if (!c)
        return fail(LBM_ERR_INVALID, "lbm_set_tiling: null context");
    if (bx != 64 && bx != 128 && bx != 256)
        return fail(LBM_ERR_INVALID, "lbm_set_tiling: bx must be 64, 128 or 256");
    if (strip_rows < kMinStrip || strip_rows > 32768)
        return fail(LBM_ERR_INVALID, "lbm_set_tiling: strip_rows must be >= %d", kMinStrip);
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->bx = bx;
    c->strip = strip_rows;
    c->ibx.assign(c->n_inst, bx);
    c->istrip.assign(c->n_inst, strip_rows);
    build_items(c);
    return upload_tables(c);
}

lbm_status lbm_set_instance_tiling(lbm_ctx* c, int32_t inst, int32_t bx, int32_t strip_rows)
{
    if (!c || inst < 0 || inst >= c->n_inst)
        return fail(LBM_ERR_INVALID, "lbm_set_instance_tiling: null context or bad instance");
    if (bx != 64 && bx != 128 && bx != 256)
        return fail(LBM_ERR_INVALID, "lbm_set_instance_tiling: bx must be 64, 128 or 256");
    if (strip_rows < kMinStrip || strip_rows > 32768)
        return fail(LBM_ERR_INVALID, "lbm_set_instance_tiling: strip_rows must be >= %d",
                    kMinStrip);
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->ibx[inst] = bx;
    c->istrip[inst] = strip_rows;
    build_items(c);
    return upload_tables(c);
}

lbm_status lbm_get_instance_tiling(const lbm_ctx* c, int32_t inst, int32_t* bx,
                                   int32_t* strip_rows)
{
    if (!c || inst < 0 || inst >= c->n_inst)
        return fail(LBM_ERR_INVALID, "lbm_get_instance_tiling: null context or bad instance");
    if (bx)
        *bx = c->ibx[inst];
    if (strip_rows)
        *strip_rows = c->istrip[inst];
    return LBM_OK;
}

lbm_status lbm_get_tiling(const lbm_ctx* c, int32_t* bx, int32_t* strip_rows, int32_t* n_items)
{
    if (!c)
        return fail(LBM_ERR_INVALID, "lbm_get_tiling: null context");
    if (bx)
        *bx = c->bx;
    if (strip_rows)
        *strip_rows = c->strip;
    if (n_items)
        *n_items = (int32_t)c->items.size();
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx* c, int32_t steps_per_trial, lbm_tune_report* report)
{
    if (!c || steps_per_trial < 2)
        return fail(LBM_ERR_INVALID, "lbm_autotune: null context or steps_per_trial < 2");
    if (c->n_active_items == 0)
        return fail(LBM_ERR_INVALID, "lbm_autotune: no active instance");
    // Buckets: active instances of equal width, largest total fluid nodes first.
    std::vector<std::pair<int64_t, int>> order;  // (fluid nodes, nx)
    for (int k = 0; k < c->n_inst; ++k) {
        if (!c->active[k])
            continue;
        int64_t nodes = 0;
        for (const Col& cc : c->ih[k].cols)
            nodes += col_nodes(cc);
        auto it = std::find_if(order.begin(), order.end(),
                               [&](const std::pair<int64_t, int>& b) { return b.second == c->ih[k].nx; });
        if (it == order.end())
            order.emplace_back(nodes, c->ih[k].nx);
        else
            it->first += nodes;
    }
    std::sort(order.begin(), order.end(), std::greater<std::pair<int64_t, int>>());

    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(LBM_ERR_DEVICE, "lbm_autotune: hipEventCreate failed");
    }
    lbm_tune_report rep{};
    lbm_status st = LBM_OK;
    // Per-step time of steps_per_trial real steps with the current tiling.
    auto trial = [&](double& ms) -> lbm_status {
        if (hipEventRecord(e0, c->stream) != hipSuccess)
            return fail(LBM_ERR_DEVICE, "lbm_autotune: event record failed");
        lbm_status s2 = lbm_step(c, steps_per_trial);
        if (s2 != LBM_OK)
            return s2;
        float t = 0.0f;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            return fail(LBM_ERR_DEVICE, "lbm_autotune: event timing failed");
        ms = (double)t / steps_per_trial;
        ++rep.trials;
        rep.steps += steps_per_trial;
        return LBM_OK;
    };
    auto apply = [&](int nx, int bx, int strip) -> lbm_status {
        HIP_TRY(hipStreamSynchronize(c->stream));
        for (int k = 0; k < c->n_inst; ++k)
            if (c->active[k] && c->ih[k].nx == nx) {
                c->ibx[k] = bx;
                c->istrip[k] = strip;
            }
        build_items(c);
        return upload_tables(c);
    };
    double best = 0.0, ms = 0.0;
    static const int kStrips[] = {4, 8, 16, 32};
    if ((st = trial(ms)) == LBM_OK)  // warm-up (graph capture, caches)
        st = trial(best);
    rep.ms_before = best;
    for (size_t b = 0; st == LBM_OK && b < order.size(); ++b) {
        const int nx = order[b].second;
        int kb = -1;
        for (int k = 0; k < c->n_inst; ++k)
            if (c->active[k] && c->ih[k].nx == nx) {
                kb = k;
                break;
            }
        int cur_bx = c->ibx[kb], cur_strip = c->istrip[kb];
        for (int cl = 0; st == LBM_OK && cl < 3; ++cl) {
            const int bx = kBxClasses[cl];
            if (bx > 64 && bx > (int)align_up((size_t)nx, 64))
                continue;
            for (int strip : kStrips) {
                if (bx == cur_bx && strip == cur_strip)
                    continue;
                if ((st = apply(nx, bx, strip)) != LBM_OK || (st = trial(ms)) != LBM_OK)
                    break;
                if (ms < best * 0.997) {
                    best = ms;
                    cur_bx = bx;
                    cur_strip = strip;
                }
            }
        }
        if (st == LBM_OK)
            st = apply(nx, cur_bx, cur_strip);
    }
    if (st == LBM_OK)
        st = trial(rep.ms_after);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != LBM_OK)
        return st;
    rep.buckets = (int32_t)order.size();
    if (report)
        *report = rep;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* c)
{
    // Queued steps (graph replays included) still use the caller's workspace:
    // drain them before the caller can free it.
    if (c)
        (void)hipStreamSynchronize(c->stream);
    delete c;
}

}  // extern "C"
