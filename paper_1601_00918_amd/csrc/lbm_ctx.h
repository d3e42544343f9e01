// Host-side context of the C ABI, shared by the runtime (lbm_runtime.cpp) and
// the critical-pressure driver (lbm_driver.cpp).  Not part of the public ABI.
#pragma once

#include "lbm.h"
#include "lbm_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

namespace lbm {

// Host description of one instance.
struct InstHost {
    int kind;
    int nx, ny;
    int pitch;
    int64_t elems;  // elements of this instance in one buffer (rstride * ny)
    int64_t f_off;
    std::vector<Col> cols;  // per column fluid runs
};

// Workspace carving (byte offsets into the caller's device workspace).
struct Layout {
    size_t buf_bytes;  // one population buffer
    size_t off_buf[2], off_snap, off_inst, off_items, off_cols, off_partial, off_mon,
        off_first, off_count, off_stage, off_seed, off_wq, total;
    int64_t n_items_max;
    int64_t max_nodes;
};


// Slugs of a SLUG initial state: the single (x0, length) when n is 0, else the
// n host pairs.  Returns false with a message on invalid input.
inline bool slug_list(int32_t n, const double* pairs, double x0, double length, double* xs,
                      double* ls, int32_t& count, std::string& err)
{
    if (n < 0 || n > LBM_MAX_SLUGS) {
        err = "n_slugs must lie in 0.." + std::to_string(LBM_MAX_SLUGS);
        return false;
    }
    if (n >= 1 && !pairs) {
        err = "n_slugs >= 1 needs the slugs array";
        return false;
    }
    count = n == 0 ? 1 : n;
    for (int k = 0; k < count; ++k) {
        xs[k] = n == 0 ? x0 : pairs[2 * k];
        ls[k] = n == 0 ? length : pairs[2 * k + 1];
        if (!std::isfinite(xs[k]) || !(ls[k] >= 0.0) || !std::isfinite(ls[k])) {
            err = "slug " + std::to_string(k) + ": x0 must be finite and length >= 0";
            return false;
        }
    }
    return true;
}

}  // namespace lbm

struct lbm_ctx {
    using InstHost = lbm::InstHost;
    using InstDev = lbm::InstDev;
    using Item = lbm::Item;
    using Layout = lbm::Layout;
    using Col = lbm::Col;
    int n_inst = 0;
    int storage = LBM_STORE_F32;
    std::vector<InstHost> ih;
    std::vector<InstDev> idv;
    std::vector<Item> items;
    std::vector<Item> act_items;  // items of the active instances (host copy)
    std::vector<int32_t> item_first, item_count;
    Layout L{};
    char* ws = nullptr;
    char* buf[2] = {nullptr, nullptr};  // population buffers (element size es)
    size_t es = 4;
    InstDev* inst_d = nullptr;
    Item* items_d = nullptr;
    Col* cols_d = nullptr;
    double* partial_d = nullptr;
    double* mon_d = nullptr;
    int32_t* first_d = nullptr;
    int32_t* count_d = nullptr;
    double* stage_d = nullptr;
    uint32_t* seed_d = nullptr;  // step number read by captured graphs
    hipStream_t stream = nullptr;
    int cur = 0;
    int64_t t = 0;
    // Tiling: per instance, columns per workgroup (64, 128, 256) and rows per
    // strip.  Items are grouped by workgroup width (one launch per width and
    // step): cls_first / cls_count index the full item list, act_first /
    // act_count the active list, in the order of kBxClasses.
    int bx = 256;    // last value set for every instance
    int strip = 8;
    std::vector<int> ibx, istrip;
    int cls_first[3] = {0, 0, 0}, cls_count[3] = {0, 0, 0};
    int act_first[3] = {0, 0, 0}, act_count[3] = {0, 0, 0};
    // Work items being stepped: a copy of the items of the active instances,
    // stored on the device after the full list (at items_d + L.n_items_max).
    std::vector<uint8_t> active;
    int n_active_items = 0;
    // Buffer (0/1) holding each instance's current state: active instances
    // follow `cur`; an inactive one stays where it was when it stopped.
    std::vector<int> ipar;
    // Snapshot buffer (optional, LBM_OPT_SNAPSHOT).
    char* snap = nullptr;
    int64_t snap_t = -1;
    // Cached graph of kGraphSteps step launches (non-null streams only).
    hipGraphExec_t graph = nullptr;
    int graph_cur = -1;
    bool graph_dirty = true;
    ~lbm_ctx();
};

namespace lbm {
// Error reporting shared by the runtime and the driver.
lbm_status fail(lbm_status st, const char* fmt, ...);
}  // namespace lbm


