// Batches of independent lattices: the entry points lbm_batch_* of lbm.h.
//
// Every item is an ordinary context (lbm_ctx) whose device buffers are
// slices of the batch's buffers 0-4, so that geometry, links, initial state
// and readback go through the single-context entry points.  The batch adds
// the item descriptor table (buffer 5), the work tables of the shared
// launches (buffer 6) and the per-item convergence state (buffer 7), and
// drives the batched kernels: tiled launches over all active items, or one
// resident workgroup per item running several steps per launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_ctx.hpp"
#include "lbm_internal.hpp"

using namespace lbmh;

struct lbm_batch {
    int n = 0;
    std::vector<lbm_ctx*> items;
    lbmi::KernelSet ks;
    void* buf[LBM_NBUF] = {};
    size_t size[LBM_NBUF] = {};
    hipStream_t stream = nullptr;
    lbm_batch_config cfg{LBM_BATCH_TILED, 256, 1, 64};
    std::string err;
    // device regions inside buffers 5-7
    char* desc = nullptr;
    uint32_t *tiles = nullptr, *ltiles = nullptr, *active = nullptr;
    uint32_t *status = nullptr, *steps = nullptr, *snap_ok = nullptr;
    double* resid = nullptr;
    size_t max_tiles = 0, max_ltiles = 0;
    // host copies: descriptors, work tables, statuses
    std::vector<char> desc_h;
    std::vector<uint32_t> tiles_h, ltiles_h, active_h, status_h;
    std::vector<uint8_t> enabled;  // items that take part in batched calls
    uint32_t n_tiles = 0, n_ltiles = 0, n_active = 0, tile = 0;
    // the device holds descriptors / work tables for the items' current state
    // (valid within one entry point: the items may change between calls)
    bool desc_valid = false, tables_valid = false;
    // captured graph and what it was captured for
    hipGraphExec_t graph = nullptr;
    hipStream_t capture_stream = nullptr;
    int graph_kind = 0;  // 1: graph_steps plain steps; 2: interval steps, then the residual check
    int graph_interval = 0;
    double graph_tol = 0.0;
};

namespace {

constexpr int kMinTile = 64;
constexpr int kLinkTile = 256;

lbm_status bset_err(lbm_batch* b, lbm_status s, const std::string& m) {
    if (b) b->err = m;
    return s;
}

lbm_status bhip(lbm_batch* b, hipError_t e, const char* what) {
    if (e == hipSuccess) return LBM_OK;
    return bset_err(b, LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool same_combo(const lbm_params& a, const lbm_params& b) {
    return a.dim == b.dim && a.fluid == b.fluid && a.scalar == b.scalar && a.magnetic == b.magnetic &&
           a.mag_ncomp == b.mag_ncomp && a.storage == b.storage;
}

int resident_limit(const lbmi::KernelSet&) { return 512; }

// Per-item buffer sizes and offsets inside the batch buffers 0-4, and the
// sizes of buffers 5-7.
struct BatchLayout {
    std::vector<size_t> item_size;  // [n][5]
    std::vector<size_t> item_off;   // [n][5]
    size_t sz[LBM_NBUF] = {};
    size_t max_tiles = 0, max_ltiles = 0;
    size_t off_ltiles = 0, off_active = 0;        // inside buffer 6
    size_t off_steps = 0, off_snap = 0, off_resid = 0;  // inside buffer 7
};

bool batch_layout(int n, const lbm_params* p, const size_t* nl, BatchLayout* L, std::string* why) {
    if (n < 1) {
        if (why) *why = "n_items must be positive";
        return false;
    }
    if (!p || !nl) {
        if (why) *why = "items or n_links is NULL";
        return false;
    }
    for (int i = 0; i < n; ++i) {
        std::string w;
        if (!valid_params(&p[i], &w)) {
            if (why) *why = "item " + std::to_string(i) + ": " + w;
            return false;
        }
        if (p[i].scalar_ncomp > 1) {
            if (why) *why = "item " + std::to_string(i) + ": several scalar components are not batched";
            return false;
        }
        if (!same_combo(p[0], p[i])) {
            if (why) *why = "item " + std::to_string(i) + " differs from item 0 in lattices or storage";
            return false;
        }
    }
    const lbmi::KernelSet ks = kernels_for(&p[0]);
    if (!ks.b_sweep) {
        if (why) *why = "no kernels for this lattice combination";
        return false;
    }
    L->item_size.assign((size_t)n * 5, 0);
    L->item_off.assign((size_t)n * 5, 0);
    for (int i = 0; i < n; ++i) {
        size_t s[LBM_NBUF];
        layout(&p[i], nl[i], s);
        for (int k = 0; k < 5; ++k) {
            L->item_size[(size_t)i * 5 + k] = s[k];
            L->item_off[(size_t)i * 5 + k] = L->sz[k];
            L->sz[k] += round_up(s[k], kAlign);
        }
        const Pad d = padding(&p[i]);
        L->max_tiles += (d.nodes + kMinTile - 1) / kMinTile;
        L->max_ltiles += (nl[i] + kLinkTile - 1) / kLinkTile;
    }
    L->sz[5] = round_up((size_t)n * ks.item_bytes, kAlign);
    L->off_ltiles = round_up(L->max_tiles * 8, kAlign);
    L->off_active = L->off_ltiles + round_up(std::max<size_t>(L->max_ltiles, 1) * 8, kAlign);
    L->sz[6] = L->off_active + round_up((size_t)n * 4, kAlign);
    L->off_steps = round_up((size_t)n * 4, kAlign);
    L->off_snap = L->off_steps + round_up((size_t)n * 4, kAlign);
    L->off_resid = L->off_snap + round_up((size_t)n * 4, kAlign);
    L->sz[7] = L->off_resid + round_up((size_t)n * 8, kAlign);
    return true;
}

void drop_bgraph(lbm_batch* b) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    b->graph_kind = 0;
}

// every enabled item set up, their times of one parity
lbm_status check_ready(lbm_batch* b) {
    int first = -1;
    for (int i = 0; i < b->n; ++i) {
        if (!b->enabled[i]) continue;
        const lbm_ctx* c = b->items[i];
        if (!c->initialized) return bset_err(b, LBM_ESTATE, "item " + std::to_string(i) + " is not initialised");
        if (first < 0) first = i;
        if ((c->t & 1) != (b->items[first]->t & 1)) return bset_err(b, LBM_ESTATE, "item times differ in parity");
    }
    return LBM_OK;
}

bool any_enabled(const lbm_batch* b) {
    for (uint8_t e : b->enabled)
        if (e) return true;
    return false;
}

int first_enabled(const lbm_batch* b) {
    for (int i = 0; i < b->n; ++i)
        if (b->enabled[i]) return i;
    return 0;
}

void advance(lbm_batch* b, int64_t k) {
    for (int i = 0; i < b->n; ++i)
        if (b->enabled[i]) b->items[i]->t += k;
}

// the residual snapshot and accumulators of an item (its buffer 4)
void aux_of(const lbm_ctx* c, void** snap, double** acc) {
    char* aux = (char*)c->buf[4];
    *snap = aux;
    *acc = (double*)(aux + round_up((size_t)(moment_planes(&c->p) - 1) * c->pad.plane * compute_bytes(c->p.storage),
                                    kAlign));
}

// item descriptors from the items' current state (links count only for items
// past time 0), uploaded synchronously
lbm_status upload_descriptors(lbm_batch* b) {
    const size_t ib = b->ks.item_bytes;
    b->desc_h.assign((size_t)b->n * ib, 0);
    for (int i = 0; i < b->n; ++i) {
        const lbm_ctx* c = b->items[i];
        lbmi::KArgs a = base_args(c);
        aux_of(c, &a.snap, &a.acc);
        a.links_ready = c->t > 0 ? 1 : 0;
        a.tbase = time_base(c);
        a.tstep = (uint32_t)c->t;
        b->ks.describe(a, b->desc_h.data() + (size_t)i * ib);
    }
    b->desc_valid = false;
    lbm_status st = bhip(b, hipMemcpyAsync(b->desc, b->desc_h.data(), b->desc_h.size(), hipMemcpyHostToDevice,
                                           b->stream), "descriptor upload");
    if (st) return st;
    // every item's time base starts at its time
    lbmi::BArgs ta;
    std::memset(&ta, 0, sizeof ta);
    ta.items = b->desc;
    ta.n_active = (uint32_t)b->n;
    ta.stream = b->stream;
    if ((st = bhip(b, b->ks.b_set_time(ta), "time base"))) return st;
    drop_bgraph(b);
    if ((st = bhip(b, hipStreamSynchronize(b->stream), "descriptor upload sync"))) return st;
    b->desc_valid = true;
    return LBM_OK;
}

// node tiles of `tile` nodes and link tiles of the items whose host status is
// active, uploaded synchronously
lbm_status build_tables(lbm_batch* b, uint32_t tile) {
    b->tiles_h.clear();
    b->ltiles_h.clear();
    b->active_h.clear();
    for (int i = 0; i < b->n; ++i) {
        if (b->status_h[i] != lbmi::BS_ACTIVE) continue;
        const lbm_ctx* c = b->items[i];
        b->active_h.push_back((uint32_t)i);
        for (size_t s = 0; s < c->pad.nodes; s += tile) {
            b->tiles_h.push_back((uint32_t)i);
            b->tiles_h.push_back((uint32_t)s);
        }
        if (c->t > 0)
            for (size_t s = 0; s < c->n_links; s += kLinkTile) {
                b->ltiles_h.push_back((uint32_t)i);
                b->ltiles_h.push_back((uint32_t)s);
            }
    }
    b->n_tiles = (uint32_t)(b->tiles_h.size() / 2);
    b->n_ltiles = (uint32_t)(b->ltiles_h.size() / 2);
    b->n_active = (uint32_t)b->active_h.size();
    b->tile = tile;
    if (b->n_tiles > b->max_tiles || b->n_ltiles > b->max_ltiles) return bset_err(b, LBM_ESIZE, "work tables overflow");
    lbm_status st;
    if (b->n_tiles &&
        (st = bhip(b, hipMemcpyAsync(b->tiles, b->tiles_h.data(), b->tiles_h.size() * 4, hipMemcpyHostToDevice,
                                     b->stream), "tile upload")))
        return st;
    if (b->n_ltiles &&
        (st = bhip(b, hipMemcpyAsync(b->ltiles, b->ltiles_h.data(), b->ltiles_h.size() * 4, hipMemcpyHostToDevice,
                                     b->stream), "link tile upload")))
        return st;
    if (b->n_active &&
        (st = bhip(b, hipMemcpyAsync(b->active, b->active_h.data(), b->active_h.size() * 4, hipMemcpyHostToDevice,
                                     b->stream), "active list upload")))
        return st;
    drop_bgraph(b);
    b->tables_valid = true;
    return bhip(b, hipStreamSynchronize(b->stream), "table upload sync");
}

lbmi::BArgs bargs(const lbm_batch* b, hipStream_t s) {
    lbmi::BArgs a;
    std::memset(&a, 0, sizeof a);
    a.items = b->desc;
    a.tiles = b->tiles;
    a.n_tiles = b->n_tiles;
    a.tile = b->tile;
    a.ltiles = b->ltiles;
    a.n_ltiles = b->n_ltiles;
    a.active = b->active;
    a.n_active = b->n_active;
    a.status = b->status;
    a.steps = b->steps;
    a.resid = b->resid;
    a.snap_ok = b->snap_ok;
    a.block = b->cfg.block;
    a.nsteps = b->cfg.steps_per_launch;
    a.stream = s;
    return a;
}

// every launch reads the descriptors; all but the clear also the work tables
lbm_status need_tables(lbm_batch* b, bool tables) {
    if (!b->desc_valid || (tables && !b->tables_valid))
        return bset_err(b, LBM_ESTATE, "batch descriptors or work tables are not on the device");
    return LBM_OK;
}

uint32_t table_tile(const lbm_batch* b) { return b->cfg.mode == LBM_BATCH_TILED ? (uint32_t)b->cfg.block : 256u; }

// every item active again, counters cleared (all items).  The clear kernel
// reads each item's accumulator address from the descriptor table, so the
// descriptors are written first.
lbm_status reset_state(lbm_batch* b) {
    lbm_status st = upload_descriptors(b);
    if (st) return st;
    b->status_h.assign(b->n, lbmi::BS_ACTIVE);
    std::vector<uint32_t> all(b->n);
    for (int i = 0; i < b->n; ++i) all[i] = (uint32_t)i;
    // enabled items start active with cleared counters; the others are frozen
    uint32_t ne = 0;
    for (int i = 0; i < b->n; ++i) {
        if (b->enabled[i]) all[ne++] = (uint32_t)i;
        else b->status_h[i] = lbmi::BS_DISABLED;
    }
    if ((st = bhip(b, hipMemcpyAsync(b->status, b->status_h.data(), (size_t)b->n * 4, hipMemcpyHostToDevice, b->stream),
                   "status upload")))
        return st;
    if (ne && (st = bhip(b, hipMemcpyAsync(b->active, all.data(), (size_t)ne * 4, hipMemcpyHostToDevice, b->stream),
                         "active list upload")))
        return st;
    if ((st = need_tables(b, false))) return st;
    lbmi::BArgs a = bargs(b, b->stream);
    a.active = b->active;
    a.n_active = ne;
    if ((st = bhip(b, b->ks.b_clear(a), "clear launch"))) return st;
    st = bhip(b, hipStreamSynchronize(b->stream), "clear sync");
    b->tables_valid = false;  // the active list was overwritten
    drop_bgraph(b);
    return st;
}

// steps [0, n) of a run starting at parity `parity`, queued on stream s
lbm_status enqueue_steps(lbm_batch* b, int64_t n, int parity, hipStream_t s) {
    if (lbm_status st = need_tables(b, true)) return st;
    lbmi::BArgs a = bargs(b, s);
    int64_t i = 0;
    if (b->cfg.mode == LBM_BATCH_RESIDENT && parity == 0) {
        const int64_t spl = b->cfg.steps_per_launch;
        while (n - i >= 2) {
            a.nsteps = (int)std::min<int64_t>(spl, (n - i) & ~int64_t(1));
            a.tstep = (uint32_t)i;
            if (hipError_t e = b->ks.b_resident(a)) return bhip(b, e, "resident launch");
            i += a.nsteps;
        }
    }
    for (; i < n; ++i) {
        a.parity = (int)((parity + i) & 1);
        a.tstep = (uint32_t)i;
        if (hipError_t e = b->ks.b_links(a)) return bhip(b, e, "link launch");
        if (hipError_t e = b->ks.b_sweep(a)) return bhip(b, e, "sweep launch");
    }
    return LBM_OK;
}

lbm_status enqueue_check(lbm_batch* b, int interval, double tol, hipStream_t s) {
    if (lbm_status st = need_tables(b, true)) return st;
    lbmi::BArgs a = bargs(b, s);
    a.parity = 0;
    a.tstep = (uint32_t)interval;  // the check runs at the end of the interval
    a.interval = interval;
    a.tol = tol;
    if (hipError_t e = b->ks.b_reduce(a)) return bhip(b, e, "reduce launch");
    if (hipError_t e = b->ks.b_judge(a)) return bhip(b, e, "judge launch");
    return LBM_OK;
}

// captures kind 1 (graph_steps steps) or kind 2 (interval steps + check)
lbm_status capture(lbm_batch* b, int kind, int interval, double tol) {
    if (b->graph && b->graph_kind == kind && b->graph_interval == interval && b->graph_tol == tol) return LBM_OK;
    drop_bgraph(b);
    if (!b->capture_stream && hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        b->capture_stream = nullptr;
        return bset_err(b, LBM_EDEVICE, "capture stream");
    }
    if (hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bset_err(b, LBM_EDEVICE, "begin capture");
    const int steps = kind == 1 ? b->cfg.graph_steps : interval;
    lbm_status st = enqueue_steps(b, steps, 0, b->capture_stream);
    if (!st && kind == 2) st = enqueue_check(b, interval, tol, b->capture_stream);
    if (!st) {
        // the time bases of the listed items follow the run
        lbmi::BArgs a = bargs(b, b->capture_stream);
        a.tstep = (uint32_t)steps;
        if (hipError_t e = b->ks.b_tick(a)) st = bhip(b, e, "time base");
    }
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(b->capture_stream, &g);
    if (st || ee != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return st ? st : bset_err(b, LBM_EDEVICE, "end capture");
    }
    hipError_t ie = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        b->graph = nullptr;
        return bset_err(b, LBM_EDEVICE, "graph instantiate");
    }
    b->graph_kind = kind;
    b->graph_interval = interval;
    b->graph_tol = tol;
    return LBM_OK;
}

// single tiled steps until every item is past time 0 and the time is even;
// returns the number of steps run (every item runs them)
lbm_status pre_steps(lbm_batch* b, int64_t budget, int64_t* done) {
    *done = 0;
    auto needs = [&]() {
        for (int i = 0; i < b->n; ++i)
            if (b->enabled[i] && (b->items[i]->t == 0 || (b->items[i]->t & 1))) return true;
        return false;
    };
    while (*done < budget && needs()) {
        lbm_status st;
        if ((st = upload_descriptors(b))) return st;
        if ((st = build_tables(b, table_tile(b)))) return st;
        if ((st = need_tables(b, true))) return st;
        lbmi::BArgs a = bargs(b, b->stream);
        a.parity = (int)(b->items[first_enabled(b)]->t & 1);
        if ((st = bhip(b, b->ks.b_links(a), "link launch"))) return st;
        if ((st = bhip(b, b->ks.b_sweep(a), "sweep launch"))) return st;
        advance(b, 1);
        ++*done;
    }
    if (*done) {
        lbm_status st = upload_descriptors(b);
        if (st) return st;
        b->tables_valid = false;
    }
    return LBM_OK;
}

bool valid_config(const lbm_batch* b, const lbm_batch_config& c, std::string* why) {
    auto fail = [&](const char* m) {
        if (why) *why = m;
        return false;
    };
    if (c.mode == LBM_BATCH_TILED) {
        if (c.block != 64 && c.block != 128 && c.block != 256) return fail("tiled block must be 64, 128 or 256");
        if (c.steps_per_launch != 1) return fail("tiled steps_per_launch must be 1");
    } else if (c.mode == LBM_BATCH_RESIDENT) {
        if (c.block < 64 || c.block % 64 || c.block > resident_limit(b->ks))
            return fail("resident block must be a multiple of 64 within the kernel's limit");
        if (c.steps_per_launch < 2 || (c.steps_per_launch & 1)) return fail("resident steps_per_launch must be even");
    } else {
        return fail("unknown mode");
    }
    if (c.graph_steps < 2 || (c.graph_steps & 1) || c.graph_steps % c.steps_per_launch)
        return fail("graph_steps must be even and a multiple of steps_per_launch");
    return true;
}

// after batched steps: an item's own residual restarts (the batch used its
// snapshot buffer)
void after_batch_steps(lbm_batch* b) {
    for (auto* c : b->items) c->snap_valid = false;
    b->desc_valid = b->tables_valid = false;
}

}  // namespace

extern "C" {

size_t lbm_batch_required_bytes(int32_t n_items, const lbm_params* items, const size_t* n_links,
                                size_t sizes_out[LBM_NBUF]) {
    BatchLayout L;
    if (!batch_layout(n_items, items, n_links, &L, nullptr)) return 0;
    size_t tot = 0;
    for (int k = 0; k < LBM_NBUF; ++k) {
        if (sizes_out) sizes_out[k] = L.sz[k];
        tot += L.sz[k];
    }
    return tot;
}

lbm_status lbm_batch_create(int32_t n_items, const lbm_params* items, const size_t* n_links,
                            void* const dev_bufs[LBM_NBUF], void* hip_stream, lbm_batch** out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    BatchLayout L;
    if (!batch_layout(n_items, items, n_links, &L, nullptr) || !dev_bufs) return LBM_EINVAL;
    for (int k = 0; k < LBM_NBUF; ++k) {
        if (L.sz[k] > 0 && !dev_bufs[k]) return LBM_EINVAL;
        if (L.sz[k] > 0 && ((uintptr_t)dev_bufs[k] % kAlign) != 0) return LBM_EINVAL;
    }
    lbm_batch* b = new lbm_batch();
    b->n = n_items;
    b->ks = kernels_for(&items[0]);
    b->stream = (hipStream_t)hip_stream;
    for (int k = 0; k < LBM_NBUF; ++k) {
        b->buf[k] = dev_bufs[k];
        b->size[k] = L.sz[k];
    }
    b->desc = (char*)dev_bufs[5];
    b->tiles = (uint32_t*)dev_bufs[6];
    b->ltiles = (uint32_t*)((char*)dev_bufs[6] + L.off_ltiles);
    b->active = (uint32_t*)((char*)dev_bufs[6] + L.off_active);
    b->status = (uint32_t*)dev_bufs[7];
    b->steps = (uint32_t*)((char*)dev_bufs[7] + L.off_steps);
    b->snap_ok = (uint32_t*)((char*)dev_bufs[7] + L.off_snap);
    b->resid = (double*)((char*)dev_bufs[7] + L.off_resid);
    b->max_tiles = L.max_tiles;
    b->max_ltiles = L.max_ltiles;
    b->status_h.assign(n_items, lbmi::BS_ACTIVE);
    b->enabled.assign(n_items, 1);
    for (int i = 0; i < n_items; ++i) {
        lbm_ctx* c = new lbm_ctx();
        c->p = items[i];
        c->pad = padding(&items[i]);
        c->ks = b->ks;
        for (int k = 0; k < LBM_NBUF; ++k) {
            c->buf[k] = nullptr;
            c->size[k] = 0;
        }
        for (int k = 0; k < 5; ++k) {
            c->size[k] = L.item_size[(size_t)i * 5 + k];
            c->buf[k] = (char*)dev_bufs[k] + L.item_off[(size_t)i * 5 + k];
        }
        c->cap_links = n_links[i];
        c->stream = b->stream;
        if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
        c->batch_owned = true;
        b->items.push_back(c);
    }
    *out = b;
    return LBM_OK;
}

lbm_ctx* lbm_batch_item(lbm_batch* b, int32_t i) {
    if (!b || i < 0 || i >= b->n) return nullptr;
    return b->items[i];
}

lbm_status lbm_batch_set_active(lbm_batch* b, const uint8_t* host_flags) {
    if (!b) return LBM_EINVAL;
    if (!host_flags) return bset_err(b, LBM_EINVAL, "flags is NULL");
    for (int i = 0; i < b->n; ++i) b->enabled[i] = host_flags[i] ? 1 : 0;
    b->desc_valid = b->tables_valid = false;
    drop_bgraph(b);
    return LBM_OK;
}

lbm_status lbm_batch_configure(lbm_batch* b, const lbm_batch_config* cfg) {
    if (!b || !cfg) return LBM_EINVAL;
    std::string why;
    if (!valid_config(b, *cfg, &why)) return bset_err(b, LBM_EINVAL, why);
    b->cfg = *cfg;
    b->tables_valid = false;
    drop_bgraph(b);
    return LBM_OK;
}

lbm_status lbm_batch_get_config(const lbm_batch* b, lbm_batch_config* cfg) {
    if (!b || !cfg) return LBM_EINVAL;
    *cfg = b->cfg;
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t n) {
    if (!b) return LBM_EINVAL;
    if (n < 0) return bset_err(b, LBM_EINVAL, "negative step count");
    lbm_status st;
    if ((st = check_ready(b))) return st;
    if (n == 0 || !any_enabled(b)) return LBM_OK;
    if ((st = reset_state(b))) return st;
    int64_t pre = 0;
    if ((st = pre_steps(b, n, &pre))) return st;
    n -= pre;
    if (n == 0) {
        after_batch_steps(b);
        return LBM_OK;
    }
    if ((st = upload_descriptors(b))) return st;
    if ((st = build_tables(b, table_tile(b)))) return st;
    const int64_t G = b->cfg.graph_steps;
    if (n >= G) {
        if ((st = capture(b, 1, 0, 0.0))) return st;
        for (; n >= G; n -= G) {
            if ((st = bhip(b, hipGraphLaunch(b->graph, b->stream), "graph launch"))) return st;
            advance(b, G);
        }
    }
    if (n > 0) {
        if ((st = enqueue_steps(b, n, 0, b->stream))) return st;
        advance(b, n);
    }
    after_batch_steps(b);
    return LBM_OK;
}

lbm_status lbm_batch_run(lbm_batch* b, double tol, int32_t interval, int64_t max_steps, int64_t* steps_out,
                         double* resid_out, int32_t* status_out) {
    if (!b) return LBM_EINVAL;
    if (interval < 2 || (interval & 1)) return bset_err(b, LBM_EINVAL, "interval must be even and >= 2");
    if (!(tol >= 0.0) || max_steps < 0) return bset_err(b, LBM_EINVAL, "bad tol or max_steps");
    lbm_status st;
    if ((st = check_ready(b))) return st;
    if ((st = reset_state(b))) return st;
    int64_t pre = 0;
    if ((st = pre_steps(b, max_steps, &pre))) return st;
    std::vector<uint32_t> steps_h(b->n, 0);
    std::vector<double> resid_h(b->n, -1.0);
    if (pre < max_steps) {
        if ((st = reset_state(b))) return st;
        if ((st = upload_descriptors(b))) return st;
        if ((st = build_tables(b, table_tile(b)))) return st;
        int64_t run = 0;
        uint32_t active_at_build = b->n_active;
        while (run < max_steps - pre && b->n_active > 0) {
            if ((st = capture(b, 2, interval, tol))) return st;
            if ((st = bhip(b, hipGraphLaunch(b->graph, b->stream), "graph launch"))) return st;
            run += interval;
            if ((st = bhip(b, hipMemcpyAsync(b->status_h.data(), b->status, (size_t)b->n * 4, hipMemcpyDeviceToHost,
                                             b->stream), "status copy")))
                return st;
            if ((st = bhip(b, hipStreamSynchronize(b->stream), "run sync"))) return st;
            uint32_t act = 0;
            for (int i = 0; i < b->n; ++i) act += b->status_h[i] == lbmi::BS_ACTIVE;
            if (act == 0) break;
            if (act * 10 <= active_at_build * 9) {
                if ((st = build_tables(b, table_tile(b)))) return st;
                active_at_build = b->n_active;
            }
        }
        if ((st = bhip(b, hipMemcpyAsync(steps_h.data(), b->steps, (size_t)b->n * 4, hipMemcpyDeviceToHost, b->stream),
                       "steps copy")))
            return st;
        if ((st = bhip(b, hipMemcpyAsync(resid_h.data(), b->resid, (size_t)b->n * 8, hipMemcpyDeviceToHost, b->stream),
                       "residual copy")))
            return st;
        if ((st = bhip(b, hipMemcpyAsync(b->status_h.data(), b->status, (size_t)b->n * 4, hipMemcpyDeviceToHost,
                                         b->stream), "status copy")))
            return st;
        if ((st = bhip(b, hipStreamSynchronize(b->stream), "run sync"))) return st;
    }
    for (int i = 0; i < b->n; ++i) {
        if (!b->enabled[i]) steps_h[i] = 0;
        b->items[i]->t += steps_h[i];
        if (steps_out) steps_out[i] = b->enabled[i] ? pre + (int64_t)steps_h[i] : 0;
        if (resid_out) resid_out[i] = resid_h[i];
        if (status_out) status_out[i] = (int32_t)b->status_h[i];
    }
    after_batch_steps(b);
    b->tables_valid = false;
    return LBM_OK;
}

lbm_status lbm_batch_tune(lbm_batch* b, int64_t trial_steps, lbm_batch_config* best, lbm_batch_config* cands,
                          double* ms_per_step, int32_t cap, int32_t* n_out) {
    if (!b) return LBM_EINVAL;
    if (trial_steps < 2) return bset_err(b, LBM_EINVAL, "trial_steps must be >= 2");
    if (cap < 0 || (cap > 0 && (!cands || !ms_per_step))) return bset_err(b, LBM_EINVAL, "bad candidate outputs");
    lbm_status st;
    if ((st = check_ready(b))) return st;
    if (!any_enabled(b)) return bset_err(b, LBM_ESTATE, "no item is enabled");
    if ((st = reset_state(b))) return st;
    int64_t pre = 0;
    if ((st = pre_steps(b, 2, &pre))) return st;
    std::vector<lbm_batch_config> list;
    for (int blk : {64, 128, 256}) list.push_back({LBM_BATCH_TILED, blk, 1, 64});
    for (int blk : {128, 256, 512})
        if (blk <= resident_limit(b->ks))
            for (int spl : {2, 8, 32}) list.push_back({LBM_BATCH_RESIDENT, blk, spl, 64});
    const lbm_batch_config keep = b->cfg;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return bset_err(b, LBM_EDEVICE, "event create");
    }
    std::vector<double> ms(list.size(), 0.0);
    const int64_t reps = std::max<int64_t>(1, (trial_steps + 63) / 64);
    for (size_t k = 0; k < list.size() && !st; ++k) {
        b->cfg = list[k];
        if ((st = build_tables(b, table_tile(b)))) break;
        if ((st = capture(b, 1, 0, 0.0))) break;
        // one untimed replay, then the timed ones
        if ((st = bhip(b, hipGraphLaunch(b->graph, b->stream), "graph launch"))) break;
        if ((st = bhip(b, hipEventRecord(e0, b->stream), "event record"))) break;
        for (int64_t r = 0; r < reps && !st; ++r) st = bhip(b, hipGraphLaunch(b->graph, b->stream), "graph launch");
        if (st || (st = bhip(b, hipEventRecord(e1, b->stream), "event record"))) break;
        if ((st = bhip(b, hipEventSynchronize(e1), "event sync"))) break;
        float el = 0.f;
        if ((st = bhip(b, hipEventElapsedTime(&el, e0, e1), "elapsed time"))) break;
        ms[k] = (double)el / (double)(reps * 64);
        advance(b, 64 * (reps + 1));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    drop_bgraph(b);
    b->tables_valid = false;
    after_batch_steps(b);
    if (st) {
        b->cfg = keep;
        return st;
    }
    size_t bi = 0;
    for (size_t k = 1; k < list.size(); ++k)
        if (ms[k] < ms[bi]) bi = k;
    b->cfg = list[bi];
    if (best) *best = list[bi];
    for (size_t k = 0; k < list.size() && (int32_t)k < cap; ++k) {
        cands[k] = list[k];
        ms_per_step[k] = ms[k];
    }
    if (n_out) *n_out = (int32_t)list.size();
    return LBM_OK;
}

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : "null batch"; }

void lbm_batch_destroy(lbm_batch* b) {
    if (!b) return;
    drop_bgraph(b);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    for (auto* c : b->items) {
        drop_graph(c);
        release_capture(c);
        delete c;
    }
    delete b;
}

}  // extern "C"
