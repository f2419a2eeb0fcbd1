// Host-side state of one lattice context and the helpers shared by the
// single-lattice entry points (lbm_host.cpp) and the batch (lbm_batch.cpp).
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"

namespace lbmh {

constexpr size_t kAlign = 256;
inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// padded grid: one halo node on each non-periodic axis
struct Pad {
    int NX, NY, NZ, hx, hy, hz;
    size_t nodes, plane;  // padded node count and the population plane stride
};

bool valid_params(const lbm_params* p, std::string* why);
Pad padding(const lbm_params* p);
size_t value_bytes(int storage);
size_t compute_bytes(int storage);
int total_planes(const lbm_params* p);
int scalar_comps(const lbm_params* p);   // scalar components (1 without several)
int moment_planes(const lbm_params* p);  // moment planes per parity: 8 + scalar components - 1
lbmi::KernelSet kernels_for(const lbm_params* p);
// device buffer sizes of one context (roles as in lbm.h)
void layout(const lbm_params* p, size_t n_links, size_t sz[LBM_NBUF]);

}  // namespace lbmh

struct lbm_ctx {
    lbm_params p;
    lbmh::Pad pad;
    lbmi::KernelSet ks;
    void* buf[LBM_NBUF];
    size_t size[LBM_NBUF];
    size_t cap_links = 0, n_links = 0;
    bool cmp_links = false;  // some link takes a comparison form (flag bit 3 or kind 8)
    hipStream_t stream = nullptr;
    int device = -1;  // HIP device current at creation
    int64_t t = 0, t_snap = 0;
    bool have_geometry = false, have_links = false, initialized = false, snap_valid = false;
    std::vector<uint8_t> mask;   // domain
    std::string err;
    // captured runs of steps (links ready), replayed by lbm_step on the
    // caller's stream: graph_steps steps from an even (run[0]) or odd (run[1])
    // time, and the last shorter run lbm_step needed (tail)
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        int parity = 0;
        int64_t steps = 0;
    };
    StepGraph run[2];
    StepGraph tail;
    hipStream_t capture_stream = nullptr;
    // lbm_set_step_overlap mode 1: a captured run overlaps each step's link
    // kernel with the previous sweep: the sweep runs as two launches over
    // 64-node waves (those that hold a link node A or its partner E, then the
    // rest) and the links of the next step, on a second stream, wait only
    // for the first
    hipStream_t capture_stream2 = nullptr;
    hipEvent_t ev_links = nullptr, ev_bnd = nullptr, ev_fork = nullptr, ev_join = nullptr;
    size_t n_wave_bnd = 0, n_wave_int = 0;  // wave lists after the flags (buffer 1)
    int overlap_mode = 0;                    // lbm_set_step_overlap
    bool graph_failed = false;
    int graph_steps = 64;
    // what lbm_step ran (lbm_step_stats): graph replays, steps inside them,
    // steps as single launches
    int64_t n_graph_launches = 0, n_graph_steps = 0, n_plain_steps = 0;
    // item of a batch: the batch owns the context and its buffers
    bool batch_owned = false;
};

namespace lbmh {

void drop_graph(lbm_ctx* c);
// destroys the capture streams and events of a context
void release_capture(lbm_ctx* c);
lbm_status set_err(lbm_ctx* c, lbm_status s, const std::string& m);
lbm_status hip_check(lbm_ctx* c, hipError_t e, const char* what);
lbmi::KArgs base_args(const lbm_ctx* c);
// device word holding the time at the start of a captured run (end of buffer 3)
uint32_t* time_base(const lbm_ctx* c);
// lbm_reduce's outputs from the 12 FP64 sums of the reduction (h[0..4] sums of
// rho, C, B; h[5..7] squared changes and h[8..10] squared norms of u, C - C0,
// B - B_ext; h[11] non-finite count); moves the residual snapshot time
lbm_status finish_reduce(lbm_ctx* c, const double h[12], double out[8]);

}  // namespace lbmh
