// Internal interface between the host side of liblbm (lbm_host.cpp) and the
// kernel instantiations (lbm_kernels_*.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbmi {

// per-node flags (one byte per padded node)
enum : uint8_t { NF_FLUID = 1, NF_LINKS = 2, NF_MOM = 4 };

// kernel modes of the observe kernel
enum : int { OBS_MOMENTS = 0, OBS_POPS = 1, OBS_REDUCE = 2, OBS_NORM = 3 };

// number of FP64 accumulators used by the reduction
constexpr int NACC = 16;

// Boundary link as the kernels read it: padded node indices, population
// planes, the lattice vector of alpha, wall data in the compute type R.
template <class R>
struct alignas(16) DevLink {
    uint32_t A;           // first fluid node
    uint32_t E, B;        // A + e_alpha and A - e_alpha (periodic wrap), fluid or not
    uint32_t mE;          // node whose moments stand for E: E if fluid, else A
    uint8_t kind;         // lbm_link_kind
    uint8_t flags;        // bit 0: u_w given; bit 1: E not fluid; bit 2: u_w cos(omega t') (oscillating);
                          // bit 3: the comparison form of the kind
    uint8_t pa, pap;      // population planes of alpha and of its opposite alpha'
    uint8_t field;        // 0 f, 1 h, 2 g
    uint8_t caxis;        // Cartesian axis of the magnetic component (g links)
    int8_t ex, ey, ez;    // e_alpha
    uint8_t need;         // bit q: the link's formula uses moment q (rho, u_x, u_y, u_z, C, B_x, B_y, B_z);
                          // bit 4 reads the moment plane cslot
    uint8_t cslot;        // moment plane of the link's scalar component: 4 (C_0), 8 (C_1), 9 (C_2)
    uint8_t pslot;        // FLUX with a bilinear term: moment planes of its components j (bits 0-3)
                          // and l (bits 4-7); 0: none
    R d;
    R value;  // given value minus its rest value (rho0, C0 or B_ext,k); FLUX with pslot: the
              // coefficient of the bilinear term (F_i += value C_j,X C_l,X)
    R a1, a3, weight, uw0, uw1, uw2;
    R quad;   // quadratic coefficient of the flux law (FLUX / MAG_FLUX)
};

// Launch description: sizes, pointers and physical parameters in double; the
// instantiation converts to the compute type.
struct KArgs {
    int NX, NY, NZ;        // padded extents
    int hx, hy, hz;        // halo widths (0 periodic, 1 otherwise)
    int n0, n1, n2;        // domain extents
    size_t plane;          // padded node count rounded up (population plane stride)
    size_t wave_fluid;     // offset in flags of one byte per 64 nodes (1 = all fluid)
    const uint32_t* waves; // sweep over a list of 64-node waves (sweep_waves): their indices
    uint32_t n_waves;
    void* S;               // populations [QT][plane]
    const uint8_t* flags;  // [plane]
    const void* links;     // DevLink<R>[n_links]
    void* M;               // R[2][MW][plane], MW = 8 + scalar components - 1
    size_t n_links;
    double tau_f, tau_c, tau_m, rho0, C0, mu;
    double tau_cs[2];      // relaxation times of scalar components 1, 2
    double wall_omega;     // angular frequency of oscillating boundary velocities (link flag bit 2)
    double Bext[3], accel[3], scale[3];
    int comp[3];           // Cartesian axis of each evolved magnetic component
    uint32_t* tbase;       // device word: the time at the start of a captured run (null: use tstep alone)
    uint32_t tstep;        // time of this step, counted from *tbase (or absolute without tbase)
    int parity;            // parity of the current time (t % 2)
    int links_ready;       // 0 at t = 0: populations are the initial state
    int cmp_links;         // some link takes a comparison form (flag bit 3 or kind 8)
    // observe / init
    int mode;              // OBS_*
    int field;             // OBS_POPS: 0 f, 1 h, 2 g; OBS_NORM: Cartesian axis
    double norm_u, norm_b; // scale: u /= norm_u, B - B_ext /= norm_u * norm_b
    void* out;             // OBS_MOMENTS: [MW][N] (out_f64 ? double : float); OBS_POPS: double
    int out_f64;
    double* acc;           // OBS_REDUCE: FP64 accumulators [NACC], or with acc_blocks the
                           // per-block records [blocks][NACC]
    int acc_blocks;        // OBS_REDUCE: 1 = each block stores its sums into its own record
                           // of acc (no atomics), 0 = FP64 atomics into acc[0..NACC)
    void* snap;            // OBS_REDUCE: R[MW - 1][plane] snapshot of u, C_0 - C0, B - B_ext, C_k - C0
    int snap_valid;
    const double *init_rho, *init_u, *init_C, *init_B;
    hipStream_t stream;
    hipEvent_t ev[3];      // optional: recorded before links, between, after sweep
};

using Launcher = hipError_t (*)(const KArgs&);

// status of one item of a batch
enum : uint32_t { BS_ACTIVE = 0, BS_STEADY = 1, BS_NONFINITE = 2, BS_DISABLED = 3 };

// Launch description of the batched kernels: the item descriptors, the
// per-launch work tables and the per-item convergence state, all on the
// device.
struct BArgs {
    const void* items;          // item descriptors, KernelSet::item_bytes each
    const uint32_t* tiles;      // node tiles: (item, first padded node) pairs
    uint32_t n_tiles, tile;     // tile = nodes per tile = threads per block
    const uint32_t* ltiles;     // link tiles: (item, first link) pairs, 256 links each
    uint32_t n_ltiles;
    const uint32_t* active;     // indices of the items a resident launch runs
    uint32_t n_active;
    uint32_t* status;           // BS_* per item
    uint32_t* steps;            // steps run per item since the counters were cleared
    double* resid;              // last steady-state residual per item (-1: none yet)
    uint32_t* snap_ok;          // per item: the residual snapshot holds a previous state
    int parity;                 // parity of the current time
    uint32_t tstep;             // time of the (first) step counted from each item's time base
    int nsteps;                 // resident launch: steps per launch (even)
    int block;                  // resident launch: threads per item
    int interval;               // steps between two residual evaluations
    double tol;                 // steady when the residual falls below it
    hipStream_t stream;
};

using BLauncher = hipError_t (*)(const BArgs&);
using Describer = size_t (*)(const KArgs&, void* out);

struct KernelSet {
    Launcher links = nullptr;    // the boundary-link kernel of a step (no-op at t = 0)
    Launcher sweep = nullptr;    // the fused sweep of a step
    Launcher sweep_waves = nullptr;  // the fused sweep over the waves listed in KArgs::waves
    Launcher step = nullptr;     // links then sweep
    Launcher observe = nullptr;  // moments / populations / reductions at the current time
    Launcher flux = nullptr;     // links of the current step with their FP64 net inflows by field
    Launcher scale = nullptr;    // OBS_NORM output [2][N] divided by norm_u and norm_u * norm_b
    Launcher init = nullptr;     // equilibrium initialisation
    Launcher set_time = nullptr; // *tbase = tstep
    Launcher tick = nullptr;     // *tbase += tstep
    int QT = 0;                  // population planes
    int MW = 8;                  // moment planes (8 + scalar components - 1)
    // batched items
    Describer describe = nullptr;  // writes one item descriptor from its launch description
    size_t item_bytes = 0;         // size of one item descriptor
    BLauncher b_sweep = nullptr;   // fused sweep over node tiles of many items
    BLauncher b_links = nullptr;   // boundary links over link tiles of many items
    BLauncher b_resident = nullptr;  // one workgroup per item, nsteps steps per launch
    BLauncher b_reduce = nullptr;  // links, then per-item FP64 sums over node tiles
    BLauncher b_judge = nullptr;   // per-item residual, steady / non-finite flags
    BLauncher b_clear = nullptr;   // zero the per-item accumulators and counters
    BLauncher b_set_time = nullptr;  // every item's time base = its time when described
    BLauncher b_tick = nullptr;    // time bases of the listed items += tstep
};

// storage codes as in lbm.h
KernelSet kernels_f64(int fl, int sl, int ml, int nc, int ns);
KernelSet kernels_f32(int fl, int sl, int ml, int nc, int ns);
KernelSet kernels_f16(int fl, int sl, int ml, int nc, int ns);
KernelSet kernels_bf16(int fl, int sl, int ml, int nc, int ns);

}  // namespace lbmi
