/*
 * lbm.h - C ABI of the fused coupled lattice Boltzmann sweep for MI355X (gfx950).
 *
 * One step advances three coupled lattices on a regular grid:
 *   f  flow, BGK (Eqs. 1-2), D2Q9 or D3Q19, with a body force and the Lorentz
 *      force J x B;
 *   h  convection-diffusion scalar C (Eqs. 3-4), D2Q5 or D3Q7, for one to
 *      three scalar components C_0, C_1, C_2, one lattice each, whose flux
 *      walls may react with each other (Section 4.2.2);
 *   g  vector-valued magnetic distributions for B (Eqs. 5-6), D2Q5 or D3Q7,
 *      one distribution per evolved Cartesian component of B;
 * and, in the same sweep, the boundary-link updates of Sections 3-4:
 * pair-wise moment conservation for a given velocity, pressure, concentration
 * or magnetic component (Eqs. 15-16, 19-20, 34-35, 43-44), the flux-increment
 * M scheme for Robin reactions and Shercliff thin walls (Eqs. 17, 23, 25-27,
 * 30-32), the moving-wall correction (Eq. 24), zero-gradient bounce-back
 * (Eqs. 21-22) and the extrapolation of unknown moments (Eq. 13), for any
 * boundary-to-node distance d in (0, 1].
 *
 * Units: lattice units, dx = dt = 1.  nu = (tau_f - 1/2)/3,
 * D = (tau_c - 1/2)/4, eta = (tau_m - 1/2)/4.
 *
 * Conventions for every entry point:
 *  - Return value: LBM_OK (0) or a negative lbm_status.  Inputs are validated
 *    before any work is queued, so a call that fails has no effect.  The text
 *    of the last error of a context is lbm_last_error(ctx).
 *  - Memory: every device buffer is allocated and owned by the caller (the
 *    library never frees caller memory and allocates no device memory); the
 *    library owns only its host-side context.  "dev" pointers are device
 *    pointers, "host" pointers are host pointers.
 *  - Streams: all device work of a context is queued on the hipStream_t given
 *    at creation (or lbm_set_stream).  lbm_reduce and lbm_save synchronise
 *    that stream; everything else is asynchronous.  Asynchronous device errors
 *    are reported by the next synchronising call.
 *  - Threads: a context is not thread-safe; use one context per stream.
 *  - Node indices: a node of the fluid domain (n[0] x n[1] x n[2] nodes) has
 *    the linear index x + n[0]*(y + n[1]*z); 2D domains have n[2] = 1.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument */
    LBM_ESIZE = -2,      /* a buffer or table is too small */
    LBM_EDEVICE = -3,    /* HIP runtime error */
    LBM_EUNSTABLE = -4,  /* non-finite values found by lbm_reduce */
    LBM_ESTATE = -5      /* call out of order (e.g. lbm_step before lbm_init) */
} lbm_status;

typedef enum { LBM_NONE = 0, LBM_D2Q9 = 1, LBM_D3Q19 = 2, LBM_D2Q5 = 3, LBM_D3Q7 = 4 } lbm_lattice;

/* Storage of the populations.  F16 and BF16 hold the deviation from the rest
 * equilibrium (w_a rho0, w_a C0, w_a B_ext,k) times store_scale; arithmetic is
 * then FP32.  F32 also stores deviations.  F64 stores deviations and computes
 * in FP64. */
typedef enum { LBM_F64 = 1, LBM_F32 = 2, LBM_F16 = 3, LBM_BF16 = 4 } lbm_storage;

/* Boundary-link kinds (Sections 3-4). */
typedef enum {
    LBM_LK_VEL = 1,      /* given velocity u_w: Eqs. 15-16 (d < 0.5), Eq. 43 (d >= 0.5) */
    LBM_LK_PRES = 2,     /* given density: zeroth-moment pair (d < 0.5), Eq. 44 (d >= 0.5) */
    LBM_LK_CONC = 3,     /* given concentration: Eqs. 19-20 */
    LBM_LK_FLUX = 4,     /* scalar flux F(C) = a1 C_X + quad C_X^2 - a3, M scheme: Eqs. 23-27 */
    LBM_LK_BB0 = 5,      /* zero normal gradient, static: Eqs. 21-22 */
    LBM_LK_MAG_DIR = 6,  /* given magnetic component B_k: Eqs. 34-35 */
    LBM_LK_MAG_FLUX = 7, /* magnetic flux F(B_k) = a1 B_X,k + quad B_X,k^2 - a3 (Shercliff, Eq. 30),
                            M scheme */
    LBM_LK_MAG_THETA = 8 /* comparison scheme: the link-based theta form of Eq. 39 (d = 0.5)
                            and Eq. 40 (d = 1) for a magnetic component.  The bounced
                            value x becomes ((theta - 1) x + theta dg_move) / (theta + 1),
                            theta = a1 >= 0 (Section 4.3: c_w H / (tau_m - 1/2));
                            combined as Eq. 43 for d >= 0.5 and applied to the Y value
                            of Eq. 35 for d < 0.5 */
} lbm_link_kind;

#define LBM_NBUF 8

typedef struct {
    int32_t dim;          /* 2 or 3 */
    int32_t n[3];         /* fluid-domain node counts (n[2] = 1 in 2D) */
    int32_t periodic[3];  /* 1 = periodic axis (2D: periodic[2] must be 1) */
    int32_t fluid;        /* LBM_D2Q9 (2D) or LBM_D3Q19 (3D) */
    int32_t scalar;       /* LBM_NONE, LBM_D2Q5 (2D) or LBM_D3Q7 (3D) */
    int32_t magnetic;     /* LBM_NONE, LBM_D2Q5 (2D), LBM_D3Q7 (3D), or LBM_D3Q19 (3D, one
                             component, no scalar lattice, c_g^2 = 1/3: the richer magnetic
                             lattice Section 6.1 suggests for conducting walls; every link
                             kind but LBM_LK_MAG_THETA) */
    int32_t mag_ncomp;    /* evolved B components: 0 (no magnetic lattice), 1..3 */
    int32_t mag_comp[3];  /* Cartesian axis (0..2) of each evolved component */
    int32_t storage;      /* lbm_storage */
    int32_t scalar_ncomp; /* scalar components (Section 4.2.2), one scalar lattice each: 0 or 1 =
                             one component C_0; 2 or 3 with a scalar lattice and no magnetic
                             lattice.  Component k relaxes with tau_c (k = 0) or tau_cs[k - 1];
                             all share the rest value C0 and the flow field */
    double tau_f, tau_c, tau_m;  /* relaxation times (> 1/2) */
    double rho0, C0, mu;         /* rest density, rest concentration, permeability */
    double B_ext[3];             /* applied field; non-evolved components stay at B_ext */
    double accel[3];             /* body force per unit mass */
    double store_scale[3];       /* F16/BF16: power-of-two scale of f, h, g deviations */
    double wall_omega;           /* angular frequency (rad per step) of oscillating boundary velocities */
    double tau_cs[2];            /* relaxation times of scalar components 1 and 2 (> 1/2 when present) */
} lbm_params;

/* One boundary link: the population entering fluid node A along e_alpha, whose
 * source node A - e_alpha lies beyond a boundary.  For a magnetic link, comp is
 * the slot (0..mag_ncomp-1) of the evolved component; for a scalar link, the
 * scalar component (0..scalar_ncomp-1). */
typedef struct {
    uint32_t node;   /* fluid node A (domain linear index) */
    uint32_t enode;  /* second fluid node E = A + e_alpha; ignored when flags bit 1 is set */
    uint8_t field;   /* 0 = f, 1 = h, 2 = g */
    uint8_t dir;     /* unknown direction alpha (lattice numbering, see lbm_lattice_table) */
    uint8_t kind;    /* lbm_link_kind */
    uint8_t comp;    /* magnetic slot or scalar component */
    uint8_t flags;   /* bit 0: u_w is the boundary velocity (else extrapolated, Eq. 13);
                        bit 1: E is not fluid, A stands in for E;
                        bit 2 (with bit 0): the boundary velocity oscillates,
                        u_w cos(wall_omega t'), evaluated at the time t' the
                        bounced population meets the boundary: t' = t - d for
                        the value entering A at time t (Section 4.1, the
                        arrival time between t - 1 and t; Eq. 45);
                        bit 3: the comparison form of Section 5 instead of the
                        method's: VEL and PRES take the extrapolated form
                        (Eqs. 15-16 and the pressure pair form) at every d, the
                        form Section 5.1 finds unstable beyond d of about 0.8;
                        FLUX and MAG_FLUX add the flux at X instead of M (Eq. 33,
                        and Y + flux + correction for d < 0.5).  Other kinds:
                        LBM_EINVAL */
    uint8_t cross_comp[2]; /* FLUX with cross != 0: the scalar components j, l of the bilinear term */
    uint8_t pad;
    double d;        /* boundary-to-node distance |AX| / |AE| in (0, 1] */
    double value;    /* PRES: rho_w; CONC: C_w; MAG_DIR: B_k */
    double a1, a3;   /* FLUX / MAG_FLUX: F(phi) = a1 phi_X - a3 (lattice units; Eq. 17 with a2 = D);
                        MAG_THETA: a1 = theta = c_w H / (tau_m - 1/2) (Eqs. 39-40), a3 = 0 */
    double weight;   /* flux share of this link (Eq. 48): on flat walls 1 / (links crossing the wall per
                        node: 1 on D2Q5 / D3Q7, 5 on D3Q19); on curved walls S_i e.n / sum e.n over
                        the links of the outer-layer node B_i */
    double u_w[3];   /* boundary velocity */
    double quad;     /* FLUX / MAG_FLUX: quadratic term of the flux law, F(phi) = a1 phi_X + quad phi_X^2
                        - a3, evaluated explicitly from the extrapolated phi_X (Eq. 13; a nonlinear
                        surface reaction, Section 4.2.2); 0 for the other kinds (else LBM_EINVAL).
                        (Eq. 17's own a2 is the coefficient of the normal derivative, D here.) */
    double cross;    /* FLUX of one of several scalar components i = comp: F_i gains cross C_j,X C_l,X with
                        (j, l) = cross_comp (any components, i included), each C_X extrapolated by Eq. 13
                        like C_i,X: a surface reaction between components (Section 4.2.2; A + B -> P
                        consumes A and B at the rate k C_A C_B and produces P), with no iteration between
                        them; 0 for the other kinds and with one scalar component (else LBM_EINVAL) */
} lbm_link;

/* How a boundary states the flux law of a FLUX or MAG_FLUX condition, or the
 * theta of MAG_THETA.  lbm_build_links forms each link's coefficients
 * (lbm_link.a1, a3, quad) from it, with the field's own transport
 * coefficient: D = c_h^2 (tau_c - 1/2) for h, eta = c_g^2 (tau_m - 1/2) for g
 * (c^2 = 1/4 on D2Q5 / D3Q7, 1/3 on D3Q19). */
typedef enum {
    LBM_LAW_COEF = 0,      /* F(phi) = a1 phi_X + quad phi_X^2 - a3 with the given a1, quad, a3
                              (Eq. 17 with a2 = D; the quadratic term: Section 4.2.2) */
    LBM_LAW_ROBIN = 1,     /* d phi / dn = k phi with n into the fluid (Eq. 17 with a2 = D):
                              F = -k D phi, i.e. a1 = -k D, a3 = 0; FLUX only */
    LBM_LAW_REACTION = 2,  /* first-order surface reaction F = -k (phi - phi_eq) (Section 5.3):
                              a1 = -k, a3 = -k phi_eq; FLUX only */
    LBM_LAW_SHERCLIFF = 3  /* thin conducting wall (Eq. 30) for the component B_k:
                              F = -eta (B_X,k - B_ext,k) / (c_w H), i.e. a1 = -eta / (c_w H),
                              a3 = a1 B_ext,k; c_w = +inf is the perfectly conducting wall (F = 0).
                              MAG_THETA: theta = c_w H / (tau_m - 1/2) (Eqs. 39-40).
                              MAG_FLUX and MAG_THETA only; c_w > 0, H > 0 */
} lbm_flux_law;

/* Boundary description consumed by lbm_build_links. */
typedef struct {
    int32_t kind;          /* lbm_link_kind, 0 = no condition for this lattice */
    int32_t u_given;       /* 1: use the boundary velocity; 0: extrapolate u (Eq. 13) */
    int32_t profile_axis;  /* axis of profile */
    int32_t profile_len;   /* 0 = no profile */
    int32_t alt;           /* 1: the comparison form of the kind (link flag bit 3); only for
                              VEL, PRES, FLUX and MAG_FLUX, else LBM_EINVAL */
    int32_t law;           /* lbm_flux_law of a FLUX, MAG_FLUX or MAG_THETA condition; must be
                              LBM_LAW_COEF (0) for the other kinds (else LBM_EINVAL) */
    double value;          /* PRES: rho_w; CONC: C_w; MAG_DIR: B_k */
    double a1, a3, quad;   /* LBM_LAW_COEF: the flux law's coefficients (MAG_THETA: a1 = theta);
                              other laws: ignored */
    const double* profile; /* host, or NULL: per coordinate of A along profile_axis, the value that
                              replaces a1 (LBM_LAW_COEF) or k (LBM_LAW_ROBIN, LBM_LAW_REACTION) */
    double k;              /* LBM_LAW_ROBIN, LBM_LAW_REACTION: the rate k (>= 0) */
    double phi_eq;         /* LBM_LAW_REACTION: equilibrium value of the reacting field */
    double c_w, H;         /* LBM_LAW_SHERCLIFF: wall conductance ratio (> 0, may be +inf) and the
                              length scale of Eq. 30 (> 0): the channel half-width or pipe radius */
    int32_t cross_comp[2]; /* FLUX, LBM_LAW_COEF, several scalar components: the components j, l
                              (0..scalar_ncomp-1) of the bilinear term */
    double cross;          /* its coefficient: F_i += cross C_j,X C_l,X (lbm_link.cross); 0 = none */
} lbm_bc;

typedef struct {
    int32_t type;     /* 0 = plane, 1 = cylinder, 2 = box */
    int32_t axis;     /* plane: normal axis; cylinder: its axis */
    int32_t side;     /* plane: 0 below node 0, 1 above node n-1 */
    int32_t is_open;  /* open boundary (inlet/outlet): loses corner ties to walls */
    double q;         /* plane: distance of the plane outside the first/last node layer */
    double center[3]; /* cylinder centre (axis coordinate ignored) */
    double radius;    /* cylinder radius; nodes strictly inside are fluid */
    double u_w[3];    /* boundary velocity */
    lbm_bc f, h, g[3];
    int32_t u_osc;    /* 1: the boundary velocity is u_w cos(wall_omega t') (link flag bit 2) */
    int32_t reserved;
    double d_scheme;  /* 0: each link uses the distance d measured from the geometry. In (0, 1]:
                         every link of this boundary uses this d in its update instead (the
                         deliberate layout/scheme mismatch of Section 5.2, e.g. the d = 0.5
                         scheme on walls that sit on the nodes, d = 1). Other values: LBM_EINVAL */
    double lo[3], hi[3]; /* box: the closed solid block lo <= x <= hi in node coordinates;
                            bounds may be infinite, lo[k] <= hi[k] (else LBM_EINVAL).
                            Nodes inside or on a face are solid; a link's d is where
                            it enters the block (walls of voxel geometries, e.g. a
                            channel between reservoirs, Section 5.1).  Along a
                            periodic axis a box must be unbounded or stay clear of
                            the domain's ends. */
    lbm_bc h_more[2]; /* conditions of scalar components 1 and 2 (h is component 0's); each must
                         have a kind exactly when h has one */
} lbm_boundary;

typedef struct lbm_ctx lbm_ctx;

/* Library version string. */
const char* lbm_version(void);

/* Lattice tables of the library: Q, e (Q x 3, row-major), w (Q), c^2 and the
 * opposite direction of each direction.  e, w, opp hold at least 19 entries. */
lbm_status lbm_lattice_table(int32_t lattice, int32_t* Q, int32_t* e, double* w, double* c2,
                             int32_t* opp);

/* Host-side geometry and link-table builder (Sections 3, 4 and 6).
 * Node classification: a node is fluid iff it lies strictly inside every
 * cylinder; planes lie outside the node range.  For every fluid node A and
 * every direction alpha of every lattice whose source A - e_alpha is not a
 * fluid node of the domain, one link (one per magnetic component) is made
 * with the crossed boundary's condition: d is q for a plane and the exact
 * ray-circle intersection for a cylinder (Section 6, per node and per
 * direction).  A link crossing several boundaries takes a wall before an open
 * boundary, then the smaller d, then the lower boundary index.  Flux links on
 * a cylinder get the surface-segment split weights of Section 6.2 / Eq. 48.
 *   p, bnds[nb]: host inputs; mask_out: host, n[0]*n[1]*n[2] bytes (1 = fluid)
 *   or NULL; links_out: host array of cap links or NULL (then only *n_out is
 *   set); n_out: number of links.  Links are ordered by node, field, comp, dir.
 * Errors: LBM_EINVAL (bad parameters, a link with no boundary condition),
 *   LBM_ESIZE (cap too small; *n_out holds the size needed). */
lbm_status lbm_build_links(const lbm_params* p, const lbm_boundary* bnds, int32_t nb,
                           uint8_t* mask_out, lbm_link* links_out, size_t cap, size_t* n_out);

/* Sizes (bytes) of the LBM_NBUF device buffers a context needs for n_links
 * links; returns their sum, 0 on invalid parameters.  Buffer roles:
 *  0 populations (AA layout, in place; boundary-link values are written into
 *    the slots the next sweep gathers them from), 1 node flags, 2 link
 *  records, 3 moment planes of the link nodes (two parities), 4 residual
 *  snapshot and FP64 accumulators; 5-7 are unused (size 0, may be NULL). */
size_t lbm_required_bytes(const lbm_params* p, size_t n_links, size_t sizes_out[LBM_NBUF]);

/* Creates a context over caller-allocated device buffers dev_bufs[i] of at
 * least sizes_out[i] bytes (256-byte aligned), working on hip_stream (a
 * hipStream_t, NULL = default stream).  The device is the current HIP device. */
lbm_status lbm_create(const lbm_params* p, size_t n_links, void* const dev_bufs[LBM_NBUF],
                      void* hip_stream, lbm_ctx** out);

/* Node classification, host array of n[0]*n[1]*n[2] bytes (nonzero = fluid). */
lbm_status lbm_set_geometry(lbm_ctx* ctx, const uint8_t* host_mask);

/* Validates the host link table against the geometry (every unknown
 * population of every fluid node has exactly one link; d in (0,1]; kinds
 * allowed for the field) and uploads it.  n must not exceed the n_links of
 * lbm_create.  Resets the time to 0 and requires lbm_init again. */
lbm_status lbm_set_links(lbm_ctx* ctx, const lbm_link* host_links, size_t n);

/* Equilibrium initialisation (Eqs. 2, 4, 6) from device FP64 fields in domain
 * layout: rho [N], u [3][N], C [scalar components][N], B [3][N] (N = domain
 * nodes); any may be NULL for the uniform rest value (rho0, 0, C0, B_ext).
 * Sets time 0. */
lbm_status lbm_init(lbm_ctx* ctx, const double* dev_rho, const double* dev_u, const double* dev_C,
                    const double* dev_B);

/* Advances n >= 0 steps (asynchronous).  One step is the boundary-link
 * update followed by the fused stream-collide sweep (Sections 2-4).  The
 * first step after lbm_init is launched singly; after that the steps run as
 * replays of captured HIP graphs: runs of 64 steps while they fit, then one
 * run of the rest (a single remaining step is launched singly).  A graph is
 * captured the first time a run of its start parity and length is needed;
 * the runs of 64 and the last shorter run are kept for replay. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/* Captures, without running anything, the graphs that lbm_step(ctx, n) would
 * replay from the current time, so that a later lbm_step(n) spends no time in
 * capture (e.g. before a timed region).  Synchronous on the host. */
lbm_status lbm_step_prepare(lbm_ctx* ctx, int64_t n);

/* What lbm_step has run since lbm_create, host outputs: out[0] graph
 * replays, out[1] steps run inside them, out[2] steps launched singly. */
lbm_status lbm_step_stats(const lbm_ctx* ctx, int64_t out[3]);

/* How a captured run orders the kernels of its steps.  mode 0 (the
 * default): the link kernel, then the whole sweep, per step.  mode 1
 * (overlap): the sweep of each step runs as two launches, first over the
 * 64-node waves that hold a link node A or its partner E = A + e_alpha, then
 * over the other waves with fluid nodes, and the link kernel of the next step
 * runs on a second captured stream beside the second launch.  It reads only
 * slots that threads of A and E write and writes only slots no sweep thread
 * touches (Section 3's link updates read the post-collision populations of A
 * and E and set the one that enters A), so the states are those of mode 0.
 * Mode 1 pays on lattices with millions of links and costs time on small
 * ones (the graph's cross-stream dependencies).  Drops captured runs.
 * Errors: LBM_EINVAL for another mode. */
lbm_status lbm_set_step_overlap(lbm_ctx* ctx, int32_t mode);

/* Durations of the two kernels of a step, for measurement: n (even, 2 to
 * 4096) launches of the boundary-link kernel back to back, captured in one
 * HIP graph and timed with HIP events on the context's stream, then n
 * launches of the fused sweep the same way (parities alternating from the
 * context's time).  Returns the mean duration per launch in ms in ms_out[0]
 * (links; 0 without links) and ms_out[1] (sweep).  These launches are not
 * steps: the populations and moments are copied into the caller's device
 * buffer dev_scratch (scratch_bytes >= lbm_timing_scratch_bytes(ctx), else
 * LBM_ESIZE) first and restored from it afterwards, so the state and the
 * time are unchanged.  Allocates no device memory.  Synchronises the stream.
 * Not for items of a batch. */
size_t lbm_timing_scratch_bytes(const lbm_ctx* ctx);
lbm_status lbm_step_timed(lbm_ctx* ctx, int64_t n, void* dev_scratch, size_t scratch_bytes, float ms_out[2]);

/* Moments at the current time into dev_out, SoA [7 + m][N] of rho, u_x, u_y,
 * u_z, C_0, B_x, B_y, B_z, then C_1 .. C_{m-1} of m >= 2 scalar components
 * (m = max(scalar_ncomp, 1); 0 at solid nodes); out_type LBM_F64 or
 * LBM_F32. */
lbm_status lbm_read_moments(lbm_ctx* ctx, void* dev_out, int32_t out_type);

/* Populations of one field at the current time (after the boundary links),
 * FP64 into dev_out as [slots][N]: f: Q planes; h: m*Q planes of the m
 * scalar components; g: ncomp*Q planes (component-major).  Solid nodes
 * hold 0. */
lbm_status lbm_read_populations(lbm_ctx* ctx, int32_t field, double* dev_out);

/* FP64 reductions at the current time, synchronising the stream:
 * out[0] steady-state residual: max over u, C - C0 (all scalar components
 *        together) and B - B_ext of
 *        ||phi(t) - phi(t0)||_2 / ((t - t0) max(||phi(t)||_2, 1e-30)), where t0
 *        is the time of the previous lbm_reduce (-1 on the first call);
 * out[1] total mass sum(rho); out[2] sum(C_0); out[3..5] sum(B);
 * out[6] t - t0; out[7] number of non-finite moments.
 * Returns LBM_EUNSTABLE when out[7] > 0. */
lbm_status lbm_reduce(lbm_ctx* ctx, double out[8]);

/* lbm_reduce for callers that cannot allocate device memory (code under HIP
 * graph capture of its neighbours, serving loops, harnesses that forbid
 * hipMalloc): the same outputs, return values and snapshot update as
 * lbm_reduce, but the reduction's scratch (one record of FP64 sums per
 * 256-node block, then their totals) lives in a device array the library
 * owns, sized for at most LBM_REDUCE_STATIC_MAX_BLOCKS blocks, i.e. lattices
 * of up to 256 * LBM_REDUCE_STATIC_MAX_BLOCKS padded nodes (16 MiB per
 * device, held until the process ends); larger lattices fail with LBM_ESIZE.
 * The records are added in a fixed order, so the sums are reproducible run to
 * run (lbm_reduce adds them with atomics and may differ in the last bits).
 * The context's device must be the current HIP device (else LBM_EINVAL).
 * Allocates no device memory.  Every call on one device shares that device's
 * array: calls that overlap in time on one device (other host threads,
 * other streams) race and must be serialised by the caller.  Synchronises
 * the stream. */
#define LBM_REDUCE_STATIC_MAX_BLOCKS 131072
lbm_status lbm_reduce_static(lbm_ctx* ctx, double out[8]);

/* The dimensionless fields of Eqs. 46-47 along one Cartesian axis (0..2),
 * FP64 into dev_out as [2][N]: u* = u_axis / U and
 * B* = (B_axis - B_ext,axis) / (U mu sqrt(rho0 nu sigma)), with
 * sigma = 1 / (mu eta) in lattice units; 0 at solid nodes.  U > 0 is the
 * velocity scale (Eq. 46: the wall speed); U = 0 takes the mean of u_axis
 * over the fluid nodes (Eq. 47: the mean flow velocity), which synchronises
 * the stream and fails with LBM_EINVAL when that mean is zero. */
lbm_status lbm_read_normalised(lbm_ctx* ctx, int32_t axis, double U, double* dev_out);

/* FP64 net inflow through the boundary links over the last step, by field:
 * out[0] f (mass), out[1] h (solute C_0), out[2..4] g (B_x, B_y, B_z).  A link
 * (A, alpha) adds the value it sets, f_alpha(A) at the current time (the
 * link updates of Sections 3-4), minus the post-collision population that A
 * sent toward the wall in the step before, f*_alpha'(A).  Collision and
 * streaming conserve each field's total, so the change of sum(rho), sum(C)
 * and sum(B_k) over a step (lbm_reduce) equals these sums, up to rounding.
 * The links of the current step are written as lbm_step would write them
 * (the state is otherwise unchanged).  Synchronises the stream.
 * LBM_ESTATE before the first step. */
lbm_status lbm_boundary_flux(lbm_ctx* ctx, double out[5]);

/* lbm_boundary_flux for every scalar component (Section 4.2.2): out[k] is the
 * net inflow of C_k through the h links over the last step, k < m (the
 * scalar components; out[k] = 0 beyond).  out[0] equals lbm_boundary_flux's
 * out[1].  Collision and streaming conserve each component's total, so the
 * change of sum(C_k) over a step equals out[k], up to rounding.  Same
 * conditions and side effects as lbm_boundary_flux. */
lbm_status lbm_boundary_flux_scalar(lbm_ctx* ctx, double out[3]);

/* Checkpoint: lbm_state_bytes() bytes of host memory hold the populations,
 * moment planes and time.  lbm_save synchronises the stream. */
size_t lbm_state_bytes(const lbm_ctx* ctx);
lbm_status lbm_save(lbm_ctx* ctx, void* host);
lbm_status lbm_load(lbm_ctx* ctx, const void* host);

/* Measurement utility (not a step of the method): the bandwidth a plain
 * streaming kernel attains on the current device, the ceiling against which
 * the sweep's share of the HBM peak is read.  kind 0 reads `bytes` from
 * dev_src (dev_dst: a 16-byte device word the kernel may write), 1 writes
 * `bytes` to dev_dst, 2 copies `bytes` from dev_src to dev_dst (not
 * overlapping).  16-byte accesses, consecutive threads on consecutive words,
 * each thread per_thread (1..1024) words at a grid stride; 256-thread blocks.
 * One untimed launch, then reps launches back to back on hip_stream between
 * two HIP events: *ms_out = mean duration per launch.  bytes a nonzero
 * multiple of 16, pointers 16-byte aligned (else LBM_EINVAL).  Synchronises
 * the stream. */
lbm_status lbm_stream_bandwidth(int32_t kind, const void* dev_src, void* dev_dst, size_t bytes, int32_t per_thread,
                                int32_t reps, void* hip_stream, float* ms_out);

int64_t lbm_time(const lbm_ctx* ctx);
lbm_status lbm_set_stream(lbm_ctx* ctx, void* hip_stream);
const char* lbm_last_error(const lbm_ctx* ctx);
void lbm_destroy(lbm_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Batches: many independent lattices ("items"), each with its own size,
 * geometry, boundary links and parameters, advanced together by shared
 * launches.  Every item runs the same step as a single context (the same
 * node update and link update), so an item evolves exactly as it would
 * alone.  All items of a batch use one lattice combination (dim, fluid,
 * scalar, magnetic, mag_ncomp) and one storage format.
 *
 * Execution modes (lbm_batch_config.mode):
 *  LBM_BATCH_TILED    one step = one boundary-link launch over link tiles of
 *                     all active items, then one sweep launch over node tiles
 *                     (block nodes each) of all active items;
 *  LBM_BATCH_RESIDENT one workgroup of `block` threads per active item runs
 *                     steps_per_launch steps inside one launch, separating the
 *                     link and sweep phases with workgroup barriers (items
 *                     never exchange data, so no grid-wide synchronisation).
 * Runs of graph_steps steps are captured once in a HIP graph and replayed.
 * Steady-state detection (lbm_batch_run) evaluates every item's residual on
 * the device every `interval` steps, in FP64, with the definition of
 * lbm_reduce out[0]; an item whose residual falls below tol, or whose moments
 * turn non-finite, is frozen by a per-item flag that every later launch reads,
 * and the host drops frozen items from the work tables.
 * --------------------------------------------------------------------------- */
typedef struct lbm_batch lbm_batch;

typedef enum { LBM_BATCH_TILED = 1, LBM_BATCH_RESIDENT = 2 } lbm_batch_mode;

/* per-item state reported by lbm_batch_run */
typedef enum { LBM_ITEM_ACTIVE = 0, LBM_ITEM_STEADY = 1, LBM_ITEM_NONFINITE = 2, LBM_ITEM_DISABLED = 3 } lbm_item_status;

typedef struct {
    int32_t mode;              /* lbm_batch_mode */
    int32_t block;             /* TILED: nodes per tile = threads per block, 64, 128 or 256;
                                  RESIDENT: threads per item, a multiple of 64 up to 512 */
    int32_t steps_per_launch;  /* RESIDENT: even, >= 2; TILED: 1 */
    int32_t graph_steps;       /* steps per captured graph: even, a multiple of steps_per_launch */
} lbm_batch_config;

/* Device buffer sizes of a batch of n_items items with parameters items[i]
 * and link capacities n_links[i] (host arrays).  Returns the sum, 0 when an
 * item's parameters are invalid or the items do not share a lattice
 * combination and storage.  Buffer roles: 0-4 the items' buffers 0-4 of
 * lbm_required_bytes back to back; 5 item descriptors; 6 work tables; 7
 * per-item convergence state. */
size_t lbm_batch_required_bytes(int32_t n_items, const lbm_params* items, const size_t* n_links,
                                size_t sizes_out[LBM_NBUF]);

/* Creates a batch over caller-allocated device buffers (256-byte aligned,
 * sizes from lbm_batch_required_bytes) on hip_stream.  The default
 * configuration is TILED, block 256, graph_steps 64. */
lbm_status lbm_batch_create(int32_t n_items, const lbm_params* items, const size_t* n_links,
                            void* const dev_bufs[LBM_NBUF], void* hip_stream, lbm_batch** out);

/* The context of item i (owned by the batch: lbm_destroy ignores it and
 * lbm_set_stream refuses it).  Set it up with lbm_set_geometry,
 * lbm_set_links and lbm_init; read it with lbm_read_moments,
 * lbm_read_populations, lbm_reduce, lbm_save; it may also be stepped alone
 * with lbm_step.  NULL when i is out of range. */
lbm_ctx* lbm_batch_item(lbm_batch* b, int32_t i);

/* Selects the items that take part in lbm_batch_step, lbm_batch_run and
 * lbm_batch_tune (host array of n_items bytes, nonzero = take part; all items
 * do after creation).  The others keep their state and time, and lbm_batch_run
 * reports them as LBM_ITEM_DISABLED. */
lbm_status lbm_batch_set_active(lbm_batch* b, const uint8_t* host_flags);

lbm_status lbm_batch_configure(lbm_batch* b, const lbm_batch_config* cfg);
lbm_status lbm_batch_get_config(const lbm_batch* b, lbm_batch_config* cfg);

/* Advances every enabled item by n >= 0 steps (asynchronous).  Every enabled
 * item must be initialised and their times must have equal parity. */
lbm_status lbm_batch_step(lbm_batch* b, int64_t n);

/* Runs every item until its residual (every `interval` steps, interval even
 * >= 2) is below tol, its moments are non-finite, or max_steps steps have
 * run; synchronises.  Host outputs, n_items entries each, may be NULL:
 * steps_out steps run by the item in this call, resid_out its last residual
 * (-1 if none was evaluated), status_out its lbm_item_status.  Each item's
 * time advances by its own step count.  At most two single steps run first
 * when an item is at time 0 or the times are odd. */
lbm_status lbm_batch_run(lbm_batch* b, double tol, int32_t interval, int64_t max_steps, int64_t* steps_out,
                         double* resid_out, int32_t* status_out);

/* Autotuner: times every candidate configuration (TILED with block 64, 128,
 * 256; RESIDENT with block 128, 256, 512 and steps_per_launch 2, 8, 32) on
 * trial_steps real steps of the batch (the items advance), with HIP events on
 * the batch's stream, and configures the fastest.  Host outputs: best (may be NULL); cands and ms_per_step (cap
 * entries each, may be NULL) every candidate and its time per step; *n_out
 * the number of candidates. */
lbm_status lbm_batch_tune(lbm_batch* b, int64_t trial_steps, lbm_batch_config* best, lbm_batch_config* cands,
                          double* ms_per_step, int32_t cap, int32_t* n_out);

const char* lbm_batch_last_error(const lbm_batch* b);
void lbm_batch_destroy(lbm_batch* b);

/* ---------------------------------------------------------------------------
 * Warm-start network: a three-level convolutional encoder-decoder mapping
 * per-node geometry and parameter maps of a cross-section (fluid mask, wall
 * distance, Hartmann number, wall conductance) to its steady fields (scaled
 * axial velocity and induced field), used to initialise a lattice through
 * lbm_init.  The lattice update always runs to convergence from that state,
 * so the network only changes where the iteration starts.
 *
 * Layers (w = width, S = size, all 3x3 convolutions with ReLU, zero padding):
 *   e1: in_ch -> w -> w        at S          (skip 1)
 *   2x2 average pooling
 *   e2: w -> 2w -> 2w          at S/2        (skip 2)
 *   2x2 average pooling
 *   e3: 2w -> 4w -> 4w         at S/4
 *   nearest x2 upsampling, concatenated with skip 2 (6w channels)
 *   d2: 6w -> 2w -> 2w         at S/2
 *   nearest x2 upsampling, concatenated with skip 1 (3w channels)
 *   d1: 3w -> w -> w           at S
 *   head: 1x1 convolution w -> out_ch, linear.
 * Parameters, FP32, in this layer order: W[c_out][c_in][ky][kx] then b[c_out]
 * per layer (w = 32, in_ch = 4, out_ch = 2: 471,874 parameters).
 * Convolutions, their input gradients and weight gradients run on the matrix
 * cores: BF16 activations and weights with FP32 accumulation (precision
 * LBM_BF16), or FP32 throughout (LBM_F32, for gradient checks).  Adam keeps
 * FP32 master weights and moments.
 * Images are NHWC FP32: x [n][S][S][in_ch], y and target [n][S][S][out_ch],
 * weight [n][S][S].  The loss is sum_p weight_p sum_c (y - target)^2 / out_ch.
 * --------------------------------------------------------------------------- */
typedef struct lbm_nn lbm_nn;

typedef struct {
    int32_t batch;      /* largest number of images per call */
    int32_t size;       /* image side S, a multiple of 8 */
    int32_t in_ch;      /* input channels, 1..16 */
    int32_t out_ch;     /* output channels, 1..32 */
    int32_t width;      /* channels of the first level, a multiple of 32 */
    int32_t precision;  /* LBM_BF16 or LBM_F32 */
} lbm_nn_desc;

/* Sizes of the 4 device buffers: 0 parameters, gradients and Adam moments
 * (FP32), 1 compute weights, 2 activations, their gradients and scratch, 3 the
 * loss accumulator.  Returns the sum, 0 on an invalid description. */
size_t lbm_nn_required_bytes(const lbm_nn_desc* d, size_t sizes_out[4]);
lbm_status lbm_nn_create(const lbm_nn_desc* d, void* const dev_bufs[4], void* hip_stream, lbm_nn** out);
int64_t lbm_nn_num_params(const lbm_nn* n);
/* Copies the parameters from dev_params (device, num_params FP32) and resets
 * the Adam state. */
lbm_status lbm_nn_set_params(lbm_nn* n, const float* dev_params);
lbm_status lbm_nn_get_params(lbm_nn* n, float* dev_out);
/* Forward pass of n <= batch images; dev_y may be NULL (the output stays
 * inside for lbm_nn_backward).  Asynchronous. */
lbm_status lbm_nn_forward(lbm_nn* n, int32_t n_images, const float* dev_x, float* dev_y);
/* Loss and parameter gradients of the last forward pass against dev_target
 * and dev_weight; host_loss (may be NULL) receives the loss after a
 * synchronisation. */
lbm_status lbm_nn_backward(lbm_nn* n, const float* dev_target, const float* dev_weight, double* host_loss);
lbm_status lbm_nn_get_grads(lbm_nn* n, float* dev_out);
/* One Adam update of the FP32 master weights with the current gradients
 * (bias-corrected moments), then the compute weights are refreshed. */
lbm_status lbm_nn_adam_step(lbm_nn* n, float lr, float beta1, float beta2, float eps);
const char* lbm_nn_last_error(const lbm_nn* n);
void lbm_nn_destroy(lbm_nn* n);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
