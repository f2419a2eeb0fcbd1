/*
 * FP64 CPU oracle for the coupled lattice Boltzmann sweep (flow f, convection-
 * diffusion h, vector magnetic g) with the paper's boundary-link updates.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU baseline
 * leg of the benchmark load this file's library.  It shares no code, header or
 * table with the HIP library: it has its own lattice tables, its own node
 * classification and its own boundary-link builder.
 *
 * Everything is plain double precision, summed in ascending direction order,
 * one node at a time, in the order the method states it:
 *   moments -> collision (Eqs. 1-6) -> propagation -> boundary links (Secs. 3-4).
 *
 * Readings where the paper is silent:
 *  - body force: Guo-Zheng-Shi forcing; u includes half the force.
 *  - Lorentz force: J x B with J = curl(B)/mu, the gradient of B taken from the
 *    local non-equilibrium first moment of g, evaluated with the velocity that
 *    carries only half the body force (explicit, local).
 *  - D2Q5 / D3Q7: rest weight 1/2 (2D) or 1/4 (3D), moving weights 1/8,
 *    c^2 = 1/4, as the paper's parameter sets imply (Secs. 5.3, 5.4, 6).
 *  - given velocity / pressure: Eqs. 15-16 (d < 0.5) and Eqs. 43-44 (d >= 0.5).
 *  - if the second fluid node E is not fluid, A stands in for E.
 *  - a link crossing several boundaries: walls win over open boundaries, then
 *    the smaller d, then the lower boundary index.
 *  - several scalar components C_1 .. C_ns (Section 4.2.2): one convection-
 *    diffusion lattice each, with its own relaxation time; a flux wall's law
 *    for component i may also depend on the other components through one
 *    bilinear term, F_i = a1 C_i + quad C_i^2 + cross C_j C_l - a3 (j, l any
 *    components, i included: the rate of a reaction A + B -> P consumes A and
 *    B and produces P), every C(X) extrapolated by Eq. 13 (no iteration
 *    couples the components).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Arithmetic type of the state and of every update.  The default build is
 * double precision; the same source compiled with -DOR_REAL="long double"
 * gives an extended-precision build used as a tighter FP64 reference. */
#ifndef OR_REAL
#define OR_REAL double
#endif
typedef OR_REAL real;

/* ------------------------------------------------------------------------- */
/* lattices (Section 2): D2Q9 / D3Q19 for f, D2Q5 / D3Q7 for h and g          */
/* ------------------------------------------------------------------------- */
enum { OR_D2Q9 = 1, OR_D3Q19 = 2, OR_D2Q5 = 3, OR_D3Q7 = 4 };

typedef struct {
    int Q;
    int e[19][3];
    real w[19];
    real c2; /* squared lattice sound speed c_s^2, c_h^2 or c_g^2 */
    int opp[19];
} or_lattice;

static void lattice_fill(or_lattice* L, int code) {
    memset(L, 0, sizeof(*L));
    if (code == OR_D2Q9) {
        /* ordering with opposite pairs 1-3, 2-4, 5-7, 6-8 (Sections 3 and 4.1) */
        static const int e[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                                    {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
        L->Q = 9;
        L->c2 = (real)1 / 3;
        for (int a = 0; a < 9; ++a) {
            L->e[a][0] = e[a][0];
            L->e[a][1] = e[a][1];
            L->w[a] = a == 0 ? (real)4 / 9 : (a < 5 ? (real)1 / 9 : (real)1 / 36);
        }
    } else if (code == OR_D3Q19) {
        static const int e[19][3] = {
            {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
            {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
            {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
        L->Q = 19;
        L->c2 = (real)1 / 3;
        for (int a = 0; a < 19; ++a) {
            for (int k = 0; k < 3; ++k) L->e[a][k] = e[a][k];
            L->w[a] = a == 0 ? (real)1 / 3 : (a < 7 ? (real)1 / 18 : (real)1 / 36);
        }
    } else if (code == OR_D2Q5) {
        static const int e[5][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}};
        L->Q = 5;
        L->c2 = 0.25;
        for (int a = 0; a < 5; ++a) {
            L->e[a][0] = e[a][0];
            L->e[a][1] = e[a][1];
            L->w[a] = a == 0 ? 0.5 : 0.125;
        }
    } else if (code == OR_D3Q7) {
        static const int e[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                                    {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
        L->Q = 7;
        L->c2 = 0.25;
        for (int a = 0; a < 7; ++a) {
            for (int k = 0; k < 3; ++k) L->e[a][k] = e[a][k];
            L->w[a] = a == 0 ? 0.25 : 0.125;
        }
    }
    for (int a = 0; a < L->Q; ++a)
        for (int b = 0; b < L->Q; ++b)
            if (L->e[a][0] == -L->e[b][0] && L->e[a][1] == -L->e[b][1] &&
                L->e[a][2] == -L->e[b][2])
                L->opp[a] = b;
}

int or_lattice_table(int code, int* Q, int* e /* Q x 3 */, double* w, double* c2, int* opp) {
    or_lattice L;
    if (code < 1 || code > 4) return -1;
    lattice_fill(&L, code);
    *Q = L.Q;
    *c2 = (double)L.c2;
    for (int a = 0; a < L.Q; ++a) {
        for (int k = 0; k < 3; ++k) e[3 * a + k] = L.e[a][k];
        w[a] = (double)L.w[a];
        opp[a] = L.opp[a];
    }
    return 0;
}

static real dot3(const real* a, const real* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static real edot(const int* e, const real* v) { return e[0] * v[0] + e[1] * v[1] + e[2] * v[2]; }

/* Eq. 2 */
static real feq(const or_lattice* L, int a, real rho, const real* u) {
    real eu = edot(L->e[a], u), cs2 = L->c2;
    return rho * L->w[a] * (1 + eu / cs2 + eu * eu / (2 * cs2 * cs2) - dot3(u, u) / (2 * cs2));
}
/* Eq. 4 */
static real heq(const or_lattice* L, int a, real C, const real* u) {
    return C * L->w[a] * (1 + edot(L->e[a], u) / L->c2);
}
/* Eq. 6, Cartesian component k of the vector equilibrium */
static real geq(const or_lattice* L, int a, int k, const real* B, const real* u) {
    real s = 0; /* e_alpha . (u B - B u), component k */
    for (int i = 0; i < 3; ++i) s += L->e[a][i] * (u[i] * B[k] - B[i] * u[k]);
    return L->w[a] * (B[k] + s / L->c2);
}

/* equilibrium vectors whose rest entry closes the zeroth moment exactly */
static void eq_closed_f(const or_lattice* L, real rho, const real* u, real* out) {
    real s = 0;
    for (int a = 1; a < L->Q; ++a) {
        out[a] = feq(L, a, rho, u);
        s += out[a];
    }
    out[0] = rho - s;
}
static void eq_closed_h(const or_lattice* L, real C, const real* u, real* out) {
    real s = 0;
    for (int a = 1; a < L->Q; ++a) {
        out[a] = heq(L, a, C, u);
        s += out[a];
    }
    out[0] = C - s;
}
static void eq_closed_g(const or_lattice* L, int k, const real* B, const real* u, real* out) {
    real s = 0;
    for (int a = 1; a < L->Q; ++a) {
        out[a] = geq(L, a, k, B, u);
        s += out[a];
    }
    out[0] = B[k] - s;
}

void or_equilibria(int code, double rho, const double* u, double C, const double* B,
                   double* f_out, double* h_out, double* g_out /* Q x 3 */) {
    or_lattice L;
    lattice_fill(&L, code);
    real ur[3] = {u[0], u[1], u[2]}, Br[3] = {B[0], B[1], B[2]};
    for (int a = 0; a < L.Q; ++a) {
        if (f_out) f_out[a] = (double)feq(&L, a, rho, ur);
        if (h_out) h_out[a] = (double)heq(&L, a, C, ur);
        if (g_out)
            for (int k = 0; k < 3; ++k) g_out[3 * a + k] = (double)geq(&L, a, k, Br, ur);
    }
}

/* ------------------------------------------------------------------------- */
/* scene description (mirrors the Python scene objects)                       */
/* ------------------------------------------------------------------------- */
enum { K_NONE = 0, K_VEL = 1, K_PRES, K_CONC, K_FLUX, K_BB0, K_MAG_DIR, K_MAG_FLUX, K_MAG_THETA };

/* how a flux wall states its law (the physical description; the builder
 * forms the coefficients of F(phi) = a1 phi + quad phi^2 - a3 itself) */
enum { LAW_COEF = 0, LAW_ROBIN = 1, LAW_REACTION = 2, LAW_SHERCLIFF = 3 };

typedef struct {
    int32_t kind;
    int32_t u_given;
    int32_t profile_axis;
    int32_t profile_len;
    int32_t alt; /* the comparison form of Section 5 (VEL, PRES, FLUX, MAG_FLUX) */
    int32_t law;
    double value;
    double a1, a3, quad; /* LAW_COEF: F = a1 phi + quad phi^2 - a3 (theta = a1 for MAG_THETA) */
    const double* profile; /* per coordinate along profile_axis: a1 (LAW_COEF) or k */
    double k;             /* LAW_ROBIN: d phi/dn = k phi; LAW_REACTION: F = -k (phi - phi_eq) */
    double phi_eq;
    double c_w, H;        /* LAW_SHERCLIFF: thin-wall conductance ratio, length scale */
    int32_t cj, cl;       /* scalar components j, l of the bilinear term (LAW_COEF, FLUX); -1: none */
    double cross;         /* F_i += cross C_j C_l */
} or_bc;

typedef struct {
    int32_t type; /* 0 plane, 1 cylinder, 2 box */
    int32_t axis, side, is_open;
    double q;
    double center[3];
    double radius;
    double u_w[3];
    or_bc f, h[3], g[3]; /* h: one condition per scalar component */
    double omega; /* the boundary velocity is u_w cos(omega t') (0: steady) */
    double d_used; /* > 0: the links take this d in their update, not the measured one */
    double lo[3], hi[3]; /* box: closed solid block lo <= x <= hi (bounds may be infinite) */
} or_boundary;

typedef struct {
    int32_t dim;
    int32_t n[3];
    int32_t periodic[3];
    int32_t fl, sl, ml; /* lattice codes; 0 = absent */
    int32_t ncomp;
    int32_t comps[3];
    double tau_f, tau_c, tau_m, rho0, C0, mu;
    double B_ext[3], accel[3];
    double init_C;
    int32_t nb;
    const or_boundary* b;
    int32_t ns;          /* scalar components (>= 1 with a scalar lattice) */
    int32_t pad;
    double tau_s[3];     /* relaxation time of each scalar component (tau_s[0] = tau_c) */
} or_scene;

typedef struct {
    int32_t A, E;     /* first fluid node, second fluid node (-1 = not fluid) */
    int32_t field;    /* 0 f, 1 h, 2 g */
    int32_t comp;     /* slot of the evolved magnetic component (g) */
    int32_t dir;      /* unknown direction alpha at A */
    int32_t kind;
    int32_t bnd;      /* boundary index */
    int32_t u_given;
    double d, value, a1, a3, weight;
    double u_w[3];
    double omega; /* of the boundary velocity, 0 = steady */
    int32_t compare; /* comparison form of the kind (Section 5) */
    int32_t pad;
    double quad;     /* quadratic term of the flux law */
    int32_t cj, cl;  /* FLUX: scalar components j, l of the bilinear term, -1 none */
    double cross;    /* FLUX: F_i += cross C_j(X) C_l(X) */
} or_link;

/* ------------------------------------------------------------------------- */
/* node classification and link building (Sections 3-4 and 6)                */
/* ------------------------------------------------------------------------- */
static int node_index(const or_scene* s, const int* c) { return c[0] + s->n[0] * (c[1] + s->n[1] * c[2]); }

/* map a coordinate into the domain; returns 0 if it falls outside a
 * non-periodic extent */
static int wrap(const or_scene* s, int* c) {
    for (int k = 0; k < 3; ++k) {
        if (c[k] < 0 || c[k] >= s->n[k]) {
            if (!s->periodic[k]) return 0;
            c[k] = ((c[k] % s->n[k]) + s->n[k]) % s->n[k];
        }
    }
    return 1;
}

static void inplane_axes(int axis, int* p, int* q) {
    *p = axis == 0 ? 1 : 0;
    *q = axis == 2 ? 1 : 2;
}

static int inside_cylinder(const or_boundary* b, const int* c) {
    int p, q;
    inplane_axes(b->axis, &p, &q);
    double dy = c[p] - b->center[p], dz = c[q] - b->center[q];
    return dy * dy + dz * dz < b->radius * b->radius;
}

/* closed solid block: a node on a face belongs to it */
static int inside_box(const or_boundary* b, const int* c) {
    for (int k = 0; k < 3; ++k)
        if (c[k] < b->lo[k] || c[k] > b->hi[k]) return 0;
    return 1;
}

/* fraction d in (0,1] of the link A -> A - e at which it enters the block:
 * the points A - s e inside the block form the s-interval where every
 * coordinate lies in [lo, hi]; d is that interval's lower end. */
static double box_d(const or_boundary* b, const int* A, const int* e) {
    double s_lo = 0.0, s_hi = 1.0;
    for (int k = 0; k < 3; ++k) {
        if (e[k] == 0) {
            if (A[k] < b->lo[k] || A[k] > b->hi[k]) return -1.0;
            continue;
        }
        /* coordinate A[k] - s e[k] in [lo, hi] for s between these two */
        double s1 = (A[k] - b->lo[k]) / e[k], s2 = (A[k] - b->hi[k]) / e[k];
        if (s1 > s2) {
            double t = s1;
            s1 = s2;
            s2 = t;
        }
        if (s1 > s_lo) s_lo = s1;
        if (s2 < s_hi) s_hi = s2;
    }
    return s_lo <= s_hi ? s_lo : -1.0;
}

/* fluid iff inside every cylinder and outside every block (flat planes lie
 * outside the node range) */
int or_fluid_mask(const or_scene* s, uint8_t* mask) {
    int c[3];
    for (c[2] = 0; c[2] < s->n[2]; ++c[2])
        for (c[1] = 0; c[1] < s->n[1]; ++c[1])
            for (c[0] = 0; c[0] < s->n[0]; ++c[0]) {
                int fl = 1;
                for (int i = 0; i < s->nb; ++i)
                    if ((s->b[i].type == 1 && !inside_cylinder(&s->b[i], c)) ||
                        (s->b[i].type == 2 && inside_box(&s->b[i], c)))
                        fl = 0;
                mask[node_index(s, c)] = (uint8_t)fl;
            }
    return 0;
}

/* fraction d in (0,1] of the link A -> A - e at which the ray leaves the
 * cylinder: |P_A - s e_perp - c|^2 = R^2, the positive root in s. */
static double cylinder_d(const or_boundary* b, const int* A, const int* e) {
    int p, q;
    inplane_axes(b->axis, &p, &q);
    double py = A[p] - b->center[p], pz = A[q] - b->center[q];
    double vy = -e[p], vz = -e[q];
    double aa = vy * vy + vz * vz, bb = py * vy + pz * vz, cc = py * py + pz * pz - b->radius * b->radius;
    if (aa == 0.0) return -1.0;
    double disc = bb * bb - aa * cc;
    if (disc < 0.0) return -1.0;
    return (-bb + sqrt(disc)) / aa;
}

static const or_bc* bc_of(const or_boundary* b, int field, int comp_slot) {
    if (field == 0) return &b->f;
    if (field == 1) return &b->h[comp_slot];
    return &b->g[comp_slot];
}

/* Surface segmentation (Section 6.2): outer solid layer B_i of a cylinder,
 * sorted by azimuth theta (then radius); S_i = (theta_{i+1} - theta_{i-1}) R / 2.
 * The flux of B_i is split over its links to fluid with e.n > 0 in proportion
 * to e.n, n the inward unit normal at B_i (Eq. 48).  Computed in one
 * cross-section; the axial extent of a node is one lattice unit. */
typedef struct {
    int y, z;        /* in-plane coordinates */
    double theta, r, S;
} or_outer;

static int cmp_outer(const void* a, const void* b) {
    const or_outer* x = (const or_outer*)a;
    const or_outer* y = (const or_outer*)b;
    if (x->theta < y->theta) return -1;
    if (x->theta > y->theta) return 1;
    if (x->r < y->r) return -1;
    if (x->r > y->r) return 1;
    return 0;
}

/* builds S_i for every outer-layer node of cylinder `b` for the in-plane
 * directions of lattice L.  Returns an array indexed by in-plane node
 * (y + ny*z) holding S_i (0 for others); also returns the count and sum. */
static double* cylinder_segments(const or_scene* s, const or_boundary* b, const or_lattice* L,
                                 int* n_outer, double* S_sum) {
    int p, q;
    inplane_axes(b->axis, &p, &q);
    int np = s->n[p], nq = s->n[q];
    double* S = (double*)calloc((size_t)np * nq, sizeof(double));
    or_outer* list = (or_outer*)malloc(sizeof(or_outer) * (size_t)np * nq);
    int cnt = 0;
    for (int j = 0; j < nq; ++j)
        for (int i = 0; i < np; ++i) {
            int c[3] = {0, 0, 0};
            c[p] = i;
            c[q] = j;
            if (inside_cylinder(b, c)) continue; /* solid nodes only */
            int linked = 0;
            for (int a = 1; a < L->Q; ++a) {
                if (L->e[a][b->axis] != 0) continue;
                int cc[3] = {c[0] + L->e[a][0], c[1] + L->e[a][1], c[2] + L->e[a][2]};
                cc[b->axis] = 0;
                if (cc[p] < 0 || cc[p] >= np || cc[q] < 0 || cc[q] >= nq) continue;
                if (inside_cylinder(b, cc)) linked = 1;
            }
            if (!linked) continue;
            double dy = i - b->center[p], dz = j - b->center[q];
            list[cnt].y = i;
            list[cnt].z = j;
            list[cnt].theta = atan2(dz, dy);
            list[cnt].r = sqrt(dy * dy + dz * dz);
            ++cnt;
        }
    qsort(list, (size_t)cnt, sizeof(or_outer), cmp_outer);
    double tot = 0.0;
    for (int k = 0; k < cnt; ++k) {
        double tprev = k > 0 ? list[k - 1].theta : list[cnt - 1].theta - 2.0 * M_PI;
        double tnext = k < cnt - 1 ? list[k + 1].theta : list[0].theta + 2.0 * M_PI;
        list[k].S = (tnext - tprev) * b->radius / 2.0;
        S[list[k].y + np * list[k].z] = list[k].S;
        tot += list[k].S;
    }
    free(list);
    *n_outer = cnt;
    *S_sum = tot;
    return S;
}

/* Eq. 48 split weight for the link entering fluid node A along e_alpha from
 * the solid node B = A - e_alpha. */
static double split_weight(const or_scene* s, const or_boundary* b, const or_lattice* L,
                           const double* S, const int* Bc, int alpha) {
    int p, q;
    inplane_axes(b->axis, &p, &q);
    int np = s->n[p], nq = s->n[q];
    double Si = 0.0;
    if (Bc[p] >= 0 && Bc[p] < np && Bc[q] >= 0 && Bc[q] < nq) Si = S[Bc[p] + np * Bc[q]];
    double ny_ = b->center[p] - Bc[p], nz_ = b->center[q] - Bc[q];
    double nn = sqrt(ny_ * ny_ + nz_ * nz_);
    ny_ /= nn;
    nz_ /= nn;
    double sum = 0.0, best = -1e300;
    int best_a = -1;
    for (int g = 1; g < L->Q; ++g) {
        /* all links of B_i across the wall: directions with an in-plane part
         * (on D3Q19 also those with an axial component) */
        if (L->e[g][p] == 0 && L->e[g][q] == 0) continue;
        int cc[3] = {Bc[0] + L->e[g][0], Bc[1] + L->e[g][1], Bc[2] + L->e[g][2]};
        cc[b->axis] = 0;
        if (cc[p] < 0 || cc[p] >= np || cc[q] < 0 || cc[q] >= nq) continue;
        if (!inside_cylinder(b, cc)) continue;
        double en = L->e[g][p] * ny_ + L->e[g][q] * nz_;
        if (en > 0.0) sum += en;
        if (en > best) {
            best = en;
            best_a = g;
        }
    }
    double en_a = L->e[alpha][p] * ny_ + L->e[alpha][q] * nz_;
    if (sum > 0.0) return en_a > 0.0 ? Si * en_a / sum : 0.0;
    return alpha == best_a ? Si : 0.0;
}

typedef struct {
    or_scene sc;
    or_lattice Lf, Lh, Lg;
    int N;
    uint8_t* fluid;
    real *f, *fs, *h, *hs, *g, *gs; /* [Q][N] (g: [ncomp][Q][N]) */
    real* mom;                     /* [N][8]: rho, ux, uy, uz, C, Bx, By, Bz */
    or_link* links;
    int nlinks;
    long t;
    double S_sum;
    int n_outer;
} or_sim;

/* The coefficients of a flux wall's law F(phi) = a1 phi + quad phi^2 - a3 from
 * its physical description.  The field's transport coefficient is
 * c^2 (tau - 1/2): D for the scalar (Section 2.2), eta for B (Section 2.3).
 *  - Robin wall d phi/dn = k phi, n into the fluid: with Eq. 17 and a2 = D,
 *    -D d phi/dn = a1 phi - a3 gives a1 = -k D, a3 = 0.
 *  - first-order surface reaction F = -k (phi - phi_eq) (Section 5.3).
 *  - Shercliff thin wall (Eq. 30): -eta dB_k/dn = -eta (B_k - B_ext,k)/(c_w H),
 *    i.e. a1 = -eta/(c_w H) and a3 = a1 B_ext,k; c_w infinite is the perfectly
 *    conducting wall, zero flux.  The theta form (Eqs. 39-40) takes
 *    theta = c_w H / (tau_m - 1/2) in a1.
 * A profile gives a1 (given coefficients) or k (Robin, reaction) per position
 * of A along its axis. */
static void flux_law(const or_scene* s, const or_bc* bc, int field, const or_lattice* L, int comp,
                     const int* c, or_link* lk) {
    double prof = 0.0;
    int has_prof = bc->profile && bc->profile_len > 0;
    if (has_prof) {
        int pos = c[bc->profile_axis];
        if (pos >= bc->profile_len) pos = bc->profile_len - 1;
        prof = bc->profile[pos];
    }
    double tau = field == 1 ? s->tau_s[comp] : s->tau_m;
    double kappa = (double)L->c2 * (tau - 0.5);
    lk->a1 = lk->a3 = lk->quad = 0.0;
    if (bc->law == LAW_ROBIN) {
        double k = has_prof ? prof : bc->k;
        lk->a1 = -k * kappa;
    } else if (bc->law == LAW_REACTION) {
        double k = has_prof ? prof : bc->k;
        lk->a1 = -k;
        lk->a3 = -k * bc->phi_eq;
    } else if (bc->law == LAW_SHERCLIFF) {
        if (bc->kind == K_MAG_THETA) {
            lk->a1 = bc->c_w * bc->H / (s->tau_m - 0.5);
        } else if (!isinf(bc->c_w)) {
            lk->a1 = -kappa / (bc->c_w * bc->H);
            lk->a3 = lk->a1 * s->B_ext[s->comps[comp]];
        }
    } else {
        lk->a1 = has_prof ? prof : bc->a1;
        lk->a3 = bc->a3;
        lk->quad = bc->quad;
    }
    lk->cj = lk->cl = -1;
    lk->cross = 0.0;
    if (field == 1 && bc->kind == K_FLUX && bc->law == LAW_COEF && bc->cj >= 0 && bc->cl >= 0) {
        lk->cj = bc->cj;
        lk->cl = bc->cl;
        lk->cross = bc->cross;
    }
}

/* collects the links of one lattice field.  Returns the number written or -1. */
static int build_field_links(or_sim* S, int field, const or_lattice* L, int ncomp, or_link* out,
                             int cap, int cnt) {
    const or_scene* s = &S->sc;
    double** seg = (double**)calloc((size_t)s->nb, sizeof(double*));
    int c[3];
    for (c[2] = 0; c[2] < s->n[2]; ++c[2])
        for (c[1] = 0; c[1] < s->n[1]; ++c[1])
            for (c[0] = 0; c[0] < s->n[0]; ++c[0]) {
                int A = node_index(s, c);
                if (!S->fluid[A]) continue;
                for (int a = 1; a < L->Q; ++a) {
                    int Bc[3] = {c[0] - L->e[a][0], c[1] - L->e[a][1], c[2] - L->e[a][2]};
                    int Bw[3] = {Bc[0], Bc[1], Bc[2]};
                    int in = wrap(s, Bw);
                    if (in && S->fluid[node_index(s, Bw)]) continue; /* known population */
                    /* choose the crossed boundary */
                    int best = -1, best_open = 1;
                    double best_d = 2.0;
                    for (int i = 0; i < s->nb; ++i) {
                        const or_boundary* b = &s->b[i];
                        double d = -1.0;
                        if (b->type == 0) {
                            int ax = b->axis;
                            int crossed = b->side == 0 ? (Bc[ax] < 0) : (Bc[ax] >= s->n[ax]);
                            if (crossed && !s->periodic[ax]) d = b->q;
                        } else if (b->type == 1) {
                            if (!inside_cylinder(b, Bc)) d = cylinder_d(b, c, L->e[a]);
                        } else if (inside_box(b, Bc)) {
                            d = box_d(b, c, L->e[a]);
                        }
                        if (d <= 0.0) continue;
                        const or_bc* bc0 = bc_of(b, field, 0);
                        if (bc0->kind == K_NONE) continue;
                        int better = 0;
                        if (best < 0) better = 1;
                        else if (best_open && !b->is_open) better = 1;
                        else if (best_open == b->is_open && d < best_d) better = 1;
                        if (better) {
                            best = i;
                            best_open = b->is_open;
                            best_d = d;
                        }
                    }
                    if (best < 0) {
                        free(seg);
                        return -1;
                    }
                    const or_boundary* b = &s->b[best];
                    int Ec[3] = {c[0] + L->e[a][0], c[1] + L->e[a][1], c[2] + L->e[a][2]};
                    int E = -1;
                    if (wrap(s, Ec) && S->fluid[node_index(s, Ec)]) E = node_index(s, Ec);
                    for (int k = 0; k < ncomp; ++k) {
                        const or_bc* bc = bc_of(b, field, k);
                        if (cnt >= cap) {
                            free(seg);
                            return -1;
                        }
                        or_link* lk = &out[cnt++];
                        memset(lk, 0, sizeof(*lk));
                        lk->A = A;
                        lk->E = E;
                        lk->field = field;
                        lk->comp = k;
                        lk->dir = a;
                        lk->kind = bc->kind;
                        lk->bnd = best;
                        lk->u_given = bc->u_given;
                        lk->d = b->d_used > 0.0 ? b->d_used : best_d;
                        lk->value = bc->value;
                        flux_law(s, bc, field, L, k, c, lk);
                        for (int j = 0; j < 3; ++j) lk->u_w[j] = b->u_w[j];
                        lk->omega = b->omega;
                        lk->compare = bc->alt;
                        /* Eq. 48 on a flat face: the node's share is spread evenly
                         * over its links through the face, as many as the lattice
                         * directions with component +1 along an axis */
                        lk->weight = 1.0;
                        if (bc->kind == K_FLUX || bc->kind == K_MAG_FLUX) {
                            int through = 0;
                            for (int g = 0; g < L->Q; ++g) through += L->e[g][0] == 1;
                            lk->weight = 1.0 / through;
                        }
                        if (b->type == 1 && (bc->kind == K_FLUX || bc->kind == K_MAG_FLUX)) {
                            if (!seg[best]) {
                                int no;
                                double ssum;
                                seg[best] = cylinder_segments(s, b, L, &no, &ssum);
                                S->S_sum = ssum;
                                S->n_outer = no;
                            }
                            lk->weight = split_weight(s, b, L, seg[best], Bc, a);
                        }
                    }
                }
            }
    for (int i = 0; i < s->nb; ++i) free(seg[i]);
    free(seg);
    return cnt;
}

static int build_links(or_sim* S) {
    const or_scene* s = &S->sc;
    int cap = 64;
    int per_node = S->Lf.Q + (s->sl ? S->Lh.Q * s->ns : 0) + (s->ml ? S->Lg.Q * s->ncomp : 0);
    /* upper bound: every fluid node next to a boundary, every direction */
    long nf = 0;
    for (int n = 0; n < S->N; ++n) nf += S->fluid[n];
    cap = (int)(nf * per_node < 64 ? 64 : nf * per_node);
    or_link* L = (or_link*)malloc(sizeof(or_link) * (size_t)cap);
    int cnt = 0;
    cnt = build_field_links(S, 0, &S->Lf, 1, L, cap, cnt);
    if (cnt >= 0 && s->sl) cnt = build_field_links(S, 1, &S->Lh, s->ns, L, cap, cnt);
    if (cnt >= 0 && s->ml) cnt = build_field_links(S, 2, &S->Lg, s->ncomp, L, cap, cnt);
    if (cnt < 0) {
        free(L);
        return -1;
    }
    S->links = L;
    S->nlinks = cnt;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* moments and collision                                                       */
/* ------------------------------------------------------------------------- */
#define IDX(q, n) ((size_t)(q) * (size_t)S->N + (size_t)(n))
#define GIDX(k, q, n) (((size_t)(k) * (size_t)S->Lg.Q + (size_t)(q)) * (size_t)S->N + (size_t)(n))
#define HIDX(k, q, n) (((size_t)(k) * (size_t)S->Lh.Q + (size_t)(q)) * (size_t)S->N + (size_t)(n))
/* moments kept per node: rho, u(3), C_0, B(3), then C_1, C_2 */
#define MOMW 10
static int cslot(int k) { return k == 0 ? 4 : 7 + k; }

/* moments at node n from the pre-collision populations: rho, u, C, B.
 * Also returns the total force F (body + Lorentz). */
static void node_moments(const or_sim* S, int n, real* rho_o, real* u, real* C_o /* [ns] */, real* B,
                         real* F) {
    const or_scene* s = &S->sc;
    const or_lattice* Lf = &S->Lf;
    real rho = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < Lf->Q; ++a) {
        real fa = S->f[IDX(a, n)];
        rho += fa;
        for (int k = 0; k < 3; ++k) m[k] += Lf->e[a][k] * fa;
    }
    if (s->sl)
        for (int k = 0; k < s->ns; ++k) {
            real C = 0.0;
            for (int a = 0; a < S->Lh.Q; ++a) C += S->h[HIDX(k, a, n)];
            C_o[k] = C;
        }
    for (int k = 0; k < 3; ++k) B[k] = s->B_ext[k];
    real Fl[3] = {0.0, 0.0, 0.0};
    if (s->ml) {
        const or_lattice* Lg = &S->Lg;
        for (int c = 0; c < s->ncomp; ++c) {
            real sum = 0.0;
            for (int a = 0; a < Lg->Q; ++a) sum += S->g[GIDX(c, a, n)];
            B[s->comps[c]] = sum;
        }
        /* velocity with half the body force only (explicit Lorentz reading) */
        real u0[3];
        for (int k = 0; k < 3; ++k) u0[k] = (m[k] + 0.5 * rho * s->accel[k]) / rho;
        /* gradient of B from the non-equilibrium first moment of g:
         * d_i B_j = -(Lambda_ij - Lambda^eq_ij) / (tau_m c_g^2), Lambda^eq = u B - B u */
        real dB[3][3] = {{0}};
        for (int c = 0; c < s->ncomp; ++c) {
            int j = s->comps[c];
            for (int i = 0; i < 3; ++i) {
                real lam = 0.0;
                for (int a = 0; a < Lg->Q; ++a) lam += Lg->e[a][i] * S->g[GIDX(c, a, n)];
                real lam_eq = u0[i] * B[j] - B[i] * u0[j];
                dB[i][j] = -(lam - lam_eq) / (s->tau_m * Lg->c2);
            }
        }
        /* J = curl(B) / mu; F_L = J x B */
        real J[3];
        J[0] = (dB[1][2] - dB[2][1]) / s->mu;
        J[1] = (dB[2][0] - dB[0][2]) / s->mu;
        J[2] = (dB[0][1] - dB[1][0]) / s->mu;
        Fl[0] = J[1] * B[2] - J[2] * B[1];
        Fl[1] = J[2] * B[0] - J[0] * B[2];
        Fl[2] = J[0] * B[1] - J[1] * B[0];
    }
    for (int k = 0; k < 3; ++k) {
        F[k] = rho * s->accel[k] + Fl[k];
        u[k] = (m[k] + 0.5 * F[k]) / rho;
    }
    *rho_o = rho;
}

static void collide_node(or_sim* S, int n) {
    const or_scene* s = &S->sc;
    real rho, u[3], C[3] = {0, 0, 0}, B[3], F[3];
    node_moments(S, n, &rho, u, C, B, F);
    real* mo = &S->mom[(size_t)n * MOMW];
    mo[0] = rho;
    mo[1] = u[0];
    mo[2] = u[1];
    mo[3] = u[2];
    mo[5] = B[0];
    mo[6] = B[1];
    mo[7] = B[2];
    for (int k = 0; k < 3; ++k) mo[cslot(k)] = C[k];
    /* Eq. 1 with the Guo source term.  The equilibria conserve the zeroth
     * moments (Section 2.4) and the force adds no mass; with weights rounded
     * to real precision that holds only if the rest entry closes the sum,
     * so the rest entries are taken as the moment minus the moving ones. */
    const or_lattice* Lf = &S->Lf;
    real tf = s->tau_f, cs2 = Lf->c2;
    real eqv[19], srcv[19];
    eq_closed_f(Lf, rho, u, eqv);
    real ssum = 0.0;
    for (int a = 1; a < Lf->Q; ++a) {
        real eu = edot(Lf->e[a], u);
        real src = 0.0;
        for (int k = 0; k < 3; ++k)
            src += ((Lf->e[a][k] - u[k]) / cs2 + eu * Lf->e[a][k] / (cs2 * cs2)) * F[k];
        srcv[a] = src * (1.0 - 0.5 / tf) * Lf->w[a];
        ssum += srcv[a];
    }
    srcv[0] = -ssum;
    for (int a = 0; a < Lf->Q; ++a) {
        real fa = S->f[IDX(a, n)];
        S->fs[IDX(a, n)] = fa + (eqv[a] - fa) / tf + srcv[a];
    }
    /* Eq. 3, for each scalar component */
    if (s->sl)
        for (int k = 0; k < s->ns; ++k) {
            eq_closed_h(&S->Lh, C[k], u, eqv);
            for (int a = 0; a < S->Lh.Q; ++a) {
                real ha = S->h[HIDX(k, a, n)];
                S->hs[HIDX(k, a, n)] = ha + (eqv[a] - ha) / s->tau_s[k];
            }
        }
    /* Eq. 5 */
    if (s->ml)
        for (int c = 0; c < s->ncomp; ++c) {
            eq_closed_g(&S->Lg, s->comps[c], B, u, eqv);
            for (int a = 0; a < S->Lg.Q; ++a) {
                real ga = S->g[GIDX(c, a, n)];
                S->gs[GIDX(c, a, n)] = ga + (eqv[a] - ga) / s->tau_m;
            }
        }
}

/* ------------------------------------------------------------------------- */
/* boundary link value (Sections 3-4)                                         */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t lattice, kind, dir, comp_axis, u_given;
    double d, value, a1, a3, weight;
    double u_w[3];
    double x_ap_E;  /* post-collision, direction alpha' (towards the wall), at E */
    double x_ap_A;  /* post-collision, direction alpha', at A */
    double x_a_A;   /* post-collision, direction alpha, at A */
    double mA[MOMW], mE[MOMW]; /* rho, u(3), C_0, B(3), C_1, C_2 at A and E at time t */
    int32_t compare;     /* the comparison form of the kind (Section 5) */
    double quad;         /* quadratic term of the flux law */
    int32_t cslot;       /* FLUX: moment slot of the link's scalar component */
    int32_t jslot, lslot; /* FLUX: moment slots of the bilinear term's components, -1: none */
    double cross;        /* FLUX: coefficient of C_j(X) C_l(X) in F_i */
} or_link_in;

/* Eq. 13: phi(X) = -d phi(E) + (d+1) phi(A) */
static real extrap(real d, real pE, real pA) { return -d * pE + (d + 1) * pA; }

/* the same inputs in the arithmetic type of the build */
typedef struct {
    int32_t lattice, kind, dir, comp_axis, u_given;
    real d, value, a1, a3, weight;
    real u_w[3];
    real x_ap_E, x_ap_A, x_a_A;
    real mA[MOMW], mE[MOMW];
    int32_t compare;
    real quad;
    int32_t cslot, jslot, lslot;
    real cross;
} or_link_in_r;

static real link_eval_r(const or_link_in_r* in) {
    or_lattice L;
    lattice_fill(&L, in->lattice);
    int a = in->dir, ap = L.opp[a];
    real d = in->d;
    real uX[3], BX[3];
    for (int k = 0; k < 3; ++k) {
        uX[k] = in->u_given ? in->u_w[k] : extrap(d, in->mE[1 + k], in->mA[1 + k]);
        BX[k] = extrap(d, in->mE[5 + k], in->mA[5 + k]);
    }
    /* Y interpolation / extrapolation (Eqs. 16, 20, 35) */
    real xY = (1 - 2 * d) * in->x_ap_E + 2 * d * in->x_ap_A;
    switch (in->kind) {
        case K_VEL: {
            real rhoX = extrap(d, in->mE[0], in->mA[0]);
            real inc = feq(&L, a, rhoX, in->u_w) - feq(&L, ap, rhoX, in->u_w);
            /* Eq. 15; the comparison run of Section 5.1 keeps it for d >= 0.5 */
            if (d < (real)0.5 || in->compare) return xY + inc;
            return ((2 * d - 1) * in->x_a_A + in->x_ap_A + inc) / (2 * d); /* Eq. 43 */
        }
        case K_PRES: {
            real uXp[3];
            for (int k = 0; k < 3; ++k) uXp[k] = extrap(d, in->mE[1 + k], in->mA[1 + k]);
            real sum = feq(&L, a, in->value, uXp) + feq(&L, ap, in->value, uXp);
            if (d < (real)0.5 || in->compare) return sum - xY;                          /* zeroth-moment pair */
            return ((2 * d - 1) * in->x_a_A - in->x_ap_A + sum) / (2 * d); /* Eq. 44 */
        }
        case K_CONC: /* Eqs. 19-20 */
            return heq(&L, a, in->value, uX) + heq(&L, ap, in->value, uX) - xY;
        case K_MAG_DIR: { /* Eqs. 34-35 */
            real Bg[3] = {BX[0], BX[1], BX[2]};
            Bg[in->comp_axis] = in->value;
            return geq(&L, a, in->comp_axis, Bg, uX) + geq(&L, ap, in->comp_axis, Bg, uX) - xY;
        }
        case K_BB0: /* Eqs. 21-22 */
            if (d < (real)0.5) return xY;
            return ((2 * d - 1) * in->x_a_A + in->x_ap_A) / (2 * d);
        case K_FLUX:
        case K_MAG_FLUX:
        case K_MAG_THETA: {
            real phiX, dmove;
            real mu_[3] = {-uX[0], -uX[1], -uX[2]};
            real cross = 0;
            if (in->kind == K_FLUX) {
                phiX = extrap(d, in->mE[in->cslot], in->mA[in->cslot]);
                dmove = heq(&L, ap, phiX, mu_) - heq(&L, a, phiX, mu_); /* Eq. 24 */
                /* other components' values at X, extrapolated the same way
                 * (Section 4.2.2): F_i(C_1, C_2, ...) needs no iteration */
                if (in->jslot >= 0 && in->lslot >= 0)
                    cross = in->cross * extrap(d, in->mE[in->jslot], in->mA[in->jslot]) *
                            extrap(d, in->mE[in->lslot], in->mA[in->lslot]);
            } else {
                phiX = BX[in->comp_axis];
                dmove = geq(&L, ap, in->comp_axis, BX, mu_) - geq(&L, a, in->comp_axis, BX, mu_);
            }
            if (in->kind == K_MAG_THETA) {
                /* Eqs. 39-40: theta = a1; the bounced population x is replaced
                 * by ((theta - 1) x + theta dmove) / (theta + 1) */
                real th = in->a1;
                if (d < (real)0.5) return ((th - 1) * xY + th * dmove) / (th + 1);
                real bounced = ((th - 1) * in->x_ap_A + th * dmove) / (th + 1);
                return ((2 * d - 1) * in->x_a_A + bounced) / (2 * d);
            }
            /* Eq. 23 with F(phi_X) = a1 phi_X + quad phi_X^2 - a3, Eq. 48 */
            real dflux = (in->a1 * phiX + in->quad * phiX * phiX + cross - in->a3) * in->weight;
            if (in->compare) { /* Eq. 33: the flux joins the bounced population at X */
                if (d < (real)0.5) return xY + dflux + dmove;
                return ((2 * d - 1) * in->x_a_A + in->x_ap_A + dflux + dmove) / (2 * d);
            }
            real xM = ((real)0.5 - d) * in->x_ap_E + ((real)0.5 + d) * in->x_ap_A;      /* Eq. 25 */
            real xM1 = xM + dflux + dmove;                                    /* Eq. 26 */
            return ((d - (real)0.5) * in->x_a_A + xM1) / (d + (real)0.5);                  /* Eq. 27 */
        }
        default:
            return NAN;
    }
}

double or_link_eval(const or_link_in* in) {
    or_link_in_r r;
    r.lattice = in->lattice;
    r.kind = in->kind;
    r.dir = in->dir;
    r.comp_axis = in->comp_axis;
    r.u_given = in->u_given;
    r.d = in->d;
    r.value = in->value;
    r.a1 = in->a1;
    r.a3 = in->a3;
    r.weight = in->weight;
    r.x_ap_E = in->x_ap_E;
    r.x_ap_A = in->x_ap_A;
    r.x_a_A = in->x_a_A;
    r.compare = in->compare;
    r.quad = in->quad;
    r.cslot = in->cslot;
    r.jslot = in->jslot;
    r.lslot = in->lslot;
    r.cross = in->cross;
    for (int k = 0; k < 3; ++k) r.u_w[k] = in->u_w[k];
    for (int k = 0; k < MOMW; ++k) {
        r.mA[k] = in->mA[k];
        r.mE[k] = in->mE[k];
    }
    return (double)link_eval_r(&r);
}

static void apply_links(or_sim* S) {
    const or_scene* s = &S->sc;
    for (int i = 0; i < S->nlinks; ++i) {
        const or_link* lk = &S->links[i];
        const or_lattice* L = lk->field == 0 ? &S->Lf : (lk->field == 1 ? &S->Lh : &S->Lg);
        const real* xs = lk->field == 0 ? S->fs : (lk->field == 1 ? S->hs : S->gs);
        real* x = lk->field == 0 ? S->f : (lk->field == 1 ? S->h : S->g);
        size_t base = lk->field != 0 ? (size_t)lk->comp * (size_t)L->Q * (size_t)S->N : 0;
        int a = lk->dir, ap = L->opp[a];
        int E = lk->E >= 0 ? lk->E : lk->A;
        or_link_in_r in;
        memset(&in, 0, sizeof(in));
        in.lattice = lk->field == 0 ? s->fl : (lk->field == 1 ? s->sl : s->ml);
        in.kind = lk->kind;
        in.dir = a;
        in.comp_axis = lk->field == 2 ? s->comps[lk->comp] : 0;
        in.u_given = lk->u_given;
        in.compare = lk->compare;
        in.quad = lk->quad;
        in.cslot = lk->field == 1 ? cslot(lk->comp) : 4;
        in.jslot = lk->field == 1 && lk->cj >= 0 ? cslot(lk->cj) : -1;
        in.lslot = lk->field == 1 && lk->cl >= 0 ? cslot(lk->cl) : -1;
        in.cross = lk->cross;
        in.d = lk->d;
        in.value = lk->value;
        in.a1 = lk->a1;
        in.a3 = lk->a3;
        in.weight = lk->weight;
        /* a time-dependent boundary velocity at the arrival time at the
         * boundary, t' = t + (1 - d) for the value at t + 1 from the
         * post-collision state at t (Section 4.1) */
        const double wall = lk->omega != 0.0 ? cos(lk->omega * ((double)S->t + 1.0 - lk->d)) : 1.0;
        for (int k = 0; k < 3; ++k) in.u_w[k] = lk->u_w[k] * wall;
        in.x_ap_E = xs[base + (size_t)ap * S->N + E];
        in.x_ap_A = xs[base + (size_t)ap * S->N + lk->A];
        in.x_a_A = xs[base + (size_t)a * S->N + lk->A];
        for (int k = 0; k < MOMW; ++k) in.mA[k] = S->mom[(size_t)lk->A * MOMW + k];
        for (int k = 0; k < MOMW; ++k) in.mE[k] = S->mom[(size_t)E * MOMW + k];
        x[base + (size_t)a * S->N + lk->A] = link_eval_r(&in);
    }
}

/* ------------------------------------------------------------------------- */
/* public API                                                                  */
/* ------------------------------------------------------------------------- */
void or_destroy(or_sim* S) {
    if (!S) return;
    free(S->fluid);
    free(S->f);
    free(S->fs);
    free(S->h);
    free(S->hs);
    free(S->g);
    free(S->gs);
    free(S->mom);
    free(S->links);
    free(S);
}

int or_init_fields(or_sim* S, const double* rho, const double* u, const double* C, const double* B);

or_sim* or_create(const or_scene* sc) {
    or_sim* S = (or_sim*)calloc(1, sizeof(or_sim));
    S->sc = *sc;
    lattice_fill(&S->Lf, sc->fl);
    if (sc->sl) lattice_fill(&S->Lh, sc->sl);
    if (sc->ml) lattice_fill(&S->Lg, sc->ml);
    S->N = sc->n[0] * sc->n[1] * sc->n[2];
    S->fluid = (uint8_t*)malloc((size_t)S->N);
    or_fluid_mask(sc, S->fluid);
    size_t N = (size_t)S->N;
    S->f = (real*)calloc(N * S->Lf.Q, sizeof(real));
    S->fs = (real*)calloc(N * S->Lf.Q, sizeof(real));
    if (sc->sl) {
        if (S->sc.ns < 1) S->sc.ns = 1;
        if (S->sc.ns > 3) {
            or_destroy(S);
            return NULL;
        }
        S->h = (real*)calloc(N * S->Lh.Q * S->sc.ns, sizeof(real));
        S->hs = (real*)calloc(N * S->Lh.Q * S->sc.ns, sizeof(real));
    }
    if (sc->ml) {
        S->g = (real*)calloc(N * S->Lg.Q * sc->ncomp, sizeof(real));
        S->gs = (real*)calloc(N * S->Lg.Q * sc->ncomp, sizeof(real));
    }
    S->mom = (real*)calloc(N * MOMW, sizeof(real));
    if (build_links(S) != 0) {
        or_destroy(S);
        return NULL;
    }
    or_init_fields(S, NULL, NULL, NULL, NULL);
    return S;
}

/* equilibrium initialisation from (rho, u, C, B) fields; NULL = uniform rest
 * state (rho0, 0, init_C, B_ext).  u, B are [N][3]; C is [ns][N]. */
int or_init_fields(or_sim* S, const double* rho, const double* u, const double* C, const double* B) {
    const or_scene* s = &S->sc;
    for (int n = 0; n < S->N; ++n) {
        real r = rho ? rho[n] : s->rho0;
        real uu[3] = {0, 0, 0}, BB[3] = {s->B_ext[0], s->B_ext[1], s->B_ext[2]};
        if (u)
            for (int k = 0; k < 3; ++k) uu[k] = u[3 * (size_t)n + k];
        if (B)
            for (int k = 0; k < 3; ++k) BB[k] = B[3 * (size_t)n + k];
        real eqv[19];
        eq_closed_f(&S->Lf, r, uu, eqv);
        for (int a = 0; a < S->Lf.Q; ++a) S->f[IDX(a, n)] = eqv[a];
        if (s->sl)
            for (int k = 0; k < s->ns; ++k) {
                real cc = C ? C[(size_t)k * S->N + n] : s->init_C;
                eq_closed_h(&S->Lh, cc, uu, eqv);
                for (int a = 0; a < S->Lh.Q; ++a) S->h[HIDX(k, a, n)] = eqv[a];
            }
        if (s->ml)
            for (int c = 0; c < s->ncomp; ++c) {
                eq_closed_g(&S->Lg, s->comps[c], BB, uu, eqv);
                for (int a = 0; a < S->Lg.Q; ++a) S->g[GIDX(c, a, n)] = eqv[a];
            }
    }
    S->t = 0;
    return 0;
}

void or_step(or_sim* S, long nsteps) {
    const or_scene* s = &S->sc;
    for (long it = 0; it < nsteps; ++it) {
        /* relaxation at every fluid node */
#pragma omp parallel for schedule(static)
        for (int n = 0; n < S->N; ++n)
            if (S->fluid[n]) collide_node(S, n);
        /* propagation: x_alpha(x, t+1) = x*_alpha(x - e_alpha, t) */
#pragma omp parallel for schedule(static)
        for (int n = 0; n < S->N; ++n) {
            if (!S->fluid[n]) continue;
            int c[3] = {n % s->n[0], (n / s->n[0]) % s->n[1], n / (s->n[0] * s->n[1])};
            for (int a = 0; a < S->Lf.Q; ++a) {
                int sc_[3] = {c[0] - S->Lf.e[a][0], c[1] - S->Lf.e[a][1], c[2] - S->Lf.e[a][2]};
                if (!wrap(s, sc_)) continue;
                int src = node_index(s, sc_);
                if (S->fluid[src]) S->f[IDX(a, n)] = S->fs[IDX(a, src)];
            }
            if (s->sl)
                for (int a = 0; a < S->Lh.Q; ++a) {
                    int sc_[3] = {c[0] - S->Lh.e[a][0], c[1] - S->Lh.e[a][1], c[2] - S->Lh.e[a][2]};
                    if (!wrap(s, sc_)) continue;
                    int src = node_index(s, sc_);
                    if (!S->fluid[src]) continue;
                    for (int k = 0; k < s->ns; ++k) S->h[HIDX(k, a, n)] = S->hs[HIDX(k, a, src)];
                }
            if (s->ml)
                for (int a = 0; a < S->Lg.Q; ++a) {
                    int sc_[3] = {c[0] - S->Lg.e[a][0], c[1] - S->Lg.e[a][1], c[2] - S->Lg.e[a][2]};
                    if (!wrap(s, sc_)) continue;
                    int src = node_index(s, sc_);
                    if (!S->fluid[src]) continue;
                    for (int k = 0; k < s->ncomp; ++k) S->g[GIDX(k, a, n)] = S->gs[GIDX(k, a, src)];
                }
        }
        /* boundary links: unknown populations entering the fluid */
        apply_links(S);
        S->t += 1;
    }
}

/* columns of or_moments: rho, u, C_0, B, then C_1 .. C_{ns-1} */
int or_moment_width(const or_sim* S) { return 8 + (S->sc.sl ? S->sc.ns - 1 : 0); }

/* moments at the current time: [N][or_moment_width] rho, u, C_0, B, C_1, ...
 * (zeros at solid nodes) */
void or_moments(const or_sim* S, double* out) {
    const int W = or_moment_width(S);
    for (int n = 0; n < S->N; ++n) {
        double* o = &out[(size_t)n * W];
        if (!S->fluid[n]) {
            memset(o, 0, sizeof(double) * W);
            continue;
        }
        real rho, u[3], C[3] = {0, 0, 0}, B[3], F[3];
        node_moments(S, n, &rho, u, C, B, F);
        o[0] = rho;
        o[1] = u[0];
        o[2] = u[1];
        o[3] = u[2];
        o[4] = C[0];
        o[5] = B[0];
        o[6] = B[1];
        o[7] = B[2];
        for (int k = 1; k < W - 7; ++k) o[7 + k] = C[k];
    }
}

/* populations of one field at the current time, [Q][N] (h: [ns][Q][N], g: [ncomp][Q][N]) */
static void copy_out(const real* src, double* dst, size_t n) {
    for (size_t i = 0; i < n; ++i) dst[i] = (double)src[i];
}
static void copy_in(const double* src, real* dst, size_t n) {
    for (size_t i = 0; i < n; ++i) dst[i] = src[i];
}

int or_populations(const or_sim* S, int field, double* out) {
    size_t N = (size_t)S->N;
    if (field == 0) copy_out(S->f, out, N * S->Lf.Q);
    else if (field == 1 && S->sc.sl) copy_out(S->h, out, N * S->Lh.Q * S->sc.ns);
    else if (field == 2 && S->sc.ml) copy_out(S->g, out, N * S->Lg.Q * S->sc.ncomp);
    else return -1;
    return 0;
}

int or_set_populations(or_sim* S, int field, const double* in) {
    size_t N = (size_t)S->N;
    if (field == 0) copy_in(in, S->f, N * S->Lf.Q);
    else if (field == 1 && S->sc.sl) copy_in(in, S->h, N * S->Lh.Q * S->sc.ns);
    else if (field == 2 && S->sc.ml) copy_in(in, S->g, N * S->Lg.Q * S->sc.ncomp);
    else return -1;
    return 0;
}

int or_real_bytes(void) { return (int)sizeof(real); }
int or_num_links(const or_sim* S) { return S->nlinks; }
void or_get_links(const or_sim* S, or_link* out) { memcpy(out, S->links, sizeof(or_link) * (size_t)S->nlinks); }
void or_get_mask(const or_sim* S, uint8_t* out) { memcpy(out, S->fluid, (size_t)S->N); }
long or_time(const or_sim* S) { return S->t; }
double or_segment_sum(const or_sim* S, int* n_outer) {
    *n_outer = S->n_outer;
    return S->S_sum;
}
int or_sizeof_link(void) { return (int)sizeof(or_link); }
int or_sizeof_link_in(void) { return (int)sizeof(or_link_in); }
int or_sizeof_scene(void) { return (int)sizeof(or_scene); }
int or_sizeof_boundary(void) { return (int)sizeof(or_boundary); }
