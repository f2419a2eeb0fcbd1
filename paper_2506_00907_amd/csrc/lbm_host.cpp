// Host side of liblbm: parameter validation, the geometry / boundary-link
// builder, the device buffer layout and the C ABI declared in include/lbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_ctx.hpp"
#include "lbm_device.hpp"
#include "lbm_internal.hpp"

using lbmi::DevLink;

namespace lbmh {

// ---------------------------------------------------------------------------
// lattice tables (host view of the device lattices)
// ---------------------------------------------------------------------------
struct HostLat {
    int Q = 0;
    int e[19][3] = {};
    double w[19] = {};
    double c2 = 1.0;
    int opp[19] = {};
    int cross = 1;  // directions crossing a flat face from one side (1 on D2Q5 / D3Q7, 5 on D3Q19)
};

template <class L>
HostLat host_lat() {
    HostLat h;
    h.Q = L::Q;
    h.c2 = L::c2;
    for (int a = 0; a < L::Q; ++a) {
        h.e[a][0] = L::ex(a);
        h.e[a][1] = L::ey(a);
        h.e[a][2] = L::ez(a);
        h.w[a] = L::w(a);
        h.opp[a] = L::opp(a);
    }
    h.cross = 0;
    for (int a = 0; a < L::Q; ++a) h.cross += L::ex(a) == 1 ? 1 : 0;
    return h;
}

HostLat lattice_of(int code) {
    switch (code) {
        case LBM_D2Q9: return host_lat<lbmi::LD2Q9>();
        case LBM_D3Q19: return host_lat<lbmi::LD3Q19>();
        case LBM_D2Q5: return host_lat<lbmi::LD2Q5>();
        case LBM_D3Q7: return host_lat<lbmi::LD3Q7>();
        default: return HostLat{};
    }
}

// ---------------------------------------------------------------------------
// parameter validation
// ---------------------------------------------------------------------------
bool valid_params(const lbm_params* p, std::string* why) {
    auto fail = [&](const char* m) {
        if (why) *why = m;
        return false;
    };
    if (!p) return fail("params is NULL");
    if (p->dim != 2 && p->dim != 3) return fail("dim must be 2 or 3");
    for (int k = 0; k < 3; ++k)
        if (p->n[k] < 1) return fail("node counts must be >= 1");
    if (p->dim == 2) {
        if (p->n[2] != 1 || !p->periodic[2]) return fail("2D domains need n[2] = 1 and periodic[2] = 1");
        if (p->fluid != LBM_D2Q9) return fail("2D flow lattice must be D2Q9");
        if (p->scalar != LBM_NONE && p->scalar != LBM_D2Q5) return fail("2D scalar lattice must be D2Q5");
        if (p->magnetic != LBM_NONE && p->magnetic != LBM_D2Q5) return fail("2D magnetic lattice must be D2Q5");
        if (p->magnetic && (p->mag_ncomp < 1 || p->mag_ncomp > 2)) return fail("2D magnetic components: 1 or 2");
    } else {
        if (p->fluid != LBM_D3Q19) return fail("3D flow lattice must be D3Q19");
        if (p->scalar != LBM_NONE && p->scalar != LBM_D3Q7) return fail("3D scalar lattice must be D3Q7");
        if (p->magnetic != LBM_NONE && p->magnetic != LBM_D3Q7 && p->magnetic != LBM_D3Q19)
            return fail("3D magnetic lattice must be D3Q7 or D3Q19");
        if (p->magnetic == LBM_D3Q19 && (p->scalar || p->mag_ncomp != 1))
            return fail("a D3Q19 magnetic lattice: one component, no scalar lattice");
        if (p->magnetic && p->mag_ncomp != 1 && p->mag_ncomp != 3) return fail("3D magnetic components: 1 or 3");
    }
    if (!p->magnetic && p->mag_ncomp != 0) return fail("mag_ncomp must be 0 without a magnetic lattice");
    for (int c = 0; c < p->mag_ncomp; ++c)
        if (p->mag_comp[c] != c) return fail("evolved magnetic component c must be Cartesian axis c");
    if (!(p->tau_f > 0.5) || (p->scalar && !(p->tau_c > 0.5)) || (p->magnetic && !(p->tau_m > 0.5)))
        return fail("relaxation times must exceed 1/2");
    if (p->scalar_ncomp < 0 || p->scalar_ncomp > 3) return fail("scalar_ncomp must be 0..3");
    if (p->scalar_ncomp > 1) {
        if (!p->scalar) return fail("several scalar components need a scalar lattice");
        if (p->magnetic) return fail("several scalar components: no magnetic lattice");
        for (int k = 0; k + 1 < p->scalar_ncomp; ++k)
            if (!(p->tau_cs[k] > 0.5)) return fail("relaxation times must exceed 1/2");
    }
    if (!(p->rho0 > 0.0)) return fail("rho0 must be positive");
    if (p->magnetic && !(p->mu > 0.0)) return fail("mu must be positive");
    if (p->storage < LBM_F64 || p->storage > LBM_BF16) return fail("unknown storage");
    for (int k = 0; k < 3; ++k)
        if (!(p->store_scale[k] > 0.0) || !std::isfinite(p->store_scale[k])) return fail("store_scale must be positive");
    if (!std::isfinite(p->wall_omega)) return fail("wall_omega must be finite");
    const double nn = (double)(p->n[0] + 2) * (p->n[1] + 2) * (p->n[2] + 2);
    if (nn > 2.0e9) return fail("lattice too large for 32-bit node indices");
    return true;
}

Pad padding(const lbm_params* p) {
    Pad d;
    d.hx = p->periodic[0] ? 0 : 1;
    d.hy = p->periodic[1] ? 0 : 1;
    d.hz = p->periodic[2] ? 0 : 1;
    d.NX = p->n[0] + 2 * d.hx;
    d.NY = p->n[1] + 2 * d.hy;
    d.NZ = p->n[2] + 2 * d.hz;
    d.nodes = (size_t)d.NX * d.NY * d.NZ;
    d.plane = round_up(d.nodes, 64);  // whole 64-node tiles (waves)
    return d;
}

size_t value_bytes(int storage) { return storage == LBM_F64 ? 8 : (storage == LBM_F32 ? 4 : 2); }
size_t compute_bytes(int storage) { return storage == LBM_F64 ? 8 : 4; }
size_t link_bytes(int storage) { return storage == LBM_F64 ? sizeof(DevLink<double>) : sizeof(DevLink<float>); }

int scalar_comps(const lbm_params* p) { return p->scalar_ncomp > 1 ? p->scalar_ncomp : 1; }

int moment_planes(const lbm_params* p) { return 8 + scalar_comps(p) - 1; }

int total_planes(const lbm_params* p) {
    int q = lattice_of(p->fluid).Q;
    if (p->scalar) q += scalar_comps(p) * lattice_of(p->scalar).Q;
    if (p->magnetic) q += p->mag_ncomp * lattice_of(p->magnetic).Q;
    return q;
}

lbmi::KernelSet kernels_for(const lbm_params* p) {
    const int nc = p->magnetic ? p->mag_ncomp : 0, ns = scalar_comps(p);
    switch (p->storage) {
        case LBM_F64: return lbmi::kernels_f64(p->fluid, p->scalar, p->magnetic, nc, ns);
        case LBM_F32: return lbmi::kernels_f32(p->fluid, p->scalar, p->magnetic, nc, ns);
        case LBM_F16: return lbmi::kernels_f16(p->fluid, p->scalar, p->magnetic, nc, ns);
        default: return lbmi::kernels_bf16(p->fluid, p->scalar, p->magnetic, nc, ns);
    }
}

// ---------------------------------------------------------------------------
// geometry and boundary-link builder
// ---------------------------------------------------------------------------
struct Cand {
    int bnd = -1;
    double d = 0.0;
    bool open = true;
};

class LinkBuilder {
   public:
    LinkBuilder(const lbm_params& p, const lbm_boundary* b, int nb) : p_(p), b_(b, b + nb) {
        N_ = (size_t)p.n[0] * p.n[1] * p.n[2];
    }

    // fluid iff strictly inside every cylinder and outside every box
    void classify() {
        mask_.assign(N_, 1);
        for (int z = 0; z < p_.n[2]; ++z)
            for (int y = 0; y < p_.n[1]; ++y)
                for (int x = 0; x < p_.n[0]; ++x) {
                    const int c[3] = {x, y, z};
                    for (const auto& bd : b_)
                        if ((bd.type == 1 && !inside(bd, c)) || (bd.type == 2 && in_box(bd, c)))
                            mask_[index(c)] = 0;
                }
    }

    std::string build(std::vector<lbm_link>* out) {
        classify();
        const int fields[3] = {p_.fluid, p_.scalar, p_.magnetic};
        for (int field = 0; field < 3; ++field) {
            if (!fields[field]) continue;
            const HostLat L = lattice_of(fields[field]);
            const int ncomp = field == 2 ? p_.mag_ncomp : (field == 1 ? scalar_comps(&p_) : 1);
            std::vector<std::vector<double>> segs(b_.size());
            for (int z = 0; z < p_.n[2]; ++z)
                for (int y = 0; y < p_.n[1]; ++y)
                    for (int x = 0; x < p_.n[0]; ++x) {
                        const int A[3] = {x, y, z};
                        const size_t ia = index(A);
                        if (!mask_[ia]) continue;
                        for (int a = 1; a < L.Q; ++a) {
                            int src[3] = {x - L.e[a][0], y - L.e[a][1], z - L.e[a][2]};
                            const int raw[3] = {src[0], src[1], src[2]};
                            if (wrap(src) && mask_[index(src)]) continue;
                            Cand best;
                            for (int i = 0; i < (int)b_.size(); ++i) {
                                const lbm_boundary& bd = b_[i];
                                if (bc_of(bd, field, 0).kind == 0) continue;
                                double d = -1.0;
                                if (bd.type == 0) {
                                    const int ax = bd.axis;
                                    const bool crossed = bd.side == 0 ? raw[ax] < 0 : raw[ax] >= p_.n[ax];
                                    if (crossed && !p_.periodic[ax]) d = bd.q;
                                } else if (bd.type == 1) {
                                    if (!inside(bd, raw)) d = cylinder_fraction(bd, A, L.e[a]);
                                } else if (in_box(bd, raw)) {
                                    d = box_fraction(bd, A, L.e[a]);
                                }
                                if (!(d > 0.0)) continue;
                                const bool open = bd.is_open != 0;
                                bool take = best.bnd < 0;
                                if (!take && best.open && !open) take = true;
                                if (!take && best.open == open && d < best.d) take = true;
                                if (take) best = Cand{i, d, open};
                            }
                            if (best.bnd < 0) {
                                char msg[160];
                                snprintf(msg, sizeof msg, "no boundary condition for node (%d,%d,%d) field %d dir %d",
                                         x, y, z, field, a);
                                return msg;
                            }
                            const lbm_boundary& bd = b_[best.bnd];
                            int E[3] = {x + L.e[a][0], y + L.e[a][1], z + L.e[a][2]};
                            const bool e_ok = wrap(E) && mask_[index(E)];
                            for (int c = 0; c < ncomp; ++c) {
                                const lbm_bc& bc = bc_of(bd, field, c);
                                lbm_link lk;
                                std::memset(&lk, 0, sizeof lk);
                                lk.node = (uint32_t)ia;
                                lk.enode = e_ok ? (uint32_t)index(E) : (uint32_t)ia;
                                lk.field = (uint8_t)field;
                                lk.dir = (uint8_t)a;
                                lk.kind = (uint8_t)bc.kind;
                                lk.comp = (uint8_t)(field == 0 ? 0 : c);
                                lk.flags = (uint8_t)((bc.u_given ? 1 : 0) | (e_ok ? 0 : 2) |
                                                     (bc.u_given && bd.u_osc ? 4 : 0) | (bc.alt ? 8 : 0));
                                lk.d = bd.d_scheme > 0.0 ? bd.d_scheme : best.d;
                                lk.value = bc.value;
                                law_coefficients(bc, field, c, A, &lk);
                                if (field == 1 && bc.kind == LBM_LK_FLUX && bc.law == LBM_LAW_COEF && bc.cross != 0.0) {
                                    lk.cross_comp[0] = (uint8_t)bc.cross_comp[0];
                                    lk.cross_comp[1] = (uint8_t)bc.cross_comp[1];
                                    lk.cross = bc.cross;
                                }
                                for (int k = 0; k < 3; ++k) lk.u_w[k] = bd.u_w[k];
                                const bool flux = bc.kind == LBM_LK_FLUX || bc.kind == LBM_LK_MAG_FLUX;
                                // flat faces: a node's flux split evenly over the
                                // links crossing the face (one on D2Q5 / D3Q7)
                                lk.weight = flux ? 1.0 / L.cross : 1.0;
                                if (bd.type == 1 && flux) {
                                    if (segs[best.bnd].empty()) segs[best.bnd] = segments(bd, L);
                                    lk.weight = split(bd, L, segs[best.bnd], raw, a);
                                }
                                out->push_back(lk);
                            }
                        }
                    }
        }
        std::stable_sort(out->begin(), out->end(), [](const lbm_link& u, const lbm_link& v) {
            if (u.node != v.node) return u.node < v.node;
            if (u.field != v.field) return u.field < v.field;
            if (u.comp != v.comp) return u.comp < v.comp;
            return u.dir < v.dir;
        });
        return std::string();
    }

    const std::vector<uint8_t>& mask() const { return mask_; }

    // The flux law of a link from the boundary's description (lbm_flux_law),
    // with the field's transport coefficient kappa = c^2 (tau - 1/2) (D for
    // h, eta for g): a Robin wall d phi/dn = k phi gives F = -k D phi (Eq. 17
    // with a2 = D); a first-order reaction F = -k (phi - phi_eq) (Section
    // 5.3); a thin conducting wall F = -eta (B_k - B_ext,k) / (c_w H) (Eq. 30),
    // where c_w = inf is the perfectly conducting wall; the theta form takes
    // theta = c_w H / (tau_m - 1/2) (Eqs. 39-40).  A profile replaces a1
    // (given coefficients) or k (Robin, reaction) by its value at A.
    void law_coefficients(const lbm_bc& bc, int field, int comp, const int* A, lbm_link* lk) const {
        double prof = 0.0;
        const bool has_prof = bc.profile && bc.profile_len > 0;
        if (has_prof) prof = bc.profile[std::min(A[bc.profile_axis], bc.profile_len - 1)];
        const int code = field == 1 ? p_.scalar : p_.magnetic;
        const double tau = field == 1 ? (comp == 0 ? p_.tau_c : p_.tau_cs[comp - 1]) : p_.tau_m;
        const double kappa = field == 0 ? 0.0 : lattice_of(code).c2 * (tau - 0.5);
        switch (bc.law) {
            case LBM_LAW_ROBIN: {
                const double k = has_prof ? prof : bc.k;
                lk->a1 = -k * kappa;
                lk->a3 = 0.0;
                break;
            }
            case LBM_LAW_REACTION: {
                const double k = has_prof ? prof : bc.k;
                lk->a1 = -k;
                lk->a3 = -k * bc.phi_eq;
                break;
            }
            case LBM_LAW_SHERCLIFF: {
                if (bc.kind == LBM_LK_MAG_THETA) {
                    lk->a1 = bc.c_w * bc.H / (p_.tau_m - 0.5);
                    lk->a3 = 0.0;
                } else if (std::isinf(bc.c_w)) {
                    lk->a1 = lk->a3 = 0.0;
                } else {
                    lk->a1 = -kappa / (bc.c_w * bc.H);
                    lk->a3 = lk->a1 * p_.B_ext[p_.mag_comp[comp]];
                }
                break;
            }
            default:
                lk->a1 = has_prof ? prof : bc.a1;
                lk->a3 = bc.a3;
                lk->quad = bc.quad;
        }
    }

   private:
    size_t index(const int* c) const { return (size_t)c[0] + (size_t)p_.n[0] * ((size_t)c[1] + (size_t)p_.n[1] * c[2]); }

    bool wrap(int* c) const {
        for (int k = 0; k < 3; ++k) {
            if (c[k] >= 0 && c[k] < p_.n[k]) continue;
            if (!p_.periodic[k]) return false;
            c[k] = ((c[k] % p_.n[k]) + p_.n[k]) % p_.n[k];
        }
        return true;
    }

    static void plane_axes(int axis, int* u, int* v) {
        static const int tab[3][2] = {{1, 2}, {0, 2}, {0, 1}};
        *u = tab[axis][0];
        *v = tab[axis][1];
    }

    static bool inside(const lbm_boundary& c, const int* q) {
        int u, v;
        plane_axes(c.axis, &u, &v);
        const double du = q[u] - c.center[u], dv = q[v] - c.center[v];
        return du * du + dv * dv < c.radius * c.radius;
    }

    // closed axis-aligned box (bounds may be infinite): a node on a face is solid
    static bool in_box(const lbm_boundary& b, const int* q) {
        for (int k = 0; k < 3; ++k)
            if (!(q[k] >= b.lo[k] && q[k] <= b.hi[k])) return false;
        return true;
    }

    // fraction s in (0, 1] of the link A -> A - e (A outside, A - e inside the
    // box) where the segment A - s e enters the box: the latest of its slab
    // entries
    static double box_fraction(const lbm_boundary& b, const int* A, const int* e) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double a = A[k];
            if (a >= b.lo[k] && a <= b.hi[k]) continue;
            if (e[k] == 0) return -1.0;
            const double face = a < b.lo[k] ? b.lo[k] : b.hi[k];
            s = std::max(s, (a - face) / (double)e[k]);
        }
        return s;
    }

    // fraction s in (0, 1] of the link A -> A - e where the ray meets the
    // circle (stable form of the quadratic's positive root)
    static double cylinder_fraction(const lbm_boundary& c, const int* A, const int* e) {
        int u, v;
        plane_axes(c.axis, &u, &v);
        const double pu = A[u] - c.center[u], pv = A[v] - c.center[v];
        const double du = -e[u], dv = -e[v];
        const double qa = du * du + dv * dv;
        if (qa == 0.0) return -1.0;
        const double qb = pu * du + pv * dv;
        const double qc = pu * pu + pv * pv - c.radius * c.radius;  // < 0 inside
        const double disc = qb * qb - qa * qc;
        if (disc < 0.0) return -1.0;
        const double sq = std::sqrt(disc);
        const double t = qb >= 0.0 ? -(qb + sq) : -(qb - sq);
        const double r1 = t / qa, r2 = qc / t;
        return r1 > 0.0 ? r1 : r2;
    }

    static const lbm_bc& bc_of(const lbm_boundary& b, int field, int comp) {
        return field == 0 ? b.f : (field == 1 ? (comp == 0 ? b.h : b.h_more[comp - 1]) : b.g[comp]);
    }

    // surface element S_i of every outer-layer solid node of a cylinder in
    // one cross-section (Section 6.2): nodes sorted by azimuth (then radius),
    // S_i = (theta_{i+1} - theta_{i-1}) R / 2 with cyclic neighbours
    std::vector<double> segments(const lbm_boundary& c, const HostLat& L) const {
        int u, v;
        plane_axes(c.axis, &u, &v);
        const int nu = p_.n[u], nv = p_.n[v];
        struct Node {
            int iu, iv;
            double th, r;
        };
        std::vector<Node> outer;
        for (int jv = 0; jv < nv; ++jv)
            for (int ju = 0; ju < nu; ++ju) {
                int q[3] = {0, 0, 0};
                q[u] = ju;
                q[v] = jv;
                if (inside(c, q)) continue;
                bool touches = false;
                for (int a = 1; a < L.Q && !touches; ++a) {
                    if (L.e[a][c.axis] != 0) continue;
                    int s[3] = {q[0] + L.e[a][0], q[1] + L.e[a][1], q[2] + L.e[a][2]};
                    s[c.axis] = 0;
                    if (s[u] < 0 || s[u] >= nu || s[v] < 0 || s[v] >= nv) continue;
                    touches = inside(c, s);
                }
                if (!touches) continue;
                const double du = ju - c.center[u], dv = jv - c.center[v];
                outer.push_back(Node{ju, jv, std::atan2(dv, du), std::hypot(du, dv)});
            }
        std::sort(outer.begin(), outer.end(), [](const Node& a, const Node& b) {
            return a.th != b.th ? a.th < b.th : a.r < b.r;
        });
        std::vector<double> S((size_t)nu * nv, 0.0);
        const size_t m = outer.size();
        const double two_pi = 2.0 * M_PI;
        for (size_t i = 0; i < m; ++i) {
            const double prev = i == 0 ? outer[m - 1].th - two_pi : outer[i - 1].th;
            const double next = i + 1 == m ? outer[0].th + two_pi : outer[i + 1].th;
            S[(size_t)outer[i].iu + (size_t)nu * outer[i].iv] = 0.5 * (next - prev) * c.radius;
        }
        return S;
    }

    // Eq. 48: the share of S_B carried by the link entering A along e_alpha
    // from the solid node B
    double split(const lbm_boundary& c, const HostLat& L, const std::vector<double>& S, const int* B,
                 int alpha) const {
        int u, v;
        plane_axes(c.axis, &u, &v);
        const int nu = p_.n[u], nv = p_.n[v];
        double SB = 0.0;
        if (B[u] >= 0 && B[u] < nu && B[v] >= 0 && B[v] < nv) SB = S[(size_t)B[u] + (size_t)nu * B[v]];
        double nx = c.center[u] - B[u], ny = c.center[v] - B[v];
        const double len = std::hypot(nx, ny);
        nx /= len;
        ny /= len;
        double total = 0.0, top = -1e300;
        int arg = -1;
        for (int g = 1; g < L.Q; ++g) {
            // every direction with an in-plane part (D3Q19: also those with an
            // axial component); the axial directions never cross the wall
            if (L.e[g][u] == 0 && L.e[g][v] == 0) continue;
            int s[3] = {B[0] + L.e[g][0], B[1] + L.e[g][1], B[2] + L.e[g][2]};
            s[c.axis] = 0;
            if (s[u] < 0 || s[u] >= nu || s[v] < 0 || s[v] >= nv || !inside(c, s)) continue;
            const double en = L.e[g][u] * nx + L.e[g][v] * ny;
            if (en > 0.0) total += en;
            if (en > top) {
                top = en;
                arg = g;
            }
        }
        const double ea = L.e[alpha][u] * nx + L.e[alpha][v] * ny;
        if (total > 0.0) return ea > 0.0 ? SB * ea / total : 0.0;
        return alpha == arg ? SB : 0.0;
    }

    const lbm_params& p_;
    std::vector<lbm_boundary> b_;
    size_t N_;
    std::vector<uint8_t> mask_;
};

}  // namespace lbmh

using namespace lbmh;

namespace lbmh {

void drop_graph(lbm_ctx* c) {
    for (lbm_ctx::StepGraph* g : {&c->run[0], &c->run[1], &c->tail}) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        *g = lbm_ctx::StepGraph();
    }
}

void release_capture(lbm_ctx* c) {
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->capture_stream2) (void)hipStreamDestroy(c->capture_stream2);
    for (hipEvent_t e : {c->ev_links, c->ev_bnd, c->ev_fork, c->ev_join})
        if (e) (void)hipEventDestroy(e);
    c->capture_stream = c->capture_stream2 = nullptr;
    c->ev_links = c->ev_bnd = c->ev_fork = c->ev_join = nullptr;
}

// first element of the wave lists in buffer 1 (after the flags and the wave
// summary): the boundary waves, then the interior ones
uint32_t* wave_lists(const lbm_ctx* c) {
    return (uint32_t*)((char*)c->buf[1] + round_up(c->pad.plane, kAlign) + round_up(c->pad.plane / 64, kAlign));
}

lbm_status finish_reduce(lbm_ctx* c, const double h[12], double out[8]) {
    const double dt = (double)(c->t - c->t_snap);
    double res = -1.0;
    if (c->snap_valid && dt > 0) {
        res = 0.0;
        for (int f = 0; f < 3; ++f) {
            const double nrm = std::sqrt(h[8 + f]);
            if (h[8 + f] == 0.0 && h[5 + f] == 0.0) continue;
            res = std::max(res, std::sqrt(h[5 + f]) / (dt * std::max(nrm, 1e-30)));
        }
    }
    out[0] = res;
    out[1] = h[0];
    out[2] = h[1];
    out[3] = h[2];
    out[4] = h[3];
    out[5] = h[4];
    out[6] = c->snap_valid ? dt : 0.0;
    out[7] = h[11];
    c->snap_valid = true;
    c->t_snap = c->t;
    if (h[11] > 0) return set_err(c, LBM_EUNSTABLE, "non-finite moments");
    return LBM_OK;
}

lbm_status set_err(lbm_ctx* c, lbm_status s, const std::string& m) {
    if (c) c->err = m;
    return s;
}

lbm_status hip_check(lbm_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return LBM_OK;
    return set_err(c, LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void layout(const lbm_params* p, size_t n_links, size_t sz[LBM_NBUF]) {
    const Pad d = padding(p);
    const size_t vb = value_bytes(p->storage), cb = compute_bytes(p->storage);
    sz[0] = round_up((size_t)total_planes(p) * d.plane * vb, kAlign);          // populations
    sz[1] = round_up(d.plane, kAlign) + round_up(d.plane / 64, kAlign) +       // node flags, wave summary,
            round_up(d.plane / 64 * 4, kAlign);                                 // wave lists
    sz[2] = round_up(std::max<size_t>(n_links, 1) * link_bytes(p->storage), kAlign);  // link records
    const size_t mw = (size_t)moment_planes(p);
    sz[3] = round_up(2 * mw * d.plane * cb, kAlign) + kAlign;                  // moment planes, time base
    sz[4] = round_up((mw - 1) * d.plane * cb, kAlign) + round_up(lbmi::NACC * sizeof(double), kAlign);  // reductions
    sz[5] = sz[6] = sz[7] = 0;
}

lbmi::KArgs base_args(const lbm_ctx* c) {
    lbmi::KArgs a;
    std::memset(&a, 0, sizeof a);
    a.NX = c->pad.NX;
    a.NY = c->pad.NY;
    a.NZ = c->pad.NZ;
    a.hx = c->pad.hx;
    a.hy = c->pad.hy;
    a.hz = c->pad.hz;
    a.n0 = c->p.n[0];
    a.n1 = c->p.n[1];
    a.n2 = c->p.n[2];
    a.plane = c->pad.plane;
    a.S = c->buf[0];
    a.flags = (const uint8_t*)c->buf[1];
    a.wave_fluid = round_up(c->pad.plane, kAlign);
    a.links = c->buf[2];
    a.M = c->buf[3];
    a.n_links = c->n_links;
    a.cmp_links = c->cmp_links ? 1 : 0;
    a.tau_f = c->p.tau_f;
    a.tau_c = c->p.scalar ? c->p.tau_c : 1.0;
    for (int k = 0; k < 2; ++k) a.tau_cs[k] = k + 1 < scalar_comps(&c->p) ? c->p.tau_cs[k] : 1.0;
    a.tau_m = c->p.magnetic ? c->p.tau_m : 1.0;
    a.rho0 = c->p.rho0;
    a.wall_omega = c->p.wall_omega;
    a.C0 = c->p.C0;
    a.mu = c->p.magnetic ? c->p.mu : 1.0;
    for (int k = 0; k < 3; ++k) {
        a.Bext[k] = c->p.B_ext[k];
        a.accel[k] = c->p.accel[k];
        const bool scaled = c->p.storage == LBM_F16 || c->p.storage == LBM_BF16;
        a.scale[k] = scaled ? c->p.store_scale[k] : 1.0;
        a.comp[k] = k;
    }
    a.parity = (int)(c->t & 1);
    a.links_ready = c->t > 0 ? 1 : 0;
    a.tbase = nullptr;
    a.tstep = (uint32_t)c->t;
    a.stream = c->stream;
    return a;
}

uint32_t* time_base(const lbm_ctx* c) {
    return (uint32_t*)((char*)c->buf[3] +
                       round_up(2 * (size_t)moment_planes(&c->p) * c->pad.plane * compute_bytes(c->p.storage), kAlign));
}

size_t domain_nodes(const lbm_params& p) { return (size_t)p.n[0] * p.n[1] * p.n[2]; }

// Moments (bit q: rho, u_x, u_y, u_z, C, B_x, B_y, B_z) a link's formula reads
// at A and E, following link_value: the velocity at X when it is extrapolated
// (Eq. 13), rho_X for the moving-wall increment of a velocity link, C_X or B_X
// of a flux link and the other components of B_X where the moving correction
// (Eq. 24) uses them.
uint8_t moments_needed(const lbm_link& k, const int* e) {
    const bool u_given = k.flags & 1;
    const bool eu_zero = u_given && e[0] * k.u_w[0] + e[1] * k.u_w[1] + e[2] * k.u_w[2] == 0.0;
    const bool uw_zero = u_given && k.u_w[0] == 0.0 && k.u_w[1] == 0.0 && k.u_w[2] == 0.0;
    const uint8_t U = 0x0E;  // u_x, u_y, u_z
    switch (k.kind) {
        case LBM_LK_VEL: return (uint8_t)((eu_zero ? 0 : 0x01) | (u_given ? 0 : U));
        case LBM_LK_PRES: return U;
        case LBM_LK_FLUX: return (uint8_t)(0x10 | (u_given ? 0 : U));
        case LBM_LK_MAG_FLUX:
            if (uw_zero) return (uint8_t)(0x20 << k.comp);
            return (uint8_t)(0xE0 | (u_given ? 0 : U));
        case LBM_LK_MAG_THETA:  // B only through the moving correction
            if (uw_zero) return 0;
            return (uint8_t)(0xE0 | (u_given ? 0 : U));
        default: return 0;  // CONC, BB0, MAG_DIR: no moments
    }
}

template <class R>
void fill_devlinks(const lbm_ctx* c, const std::vector<lbm_link>& L, const std::vector<uint32_t>& padA,
                   const std::vector<uint32_t>& padE, const std::vector<uint32_t>& padB,
                   std::vector<unsigned char>* bytes) {
    const HostLat Lf = lattice_of(c->p.fluid), Lh = lattice_of(c->p.scalar), Lg = lattice_of(c->p.magnetic);
    const int QF = Lf.Q, QH = c->p.scalar ? Lh.Q : 0, QG = Lg.Q, NS = scalar_comps(&c->p);
    auto cslot = [](int k) { return k == 0 ? 4 : 7 + k; };  // moment plane of scalar component k
    bytes->assign(std::max<size_t>(L.size(), 1) * sizeof(DevLink<R>), 0);
    DevLink<R>* out = (DevLink<R>*)bytes->data();
    for (size_t i = 0; i < L.size(); ++i) {
        const lbm_link& s = L[i];
        const HostLat& lat = s.field == 0 ? Lf : (s.field == 1 ? Lh : Lg);
        const int base = s.field == 0 ? 0 : (s.field == 1 ? QF + s.comp * QH : QF + NS * QH + s.comp * QG);
        DevLink<R> d;
        std::memset(&d, 0, sizeof d);
        d.A = padA[i];
        d.E = padE[i];
        d.B = padB[i];
        d.mE = (s.flags & 2) ? padA[i] : padE[i];
        d.kind = s.kind;
        d.flags = s.flags & 15;
        d.pa = (uint8_t)(base + s.dir);
        d.pap = (uint8_t)(base + lat.opp[s.dir]);
        d.field = s.field;
        d.caxis = s.field == 2 ? s.comp : 0;
        d.ex = (int8_t)lat.e[s.dir][0];
        d.ey = (int8_t)lat.e[s.dir][1];
        d.ez = (int8_t)lat.e[s.dir][2];
        d.d = (R)s.d;
        // given values enter as deviations from the rest state, formed in
        // double precision so that small differences survive FP32
        double rest = 0.0;
        if (s.kind == LBM_LK_PRES) rest = c->p.rho0;
        else if (s.kind == LBM_LK_CONC) rest = c->p.C0;
        else if (s.kind == LBM_LK_MAG_DIR) rest = c->p.B_ext[s.comp];
        d.value = (R)(s.value - rest);
        d.a1 = (R)s.a1;
        d.a3 = (R)s.a3;
        d.quad = (R)s.quad;
        d.weight = (R)s.weight;
        d.uw0 = (R)s.u_w[0];
        d.uw1 = (R)s.u_w[1];
        d.uw2 = (R)s.u_w[2];
        d.need = moments_needed(s, lat.e[s.dir]);
        d.cslot = (uint8_t)(s.field == 1 ? cslot(s.comp) : 4);
        if (s.field == 1 && s.kind == LBM_LK_FLUX && s.cross != 0.0) {
            d.pslot = (uint8_t)(cslot(s.cross_comp[0]) | (cslot(s.cross_comp[1]) << 4));
            d.value = (R)s.cross;  // a FLUX link has no given value
        }
        out[i] = d;
    }
}

// A boundary's flux law (lbm_flux_law) fits its kind and has valid data.
bool valid_law(const lbm_bc& bc) {
    if (bc.profile_len < 0 || (bc.profile_len > 0 && (!bc.profile || bc.profile_axis < 0 || bc.profile_axis > 2)))
        return false;
    switch (bc.law) {
        case LBM_LAW_COEF:
            return true;
        case LBM_LAW_ROBIN:
        case LBM_LAW_REACTION:
            if (bc.kind != LBM_LK_FLUX || !(bc.k >= 0.0) || !std::isfinite(bc.k) || !std::isfinite(bc.phi_eq))
                return false;
            for (int i = 0; i < bc.profile_len; ++i)
                if (!(bc.profile[i] >= 0.0) || !std::isfinite(bc.profile[i])) return false;
            return true;
        case LBM_LAW_SHERCLIFF:
            if (bc.kind != LBM_LK_MAG_FLUX && bc.kind != LBM_LK_MAG_THETA) return false;
            if (bc.profile_len > 0 || !(bc.c_w > 0.0) || !(bc.H > 0.0) || !std::isfinite(bc.H)) return false;
            return bc.kind == LBM_LK_MAG_FLUX || std::isfinite(bc.c_w);
        default:
            return false;
    }
}

}  // namespace lbmh

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* lbm_version(void) { return "liblbm 0.1 (gfx950, AA-pattern fused coupled sweep)"; }

lbm_status lbm_lattice_table(int32_t lattice, int32_t* Q, int32_t* e, double* w, double* c2, int32_t* opp) {
    if (lattice < LBM_D2Q9 || lattice > LBM_D3Q7 || !Q || !e || !w || !c2 || !opp) return LBM_EINVAL;
    const HostLat L = lattice_of(lattice);
    *Q = L.Q;
    *c2 = L.c2;
    for (int a = 0; a < L.Q; ++a) {
        for (int k = 0; k < 3; ++k) e[3 * a + k] = L.e[a][k];
        w[a] = L.w[a];
        opp[a] = L.opp[a];
    }
    return LBM_OK;
}

lbm_status lbm_build_links(const lbm_params* p, const lbm_boundary* bnds, int32_t nb, uint8_t* mask_out,
                           lbm_link* links_out, size_t cap, size_t* n_out) {
    std::string why;
    if (!valid_params(p, &why) || nb < 0 || (nb > 0 && !bnds) || !n_out) return LBM_EINVAL;
    for (int i = 0; i < nb; ++i) {
        const lbm_boundary& b = bnds[i];
        if (b.type < 0 || b.type > 2) return LBM_EINVAL;
        if (b.axis < 0 || b.axis > 2) return LBM_EINVAL;
        if (b.type == 0 && !(b.q > 0.0 && b.q <= 1.0)) return LBM_EINVAL;
        if (b.type == 1 && !(b.radius > 0.0)) return LBM_EINVAL;
        if (b.type == 2)
            for (int k = 0; k < 3; ++k)
                if (!(b.lo[k] <= b.hi[k])) return LBM_EINVAL;
        if (!(b.d_scheme == 0.0 || (b.d_scheme > 0.0 && b.d_scheme <= 1.0))) return LBM_EINVAL;
        const int ns = scalar_comps(p);
        for (int k = 1; k < ns; ++k)
            if ((b.h_more[k - 1].kind != 0) != (b.h.kind != 0)) return LBM_EINVAL;
        for (int k = 0; k < 3; ++k) {
            const lbm_bc& bc = k == 0 ? b.h : b.h_more[k - 1];
            if (!std::isfinite(bc.cross)) return LBM_EINVAL;
            if (bc.cross == 0.0 || k >= ns) continue;
            if (bc.kind != LBM_LK_FLUX || bc.law != LBM_LAW_COEF || ns < 2)
                return LBM_EINVAL;
            for (int j = 0; j < 2; ++j)
                if (bc.cross_comp[j] < 0 || bc.cross_comp[j] >= ns) return LBM_EINVAL;
        }
        const lbm_bc* bcs[7] = {&b.f, &b.h, &b.g[0], &b.g[1], &b.g[2], &b.h_more[0], &b.h_more[1]};
        for (const lbm_bc* bc : bcs) {
            if (bc->alt && !(bc->kind == LBM_LK_VEL || bc->kind == LBM_LK_PRES || bc->kind == LBM_LK_FLUX ||
                             bc->kind == LBM_LK_MAG_FLUX))
                return LBM_EINVAL;
            if (!valid_law(*bc)) return LBM_EINVAL;
        }
    }
    LinkBuilder lb(*p, bnds, nb);
    std::vector<lbm_link> links;
    const std::string e = lb.build(&links);
    if (!e.empty()) return LBM_EINVAL;
    *n_out = links.size();
    if (mask_out) std::memcpy(mask_out, lb.mask().data(), lb.mask().size());
    if (links_out) {
        if (cap < links.size()) return LBM_ESIZE;
        std::memcpy(links_out, links.data(), links.size() * sizeof(lbm_link));
    }
    return LBM_OK;
}

size_t lbm_required_bytes(const lbm_params* p, size_t n_links, size_t sizes_out[LBM_NBUF]) {
    if (!valid_params(p, nullptr)) return 0;
    size_t sz[LBM_NBUF];
    layout(p, n_links, sz);
    size_t tot = 0;
    for (int i = 0; i < LBM_NBUF; ++i) {
        if (sizes_out) sizes_out[i] = sz[i];
        tot += sz[i];
    }
    return tot;
}

lbm_status lbm_create(const lbm_params* p, size_t n_links, void* const dev_bufs[LBM_NBUF], void* hip_stream,
                      lbm_ctx** out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    std::string why;
    if (!valid_params(p, &why) || !dev_bufs) return LBM_EINVAL;
    lbmi::KernelSet ks = kernels_for(p);
    if (!ks.step) return LBM_EINVAL;
    size_t sz[LBM_NBUF];
    layout(p, n_links, sz);
    for (int i = 0; i < LBM_NBUF; ++i) {
        if (sz[i] > 0 && !dev_bufs[i]) return LBM_EINVAL;
        if (sz[i] > 0 && ((uintptr_t)dev_bufs[i] % kAlign) != 0) return LBM_EINVAL;
    }
    lbm_ctx* c = new lbm_ctx();
    c->p = *p;
    c->pad = padding(p);
    c->ks = ks;
    for (int i = 0; i < LBM_NBUF; ++i) {
        c->buf[i] = dev_bufs[i];
        c->size[i] = sz[i];
    }
    c->cap_links = n_links;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
    *out = c;
    return LBM_OK;
}

lbm_status lbm_set_geometry(lbm_ctx* c, const uint8_t* host_mask) {
    if (!c) return LBM_EINVAL;
    if (!host_mask) return set_err(c, LBM_EINVAL, "mask is NULL");
    const size_t N = domain_nodes(c->p);
    c->mask.assign(host_mask, host_mask + N);
    for (auto& m : c->mask) m = m ? 1 : 0;
    c->have_geometry = true;
    c->have_links = false;
    c->initialized = false;
    return LBM_OK;
}

lbm_status lbm_set_links(lbm_ctx* c, const lbm_link* L, size_t n) {
    if (!c) return LBM_EINVAL;
    if (!c->have_geometry) return set_err(c, LBM_ESTATE, "lbm_set_geometry must come first");
    if (n > c->cap_links) return set_err(c, LBM_ESIZE, "more links than the context was created for");
    if (n > 0 && !L) return set_err(c, LBM_EINVAL, "links is NULL");
    const lbm_params& p = c->p;
    const Pad& d = c->pad;
    const size_t N = domain_nodes(p);
    const int codes[3] = {p.fluid, p.scalar, p.magnetic};
    HostLat lats[3] = {lattice_of(p.fluid), lattice_of(p.scalar), lattice_of(p.magnetic)};
    auto coords = [&](uint32_t i, int* q) {
        q[0] = (int)(i % (uint32_t)p.n[0]);
        q[1] = (int)((i / (uint32_t)p.n[0]) % (uint32_t)p.n[1]);
        q[2] = (int)(i / ((uint32_t)p.n[0] * (uint32_t)p.n[1]));
    };
    auto wrap = [&](int* q) {
        for (int k = 0; k < 3; ++k) {
            if (q[k] >= 0 && q[k] < p.n[k]) continue;
            if (!p.periodic[k]) return false;
            q[k] = ((q[k] % p.n[k]) + p.n[k]) % p.n[k];
        }
        return true;
    };
    auto dom = [&](const int* q) { return (size_t)q[0] + (size_t)p.n[0] * ((size_t)q[1] + (size_t)p.n[1] * q[2]); };
    auto padidx = [&](const int* q) {
        return (uint32_t)((q[0] + d.hx) + (size_t)d.NX * ((q[1] + d.hy) + (size_t)d.NY * (q[2] + d.hz)));
    };

    // validate each link; mark the (node, slot) pairs it covers
    const int QF = lats[0].Q, QH = p.scalar ? lats[1].Q : 0, QG = p.magnetic ? lats[2].Q : 0;
    const int NS = scalar_comps(&p);
    const int QT = QF + NS * QH + p.mag_ncomp * QG;
    auto plane_base = [&](int field, int comp) {
        return field == 0 ? 0 : (field == 1 ? QF + comp * QH : QF + NS * QH + comp * QG);
    };
    std::vector<uint8_t> covered(N * (size_t)QT, 0);
    std::vector<lbm_link> links(L, L + n);
    for (size_t i = 0; i < n; ++i) {
        const lbm_link& k = links[i];
        char msg[200];
        auto bad = [&](const char* why) {
            snprintf(msg, sizeof msg, "link %zu (node %u field %u dir %u): %s", i, k.node, k.field, k.dir, why);
            return set_err(c, LBM_EINVAL, msg);
        };
        if (k.node >= N || !c->mask[k.node]) return bad("A is not a fluid node");
        if (k.field > 2 || !codes[k.field]) return bad("field has no lattice");
        const HostLat& lat = lats[k.field];
        if (k.dir < 1 || k.dir >= lat.Q) return bad("direction out of range");
        if (k.field == 2 ? k.comp >= p.mag_ncomp : (k.field == 1 ? k.comp >= NS : k.comp != 0))
            return bad("component out of range");
        const bool okkind = k.field == 0 ? (k.kind == LBM_LK_VEL || k.kind == LBM_LK_PRES)
                            : k.field == 1 ? (k.kind == LBM_LK_CONC || k.kind == LBM_LK_FLUX || k.kind == LBM_LK_BB0)
                                           : (k.kind == LBM_LK_MAG_DIR || k.kind == LBM_LK_MAG_FLUX || k.kind == LBM_LK_BB0 ||
                                              k.kind == LBM_LK_MAG_THETA);
        if (!okkind) return bad("kind not allowed for this field");
        if (!(k.d > 0.0 && k.d <= 1.0)) return bad("d outside (0, 1]");
        if (k.flags & ~15u) return bad("unknown flag bits");
        if ((k.flags & 8) && !(k.kind == LBM_LK_VEL || k.kind == LBM_LK_PRES || k.kind == LBM_LK_FLUX ||
                               k.kind == LBM_LK_MAG_FLUX))
            return bad("flag bit 3 (comparison form) needs kind VEL, PRES, FLUX or MAG_FLUX");
        if (k.kind == LBM_LK_MAG_THETA && !(k.a1 >= 0.0)) return bad("theta (a1) must be >= 0");
        // the theta form assumes one crossing link per wall node (D2Q5 / D3Q7)
        if (k.field == 2 && p.magnetic == LBM_D3Q19 && k.kind == LBM_LK_MAG_THETA)
            return bad("the theta form needs a D2Q5 or D3Q7 magnetic lattice");
        if ((k.flags & 4) && !(k.flags & 1)) return bad("an oscillating boundary velocity needs flag bit 0 (u_w given)");
        if (!std::isfinite(k.value) || !std::isfinite(k.a1) || !std::isfinite(k.a3) || !std::isfinite(k.weight) ||
            !std::isfinite(k.quad))
            return bad("non-finite wall data");
        if (k.quad != 0.0 && k.kind != LBM_LK_FLUX && k.kind != LBM_LK_MAG_FLUX)
            return bad("quad (quadratic flux term) needs kind FLUX or MAG_FLUX");
        if (!std::isfinite(k.cross)) return bad("non-finite cross coefficient");
        if (k.cross != 0.0 && (k.kind != LBM_LK_FLUX || NS < 2 || k.cross_comp[0] >= NS || k.cross_comp[1] >= NS))
            return bad("a bilinear flux term needs kind FLUX, several scalar components and components below "
                       "scalar_ncomp");
        int q[3];
        coords(k.node, q);
        int s[3] = {q[0] - lat.e[k.dir][0], q[1] - lat.e[k.dir][1], q[2] - lat.e[k.dir][2]};
        if (wrap(s) && c->mask[dom(s)]) return bad("the source node is fluid (population is known)");
        if (!(k.flags & 2)) {
            int e[3] = {q[0] + lat.e[k.dir][0], q[1] + lat.e[k.dir][1], q[2] + lat.e[k.dir][2]};
            if (!wrap(e) || !c->mask[dom(e)] || dom(e) != k.enode) return bad("enode is not the fluid node A + e_alpha");
        }
        const int base = plane_base(k.field, k.comp);
        uint8_t& cov = covered[(size_t)k.node * QT + base + k.dir];
        if (cov) return bad("duplicate link");
        cov = 1;
    }
    // completeness: every unknown population has a link
    for (size_t i = 0; i < N; ++i) {
        if (!c->mask[i]) continue;
        int q[3];
        coords((uint32_t)i, q);
        for (int f = 0; f < 3; ++f) {
            if (!codes[f]) continue;
            const HostLat& lat = lats[f];
            const int nc = f == 2 ? p.mag_ncomp : (f == 1 ? NS : 1);
            for (int a = 1; a < lat.Q; ++a) {
                int s[3] = {q[0] - lat.e[a][0], q[1] - lat.e[a][1], q[2] - lat.e[a][2]};
                if (wrap(s) && c->mask[dom(s)]) continue;
                for (int cc = 0; cc < nc; ++cc) {
                    const int base = plane_base(f, cc);
                    if (!covered[i * QT + base + a]) {
                        char msg[160];
                        snprintf(msg, sizeof msg, "node %zu field %d dir %d comp %d has no boundary link", i, f, a, cc);
                        return set_err(c, LBM_EINVAL, msg);
                    }
                }
            }
        }
    }

    // order by padded node; padded indices of A, of E = A + e_alpha and of
    // B = A - e_alpha (the latter two with periodic wrap, fluid or not)
    auto padwrap = [&](const int* q) {
        int w[3];
        for (int k = 0; k < 3; ++k) {
            w[k] = q[k];
            if (p.periodic[k]) w[k] = ((w[k] % p.n[k]) + p.n[k]) % p.n[k];
        }
        return (uint32_t)((w[0] + d.hx) + (size_t)d.NX * ((w[1] + d.hy) + (size_t)d.NY * (w[2] + d.hz)));
    };
    std::vector<uint32_t> padA(n), padE(n), padB(n);
    for (size_t i = 0; i < n; ++i) {
        const HostLat& lat = lats[links[i].field];
        int q[3];
        coords(links[i].node, q);
        padA[i] = padidx(q);
        const int* e = lat.e[links[i].dir];
        const int qe[3] = {q[0] + e[0], q[1] + e[1], q[2] + e[2]};
        const int qb[3] = {q[0] - e[0], q[1] - e[1], q[2] - e[2]};
        padE[i] = padwrap(qe);
        padB[i] = padwrap(qb);
    }
    std::vector<size_t> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = i;
    // device order (the result does not depend on it: no link reads a slot
    // another link writes).  3D lattices and items of a batch: by plane
    // (field, component, direction), then node, so that the links of one
    // direction along a wall share a wave and their population accesses
    // coalesce.  2D single lattices: by node, then plane; plane order made the
    // step of the 512 x 256 reactive channel 15 % slower.
    const bool plane_first = c->p.dim == 3 || c->batch_owned;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        const lbm_link &u = links[a], &v = links[b];
        if (!plane_first && padA[a] != padA[b]) return padA[a] < padA[b];
        if (u.field != v.field) return u.field < v.field;
        if (u.comp != v.comp) return u.comp < v.comp;
        if (u.dir != v.dir) return u.dir < v.dir;
        return padA[a] < padA[b];
    });
    std::vector<lbm_link> sl(n);
    std::vector<uint32_t> sA(n), sE(n), sB(n);
    for (size_t i = 0; i < n; ++i) {
        sl[i] = links[order[i]];
        sA[i] = padA[order[i]];
        sE[i] = padE[order[i]];
        sB[i] = padB[order[i]];
    }
    std::vector<uint8_t> flags(round_up(d.plane, kAlign) + d.plane / 64, 0);
    for (size_t i = 0; i < N; ++i)
        if (c->mask[i]) {
            int q[3];
            coords((uint32_t)i, q);
            flags[padidx(q)] = lbmi::NF_FLUID;
        }
    for (size_t i = 0; i < n; ++i) {
        flags[sA[i]] |= lbmi::NF_LINKS | lbmi::NF_MOM;
        if (!(sl[i].flags & 2)) flags[sE[i]] |= lbmi::NF_MOM;
    }
    // one byte per 64 padded nodes: 1 when every node of the group is fluid
    const size_t wf0 = round_up(d.plane, kAlign);
    for (size_t g = 0; g < d.plane / 64; ++g) {
        bool all = true;
        for (size_t k = 64 * g; k < 64 * g + 64 && all; ++k) all = k < d.nodes && (flags[k] & lbmi::NF_FLUID);
        flags[wf0 + g] = all ? 1 : 0;
    }
    // waves of the link nodes A and their partners E (their slots carry the
    // link kernel's inputs and its result), then every other wave with a
    // fluid node; the two lists are swept as separate launches in captured runs
    const size_t nw = d.plane / 64;
    std::vector<uint8_t> bnd(nw, 0);
    for (size_t i = 0; i < n; ++i) {
        bnd[sA[i] / 64] = 1;
        bnd[sE[i] / 64] = 1;
    }
    std::vector<uint32_t> wl;
    wl.reserve(nw);
    for (size_t g = 0; g < nw; ++g)
        if (bnd[g]) wl.push_back((uint32_t)g);
    const size_t n_bnd = wl.size();
    for (size_t g = 0; g < nw; ++g) {
        if (bnd[g]) continue;
        bool any = false;
        for (size_t k = 64 * g; k < 64 * g + 64 && !any; ++k) any = k < d.nodes && (flags[k] & lbmi::NF_FLUID);
        if (any) wl.push_back((uint32_t)g);
    }

    std::vector<unsigned char> dl;
    if (p.storage == LBM_F64) fill_devlinks<double>(c, sl, sA, sE, sB, &dl);
    else fill_devlinks<float>(c, sl, sA, sE, sB, &dl);

    lbm_status st;
    if ((st = hip_check(c, hipMemcpyAsync(c->buf[1], flags.data(), flags.size(), hipMemcpyHostToDevice, c->stream), "flags upload")))
        return st;
    if ((st = hip_check(c, hipMemcpyAsync(c->buf[2], dl.data(), dl.size(), hipMemcpyHostToDevice, c->stream), "links upload")))
        return st;
    if (!wl.empty() && (st = hip_check(c, hipMemcpyAsync(wave_lists(c), wl.data(), wl.size() * 4,
                                                          hipMemcpyHostToDevice, c->stream), "wave list upload")))
        return st;
    if ((st = hip_check(c, hipMemsetAsync(c->buf[3], 0, c->size[3], c->stream), "moment clear"))) return st;
    if ((st = hip_check(c, hipStreamSynchronize(c->stream), "link upload sync"))) return st;
    c->n_links = n;
    c->n_wave_bnd = n_bnd;
    c->n_wave_int = wl.size() - n_bnd;
    c->cmp_links = false;
    for (size_t i = 0; i < n; ++i)
        if ((L[i].flags & 8) || L[i].kind == LBM_LK_MAG_THETA) c->cmp_links = true;
    drop_graph(c);
    c->have_links = true;
    c->initialized = false;
    c->t = 0;
    c->snap_valid = false;
    return LBM_OK;
}

lbm_status lbm_init(lbm_ctx* c, const double* rho, const double* u, const double* C, const double* B) {
    if (!c) return LBM_EINVAL;
    if (!c->have_links) return set_err(c, LBM_ESTATE, "lbm_set_links must come first");
    lbm_status st;
    if ((st = hip_check(c, hipMemsetAsync(c->buf[0], 0, c->size[0], c->stream), "population clear"))) return st;
    lbmi::KArgs a = base_args(c);
    a.init_rho = rho;
    a.init_u = u;
    a.init_C = C;
    a.init_B = B;
    if ((st = hip_check(c, c->ks.init(a), "init launch"))) return st;
    c->t = 0;
    c->initialized = true;
    c->snap_valid = false;
    return LBM_OK;
}

namespace {

// Captures `steps` steps starting at a time of the given parity with links
// ready.  The capture runs on a private stream (the caller's stream may be the
// legacy default stream, which cannot be captured); the launch arguments do
// not depend on the time beyond its parity: each launch reads the time of its
// step from the time-base word, which the run advances at its end.
lbm_status make_graph(lbm_ctx* c, int parity, int64_t steps, lbm_ctx::StepGraph* out) {
    if (!c->capture_stream) {
        if (hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess) {
            c->capture_stream = nullptr;
            return LBM_EDEVICE;
        }
    }
    if (out->exec) (void)hipGraphExecDestroy(out->exec);
    *out = lbm_ctx::StepGraph();
    lbmi::KArgs a = base_args(c);
    a.stream = c->capture_stream;
    a.links_ready = 1;
    a.tbase = time_base(c);
    const bool split = c->n_links > 0 && c->n_wave_bnd > 0 && c->overlap_mode == 1;
    if (split && !c->capture_stream2) {
        if (hipStreamCreateWithFlags(&c->capture_stream2, hipStreamNonBlocking) != hipSuccess) {
            c->capture_stream2 = nullptr;
            return LBM_EDEVICE;
        }
        for (hipEvent_t* e : {&c->ev_links, &c->ev_bnd, &c->ev_fork, &c->ev_join})
            if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
                *e = nullptr;
                return LBM_EDEVICE;
            }
    }
    if (hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return LBM_EDEVICE;
    hipError_t le = hipSuccess;
    if (!split) {
        for (int64_t i = 0; i < steps && le == hipSuccess; ++i) {
            a.parity = (int)((parity + i) & 1);
            a.tstep = (uint32_t)i;
            le = c->ks.step(a);
        }
    } else {
        // Step i: links(i) on the second stream; then, on the first, the
        // sweep of the boundary waves (after links(i)) and of the interior
        // waves.  links(i + 1) waits for the boundary sweep of step i only:
        // it reads slots that only threads of A and E nodes write, and writes
        // slots no thread of either sweep touches, so it overlaps the
        // interior sweep of step i.
        const hipStream_t s0 = c->capture_stream, s1 = c->capture_stream2;
        uint32_t* wl = wave_lists(c);
        auto ok = [&](hipError_t e) { if (le == hipSuccess) le = e; return le == hipSuccess; };
        ok(hipEventRecord(c->ev_fork, s0));
        ok(hipStreamWaitEvent(s1, c->ev_fork, 0));
        for (int64_t i = 0; i < steps && le == hipSuccess; ++i) {
            a.parity = (int)((parity + i) & 1);
            a.tstep = (uint32_t)i;
            a.stream = s1;
            if (!ok(c->ks.links(a)) || !ok(hipEventRecord(c->ev_links, s1))) break;
            a.stream = s0;
            if (!ok(hipStreamWaitEvent(s0, c->ev_links, 0))) break;
            a.waves = wl;
            a.n_waves = (uint32_t)c->n_wave_bnd;
            if (!ok(c->ks.sweep_waves(a)) || !ok(hipEventRecord(c->ev_bnd, s0))) break;
            a.waves = wl + c->n_wave_bnd;
            a.n_waves = (uint32_t)c->n_wave_int;
            if (!ok(c->ks.sweep_waves(a)) || !ok(hipStreamWaitEvent(s1, c->ev_bnd, 0))) break;
        }
        // the second stream joins the first before the capture ends
        ok(hipEventRecord(c->ev_join, s1));
        ok(hipStreamWaitEvent(s0, c->ev_join, 0));
        a.stream = s0;
        a.waves = nullptr;
        a.n_waves = 0;
    }
    if (le == hipSuccess) {
        // the time base follows the run
        a.tstep = (uint32_t)steps;
        le = c->ks.tick(a);
    }
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(c->capture_stream, &g);
    if (le != hipSuccess || ee != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return LBM_EDEVICE;
    }
    hipGraphExec_t exec = nullptr;
    hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return LBM_EDEVICE;
    out->exec = exec;
    out->parity = parity;
    out->steps = steps;
    return LBM_OK;
}

// The captured run lbm_step replays next from a time of parity `par` with n
// steps left (n >= 2): graph_steps steps when n allows, else all n.  Captures
// it when missing; null when capture failed (lbm_step then launches singly).
lbm_ctx::StepGraph* run_for(lbm_ctx* c, int par, int64_t n) {
    if (c->graph_failed) return nullptr;
    lbm_ctx::StepGraph* g = n >= c->graph_steps ? &c->run[par] : &c->tail;
    const int64_t steps = n >= c->graph_steps ? c->graph_steps : n;
    if (g->exec && g->parity == par && g->steps == steps) return g;
    if (make_graph(c, par, steps, g) != LBM_OK) {
        c->graph_failed = true;  // fall back to single launches of the same kernels
        (void)hipGetLastError();
        return nullptr;
    }
    return g;
}

lbm_status step_launches(lbm_ctx* c, int64_t n) {
    lbmi::KArgs a = base_args(c);
    for (int64_t i = 0; i < n; ++i) {
        a.parity = (int)(c->t & 1);
        a.links_ready = c->t > 0 ? 1 : 0;
        a.tstep = (uint32_t)c->t;
        lbm_status st = hip_check(c, c->ks.step(a), "step launch");
        if (st) return st;
        c->t++;
    }
    return LBM_OK;
}

}  // namespace

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
    if (!c) return LBM_EINVAL;
    if (n < 0) return set_err(c, LBM_EINVAL, "negative step count");
    if (!c->initialized) return set_err(c, LBM_ESTATE, "lbm_init must come first");
    lbm_status st;
    // the first step reads the initial populations (no link values yet)
    if (n > 0 && c->t == 0) {
        if ((st = step_launches(c, 1))) return st;
        c->n_plain_steps++;
        --n;
    }
    // captured runs: graph_steps steps while they fit, then one run of the
    // rest; runs start from the context's time, whatever its parity
    bool timed = false;
    while (n >= 2) {
        lbm_ctx::StepGraph* g = run_for(c, (int)(c->t & 1), n);
        if (!g) break;
        if (!timed) {
            lbmi::KArgs a = base_args(c);
            a.tbase = time_base(c);
            a.tstep = (uint32_t)c->t;
            if ((st = hip_check(c, c->ks.set_time(a), "time base"))) return st;
            timed = true;
        }
        if ((st = hip_check(c, hipGraphLaunch(g->exec, c->stream), "graph launch"))) return st;
        c->t += g->steps;
        n -= g->steps;
        c->n_graph_launches++;
        c->n_graph_steps += g->steps;
    }
    c->n_plain_steps += n;
    return step_launches(c, n);
}

lbm_status lbm_step_prepare(lbm_ctx* c, int64_t n) {
    if (!c) return LBM_EINVAL;
    if (n < 0) return set_err(c, LBM_EINVAL, "negative step count");
    if (!c->initialized) return set_err(c, LBM_ESTATE, "lbm_init must come first");
    int64_t t = c->t;
    if (n > 0 && t == 0) {
        ++t;
        --n;
    }
    // graph_steps is even: every full run starts at the same parity
    if (n >= c->graph_steps && !run_for(c, (int)(t & 1), n)) return set_err(c, LBM_EDEVICE, "graph capture");
    const int64_t r = n % c->graph_steps;
    if (r >= 2 && !run_for(c, (int)((t + n - r) & 1), r)) return set_err(c, LBM_EDEVICE, "graph capture");
    return LBM_OK;
}

lbm_status lbm_set_step_overlap(lbm_ctx* c, int32_t mode) {
    if (!c) return LBM_EINVAL;
    if (mode < 0 || mode > 1) return set_err(c, LBM_EINVAL, "overlap mode must be 0 or 1");
    if (mode != c->overlap_mode) drop_graph(c);
    c->overlap_mode = mode;
    return LBM_OK;
}

lbm_status lbm_step_stats(const lbm_ctx* c, int64_t out[3]) {
    if (!c || !out) return LBM_EINVAL;
    out[0] = c->n_graph_launches;
    out[1] = c->n_graph_steps;
    out[2] = c->n_plain_steps;
    return LBM_OK;
}

namespace {

// One graph of n launches of a single kernel of the step (links or sweep),
// parities alternating from the context's time.
lbm_status capture_kernel(lbm_ctx* c, int64_t n, bool links, hipGraphExec_t* out) {
    *out = nullptr;
    if (!c->capture_stream && hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        c->capture_stream = nullptr;
        return set_err(c, LBM_EDEVICE, "capture stream");
    }
    lbmi::KArgs a = base_args(c);
    a.stream = c->capture_stream;
    a.links_ready = 1;
    if (hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return set_err(c, LBM_EDEVICE, "begin capture");
    hipError_t le = hipSuccess;
    for (int64_t i = 0; i < n && le == hipSuccess; ++i) {
        a.parity = (int)((c->t + i) & 1);
        a.tstep = (uint32_t)(c->t + i);
        le = links ? c->ks.links(a) : c->ks.sweep(a);
    }
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(c->capture_stream, &g);
    if (le != hipSuccess || ee != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return set_err(c, LBM_EDEVICE, "kernel capture");
    }
    hipError_t ie = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        *out = nullptr;
        return set_err(c, LBM_EDEVICE, "graph instantiate");
    }
    return LBM_OK;
}

}  // namespace

size_t lbm_timing_scratch_bytes(const lbm_ctx* c) { return c ? c->size[0] + c->size[3] : 0; }

lbm_status lbm_step_timed(lbm_ctx* c, int64_t n, void* dev_scratch, size_t scratch_bytes, float ms_out[2]) {
    if (!c || !ms_out) return LBM_EINVAL;
    if (n < 2 || n > 4096 || (n & 1)) return set_err(c, LBM_EINVAL, "launch count must be even, 2 to 4096");
    if (!c->initialized) return set_err(c, LBM_ESTATE, "lbm_init must come first");
    if (c->batch_owned) return set_err(c, LBM_EINVAL, "an item of a batch is timed through the batch");
    // the launches below do not form steps: populations and moments (with the
    // time base word) are saved into the caller's scratch first and restored
    // afterwards
    const size_t s0 = c->size[0], s3 = c->size[3];
    if (!dev_scratch) return set_err(c, LBM_EINVAL, "no scratch buffer");
    if (scratch_bytes < s0 + s3) return set_err(c, LBM_ESIZE, "scratch buffer smaller than lbm_timing_scratch_bytes");
    ms_out[0] = ms_out[1] = 0.f;
    void* save = dev_scratch;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipGraphExec_t g[2] = {nullptr, nullptr};
    lbm_status st = hip_check(c, hipMemcpyAsync(save, c->buf[0], s0, hipMemcpyDeviceToDevice, c->stream), "state save");
    if (!st) st = hip_check(c, hipMemcpyAsync((char*)save + s0, c->buf[3], s3, hipMemcpyDeviceToDevice, c->stream),
                            "state save");
    if (!st && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = set_err(c, LBM_EDEVICE, "event create");
    for (int k = 0; k < 2 && !st; ++k) {
        const bool links = k == 0;
        if (links && c->n_links == 0) continue;
        if ((st = capture_kernel(c, n, links, &g[k]))) break;
        // one untimed replay, then the timed one
        if ((st = hip_check(c, hipGraphLaunch(g[k], c->stream), "graph launch"))) break;
        if ((st = hip_check(c, hipEventRecord(e0, c->stream), "event record"))) break;
        if ((st = hip_check(c, hipGraphLaunch(g[k], c->stream), "graph launch"))) break;
        if ((st = hip_check(c, hipEventRecord(e1, c->stream), "event record"))) break;
        if ((st = hip_check(c, hipEventSynchronize(e1), "event sync"))) break;
        float ms = 0.f;
        if ((st = hip_check(c, hipEventElapsedTime(&ms, e0, e1), "event elapsed time"))) break;
        ms_out[k] = ms / (float)n;
    }
    // the restore runs whatever happened above
    lbm_status rs = hip_check(c, hipMemcpyAsync(c->buf[0], save, s0, hipMemcpyDeviceToDevice, c->stream), "state restore");
    if (!rs) rs = hip_check(c, hipMemcpyAsync(c->buf[3], (char*)save + s0, s3, hipMemcpyDeviceToDevice, c->stream),
                            "state restore");
    if (!rs) rs = hip_check(c, hipStreamSynchronize(c->stream), "state restore");
    for (auto& x : g)
        if (x) (void)hipGraphExecDestroy(x);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return st ? st : rs;
}

lbm_status lbm_read_moments(lbm_ctx* c, void* dev_out, int32_t out_type) {
    if (!c) return LBM_EINVAL;
    if (!dev_out || (out_type != LBM_F64 && out_type != LBM_F32)) return set_err(c, LBM_EINVAL, "bad output");
    if (!c->initialized) return set_err(c, LBM_ESTATE, "lbm_init must come first");
    lbmi::KArgs a = base_args(c);
    a.mode = lbmi::OBS_MOMENTS;
    a.out = dev_out;
    a.out_f64 = out_type == LBM_F64;
    return hip_check(c, c->ks.observe(a), "moments launch");
}

lbm_status lbm_read_populations(lbm_ctx* c, int32_t field, double* dev_out) {
    if (!c) return LBM_EINVAL;
    const int codes[3] = {c->p.fluid, c->p.scalar, c->p.magnetic};
    if (!dev_out || field < 0 || field > 2 || !codes[field]) return set_err(c, LBM_EINVAL, "bad field or output");
    if (!c->initialized) return set_err(c, LBM_ESTATE, "lbm_init must come first");
    lbmi::KArgs a = base_args(c);
    a.mode = lbmi::OBS_POPS;
    a.field = field;
    a.out = dev_out;
    return hip_check(c, c->ks.observe(a), "populations launch");
}

lbm_status lbm_read_normalised(lbm_ctx* c, int32_t axis, double U, double* dev_out) {
    if (!c) return LBM_EINVAL;
    if (!dev_out || axis < 0 || axis > 2 || !(U >= 0.0) || !std::isfinite(U))
        return set_err(c, LBM_EINVAL, "bad axis, velocity scale or output");
    if (!c->initialized) return set_err(c, LBM_ESTATE, "lbm_init must come first");
    const size_t cb = compute_bytes(c->p.storage);
    double* acc = (double*)((char*)c->buf[4] + round_up((size_t)(moment_planes(&c->p) - 1) * c->pad.plane * cb, kAlign));
    lbm_status st;
    if ((st = hip_check(c, hipMemsetAsync(acc, 0, lbmi::NACC * sizeof(double), c->stream), "accumulator clear")))
        return st;
    lbmi::KArgs a = base_args(c);
    a.mode = lbmi::OBS_NORM;
    a.field = axis;
    a.out = dev_out;
    a.acc = acc;
    if ((st = hip_check(c, c->ks.observe(a), "normalised moments launch"))) return st;
    if (U == 0.0) {  // the mean velocity over the fluid nodes
        double h[2];
        if ((st = hip_check(c, hipMemcpyAsync(h, acc, sizeof h, hipMemcpyDeviceToHost, c->stream), "mean copy")))
            return st;
        if ((st = hip_check(c, hipStreamSynchronize(c->stream), "mean sync"))) return st;
        U = h[1] > 0.0 ? h[0] / h[1] : 0.0;
        if (!(U != 0.0) || !std::isfinite(U)) return set_err(c, LBM_EINVAL, "the mean velocity is zero or not finite");
    }
    // B* = B / (U mu sqrt(rho0 nu sigma)), sigma = 1 / (mu eta): sqrt(rho0 nu mu / eta)
    const double nu = (c->p.tau_f - 0.5) / 3.0;
    const double cg2 = c->p.magnetic == LBM_D3Q19 ? 1.0 / 3.0 : 0.25;
    const double eta = c->p.magnetic ? cg2 * (c->p.tau_m - 0.5) : 1.0;
    const double mu = c->p.magnetic ? c->p.mu : 1.0;
    a.norm_u = U;
    a.norm_b = std::sqrt(c->p.rho0 * nu * mu / eta);
    return hip_check(c, c->ks.scale(a), "normalisation launch");
}

namespace {

// the link kernel of the current step with its net inflows by slot: 0 f,
// 1 h (C_0), 2..4 g (B_x, B_y, B_z), 5..6 C_1, C_2
lbm_status run_flux(lbm_ctx* c, double h[7]) {
    for (int q = 0; q < 7; ++q) h[q] = 0.0;
    if (!c->initialized) return set_err(c, LBM_ESTATE, "lbm_init must come first");
    if (c->t == 0) return set_err(c, LBM_ESTATE, "no step has been taken");
    if (c->n_links == 0) return LBM_OK;
    const size_t cb = compute_bytes(c->p.storage);
    char* aux = (char*)c->buf[4];
    double* acc = (double*)(aux + round_up((size_t)(moment_planes(&c->p) - 1) * c->pad.plane * cb, kAlign));  // the reduction accumulators
    lbm_status st;
    if ((st = hip_check(c, hipMemsetAsync(acc, 0, lbmi::NACC * sizeof(double), c->stream), "accumulator clear")))
        return st;
    lbmi::KArgs a = base_args(c);
    a.acc = acc;
    if ((st = hip_check(c, c->ks.flux(a), "flux launch"))) return st;
    if ((st = hip_check(c, hipMemcpyAsync(h, acc, 7 * sizeof(double), hipMemcpyDeviceToHost, c->stream),
                        "flux copy")))
        return st;
    return hip_check(c, hipStreamSynchronize(c->stream), "flux sync");
}

}  // namespace

lbm_status lbm_boundary_flux(lbm_ctx* c, double out[5]) {
    if (!c || !out) return LBM_EINVAL;
    double h[7];
    const lbm_status st = run_flux(c, h);
    for (int q = 0; q < 5; ++q) out[q] = st ? 0.0 : h[q];
    return st;
}

lbm_status lbm_boundary_flux_scalar(lbm_ctx* c, double out[3]) {
    if (!c || !out) return LBM_EINVAL;
    double h[7];
    const lbm_status st = run_flux(c, h);
    out[0] = st ? 0.0 : h[1];
    out[1] = st ? 0.0 : h[5];
    out[2] = st ? 0.0 : h[6];
    return st;
}

lbm_status lbm_reduce(lbm_ctx* c, double out[8]) {
    if (!c || !out) return LBM_EINVAL;
    if (!c->initialized) return set_err(c, LBM_ESTATE, "lbm_init must come first");
    const size_t cb = compute_bytes(c->p.storage);
    char* aux = (char*)c->buf[4];
    double* acc = (double*)(aux + round_up((size_t)(moment_planes(&c->p) - 1) * c->pad.plane * cb, kAlign));
    lbm_status st;
    if ((st = hip_check(c, hipMemsetAsync(acc, 0, lbmi::NACC * sizeof(double), c->stream), "accumulator clear")))
        return st;
    lbmi::KArgs a = base_args(c);
    a.mode = lbmi::OBS_REDUCE;
    a.acc = acc;
    a.snap = aux;
    a.snap_valid = c->snap_valid ? 1 : 0;
    if ((st = hip_check(c, c->ks.observe(a), "reduce launch"))) return st;
    double h[lbmi::NACC];
    if ((st = hip_check(c, hipMemcpyAsync(h, acc, sizeof h, hipMemcpyDeviceToHost, c->stream), "reduce copy")))
        return st;
    if ((st = hip_check(c, hipStreamSynchronize(c->stream), "reduce sync"))) return st;
    return finish_reduce(c, h, out);
}


size_t lbm_state_bytes(const lbm_ctx* c) {
    if (!c) return 0;
    return 64 + c->size[0] + c->size[3];
}

lbm_status lbm_save(lbm_ctx* c, void* host) {
    if (!c || !host) return LBM_EINVAL;
    if (!c->initialized) return set_err(c, LBM_ESTATE, "nothing to save");
    char* h = (char*)host;
    std::memset(h, 0, 64);
    std::memcpy(h, &c->t, sizeof c->t);
    const uint64_t magic = 0x4C424D53544154ull;  // "LBMSTAT"
    std::memcpy(h + 8, &magic, 8);
    size_t o = 64;
    lbm_status st;
    const int ids[2] = {0, 3};
    for (int i : ids) {
        if ((st = hip_check(c, hipMemcpyAsync(h + o, c->buf[i], c->size[i], hipMemcpyDeviceToHost, c->stream), "save copy")))
            return st;
        o += c->size[i];
    }
    return hip_check(c, hipStreamSynchronize(c->stream), "save sync");
}

lbm_status lbm_load(lbm_ctx* c, const void* host) {
    if (!c || !host) return LBM_EINVAL;
    if (!c->have_links) return set_err(c, LBM_ESTATE, "lbm_set_links must come first");
    const char* h = (const char*)host;
    uint64_t magic;
    std::memcpy(&magic, h + 8, 8);
    if (magic != 0x4C424D53544154ull) return set_err(c, LBM_EINVAL, "not a saved state");
    int64_t t;
    std::memcpy(&t, h, sizeof t);
    size_t o = 64;
    lbm_status st;
    const int ids[2] = {0, 3};
    for (int i : ids) {
        if ((st = hip_check(c, hipMemcpyAsync(c->buf[i], h + o, c->size[i], hipMemcpyHostToDevice, c->stream), "load copy")))
            return st;
        o += c->size[i];
    }
    if ((st = hip_check(c, hipStreamSynchronize(c->stream), "load sync"))) return st;
    c->t = t;
    c->initialized = true;
    c->snap_valid = false;
    return LBM_OK;
}

int64_t lbm_time(const lbm_ctx* c) { return c ? c->t : -1; }

lbm_status lbm_set_stream(lbm_ctx* c, void* s) {
    if (!c) return LBM_EINVAL;
    if (c->batch_owned) return set_err(c, LBM_EINVAL, "an item of a batch runs on the batch's stream");
    c->stream = (hipStream_t)s;
    drop_graph(c);
    return LBM_OK;
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : "null context"; }

void lbm_destroy(lbm_ctx* c) {
    if (!c || c->batch_owned) return;
    drop_graph(c);
    release_capture(c);
    delete c;
}

}  // extern "C"
