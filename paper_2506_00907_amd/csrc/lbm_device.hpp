// Fused stream-collide node update for gfx950: BGK flow f (Eqs. 1-2, Guo
// forcing, Lorentz force), convection-diffusion h (Eqs. 3-4) and the vector
// magnetic distributions g (Eqs. 5-6), with the boundary links of Sections 3-4
// applied in the same sweep.
//
// Layout: structure of arrays, one plane of `plane` nodes per population,
// padded grid with a one-node halo on non-periodic axes.  Streaming is the AA
// pattern, in place:
//   even step: node x reads slot i at x and writes its post-collision value
//              of direction i into slot opp(i) at x;
//   odd step:  node x reads slot opp(i) at x - e_i and writes its
//              post-collision value of direction i into slot i at x + e_i.
// Each location is read and written by one thread only, so one array holds
// the state.  Populations are stored as deviations from the rest
// equilibrium (w rho0, w C0, w B_ext,k), scaled by a power of two for the
// 16-bit formats.
//
// Boundary links.  The unknown population f_alpha(A, t+1) needs, from time t,
// the post-collision values f*_alpha'(A), f*_alpha(A), f*_alpha'(E) and the
// moments at A and E (Eq. 13).  After a sweep all three values sit in the
// population array at slots fixed by the parity (f*_alpha'(E) is what A
// receives along alpha' by streaming), and the slot the next sweep gathers
// f_alpha(A) from holds nothing else (a halo or solid slot, or A's own slot
// that no node streams into).  A short kernel, one thread per link, therefore
// reads its inputs from the array and writes the link value straight into
// that slot; the fused sweep needs no link code at all.  Moments of the
// link nodes go to one of two moment planes by parity.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "lbm_internal.hpp"

namespace lbmi {

// ---------------------------------------------------------------------------
// lattices
// ---------------------------------------------------------------------------
struct NoLat {
    static constexpr int Q = 0;
    __host__ __device__ static constexpr int ex(int) { return 0; }
    __host__ __device__ static constexpr int ey(int) { return 0; }
    __host__ __device__ static constexpr int ez(int) { return 0; }
    __host__ __device__ static constexpr int opp(int a) { return a; }
    __host__ __device__ static constexpr double w(int) { return 0.0; }
    static constexpr double c2 = 1.0;
};

// D2Q9: 0 rest, 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1), 5 (1,1), 6 (-1,1),
// 7 (-1,-1), 8 (1,-1); opposite pairs 1-3, 2-4, 5-7, 6-8.
struct LD2Q9 {
    static constexpr int Q = 9;
    __host__ __device__ static constexpr int ex(int a) {
        return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0);
    }
    __host__ __device__ static constexpr int ey(int a) {
        return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0);
    }
    __host__ __device__ static constexpr int ez(int) { return 0; }
    __host__ __device__ static constexpr int opp(int a) {
        return a == 0 ? 0 : (a < 5 ? ((a + 1) & 3) + 1 : ((a - 3) & 3) + 5);
    }
    __host__ __device__ static constexpr double w(int a) {
        return a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    static constexpr double c2 = 1.0 / 3.0;
};

// D3Q19: rest, the six axis directions in +/- pairs, then the twelve edge
// directions in +/- pairs; opp(a) = a + 1 for odd a, a - 1 for even a > 0.
struct LD3Q19 {
    static constexpr int Q = 19;
    __host__ __device__ static constexpr int e(int a, int k) {
        constexpr signed char t[19][3] = {
            {0, 0, 0},   {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
            {1, 1, 0},   {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
            {-1, 0, 1},  {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
        return t[a][k];
    }
    __host__ __device__ static constexpr int ex(int a) { return e(a, 0); }
    __host__ __device__ static constexpr int ey(int a) { return e(a, 1); }
    __host__ __device__ static constexpr int ez(int a) { return e(a, 2); }
    __host__ __device__ static constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
    __host__ __device__ static constexpr double w(int a) {
        return a == 0 ? 1.0 / 3.0 : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    static constexpr double c2 = 1.0 / 3.0;
};

// D2Q5: rest, (1,0), (-1,0), (0,1), (0,-1); weights 1/2 and 1/8, c^2 = 1/4.
struct LD2Q5 {
    static constexpr int Q = 5;
    __host__ __device__ static constexpr int ex(int a) { return a == 1 ? 1 : (a == 2 ? -1 : 0); }
    __host__ __device__ static constexpr int ey(int a) { return a == 3 ? 1 : (a == 4 ? -1 : 0); }
    __host__ __device__ static constexpr int ez(int) { return 0; }
    __host__ __device__ static constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
    __host__ __device__ static constexpr double w(int a) { return a == 0 ? 0.5 : 0.125; }
    static constexpr double c2 = 0.25;
};

// D3Q7: rest, (+-1,0,0), (0,+-1,0), (0,0,+-1); weights 1/4 and 1/8, c^2 = 1/4.
struct LD3Q7 {
    static constexpr int Q = 7;
    __host__ __device__ static constexpr int ex(int a) { return a == 1 ? 1 : (a == 2 ? -1 : 0); }
    __host__ __device__ static constexpr int ey(int a) { return a == 3 ? 1 : (a == 4 ? -1 : 0); }
    __host__ __device__ static constexpr int ez(int a) { return a == 5 ? 1 : (a == 6 ? -1 : 0); }
    __host__ __device__ static constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
    __host__ __device__ static constexpr double w(int a) { return a == 0 ? 0.25 : 0.125; }
    static constexpr double c2 = 0.25;
};

template <int CODE> struct LatOf { using T = NoLat; };
template <> struct LatOf<1> { using T = LD2Q9; };
template <> struct LatOf<2> { using T = LD3Q19; };
template <> struct LatOf<3> { using T = LD2Q5; };
template <> struct LatOf<4> { using T = LD3Q7; };

// ---------------------------------------------------------------------------
// storage formats
// ---------------------------------------------------------------------------
struct F64S { using T = double; using R = double; };
struct F32S { using T = float; using R = float; };
struct F16S { using T = uint16_t; using R = float; };
struct BF16S { using T = uint16_t; using R = float; };

// Element i of a plane.  The byte offset is formed in 32 bits (a plane is
// below 4 GiB, checked on the host), so the access is a uniform 64-bit base
// plus a 32-bit per-lane offset: one VGPR of address per access, not two.
template <class T>
__device__ __forceinline__ const T& at(const T* p, uint32_t i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + (uint32_t)(i * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ T& at(T* p, uint32_t i) {
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(p) + (uint32_t)(i * (uint32_t)sizeof(T)));
}

template <class SF> __device__ __forceinline__ typename SF::R ld(const typename SF::T* p, uint32_t i);
template <> __device__ __forceinline__ double ld<F64S>(const double* p, uint32_t i) { return at(p, i); }
template <> __device__ __forceinline__ float ld<F32S>(const float* p, uint32_t i) { return at(p, i); }
template <> __device__ __forceinline__ float ld<F16S>(const uint16_t* p, uint32_t i) {
    return (float)__builtin_bit_cast(_Float16, at(p, i));
}
template <> __device__ __forceinline__ float ld<BF16S>(const uint16_t* p, uint32_t i) {
    return __builtin_bit_cast(float, (uint32_t)at(p, i) << 16);
}

template <class SF> __device__ __forceinline__ void st(typename SF::T* p, uint32_t i, typename SF::R v);
template <> __device__ __forceinline__ void st<F64S>(double* p, uint32_t i, double v) { at(p, i) = v; }
template <> __device__ __forceinline__ void st<F32S>(float* p, uint32_t i, float v) { at(p, i) = v; }
template <> __device__ __forceinline__ void st<F16S>(uint16_t* p, uint32_t i, float v) {
    at(p, i) = __builtin_bit_cast(uint16_t, (_Float16)v);  // round to nearest even
}
template <> __device__ __forceinline__ void st<BF16S>(uint16_t* p, uint32_t i, float v) {
    // round to nearest even on the upper 16 bits (finite inputs)
    uint32_t b = __builtin_bit_cast(uint32_t, v);
    b += 0x7FFFu + ((b >> 16) & 1u);
    at(p, i) = (uint16_t)(b >> 16);
}

// Stores with stochastic rounding for the 16-bit formats: a value rounds up
// with probability equal to its distance from the lower neighbour, in units
// of the last place, so increments smaller than half a unit survive on
// average instead of being rounded away.  The random bits come from a
// counter-based hash (the 32-bit finaliser of MurmurHash3): a link store
// hashes (slot, node, time); the sweep hashes (writing node, time) once per
// node and mixes in each slot with one more multiply-xorshift round.  Either
// way a slot written at a given time gets the same rounding on every path.
__device__ __forceinline__ uint32_t dither(uint32_t node, uint32_t slot, uint32_t t) {
    uint32_t h = node * 0x9E3779B1u + slot * 0x85EBCA77u + t * 0xC2B2AE3Du;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}
// the sweep's per-store random bits: the node's hash hn mixed with the slot
__device__ __forceinline__ uint32_t slot_dither(uint32_t hn, int slot) {
    uint32_t h = hn + (uint32_t)slot * 0x9E3779B9u;
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    return h;
}

// the stored form of v (16-bit formats: stochastically rounded with the
// random bits r)
template <class SF>
__device__ __forceinline__ typename SF::T to_store(typename SF::R v, uint32_t r) {
    return v;
}
// gfx950 converts with stochastic rounding in one instruction
// (v_cvt_sr_f16_f32, v_cvt_sr_bf16_f32), taking its random bits from r
typedef _Float16 lbm_half2 __attribute__((ext_vector_type(2)));
typedef __bf16 lbm_bf162 __attribute__((ext_vector_type(2)));
template <> __device__ __forceinline__ uint16_t to_store<F16S>(float v, uint32_t r) {
    lbm_half2 h = {0, 0};
    h = __builtin_amdgcn_cvt_sr_f16_f32(h, v, r, false);
    return __builtin_bit_cast(uint16_t, h[0]);
}
template <> __device__ __forceinline__ uint16_t to_store<BF16S>(float v, uint32_t r) {
    lbm_bf162 h = {0, 0};
    h = __builtin_amdgcn_cvt_sr_bf16_f32(h, v, r, false);
    return __builtin_bit_cast(uint16_t, h[0]);
}
template <class SF>
__device__ __forceinline__ void st_sr(typename SF::T* p, uint32_t i, typename SF::R v, uint32_t r) {
    if (sizeof(typename SF::T) == 2) at(p, i) = to_store<SF>(v, r);
    else st<SF>(p, i, v);
}
// Population layout: tiles of 64 consecutive padded nodes (one wave) hold the
// QT populations of those nodes, population after population, so element
// (p, n) sits at ((n / 64) QT + p) 64 + n % 64.  The populations a wave
// streams lie in one contiguous QT x 64-element range instead of QT planes
// far apart: fewer DRAM pages and translations per wave (the HBM-bound sweeps
// run 4-7 % faster than with one plane per population).
constexpr uint32_t kTile = 64;
template <int QT>
__device__ __forceinline__ size_t pidx(int p, uint32_t n) {
    return ((size_t)(n / kTile) * QT + (size_t)p) * kTile + (n % kTile);
}
// element (0, n); element (p, n) is p * kTile further, a constant the memory
// instructions take as an immediate offset, so the sweep forms one address
// per node it touches rather than one per population
template <int QT, class T>
__device__ __forceinline__ T* node_base(T* S, uint32_t n) {
    return S + ((size_t)(n / kTile) * (size_t)(QT * kTile) + (n % kTile));
}

// the value of a stored element
template <class SF> __device__ __forceinline__ typename SF::R from_store(typename SF::T t) { return t; }
template <> __device__ __forceinline__ float from_store<F16S>(uint16_t t) {
    return (float)__builtin_bit_cast(_Float16, t);
}
template <> __device__ __forceinline__ float from_store<BF16S>(uint16_t t) {
    return __builtin_bit_cast(float, (uint32_t)t << 16);
}

// ---------------------------------------------------------------------------
// configuration bundle
// ---------------------------------------------------------------------------
template <int FLC, int SLC, int MLC, int NC, class SF, int NSC = 1>
struct Cfg {
    using FL = typename LatOf<FLC>::T;
    using HL = typename LatOf<SLC>::T;
    using GL = typename LatOf<MLC>::T;
    using S = SF;
    using T = typename SF::T;
    using R = typename SF::R;
    static constexpr int QF = FL::Q;
    static constexpr int QH = HL::Q;
    static constexpr int QG = GL::Q;
    static constexpr int NCOMP = (MLC == 0) ? 0 : NC;
    static constexpr int NS = (SLC == 0) ? 1 : NSC;  // scalar components, one h lattice each
    static constexpr int QT = QF + NS * QH + NCOMP * QG;
    static constexpr int H0 = QF;          // first h plane (component k: H0 + k QH)
    static constexpr int G0 = QF + NS * QH;  // first g plane
    static constexpr int MW = 8 + NS - 1;  // moment planes: rho, u, C_0, B, then C_1, C_2
    static constexpr bool SCALED = sizeof(T) == 2;  // 16-bit storage carries a power-of-two scale
};

// physical parameters in the compute type
template <class R>
struct Phys {
    R omf, omc, omm, guo;          // 1/tau_f, 1/tau_c, 1/tau_m, 1 - 1/(2 tau_f)
    R omcx[2];                     // 1/tau of scalar components 1, 2
    R rho0, C0, inv_mu, grad_c;    // grad_c = 1/(tau_m c_g^2)
    R Bext[3], acc[3];
    R sc[3], isc[3];               // storage scale and inverse (f, h, g)
    double womega;                 // angular frequency of oscillating boundary velocities
};

template <class R>
__host__ Phys<R> make_phys(const KArgs& a, double cg2) {
    Phys<R> p;
    p.omf = (R)(1.0 / a.tau_f);
    p.omc = (R)(1.0 / a.tau_c);
    for (int k = 0; k < 2; ++k) p.omcx[k] = (R)(a.tau_cs[k] > 0.0 ? 1.0 / a.tau_cs[k] : 1.0);
    p.omm = (R)(1.0 / a.tau_m);
    p.guo = (R)(1.0 - 0.5 / a.tau_f);
    p.rho0 = (R)a.rho0;
    p.womega = a.wall_omega;
    p.C0 = (R)a.C0;
    p.inv_mu = (R)(1.0 / a.mu);
    p.grad_c = (R)(1.0 / (a.tau_m * cg2));
    for (int k = 0; k < 3; ++k) {
        p.Bext[k] = (R)a.Bext[k];
        p.acc[k] = (R)a.accel[k];
        p.sc[k] = (R)a.scale[k];
        p.isc[k] = (R)(1.0 / a.scale[k]);
    }
    return p;
}

// division of a 32-bit index by a fixed divisor with a multiply-high
// (round-up reciprocal, valid for every 32-bit dividend)
struct FastDiv {
    uint32_t m, s1, s2;
};
inline FastDiv make_fastdiv(uint32_t d) {
    if (d <= 1) return FastDiv{0u, 0u, 0u};
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    const uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
    return FastDiv{(uint32_t)m, 1u, l - 1};
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
    const uint32_t t = __umulhi(n, f.m);
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

// Grid geometry of one launch.
struct Geo {
    int NX, NY, NZ;
    int hx, hy, hz, n0, n1, n2;
    uint32_t plane;
    uint32_t wave_fluid;  // offset in the flag array of one byte per 64 nodes: 1 = all fluid
    FastDiv dx, dy;
};

// logical workgroup index: consecutive blocks are dispatched round-robin over
// the 8 XCDs; give each XCD a contiguous range of the grid so that the rows a
// block streams from are mostly in its own L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t G) {
    uint32_t G8 = G & ~7u;
    if (b >= G8) return b;
    return (b & 7u) * (G8 >> 3) + (b >> 3);
}

// moments of one node (compute type)
template <class R>
struct Mom {
    R drho, u[3], dC, dB[3];  // deviations from rho0, C0 and B_ext (all three axes)
    R dCx[2];                 // deviations of scalar components 1, 2 from C0
};

// ---------------------------------------------------------------------------
// boundary link value (deviation form; Sections 3-4)
// ---------------------------------------------------------------------------
// x_a:   post-collision deviation of A along alpha
// x_apA: post-collision deviation of A along alpha'
// x_apE: post-collision deviation of E along alpha' (streamed value)
// mA, mE: moments at A and E at the previous time (deviations + u); slot 4
// holds the link's own scalar component, slots 8 and 9 (XS) the components
// of a bilinear flux term
// t: time of the value being set (the bounced population meets the boundary
// at t - d, where an oscillating boundary velocity is evaluated)
// CMP: the comparison forms (link flag bit 3, kind 8) are compiled in; the
// method-only instantiation keeps the link kernel of the hot path lean.
// XS: several scalar components (a FLUX link may carry a cross term).
template <class R, bool CMP = true, bool XS = false>
__device__ __forceinline__ R link_value(const DevLink<R>& L, const Phys<R>& P, R x_a, R x_apA,
                                        R x_apE, const R* mA, const R* mE, R w, R c2, uint32_t t) {
    const R d = L.d;
    const R one = (R)1, two = (R)2, half = (R)0.5;
    const R cE = -d, cA = d + one;  // Eq. 13 coefficients
    const R ex = (R)L.ex, ey = (R)L.ey, ez = (R)L.ez;
    // boundary velocity: given, or extrapolated (Eq. 13)
    R ux, uy, uz;
    if (L.flags & 1) {
        ux = L.uw0;
        uy = L.uw1;
        uz = L.uw2;
        if (L.flags & 4) {  // u_w cos(omega t'), t' = t - d
            const R c = (R)cos(P.womega * ((double)t - (double)L.d));
            ux *= c;
            uy *= c;
            uz *= c;
        }
    } else {
        ux = cE * mE[1] + cA * mA[1];
        uy = cE * mE[2] + cA * mA[2];
        uz = cE * mE[3] + cA * mA[3];
    }
    const R Y = (one - two * d) * x_apE + two * d * x_apA;  // Eqs. 16, 20, 35
    const bool lo = d < half;
    const bool alt = CMP && (L.flags & 8) != 0;  // the comparison forms of Section 5
    switch (L.kind) {
        case 1: {  // VEL
            R rhoX = P.rho0 + cE * mE[0] + cA * mA[0];
            R inc = two * w * rhoX * (ex * ux + ey * uy + ez * uz) / c2;
            // Eq. 15 (at every d with the comparison flag) / Eq. 43
            return (lo || alt) ? Y + inc : ((two * d - one) * x_a + x_apA + inc) / (two * d);
        }
        case 2: {  // PRES: u_X always extrapolated
            R vx = cE * mE[1] + cA * mA[1], vy = cE * mE[2] + cA * mA[2], vz = cE * mE[3] + cA * mA[3];
            R eu = ex * vx + ey * vy + ez * vz;
            R rw = P.rho0 + L.value;  // value holds rho_w - rho0
            R sdev = two * w * (L.value + rw * (eu * eu / (two * c2 * c2) - (vx * vx + vy * vy + vz * vz) / (two * c2)));
            return (lo || alt) ? sdev - Y : ((two * d - one) * x_a - x_apA + sdev) / (two * d);  // pair / Eq. 44
        }
        case 3:  // CONC (Eqs. 19-20); the velocity terms of the pair cancel; value = C_w - C0
        case 6:  // MAG_DIR (Eqs. 34-35); value = B_k - B_ext,k
            return two * w * L.value - Y;
        case 5:  // BB0 (Eqs. 21-22)
            return lo ? Y : ((two * d - one) * x_a + x_apA) / (two * d);
        case 4:
        case 7:
        case 8: {  // FLUX / MAG_FLUX: M scheme (Eqs. 23-27) with the moving correction (Eq. 24)
            R phiX, dmove;
            const R eu = ex * ux + ey * uy + ez * uz;
            if (L.kind == 4) {
                phiX = P.C0 + cE * mE[4] + cA * mA[4];
                dmove = two * w * phiX * eu / c2;
            } else {
                const int k = L.caxis;
                R Bx = P.Bext[0] + cE * mE[5] + cA * mA[5];
                R By = P.Bext[1] + cE * mE[6] + cA * mA[6];
                R Bz = P.Bext[2] + cE * mE[7] + cA * mA[7];
                phiX = k == 0 ? Bx : (k == 1 ? By : Bz);
                R uk = k == 0 ? ux : (k == 1 ? uy : uz);
                dmove = two * w * (eu * phiX - (ex * Bx + ey * By + ez * Bz) * uk) / c2;
            }
            if (CMP && L.kind == 8) {
                // link-based theta form (Eqs. 39-40): the bounced value x
                // becomes ((theta - 1) x + theta dmove) / (theta + 1), written
                // for deviations from w B_ext,k; theta = a1
                const R th = L.a1, Bk = P.Bext[L.caxis];
                const R bx = lo ? Y : x_apA;
                const R tb = ((th - one) * bx + th * dmove - two * w * Bk) / (th + one);
                return lo ? tb : ((two * d - one) * x_a + tb) / (two * d);
            }
            // F(phi_X), explicit; a bilinear term in components j, l
            // (Section 4.2.2) takes their values at X extrapolated the same way
            R dflux;
            if (XS && L.pslot) {
                const R JX = P.C0 + cE * mE[8] + cA * mA[8];
                const R LX = P.C0 + cE * mE[9] + cA * mA[9];
                dflux = ((L.a1 + L.quad * phiX) * phiX + L.value * JX * LX - L.a3) * L.weight;
            } else {
                dflux = ((L.a1 + L.quad * phiX) * phiX - L.a3) * L.weight;
            }
            if (alt)  // flux added at X, not at M (Eq. 33 and its d < 0.5 analogue)
                return lo ? Y + dflux + dmove : ((two * d - one) * x_a + x_apA + dflux + dmove) / (two * d);
            R xM = (half - d) * x_apE + (half + d) * x_apA + dflux + dmove;
            return ((d - half) * x_a + xM) / (d + half);
        }
        default:
            return x_apA;
    }
}

// One thread per link: the unknown population entering A along alpha at time
// t (parity ODD), from the state after step t-1, written into the slot the
// sweep of step t gathers it from.
//   t odd  (t-1 even: x*_i(x) sits at slot opp(i) of x):
//     x*_alpha(A) = [alpha', A], x*_alpha'(A) = [alpha, A],
//     streamed x*_alpha'(E) = [alpha, E]; target [alpha', B]
//   t even (t-1 odd: x*_i(x) sits at slot i of x + e_i):
//     x*_alpha(A) = [alpha, E], x*_alpha'(A) = [alpha', B],
//     streamed x*_alpha'(E) = [alpha', A]; target [alpha, A]
// with E = A + e_alpha and B = A - e_alpha.  No other link of the launch
// reads a target slot, so the kernel is race-free.
// a link record into registers with 16-byte loads (the fields are then read
// from registers, not fetched one by one inside the dependent chain)
template <class R>
__device__ __forceinline__ DevLink<R> load_link(const DevLink<R>* __restrict__ p) {
    static_assert(sizeof(DevLink<R>) % 16 == 0, "link records are whole 16-byte words");
    DevLink<R> L;
    const uint4* s = reinterpret_cast<const uint4*>(p);
    uint4* d = reinterpret_cast<uint4*>(&L);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(DevLink<R>) / 16); ++i) d[i] = s[i];
    return L;
}

// t: time of the value being set (also the dither seed of 16-bit storage).
// Returns the link's net inflow into A over the step: the value it sets
// minus the post-collision population A sent toward the wall, x*_alpha'(A).
template <class C, int ODD, bool CMP = true>
__device__ __forceinline__ typename C::R link_update(const Geo& G, const Phys<typename C::R>& P,
                                                     typename C::T* __restrict__ S,
                                                     const DevLink<typename C::R>& L,
                                                     const typename C::R* __restrict__ M, uint32_t t) {
    const uint32_t seed = t;
    using R = typename C::R;
    using SF = typename C::S;
    const size_t PL = G.plane;
    auto pe = [&](int p, uint32_t n) -> typename C::T* { return S + pidx<C::QT>(p, n); };
    R x_a, x_apA, xs;
    if (ODD) {
        x_a = ld<SF>(pe(L.pap, L.A), 0);
        x_apA = ld<SF>(pe(L.pa, L.A), 0);
        xs = (L.flags & 2) ? x_apA : ld<SF>(pe(L.pa, L.E), 0);
    } else {
        x_a = ld<SF>(pe(L.pa, L.E), 0);
        x_apA = ld<SF>(pe(L.pap, L.B), 0);
        xs = (L.flags & 2) ? x_apA : ld<SF>(pe(L.pap, L.A), 0);
    }
    R isc = (R)1, sc = (R)1;
    if (C::SCALED) {
        isc = L.field == 0 ? P.isc[0] : (L.field == 1 ? P.isc[1] : P.isc[2]);
        sc = L.field == 0 ? P.sc[0] : (L.field == 1 ? P.sc[1] : P.sc[2]);
        x_a *= isc;
        x_apA *= isc;
        xs *= isc;
    }
    const R* Mp = M + (size_t)(ODD ^ 1) * C::MW * PL;  // moments of the previous time
    // only the moments this link's formula uses are read (the rest stay 0);
    // the scalar slot reads the link's own component, slots 8 and 9 the
    // components of a bilinear term
    R mA[10], mE[10];
    const uint32_t need = L.need;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        mA[q] = (R)0;
        mE[q] = (R)0;
        if (need & (1u << q)) {
            const size_t src = (C::NS > 1 && q == 4) ? (size_t)L.cslot : (size_t)q;
            mA[q] = Mp[src * PL + L.A];
            mE[q] = Mp[src * PL + L.mE];
        }
    }
    mA[8] = mE[8] = mA[9] = mE[9] = (R)0;
    if (C::NS > 1 && L.pslot) {
        const size_t j = L.pslot & 15u, l = L.pslot >> 4;
        mA[8] = Mp[j * PL + L.A];
        mE[8] = Mp[j * PL + L.mE];
        mA[9] = Mp[l * PL + L.A];
        mE[9] = Mp[l * PL + L.mE];
    }
    const int e2 = L.ex * L.ex + L.ey * L.ey + L.ez * L.ez;
    R w, c2;
    if (L.field == 0) {
        w = (R)(C::QF == 9 ? (e2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0) : (e2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0));
        c2 = (R)(1.0 / 3.0);
    } else if (L.field == 2 && C::QG == 19) {  // D3Q19 magnetic lattice
        w = (R)(e2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        c2 = (R)(1.0 / 3.0);
    } else {  // D2Q5 / D3Q7
        w = (R)0.125;
        c2 = (R)0.25;
    }
    const R v = link_value<R, CMP, (C::NS > 1)>(L, P, x_a, x_apA, xs, mA, mE, w, c2, t);
    if (ODD) st_sr<SF>(pe(L.pap, L.B), 0, C::SCALED ? v * sc : v, C::SCALED ? dither(L.B, L.pap, seed) : 0u);
    else st_sr<SF>(pe(L.pa, L.A), 0, C::SCALED ? v * sc : v, C::SCALED ? dither(L.A, L.pa, seed) : 0u);
    return v - x_apA;
}

// time of the step being taken: base word (if any) plus offset
__device__ __forceinline__ uint32_t step_time(const uint32_t* tbase, uint32_t tstep) {
    return (tbase ? *tbase : 0u) + tstep;
}

template <class C, int ODD, bool CMP>
__global__ __launch_bounds__(256) void k_links(Geo G, Phys<typename C::R> P, typename C::T* __restrict__ S,
                                               const DevLink<typename C::R>* __restrict__ links,
                                               const typename C::R* __restrict__ M, uint32_t nlinks,
                                               const uint32_t* __restrict__ tbase, uint32_t tstep) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nlinks) return;
    link_update<C, ODD, CMP>(G, P, S, load_link(links + k), M, step_time(tbase, tstep));
}

// sum over the 64 lanes of a wave (lane 0 holds the total)
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// The links of the current step as k_links, plus the FP64 sums of their net
// inflows by field slot: 0 f (mass), 1 h (solute C_0), 2 + axis g (B_x, B_y,
// B_z), 5 and 6 the scalar components C_1 and C_2; one FP64 atomic per slot
// and block.
template <class C, int ODD>
__global__ __launch_bounds__(256) void k_flux(Geo G, Phys<typename C::R> P, typename C::T* __restrict__ S,
                                              const DevLink<typename C::R>* __restrict__ links,
                                              const typename C::R* __restrict__ M, uint32_t nlinks, uint32_t tstep,
                                              double* __restrict__ acc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    constexpr int NV = 7;
    double v[NV] = {0, 0, 0, 0, 0, 0, 0};
    if (k < nlinks) {
        const DevLink<typename C::R> L = load_link(links + k);
        const double net = (double)link_update<C, ODD>(G, P, S, L, M, tstep);
        // scalar component k's moment plane is 4 (k = 0) or 7 + k
        int slot = L.field == 2 ? 2 + L.caxis : L.field;
        if (C::NS > 1 && L.field == 1 && L.cslot != 4) slot = L.cslot - 3;
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = q == slot ? net : 0.0;
    }
    __shared__ double red[NV][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double sum = wave_sum(v[q]);
        if (lane == 0) red[q][wv] = sum;
    }
    __syncthreads();
    if (threadIdx.x < NV) atomicAdd(&acc[threadIdx.x], red[threadIdx.x][0] + red[threadIdx.x][1] +
                                                           red[threadIdx.x][2] + red[threadIdx.x][3]);
}

// ---------------------------------------------------------------------------
// the fused node update
// ---------------------------------------------------------------------------
template <class C>
struct NodeRes {
    typename C::R x[C::QT];  // populations (deviations), post-collision after MODE 0
    Mom<typename C::R> m;
};

// e . v for a lattice vector e whose components (-1, 0 or 1) are known at
// compile time: a zero component contributes -0.0, which the compiler drops
// exactly, so only the nonzero terms are formed (0 * v would have to be
// computed, since it is not exactly zero for every v)
template <class R>
__device__ __forceinline__ R edot(int ex, int ey, int ez, R x, R y, R z) {
    auto t = [](int e, R v) -> R { return e == 0 ? (R)-0.0 : (e > 0 ? v : -v); };
    return t(ex, x) + t(ey, y) + t(ez, z);
}

// Padded node and its wrapped neighbour offsets (fluid nodes never touch a
// non-periodic edge of the padded grid, so wrapping only ever applies on
// periodic axes).
struct Nbr {
    uint32_t n;
    int oxm, oxp, oym, oyp, ozm, ozp;
    __device__ __forceinline__ uint32_t at(int ex, int ey, int ez) const {
        return (uint32_t)((int)n + (ex > 0 ? oxp : (ex < 0 ? oxm : 0)) + (ey > 0 ? oyp : (ey < 0 ? oym : 0)) +
                          (ez > 0 ? ozp : (ez < 0 ? ozm : 0)));
    }
};

__device__ __forceinline__ Nbr nbr_of(const Geo& G, uint32_t n) {
    Nbr q;
    q.n = n;
    const uint32_t t1 = fdiv(n, G.dx);
    const int x = (int)(n - t1 * (uint32_t)G.NX);
    const uint32_t zz = fdiv(t1, G.dy);
    const int y = (int)(t1 - zz * (uint32_t)G.NY);
    const int z = (int)zz;
    const int sx = G.NX * G.NY;
    q.oxm = x == 0 ? G.NX - 1 : -1;
    q.oxp = x == G.NX - 1 ? -(G.NX - 1) : 1;
    q.oym = y == 0 ? (G.NY - 1) * G.NX : -G.NX;
    q.oyp = y == G.NY - 1 ? -(G.NY - 1) * G.NX : G.NX;
    q.ozm = z == 0 ? (G.NZ - 1) * sx : -sx;
    q.ozp = z == G.NZ - 1 ? -(G.NZ - 1) * sx : sx;
    return q;
}

// gather (streaming) of one fluid node's populations, unscaled deviations
template <class C, int ODD>
__device__ __forceinline__ void gather(const Geo& G, const Phys<typename C::R>& P, typename C::T* __restrict__ S,
                                       const Nbr& q, typename C::R* x_) {
    using R = typename C::R;
    using SF = typename C::S;
    using FL = typename C::FL;
    using HL = typename C::HL;
    using GL = typename C::GL;
    constexpr int QF = C::QF, QH = C::QH, QG = C::QG, NCP = C::NCOMP;
    const uint32_t n = q.n;
    auto ldp = [&](int p, uint32_t m) -> R { return ld<SF>(node_base<C::QT>(S, m) + p * kTile, 0); };
#pragma unroll
    for (int i = 0; i < QF; ++i) {
        R v = ODD ? ldp(FL::opp(i), q.at(-FL::ex(i), -FL::ey(i), -FL::ez(i))) : ldp(i, n);
        x_[i] = C::SCALED ? v * P.isc[0] : v;
    }
#pragma unroll
    for (int k = 0; k < C::NS; ++k)
#pragma unroll
        for (int i = 0; i < QH; ++i) {
            const int b = C::H0 + k * QH;
            R v = ODD ? ldp(b + HL::opp(i), q.at(-HL::ex(i), -HL::ey(i), -HL::ez(i))) : ldp(b + i, n);
            x_[b + i] = C::SCALED ? v * P.isc[1] : v;
        }
#pragma unroll
    for (int c = 0; c < NCP; ++c)
#pragma unroll
        for (int i = 0; i < QG; ++i) {
            const int b = C::G0 + c * QG;
            R v = ODD ? ldp(b + GL::opp(i), q.at(-GL::ex(i), -GL::ey(i), -GL::ez(i))) : ldp(b + i, n);
            x_[b + i] = C::SCALED ? v * P.isc[2] : v;
        }
}

// Everything after the gather: moments, moment store of link nodes,
// collision, scatter.  MODE 0: full step; MODE 1: observe (moments only).
template <class C, int ODD, int MODE>
__device__ __forceinline__ void finish(const Geo& G, const Phys<typename C::R>& P, typename C::T* __restrict__ S,
                                       uint8_t fl, typename C::R* __restrict__ M,
                                       const Nbr& q, NodeRes<C>& res, uint32_t seed) {
    using R = typename C::R;
    using SF = typename C::S;
    using FL = typename C::FL;
    using HL = typename C::HL;
    using GL = typename C::GL;
    constexpr int QF = C::QF, QH = C::QH, QG = C::QG, NCP = C::NCOMP;
    const uint32_t PL = G.plane, n = q.n;
    auto stp = [&](int p, uint32_t m, R v, uint32_t r) { st_sr<SF>(node_base<C::QT>(S, m) + p * kTile, 0, v, r); };
    R* x_ = res.x;
    // ---- moments ----
    Mom<R>& m = res.m;
    R jx = 0, jy = 0, jz = 0, drho = 0;
#pragma unroll
    for (int i = 0; i < QF; ++i) {
        drho += x_[i];
        if (FL::ex(i)) jx += (R)FL::ex(i) * x_[i];
        if (FL::ey(i)) jy += (R)FL::ey(i) * x_[i];
        if (FL::ez(i)) jz += (R)FL::ez(i) * x_[i];
    }
    const R rho = P.rho0 + drho;
    const R irho = (R)1 / rho;
    R dCs[C::NS];
#pragma unroll
    for (int k = 0; k < C::NS; ++k) {
        dCs[k] = 0;
#pragma unroll
        for (int i = 0; i < QH; ++i) dCs[k] += x_[C::H0 + k * QH + i];
    }
    const R dC = dCs[0];
    R dB[3] = {0, 0, 0}, B[3] = {P.Bext[0], P.Bext[1], P.Bext[2]};
    R lam[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // lam[c][i] = sum_a e_ai g_a,c
#pragma unroll
    for (int c = 0; c < NCP; ++c) {
        R s = 0, l0 = 0, l1 = 0, l2 = 0;
#pragma unroll
        for (int i = 0; i < QG; ++i) {
            const R g = x_[C::G0 + c * QG + i];
            s += g;
            if (GL::ex(i)) l0 += (R)GL::ex(i) * g;
            if (GL::ey(i)) l1 += (R)GL::ey(i) * g;
            if (GL::ez(i)) l2 += (R)GL::ez(i) * g;
        }
        // evolved component slot c is Cartesian axis c
        dB[c] = s;
        B[c] = P.Bext[c] + s;
        lam[c][0] = l0;
        lam[c][1] = l1;
        lam[c][2] = l2;
    }
    R F[3] = {rho * P.acc[0], rho * P.acc[1], rho * P.acc[2]};
    if (NCP > 0) {
        // grad B from the non-equilibrium first moment of g, evaluated with the
        // velocity that carries half the body force only (explicit current)
        const R u0[3] = {(jx + (R)0.5 * F[0]) * irho, (jy + (R)0.5 * F[1]) * irho, (jz + (R)0.5 * F[2]) * irho};
        R gB[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // gB[i][k] = d_i B_k
#pragma unroll
        for (int c = 0; c < NCP; ++c) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const R leq = u0[i] * B[c] - B[i] * u0[c];
                gB[i][c] = -(lam[c][i] - leq) * P.grad_c;
            }
        }
        const R J0 = (gB[1][2] - gB[2][1]) * P.inv_mu;
        const R J1 = (gB[2][0] - gB[0][2]) * P.inv_mu;
        const R J2 = (gB[0][1] - gB[1][0]) * P.inv_mu;
        F[0] += J1 * B[2] - J2 * B[1];
        F[1] += J2 * B[0] - J0 * B[2];
        F[2] += J0 * B[1] - J1 * B[0];
    }
    const R ux = (jx + (R)0.5 * F[0]) * irho, uy = (jy + (R)0.5 * F[1]) * irho, uz = (jz + (R)0.5 * F[2]) * irho;
    m.drho = drho;
    m.u[0] = ux;
    m.u[1] = uy;
    m.u[2] = uz;
    m.dC = dC;
    m.dB[0] = dB[0];
    m.dB[1] = dB[1];
    m.dB[2] = dB[2];
#pragma unroll
    for (int k = 1; k < C::NS; ++k) m.dCx[k - 1] = dCs[k];
    if (MODE != 0) return;

    // moments of link nodes for the next step's extrapolations (Eq. 13)
    if (fl & NF_MOM) {
        R* Mc = M + (size_t)ODD * C::MW * PL;
        Mc[0 * (size_t)PL + n] = drho;
        Mc[1 * (size_t)PL + n] = ux;
        Mc[2 * (size_t)PL + n] = uy;
        Mc[3 * (size_t)PL + n] = uz;
        Mc[4 * (size_t)PL + n] = dC;
        Mc[5 * (size_t)PL + n] = dB[0];
        Mc[6 * (size_t)PL + n] = dB[1];
        Mc[7 * (size_t)PL + n] = dB[2];
#pragma unroll
        for (int k = 1; k < C::NS; ++k) Mc[(size_t)(7 + k) * PL + n] = dCs[k];
    }

    // ---- collision (deviation form), opposite directions in pairs: the
    // equilibrium and the Guo source split into a part even in e (shared by
    // the pair) and a part odd in e (opposite signs).  Per pair of the fluid
    // and magnetic lattices,
    //   x_a' = (1 - om) x_a + S + D,   x_b' = (1 - om) x_b + S - D,
    // with S = om ev + evs and D = om od + ods gathered into per-node factors
    // that only the lattice weight w multiplies (fewer instructions, and in
    // FP32 closer to the oracle than x + om (x_eq - x) after long runs) ----
    const R usq = ux * ux + uy * uy + uz * uz;
    const R uF = ux * F[0] + uy * F[1] + uz * F[2];
    const R omf = P.omf, guo = P.guo;
    {
        const R w0 = (R)FL::w(0);
        const R feq = w0 * (drho - (R)1.5 * rho * usq);
        x_[0] += omf * (feq - x_[0]) - (R)3 * guo * w0 * uF;
    }
    {
        // om ev + evs = w (s0 + eu (s2 eu + s1 eF)), om od + ods = w (d1 eu + d2 eF)
        const R om1 = (R)1 - omf;
        const R s0 = omf * (drho - (R)1.5 * rho * usq) - (R)3 * guo * uF;
        const R s2 = (R)4.5 * omf * rho, s1 = (R)9 * guo;
        const R d1 = (R)3 * omf * rho, d2 = (R)3 * guo;
#pragma unroll
        for (int a = 1; a < QF; ++a) {
            if (FL::opp(a) < a) continue;
            const int b = FL::opp(a);
            const R w = (R)FL::w(a);
            const R eu = edot(FL::ex(a), FL::ey(a), FL::ez(a), ux, uy, uz);
            const R eF = edot(FL::ex(a), FL::ey(a), FL::ez(a), F[0], F[1], F[2]);
            const R S = w * s0 + eu * ((w * s2) * eu + (w * s1) * eF);
            const R D = (w * d1) * eu + (w * d2) * eF;
            const R xa = x_[a], xb = x_[b];
            x_[a] = om1 * xa + (S + D);
            x_[b] = om1 * xb + (S - D);
        }
    }
#pragma unroll
    for (int k = 0; k < (QH > 0 ? C::NS : 0); ++k) {
        const int h0 = C::H0 + k * QH;
        const R dCk = dCs[k];
        const R Cc = P.C0 + dCk, omc = k == 0 ? P.omc : P.omcx[k - 1];
        x_[h0] += omc * ((R)HL::w(0) * dCk - x_[h0]);
        // relaxed toward the pair's equilibrium directly: in FP32 this kept
        // the steady solute field of the reactive channel 3 times closer to
        // the oracle's than the (1 - om) x + S + D form of f and g
#pragma unroll
        for (int a = 1; a < QH; ++a) {
            if (HL::opp(a) < a) continue;
            const int b = HL::opp(a);
            const R w = (R)HL::w(a);
            const R eu = edot(HL::ex(a), HL::ey(a), HL::ez(a), ux, uy, uz);
            const R ev = w * dCk, od = (R)4 * w * Cc * eu;
            const R xa = x_[h0 + a], xb = x_[h0 + b];
            x_[h0 + a] = xa + omc * (ev + od - xa);
            x_[h0 + b] = xb + omc * (ev - od - xb);
        }
    }
#pragma unroll
    for (int c = 0; c < NCP; ++c) {
        const R Bk = B[c];
        const R uk = c == 0 ? ux : (c == 1 ? uy : uz);
        const R omm = P.omm;
        const int p0 = C::G0 + c * QG;
        x_[p0] += omm * ((R)GL::w(0) * dB[c] - x_[p0]);
        // om ev = w om dB_k, om od = w (om / c2) (e.u B_k - e.B u_k)
        const R om1 = (R)1 - omm, sg = omm * dB[c], dg = (R)(1.0 / GL::c2) * omm;
#pragma unroll
        for (int a = 1; a < QG; ++a) {
            if (GL::opp(a) < a) continue;
            const int b = GL::opp(a);
            const R w = (R)GL::w(a);
            const R s = edot(GL::ex(a), GL::ey(a), GL::ez(a), ux, uy, uz) * Bk -
                        edot(GL::ex(a), GL::ey(a), GL::ez(a), B[0], B[1], B[2]) * uk;
            const R S = w * sg, D = (w * dg) * s;
            const R xa = x_[p0 + a], xb = x_[p0 + b];
            x_[p0 + a] = om1 * xa + (S + D);
            x_[p0 + b] = om1 * xb + (S - D);
        }
    }

    auto nb = [&](int ex, int ey, int ez) -> uint32_t { return q.at(ex, ey, ez); };

    // ---- scatter (streaming); 16-bit formats round stochastically with a
    // dither of (writing node, time), then the slot ----
    // one full hash of (writing node n, time), then one multiply-xorshift
    // round per store mixes in the slot
    const uint32_t hn = C::SCALED ? dither(n, 0u, seed) : 0u;
    auto put = [&](int slot, uint32_t dest, R v) {
        stp(slot, dest, v, C::SCALED ? slot_dither(hn, slot) : 0u);
    };
#pragma unroll
    for (int i = 0; i < QF; ++i) {
        const R v = C::SCALED ? x_[i] * P.sc[0] : x_[i];
        if (ODD) put(i, nb(FL::ex(i), FL::ey(i), FL::ez(i)), v);
        else put(FL::opp(i), n, v);
    }
#pragma unroll
    for (int k = 0; k < C::NS; ++k)
#pragma unroll
        for (int i = 0; i < QH; ++i) {
            const int b = C::H0 + k * QH;
            const R v = C::SCALED ? x_[b + i] * P.sc[1] : x_[b + i];
            if (ODD) put(b + i, nb(HL::ex(i), HL::ey(i), HL::ez(i)), v);
            else put(b + HL::opp(i), n, v);
        }
#pragma unroll
    for (int c = 0; c < NCP; ++c)
#pragma unroll
        for (int i = 0; i < QG; ++i) {
            const int b = C::G0 + c * QG;
            const R v = C::SCALED ? x_[b + i] * P.sc[2] : x_[b + i];
            if (ODD) put(b + i, nb(GL::ex(i), GL::ey(i), GL::ez(i)), v);
            else put(b + GL::opp(i), n, v);
        }
}

// Updates node n if it is fluid; returns whether it is.  The 64 nodes of a
// wave are contiguous and 64-aligned; where all of them are fluid (one
// wave-uniform byte of the flag array, a scalar load), the gathers are issued
// without waiting for the per-node flag.
template <class C, int ODD, int MODE>
__device__ __forceinline__ bool node_update(const Geo& G, const Phys<typename C::R>& P,
                                            typename C::T* __restrict__ S,
                                            const uint8_t* __restrict__ flags,
                                            typename C::R* __restrict__ M, uint32_t n,
                                            NodeRes<C>& res, uint32_t seed = 0u) {
    const uint32_t wg = __builtin_amdgcn_readfirstlane(n >> 6);
    const uint32_t wword = reinterpret_cast<const uint32_t*>(flags + G.wave_fluid)[wg >> 2];
    const uint8_t fl = flags[n];  // issued before the gathers, used after them
    if ((wword >> (8 * (wg & 3))) & 0xFFu) {  // uniform branch: no wait for the node's flag
        const Nbr q = nbr_of(G, n);
        gather<C, ODD>(G, P, S, q, res.x);
        finish<C, ODD, MODE>(G, P, S, fl, M, q, res, seed);
        return true;
    }
    if (!(fl & NF_FLUID)) return false;
    const Nbr q = nbr_of(G, n);
    gather<C, ODD>(G, P, S, q, res.x);
    finish<C, ODD, MODE>(G, P, S, fl, M, q, res, seed);
    return true;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <class C, int ODD>
__global__ __launch_bounds__(256) void k_step(Geo G, Phys<typename C::R> P, typename C::T* __restrict__ S,
                                              const uint8_t* __restrict__ flags,
                                              typename C::R* __restrict__ M, uint32_t nnodes,
                                              const uint32_t* __restrict__ tbase, uint32_t tstep) {
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t n = b * 256u + threadIdx.x;
    if (n >= nnodes) return;
    NodeRes<C> r;
    node_update<C, ODD, 0>(G, P, S, flags, M, n, r, C::SCALED ? step_time(tbase, tstep) : 0u);
}

// The same update over a list of 64-node waves (four per block): a step's
// sweep split into the waves that hold link nodes or their partners and the
// rest, so that the link kernel of the next step can run beside the rest.
template <class C, int ODD>
__global__ __launch_bounds__(256) void k_step_waves(Geo G, Phys<typename C::R> P, typename C::T* __restrict__ S,
                                                    const uint8_t* __restrict__ flags,
                                                    typename C::R* __restrict__ M, uint32_t nnodes,
                                                    const uint32_t* __restrict__ waves, uint32_t nwaves,
                                                    const uint32_t* __restrict__ tbase, uint32_t tstep) {
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t w = b * 4u + (threadIdx.x >> 6);
    if (w >= nwaves) return;
    const uint32_t n = waves[w] * 64u + (threadIdx.x & 63u);
    if (n >= nnodes) return;
    NodeRes<C> r;
    node_update<C, ODD, 0>(G, P, S, flags, M, n, r, C::SCALED ? step_time(tbase, tstep) : 0u);
}

// time base of a captured run: *tbase = t (set) or *tbase += t (tick); one
// lane, through a vector-memory atomic
template <class C>
__global__ void k_time(uint32_t* tbase, uint32_t t, int add) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (add) atomicAdd(tbase, t);
        else atomicExch(tbase, t);
    }
}

// Per-node terms of the FP64 reductions: sums of rho, C_0, B (0..4); squared
// change of u, C - C0 (every scalar component), B - B_ext since the snapshot
// (5..7) and their squared norms (8..10); a non-finite flag (11).  The
// snapshot is replaced by the current values.
template <class C>
__device__ __forceinline__ void reduce_node(const Phys<typename C::R>& P, const NodeRes<C>& r, bool fluid,
                                            typename C::R* snap, int snap_valid, uint32_t PL, uint32_t n,
                                            double v[NACC]) {
    using R = typename C::R;
    for (int q = 0; q < NACC; ++q) v[q] = 0.0;
    if (!fluid) return;
    constexpr int NP = C::MW - 1;  // u, C_0, B, C_1, C_2
    double phi[9] = {r.m.u[0], r.m.u[1], r.m.u[2], r.m.dC, r.m.dB[0], r.m.dB[1], r.m.dB[2], 0.0, 0.0};
    for (int k = 1; k < C::NS; ++k) phi[6 + k] = r.m.dCx[k - 1];
    v[0] = (double)P.rho0 + (double)r.m.drho;
    v[1] = (double)P.C0 + (double)r.m.dC;
    for (int k = 0; k < 3; ++k) v[2 + k] = (double)P.Bext[k] + (double)r.m.dB[k];
    for (int q = 0; q < NP; ++q) {
        const double s = snap_valid ? (double)snap[(size_t)q * PL + n] : 0.0;
        const double dd = phi[q] - s;
        const int fld = q < 3 ? 0 : ((q == 3 || q > 6) ? 1 : 2);
        v[5 + fld] += dd * dd;
        v[8 + fld] += phi[q] * phi[q];
        snap[(size_t)q * PL + n] = (R)phi[q];
    }
    bool bad = false;
    for (int q = 0; q < 5; ++q) bad = bad || !(v[q] - v[q] == 0.0);
    for (int q = 0; q < NP; ++q) bad = bad || !(phi[q] - phi[q] == 0.0);
    v[11] = bad ? 1.0 : 0.0;
}

// block sum of the first 12 accumulators: wave shuffles, then LDS, then one
// FP64 atomic per value and block into acc, or (store) a plain store of the
// block's sums into acc
__device__ __forceinline__ void block_accumulate(const double v[NACC], double* acc, bool store = false) {
    __shared__ double red[12][16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int q = 0; q < 12; ++q) {
        double s = wave_sum(v[q]);
        if (lane == 0) red[q][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        double s = 0.0;
        for (int k = 0; k < (int)((blockDim.x + 63) >> 6); ++k) s += red[threadIdx.x][k];
        if (store) acc[threadIdx.x] = s;
        else atomicAdd(&acc[threadIdx.x], s);
    }
}

// observe: moments / populations / FP64 reductions at the current time
template <class C, int ODD>
__global__ __launch_bounds__(256) void k_observe(Geo G, Phys<typename C::R> P, typename C::T* __restrict__ S,
                                                 const uint8_t* __restrict__ flags,
                                                 typename C::R* __restrict__ M,
                                                 uint32_t nnodes, int mode, int field, void* out,
                                                 int out_f64, double* acc, int acc_blocks,
                                                 typename C::R* snap, int snap_valid) {
    using R = typename C::R;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    NodeRes<C> r;
    bool fluid = false;
    if (n < nnodes) fluid = node_update<C, ODD, 1>(G, P, S, flags, M, n, r);
    // domain index of this node (if inside the domain)
    int dom = -1;
    if (n < nnodes) {
        const int x = (int)(n % (uint32_t)G.NX);
        const uint32_t t1 = n / (uint32_t)G.NX;
        const int y = (int)(t1 % (uint32_t)G.NY);
        const int z = (int)(t1 / (uint32_t)G.NY);
        const int dx = x - G.hx, dy = y - G.hy, dz = z - G.hz;
        if (dx >= 0 && dx < G.n0 && dy >= 0 && dy < G.n1 && dz >= 0 && dz < G.n2)
            dom = dx + G.n0 * (dy + G.n1 * dz);
    }
    const size_t N = (size_t)G.n0 * G.n1 * G.n2;
    if (mode == OBS_MOMENTS) {
        if (dom < 0) return;
        double v[C::MW];
        for (int q = 0; q < C::MW; ++q) v[q] = 0.0;
        if (fluid) {
            v[0] = (double)P.rho0 + (double)r.m.drho;
            v[1] = r.m.u[0];
            v[2] = r.m.u[1];
            v[3] = r.m.u[2];
            v[4] = (double)P.C0 + (double)r.m.dC;
            for (int k = 0; k < 3; ++k) v[5 + k] = (double)P.Bext[k] + (double)r.m.dB[k];
            for (int k = 1; k < C::NS; ++k) v[7 + k] = (double)P.C0 + (double)r.m.dCx[k - 1];
        }
        for (int q = 0; q < C::MW; ++q) {
            if (out_f64) ((double*)out)[(size_t)q * N + dom] = v[q];
            else ((float*)out)[(size_t)q * N + dom] = (float)v[q];
        }
        return;
    }
    if (mode == OBS_POPS) {
        if (dom < 0) return;
        double* o = (double*)out;
        if (field == 0) {
            for (int i = 0; i < C::QF; ++i)
                o[(size_t)i * N + dom] = fluid ? (double)r.x[i] + C::FL::w(i) * (double)P.rho0 : 0.0;
        } else if (field == 1) {
            for (int k = 0; k < C::NS; ++k)
                for (int i = 0; i < C::QH; ++i)
                    o[(size_t)(k * C::QH + i) * N + dom] =
                        fluid ? (double)r.x[C::H0 + k * C::QH + i] + C::HL::w(i) * (double)P.C0 : 0.0;
        } else {
            for (int c = 0; c < C::NCOMP; ++c)
                for (int i = 0; i < C::QG; ++i)
                    o[(size_t)(c * C::QG + i) * N + dom] =
                        fluid ? (double)r.x[C::G0 + c * C::QG + i] + C::GL::w(i) * (double)P.Bext[c] : 0.0;
        }
        return;
    }
    if (mode == OBS_NORM) {
        // u and B - B_ext along one axis, raw (k_scale divides them), and the
        // sums of u and of the fluid nodes for a mean velocity
        double v[NACC];
        for (int q = 0; q < NACC; ++q) v[q] = 0.0;
        if (dom >= 0) {
            double* o = (double*)out;
            o[dom] = fluid ? (double)r.m.u[field] : 0.0;
            o[N + dom] = fluid ? (double)r.m.dB[field] : 0.0;
            if (fluid) {
                v[0] = r.m.u[field];
                v[1] = 1.0;
            }
        }
        block_accumulate(v, acc);
        return;
    }
    // OBS_REDUCE
    double v[NACC];
    reduce_node<C>(P, r, fluid, snap, snap_valid, G.plane, n, v);
    if (acc_blocks) block_accumulate(v, acc + (size_t)blockIdx.x * NACC, true);
    else block_accumulate(v, acc);
}

// the normalisation of the OBS_NORM output: out[0][i] /= U,
// out[1][i] /= U * bfac
template <class C>
__global__ __launch_bounds__(256) void k_scale(double* __restrict__ out, uint32_t N, double U, double bfac) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    out[i] /= U;
    out[N + i] /= U * bfac;
}

// equilibrium initialisation: canonical layout slot i at node n holds x_i
template <class C>
__global__ __launch_bounds__(256) void k_init(Geo G, Phys<typename C::R> P, typename C::T* __restrict__ S,
                                              const uint8_t* __restrict__ flags, uint32_t nnodes,
                                              const double* __restrict__ rho_in,
                                              const double* __restrict__ u_in,
                                              const double* __restrict__ C_in,
                                              const double* __restrict__ B_in) {
    using R = typename C::R;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nnodes || !(flags[n] & NF_FLUID)) return;
    const int x = (int)(n % (uint32_t)G.NX);
    const uint32_t t1 = n / (uint32_t)G.NX;
    const int y = (int)(t1 % (uint32_t)G.NY);
    const int z = (int)(t1 / (uint32_t)G.NY);
    const size_t N = (size_t)G.n0 * G.n1 * G.n2;
    const size_t dom = (size_t)(x - G.hx) + (size_t)G.n0 * ((size_t)(y - G.hy) + (size_t)G.n1 * (size_t)(z - G.hz));
    const R rho = rho_in ? (R)rho_in[dom] : P.rho0;
    const R drho = rho_in ? (R)(rho_in[dom] - (double)P.rho0) : (R)0;
    R u[3] = {0, 0, 0};
    if (u_in)
        for (int k = 0; k < 3; ++k) u[k] = (R)u_in[(size_t)k * N + dom];
    R B[3] = {P.Bext[0], P.Bext[1], P.Bext[2]}, dB[3] = {0, 0, 0};
    if (B_in)
        for (int k = 0; k < 3; ++k) {
            dB[k] = (R)(B_in[(size_t)k * N + dom] - (double)P.Bext[k]);
            B[k] = P.Bext[k] + dB[k];
        }
    const R usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    using FL = typename C::FL;
    using HL = typename C::HL;
    using GL = typename C::GL;
#pragma unroll
    for (int i = 0; i < C::QF; ++i) {
        const R eu = (R)FL::ex(i) * u[0] + (R)FL::ey(i) * u[1] + (R)FL::ez(i) * u[2];
        const R v = (R)FL::w(i) * (drho + rho * ((R)3 * eu + (R)4.5 * eu * eu - (R)1.5 * usq));
        st<typename C::S>(S + pidx<C::QT>(i, (uint32_t)n), 0, C::SCALED ? v * P.sc[0] : v);
    }
#pragma unroll
    for (int k = 0; k < C::NS; ++k) {
        const R dC = C_in ? (R)(C_in[(size_t)k * N + dom] - (double)P.C0) : (R)0;
        const R Cc = P.C0 + dC;
#pragma unroll
        for (int i = 0; i < C::QH; ++i) {
            const R eu = (R)HL::ex(i) * u[0] + (R)HL::ey(i) * u[1] + (R)HL::ez(i) * u[2];
            const R v = (R)HL::w(i) * (dC + Cc * eu * (R)4);
            st<typename C::S>(S + pidx<C::QT>(C::H0 + k * C::QH + i, (uint32_t)n), 0,
                              C::SCALED ? v * P.sc[1] : v);
        }
    }
#pragma unroll
    for (int c = 0; c < C::NCOMP; ++c) {
        const R uk = u[c];
#pragma unroll
        for (int i = 0; i < C::QG; ++i) {
            const R ex = (R)GL::ex(i), ey = (R)GL::ey(i), ez = (R)GL::ez(i);
            const R s = (ex * u[0] + ey * u[1] + ez * u[2]) * B[c] - (ex * B[0] + ey * B[1] + ez * B[2]) * uk;
            const R v = (R)GL::w(i) * (dB[c] + s * (R)(1.0 / GL::c2));
            st<typename C::S>(S + pidx<C::QT>(C::G0 + c * C::QG + i, (uint32_t)n), 0,
                              C::SCALED ? v * P.sc[2] : v);
        }
    }
}

// ---------------------------------------------------------------------------
// batched items: many independent lattices of one lattice combination and
// storage format, each with its own geometry, links and parameters
// ---------------------------------------------------------------------------
template <class C>
struct BItem {
    Geo G;
    Phys<typename C::R> P;
    typename C::T* S;
    const uint8_t* flags;
    const DevLink<typename C::R>* links;
    typename C::R* M;
    typename C::R* snap;  // [MW - 1][plane] residual snapshot
    double* acc;          // [NACC] FP64 accumulators
    uint32_t* tbase;      // time base word of the item
    uint32_t t0;          // the item's time when the descriptor was written
    uint32_t nnodes, nlinks;
};

// fused sweep over node tiles; the tile table lists (item, first node)
template <class C, int ODD>
__global__ __launch_bounds__(256) void kb_sweep(const BItem<C>* __restrict__ items,
                                                const uint32_t* __restrict__ tiles,
                                                const uint32_t* __restrict__ status, uint32_t ntiles,
                                                uint32_t tstep) {
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    if (b >= ntiles) return;
    const uint32_t it = tiles[2 * b];
    if (status[it] != BS_ACTIVE) return;
    const BItem<C>& I = items[it];
    const uint32_t n = tiles[2 * b + 1] + threadIdx.x;
    if (n >= I.nnodes) return;
    NodeRes<C> r;
    node_update<C, ODD, 0>(I.G, I.P, I.S, I.flags, I.M, n, r, C::SCALED ? step_time(I.tbase, tstep) : 0u);
}

template <class C, int ODD>
__global__ __launch_bounds__(256) void kb_links(const BItem<C>* __restrict__ items,
                                                const uint32_t* __restrict__ ltiles,
                                                const uint32_t* __restrict__ status, uint32_t nltiles,
                                                uint32_t tstep) {
    const uint32_t b = blockIdx.x;
    if (b >= nltiles) return;
    const uint32_t it = ltiles[2 * b];
    if (status[it] != BS_ACTIVE) return;
    const BItem<C>& I = items[it];
    const uint32_t k = ltiles[2 * b + 1] + threadIdx.x;
    if (k >= I.nlinks) return;
    link_update<C, ODD>(I.G, I.P, I.S, load_link(I.links + k), I.M, step_time(I.tbase, tstep));
}

// item time bases: set from the descriptors (all items), or advanced for the
// listed items
template <class C>
__global__ __launch_bounds__(256) void kb_time(const BItem<C>* __restrict__ items, const uint32_t* __restrict__ active,
                                               uint32_t n, uint32_t add) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (active) atomicAdd(items[active[i]].tbase, add);
    else atomicExch(items[i].tbase, items[i].t0);
}

// One workgroup advances one item by nsteps steps (nsteps even, starting at
// an even time with links ready): per step the links, a workgroup barrier, the
// sweep over all nodes of the item, a barrier.  The barriers order the
// global-memory writes of one phase before the reads of the next within the
// workgroup; items never touch each other's memory.
template <class C>
__global__ __launch_bounds__(512) void kb_resident(const BItem<C>* __restrict__ items,
                                                                      const uint32_t* __restrict__ active,
                                                                      const uint32_t* __restrict__ status,
                                                                      int nsteps, uint32_t tstep) {
    const uint32_t it = active[blockIdx.x];
    if (status[it] != BS_ACTIVE) return;
    const BItem<C>& I = items[it];
    const Geo G = I.G;
    const Phys<typename C::R> P = I.P;
    typename C::T* S = I.S;
    typename C::R* M = I.M;
    const uint8_t* flags = I.flags;
    const DevLink<typename C::R>* links = I.links;
    const uint32_t nn = I.nnodes, nl = I.nlinks, bd = blockDim.x;
    const uint32_t t0 = step_time(I.tbase, tstep);
    for (int s = 0; s < nsteps; s += 2) {
        const uint32_t te = t0 + (uint32_t)s, to = te + 1u;
        for (uint32_t k = threadIdx.x; k < nl; k += bd) link_update<C, 0>(G, P, S, load_link(links + k), M, te);
        __syncthreads();
        for (uint32_t n = threadIdx.x; n < nn; n += bd) {
            NodeRes<C> r;
            node_update<C, 0, 0>(G, P, S, flags, M, n, r, te);
        }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < nl; k += bd) link_update<C, 1>(G, P, S, load_link(links + k), M, to);
        __syncthreads();
        for (uint32_t n = threadIdx.x; n < nn; n += bd) {
            NodeRes<C> r;
            node_update<C, 1, 0>(G, P, S, flags, M, n, r, to);
        }
        __syncthreads();
    }
}

// per-item FP64 sums over node tiles (after the links of the current time)
template <class C, int ODD>
__global__ __launch_bounds__(256) void kb_reduce(const BItem<C>* __restrict__ items,
                                                 const uint32_t* __restrict__ tiles,
                                                 const uint32_t* __restrict__ status,
                                                 const uint32_t* __restrict__ snap_ok, uint32_t ntiles) {
    const uint32_t b = blockIdx.x;
    if (b >= ntiles) return;
    const uint32_t it = tiles[2 * b];
    if (status[it] != BS_ACTIVE) return;
    const BItem<C>& I = items[it];
    const uint32_t n = tiles[2 * b + 1] + threadIdx.x;
    NodeRes<C> r;
    bool fluid = false;
    if (n < I.nnodes) fluid = node_update<C, ODD, 1>(I.G, I.P, I.S, I.flags, I.M, n, r);
    double v[NACC];
    reduce_node<C>(I.P, r, fluid, I.snap, (int)snap_ok[it], I.G.plane, n, v);
    block_accumulate(v, I.acc);
}

// One thread per active item: the steady-state residual from the sums of
// kb_reduce (the largest over u, C - C0, B - B_ext of |change| / (interval
// |value|)), the item's flags, then the accumulators cleared for the next
// evaluation.
template <class C>
__global__ __launch_bounds__(256) void kb_judge(const BItem<C>* __restrict__ items,
                                                const uint32_t* __restrict__ active, uint32_t nact,
                                                uint32_t* status, uint32_t* steps, double* resid,
                                                uint32_t* snap_ok, int interval, double tol) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nact) return;
    const uint32_t it = active[i];
    if (status[it] != BS_ACTIVE) return;
    double* a = items[it].acc;
    steps[it] += (uint32_t)interval;
    double res = -1.0;
    if (snap_ok[it]) {
        res = 0.0;
        for (int f = 0; f < 3; ++f) {
            if (a[8 + f] == 0.0 && a[5 + f] == 0.0) continue;
            res = fmax(res, sqrt(a[5 + f]) / ((double)interval * fmax(sqrt(a[8 + f]), 1e-30)));
        }
    }
    resid[it] = res;
    if (a[11] > 0.0) status[it] = BS_NONFINITE;
    else if (res >= 0.0 && res < tol) status[it] = BS_STEADY;
    snap_ok[it] = 1u;
    for (int q = 0; q < NACC; ++q) a[q] = 0.0;
}

// accumulators, counters and flags of the listed items back to their start
template <class C>
__global__ __launch_bounds__(256) void kb_clear(const BItem<C>* __restrict__ items,
                                                const uint32_t* __restrict__ active, uint32_t nact,
                                                uint32_t* status, uint32_t* steps, double* resid,
                                                uint32_t* snap_ok) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nact) return;
    const uint32_t it = active[i];
    double* a = items[it].acc;
    for (int q = 0; q < NACC; ++q) a[q] = 0.0;
    status[it] = BS_ACTIVE;
    steps[it] = 0u;
    resid[it] = -1.0;
    snap_ok[it] = 0u;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
inline Geo make_geo(const KArgs& a) {
    Geo g;
    g.NX = a.NX;
    g.NY = a.NY;
    g.NZ = a.NZ;
    g.hx = a.hx;
    g.hy = a.hy;
    g.hz = a.hz;
    g.n0 = a.n0;
    g.n1 = a.n1;
    g.n2 = a.n2;
    g.plane = (uint32_t)a.plane;
    g.wave_fluid = (uint32_t)a.wave_fluid;
    g.dx = make_fastdiv((uint32_t)a.NX);
    g.dy = make_fastdiv((uint32_t)a.NY);
    return g;
}

template <class C>
struct Launch {
    using R = typename C::R;
    static double cg2() { return C::QG == 19 ? 1.0 / 3.0 : (C::QG ? 0.25 : 1.0); }
    // Few links (a 2D channel's few thousand): 64 threads per block, so they
    // spread over four times as many CUs (3.1 -> 2.8 us per launch on the
    // 512 x 256 reactive channel).  Millions of links: 256 (with 64, the
    // pipe 1024 x 128 x 128 took 48 us instead of 37).
    static hipError_t links(const KArgs& a, const Geo& G, const Phys<R>& P) {
        if (!a.links_ready || a.n_links == 0) return hipSuccess;
        const int LB = a.n_links < 65536 ? 64 : 256;
        dim3 grid((unsigned)((a.n_links + LB - 1) / LB));
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, dim3(LB), 0, a.stream, G, P, (typename C::T*)a.S,
                               (const DevLink<R>*)a.links, (const R*)a.M, (uint32_t)a.n_links, a.tbase, a.tstep);
        };
        if (a.cmp_links)
            a.parity ? go(k_links<C, 1, true>) : go(k_links<C, 0, true>);
        else
            a.parity ? go(k_links<C, 1, false>) : go(k_links<C, 0, false>);
        return hipGetLastError();
    }
    static hipError_t flux(const KArgs& a) {
        if (a.n_links == 0) return hipSuccess;
        dim3 grid((unsigned)((a.n_links + 255) / 256));
        const Phys<R> P = make_phys<R>(a, cg2());
        const Geo G = make_geo(a);
        if (a.parity)
            hipLaunchKernelGGL((k_flux<C, 1>), grid, dim3(256), 0, a.stream, G, P, (typename C::T*)a.S,
                               (const DevLink<R>*)a.links, (const R*)a.M, (uint32_t)a.n_links, a.tstep, a.acc);
        else
            hipLaunchKernelGGL((k_flux<C, 0>), grid, dim3(256), 0, a.stream, G, P, (typename C::T*)a.S,
                               (const DevLink<R>*)a.links, (const R*)a.M, (uint32_t)a.n_links, a.tstep, a.acc);
        return hipGetLastError();
    }
    static hipError_t scale(const KArgs& a) {
        const uint32_t N = (uint32_t)((size_t)a.n0 * a.n1 * a.n2);
        hipLaunchKernelGGL((k_scale<C>), dim3((N + 255) / 256), dim3(256), 0, a.stream, (double*)a.out, N, a.norm_u,
                           a.norm_b);
        return hipGetLastError();
    }
    static hipError_t links_only(const KArgs& a) {
        return links(a, make_geo(a), make_phys<R>(a, cg2()));
    }
    static hipError_t step(const KArgs& a) {
        hipError_t e = links_only(a);
        if (e != hipSuccess) return e;
        return sweep(a);
    }
    static hipError_t sweep(const KArgs& a) {
        const uint32_t nn = (uint32_t)((size_t)a.NX * a.NY * a.NZ);
        const int bs = 256;
        dim3 grid((nn + bs - 1) / bs);
        const Phys<R> P = make_phys<R>(a, cg2());
        const Geo G = make_geo(a);
        if (a.parity)
            hipLaunchKernelGGL((k_step<C, 1>), grid, dim3(bs), 0, a.stream, G, P, (typename C::T*)a.S, a.flags,
                               (R*)a.M, nn, a.tbase, a.tstep);
        else
            hipLaunchKernelGGL((k_step<C, 0>), grid, dim3(bs), 0, a.stream, G, P, (typename C::T*)a.S, a.flags,
                               (R*)a.M, nn, a.tbase, a.tstep);
        return hipGetLastError();
    }
    static hipError_t sweep_waves(const KArgs& a) {
        if (a.n_waves == 0) return hipSuccess;
        const uint32_t nn = (uint32_t)((size_t)a.NX * a.NY * a.NZ);
        dim3 grid((a.n_waves + 3) / 4);
        const Phys<R> P = make_phys<R>(a, cg2());
        const Geo G = make_geo(a);
        if (a.parity)
            hipLaunchKernelGGL((k_step_waves<C, 1>), grid, dim3(256), 0, a.stream, G, P, (typename C::T*)a.S,
                               a.flags, (R*)a.M, nn, a.waves, a.n_waves, a.tbase, a.tstep);
        else
            hipLaunchKernelGGL((k_step_waves<C, 0>), grid, dim3(256), 0, a.stream, G, P, (typename C::T*)a.S,
                               a.flags, (R*)a.M, nn, a.waves, a.n_waves, a.tbase, a.tstep);
        return hipGetLastError();
    }
    static hipError_t set_time(const KArgs& a) {
        hipLaunchKernelGGL((k_time<C>), dim3(1), dim3(64), 0, a.stream, a.tbase, a.tstep, 0);
        return hipGetLastError();
    }
    static hipError_t tick(const KArgs& a) {
        hipLaunchKernelGGL((k_time<C>), dim3(1), dim3(64), 0, a.stream, a.tbase, a.tstep, 1);
        return hipGetLastError();
    }
    static hipError_t observe(const KArgs& a) {
        const uint32_t nn = (uint32_t)((size_t)a.NX * a.NY * a.NZ);
        dim3 grid((nn + 255) / 256);
        const Phys<R> P = make_phys<R>(a, cg2());
        const Geo G = make_geo(a);
        hipError_t e = links(a, G, P);
        if (e != hipSuccess) return e;
        if (a.parity)
            hipLaunchKernelGGL((k_observe<C, 1>), grid, dim3(256), 0, a.stream, G, P, (typename C::T*)a.S, a.flags,
                               (R*)a.M, nn, a.mode, a.field, a.out, a.out_f64, a.acc, a.acc_blocks, (R*)a.snap,
                               a.snap_valid);
        else
            hipLaunchKernelGGL((k_observe<C, 0>), grid, dim3(256), 0, a.stream, G, P, (typename C::T*)a.S, a.flags,
                               (R*)a.M, nn, a.mode, a.field, a.out, a.out_f64, a.acc, a.acc_blocks, (R*)a.snap,
                               a.snap_valid);
        return hipGetLastError();
    }
    static hipError_t init(const KArgs& a) {
        const uint32_t nn = (uint32_t)((size_t)a.NX * a.NY * a.NZ);
        dim3 grid((nn + 255) / 256);
        const Phys<R> P = make_phys<R>(a, cg2());
        const Geo G = make_geo(a);
        hipLaunchKernelGGL((k_init<C>), grid, dim3(256), 0, a.stream, G, P, (typename C::T*)a.S, a.flags, nn,
                           a.init_rho, a.init_u, a.init_C, a.init_B);
        return hipGetLastError();
    }
    // ---- batched items ----
    static size_t describe(const KArgs& a, void* out) {
        BItem<C> d;
        memset(&d, 0, sizeof d);
        d.G = make_geo(a);
        d.P = make_phys<R>(a, cg2());
        d.S = (typename C::T*)a.S;
        d.flags = a.flags;
        d.links = (const DevLink<R>*)a.links;
        d.M = (R*)a.M;
        d.snap = (R*)a.snap;
        d.acc = a.acc;
        d.tbase = a.tbase;
        d.t0 = a.tstep;
        d.nnodes = (uint32_t)((size_t)a.NX * a.NY * a.NZ);
        d.nlinks = a.links_ready ? (uint32_t)a.n_links : 0u;
        if (out) memcpy(out, &d, sizeof d);
        return sizeof d;
    }
    static hipError_t b_sweep(const BArgs& b) {
        if (b.n_tiles == 0) return hipSuccess;
        const BItem<C>* it = (const BItem<C>*)b.items;
        if (b.parity)
            hipLaunchKernelGGL((kb_sweep<C, 1>), dim3(b.n_tiles), dim3(b.tile), 0, b.stream, it, b.tiles, b.status,
                               b.n_tiles, b.tstep);
        else
            hipLaunchKernelGGL((kb_sweep<C, 0>), dim3(b.n_tiles), dim3(b.tile), 0, b.stream, it, b.tiles, b.status,
                               b.n_tiles, b.tstep);
        return hipGetLastError();
    }
    static hipError_t b_links(const BArgs& b) {
        if (b.n_ltiles == 0) return hipSuccess;
        const BItem<C>* it = (const BItem<C>*)b.items;
        if (b.parity)
            hipLaunchKernelGGL((kb_links<C, 1>), dim3(b.n_ltiles), dim3(256), 0, b.stream, it, b.ltiles, b.status,
                               b.n_ltiles, b.tstep);
        else
            hipLaunchKernelGGL((kb_links<C, 0>), dim3(b.n_ltiles), dim3(256), 0, b.stream, it, b.ltiles, b.status,
                               b.n_ltiles, b.tstep);
        return hipGetLastError();
    }
    static hipError_t b_resident(const BArgs& b) {
        if (b.n_active == 0) return hipSuccess;
        hipLaunchKernelGGL((kb_resident<C>), dim3(b.n_active), dim3(b.block), 0, b.stream,
                           (const BItem<C>*)b.items, b.active, b.status, b.nsteps, b.tstep);
        return hipGetLastError();
    }
    static hipError_t b_reduce(const BArgs& b) {
        hipError_t e = b_links(b);
        if (e != hipSuccess || b.n_tiles == 0) return e;
        const BItem<C>* it = (const BItem<C>*)b.items;
        if (b.parity)
            hipLaunchKernelGGL((kb_reduce<C, 1>), dim3(b.n_tiles), dim3(b.tile), 0, b.stream, it, b.tiles, b.status,
                               b.snap_ok, b.n_tiles);
        else
            hipLaunchKernelGGL((kb_reduce<C, 0>), dim3(b.n_tiles), dim3(b.tile), 0, b.stream, it, b.tiles, b.status,
                               b.snap_ok, b.n_tiles);
        return hipGetLastError();
    }
    static hipError_t b_judge(const BArgs& b) {
        if (b.n_active == 0) return hipSuccess;
        hipLaunchKernelGGL((kb_judge<C>), dim3((b.n_active + 255) / 256), dim3(256), 0, b.stream,
                           (const BItem<C>*)b.items, b.active, b.n_active, b.status, b.steps, b.resid, b.snap_ok,
                           b.interval, b.tol);
        return hipGetLastError();
    }
    static hipError_t b_clear(const BArgs& b) {
        if (b.n_active == 0) return hipSuccess;
        hipLaunchKernelGGL((kb_clear<C>), dim3((b.n_active + 255) / 256), dim3(256), 0, b.stream,
                           (const BItem<C>*)b.items, b.active, b.n_active, b.status, b.steps, b.resid, b.snap_ok);
        return hipGetLastError();
    }

    static hipError_t b_set_time(const BArgs& b) {
        if (b.n_active == 0) return hipSuccess;
        hipLaunchKernelGGL((kb_time<C>), dim3((b.n_active + 255) / 256), dim3(256), 0, b.stream,
                           (const BItem<C>*)b.items, (const uint32_t*)nullptr, b.n_active, 0u);
        return hipGetLastError();
    }
    static hipError_t b_tick(const BArgs& b) {
        if (b.n_active == 0) return hipSuccess;
        hipLaunchKernelGGL((kb_time<C>), dim3((b.n_active + 255) / 256), dim3(256), 0, b.stream,
                           (const BItem<C>*)b.items, b.active, b.n_active, b.tstep);
        return hipGetLastError();
    }

    static KernelSet set() {
        KernelSet k;
        k.set_time = &set_time;
        k.tick = &tick;
        k.b_set_time = &b_set_time;
        k.b_tick = &b_tick;
        k.describe = &describe;
        k.item_bytes = sizeof(BItem<C>);
        k.b_sweep = &b_sweep;
        k.b_links = &b_links;
        k.b_resident = &b_resident;
        k.b_reduce = &b_reduce;
        k.b_judge = &b_judge;
        k.b_clear = &b_clear;
        k.links = &links_only;
        k.sweep = &sweep;
        k.sweep_waves = &sweep_waves;
        k.step = &step;
        k.flux = &flux;
        k.scale = &scale;
        k.observe = &observe;
        k.init = &init;
        k.QT = C::QT;
        k.MW = C::MW;
        return k;
    }
};

// the lattice combinations the library instantiates
template <class SF>
KernelSet select_kernels(int fl, int sl, int ml, int nc, int ns) {
#define LBM_CASE(F, H, M, N)                                                \
    if (fl == F && sl == H && ml == M && (M == 0 || nc == N) && ns <= 1) \
        return Launch<Cfg<F, H, M, N, SF>>::set();
    // several scalar components: flow and scalar lattices only
#define LBM_CASE_NS(F, H, S)                          \
    if (fl == F && sl == H && ml == 0 && ns == S) \
        return Launch<Cfg<F, H, 0, 0, SF, S>>::set();
    LBM_CASE_NS(1, 3, 2)
    LBM_CASE_NS(1, 3, 3)
    LBM_CASE_NS(2, 4, 2)
    LBM_CASE_NS(2, 4, 3)
#undef LBM_CASE_NS
    LBM_CASE(1, 0, 0, 0)
    LBM_CASE(1, 3, 0, 0)
    LBM_CASE(1, 0, 3, 1)
    LBM_CASE(1, 0, 3, 2)
    LBM_CASE(1, 3, 3, 1)
    LBM_CASE(1, 3, 3, 2)
    LBM_CASE(2, 0, 0, 0)
    LBM_CASE(2, 4, 0, 0)
    LBM_CASE(2, 0, 4, 1)
    LBM_CASE(2, 0, 4, 3)
    LBM_CASE(2, 4, 4, 1)
    LBM_CASE(2, 4, 4, 3)
    LBM_CASE(2, 0, 2, 1)
#undef LBM_CASE
    return KernelSet{};
}

}  // namespace lbmi
