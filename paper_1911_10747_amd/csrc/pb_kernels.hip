// HIP kernels (gfx950) for one time step of the hybrid pseudopotential
// phase-change LBM with conjugate heat transfer (arXiv:1911.10747, Section 2).
//
// Two launches per step, both stencils with no dense contraction (no MFMA); the
// flow launch is bound by HBM traffic, the energy-equation launch by VALU
// issue:
//   k_flow     pull streaming (Eq. 8, halfway bounce-back, periodic x), the
//              macroscopic update (Eq. 10), psi from the Peng-Robinson EOS
//              (Eqs. 12-13) staged with a one-node halo in LDS, the forces
//              (Eqs. 11, 14, 15), MRT collision with the improved forcing
//              (Eqs. 3-7, 9) and the store of f*, rho(t), v(t).
//   k_thermal  the energy equation (Eq. 24) advanced by RK4 (Eqs. 25-26) with
//              the isotropic stencils (Eqs. 27-28) over fluid and heater; one
//              wavefront sweeps a strip of columns upwards with the four
//              stages pipelined over consecutive rows in registers, so T, rho
//              and v are read from HBM once per step (plus the strip halos).
// plus k_flux (heat flux of Eqs. 36, 38-39, FP64, fixed reduction order),
// k_init (rest equilibrium) and k_advance (time/parity bookkeeping on device).
//
// Layout: SoA populations f[i][y][x] with x fastest and a padded row pitch; a
// wavefront covers 64 consecutive x of one row, so every pull and store is a
// coalesced row segment.  The flow step computes in FP64; PB_FP32_DEV stores
// rho(x) in FP32 and f*_i - w_i rho(x) in FP32 against that stored density
// (so the FP64 rebuild on load is exact up to the rounding of the deviation),
// and runs the energy equation in FP32 increments over FP64 T (see the FP32
// sweep below).
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "pb_internal.h"

namespace {

// D2Q9 velocities in the order of Eq. 2 and the opposite directions.
__device__ constexpr int kEX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kEY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// lattice weights (rest equilibrium, Eqs. 27-28)
__device__ constexpr double kW[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                                     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
// interaction-force weights w(|e|^2) of Eq. 11: 1/3 (axis), 1/12 (diagonal)
__device__ constexpr double kWF[9] = {0.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0,
                                      1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0};

constexpr uint32_t F_PERY = 0x1u, F_FROZEN = 0x4u, F_FMONLY = 0x10u;

__device__ __forceinline__ int wrap_once(int v, int n) {
    v += (v < 0) ? n : 0;
    v -= (v >= n) ? n : 0;
    return v;
}

// Address-space views: descriptors are read through the constant space
// (scalar loads), field arrays through the global space.
#define PB_CAS __attribute__((address_space(4)))
#define PB_GAS __attribute__((address_space(1)))
typedef const PbDesc PB_CAS cdesc;

template <typename T>
__device__ __forceinline__ const T PB_GAS *gcast(const void *p) { return (const T PB_GAS *)p; }
template <typename T>
__device__ __forceinline__ T PB_GAS *gcast_w(void *p) { return (T PB_GAS *)p; }

__device__ __forceinline__ void flag_error(cdesc &d) { atomicOr(d.err, 1); }

// The element at a 32-bit byte offset from a base that is the same for every
// lane, written so that the access can take the base from scalar registers
// and the offset from one vector register instead of a 64-bit address per
// lane (the flow's stores compile so: 12 fewer vector instructions a node).
template <typename V>
__device__ __forceinline__ V at_byte(const V PB_GAS *base, uint32_t boff) {
    return *(const V PB_GAS *)((const char PB_GAS *)base + boff);
}
template <typename V>
__device__ __forceinline__ V PB_GAS *at_byte_w(V PB_GAS *base, uint32_t boff) {
    return (V PB_GAS *)((char PB_GAS *)base + boff);
}

// reciprocal and square root from the hardware approximations refined by
// Newton steps (within about one ulp of the correctly rounded values)
__device__ __forceinline__ double frcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}
__device__ __forceinline__ double fsqrt(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * y, g = x * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double e = fma(-g, g, x);
    g = fma(e, h, g);
    return x == 0.0 ? 0.0 : g;   // negative x gives NaN through rsq
}

// Eq. 13 and Eq. 12 (c = 1, c_s^2 = 1/3) with a single division; sets bad on a
// negative radicand.
__device__ __forceinline__ double eos_psi(cdesc &d, double rho, double T, bool &bad) {
    const double s = d.eos_s0 - d.eos_s1 * fsqrt(T);    // 1 + kappa (1 - sqrt(T / Tc))
    const double br = d.b * rho;
    const double den1 = 1.0 - br, den2 = 1.0 + 2.0 * br - br * br;
    const double P = (rho * d.R * T * den2 - d.a * (s * s) * rho * rho * den1) * frcp(den1 * den2);
    const double rad = (P - rho * (1.0 / 3.0)) * d.two_invG;
    bad = bad || !(rad >= 0.0);
    return fsqrt(rad);
}

// Pull f_i(x, y, t) = f*_i(x - e_i, t-1), halfway bounce-back at the walls
// (general path, any node).  FP32 deviation storage rebuilds
// f* = w_i rho_ref + delta with rho_ref the stored (FP32) density of the node
// the value was stored at, the same value its encoding used.
template <typename FT>
__device__ __forceinline__ void pull_node(cdesc &d, const FT PB_GAS *fin, const FT PB_GAS *rin, int x, int y,
                                          bool pery, double f[9]) {
    const uint32_t plane = (uint32_t)d.nyf * (uint32_t)d.pitch;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int xs = wrap_once(x - kEX[i], d.nx);
        int ys = y - kEY[i];
        int ii = i;
        if (pery) {
            ys = wrap_once(ys, d.nyf);
        } else if (ys < 0 || ys >= d.nyf) {
            ii = kOPP[i];
            xs = x;
            ys = y;
        }
        const uint32_t idx = (uint32_t)ys * (uint32_t)d.pitch + (uint32_t)xs;
        const FT v = fin[(uint32_t)ii * plane + idx];
        if constexpr (std::is_same<FT, float>::value)
            f[i] = kW[i] * (double)rin[idx] + (double)v;
        else
            f[i] = v;
    }
}

// Same pull for a node whose nine sources are all inside the fluid and away
// from the x edges: constant offsets, no branches.
template <typename FT>
__device__ __forceinline__ void pull_inner(const FT PB_GAS *fin, const FT PB_GAS *rin, uint32_t plane,
                                           uint32_t pitch, uint32_t idx, double f[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const uint32_t src = idx - (uint32_t)(kEY[i] * (int)pitch) - (uint32_t)kEX[i];
        const FT v = (fin + (uint32_t)i * plane)[src];
        if constexpr (std::is_same<FT, float>::value)
            f[i] = kW[i] * (double)rin[src] + (double)v;
        else
            f[i] = v;
    }
}

// Same pull split in two for FP32 storage, with the reference densities of
// the decode taken from an LDS copy of rho(t-1) over the tile plus two rings
// (row stride RW, node at (lx, ly) of that copy), so that the loads of a tile
// can be in flight before that copy is complete.
__device__ __forceinline__ void load_inner_raw(const float PB_GAS *fin, uint32_t plane, uint32_t pitch, uint32_t idx,
                                               float v[9]) {
    // raw buffer loads: a descriptor per shifted plane (its base the plane's
    // element -e_i, so every address is at or above the array's start) in
    // scalar registers, and the node's 32-bit byte offset in one vector
    // register, so no lane computes a 64-bit address (the kernel measured
    // 1.0 us faster than with global loads)
    const uint32_t boff = idx * 4u;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const float PB_GAS *b = fin + ((int64_t)i * plane - (int64_t)kEY[i] * pitch - kEX[i]);
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void *)b, (short)0, -1, 0x00020000);
        v[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, boff, 0, 0));
    }
}
// load_inner_raw for a node within a row of the fluid whose x neighbours
// wrap periodically (the tiles at the x edges): the source column of each
// population is x - 1, x or x + 1 taken modulo nx, per lane
__device__ __forceinline__ void load_wrap_raw(const float PB_GAS *fin, uint32_t plane, uint32_t pitch, int x, int y,
                                              int nx, float v[9]) {
    const uint32_t xm = (uint32_t)wrap_once(x - 1, nx), xp = (uint32_t)wrap_once(x + 1, nx);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const uint32_t xs = kEX[i] == 0 ? (uint32_t)x : (kEX[i] > 0 ? xm : xp);   // x - e_x
        const uint32_t boff = ((uint32_t)(y - kEY[i]) * pitch + xs) * 4u;
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc((void *)(fin + (uint32_t)i * plane), (short)0, -1, 0x00020000);
        v[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, boff, 0, 0));
    }
}
template <int RW>
__device__ __forceinline__ void decode_lds(const float *s_rho, int lx, int ly, const float v[9], double f[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = kW[i] * (double)s_rho[(ly - kEY[i]) * RW + lx - kEX[i]] + (double)v[i];
}

// Where a node's outputs go: global pointers at element offset oidx.  The
// stores are non-temporal: the next reader is the next launch, after the whole
// domain has streamed through L2, so keeping them out of L2 leaves it to the
// halo re-reads (4096 x 2112, FP32: flow 191 -> 185 us, and the energy launch
// after it 74.9 -> 71.9 us).
template <typename FT>
struct GlobalStore {
    FT PB_GAS *f;
    FT PB_GAS *rho;
    FT PB_GAS *vx;
    FT PB_GAS *vy;
    uint32_t plane, oidx;
    __device__ __forceinline__ void pop(int i, FT v) const {
        __builtin_nontemporal_store(v, at_byte_w(f + (size_t)i * plane, oidx * (uint32_t)sizeof(FT)));
    }
    __device__ __forceinline__ void fields(double r, FT ux, FT uy) const {
        const uint32_t boff = oidx * (uint32_t)sizeof(FT);
        __builtin_nontemporal_store((FT)r, at_byte_w(rho, boff));
        __builtin_nontemporal_store(ux, at_byte_w(vx, boff));
        __builtin_nontemporal_store(uy, at_byte_w(vy, boff));
    }
};



// ------------------------------------------------------------ node update
// Moments of the pulled populations: rho and j (Eq. 10 without the force)
// and the non-conserved rows of m = M f (Eq. 6) the collision relaxes.
struct Mom {
    double rho, jx, jy, m1, m2, m4, m6, m7, m8;
};
// rho = sum of the f_i in one fixed grouping, used wherever a density is
// summed from pulled populations (a node's own tile and the tiles that hold
// it in their psi ring must get the same bits)
__device__ __forceinline__ double node_rho(const double f[9]) {
    return f[0] + (((f[1] + f[3]) + (f[2] + f[4])) + ((f[5] + f[7]) + (f[6] + f[8])));
}
__device__ __forceinline__ Mom node_moments(const double f[9]) {
    // the rows of M from shared partial sums (e_1..e_8 = E, N, W, S, NE, NW,
    // SW, SE): a = f1 - f3, b = f2 - f4, c = f5 - f7, e = f6 - f8
    const double a = f[1] - f[3], b = f[2] - f[4], c = f[5] - f[7], e = f[6] - f[8];
    const double sa = (f[1] + f[3]) + (f[2] + f[4]), sd = (f[5] + f[7]) + (f[6] + f[8]);
    const double cme = c - e, cpe = c + e;
    Mom m;
    m.rho = node_rho(f);
    m.jx = a + cme;                       // f1 - f3 + f5 - f6 - f7 + f8
    m.jy = b + cpe;                       // f2 - f4 + f5 + f6 - f7 - f8
    m.m1 = -4.0 * f[0] - sa + 2.0 * sd;
    m.m2 = 4.0 * f[0] - 2.0 * sa + sd;
    m.m4 = -2.0 * a + cme;
    m.m6 = -2.0 * b + cpe;
    m.m7 = (f[1] + f[3]) - (f[2] + f[4]);
    m.m8 = (f[5] + f[7]) - (f[6] + f[8]);
    return m;
}

// sum over i = 1..8 of w(|e_i|^2) e_i p_i (Eqs. 11 and 14) from the
// differences of opposite neighbours: (1/3)(p1 - p3, p2 - p4) plus
// (1/12)(c - e, c + e) with c = p5 - p7, e = p6 - p8
__device__ __forceinline__ void weighted_sum(const double p[9], double &sx, double &sy) {
    const double c = p[5] - p[7], e = p[6] - p[8];
    sx = kWF[1] * (p[1] - p[3]) + kWF[5] * (c - e);
    sy = kWF[2] * (p[2] - p[4]) + kWF[5] * (c + e);
}

// Forces, velocity and collision of one fluid node from the moments mo of its
// pulled populations f (f itself is used in read mode only), its psi and,
// for i = 1..8, psi of the neighbour
// x + e_i (pn[i]) or, where bit i of wmask marks that neighbour as a wall,
// the wall's adhesion gamma (gw[i]).  Writes f*, rho(t), v(t) at oidx (or, in
// read mode, the pulled state).  Returns true if the node is not finite.
// Every flow kernel updates its nodes through this one function, so a node
// gives the same bits whatever the launch shape.
template <typename FT, int MODE>
__device__ __forceinline__ bool node_update(cdesc &d, const double f[9], const Mom &mo, double psi,
                                            const double pn[9], const double gw[9], uint32_t wmask, uint32_t oidx,
                                            const GlobalStore<FT> &st) {
    const double rho = mo.rho, jx = mo.jx, jy = mo.jy;
    const bool frozen = (d.flags & F_FROZEN) != 0;
    // Eq. 11 over fluid neighbours (a wall neighbour's psi counts as 0), Eq. 14
    // over wall neighbours (gw is 0 off the walls)
    double pf[9];
#pragma unroll
    for (int i = 1; i < 9; ++i) pf[i] = ((wmask >> i) & 1u) ? 0.0 : pn[i];
    double sfx, sfy, sax, say;
    weighted_sum(pf, sfx, sfy);
    const double Fmx = -d.G * psi * sfx, Fmy = -d.G * psi * sfy;
    // a node with no wall neighbour (every node of an inner tile) has F_ads = 0
    // and skips it
    const bool walls = wmask != 0u;
    double Fsx = Fmx, Fsy = Fmy;            // F_m + F_ads
    if (walls) {
        weighted_sum(gw, sax, say);
        Fsx = Fmx - psi * sax;
        Fsy = Fmy - psi * say;
    }
    const double Fx = Fsx;
    const double Fy = Fsy - (rho - d.rho_bar) * d.g;       // Eq. 15
    // 1/rho, 1/psi^2 and s_nu = 1/tau(rho) (Eq. 5) from one reciprocal of
    // their product (batch inversion)
    const double psi2 = psi * psi, tau = d.tau_V + (rho - d.rho_V) * d.ktau;
    const double pr = rho * psi2;
    double rr = frcp(pr * tau);
    const double snu = rr * pr;
    rr = rr * tau;
    const double inv_rho = rr * psi2, inv_psi2 = rr * rho;
    double vx = (jx + 0.5 * Fx) * inv_rho;                         // Eq. 10
    double vy = (jy + 0.5 * Fy) * inv_rho;
    if (frozen) { vx = 0.0; vy = 0.0; }

    if constexpr (MODE == PB_MODE_READ) {
        // the read-back staging holds dense rows ([nyf][nx] per field), so the
        // host copies it out in one contiguous piece per field
        const uint32_t y = oidx / (uint32_t)d.pitch, x = oidx - y * (uint32_t)d.pitch;
        const uint32_t didx = y * (uint32_t)d.nx + x, dplane = (uint32_t)d.nyf * (uint32_t)d.nx;
        double PB_GAS *rdf = gcast_w<double>(d.rd_f);
#pragma unroll
        for (int i = 0; i < 9; ++i) (rdf + (uint32_t)i * dplane)[didx] = f[i];
        gcast_w<double>(d.rd_rho)[didx] = rho;
        gcast_w<double>(d.rd_vx)[didx] = vx;
        gcast_w<double>(d.rd_vy)[didx] = vy;
    } else {
        const double m1 = mo.m1, m2 = mo.m2, m4 = mo.m4, m6 = mo.m6, m7 = mo.m7, m8 = mo.m8;
        // equilibria (Eq. 6) with u = v of Eq. 10
        const double u2 = vx * vx + vy * vy;
        const double meq1 = rho * (-2.0 + 3.0 * u2), meq2 = rho * (1.0 - 3.0 * u2);
        const double meq4 = -rho * vx, meq6 = -rho * vy;
        const double meq7 = rho * (vx * vx - vy * vy), meq8 = rho * vx * vy;
        // forcing of Eq. 9; the varpi term times (1 - s_e/2) equals
        // 12 varpi s_e |F|^2 / psi^2 because tau_e = 1/s_e
        const double Fwx = (d.flags & F_FMONLY) ? Fmx : Fsx;
        const double Fwy = (d.flags & F_FMONLY) ? Fmy : Fsy;
        const double uF = vx * Fx + vy * Fy;
        const double cw = d.cw_k * (Fwx * Fwx + Fwy * Fwy) * inv_psi2;
        const double cw2 = d.s2sign * cw;
        const double se = d.s_e, sq = d.s_q;
        const double ms1 = m1 - se * (m1 - meq1) + d.hse * (6.0 * uF) + cw;
        const double ms2 = m2 - se * (m2 - meq2) + d.hse * (-6.0 * uF) + cw2;
        const double ms3 = jx + Fx;                       // s_j drops out (Eq. 7 + Eq. 10)
        const double ms4 = m4 - sq * (m4 - meq4) + d.hsq * (-Fx);
        const double ms5 = jy + Fy;
        const double ms6 = m6 - sq * (m6 - meq6) + d.hsq * (-Fy);
        const double ms7 = m7 - snu * (m7 - meq7) + (1.0 - 0.5 * snu) * (2.0 * (vx * Fx - vy * Fy));
        const double ms8 = m8 - snu * (m8 - meq8) + (1.0 - 0.5 * snu) * (vx * Fy + vy * Fx);
        // f* = M^{-1} m*, M^{-1} = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
        const double a0 = rho * (1.0 / 9.0), a1 = ms1 * (1.0 / 36.0), a2 = ms2 * (1.0 / 36.0);
        const double a3 = ms3 * (1.0 / 6.0), a4 = ms4 * (1.0 / 12.0), a5 = ms5 * (1.0 / 6.0);
        const double a6 = ms6 * (1.0 / 12.0), a7 = ms7 * 0.25, a8 = ms8 * 0.25;
        // FP32 storage keeps f* - w_i rho_ref (the deviation) with rho_ref =
        // rho(t) rounded to FP32, the density stored beside it: w_i rho_ref is
        // taken off the rest term and the terms common to the axis and to the
        // diagonal populations.  FP64 storage keeps f* itself.
        double p0, c0, cd;
        if constexpr (std::is_same<FT, float>::value) {
            const double rref = (double)(float)rho;
            p0 = a0 - 4.0 * a1 + 4.0 * a2 - kW[0] * rref;
            c0 = a0 - a1 - 2.0 * a2 - kW[1] * rref;
            cd = a0 + 2.0 * a1 + a2 - kW[5] * rref;
        } else {
            p0 = a0 - 4.0 * a1 + 4.0 * a2;
            c0 = a0 - a1 - 2.0 * a2;       // axis-common part
            cd = a0 + 2.0 * a1 + a2;       // diagonal-common part
        }
        st.pop(0, (FT)p0);
        st.pop(1, (FT)(c0 + a3 - 2.0 * a4 + a7));
        st.pop(2, (FT)(c0 + a5 - 2.0 * a6 - a7));
        st.pop(3, (FT)(c0 - a3 + 2.0 * a4 + a7));
        st.pop(4, (FT)(c0 - a5 + 2.0 * a6 - a7));
        st.pop(5, (FT)(cd + a3 + a4 + a5 + a6 + a8));
        st.pop(6, (FT)(cd - a3 - a4 + a5 + a6 - a8));
        st.pop(7, (FT)(cd - a3 - a4 - a5 - a6 + a8));
        st.pop(8, (FT)(cd + a3 + a4 - a5 - a6 - a8));
        st.fields(rho, (FT)vx, (FT)vy);      // rho and v in FP32 with FP32 storage
    }
    return !(rho == rho) || !__builtin_isfinite(vx) || !__builtin_isfinite(vy);
}

// ---------------------------------------------------------------- flow step
// Code paths of a flow tile.  PATH_INNER: every node of the tile and its ring
// is at least two nodes from the x edges and from the walls.  PATH_XWRAP
// (FP32 storage): the same two nodes from the walls, a periodic y absent, and
// x positions taken modulo nx (nx >= BX + 4, so one wrap reaches every
// position the tile uses).  PATH_GENERAL: any tile.
enum : int { PATH_GENERAL = 0, PATH_INNER = 1, PATH_XWRAP = 2 };

// One tile: psi over the tile plus a one-node ring in LDS, then forces,
// velocity and collision on the tile.
template <typename FT, int BX, int BY, int MODE, int PATH>
__device__ __forceinline__ void flow_tile(cdesc &d, const PbTile &te, int k, double *s_psi, FT *s_rho,
                                          int *s_bad) {
    constexpr bool INNER = PATH == PATH_INNER, XWRAP = PATH == PATH_XWRAP;
    static_assert(!XWRAP || std::is_same<FT, float>::value, "x-wrapped tiles use the FP32 LDS decode");
    constexpr int RW = BX + 4, RH = BY + 4;        // rho(t-1) copy: tile plus two rings
    constexpr bool RLDS = (INNER || XWRAP) && std::is_same<FT, float>::value;
    constexpr int LW = BX + 2, LH = BY + 2;
    constexpr int NHALO = 2 * LW + 2 * BY;
    // the thread index through an empty asm, so that what is derived from it
    // is formed per tile instead of being hoisted out of the tile loop and
    // held in registers across it
    int tid = (int)threadIdx.x;
    __asm__ volatile("" : "+v"(tid));
    const int tx = tid % BX, ty = tid / BX;
    const bool pery = (d.flags & F_PERY) != 0;
    const int pin = (int)((d.par0 + k) & 1), pout = pin ^ 1;
    const FT PB_GAS *fin = gcast<FT>(d.f[pin]);
    const FT PB_GAS *rin = gcast<FT>(d.rho[pin]);
    const double PB_GAS *Tt = gcast<double>(d.T[pin]);
    const uint32_t pitch = (uint32_t)d.pitch, plane = (uint32_t)d.nyf * pitch;
    const uint32_t toff = (uint32_t)d.nys * pitch;           // fluid row 0 in the T array
    bool bad = false;

    // this thread's node; positions past the edge wrap once so that the first
    // column/row beyond holds the periodic neighbour
    const int xr = te.x0 + tx, yr = te.y0 + ty;
    const bool own = INNER || (xr < d.nx && yr < d.nyf);
    const int xw = INNER ? xr : xr - (xr >= d.nx ? d.nx : 0);
    const int yw = (INNER || !pery) ? yr : yr - (yr >= d.nyf ? d.nyf : 0);
    const bool live = INNER || (xw < d.nx && yw < d.nyf);
    double f[9], psi = 0.0;
    Mom mo{};
    const uint32_t idx = (uint32_t)yw * pitch + (uint32_t)xw;

    // ring node of psi around the tile handled by this thread, if any
    const bool has_h = tid < NHALO;
    int lx = 0, ly = 0;
    {
        const int h = tid;
        if (h < LW) { lx = h; ly = 0; }
        else if (h < 2 * LW) { lx = h - LW; ly = LH - 1; }
        else if (h < 2 * LW + BY) { lx = 0; ly = h - 2 * LW + 1; }
        else { lx = LW - 1; ly = h - 2 * LW - BY + 1; }
    }

    if constexpr (RLDS) {
        // Every load of the tile is issued before the first wait: the rho(t-1)
        // copy (tile plus two rings, all inside the fluid since the tile is two
        // nodes from the walls; columns modulo nx on the x-wrapped path), then
        // the populations and T of this thread's node and of its ring node.
        // thread (tx, ty) copies columns tx + i BX of rows ty + j BY, so the
        // copy needs no index arithmetic beyond the thread's own position
        constexpr int NI = (RW + BX - 1) / BX, NJ = (RH + BY - 1) / BY;
        float rq[NJ][NI];
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                const int c = tx + i * BX, r = ty + j * BY;
                const int xc = XWRAP ? wrap_once(te.x0 - 2 + c, d.nx) : te.x0 - 2 + c;
                if (c < RW && r < RH) rq[j][i] = rin[(uint32_t)(te.y0 - 2 + r) * pitch + (uint32_t)xc];
            }
        float v[9], vh[9];
        if (XWRAP) load_wrap_raw(fin, plane, pitch, xw, yw, d.nx, v);
        else load_inner_raw(fin, plane, pitch, idx, v);
        const double Tn = at_byte(Tt + toff, idx * 8u);
        const int xh = XWRAP ? wrap_once(te.x0 + lx - 1, d.nx) : te.x0 + lx - 1, yh = te.y0 + ly - 1;
        const uint32_t hidx = (uint32_t)yh * pitch + (uint32_t)xh;
        double Th = 0.0;
        if (has_h) {
            if (XWRAP) load_wrap_raw(fin, plane, pitch, xh, yh, d.nx, vh);
            else load_inner_raw(fin, plane, pitch, hidx, vh);
            Th = at_byte(Tt + toff, hidx * 8u);
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                const int c = tx + i * BX, r = ty + j * BY;
                if (c < RW && r < RH) s_rho[r * RW + c] = rq[j][i];
            }
        __syncthreads();
        // a block past its loads computes at raised wave priority, so it gets
        // to its stores and frees its slot sooner (0.7 us per launch)
        __builtin_amdgcn_s_setprio(2);
        decode_lds<RW>(s_rho, tx + 2, ty + 2, v, f);
        mo = node_moments(f);
        psi = eos_psi(d, mo.rho, Tn, bad);
        s_psi[(ty + 1) * LW + tx + 1] = psi;
        if (has_h) {
            double fh[9];
            decode_lds<RW>(s_rho, lx + 1, ly + 1, vh, fh);
            const double rh = node_rho(fh);
            bool dummy = false;  // errors are flagged by the owning tile
            s_psi[ly * LW + lx] = eos_psi(d, rh, Th, dummy);
        }
    } else {
        if (live) {
            if (INNER) pull_inner<FT>(fin, rin, plane, pitch, idx, f);
            else pull_node<FT>(d, fin, rin, xw, yw, pery, f);
            mo = node_moments(f);
            psi = eos_psi(d, mo.rho, Tt[toff + idx], bad);
        }
        s_psi[(ty + 1) * LW + tx + 1] = psi;
        if (has_h) {
            int xh = te.x0 + lx - 1, yh = te.y0 + ly - 1;
            bool ok = true;
            if (!INNER) {
                xh = wrap_once(xh, d.nx);
                ok = xh >= 0 && xh < d.nx;
                if (pery) yh = wrap_once(yh, d.nyf);
                ok = ok && yh >= 0 && yh < d.nyf;
            }
            double ph = 0.0;
            if (ok) {
                double fh[9];
                const uint32_t hidx = (uint32_t)yh * pitch + (uint32_t)xh;
                if (INNER) pull_inner<FT>(fin, rin, plane, pitch, hidx, fh);
                else pull_node<FT>(d, fin, rin, xh, yh, pery, fh);
                const double rh = node_rho(fh);
                bool dummy = false;  // errors are flagged by the owning tile
                ph = eos_psi(d, rh, Tt[toff + hidx], dummy);
            }
            s_psi[ly * LW + lx] = ph;
        }
    }
    __syncthreads();

    if (own) {
        double pn[9], gw[9];
        uint32_t wmask = 0;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const int yn = yr + kEY[i];
            const bool wall = PATH == PATH_GENERAL && !pery && (yn < 0 || yn >= d.nyf);
            pn[i] = s_psi[(ty + 1 + kEY[i]) * LW + tx + 1 + kEX[i]];
            gw[i] = 0.0;
            if (wall) {
                const int xn = wrap_once(xr + kEX[i], d.nx);
                gw[i] = (yn < 0) ? d.gbot[xn] : d.gtop[xn];
                wmask |= 1u << i;
            }
        }
        const uint32_t oidx = (uint32_t)yr * pitch + (uint32_t)xr;
        const GlobalStore<FT> st{gcast_w<FT>(d.f[pout]), gcast_w<FT>(d.rho[pout]), gcast_w<FT>(d.vx),
                                 gcast_w<FT>(d.vy), plane, oidx};
        if (node_update<FT, MODE>(d, f, mo, psi, pn, gw, wmask, oidx, st) || bad)
            *s_bad = 1;
    }
}

// One tile of shape TX x TY by the path its position allows.
template <typename FT, int TX, int TY, int MODE>
__device__ __forceinline__ void flow_tile_any(cdesc &d, const PbTile &te, int k, double *s_psi, FT *s_rho,
                                              int *s_bad) {
    const bool yin = !(d.flags & F_PERY) && te.y0 >= 2 && te.y0 + TY + 2 <= d.nyf;
    if (yin && te.x0 >= 2 && te.x0 + TX + 2 <= d.nx) {
        flow_tile<FT, TX, TY, MODE, PATH_INNER>(d, te, k, s_psi, s_rho, s_bad);
    } else if constexpr (std::is_same<FT, float>::value) {
        if (yin && d.nx >= TX + 4) flow_tile<FT, TX, TY, MODE, PATH_XWRAP>(d, te, k, s_psi, s_rho, s_bad);
        else flow_tile<FT, TX, TY, MODE, PATH_GENERAL>(d, te, k, s_psi, s_rho, s_bad);
    } else {
        flow_tile<FT, TX, TY, MODE, PATH_GENERAL>(d, te, k, s_psi, s_rho, s_bad);
    }
}

// Alternate tile of 512-thread FP32 launches wider than 32: 32 x 16, for the
// columns past a domain's last full tile (a partial tile computes as much as
// a full one, so a remainder of 32 columns or fewer costs half as much in
// 32 x 16 tiles)
template <typename FT, int BX, int BY>
constexpr bool kFlowAlt = std::is_same<FT, float>::value && BX * BY == 512 && BX > 32;
constexpr int kAltX = 32, kAltY = 16;

// 512-thread stepping blocks are held to 80 VGPRs with FP32 storage, 6
// waves per SIMD (three blocks per CU), and to 64 with FP64 storage, 8 waves
// per SIMD (four blocks per CU).  ALT: the work list holds alternate tiles (a
// separate kernel, so that launches without them keep the smaller code)
template <typename FT, int BX, int BY, int MODE, bool ALT>
__global__ __launch_bounds__(BX *BY, (BX * BY == 512 && MODE == PB_MODE_STEP ? (sizeof(FT) == 8 ? 8 : 6) : 1))
void k_flow(const PbDesc *const *__restrict__ dps, const PbTile *__restrict__ tiles, int ntiles, int k) {
    static_assert(!ALT || kFlowAlt<FT, BX, BY>, "no alternate tiles for this launch shape");
    constexpr int NPSI = std::max((BX + 2) * (BY + 2), ALT ? (kAltX + 2) * (kAltY + 2) : 0);
    constexpr int NRHO = std::max((BX + 4) * (BY + 4), ALT ? (kAltX + 4) * (kAltY + 4) : 0);
    static_assert(2 * (BX + 2) + 2 * BY <= BX * BY, "halo larger than block");
    __shared__ double s_psi[NPSI];
    __shared__ FT s_rho[NRHO];
    __shared__ int s_bad;
    for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const PbTile te = tiles[tl];
        cdesc &d = *(const PbDesc PB_CAS *)dps[te.dom];
        if (threadIdx.x == 0) s_bad = 0;
        if constexpr (ALT) {
            if (te.alt) flow_tile_any<FT, kAltX, kAltY, MODE>(d, te, k, s_psi, s_rho, &s_bad);
            else flow_tile_any<FT, BX, BY, MODE>(d, te, k, s_psi, s_rho, &s_bad);
        } else {
            flow_tile_any<FT, BX, BY, MODE>(d, te, k, s_psi, s_rho, &s_bad);
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        if (threadIdx.x == 0 && s_bad) flag_error(d);
        __syncthreads();
    }
}

// Thermal node kinds.
enum : int { KIND_NONE = 0, KIND_FIXED = 1, KIND_SOLID = 2, KIND_FLUID = 3 };

// ----------------------------------------------------- energy step (sweep)
// Column-sweep form of the same RK4 update.  One wavefront owns 64
// consecutive columns (56 are written; four on each side are halo) and walks
// up a strip of H thermal rows plus four halo rows below and above.  At the
// row n it has just loaded it builds the operator of row n-1 and runs stage 1
// there, stage 2 on row n-2, stage 3 on row n-3 and stage 4 (the update) on
// row n-4, so every intermediate lives in registers; x-neighbours come from
// the adjacent lanes.  The operator of Eq. 24 at a node is folded once per step
// into  K(T) = sum_i k_i T(x + e_i) + beta sqrt(T(x))  (i = 0..8): diffusion
// (conservative Eq. 28 with harmonic-mean links), advection (Eq. 27 on T) and
// the latent term, whose (dP/dT)_rho part A(rho) + B(rho) g(T) gives
// T (A + B g(T)) = (A - B kappa/Tc) T + B (1 + kappa)/sqrt(Tc) sqrt(T).
struct Coef9 {
    double k0, k1, k2, k3, k4, k5, k6, k7, k8, beta;
};

// Lane exchange with DPP wave shifts (a VALU move, no LDS round trip): wave_shr:1
// gives lane i the value of lane i-1 (column x-1), wave_shl:1 that of lane i+1.
// The end lanes receive 0; they are halo columns whose results are discarded.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double from_left(double v) { return dpp_move<0x138>(v); }   // value at x-1
__device__ __forceinline__ double from_right(double v) { return dpp_move<0x130>(v); }  // value at x+1
__device__ __forceinline__ float from_left(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_right(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}

// Harmonic-mean link conductance 2ab/(a+b) in two halves around a shared
// reciprocal: the divisor to invert (1 where none is needed) and the link
// from the inverted sum.  A negative value marks the T_top row, whose links
// take the conductance of the other node; a zero sum gives a zero link.  FL:
// both conductances are fluid ones, positive in any physical state.
template <bool FL, typename R>
__device__ __forceinline__ R hlink_div(R a, R b, R s) {
    if constexpr (FL) return s;
    return (a < R(0) || b < R(0) || !(s > R(0))) ? R(1) : s;
}
template <bool FL, typename R>
__device__ __forceinline__ R hlink_sel(R a, R b, R s, R inv_s) {
    const R h = R(2) * a * b * inv_s;
    if constexpr (FL) return h;
    if (a < R(0)) return b;
    if (b < R(0)) return a;
    return s > R(0) ? h : R(0);
}

struct RowIn {
    int kind;
    double T0, lam, rho, vx, vy;
};

// Thermal row n at column xg.  FL: the row is known to be a fluid row (no
// wrap, no kind tests).
template <typename VT, bool FL>
__device__ __forceinline__ RowIn load_row(cdesc &d, const double PB_GAS *Tin, const double PB_GAS *rho,
                                          const VT PB_GAS *vxg, const VT PB_GAS *vyg, int n, int xg, bool pery) {
    RowIn r{KIND_NONE, 0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (FL) {
        const uint32_t fi = (uint32_t)(n - d.nys) * (uint32_t)d.pitch + (uint32_t)xg;
        r.T0 = Tin[(uint32_t)n * (uint32_t)d.pitch + (uint32_t)xg];
        r.rho = rho[fi];
        r.lam = d.Cvchi * r.rho;
        r.vx = vxg[fi];
        r.vy = vyg[fi];
        r.kind = KIND_FLUID;
        return r;
    }
    int rr = n;
    if (pery) {
        rr %= d.nr;
        if (rr < 0) rr += d.nr;
    }
    if (rr >= 0 && rr < d.nr) {
        r.T0 = Tin[(uint32_t)rr * (uint32_t)d.pitch + (uint32_t)xg];
        if (rr < d.nys) {
            r.lam = d.lambda_S;
            r.kind = (rr == 0 && !pery) ? KIND_FIXED : KIND_SOLID;
        } else {
            const uint32_t fi = (uint32_t)(rr - d.nys) * (uint32_t)d.pitch + (uint32_t)xg;
            r.rho = rho[fi];
            r.lam = d.Cvchi * r.rho;
            r.vx = vxg[fi];
            r.vy = vyg[fi];
            r.kind = KIND_FLUID;
        }
    } else if (!pery && rr == d.nr) {
        r.T0 = d.T_top;
        r.lam = -1.0;
        r.kind = KIND_FIXED;
    }
    return r;
}

template <bool FL>
__device__ __forceinline__ double apply9(const Coef9 &c, int kind, double Sc, double SR, double SL, double Nc,
                                         double NR, double NL, double Sc_, double SR_, double SL_) {
    // rows: S* centre row, N* row above, *_ row below; order of Eq. 2.  One
    // multiply-add chain, the centre and lower rows (known a row earlier)
    // first, so the row above, computed last, enters through three of them
    double K = c.k0 * Sc;
    K = fma(c.k1, SR, K);
    K = fma(c.k3, SL, K);
    K = fma(c.k4, Sc_, K);
    K = fma(c.k7, SL_, K);
    K = fma(c.k8, SR_, K);
    K = fma(c.k2, Nc, K);
    K = fma(c.k5, NR, K);
    K = fma(c.k6, NL, K);
    if (FL || kind == KIND_FLUID) K += c.beta * fsqrt(Sc);
    return K;
}

// One strip: 64 lanes (56 written columns) by H rows, swept upwards.  The
// operator rows of the three previous rows stay in registers (the strip is
// unrolled); rows n+1 and n+2 are prefetched from HBM.  FL: every row the
// strip reads (H plus four halo rows on each side) is a fluid row, so the
// kind tests fold away; the arithmetic per node is the same as the general
// form, so a node gives the same bits in either.
template <typename VT, int H, int UNR, bool FL>
__device__ __forceinline__ void thermal_strip(cdesc &d, const PbTile &te, int k, int lane) {
    const bool pery = !FL && (d.flags & F_PERY) != 0;
    const int pin = (int)((d.par0 + k) & 1), pout = pin ^ 1;
    const int64_t t1 = d.t0 + k + 1;
    const double PB_GAS *Tin = gcast<double>(d.T[pin]);
    double PB_GAS *Tout = gcast_w<double>(d.T[pout]);
    const double PB_GAS *rhog = gcast<double>(d.rho[pout]);   // rho(t) written by this step's flow
    const VT PB_GAS *vxg = gcast<VT>(d.vx);
    const VT PB_GAS *vyg = gcast<VT>(d.vy);
    int xg = (te.x0 - 4 + lane) % d.nx;
    if (xg < 0) xg += d.nx;
    const bool out_lane = lane >= 4 && lane < 60 && (te.x0 + lane - 4) < d.nx;
    const double c1_solid = 1.0 / (d.rho_S * d.C_S);
    const double lat_a = d.kappa / d.Tc, lat_b = (1.0 + d.kappa) * d.inv_sqrtTc;
    const double W1 = 6.0 / 9.0, W2 = 6.0 / 36.0, A1 = 3.0 / 9.0, A2 = 3.0 / 36.0;

    // carried state; "_1" = row n-1, "_2" = row n-2 and so on
    int kind_1 = KIND_NONE;
    double lam_1 = 0.0, lamR_1 = 0.0, rho_1 = 0.0;
    double vx_1 = 0.0, vy_1 = 0.0, vy_2 = 0.0;
    double p_1 = 0.0, m_1 = 0.0, p_2 = 0.0, m_2 = 0.0;   // vx + vy and vx - vy
    double lN_2 = 0.0, lNEL_2 = 0.0, lNWR_2 = 0.0;       // links of row n-2 seen from row n-1
    double T0_1 = 0.0, T0_2 = 0.0, T0_3 = 0.0, T0_4 = 0.0;
    double T0L_1 = 0.0, T0R_1 = 0.0, T0L_2 = 0.0, T0R_2 = 0.0;
    double s1_2 = 0.0, s1L_2 = 0.0, s1R_2 = 0.0, s1_3 = 0.0, s1L_3 = 0.0, s1R_3 = 0.0;
    double s2_3 = 0.0, s2L_3 = 0.0, s2R_3 = 0.0, s2_4 = 0.0, s2L_4 = 0.0, s2R_4 = 0.0;
    double s3_4 = 0.0, s3L_4 = 0.0, s3R_4 = 0.0, s3_5 = 0.0, s3L_5 = 0.0, s3R_5 = 0.0;
    double acc_2 = 0.0, acc_3 = 0.0, acc_4 = 0.0;
    int kd_2 = KIND_NONE, kd_3 = KIND_NONE, kd_4 = KIND_NONE;
    Coef9 cf_2{}, cf_3{}, cf_4{};
    bool bad = false;

    const int nbeg = te.y0 - 4, nend = te.y0 + H + 3;
    RowIn nx1 = load_row<VT, FL>(d, Tin, rhog, vxg, vyg, nbeg, xg, pery);
    RowIn nx2 = load_row<VT, FL>(d, Tin, rhog, vxg, vyg, nbeg + 1, xg, pery);
#pragma unroll UNR
    for (int j = 0; j < H + 8; ++j) {
        const int n = nbeg + j;
        const RowIn cur = nx1;
        nx1 = nx2;
        if (n + 2 <= nend) nx2 = load_row<VT, FL>(d, Tin, rhog, vxg, vyg, n + 2, xg, pery);

        // new row n: neighbours across lanes
        const double lamL = from_left(cur.lam), lamR = from_right(cur.lam);
        const double T0L = from_left(cur.T0), T0R = from_right(cur.T0);
        const double p = cur.vx + cur.vy, m = cur.vx - cur.vy;

        // operator of row a = n-1
        // The row's six divisions share one reciprocal (product chain and
        // back-substitution, Montgomery's batch inversion): the four link
        // sums of the harmonic means, rho C_V, and the two Peng-Robinson
        // denominators (1 - b rho)(1 + 2 b rho - b^2 rho^2) of (dP/dT)_rho.
        // A divisor that is not used (link special case, non-fluid row) is
        // replaced by 1.
        const double sE = lam_1 + lamR_1, sN = lam_1 + cur.lam, sNE = lam_1 + lamR, sNW = lam_1 + lamL;
        const bool fluid_1 = FL || kind_1 == KIND_FLUID;
        const double br = d.b * rho_1;
        const double q1 = 1.0 - br, q2 = 1.0 + 2.0 * br - br * br;
        const double dE = hlink_div<FL>(lam_1, lamR_1, sE), dN = hlink_div<FL>(lam_1, cur.lam, sN);
        const double dNE = hlink_div<FL>(lam_1, lamR, sNE), dNW = hlink_div<FL>(lam_1, lamL, sNW);
        const double dC = fluid_1 ? rho_1 * d.Cv : 1.0, dAB = fluid_1 ? q1 * q2 : 1.0;
        const double p1 = dE * dN, p2 = p1 * dNE, p3 = p2 * dNW, p4 = p3 * dC, p5 = p4 * dAB;
        double rr = frcp(p5);
        const double iAB = rr * p4;
        rr = rr * dAB;
        const double iC = rr * p3;
        rr = rr * dC;
        const double iNW = rr * p2;
        rr = rr * dNW;
        const double iNE = rr * p1;
        rr = rr * dNE;
        const double iN = rr * dE, iE = rr * dN;
        const double lE = hlink_sel<FL>(lam_1, lamR_1, sE, iE), lN = hlink_sel<FL>(lam_1, cur.lam, sN, iN);
        const double lNE = hlink_sel<FL>(lam_1, lamR, sNE, iNE), lNW = hlink_sel<FL>(lam_1, lamL, sNW, iNW);
        const double lW = from_left(lE);
        // Eq. 27 on v (v = 0 outside the fluid): 3 sum_i w_i e_i . v(x + e_i),
        // grouped as U(x+1) - V(x-1) + (vy(above) - vy(below)) / 9
        const double U = (1.0 / 9.0) * vx_1 + (1.0 / 36.0) * (p + m_2);
        const double V = (1.0 / 9.0) * vx_1 + (1.0 / 36.0) * (m + p_2);
        const double UR = from_right(U), VL = from_left(V);
        Coef9 cf{};
        if (FL || kind_1 == KIND_FLUID || kind_1 == KIND_SOLID) {
            const double C1 = fluid_1 ? iC : c1_solid;
            const double c1 = W1 * C1 * lE, c2 = W1 * C1 * lN, c3 = W1 * C1 * lW, c4 = W1 * C1 * lN_2;
            const double c5 = W2 * C1 * lNE, c6 = W2 * C1 * lNW, c7 = W2 * C1 * lNEL_2, c8 = W2 * C1 * lNWR_2;
            cf.k0 = -(((c1 + c2) + (c3 + c4)) + ((c5 + c6) + (c7 + c8)));
            cf.k1 = c1; cf.k2 = c2; cf.k3 = c3; cf.k4 = c4;
            cf.k5 = c5; cf.k6 = c6; cf.k7 = c7; cf.k8 = c8;
            if (fluid_1) {
                const double divv = 3.0 * ((UR - VL) + (1.0 / 9.0) * (cur.vy - vy_2));
                const double A = rho_1 * d.R * q2 * iAB;                     // rho R / (1 - b rho)
                const double B = d.a * d.kappa * rho_1 * rho_1 * q1 * iAB;   // a kappa rho^2 / (1 + 2 b rho - b^2 rho^2)
                const double AL = -C1 * divv * A, BE = -C1 * divv * B;
                cf.k0 += AL - BE * lat_a;
                cf.beta = BE * lat_b;
                // advection -v.grad T with Eq. 27
                cf.k1 -= A1 * vx_1;  cf.k3 += A1 * vx_1;
                cf.k2 -= A1 * vy_1;  cf.k4 += A1 * vy_1;
                cf.k5 -= A2 * p_1;  cf.k7 += A2 * p_1;
                cf.k6 += A2 * m_1;  cf.k8 -= A2 * m_1;
            }
        }

        // stage 1 on row n-1 (input T0 rows n-2, n-1, n)
        const double K1 = apply9<FL>(cf, kind_1, T0_1, T0R_1, T0L_1, cur.T0, T0R, T0L, T0_2, T0R_2, T0L_2);
        const double s1 = T0_1 + 0.5 * K1;
        const double acc1 = K1;
        const double s1L = from_left(s1), s1R = from_right(s1);
        // stage 2 on row n-2 (input s1 rows n-3, n-2, n-1)
        const double K2 = apply9<FL>(cf_2, kd_2, s1_2, s1R_2, s1L_2, s1, s1R, s1L, s1_3, s1R_3, s1L_3);
        const double s2 = T0_2 + 0.5 * K2;
        const double acc2 = acc_2 + 2.0 * K2;
        const double s2L = from_left(s2), s2R = from_right(s2);
        // stage 3 on row n-3 (input s2 rows n-4, n-3, n-2)
        const double K3 = apply9<FL>(cf_3, kd_3, s2_3, s2R_3, s2L_3, s2, s2R, s2L, s2_4, s2R_4, s2L_4);
        const double s3 = T0_3 + K3;
        const double acc3 = acc_3 + 2.0 * K3;
        const double s3L = from_left(s3), s3R = from_right(s3);
        // stage 4 and the update on row e = n-4 (input s3 rows n-5, n-4, n-3)
        const double K4 = apply9<FL>(cf_4, kd_4, s3_4, s3R_4, s3L_4, s3, s3R, s3L, s3_5, s3R_5, s3L_5);
        const int e = n - 4;
        if (out_lane && e >= te.y0 && e < te.y0 + H && e >= 0 && e < d.nr) {
            double Tn;
            if (!FL && kd_4 == KIND_FIXED) {
                Tn = (t1 >= d.alt_t0 && t1 < d.alt_t1) ? gcast<double>(d.Tb_alt)[xg]
                                                       : gcast<double>(d.Tb)[xg];   // T_b(x, t+1)
            } else {
                Tn = T0_4 + (1.0 / 6.0) * (acc_4 + K4);
            }
            Tout[(uint32_t)e * (uint32_t)d.pitch + (uint32_t)xg] = Tn;
            bad = bad || !__builtin_isfinite(Tn);
        }

        // shift the windows by one row
        cf_4 = cf_3; cf_3 = cf_2; cf_2 = cf;
        s3_5 = s3_4; s3L_5 = s3L_4; s3R_5 = s3R_4;
        s3_4 = s3; s3L_4 = s3L; s3R_4 = s3R;
        s2_4 = s2_3; s2L_4 = s2L_3; s2R_4 = s2R_3;
        s2_3 = s2; s2L_3 = s2L; s2R_3 = s2R;
        s1_3 = s1_2; s1L_3 = s1L_2; s1R_3 = s1R_2;
        s1_2 = s1; s1L_2 = s1L; s1R_2 = s1R;
        acc_4 = acc3; acc_3 = acc2; acc_2 = acc1;
        kd_4 = kd_3; kd_3 = kd_2; kd_2 = kind_1;
        T0_4 = T0_3; T0_3 = T0_2;
        T0_2 = T0_1; T0L_2 = T0L_1; T0R_2 = T0R_1;
        T0_1 = cur.T0; T0L_1 = T0L; T0R_1 = T0R;
        lN_2 = lN; lNEL_2 = from_left(lNE); lNWR_2 = from_right(lNW);
        vy_2 = vy_1; p_2 = p_1; m_2 = m_1;
        vx_1 = cur.vx; vy_1 = cur.vy; p_1 = p; m_1 = m;
        lam_1 = cur.lam; lamR_1 = lamR; rho_1 = cur.rho; kind_1 = cur.kind;
    }
    if (bad) flag_error(d);
}

// ------------------------------------------- energy step, FP32 arithmetic
// The same sweep for FP32-deviation storage with the energy equation's
// arithmetic in FP32 (the FP32 VALU issues twice as many instructions per
// cycle as the FP64 one).  What stays FP64: T in HBM, the EOS-derivative
// coefficients A(rho), B(rho) of the latent term (from the stored FP32 rho), the
// differences T(x + e_i) - T(x) that enter stage 1, and the final update
// T(t+1) = T(t) + (h1 + 2 h2 + 2 h3 + h4) / 6, whose FP32 increment is added to
// the FP64 T.  The stages are carried as increments: with the operator
// K(T) = L T + beta sqrt(T) (L linear, L T = sum_i k_i T(x + e_i)),
//   h1 = L T + beta sqrt(T),
//   h_k = L T + c_k L h_(k-1) + beta sqrt(T + c_k h_(k-1)),  c = 1/2, 1/2, 1,
// and L T = sum_(i>0) k_i (T(x + e_i) - T(x)) + (sum_i k_i) T(x), where the
// diffusion and advection weights sum to zero and sum_i k_i is the linear part
// of the latent term.  Every rounding error is then relative to an increment
// or a local difference, never to T itself, so a steady field (the heater)
// gets no spurious source.
struct Coef9s {
    float k0, k1, k2, k3, k4, k5, k6, k7, k8, beta;
};

// A row as loaded: raw values only, so that nothing waits on the loads
// before the row is used two iterations later.  lam is set for the rows that
// need no load (heater, T_top); a fluid row's comes from rho when used.
struct RowInS {
    int kind;
    double T0;
    float rho, lam, vx, vy;   // rho as stored: converted where used, so a prefetch does not wait on it
};

// Element x of row r of a plane: a row address computed in scalar registers
// plus the lane's byte offset (xb = 4 x or 8 x, a 32-bit value fixed for the
// strip), so a row load costs no vector address arithmetic.
template <typename V>
__device__ __forceinline__ V row_elem(const V PB_GAS *base, uint32_t row, uint32_t pitch, uint32_t xb) {
    const char PB_GAS *rb = (const char PB_GAS *)(base + (size_t)(row * pitch));
    return *(const V PB_GAS *)(rb + xb);
}

template <bool FL>
__device__ __forceinline__ RowInS load_row_s(cdesc &d, const double PB_GAS *Tin, const float PB_GAS *rho,
                                             const float PB_GAS *vxg, const float PB_GAS *vyg, int n, uint32_t xb4,
                                             bool pery, float lam_s) {
    RowInS r{KIND_NONE, 0.0, 0.0f, 0.0f, 0.0f, 0.0f};
    const uint32_t pitch = (uint32_t)d.pitch, xb8 = xb4 * 2u;
    if constexpr (FL) {
        const uint32_t fr = (uint32_t)(n - d.nys);
        r.T0 = row_elem(Tin, (uint32_t)n, pitch, xb8);
        r.rho = row_elem(rho, fr, pitch, xb4);
        r.vx = row_elem(vxg, fr, pitch, xb4);
        r.vy = row_elem(vyg, fr, pitch, xb4);
        r.kind = KIND_FLUID;
        return r;
    }
    int rr = n;
    if (pery) {
        rr %= d.nr;
        if (rr < 0) rr += d.nr;
    }
    if (rr >= 0 && rr < d.nr) {
        r.T0 = row_elem(Tin, (uint32_t)rr, pitch, xb8);
        if (rr < d.nys) {
            r.lam = lam_s;
            r.kind = (rr == 0 && !pery) ? KIND_FIXED : KIND_SOLID;
        } else {
            const uint32_t fr = (uint32_t)(rr - d.nys);
            r.rho = row_elem(rho, fr, pitch, xb4);
            r.vx = row_elem(vxg, fr, pitch, xb4);
            r.vy = row_elem(vyg, fr, pitch, xb4);
            r.kind = KIND_FLUID;
        }
    } else if (!pery && rr == d.nr) {
        r.T0 = d.T_top;
        r.lam = -1.0f;
        r.kind = KIND_FIXED;
    }
    return r;
}

__device__ __forceinline__ float frcp_s(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(__builtin_fmaf(-x, r, 1.0f), r, r);
}

// L applied to nine values (centre row S*, row above N*, row below *_): one
// multiply-add chain, the centre and lower rows (known a row earlier) first,
// so the row above, computed last, enters through three multiply-adds
__device__ __forceinline__ float lin9s(const Coef9s &c, float Sc, float SR, float SL, float Nc, float NR, float NL,
                                       float Sc_, float SR_, float SL_) {
    float r = c.k0 * Sc;
    r = __builtin_fmaf(c.k1, SR, r);
    r = __builtin_fmaf(c.k3, SL, r);
    r = __builtin_fmaf(c.k4, Sc_, r);
    r = __builtin_fmaf(c.k7, SL_, r);
    r = __builtin_fmaf(c.k8, SR_, r);
    r = __builtin_fmaf(c.k2, Nc, r);
    r = __builtin_fmaf(c.k5, NR, r);
    return __builtin_fmaf(c.k6, NL, r);
}

// stage k >= 2: h_k = L T + c L h_(k-1) + beta sqrt(T + c h_(k-1)); sqrt is
// the hardware square root (about 1 ulp)
template <bool FL>
__device__ __forceinline__ float stage_s(const Coef9s &c, int kind, float LT, float ck, float Tf, float Sc, float SR,
                                         float SL, float Nc, float NR, float NL, float Sc_, float SR_, float SL_) {
    float K = LT + ck * lin9s(c, Sc, SR, SL, Nc, NR, NL, Sc_, SR_, SL_);
    if (FL || kind == KIND_FLUID) K += c.beta * __builtin_amdgcn_sqrtf(Tf + ck * Sc);
    return K;
}

template <int H, int UNR, bool FL>
__device__ __forceinline__ void thermal_strip_sp(cdesc &d, const PbTile &te, int k, int lane) {
    const bool pery = !FL && (d.flags & F_PERY) != 0;
    const int pin = (int)((d.par0 + k) & 1), pout = pin ^ 1;
    const int64_t t1 = d.t0 + k + 1;
    const double PB_GAS *Tin = gcast<double>(d.T[pin]);
    double PB_GAS *Tout = gcast_w<double>(d.T[pout]);
    const float PB_GAS *rhog = gcast<float>(d.rho[pout]);     // rho(t) written by this step's flow
    const float PB_GAS *vxg = gcast<float>(d.vx);
    const float PB_GAS *vyg = gcast<float>(d.vy);
    int xg = (te.x0 - 4 + lane) % d.nx;
    if (xg < 0) xg += d.nx;
    const bool out_lane = lane >= 4 && lane < 60 && (te.x0 + lane - 4) < d.nx;
    double PB_GAS *Tst = out_lane ? Tout : gcast_w<double>(d.sink);
    const uint32_t xb4 = (uint32_t)xg * 4u;
    const float cvchi = (float)d.Cvchi, lam_s = (float)d.lambda_S, cv = (float)d.Cv;
    const float c1_solid = (float)(1.0 / (d.rho_S * d.C_S));
    const float lat_a = (float)(d.kappa / d.Tc), lat_b = (float)((1.0 + d.kappa) * d.inv_sqrtTc);
    const float eos_b = (float)d.b, eos_R = (float)d.R, eos_ak = (float)(d.a * d.kappa);
    const float W1 = 6.0f / 9.0f, W2 = 6.0f / 36.0f, A1 = 3.0f / 9.0f, A2 = 3.0f / 36.0f;

    // carried state; "_1" = row n-1, "_2" = row n-2 and so on
    int kind_1 = KIND_NONE;
    float lam_1 = 0.0f, lamR_1 = 0.0f;
    float rho_1 = 0.0f;
    float vx_1 = 0.0f, vy_1 = 0.0f, vy_2 = 0.0f;
    float p_1 = 0.0f, m_1 = 0.0f, p_2 = 0.0f, m_2 = 0.0f;
    float lN_2 = 0.0f, lNEL_2 = 0.0f, lNWR_2 = 0.0f;
    double T0_1 = 0.0, T0_2 = 0.0, T0_3 = 0.0, T0_4 = 0.0;
    float Tf_1 = 0.0f, Tf_2 = 0.0f, Tf_3 = 0.0f, Tf_4 = 0.0f;   // the same rows rounded to FP32
    // FP64 differences rounded to FP32: T(x+1) - T(x) and T(x-1) - T(x) of a
    // row, and T(row n-1) - T(row n-2)
    float dR_1 = 0.0f, dL_1 = 0.0f, dR_2 = 0.0f, dL_2 = 0.0f, dV_1 = 0.0f;
    float LT_2 = 0.0f, LT_3 = 0.0f, LT_4 = 0.0f;              // L T(t) of the row
    float h1_2 = 0.0f, h1L_2 = 0.0f, h1R_2 = 0.0f, h1_3 = 0.0f, h1L_3 = 0.0f, h1R_3 = 0.0f;
    float h2_3 = 0.0f, h2L_3 = 0.0f, h2R_3 = 0.0f, h2_4 = 0.0f, h2L_4 = 0.0f, h2R_4 = 0.0f;
    float h3_4 = 0.0f, h3L_4 = 0.0f, h3R_4 = 0.0f, h3_5 = 0.0f, h3L_5 = 0.0f, h3R_5 = 0.0f;
    float acc_2 = 0.0f, acc_3 = 0.0f, acc_4 = 0.0f;
    int kd_2 = KIND_NONE, kd_3 = KIND_NONE, kd_4 = KIND_NONE;
    Coef9s cf_2{}, cf_3{}, cf_4{};
    bool bad = false;

    const int nbeg = te.y0 - 4, nend = te.y0 + H + 3;
    RowInS nx1 = load_row_s<FL>(d, Tin, rhog, vxg, vyg, nbeg, xb4, pery, lam_s);
    RowInS nx2 = load_row_s<FL>(d, Tin, rhog, vxg, vyg, nbeg + 1, xb4, pery, lam_s);
#pragma unroll UNR
    for (int j = 0; j < H + 8; ++j) {
        const int n = nbeg + j;
        RowInS cur = nx1;
        nx1 = nx2;
        if (n + 2 <= nend) nx2 = load_row_s<FL>(d, Tin, rhog, vxg, vyg, n + 2, xb4, pery, lam_s);
        // keep the loads of row n+2 here: the scheduler would otherwise sink
        // them next to their use to save registers and lose the prefetch
        __builtin_amdgcn_sched_barrier(0);
        if (FL || cur.kind == KIND_FLUID) cur.lam = cvchi * cur.rho;

        const float lamL = from_left(cur.lam), lamR = from_right(cur.lam);
        const float dR = (float)(from_right(cur.T0) - cur.T0), dL = (float)(from_left(cur.T0) - cur.T0);
        const float dV = (float)(cur.T0 - T0_1);
        const float p = cur.vx + cur.vy, m = cur.vx - cur.vy;

        // operator of row a = n-1: the four link sums, rho C_V and the
        // Peng-Robinson denominator (1 - b rho)(1 + 2 b rho - b^2 rho^2) share
        // one reciprocal (batch inversion)
        const float sE = lam_1 + lamR_1, sN = lam_1 + cur.lam, sNE = lam_1 + lamR, sNW = lam_1 + lamL;
        const bool fluid_1 = FL || kind_1 == KIND_FLUID;
        const float dE = hlink_div<FL>(lam_1, lamR_1, sE), dN = hlink_div<FL>(lam_1, cur.lam, sN);
        const float dNE = hlink_div<FL>(lam_1, lamR, sNE), dNW = hlink_div<FL>(lam_1, lamL, sNW);
        const float dC = fluid_1 ? rho_1 * cv : 1.0f;
        const float br = eos_b * rho_1;
        const float q1 = 1.0f - br, q2 = 1.0f + br * (2.0f - br);
        const float dQ = fluid_1 ? q1 * q2 : 1.0f;
        const float p1 = dE * dN, p2 = p1 * dNE, p3 = p2 * dNW, p4 = p3 * dC, p5 = p4 * dQ;
        float rr = frcp_s(p5);
        const float iQ = rr * p4;
        rr = rr * dQ;
        const float iC = rr * p3;
        rr = rr * dC;
        const float iNW = rr * p2;
        rr = rr * dNW;
        const float iNE = rr * p1;
        rr = rr * dNE;
        const float iN = rr * dE, iE = rr * dN;
        const float lE = hlink_sel<FL>(lam_1, lamR_1, sE, iE), lN = hlink_sel<FL>(lam_1, cur.lam, sN, iN);
        const float lNE = hlink_sel<FL>(lam_1, lamR, sNE, iNE), lNW = hlink_sel<FL>(lam_1, lamL, sNW, iNW);
        const float lW = from_left(lE);
        // Eq. 27 on v, grouped as U(x+1) - V(x-1) + (vy(above) - vy(below)) / 9
        const float U = (1.0f / 9.0f) * vx_1 + (1.0f / 36.0f) * (p + m_2);
        const float V = (1.0f / 9.0f) * vx_1 + (1.0f / 36.0f) * (m + p_2);
        const float UR = from_right(U), VL = from_left(V);
        Coef9s cf{};
        float lin = 0.0f;
        if (FL || kind_1 == KIND_FLUID || kind_1 == KIND_SOLID) {
            const float C1 = fluid_1 ? iC : c1_solid;
            const float c1 = W1 * C1 * lE, c2 = W1 * C1 * lN, c3 = W1 * C1 * lW, c4 = W1 * C1 * lN_2;
            const float c5 = W2 * C1 * lNE, c6 = W2 * C1 * lNW, c7 = W2 * C1 * lNEL_2, c8 = W2 * C1 * lNWR_2;
            cf.k0 = -(((c1 + c2) + (c3 + c4)) + ((c5 + c6) + (c7 + c8)));
            cf.k1 = c1; cf.k2 = c2; cf.k3 = c3; cf.k4 = c4;
            cf.k5 = c5; cf.k6 = c6; cf.k7 = c7; cf.k8 = c8;
            if (fluid_1) {
                const float A = eos_R * rho_1 * q2 * iQ;              // rho R / (1 - b rho)
                const float B = eos_ak * rho_1 * rho_1 * q1 * iQ;     // a kappa rho^2 / (1 + 2 b rho - b^2 rho^2)
                const float divv = 3.0f * ((UR - VL) + (1.0f / 9.0f) * (cur.vy - vy_2));
                const float AL = -C1 * divv * A, BE = -C1 * divv * B;
                lin = AL - BE * lat_a;
                cf.k0 += lin;
                cf.beta = BE * lat_b;
                // advection -v.grad T with Eq. 27
                cf.k1 -= A1 * vx_1;  cf.k3 += A1 * vx_1;
                cf.k2 -= A1 * vy_1;  cf.k4 += A1 * vy_1;
                cf.k5 -= A2 * p_1;  cf.k7 += A2 * p_1;
                cf.k6 += A2 * m_1;  cf.k8 -= A2 * m_1;
            }
        }

        // stage 1 on row n-1 from the differences to T(x) (input T rows n-2,
        // n-1, n); a diagonal difference is a row difference plus a column one
        const float dS = -dV_1;
        float LT = lin * Tf_1;
        LT = __builtin_fmaf(cf.k1, dR_1, LT);
        LT = __builtin_fmaf(cf.k3, dL_1, LT);
        LT = __builtin_fmaf(cf.k4, dS, LT);
        LT = __builtin_fmaf(cf.k7, dS + dL_2, LT);
        LT = __builtin_fmaf(cf.k8, dS + dR_2, LT);
        LT = __builtin_fmaf(cf.k2, dV, LT);
        LT = __builtin_fmaf(cf.k5, dV + dR, LT);
        LT = __builtin_fmaf(cf.k6, dV + dL, LT);
        float h1 = LT;
        if (FL || kind_1 == KIND_FLUID) h1 += cf.beta * __builtin_amdgcn_sqrtf(Tf_1);
        const float acc1 = h1;
        const float h1L = from_left(h1), h1R = from_right(h1);
        // stage 2 on row n-2 (input h1 rows n-3, n-2, n-1)
        const float h2 = stage_s<FL>(cf_2, kd_2, LT_2, 0.5f, Tf_2, h1_2, h1R_2, h1L_2, h1, h1R, h1L, h1_3,
                                     h1R_3, h1L_3);
        const float acc2 = acc_2 + 2.0f * h2;
        const float h2L = from_left(h2), h2R = from_right(h2);
        // stage 3 on row n-3 (input h2 rows n-4, n-3, n-2)
        const float h3 = stage_s<FL>(cf_3, kd_3, LT_3, 0.5f, Tf_3, h2_3, h2R_3, h2L_3, h2, h2R, h2L, h2_4,
                                     h2R_4, h2L_4);
        const float acc3 = acc_3 + 2.0f * h3;
        const float h3L = from_left(h3), h3R = from_right(h3);
        // stage 4 and the update on row e = n-4 (input h3 rows n-5, n-4, n-3)
        const float h4 = stage_s<FL>(cf_4, kd_4, LT_4, 1.0f, Tf_4, h3_4, h3R_4, h3L_4, h3, h3R, h3L, h3_5,
                                     h3R_5, h3L_5);
        const int e = n - 4;
        if constexpr (FL) {
            // every row of the strip is in the domain: the halo lanes store to
            // the sink instead of branching around the store, so the rows form
            // one straight-line block the compiler can schedule across
            if (j >= 8) {
                const double Tn = T0_4 + (double)((1.0f / 6.0f) * (acc_4 + h4));
                const uint32_t off = out_lane ? (uint32_t)e * (uint32_t)d.pitch + (uint32_t)xg : (uint32_t)lane;
                Tst[off] = Tn;
                bad = bad || (out_lane && !__builtin_isfinite(Tn));
            }
        } else if (out_lane && e >= te.y0 && e < te.y0 + H && e >= 0 && e < d.nr) {
            double Tn;
            if (kd_4 == KIND_FIXED) {
                Tn = (t1 >= d.alt_t0 && t1 < d.alt_t1) ? gcast<double>(d.Tb_alt)[xg]
                                                       : gcast<double>(d.Tb)[xg];   // T_b(x, t+1)
            } else {
                Tn = T0_4 + (double)((1.0f / 6.0f) * (acc_4 + h4));
            }
            Tout[(uint32_t)e * (uint32_t)d.pitch + (uint32_t)xg] = Tn;
            bad = bad || !__builtin_isfinite(Tn);
        }

        // shift the windows by one row
        cf_4 = cf_3; cf_3 = cf_2; cf_2 = cf;
        LT_4 = LT_3; LT_3 = LT_2; LT_2 = LT;
        h3_5 = h3_4; h3L_5 = h3L_4; h3R_5 = h3R_4;
        h3_4 = h3; h3L_4 = h3L; h3R_4 = h3R;
        h2_4 = h2_3; h2L_4 = h2L_3; h2R_4 = h2R_3;
        h2_3 = h2; h2L_3 = h2L; h2R_3 = h2R;
        h1_3 = h1_2; h1L_3 = h1L_2; h1R_3 = h1R_2;
        h1_2 = h1; h1L_2 = h1L; h1R_2 = h1R;
        acc_4 = acc3; acc_3 = acc2; acc_2 = acc1;
        kd_4 = kd_3; kd_3 = kd_2; kd_2 = kind_1;
        T0_4 = T0_3; T0_3 = T0_2; T0_2 = T0_1; T0_1 = cur.T0;
        Tf_4 = Tf_3; Tf_3 = Tf_2; Tf_2 = Tf_1; Tf_1 = (float)cur.T0;
        dR_2 = dR_1; dL_2 = dL_1; dR_1 = dR; dL_1 = dL; dV_1 = dV;
        lN_2 = lN; lNEL_2 = from_left(lNE); lNWR_2 = from_right(lNW);
        vy_2 = vy_1; p_2 = p_1; m_2 = m_1;
        vx_1 = cur.vx; vy_1 = cur.vy; p_1 = p; m_1 = m;
        lam_1 = cur.lam; lamR_1 = lamR; rho_1 = cur.rho; kind_1 = cur.kind;
    }
    if (bad) flag_error(d);
}

// One strip of H rows: the specialised path where every row it reads is a
// fluid row, else the general one.
template <typename VT, int H, int UNR>
__device__ __forceinline__ void thermal_tile(cdesc &d, const PbTile &te, int k, int lane) {
    const bool fl = !(d.flags & F_PERY) && te.y0 - 4 >= d.nys && te.y0 + H + 3 < d.nr;
    if constexpr (std::is_same<VT, float>::value) {
        if (fl) thermal_strip_sp<H, UNR, true>(d, te, k, lane);
        else thermal_strip_sp<H, UNR, false>(d, te, k, lane);
    } else {
        if (fl) thermal_strip<VT, H, UNR, true>(d, te, k, lane);
        else thermal_strip<VT, H, UNR, false>(d, te, k, lane);
    }
}

// A tile with alt set is an 8-row strip: the work-list ends with such strips
// so that the last wavefronts to start are short ones.
template <typename VT, int H, int WPE, int UNR>
__global__ __launch_bounds__(64, WPE) void k_thermal_sweep(const PbDesc *const *__restrict__ dps,
                                                            const PbTile *__restrict__ tiles, int ntiles, int k) {
    const int lane = threadIdx.x;
    for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const PbTile te = tiles[tl];
        cdesc &d = *(const PbDesc PB_CAS *)dps[te.dom];
        if (te.alt) thermal_tile<VT, 8, 16>(d, te, k, lane);
        else thermal_tile<VT, H, UNR>(d, te, k, lane);
    }
}

// --------------------------------------------------------- heat-flux sample
// One block per domain; fixed-order tree reduction so the result does not
// depend on what else runs.  With fewer than three heater rows (model A of
// Section 4.1: the Dirichlet row directly under the fluid) Eq. 36 has no
// heater rows to difference and the bottom flux is the link flux into the
// fluid.
constexpr int kFluxThreads = 1024;   // one block per domain; few columns per thread keep it short
template <typename RT>
__global__ __launch_bounds__(kFluxThreads) void k_flux(const PbDesc *const *__restrict__ dps, int k) {
    cdesc &d = *(const PbDesc PB_CAS *)dps[blockIdx.x];
    const int64_t t = d.t0 + k + 1;
    if ((d.flags & F_PERY) || d.nys < 1 || d.nyf < 1) return;
    if (t < d.fl_ta || t >= d.fl_tb || ((t - d.fl_ta) % d.fl_every) != 0) return;
    const int pout = (int)((d.par0 + k + 1) & 1);
    const double PB_GAS *T = gcast<double>(d.T[pout]);
    const RT PB_GAS *rho = gcast<RT>(d.rho[pout]);
    __shared__ double sb[kFluxThreads], st[kFluxThreads], sw[kFluxThreads];
    double ab = 0.0, at = 0.0, aw = 0.0;
    const int r = d.nys - 1;
    for (int x = threadIdx.x; x < d.nx; x += kFluxThreads) {
        if (d.nys >= 3) {
            const double T0 = T[x], T1 = T[d.pitch + x], T2 = T[2 * (size_t)d.pitch + x];
            ab += -d.lambda_S * ((4.0 * T1 - T2 - 3.0 * T0) * 0.5);       // Eq. 36
        }
        const double Tr = T[(size_t)r * d.pitch + x];
        double link = 0.0;
        const int xs[3] = {x, x + 1 < d.nx ? x + 1 : 0, x > 0 ? x - 1 : d.nx - 1};
        const double ws[3] = {1.0 / 9.0, 1.0 / 36.0, 1.0 / 36.0};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double lf = d.Cvchi * (double)rho[xs[j]];
            const double lh = 2.0 * d.lambda_S * lf / (d.lambda_S + lf);
            link += ws[j] * lh * (T[(size_t)(r + 1) * d.pitch + xs[j]] - Tr);
        }
        at += -6.0 * link;
        aw += Tr;
    }
    sb[threadIdx.x] = ab;
    st[threadIdx.x] = at;
    sw[threadIdx.x] = aw;
    __syncthreads();
    for (int s = kFluxThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sb[threadIdx.x] += sb[threadIdx.x + s];
            st[threadIdx.x] += st[threadIdx.x + s];
            sw[threadIdx.x] += sw[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double inx = 1.0 / (double)d.nx;
        const double qt = st[0] * inx, tw = sw[0] * inx;
        const double qb = d.nys >= 3 ? sb[0] * inx : qt;
        double PB_GAS *fl = gcast_w<double>(d.flux);
        fl[0] = qb;
        fl[1] = qt;
        fl[2] = tw;
        fl[3] += qb;
        fl[4] += qt;
        fl[5] += tw;
        fl[6] += 1.0;
    }
}

// ------------------------------------------------------------------ set-up
// Initial state f_i(x, 0) = w_i rho(x) (rest equilibrium).  Storage holds
// post-collision values at the source node, so slot (i, y) receives the value
// node y + e_i will pull, or, when y + e_i is a wall, the value y pulls back
// as f_opp(i); both buffers are written so frozen-flow runs see the same
// state on either parity.  rho (FP64, dense [nyf][nx] at rsrc) is stored in both
// rho buffers (as FP32 with FP32 storage, the reference of the deviations,
// which are taken against that stored value); v = 0.
template <typename FT>
__global__ __launch_bounds__(256) void k_init(const PbDesc *__restrict__ dp, const double *__restrict__ rsrc) {
    const PbDesc &d = *dp;
    const bool pery = (d.flags & F_PERY) != 0;
    const size_t plane = (size_t)d.nyf * d.pitch;
    const size_t nn = (size_t)d.nyf * d.nx;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < nn; q += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(q / d.nx), x = (int)(q % d.nx);
        const size_t idx = (size_t)y * d.pitch + x;
        const double r = rsrc[q];
        const FT rs = (FT)r;
        ((FT *)d.rho[0])[idx] = rs;
        ((FT *)d.rho[1])[idx] = rs;
        ((FT *)d.vx)[idx] = (FT)0;
        ((FT *)d.vy)[idx] = (FT)0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int xd = wrap_once(x + kEX[i], d.nx);
            int yd = y + kEY[i];
            if (pery) yd = wrap_once(yd, d.nyf);
            const double rd = (yd >= 0 && yd < d.nyf) ? rsrc[(size_t)yd * d.nx + xd] : r;
            const double fe = kW[i] * rd;
            for (int b = 0; b < 2; ++b) {
                FT *fo = (FT *)d.f[b];
                if constexpr (std::is_same<FT, float>::value)
                    fo[(size_t)i * plane + idx] = (float)(fe - kW[i] * (double)rs);
                else
                    fo[(size_t)i * plane + idx] = fe;
            }
        }
    }
}

// Advance every listed domain by nsteps: t0 += nsteps, parity flips with odd
// nsteps.  Runs on the device so captured step batches can be replayed.
__global__ void k_advance(PbDesc *const *__restrict__ dps, int ndom, int nsteps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ndom) {
        PbDesc *d = dps[i];
        d->t0 += nsteps;
        d->par0 ^= (nsteps & 1);
    }
}

}  // namespace

// ------------------------------------------------------------ launch helpers
// Flow tile variants: (BX, BY) with BX * BY threads per block.
// tiles of BX x BY nodes, one block of BX * BY threads each
static const int kFlowShapes[][2] = {{64, 4}, {64, 8}, {32, 8}, {128, 4}, {32, 16}, {64, 16}};
// column sweeps of 56 written columns x H rows
// the whole strip is unrolled so the operator ring lives in registers
static const int kThermalShapes[][2] = {{56, 28}, {56, 20}, {56, 24}, {56, 16}, {56, 12}, {56, 8}, {56, 36}};

int pb_flow_variants() { return (int)(sizeof(kFlowShapes) / sizeof(kFlowShapes[0])); }
int pb_thermal_variants() { return (int)(sizeof(kThermalShapes) / sizeof(kThermalShapes[0])); }
void pb_flow_tile_shape(int v, int *bx, int *by) {
    *bx = kFlowShapes[v][0];
    *by = kFlowShapes[v][1];
}
int pb_flow_alt_shape(int prec, int v, int *ax, int *ay) {
    *ax = kAltX;
    *ay = kAltY;
    const int bx = kFlowShapes[v][0], by = kFlowShapes[v][1];
    return prec == 1 && bx * by == 512 && bx > kAltX;
}
void pb_thermal_tile_shape(int v, int *bx, int *by) {
    *bx = kThermalShapes[v][0];
    *by = kThermalShapes[v][1];
}

template <typename FT, int BX, int BY, int MODE>
static hipError_t launch_flow_shape(bool alt, const PbDesc *const *dps, const PbTile *t, int nt, int grid, int k,
                                    hipStream_t s) {
    if constexpr (kFlowAlt<FT, BX, BY>) {
        if (alt) {
            hipLaunchKernelGGL((k_flow<FT, BX, BY, MODE, true>), dim3(grid), dim3(BX * BY), 0, s, dps, t, nt, k);
            return hipGetLastError();
        }
    } else {
        if (alt) return hipErrorInvalidValue;   // this shape has no alternate tiles
    }
    hipLaunchKernelGGL((k_flow<FT, BX, BY, MODE, false>), dim3(grid), dim3(BX * BY), 0, s, dps, t, nt, k);
    return hipGetLastError();
}

template <typename FT, int MODE>
static hipError_t launch_flow_t(int variant, const PbDesc *const *dps, const PbTile *t, int nt, int grid, int k,
                                hipStream_t s) {
    const bool alt = (variant & PB_FLOW_ALT_TILES) != 0;
    switch (variant & ~PB_FLOW_ALT_TILES) {
#define PB_FLOW_CASE(V, BX, BY) \
    case V:                    \
        return launch_flow_shape<FT, BX, BY, MODE>(alt, dps, t, nt, grid, k, s);
        PB_FLOW_CASE(0, 64, 4)
        PB_FLOW_CASE(1, 64, 8)
        PB_FLOW_CASE(2, 32, 8)
        PB_FLOW_CASE(3, 128, 4)
        PB_FLOW_CASE(4, 32, 16)
        PB_FLOW_CASE(5, 64, 16)
#undef PB_FLOW_CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t pb_launch_flow(int prec, int mode, int variant, const PbDesc *const *d_descs, const PbTile *d_tiles, int ntiles,
                          int grid, int k, hipStream_t s) {
    if (prec == 0)
        return mode == PB_MODE_READ ? launch_flow_t<double, PB_MODE_READ>(variant, d_descs, d_tiles, ntiles, grid, k, s)
                                    : launch_flow_t<double, PB_MODE_STEP>(variant, d_descs, d_tiles, ntiles, grid, k, s);
    return mode == PB_MODE_READ ? launch_flow_t<float, PB_MODE_READ>(variant, d_descs, d_tiles, ntiles, grid, k, s)
                                : launch_flow_t<float, PB_MODE_STEP>(variant, d_descs, d_tiles, ntiles, grid, k, s);
}

template <typename VT>
static hipError_t launch_thermal_t(int variant, const PbDesc *const *dps, const PbTile *d_tiles, int ntiles, int grid,
                                   int k, hipStream_t s) {
    switch (variant) {
        case 0: hipLaunchKernelGGL((k_thermal_sweep<VT, 28, 2, 36>), dim3(grid), dim3(64), 0, s, dps, d_tiles, ntiles, k); break;
        case 1: hipLaunchKernelGGL((k_thermal_sweep<VT, 20, 2, 28>), dim3(grid), dim3(64), 0, s, dps, d_tiles, ntiles, k); break;
        case 2: hipLaunchKernelGGL((k_thermal_sweep<VT, 24, 2, 32>), dim3(grid), dim3(64), 0, s, dps, d_tiles, ntiles, k); break;
        case 3: hipLaunchKernelGGL((k_thermal_sweep<VT, 16, 2, 24>), dim3(grid), dim3(64), 0, s, dps, d_tiles, ntiles, k); break;
        case 4: hipLaunchKernelGGL((k_thermal_sweep<VT, 12, 2, 20>), dim3(grid), dim3(64), 0, s, dps, d_tiles, ntiles, k); break;
        case 5: hipLaunchKernelGGL((k_thermal_sweep<VT, 8, 2, 16>), dim3(grid), dim3(64), 0, s, dps, d_tiles, ntiles, k); break;
        case 6: hipLaunchKernelGGL((k_thermal_sweep<VT, 36, 2, 44>), dim3(grid), dim3(64), 0, s, dps, d_tiles, ntiles, k); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t pb_launch_thermal(int prec, int variant, const PbDesc *const *dps, const PbTile *d_tiles, int ntiles,
                             int grid, int k, hipStream_t s) {
    return prec == 0 ? launch_thermal_t<double>(variant, dps, d_tiles, ntiles, grid, k, s)
                     : launch_thermal_t<float>(variant, dps, d_tiles, ntiles, grid, k, s);
}

hipError_t pb_launch_flux(int prec, const PbDesc *const *d_descs, int ndom, int k, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL(k_flux<double>, dim3(ndom), dim3(kFluxThreads), 0, s, d_descs, k);
    else
        hipLaunchKernelGGL(k_flux<float>, dim3(ndom), dim3(kFluxThreads), 0, s, d_descs, k);
    return hipGetLastError();
}

hipError_t pb_launch_advance(PbDesc *const *d_descs, int ndom, int nsteps, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3((ndom + 63) / 64), dim3(64), 0, s, d_descs, ndom, nsteps);
    return hipGetLastError();
}

hipError_t pb_launch_init(int prec, const PbDesc *d_desc, const double *rho_src, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL(k_init<double>, dim3(1024), dim3(256), 0, s, d_desc, rho_src);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(1024), dim3(256), 0, s, d_desc, rho_src);
    return hipGetLastError();
}

// rows x width elements from rows spitch elements apart to rows dpitch
// elements apart (device to device), so that host transfers of pitched arrays
// are single contiguous copies whatever the row length
template <typename V>
__global__ __launch_bounds__(256) void k_repitch(V *__restrict__ dst, size_t dpitch, const V *__restrict__ src,
                                                 size_t spitch, size_t width, size_t n) {
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        const size_t y = q / width, x = q - y * width;
        dst[y * dpitch + x] = src[y * spitch + x];
    }
}

hipError_t pb_launch_repitch(int elem_bytes, void *dst, size_t dpitch, const void *src, size_t spitch, size_t width,
                             size_t rows, hipStream_t s) {
    const size_t n = width * rows;
    if (n == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_repitch<double>, dim3(grid), dim3(256), 0, s, (double *)dst, dpitch, (const double *)src,
                           spitch, width, n);
    else if (elem_bytes == 4)
        hipLaunchKernelGGL(k_repitch<float>, dim3(grid), dim3(256), 0, s, (float *)dst, dpitch, (const float *)src,
                           spitch, width, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------- fixed read-back staging
// Staging for pb_read_fields_noalloc: every GPU the library runs on holds one
// copy of this array for the life of the process, so that call allocates
// nothing.  Host code never passes the array's name to a kernel (in host code
// it is a stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device.
static __device__ __align__(256) double scratch[PB_SCRATCH_BYTES / sizeof(double)];

hipError_t pb_scratch_address(void **ptr, size_t *bytes) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = PB_SCRATCH_BYTES;
    return hipSuccess;
}
