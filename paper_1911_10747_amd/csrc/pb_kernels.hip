// HIP kernels (gfx950) for one time step of the hybrid pseudopotential
// phase-change LBM with conjugate heat transfer (arXiv:1911.10747, Section 2).
//
// Two launches per step, both bandwidth-bound stencils (no MFMA):
//   k_flow     pull streaming (Eq. 8, halfway bounce-back, periodic x), the
//              macroscopic update (Eq. 10), psi from the Peng-Robinson EOS
//              (Eqs. 12-13) staged with a one-node halo in LDS, the forces
//              (Eqs. 11, 14, 15), MRT collision with the improved forcing
//              (Eqs. 3-7, 9) and the store of f*, rho(t), v(t).
//   k_thermal  the energy equation (Eq. 24) advanced by RK4 (Eqs. 25-26) with
//              the isotropic stencils (Eqs. 27-28) over fluid and heater; the
//              four stages run inside one tile held in LDS with a four-node
//              halo, so T, rho and v are read from HBM once per step.
// plus k_flux (heat flux of Eqs. 36, 38-39, FP64, fixed reduction order),
// k_init (rest equilibrium) and k_advance (time/parity bookkeeping on device).
//
// Layout: SoA populations f[i][y][x] with x fastest and a padded row pitch; a
// wavefront covers 64 consecutive x of one row, so every pull and store is a
// coalesced row segment.  All arithmetic is FP64; PB_FP32_DEV stores
// f*_i - w_i rho(x) in FP32 and rebuilds f in FP64 on load.
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

constexpr uint32_t F_PERY = 0x1u, F_FROZEN = 0x4u, F_S2PLUS = 0x8u, F_FMONLY = 0x10u;

__device__ __forceinline__ int wrap_once(int v, int n) {
    v += (v < 0) ? n : 0;
    v -= (v >= n) ? n : 0;
    return v;
}

__device__ __forceinline__ void flag_error(const PbDesc &d) { atomicOr(d.err, 1); }

// Eq. 13 and Eq. 12 (c = 1, c_s^2 = 1/3); sets bad on a negative radicand.
__device__ __forceinline__ double eos_psi(const PbDesc &d, double rho, double T, bool &bad) {
    const double st = sqrt(T) * d.inv_sqrtTc;          // sqrt(T / Tc)
    const double s = 1.0 + d.kappa * (1.0 - st);
    const double br = d.b * rho;
    const double P = rho * d.R * T / (1.0 - br) - d.a * (s * s) * rho * rho / (1.0 + 2.0 * br - br * br);
    const double rad = 2.0 * (P - rho * (1.0 / 3.0)) / d.G;
    bad = bad || !(rad >= 0.0);
    return sqrt(rad);
}

// Pull f_i(x, y, t) = f*_i(x - e_i, t-1), halfway bounce-back at the walls.
// FP32 deviation storage rebuilds f* = w_i rho_ref + delta with rho_ref the
// density of the node the value was stored at.
template <typename FT>
__device__ __forceinline__ void pull_node(const PbDesc &d, const FT *__restrict__ fin,
                                          const double *__restrict__ rin, int x, int y, bool pery,
                                          double f[9]) {
    const size_t plane = (size_t)d.nyf * d.pitch;
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
        const size_t idx = (size_t)ys * d.pitch + xs;
        const FT v = fin[(size_t)ii * plane + idx];
        if constexpr (std::is_same<FT, float>::value)
            f[i] = kW[i] * rin[idx] + (double)v;
        else
            f[i] = v;
    }
}

template <typename FT>
__device__ __forceinline__ void store_pop(FT *__restrict__ fout, size_t plane, size_t idx, int i, double fs,
                                          double rho) {
    if constexpr (std::is_same<FT, float>::value)
        fout[(size_t)i * plane + idx] = (float)(fs - kW[i] * rho);
    else
        fout[(size_t)i * plane + idx] = fs;
}

// ---------------------------------------------------------------- flow step
template <typename FT, int BX, int BY, int MODE>
__global__ __launch_bounds__(BX *BY) void k_flow(const PbDesc *const *__restrict__ dps,
                                                  const PbTile *__restrict__ tiles, int ntiles, int k) {
    constexpr int LW = BX + 2, LH = BY + 2;
    constexpr int NHALO = 2 * LW + 2 * BY;
    static_assert(NHALO <= BX * BY, "halo larger than block");
    __shared__ double s_psi[LW * LH];
    __shared__ int s_bad;

    const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
    for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const PbTile te = tiles[tl];
        const PbDesc &d = *dps[te.dom];
        const bool pery = (d.flags & F_PERY) != 0;
        const bool frozen = (d.flags & F_FROZEN) != 0;
        const int pin = (int)((d.par0 + k) & 1), pout = pin ^ 1;
        const FT *__restrict__ fin = (const FT *)d.f[pin];
        const double *__restrict__ rin = d.rho[pin];
        const double *__restrict__ Tt = d.T[pin];
        if (threadIdx.x == 0) s_bad = 0;
        bool bad = false;

        // interior node of this thread (positions past the edge wrap once so
        // that the first column/row beyond holds the periodic neighbour)
        const int xr = te.x0 + tx, yr = te.y0 + ty;
        const bool own = xr < d.nx && yr < d.nyf;
        const int xw = xr - (xr >= d.nx ? d.nx : 0);
        const int yw = pery ? yr - (yr >= d.nyf ? d.nyf : 0) : yr;
        const bool live = xw < d.nx && yw < d.nyf;
        double f[9], rho = 0.0, jx = 0.0, jy = 0.0, psi = 0.0;
        if (live) {
            pull_node<FT>(d, fin, rin, xw, yw, pery, f);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                rho += f[i];
                jx += kEX[i] * f[i];
                jy += kEY[i] * f[i];
            }
            psi = eos_psi(d, rho, Tt[(size_t)(d.nys + yw) * d.pitch + xw], bad);
        }
        s_psi[(ty + 1) * LW + tx + 1] = psi;

        // halo ring of psi
        if ((int)threadIdx.x < NHALO) {
            int h = threadIdx.x, lx, ly;
            if (h < LW) { lx = h; ly = 0; }
            else if (h < 2 * LW) { lx = h - LW; ly = LH - 1; }
            else if (h < 2 * LW + BY) { lx = 0; ly = h - 2 * LW + 1; }
            else { lx = LW - 1; ly = h - 2 * LW - BY + 1; }
            int xh = te.x0 + lx - 1, yh = te.y0 + ly - 1;
            xh = wrap_once(xh, d.nx);
            bool ok = xh >= 0 && xh < d.nx;
            if (pery) yh = wrap_once(yh, d.nyf);
            ok = ok && yh >= 0 && yh < d.nyf;
            double ph = 0.0;
            if (ok) {
                double fh[9], rh = 0.0;
                pull_node<FT>(d, fin, rin, xh, yh, pery, fh);
#pragma unroll
                for (int i = 0; i < 9; ++i) rh += fh[i];
                bool dummy = false;  // errors are flagged by the owning tile
                ph = eos_psi(d, rh, Tt[(size_t)(d.nys + yh) * d.pitch + xh], dummy);
            }
            s_psi[ly * LW + lx] = ph;
        }
        __syncthreads();

        if (own) {
            // Eq. 11 over fluid neighbours, Eq. 14 over wall neighbours
            double sfx = 0.0, sfy = 0.0, sax = 0.0, say = 0.0;
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const int yn = yr + kEY[i];
                const bool wall = !pery && (yn < 0 || yn >= d.nyf);
                if (!wall) {
                    const double pn = s_psi[(ty + 1 + kEY[i]) * LW + tx + 1 + kEX[i]];
                    sfx += kWF[i] * kEX[i] * pn;
                    sfy += kWF[i] * kEY[i] * pn;
                } else {
                    const int xn = wrap_once(xr + kEX[i], d.nx);
                    const double gam = (yn < 0) ? d.gbot[xn] : d.gtop[xn];
                    sax += kWF[i] * kEX[i] * gam;
                    say += kWF[i] * kEY[i] * gam;
                }
            }
            const double Fmx = -d.G * psi * sfx, Fmy = -d.G * psi * sfy;
            const double Fax = -psi * sax, Fay = -psi * say;
            const double Fx = Fmx + Fax;
            const double Fy = Fmy + Fay - (rho - d.rho_bar) * d.g;       // Eq. 15
            const double inv_rho = 1.0 / rho;
            double vx = (jx + 0.5 * Fx) * inv_rho;                         // Eq. 10
            double vy = (jy + 0.5 * Fy) * inv_rho;
            if (frozen) { vx = 0.0; vy = 0.0; }
            const size_t plane = (size_t)d.nyf * d.pitch;
            const size_t idx = (size_t)yr * d.pitch + xr;

            if constexpr (MODE == PB_MODE_READ) {
#pragma unroll
                for (int i = 0; i < 9; ++i) d.rd_f[(size_t)i * plane + idx] = f[i];
                d.rd_rho[idx] = rho;
                d.rd_vx[idx] = vx;
                d.rd_vy[idx] = vy;
            } else {
                // moments m = M f (Eq. 6)
                const double sa = f[1] + f[2] + f[3] + f[4];
                const double sd = f[5] + f[6] + f[7] + f[8];
                const double m1 = -4.0 * f[0] - sa + 2.0 * sd;
                const double m2 = 4.0 * f[0] - 2.0 * sa + sd;
                const double m4 = -2.0 * f[1] + 2.0 * f[3] + f[5] - f[6] - f[7] + f[8];
                const double m6 = -2.0 * f[2] + 2.0 * f[4] + f[5] + f[6] - f[7] - f[8];
                const double m7 = f[1] - f[2] + f[3] - f[4];
                const double m8 = f[5] - f[6] + f[7] - f[8];
                // equilibria (Eq. 6) with u = v of Eq. 10
                const double u2 = vx * vx + vy * vy;
                const double meq1 = rho * (-2.0 + 3.0 * u2), meq2 = rho * (1.0 - 3.0 * u2);
                const double meq4 = -rho * vx, meq6 = -rho * vy;
                const double meq7 = rho * (vx * vx - vy * vy), meq8 = rho * vx * vy;
                // forcing of Eq. 9; the varpi term times (1 - s_e/2) equals
                // 12 varpi s_e |F|^2 / psi^2 because tau_e = 1/s_e
                const double Fwx = (d.flags & F_FMONLY) ? Fmx : Fmx + Fax;
                const double Fwy = (d.flags & F_FMONLY) ? Fmy : Fmy + Fay;
                const double uF = vx * Fx + vy * Fy;
                const double cw = 12.0 * d.varpi * d.s_e * (Fwx * Fwx + Fwy * Fwy) / (psi * psi);
                const double cw2 = (d.flags & F_S2PLUS) ? cw : -cw;
                const double se = d.s_e, sq = d.s_q;
                const double snu = 1.0 / (d.tau_V + (rho - d.rho_V) * d.ktau);   // Eq. 5
                const double ms1 = m1 - se * (m1 - meq1) + (1.0 - 0.5 * se) * (6.0 * uF) + cw;
                const double ms2 = m2 - se * (m2 - meq2) + (1.0 - 0.5 * se) * (-6.0 * uF) + cw2;
                const double ms3 = jx + Fx;                       // s_j drops out (Eq. 7 + Eq. 10)
                const double ms4 = m4 - sq * (m4 - meq4) + (1.0 - 0.5 * sq) * (-Fx);
                const double ms5 = jy + Fy;
                const double ms6 = m6 - sq * (m6 - meq6) + (1.0 - 0.5 * sq) * (-Fy);
                const double ms7 = m7 - snu * (m7 - meq7) + (1.0 - 0.5 * snu) * (2.0 * (vx * Fx - vy * Fy));
                const double ms8 = m8 - snu * (m8 - meq8) + (1.0 - 0.5 * snu) * (vx * Fy + vy * Fx);
                // f* = M^{-1} m*, M^{-1} = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
                const double a0 = rho * (1.0 / 9.0), a1 = ms1 * (1.0 / 36.0), a2 = ms2 * (1.0 / 36.0);
                const double a3 = ms3 * (1.0 / 6.0), a4 = ms4 * (1.0 / 12.0), a5 = ms5 * (1.0 / 6.0);
                const double a6 = ms6 * (1.0 / 12.0), a7 = ms7 * 0.25, a8 = ms8 * 0.25;
                const double c0 = a0 - a1 - 2.0 * a2;       // axis-common part
                const double cd = a0 + 2.0 * a1 + a2;       // diagonal-common part
                FT *__restrict__ fout = (FT *)d.f[pout];
                store_pop<FT>(fout, plane, idx, 0, a0 - 4.0 * a1 + 4.0 * a2, rho);
                store_pop<FT>(fout, plane, idx, 1, c0 + a3 - 2.0 * a4 + a7, rho);
                store_pop<FT>(fout, plane, idx, 2, c0 + a5 - 2.0 * a6 - a7, rho);
                store_pop<FT>(fout, plane, idx, 3, c0 - a3 + 2.0 * a4 + a7, rho);
                store_pop<FT>(fout, plane, idx, 4, c0 - a5 + 2.0 * a6 - a7, rho);
                store_pop<FT>(fout, plane, idx, 5, cd + a3 + a4 + a5 + a6 + a8, rho);
                store_pop<FT>(fout, plane, idx, 6, cd - a3 - a4 + a5 + a6 - a8, rho);
                store_pop<FT>(fout, plane, idx, 7, cd - a3 - a4 - a5 - a6 + a8, rho);
                store_pop<FT>(fout, plane, idx, 8, cd + a3 + a4 - a5 - a6 - a8, rho);
                d.rho[pout][idx] = rho;
                d.vx[idx] = vx;
                d.vy[idx] = vy;
            }
            if (bad || !(rho == rho) || !(vx - vx == 0.0) || !(vy - vy == 0.0)) s_bad = 1;
        }
        __syncthreads();
        if (threadIdx.x == 0 && s_bad) flag_error(d);
    }
}

// ------------------------------------------------------------- energy step
// Thermal node kinds in the LDS tile.
enum : unsigned char { KIND_NONE = 0, KIND_FIXED = 1, KIND_SOLID = 2, KIND_FLUID = 3 };

template <int BX, int BY>
__global__ __launch_bounds__(256) void k_thermal(const PbDesc *const *__restrict__ dps,
                                                  const PbTile *__restrict__ tiles, int ntiles, int k) {
    constexpr int H = 4;                        // one ring per RK4 stage
    constexpr int RW = BX + 2 * H, RH = BY + 2 * H, RN = RW * RH;
    constexpr int NT = 256;
    __shared__ double sT0[RN];                  // T(t) (and fixed values)
    __shared__ double sA[RN], sB[RN];           // stage values (sB holds lambda during set-up)
    __shared__ double sLE[RN], sLN[RN], sLNE[RN], sLNW[RN];   // link conductances owned by a node
    __shared__ double sC1[RN], sAL[RN], sBE[RN], sVX[RN], sVY[RN];
    __shared__ double sAcc[BX * BY];
    __shared__ unsigned char sKind[RN];
    __shared__ int s_bad;

    for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const PbTile te = tiles[tl];
        const PbDesc &d = *dps[te.dom];
        const bool pery = (d.flags & F_PERY) != 0;
        const int pin = (int)((d.par0 + k) & 1), pout = pin ^ 1;
        const int64_t t = d.t0 + k;
        const double *__restrict__ Tin = d.T[pin];
        const double *__restrict__ rho = d.rho[pout];   // rho(t) written by this step's flow
        const double *__restrict__ vxg = d.vx;
        const double *__restrict__ vyg = d.vy;
        if (threadIdx.x == 0) s_bad = 0;

        // (1) load T(t), lambda, v over the tile plus four rings
        for (int n = threadIdx.x; n < RN; n += NT) {
            const int lx = n % RW, ly = n / RW;
            int xg = te.x0 - H + lx;
            xg %= d.nx;
            if (xg < 0) xg += d.nx;
            int rg = te.y0 - H + ly;
            unsigned char kind = KIND_NONE;
            double T0 = 0.0, lam = 0.0, vx = 0.0, vy = 0.0, c1 = 0.0, rh = 0.0;
            if (pery) {
                rg %= d.nr;
                if (rg < 0) rg += d.nr;
            }
            if (rg >= 0 && rg < d.nr) {
                T0 = Tin[(size_t)rg * d.pitch + xg];
                if (rg < d.nys) {
                    lam = d.lambda_S;
                    kind = (rg == 0 && !pery) ? KIND_FIXED : KIND_SOLID;
                    c1 = 1.0 / (d.rho_S * d.C_S);
                } else {
                    const size_t fi = (size_t)(rg - d.nys) * d.pitch + xg;
                    rh = rho[fi];
                    lam = d.Cvchi * rh;
                    vx = vxg[fi];
                    vy = vyg[fi];
                    kind = KIND_FLUID;
                    c1 = 1.0 / (rh * d.Cv);
                }
            } else if (!pery && rg == d.nr) {           // virtual row at T_top
                T0 = d.T_top;
                lam = -1.0;                              // marker: link takes the other side
                kind = KIND_FIXED;
            }
            sT0[n] = T0;
            sB[n] = lam;
            sVX[n] = vx;
            sVY[n] = vy;
            sC1[n] = c1;
            sAL[n] = rh;
            sKind[n] = kind;
        }
        __syncthreads();

        // (2) link conductances (harmonic mean, flux-continuous at the heater
        //     top) and the per-node latent-heat coefficients
        for (int n = threadIdx.x; n < RN; n += NT) {
            const int lx = n % RW, ly = n / RW;
            const double la = sB[n];
            auto link = [&](int m) -> double {
                const double lb = sB[m];
                if (la < 0.0) return lb;
                if (lb < 0.0) return la;
                const double s = la + lb;
                return s > 0.0 ? 2.0 * la * lb / s : 0.0;
            };
            sLE[n] = (lx + 1 < RW) ? link(n + 1) : 0.0;
            sLN[n] = (ly + 1 < RH) ? link(n + RW) : 0.0;
            sLNE[n] = (lx + 1 < RW && ly + 1 < RH) ? link(n + RW + 1) : 0.0;
            sLNW[n] = (lx >= 1 && ly + 1 < RH) ? link(n + RW - 1) : 0.0;
            double al = 0.0, be = 0.0;
            if (sKind[n] == KIND_FLUID && lx >= 1 && lx < RW - 1 && ly >= 1 && ly < RH - 1) {
                // Eq. 27 on v (v = 0 on solid and virtual nodes)
                const double divv =
                    3.0 * ((1.0 / 9.0) * (sVX[n + 1] - sVX[n - 1] + sVY[n + RW] - sVY[n - RW]) +
                           (1.0 / 36.0) * (sVX[n + RW + 1] - sVX[n + RW - 1] - sVX[n - RW - 1] + sVX[n - RW + 1] +
                                           sVY[n + RW + 1] + sVY[n + RW - 1] - sVY[n - RW - 1] - sVY[n - RW + 1]));
                // (dP/dT)_rho = A(rho) + B(rho) g(T), g = (1 + kappa(1 - sqrt(T/Tc))) / sqrt(T Tc)
                const double rh = sAL[n], br = d.b * rh;
                const double A = rh * d.R / (1.0 - br);
                const double B = d.a * rh * rh * d.kappa / (1.0 + 2.0 * br - br * br);
                const double c = -sC1[n] * divv;
                al = c * A;
                be = c * B;
            }
            sAL[n] = al;   // only this thread reads or writes sAL[n], sBE[n] in this pass
            sBE[n] = be;
        }
        __syncthreads();

        // (3) RK4 stages on shrinking regions: h1 on ring 3, h2 on ring 2,
        //     h3 on ring 1, h4 on the tile
#pragma unroll 1
        for (int st = 1; st <= 4; ++st) {
            const double *S = (st == 1) ? sT0 : ((st == 3) ? sB : sA);
            double *O = (st == 2) ? sB : sA;
            const int m = st;                          // stage st runs on the tile plus (4 - st) rings
            const int w = RW - 2 * m, h = RH - 2 * m;
            for (int q = threadIdx.x; q < w * h; q += NT) {
                const int lx = m + q % w, ly = m + q / w;
                const int n = ly * RW + lx;
                const unsigned char kind = sKind[n];
                const double Tc = S[n];
                double K = 0.0;
                if (kind >= KIND_SOLID) {
                    const double TE = S[n + 1], TW = S[n - 1], TN = S[n + RW], TS = S[n - RW];
                    const double TNE = S[n + RW + 1], TNW = S[n + RW - 1], TSW = S[n - RW - 1], TSE = S[n - RW + 1];
                    const double diff =
                        6.0 * ((1.0 / 9.0) * (sLE[n] * (TE - Tc) + sLN[n] * (TN - Tc) + sLE[n - 1] * (TW - Tc) +
                                              sLN[n - RW] * (TS - Tc)) +
                               (1.0 / 36.0) * (sLNE[n] * (TNE - Tc) + sLNW[n] * (TNW - Tc) +
                                               sLNE[n - RW - 1] * (TSW - Tc) + sLNW[n - RW + 1] * (TSE - Tc)));
                    K = sC1[n] * diff;
                    if (kind == KIND_FLUID) {
                        const double gx = 3.0 * ((1.0 / 9.0) * (TE - TW) + (1.0 / 36.0) * (TNE - TNW - TSW + TSE));
                        const double gy = 3.0 * ((1.0 / 9.0) * (TN - TS) + (1.0 / 36.0) * (TNE + TNW - TSW - TSE));
                        const double sq = sqrt(Tc);
                        const double gT = (1.0 + d.kappa * (1.0 - sq * d.inv_sqrtTc)) / (sq * d.sqrtTc);
                        K += -(sVX[n] * gx + sVY[n] * gy) + Tc * (sAL[n] + sBE[n] * gT);
                    }
                }
                const double T0 = sT0[n];
                const bool in_tile = lx >= H && lx < H + BX && ly >= H && ly < H + BY;
                const int ti = (ly - H) * BX + (lx - H);
                if (st == 1) {
                    O[n] = T0 + 0.5 * K;
                    if (in_tile) sAcc[ti] = K;
                } else if (st == 2) {
                    O[n] = T0 + 0.5 * K;
                    if (in_tile) sAcc[ti] += 2.0 * K;
                } else if (st == 3) {
                    O[n] = T0 + K;
                    if (in_tile) sAcc[ti] += 2.0 * K;
                } else {
                    // final update and store of the tile
                    const int xg = te.x0 + (lx - H), rg = te.y0 + (ly - H);
                    if (xg < d.nx && rg < d.nr) {
                        double Tn;
                        if (kind == KIND_FIXED) {                     // Dirichlet row: T_b(x, t+1)
                            const int64_t t1 = t + 1;
                            Tn = (t1 >= d.alt_t0 && t1 < d.alt_t1) ? d.Tb_alt[xg] : d.Tb[xg];
                        } else {
                            const double acc = sAcc[ti] + K;
                            Tn = T0 + (1.0 / 6.0) * acc;
                        }
                        d.T[pout][(size_t)rg * d.pitch + xg] = Tn;
                        if (!(Tn - Tn == 0.0)) s_bad = 1;
                    }
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0 && s_bad) flag_error(d);
        __syncthreads();
    }
}

// --------------------------------------------------------- heat-flux sample
// One block per domain; fixed-order tree reduction so the result does not
// depend on what else runs.
__global__ __launch_bounds__(256) void k_flux(const PbDesc *const *__restrict__ dps, int k) {
    const PbDesc &d = *dps[blockIdx.x];
    const int64_t t = d.t0 + k + 1;
    if ((d.flags & F_PERY) || d.nys < 3 || d.nyf < 1) return;
    if (t < d.fl_ta || t >= d.fl_tb || ((t - d.fl_ta) % d.fl_every) != 0) return;
    const int pout = (int)((d.par0 + k + 1) & 1);
    const double *T = d.T[pout];
    const double *rho = d.rho[pout];
    __shared__ double sb[256], st[256], sw[256];
    double ab = 0.0, at = 0.0, aw = 0.0;
    const int r = d.nys - 1;
    for (int x = threadIdx.x; x < d.nx; x += 256) {
        const double T0 = T[x], T1 = T[d.pitch + x], T2 = T[2 * (size_t)d.pitch + x];
        ab += -d.lambda_S * ((4.0 * T1 - T2 - 3.0 * T0) * 0.5);           // Eq. 36
        const double Tr = T[(size_t)r * d.pitch + x];
        double link = 0.0;
        const int xs[3] = {x, x + 1 < d.nx ? x + 1 : 0, x > 0 ? x - 1 : d.nx - 1};
        const double ws[3] = {1.0 / 9.0, 1.0 / 36.0, 1.0 / 36.0};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double lf = d.Cvchi * rho[xs[j]];
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
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sb[threadIdx.x] += sb[threadIdx.x + s];
            st[threadIdx.x] += st[threadIdx.x + s];
            sw[threadIdx.x] += sw[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double inx = 1.0 / (double)d.nx;
        const double qb = sb[0] * inx, qt = st[0] * inx, tw = sw[0] * inx;
        d.flux[0] = qb;
        d.flux[1] = qt;
        d.flux[2] = tw;
        d.flux[3] += qb;
        d.flux[4] += qt;
        d.flux[5] += tw;
        d.flux[6] += 1.0;
    }
}

// ------------------------------------------------------------------ set-up
// Initial state f_i(x, 0) = w_i rho(x) (rest equilibrium).  Storage holds
// post-collision values at the source node, so slot (i, y) receives the value
// node y + e_i will pull, or, when y + e_i is a wall, the value y pulls back
// as f_opp(i); both buffers are written so frozen-flow runs see the same
// state on either parity.  rho is copied to both rho buffers; v = 0.
template <typename FT>
__global__ __launch_bounds__(256) void k_init(const PbDesc *__restrict__ dp, int par) {
    const PbDesc &d = *dp;
    const bool pery = (d.flags & F_PERY) != 0;
    const size_t plane = (size_t)d.nyf * d.pitch;
    const size_t nn = (size_t)d.nyf * d.nx;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < nn; q += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(q / d.nx), x = (int)(q % d.nx);
        const size_t idx = (size_t)y * d.pitch + x;
        const double r = d.rho[par][idx];
        d.rho[par ^ 1][idx] = r;
        d.vx[idx] = 0.0;
        d.vy[idx] = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int xd = wrap_once(x + kEX[i], d.nx);
            int yd = y + kEY[i];
            if (pery) yd = wrap_once(yd, d.nyf);
            const double rd = (yd >= 0 && yd < d.nyf) ? d.rho[par][(size_t)yd * d.pitch + xd] : r;
            const double fe = kW[i] * rd;
            for (int b = 0; b < 2; ++b) {
                FT *fo = (FT *)d.f[b];
                if constexpr (std::is_same<FT, float>::value)
                    fo[(size_t)i * plane + idx] = (float)(fe - kW[i] * r);
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
static const int kFlowShapes[][2] = {{64, 4}, {64, 8}, {32, 8}, {128, 4}, {32, 16}, {64, 16}};
static const int kThermalShapes[][2] = {{32, 8}, {64, 4}, {16, 16}, {32, 16}};

int pb_flow_variants() { return (int)(sizeof(kFlowShapes) / sizeof(kFlowShapes[0])); }
int pb_thermal_variants() { return (int)(sizeof(kThermalShapes) / sizeof(kThermalShapes[0])); }
void pb_flow_tile_shape(int v, int *bx, int *by) {
    *bx = kFlowShapes[v][0];
    *by = kFlowShapes[v][1];
}
void pb_thermal_tile_shape(int v, int *bx, int *by) {
    *bx = kThermalShapes[v][0];
    *by = kThermalShapes[v][1];
}

template <typename FT, int MODE>
static hipError_t launch_flow_t(int variant, const PbDesc *const *dps, const PbTile *t, int nt, int grid, int k,
                                hipStream_t s) {
    switch (variant) {
#define PB_FLOW_CASE(V, BX, BY)                                                                       \
    case V:                                                                                          \
        hipLaunchKernelGGL((k_flow<FT, BX, BY, MODE>), dim3(grid), dim3(BX * BY), 0, s, dps, t, nt, k); \
        break;
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
    return hipGetLastError();
}

hipError_t pb_launch_flow(int prec, int mode, int variant, const PbDesc *const *d_descs, const PbTile *d_tiles, int ntiles,
                          int grid, int k, hipStream_t s) {
    if (prec == 0)
        return mode == PB_MODE_READ ? launch_flow_t<double, PB_MODE_READ>(variant, d_descs, d_tiles, ntiles, grid, k, s)
                                    : launch_flow_t<double, PB_MODE_STEP>(variant, d_descs, d_tiles, ntiles, grid, k, s);
    return mode == PB_MODE_READ ? launch_flow_t<float, PB_MODE_READ>(variant, d_descs, d_tiles, ntiles, grid, k, s)
                                : launch_flow_t<float, PB_MODE_STEP>(variant, d_descs, d_tiles, ntiles, grid, k, s);
}

hipError_t pb_launch_thermal(int variant, const PbDesc *const *dps, const PbTile *d_tiles, int ntiles, int grid, int k,
                             hipStream_t s) {
    switch (variant) {
        case 0: hipLaunchKernelGGL((k_thermal<32, 8>), dim3(grid), dim3(256), 0, s, dps, d_tiles, ntiles, k); break;
        case 1: hipLaunchKernelGGL((k_thermal<64, 4>), dim3(grid), dim3(256), 0, s, dps, d_tiles, ntiles, k); break;
        case 2: hipLaunchKernelGGL((k_thermal<16, 16>), dim3(grid), dim3(256), 0, s, dps, d_tiles, ntiles, k); break;
        case 3: hipLaunchKernelGGL((k_thermal<32, 16>), dim3(grid), dim3(256), 0, s, dps, d_tiles, ntiles, k); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t pb_launch_flux(const PbDesc *const *d_descs, int ndom, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_flux, dim3(ndom), dim3(256), 0, s, d_descs, k);
    return hipGetLastError();
}

hipError_t pb_launch_advance(PbDesc *const *d_descs, int ndom, int nsteps, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3((ndom + 63) / 64), dim3(64), 0, s, d_descs, ndom, nsteps);
    return hipGetLastError();
}

hipError_t pb_launch_init(int prec, const PbDesc *d_desc, int par, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL(k_init<double>, dim3(1024), dim3(256), 0, s, d_desc, par);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(1024), dim3(256), 0, s, d_desc, par);
    return hipGetLastError();
}
