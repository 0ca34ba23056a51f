/*
 * ORACLE -- test infrastructure only.
 *
 * Plain, serial, FP64 CPU reference of one time step of the hybrid
 * pseudopotential phase-change lattice Boltzmann method with conjugate heat
 * transfer (Zhao, Liang, Sun, Cai, Li, arXiv:1911.10747, Section 2).  It is
 * written from the paper's equations in the paper's order, with plain nested
 * loops and no blocking, fusion or reordering.  Only tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header or constant table with the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 *
 * Readings of the paper that this code takes (each is a switch or a parameter
 * where a choice exists):
 *   - interaction strength G = -1 (Eq. 12 needs G < 0 for a real psi);
 *   - the switch s of Eq. 14 is 1 on wall nodes and 0 on fluid nodes: the
 *     Shan-Chen sum of Eq. 11 runs over fluid neighbours and the adhesion sum
 *     of Eq. 14 over wall neighbours, each wall node carrying its own
 *     gamma = G_w * psi(rho_w);
 *   - row 8 of the forcing vector of Eq. 9 is u_x F_y + u_y F_x (the
 *     projection of the standard forcing term; the printed minus sign does not
 *     follow from Eq. 6);
 *   - the ||F_m||^2 term enters row 2 of Eq. 9 with a minus sign unless
 *     sbar2_plus is set;
 *   - the force in that term is the whole pseudopotential interaction
 *     F_m + F_ads (so a liquid at rest beside a neutral wall stays at rest);
 *     varpi_fm_only selects the fluid-fluid part of Eq. 11 alone;
 *   - rho_v of Eq. 15 is the mean fluid density, fixed when the fields are set
 *     (mass is conserved exactly);
 *   - the derivative written (dP/dt) in Eqs. 21-24 is (dP_EOS/dT) at fixed rho;
 *   - the weights of Eqs. 27-28 are the D2Q9 lattice weights 4/9, 1/9, 1/36;
 *   - div(lambda grad T) is the conservative sum 6 * sum_i w_i lambda_h,i
 *     (T_i - T) with a harmonic-mean link conductance (flux continuous at the
 *     fluid/heater interface; equals lambda times Eq. 28 for uniform lambda);
 *   - within a step: psi and the forces use T(t); the RK4 of Eqs. 25-26 uses
 *     rho(t), v(t) frozen and evaluates T-dependent terms at the stage value;
 *   - periodic direction is x; halfway bounce-back walls sit below the first
 *     and above the last fluid row; thermal row 0 (heater bottom) is
 *     Dirichlet T_b(x,t); a virtual row above the fluid holds T_top.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Flat parameter block.  The same field order is mirrored by the ctypes
 * structure in oracle/orc.py. */
typedef struct {
    int32_t nx, nyf, nys;
    int32_t periodic_y, isothermal, frozen_flow, sbar2_plus, varpi_fm_only;
    double a, b, R, omega, Tc, G;          /* Eq. 13 and Eq. 11-12            */
    double s_e, s_q, varpi;                /* Eq. 3 (s1=s2=s_e, s4=s6=s_q), Eq. 9 */
    double tau_L, tau_V, rho_L, rho_V;     /* Eq. 5                            */
    double g;                              /* Eq. 15, gravity (0,-g)           */
    double Cv, Cvchi, rho_S, C_S, lambda_S;/* Section 2.2, Section 3.1          */
} orc_params;

/* D2Q9 velocities in the order of Eq. 2. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* Transform matrix of Eq. 6, row by row as printed. */
static const double MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

static double lattice_w(int i) { return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }
/* Weights w(|e|^2) of the interaction force, Eq. 11: w(1)=1/3, w(2)=1/12. */
static double force_w(int i) { return i == 0 ? 0.0 : (i < 5 ? 1.0 / 3.0 : 1.0 / 12.0); }

typedef struct {
    orc_params p;
    int nx, nyf, nys, nr;          /* nr = thermal rows = nys + nyf          */
    int64_t t;                     /* current time step                      */
    double *f;                     /* f(t), post streaming: [9][nyf][nx]      */
    double *fs;                    /* scratch for f* : [9][nyf][nx]           */
    double *T;                     /* T(t): [nr][nx]                          */
    double *rho, *jx, *jy, *psi, *Fx, *Fy, *Fmx, *Fmy, *Fax, *Fay, *ux, *uy; /* [nyf][nx] */
    double *Tb, *Tb_alt, *gbot, *gtop;                            /* [nx]      */
    int64_t alt_t0, alt_t1;
    double T_top;
    double rho_bar;
    int err;
    /* heat-flux window */
    int64_t fl_ta, fl_tb; int fl_every;
    double q_bot_inst, q_top_inst, Tw_inst;
    double q_bot_sum, q_top_sum, Tw_sum; int64_t n_samples;
    /* RK4 work arrays [nr][nx] */
    double *Ts, *K, *acc;
} orc_dom;

static double *zalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

/* ---------------- Thermodynamics (Eq. 13 and its T-derivative) ---------- */
static double pr_kappa(const orc_params *p) {
    return 0.37464 + 1.54226 * p->omega - 0.26992 * p->omega * p->omega;
}
double orc_pressure(const orc_params *p, double rho, double T) {
    double k = pr_kappa(p);
    double s = 1.0 + k * (1.0 - sqrt(T / p->Tc));
    double phi = s * s;
    return rho * p->R * T / (1.0 - p->b * rho)
         - p->a * phi * rho * rho / (1.0 + 2.0 * p->b * rho - p->b * p->b * rho * rho);
}
/* (dP_EOS/dT) at constant rho, differentiated by hand from Eq. 13. */
double orc_dpdt(const orc_params *p, double rho, double T) {
    double k = pr_kappa(p);
    double s = 1.0 + k * (1.0 - sqrt(T / p->Tc));
    double dphi_dT = 2.0 * s * (-k / (2.0 * sqrt(T * p->Tc)));
    return rho * p->R / (1.0 - p->b * rho)
         - p->a * dphi_dT * rho * rho / (1.0 + 2.0 * p->b * rho - p->b * p->b * rho * rho);
}
/* Eq. 12 with c = 1 and c_s^2 = 1/3; returns the radicand through *rad. */
double orc_psi(const orc_params *p, double rho, double T, double *rad) {
    double cs2 = 1.0 / 3.0, c = 1.0;
    double r = 2.0 * (orc_pressure(p, rho, T) - rho * cs2) / (p->G * c * c);
    if (rad) *rad = r;
    return sqrt(r);
}

/* ---------------- MRT collision of one node (Eqs. 3, 5, 6, 7, 9) ------- */
/* f in, f* out.  F is the total force, Fm the pseudopotential part, psi the
 * node's pseudopotential; (ux, uy) the velocity of Eq. 10. */
void orc_collide_node(const orc_params *p, const double *f, double rho, double ux, double uy,
                      double Fx, double Fy, double Fmx, double Fmy, double psi, double *fout) {
    double m[9], meq[9], S[9], s[9], ms[9];
    for (int k = 0; k < 9; ++k) {
        m[k] = 0.0;
        for (int i = 0; i < 9; ++i) m[k] += MM[k][i] * f[i];
    }
    double u2 = ux * ux + uy * uy;
    meq[0] = rho;
    meq[1] = rho * (-2.0 + 3.0 * u2);
    meq[2] = rho * (1.0 - 3.0 * u2);
    meq[3] = rho * ux;
    meq[4] = -rho * ux;
    meq[5] = rho * uy;
    meq[6] = -rho * uy;
    meq[7] = rho * (ux * ux - uy * uy);
    meq[8] = rho * ux * uy;

    /* Eq. 5: density-interpolated viscous relaxation time. */
    double tau_v = p->tau_V + (rho - p->rho_V) / (p->rho_L - p->rho_V) * (p->tau_L - p->tau_V);
    double tau_e = 1.0 / p->s_e, tau_z = 1.0 / p->s_e; /* s1 = s2 */
    s[0] = 1.0; s[1] = p->s_e; s[2] = p->s_e;
    s[3] = 1.0; s[4] = p->s_q; s[5] = 1.0; s[6] = p->s_q;
    s[7] = 1.0 / tau_v; s[8] = 1.0 / tau_v;

    double uF = ux * Fx + uy * Fy;
    double Fm2 = Fmx * Fmx + Fmy * Fmy;
    double dt = 1.0;
    double sgn2 = p->sbar2_plus ? 1.0 : -1.0;
    S[0] = 0.0;
    S[1] = 6.0 * uF + 12.0 * p->varpi * Fm2 / (psi * psi * dt * (tau_e - 0.5));
    S[2] = -6.0 * uF + sgn2 * 12.0 * p->varpi * Fm2 / (psi * psi * dt * (tau_z - 0.5));
    S[3] = Fx;
    S[4] = -Fx;
    S[5] = Fy;
    S[6] = -Fy;
    S[7] = 2.0 * (ux * Fx - uy * Fy);
    S[8] = ux * Fy + uy * Fx;

    for (int k = 0; k < 9; ++k)
        ms[k] = m[k] - s[k] * (m[k] - meq[k]) + dt * (1.0 - 0.5 * s[k]) * S[k];

    /* f* = M^{-1} m*; M is orthogonal so M^{-1} = M^T diag(1/|row k|^2). */
    for (int i = 0; i < 9; ++i) {
        double acc = 0.0;
        for (int k = 0; k < 9; ++k) {
            double nk = 0.0;
            for (int j = 0; j < 9; ++j) nk += MM[k][j] * MM[k][j];
            acc += MM[k][i] * ms[k] / nk;
        }
        fout[i] = acc;
    }
}

void orc_moment_matrix(double *out81) {
    for (int k = 0; k < 9; ++k)
        for (int i = 0; i < 9; ++i) out81[k * 9 + i] = MM[k][i];
}

/* ---------------- Domain lifecycle -------------------------------------- */
orc_dom *orc_create(const orc_params *p) {
    orc_dom *d = (orc_dom *)calloc(1, sizeof(orc_dom));
    d->p = *p;
    d->nx = p->nx; d->nyf = p->nyf; d->nys = p->nys; d->nr = p->nys + p->nyf;
    size_t nf = (size_t)p->nx * p->nyf, nt = (size_t)p->nx * d->nr;
    d->f = zalloc(9 * nf); d->fs = zalloc(9 * nf);
    d->T = zalloc(nt); d->Ts = zalloc(nt); d->K = zalloc(nt); d->acc = zalloc(nt);
    d->rho = zalloc(nf); d->jx = zalloc(nf); d->jy = zalloc(nf); d->psi = zalloc(nf);
    d->Fx = zalloc(nf); d->Fy = zalloc(nf); d->Fmx = zalloc(nf); d->Fmy = zalloc(nf); d->Fax = zalloc(nf); d->Fay = zalloc(nf);
    d->ux = zalloc(nf); d->uy = zalloc(nf);
    d->Tb = zalloc(p->nx); d->Tb_alt = zalloc(p->nx);
    d->gbot = zalloc(p->nx); d->gtop = zalloc(p->nx);
    d->alt_t0 = d->alt_t1 = 0;
    d->fl_ta = 0; d->fl_tb = 0; d->fl_every = 1;
    return d;
}

void orc_destroy(orc_dom *d) {
    if (!d) return;
    double *ptrs[] = {d->f, d->fs, d->T, d->Ts, d->K, d->acc, d->rho, d->jx, d->jy, d->psi,
                      d->Fx, d->Fy, d->Fmx, d->Fmy, d->Fax, d->Fay, d->ux, d->uy, d->Tb, d->Tb_alt, d->gbot, d->gtop};
    for (size_t k = 0; k < sizeof(ptrs) / sizeof(ptrs[0]); ++k) free(ptrs[k]);
    free(d);
}

#define FI(d, i, y, x) ((size_t)(i) * (d)->nyf * (d)->nx + (size_t)(y) * (d)->nx + (size_t)(x))
#define NI(d, y, x) ((size_t)(y) * (d)->nx + (size_t)(x))

static double bottom_T(const orc_dom *d, int x, int64_t t) {
    if (t >= d->alt_t0 && t < d->alt_t1) return d->Tb_alt[x];
    return d->Tb[x];
}

void orc_set_bc(orc_dom *d, double T_top, const double *Tb, const double *Tb_alt, int64_t t0,
                int64_t t1, const double *gbot, const double *gtop) {
    d->T_top = T_top;
    for (int x = 0; x < d->nx; ++x) {
        d->Tb[x] = Tb ? Tb[x] : T_top;
        d->Tb_alt[x] = Tb_alt ? Tb_alt[x] : d->Tb[x];
        d->gbot[x] = gbot ? gbot[x] : 0.0;
        d->gtop[x] = gtop ? gtop[x] : 0.0;
    }
    d->alt_t0 = Tb_alt ? t0 : 0;
    d->alt_t1 = Tb_alt ? t1 : 0;
}

static void apply_dirichlet(orc_dom *d, double *T, int64_t t) {
    if (d->p.periodic_y || d->nys < 1) return;
    for (int x = 0; x < d->nx; ++x) T[NI(d, 0, x)] = bottom_T(d, x, t);
}

/* Initial state: f = f^eq(rho, 0) = w_i rho, T given; rho_bar = mean fluid rho. */
void orc_set_fields(orc_dom *d, const double *rho, const double *T) {
    double sum = 0.0;
    for (int y = 0; y < d->nyf; ++y)
        for (int x = 0; x < d->nx; ++x) {
            double r = rho[NI(d, y, x)];
            sum += r;
            for (int i = 0; i < 9; ++i) d->f[FI(d, i, y, x)] = lattice_w(i) * r;
        }
    d->rho_bar = sum / ((double)d->nx * d->nyf);
    memcpy(d->T, T, sizeof(double) * (size_t)d->nx * d->nr);
    d->t = 0;
    apply_dirichlet(d, d->T, d->t);
    d->err = 0;
}

/* Full state (checkpoint): f(t) post streaming, T(t), time t. rho_bar given. */
void orc_set_state(orc_dom *d, const double *f, const double *T, int64_t t, double rho_bar) {
    memcpy(d->f, f, sizeof(double) * 9 * (size_t)d->nx * d->nyf);
    memcpy(d->T, T, sizeof(double) * (size_t)d->nx * d->nr);
    d->t = t;
    d->rho_bar = rho_bar;
    d->err = 0;
}

double orc_rho_bar(const orc_dom *d) { return d->rho_bar; }
int64_t orc_time(const orc_dom *d) { return d->t; }
int orc_error(const orc_dom *d) { return d->err; }

/* ---------------- Step pieces ------------------------------------------- */
/* Eq. 10: density and bare momentum from f. */
static void macroscopic(orc_dom *d) {
    for (int y = 0; y < d->nyf; ++y)
        for (int x = 0; x < d->nx; ++x) {
            double r = 0, jx = 0, jy = 0;
            for (int i = 0; i < 9; ++i) {
                double fi = d->f[FI(d, i, y, x)];
                r += fi; jx += EX[i] * fi; jy += EY[i] * fi;
            }
            d->rho[NI(d, y, x)] = r; d->jx[NI(d, y, x)] = jx; d->jy[NI(d, y, x)] = jy;
        }
}

/* Eqs. 12-13 at T(t). */
static void pseudopotential(orc_dom *d) {
    for (int y = 0; y < d->nyf; ++y)
        for (int x = 0; x < d->nx; ++x) {
            double rad;
            double T = d->T[NI(d, d->nys + y, x)];
            double ps = orc_psi(&d->p, d->rho[NI(d, y, x)], T, &rad);
            if (!(rad >= 0.0) || !isfinite(ps)) d->err = 1;
            d->psi[NI(d, y, x)] = ps;
        }
}

/* Eq. 11 (fluid neighbours), Eq. 14 (wall neighbours), Eq. 15, and v of Eq. 10. */
static void forces_and_velocity(orc_dom *d) {
    const orc_params *p = &d->p;
    for (int y = 0; y < d->nyf; ++y)
        for (int x = 0; x < d->nx; ++x) {
            double sfx = 0, sfy = 0, sax = 0, say = 0;
            for (int i = 1; i < 9; ++i) {
                int xn = (x + EX[i] + d->nx) % d->nx;
                int yn = y + EY[i];
                if (p->periodic_y) yn = (yn + d->nyf) % d->nyf;
                if (yn >= 0 && yn < d->nyf) {
                    double pn = d->psi[NI(d, yn, xn)];
                    sfx += force_w(i) * pn * EX[i];
                    sfy += force_w(i) * pn * EY[i];
                } else {
                    double gam = (yn < 0) ? d->gbot[xn] : d->gtop[xn];
                    sax += force_w(i) * gam * EX[i];
                    say += force_w(i) * gam * EY[i];
                }
            }
            size_t n = NI(d, y, x);
            double ps = d->psi[n];
            double Fmx = -p->G * ps * sfx, Fmy = -p->G * ps * sfy;
            double Fax = -ps * sax, Fay = -ps * say;
            double Fgx = 0.0, Fgy = (d->rho[n] - d->rho_bar) * (-p->g);
            d->Fmx[n] = Fmx; d->Fmy[n] = Fmy;
            d->Fax[n] = Fax; d->Fay[n] = Fay;
            d->Fx[n] = Fmx + Fax + Fgx;
            d->Fy[n] = Fmy + Fay + Fgy;
            double dt = 1.0;
            d->ux[n] = (d->jx[n] + dt * d->Fx[n] / 2.0) / d->rho[n];
            d->uy[n] = (d->jy[n] + dt * d->Fy[n] / 2.0) / d->rho[n];
        }
}

/* ---------------- Energy equation (Eqs. 24-28) -------------------------- */
/* Conductivity of a thermal node: lambda_S in the heater, Cv*chi*rho in the fluid. */
static double node_lambda(const orc_dom *d, const double *rho, int r, int x) {
    if (r < d->nys) return d->p.lambda_S;
    return d->p.Cvchi * rho[NI(d, r - d->nys, x)];
}

/* K(T) of Eq. 24 for every non-Dirichlet thermal node, with rho, v frozen.
 * rho, vx, vy are [nyf][nx] fluid fields.  Rows without a fluid node carry
 * v = 0.  Exposed so tests can evaluate the right-hand side on its own. */
void orc_thermal_rhs(const orc_dom *d, const double *Tst, const double *rho, const double *vx,
                     const double *vy, double *K) {
    const orc_params *p = &d->p;
    const double cs2 = 1.0 / 3.0, dt = 1.0;
    int r0 = (p->periodic_y || d->nys < 1) ? 0 : 1;
    for (int r = 0; r < d->nr; ++r)
        for (int x = 0; x < d->nx; ++x) K[NI(d, r, x)] = 0.0;
    for (int r = r0; r < d->nr; ++r)
        for (int x = 0; x < d->nx; ++x) {
            double Tc0 = Tst[NI(d, r, x)];
            double lam0 = node_lambda(d, rho, r, x);
            double diff = 0.0, gx = 0.0, gy = 0.0, divv = 0.0;
            for (int i = 1; i < 9; ++i) {
                int xn = (x + EX[i] + d->nx) % d->nx;
                int rn = r + EY[i];
                double Tn, lamh, vxn = 0.0, vyn = 0.0;
                if (p->periodic_y) rn = (rn + d->nr) % d->nr;
                if (rn == d->nr) { /* virtual row above the fluid: T_top, v = 0 */
                    Tn = d->T_top;
                    lamh = lam0;
                } else {
                    Tn = Tst[NI(d, rn, xn)];   /* row 0 already holds T_b(t) */
                    double lamn = node_lambda(d, rho, rn, xn);
                    lamh = 2.0 * lam0 * lamn / (lam0 + lamn);
                    if (rn >= d->nys) { vxn = vx[NI(d, rn - d->nys, xn)]; vyn = vy[NI(d, rn - d->nys, xn)]; }
                }
                double w = lattice_w(i);
                diff += w * lamh * (Tn - Tc0);                 /* conservative Eq. 28 */
                gx += w * Tn * EX[i]; gy += w * Tn * EY[i];    /* Eq. 27 on T         */
                divv += w * (vxn * EX[i] + vyn * EY[i]);       /* Eq. 27 on v         */
            }
            diff *= 2.0 / (cs2 * dt * dt);
            gx /= cs2 * dt; gy /= cs2 * dt; divv /= cs2 * dt;
            double k;
            if (r < d->nys) {
                k = diff / (p->rho_S * p->C_S);
            } else {
                size_t n = NI(d, r - d->nys, x);
                double rh = rho[n];
                k = -(vx[n] * gx + vy[n] * gy) + diff / (rh * p->Cv)
                    - Tc0 / (rh * p->Cv) * orc_dpdt(p, rh, Tc0) * divv;
            }
            K[NI(d, r, x)] = k;
        }
}

/* Eqs. 25-26: classical RK4 with Dirichlet rows held at T_b(t) in every stage
 * and set to T_b(t+1) at the end. */
static void thermal_rk4(orc_dom *d, const double *vx, const double *vy) {
    size_t nt = (size_t)d->nx * d->nr;
    const double dt = 1.0;
    int64_t t = d->t;
    orc_thermal_rhs(d, d->T, d->rho, vx, vy, d->K);                  /* h1 */
    for (size_t n = 0; n < nt; ++n) { d->acc[n] = d->K[n]; d->Ts[n] = d->T[n] + dt / 2.0 * d->K[n]; }
    apply_dirichlet(d, d->Ts, t);
    orc_thermal_rhs(d, d->Ts, d->rho, vx, vy, d->K);                 /* h2 */
    for (size_t n = 0; n < nt; ++n) { d->acc[n] += 2.0 * d->K[n]; d->Ts[n] = d->T[n] + dt / 2.0 * d->K[n]; }
    apply_dirichlet(d, d->Ts, t);
    orc_thermal_rhs(d, d->Ts, d->rho, vx, vy, d->K);                 /* h3 */
    for (size_t n = 0; n < nt; ++n) { d->acc[n] += 2.0 * d->K[n]; d->Ts[n] = d->T[n] + dt * d->K[n]; }
    apply_dirichlet(d, d->Ts, t);
    orc_thermal_rhs(d, d->Ts, d->rho, vx, vy, d->K);                 /* h4 */
    for (size_t n = 0; n < nt; ++n) {
        d->acc[n] += d->K[n];
        d->T[n] = d->T[n] + dt / 6.0 * d->acc[n];
    }
    apply_dirichlet(d, d->T, t + 1);
}

/* Eq. 7 at every fluid node, then Eq. 8 by pulling with halfway bounce-back. */
static void collide_and_stream(orc_dom *d) {
    double fin[9], fout[9];
    for (int y = 0; y < d->nyf; ++y)
        for (int x = 0; x < d->nx; ++x) {
            size_t n = NI(d, y, x);
            for (int i = 0; i < 9; ++i) fin[i] = d->f[FI(d, i, y, x)];
            /* force entering the varpi term of Eq. 9 */
            double fwx = d->Fmx[n], fwy = d->Fmy[n];
            if (!d->p.varpi_fm_only) { fwx += d->Fax[n]; fwy += d->Fay[n]; }
            orc_collide_node(&d->p, fin, d->rho[n], d->ux[n], d->uy[n], d->Fx[n], d->Fy[n],
                             fwx, fwy, d->psi[n], fout);
            for (int i = 0; i < 9; ++i) d->fs[FI(d, i, y, x)] = fout[i];
        }
    for (int y = 0; y < d->nyf; ++y)
        for (int x = 0; x < d->nx; ++x)
            for (int i = 0; i < 9; ++i) {
                int xs = (x - EX[i] + d->nx) % d->nx;
                int ys = y - EY[i];
                if (d->p.periodic_y) ys = (ys + d->nyf) % d->nyf;
                if (ys >= 0 && ys < d->nyf) d->f[FI(d, i, y, x)] = d->fs[FI(d, i, ys, xs)];
                else d->f[FI(d, i, y, x)] = d->fs[FI(d, OPP[i], y, x)];
            }
}

/* Eq. 36 at the heater bottom (Eq. 39), link flux and mean T at the heater top.
 * With fewer than three heater rows (model A of Section 4.1 has none: the
 * Dirichlet row sits directly under the fluid) Eq. 36 has no heater rows to
 * difference, and the bottom flux is the link flux into the fluid. */
static void sample_flux(orc_dom *d) {
    const orc_params *p = &d->p;
    double sb = 0.0, st = 0.0, sw = 0.0;
    if (d->nys >= 3) {
        for (int x = 0; x < d->nx; ++x) {
            double dTdy = (4.0 * d->T[NI(d, 1, x)] - d->T[NI(d, 2, x)] - 3.0 * d->T[NI(d, 0, x)]) / 2.0;
            sb += -p->lambda_S * dTdy;
        }
    }
    int r = d->nys - 1;
    for (int x = 0; x < d->nx; ++x) {
        double lam0 = node_lambda(d, d->rho, r, x), link = 0.0;
        for (int i = 1; i < 9; ++i) {
            if (EY[i] != 1) continue;
            int xn = (x + EX[i] + d->nx) % d->nx, rn = r + 1;
            double Tn, lamh;
            if (rn == d->nr) { Tn = d->T_top; lamh = lam0; }
            else {
                double lamn = node_lambda(d, d->rho, rn, xn);
                Tn = d->T[NI(d, rn, xn)];
                lamh = 2.0 * lam0 * lamn / (lam0 + lamn);
            }
            link += lattice_w(i) * lamh * (Tn - d->T[NI(d, r, x)]);
        }
        st += -6.0 * link;
        sw += d->T[NI(d, r, x)];
    }
    d->q_top_inst = st / d->nx;
    d->q_bot_inst = d->nys >= 3 ? sb / d->nx : d->q_top_inst;
    d->Tw_inst = sw / d->nx;
    d->q_bot_sum += d->q_bot_inst; d->q_top_sum += d->q_top_inst; d->Tw_sum += d->Tw_inst;
    d->n_samples += 1;
}

void orc_flux_window(orc_dom *d, int64_t ta, int64_t tb, int every) {
    d->fl_ta = ta; d->fl_tb = tb; d->fl_every = every > 0 ? every : 1;
    d->q_bot_sum = d->q_top_sum = d->Tw_sum = 0.0; d->n_samples = 0;
    d->q_bot_inst = d->q_top_inst = d->Tw_inst = 0.0;
}

/* out: q_bottom_inst, q_top_inst, T_w_inst, q_bottom_mean, q_top_mean, T_w_mean, n_samples */
void orc_heat_flux(const orc_dom *d, double *out) {
    double n = (double)d->n_samples;
    out[0] = d->q_bot_inst; out[1] = d->q_top_inst; out[2] = d->Tw_inst;
    out[3] = n > 0 ? d->q_bot_sum / n : 0.0;
    out[4] = n > 0 ? d->q_top_sum / n : 0.0;
    out[5] = n > 0 ? d->Tw_sum / n : 0.0;
    out[6] = n;
}

/* One time step t -> t+1 in the order: Eq. 10, Eqs. 12-13, Eqs. 11/14/15,
 * Eqs. 24-28 (RK4), Eq. 7, Eq. 8, then the optional heat-flux sample. */
static void one_step(orc_dom *d) {
    const orc_params *p = &d->p;
    macroscopic(d);
    if (p->frozen_flow) {
        size_t nf = (size_t)d->nx * d->nyf;
        for (size_t n = 0; n < nf; ++n) { d->ux[n] = 0.0; d->uy[n] = 0.0; }
    } else {
        pseudopotential(d);
        forces_and_velocity(d);
    }
    if (!p->isothermal) thermal_rk4(d, d->ux, d->uy);
    if (!p->frozen_flow) collide_and_stream(d);
    d->t += 1;
    if (!p->periodic_y && d->nys >= 1 && d->t >= d->fl_ta && d->t < d->fl_tb &&
        (d->t - d->fl_ta) % d->fl_every == 0)
        sample_flux(d);
    size_t nt = (size_t)d->nx * d->nr;
    for (size_t n = 0; n < nt; ++n) if (!isfinite(d->T[n])) d->err = 1;
}

int orc_step(orc_dom *d, int64_t n) {
    for (int64_t k = 0; k < n; ++k) one_step(d);
    return d->err;
}

/* Fields at the current time t: rho(t), v(t) of Eq. 10 (forces at T(t)),
 * T(t) and, if f is not NULL, f(t). */
void orc_read(orc_dom *d, double *rho, double *ux, double *uy, double *T, double *f) {
    macroscopic(d);
    size_t nf = (size_t)d->nx * d->nyf;
    if (d->p.frozen_flow) {
        for (size_t n = 0; n < nf; ++n) { d->ux[n] = 0.0; d->uy[n] = 0.0; }
    } else {
        pseudopotential(d);
        forces_and_velocity(d);
    }
    if (rho) memcpy(rho, d->rho, sizeof(double) * nf);
    if (ux) memcpy(ux, d->ux, sizeof(double) * nf);
    if (uy) memcpy(uy, d->uy, sizeof(double) * nf);
    if (T) memcpy(T, d->T, sizeof(double) * (size_t)d->nx * d->nr);
    if (f) memcpy(f, d->f, sizeof(double) * 9 * nf);
}

/* Forces at the current state, for tests: Fm, total F, psi.  [nyf][nx] each. */
void orc_read_forces(orc_dom *d, double *Fmx, double *Fmy, double *Fx, double *Fy, double *psi) {
    macroscopic(d);
    pseudopotential(d);
    forces_and_velocity(d);
    size_t nf = (size_t)d->nx * d->nyf, b = sizeof(double) * nf;
    if (Fmx) memcpy(Fmx, d->Fmx, b);
    if (Fmy) memcpy(Fmy, d->Fmy, b);
    if (Fx) memcpy(Fx, d->Fx, b);
    if (Fy) memcpy(Fy, d->Fy, b);
    if (psi) memcpy(psi, d->psi, b);
}
