/*
 * poolboil.h -- C ABI of the MI355X (gfx950) implementation of the time step
 * of the hybrid pseudopotential phase-change lattice Boltzmann method for pool
 * boiling with conjugate heat transfer (Zhao, Liang, Sun, Cai, Li,
 * arXiv:1911.10747, Section 2; set-up of Section 3.1).
 *
 * One time step t -> t+1 of a domain is
 *   (1) pull streaming of the post-collision populations with halfway
 *       bounce-back at the walls and periodic x (Eq. 8, Section 3.1);
 *   (2) the macroscopic update rho = sum f, rho v = sum e f + F/2 (Eq. 10);
 *   (3) the pseudopotential psi(rho, T(t)) from the Peng-Robinson EOS
 *       (Eqs. 12-13) and the forces F = F_m + F_ads + F_g (Eqs. 11, 14, 15);
 *   (4) the energy equation (Eq. 24) advanced by RK4 (Eqs. 25-26) with the
 *       isotropic stencils (Eqs. 27-28) over the fluid and the solid heater,
 *       with rho(t), v(t) frozen inside the step;
 *   (5) the MRT collision with the improved forcing (Eqs. 3-7, 9);
 *   (6) optionally, the wall heat-flux sample (Eqs. 36, 38, 39).
 *
 * Grid and layout.  A domain has nx columns (periodic), ny_fluid fluid rows
 * and ny_solid heater rows below them.  Thermal rows are numbered
 * 0 .. ny_solid+ny_fluid-1 from the heater bottom up: rows < ny_solid are
 * solid, row 0 is held at the Dirichlet value T_b(x, t), and a virtual row
 * above the last fluid row is held at T_top.  Halfway bounce-back walls sit
 * between the heater and the first fluid row and above the last fluid row.
 * Every host array passed in or out is row-major with x fastest:
 *   rho, ux, uy : [ny_fluid][nx]             (fluid rows, y up)
 *   T           : [ny_solid + ny_fluid][nx]  (thermal rows, row 0 = heater bottom)
 *   f           : [9][ny_fluid][nx]          (D2Q9 in the order of Eq. 2)
 * All values are FP64 at the boundary.  Host arrays are copied; the caller
 * keeps ownership.  The library never retains a caller pointer after a call
 * returns, except the device memory given to pb_create_domain.
 *
 * Errors.  Every int-returning call returns PB_OK (0) or a negative PB_E*
 * code; pb_last_error() then gives a message (thread-local).  A handle must
 * not be used from two threads at once.  Calls that enqueue work are
 * asynchronous on the domain's stream; pb_sync() waits and reports the sticky
 * non-finite flag (negative psi radicand, NaN or Inf) as PB_ENONFINITE.
 */
#ifndef POOLBOIL_H
#define POOLBOIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PB_VERSION 1

enum {
    PB_OK = 0,
    PB_EINVAL = -1,      /* bad argument or configuration               */
    PB_ENOMEM = -2,      /* device allocation failed / buffer too small  */
    PB_EDEVICE = -3,     /* HIP runtime error                            */
    PB_ENONFINITE = -4,  /* sticky flag: negative psi radicand or NaN/Inf */
    PB_ESTATE = -5       /* call not valid in the current state          */
};

/* Storage precision.  PB_FP64: everything FP64.  PB_FP32_DEV stores rho(x)
 * and v in FP32 and the populations as f*_i - w_i rho(x) in FP32, taken
 * against that stored FP32 density, so rebuilding f in FP64 on load is exact
 * up to the rounding of the deviation; T stays FP64.  The flow step (moments,
 * psi and the EOS, forces, collision) computes in FP64 in both modes;
 * with PB_FP32_DEV the energy equation computes its operator and stages in
 * FP32 as increments over the FP64 T (FP64 for the differences
 * T(x + e_i) - T(x) and the update), within the FP32 tolerance of the
 * oracle comparisons. */
enum { PB_FP64 = 0, PB_FP32_DEV = 1 };

/* Configuration flags (pb_config.flags). */
#define PB_PERIODIC_Y    0x1u  /* periodic in y too: no walls, ny_solid = 0        */
#define PB_ISOTHERMAL    0x2u  /* skip the energy equation: T stays as set          */
#define PB_FROZEN_FLOW   0x4u  /* skip the flow: f fixed, v = 0 in Eq. 24           */
#define PB_SBAR2_PLUS    0x8u  /* + sign of the varpi term in row 2 of Eq. 9        */
#define PB_VARPI_FM_ONLY 0x10u /* varpi term of Eq. 9 uses F_m of Eq. 11 only
                                  (default: F_m + F_ads)                          */

/* Flat configuration, copied by pb_create_domain.  Every physical constant is
 * explicit; the library derives only rho_bar (Eq. 15, mean initial fluid
 * density) and per-step invariants from it. */
typedef struct pb_config {
    int32_t nx, ny_fluid, ny_solid;  /* ny_solid >= 1 unless PB_PERIODIC_Y (then 0);
                                        ny_solid = 1 is model A of Section 4.1
                                        (the Dirichlet row under the fluid)   */
    int32_t precision;               /* PB_FP64 or PB_FP32_DEV                   */
    uint32_t flags;                  /* PB_* flags                               */
    int32_t tile_x, tile_y;          /* flow-kernel tile: 64x4, 64x8, 32x8,       */
                                     /* 128x4, 32x16 or 64x16 nodes; 0,0 = 64x8;  */
                                     /* every tile gives the same bits           */
    int32_t thermal_tile;            /* energy-equation strips of 56 columns by */
                                     /* 28, 20, 24, 16, 12, 8 or 36 rows (1..7); */
                                     /* 0 = chosen from the domain size (tall    */
                                     /* strips for large domains, short ones for */
                                     /* small); every variant gives the same bits */
    double a, b, R, omega, Tc;       /* Eq. 13 (Tc explicit)                     */
    double G;                        /* Eq. 11-12 interaction strength (< 0)     */
    double s_e, s_q, varpi;          /* Eq. 3: s1 = s2 = s_e, s4 = s6 = s_q; Eq. 9 */
    double tau_L, tau_V, rho_L, rho_V; /* Eq. 5                                  */
    double g;                        /* Eq. 15: gravity (0, -g)                  */
    double Cv, Cvchi;                /* fluid C_V and lambda = Cvchi * rho        */
    double rho_S, C_S, lambda_S;     /* heater density, heat capacity, conductivity */
} pb_config;

/* Boundary data.  T_bottom_alt (if not NULL) replaces T_bottom for
 * alt_t0 <= t < alt_t1 (the fluctuating trigger of Section 3.2).  gamma_* are
 * the per-wall-node adhesion coefficients G_w psi(rho_w) of Eq. 14 (NULL = 0). */
typedef struct pb_bc {
    double T_top;
    const double *T_bottom;      /* [nx], required unless PB_PERIODIC_Y */
    const double *T_bottom_alt;  /* [nx] or NULL                         */
    int64_t alt_t0, alt_t1;
    const double *gamma_bottom;  /* [nx] or NULL                         */
    const double *gamma_top;     /* [nx] or NULL                         */
} pb_bc;

/* Heat flux (lattice units).  q_bottom: -lambda_S dT/dy at the heater bottom
 * with the one-sided second-order difference of Eq. 36 (the quantity of
 * Eq. 39 before scaling), averaged over x; with ny_solid < 3 (model A) there
 * are no heater rows to difference and q_bottom = q_top.  q_top: conductive
 * link flux from the heater top row into the fluid, averaged over x (uses the
 * conductances of the last completed step).  T_w: mean heater-top temperature
 * (Section 3.2).  *_mean: averages over the samples of the window (Eq. 38). */
typedef struct pb_flux {
    double q_bottom_inst, q_top_inst, T_w_inst;
    double q_bottom_mean, q_top_mean, T_w_mean;
    int64_t n_samples;
} pb_flux;

typedef struct pb_domain pb_domain;
typedef struct pb_batch pb_batch;

/* Device bytes a domain with this configuration needs (state, boundary data,
 * flags and flux accumulators; read-back staging is allocated on first read). */
int pb_domain_bytes(const pb_config *cfg, size_t *bytes);

/* Rows of the energy-equation strips (56 columns wide, Eqs. 24-28 swept upwards
 * by one wavefront each) a domain with this configuration uses: the explicit
 * thermal_tile, or for thermal_tile = 0 the tallest strips that still give
 * about 3072 strips (one per SIMD slot; at most 28 rows for PB_FP64), else
 * the shortest.  Host only;
 * PB_EINVAL for an invalid configuration. */
int pb_thermal_strip_rows(const pb_config *cfg, int *rows);

/* The energy launch's work list for n domains stepped together (n = 1: one
 * domain stepped alone by pb_step; n > 1: the batch pb_batch_create makes of
 * them, without persistent_blocks), in launch order, as (domain index, x0,
 * y0, rows) quadruples in out[4 * i .. 4 * i + 3]: a strip covers columns
 * x0 .. x0 + 55 and thermal rows y0 .. y0 + rows - 1 (clipped to the domain).
 * Strip height as pb_thermal_strip_rows gives for one domain (for several:
 * the first configuration's, or, when all have thermal_tile = 0, chosen for
 * their total size); when the strips outnumber the wavefront slots of the
 * chip, the top rows of each domain come as 8-row strips at the end of the
 * list.  Isothermal domains are left out.  *count receives the number of
 * strips; out may be NULL to query it, else cap (quadruples) must hold them
 * (PB_EINVAL otherwise).  Host only: for tests and tools. */
int pb_thermal_work_list(const pb_config *const *cfgs, int32_t n, int32_t *out, int64_t cap, int64_t *count);

/* The flow launch's work list of one domain stepped alone (a batch holds the
 * same tiles for each member, with the first member's tile shape), as (x0,
 * y0, width, height, alt) quintuples in out[5 * i .. 5 * i + 4]: a tile
 * covers fluid columns x0 .. x0 + width - 1 and rows y0 .. y0 + height - 1
 * (clipped to the domain), in the order built before the XCD ordering.
 * alt = 1 marks a 32 x 16 tile: with FP32-deviation storage and a 512-thread
 * tile shape wider than 32, the columns past the domain's last full tile go
 * to such tiles when that takes fewer tiles than partial ones.  *count
 * receives the number of tiles; out may be NULL to query it, else cap
 * (quintuples) must hold them (PB_EINVAL otherwise).  Host only: for tests
 * and tools.  PB_EINVAL for an invalid configuration. */
int pb_flow_work_list(const pb_config *cfg, int32_t *out, int64_t cap, int64_t *count);

/* Create a domain.  stream: a hipStream_t (NULL = the null stream).  dev_mem:
 * NULL to let the library allocate, or caller-owned device memory of at least
 * pb_domain_bytes() bytes (256-byte aligned) that must outlive the domain.
 * Fields start at zero; call pb_set_bc and pb_set_fields before stepping. */
int pb_create_domain(const pb_config *cfg, void *stream, void *dev_mem, size_t dev_bytes, pb_domain **out);
void pb_destroy_domain(pb_domain *dom);

/* Boundary data (Section 3.1 Dirichlet rows, Section 3.2 trigger, Eq. 14). */
int pb_set_bc(pb_domain *dom, const pb_bc *bc);

/* Initial state: f = w_i rho (rest equilibrium), T as given (row 0 is then set
 * to T_b(x, 0)), t = 0, rho_bar = mean of rho, error flag cleared. */
int pb_set_fields(pb_domain *dom, const double *rho, const double *T);

/* Full state for checkpoint/resume: f(t) after streaming, T(t), the time t and
 * rho_bar (Eq. 15), all exactly as pb_read_fields/pb_rho_bar returned them. */
int pb_set_fields_full(pb_domain *dom, const double *f, const double *T, int64_t t, double rho_bar);

/* Enqueue exactly n steps (asynchronous). */
int pb_step(pb_domain *dom, int64_t n);

/* Wait for the domain's work; PB_ENONFINITE if the sticky flag is set. */
int pb_sync(pb_domain *dom);

/* Synchronous read of rho(t), v(t) (Eq. 10 with the forces at T(t)), T(t) and,
 * if f is not NULL, f(t) after streaming.  Any output pointer may be NULL. */
int pb_read_fields(pb_domain *dom, double *rho, double *ux, double *uy, double *T, double *f);

/* pb_read_fields for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same outputs, bit for bit, but the FP64 read-back staging is a fixed
 * device array of PB_READ_NOALLOC_MAX_BYTES that every GPU the library runs
 * on holds for the life of the process, instead of memory allocated on the
 * first read.  The domain needs (13 * ny_fluid + ny_solid) * nx * 8 bytes of
 * it (so (13 * ny_fluid + ny_solid) * nx <= 8388608); a larger domain gets
 * PB_EINVAL before any device work.  No hipMalloc/hipFree is called.  Every
 * call on a GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (other threads or streams) race.
 * Synchronous, like pb_read_fields. */
#define PB_READ_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int pb_read_fields_noalloc(pb_domain *dom, double *rho, double *ux, double *uy, double *T, double *f);

/* Heat-flux sampling: a sample is taken after every step that ends at a time
 * t with t_a <= t < t_b and (t - t_a) % every == 0.  Resets the accumulators. */
int pb_flux_window(pb_domain *dom, int64_t t_a, int64_t t_b, int32_t every);
int pb_heat_flux(pb_domain *dom, pb_flux *out);   /* synchronous */

/* Diagnostics: enqueue n steps exactly as pb_step does, with HIP events
 * recorded on the domain's stream around every flow and thermal launch; wait
 * for them and return the mean launch durations in milliseconds:
 * avg_ms[0] = flow kernel, avg_ms[1] = thermal kernel, avg_ms[2] = elapsed
 * time of the whole sequence divided by n.  The steps are real steps.  The
 * events (2n + 1) stay with the domain and are reused by later calls; the
 * ones missing are created first, on the current device.
 * pb_profile_reserve creates them for up to n steps ahead of time, so that a
 * timed call creates none.  n in [1, 2^20]; PB_EDEVICE if an event cannot be
 * created. */
int pb_profile_steps(pb_domain *dom, int64_t n, double *avg_ms);
int pb_profile_reserve(pb_domain *dom, int64_t n);

int64_t pb_time(const pb_domain *dom);            /* current t              */
double pb_rho_bar(const pb_domain *dom);          /* rho_bar of Eq. 15      */

/* Batched stepping of many domains in shared launches (one flow and one
 * thermal launch per step for the whole set, tiles of every domain in one
 * work-list; frozen-flow domains are left out of the flow launch and
 * isothermal ones out of the thermal launch), optionally replayed from a
 * captured HIP graph of steps_per_graph steps (even).  All domains must share
 * the precision; they are stepped in lock-step on `stream`, or on a stream of
 * the batch's own if it is NULL, each pb_batch_step ordered after the work
 * already queued on the domains' streams and before work queued there later.
 * Each member keeps its own time t (members may have started at different
 * times).  Per-node arithmetic does not depend on the batch, so each domain's
 * result is bit-identical to stepping it alone.  Tile shapes come from the
 * first member's configuration; when every member has thermal_tile = 0 the
 * energy strips are chosen for the batch's total size (pb_thermal_strip_rows's
 * rule over all members).  persistent_blocks > 0 caps the grid (blocks then
 * loop over the work-list).  A domain must stay alive while it is a member. */
int pb_batch_create(pb_domain *const *doms, int32_t n, int32_t steps_per_graph, int32_t persistent_blocks,
                    void *stream, pb_batch **out);
int pb_batch_step(pb_batch *batch, int64_t n);
void pb_batch_destroy(pb_batch *batch);

/* Membership changes between steps, for continuous batching (jobs join and
 * leave a batch that keeps running).  pb_batch_add appends a domain (fields
 * set, the batch's precision, not already a member); pb_batch_remove takes one
 * out.  The launches' work lists and descriptor table are rebuilt on the host
 * and uploaded on the batch stream, ordered after the steps already queued
 * (those still step the previous members); no member stream is synchronised,
 * and the captured step graph is captured again at the next graph-length step.
 * A batch may become empty (pb_batch_step then does nothing).  Work queued
 * before a removal still reaches the removed domain and its stream waits for
 * that work, so the domain may be destroyed right after pb_batch_remove.
 * Errors: PB_EINVAL (NULL, not a member / already a member, other precision),
 * PB_ESTATE (no fields), PB_ENOMEM, PB_EDEVICE; on error the membership is
 * unchanged. */
int pb_batch_add(pb_batch *batch, pb_domain *dom);
int pb_batch_remove(pb_batch *batch, pb_domain *dom);
int32_t pb_batch_size(const pb_batch *batch);   /* members, or -1 for NULL */

/* Host helpers for configuration (no device work): the critical temperature
 * implied by a = 0.45724 R^2 Tc^2/Pc and b = 0.0778 R Tc/Pc (Section 2.1), and
 * the Maxwell coexistence densities of Eq. 13 at temperature T (Section 3.1). */
int pb_eos_critical_temperature(double a, double b, double R, double *Tc);
int pb_eos_coexistence(double a, double b, double R, double omega, double Tc, double T, double *rho_L,
                       double *rho_V);

/* Latent heat h_fg at T < Tc for Eq. 13 by the Clausius-Clapeyron relation
 * h_fg = T (1/rho_V - 1/rho_L) dP_sat/dT, with dP_sat/dT from centred
 * differences of the Maxwell saturation pressure (Section 3.1, Eq. 37 uses it
 * for the Jakob number). */
int pb_eos_latent_heat(double a, double b, double R, double omega, double Tc, double T, double *h_fg);

/* psi of Eq. 12 (c = 1, c_s^2 = 1/3) with P_EOS of Eq. 13 at (rho, T); used
 * to express wall adhesion gamma = G_w psi(rho_w) of Eq. 14. */
int pb_eos_psi(double a, double b, double R, double omega, double Tc, double G, double rho, double T, double *psi);

const char *pb_last_error(void);
int pb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* POOLBOIL_H */
