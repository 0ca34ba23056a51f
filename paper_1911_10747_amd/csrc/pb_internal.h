// Internal structures shared by the host API (pb_api.cpp) and the kernels
// (pb_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Per-domain descriptor read by every kernel (one per domain of a launch).
// Buffers come in A/B pairs; step k of a launch sequence reads buffer
// (par0 + k) & 1 and writes the other.  t = t0 + k.
struct PbDesc {
    // geometry
    int32_t nx, nyf, nys, nr, pitch;
    uint32_t flags;
    int32_t par0;
    int32_t pad0;
    int64_t t0;
    int64_t fl_ta, fl_tb;
    int32_t fl_every;
    int32_t pad1;
    // state
    void *f[2];          // populations [9][nyf][pitch], double or float (deviation)
    void *rho[2];        // rho(t) written by the flow kernel, [nyf][pitch]; FP32 with FP32 storage
    void *vx, *vy;       // v(t) written by the flow kernel, [nyf][pitch]; FP32 with FP32 storage
    double *T[2];        // temperature [nr][pitch]
    // boundary data [nx]
    const double *Tb, *Tb_alt, *gbot, *gtop;
    int64_t alt_t0, alt_t1;
    double T_top;
    // diagnostics
    int32_t *err;        // sticky non-finite flag
    double *sink;        // [64]: where the energy sweep's halo lanes send their discarded stores
    double *flux;        // [8]: q_bot, q_top, Tw (inst), their sums, count
    // read-back staging (FP64, [9][nyf][pitch] + 3 x [nyf][pitch])
    double *rd_f, *rd_rho, *rd_vx, *rd_vy;
    // constants
    double a, b, R, kappa, Tc, sqrtTc, inv_sqrtTc, G, invG;
    double s_e, s_q, varpi;
    double tau_V, rho_V, ktau;   // tau(rho) = tau_V + (rho - rho_V) * ktau  (Eq. 5)
    double g, rho_bar;
    double Cv, Cvchi, rho_S, C_S, lambda_S;
    // uniform factors of the flow update, derived once from the constants above
    double eos_s0, eos_s1;   // s(T) = 1 + kappa (1 - sqrt(T / Tc)) = eos_s0 - eos_s1 sqrt(T)  (Eq. 13)
    double two_invG;         // 2 / G  (Eq. 12)
    double cw_k;             // 12 varpi s_e  (varpi term of Eq. 9)
    double hse, hsq;         // 1 - s_e / 2, 1 - s_q / 2  (Eq. 7)
    double s2sign;           // +1 with PB_SBAR2_PLUS (row 2 adds the varpi term), else -1
};

struct PbTile {
    int32_t dom, x0, y0;
    // 1 = the launch's alternate shape: in the energy sweep an 8-row strip,
    // whatever the launch's strip height; in a 512-thread FP32 flow launch a
    // 32 x 16 tile (the columns past a domain's last full tile)
    int32_t alt;
};

enum { PB_MODE_STEP = 0, PB_MODE_READ = 1 };

// Launch helpers implemented in pb_kernels.hip.  All return hipError_t.
// prec: 0 = FP64 storage, 1 = FP32 deviation storage.
// d_descs is a device array of device pointers to the domains' descriptors.
// tile_variant may carry PB_FLOW_ALT_TILES: the work list holds alternate
// tiles (pb_flow_alt_shape), launched with the kernel that handles them.
#define PB_FLOW_ALT_TILES 0x100
hipError_t pb_launch_flow(int prec, int mode, int tile_variant, const PbDesc *const *d_descs, const PbTile *d_tiles,
                          int ntiles, int grid, int k, hipStream_t s);
hipError_t pb_launch_thermal(int prec, int tile_variant, const PbDesc *const *d_descs, const PbTile *d_tiles,
                             int ntiles, int grid, int k, hipStream_t s);
hipError_t pb_launch_flux(int prec, const PbDesc *const *d_descs, int ndom, int k, hipStream_t s);
hipError_t pb_launch_advance(PbDesc *const *d_descs, int ndom, int nsteps, hipStream_t s);
hipError_t pb_launch_init(int prec, const PbDesc *d_desc, const double *rho_src, hipStream_t s);
// 2D copy on the device: rows x width elements of elem_bytes (4 or 8) from
// rows spitch elements apart to rows dpitch elements apart
hipError_t pb_launch_repitch(int elem_bytes, void *dst, size_t dpitch, const void *src, size_t spitch, size_t width,
                             size_t rows, hipStream_t s);

// Fixed read-back staging of pb_read_fields_noalloc: a file-scope device array
// of PB_SCRATCH_BYTES in pb_kernels.hip, one per GPU for the life of the
// process.  pb_scratch_address gives its device address on the current device
// (looked up once per device with hipGetSymbolAddress).
#define PB_SCRATCH_BYTES ((size_t)64 << 20)
hipError_t pb_scratch_address(void **ptr, size_t *bytes);

// Tile geometry of the variants (x, y extents of one block's tile).
void pb_flow_tile_shape(int variant, int *bx, int *by);
// Whether flow launches of this precision (0 FP64, 1 FP32 deviation) and
// variant take tiles of the alternate shape (PbTile.alt), and that shape.
int pb_flow_alt_shape(int prec, int variant, int *ax, int *ay);
void pb_thermal_tile_shape(int variant, int *bx, int *by);
int pb_flow_variants();
int pb_thermal_variants();
