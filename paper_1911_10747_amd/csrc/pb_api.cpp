// Host side of the C ABI declared in include/poolboil.h: domain lifecycle,
// boundary data, state upload/read-back, stepping, heat flux, batched and
// graph-replayed stepping, and host EOS helpers for building configurations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/poolboil.h"
#include "pb_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define PB_HIP(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return fail(PB_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));     \
    } while (0)

constexpr size_t kAlign = 256;
static_assert(PB_SCRATCH_BYTES == PB_READ_NOALLOC_MAX_BYTES, "fixed read-back staging size");
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

const double kWh[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
const int kEXh[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int kEYh[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const int kOPPh[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

int flow_variant_of(const pb_config &c) {
    if (c.tile_x == 0 && c.tile_y == 0) return 1;   // 64x8
    for (int v = 0; v < pb_flow_variants(); ++v) {
        int bx, by;
        pb_flow_tile_shape(v, &bx, &by);
        if (bx == c.tile_x && by == c.tile_y) return v;
    }
    return -1;
}

int ntiles_for(int nx, int ny, int bx, int by) { return ((nx + bx - 1) / bx) * ((ny + by - 1) / by); }

// Thermal strip variant chosen from the sizes (nx, rows) of the domains one
// launch steps: the tallest strips whose count over those domains still gives
// about one strip per SIMD slot (3072 at 3 waves per SIMD on 256 CUs), else
// the shortest, since a small domain's step time is the sweep of one strip.
int thermal_variant_for(int precision, const std::vector<std::pair<int, int>> &doms) {
    int best = -1, best_h = 0, shortest = 0, shortest_h = 1 << 30;
    for (int v = 0; v < pb_thermal_variants(); ++v) {
        int bx, by;
        pb_thermal_tile_shape(v, &bx, &by);
        // FP64 strips stop at 28 rows: its sweep measured slower with 36
        // (4096 x 2112: 132 us against 127.5; FP32: 76.3 against 79.7)
        if (precision == PB_FP64 && by > 28) continue;
        int64_t strips = 0;
        for (const auto &d : doms) strips += ntiles_for(d.first, d.second, bx, by);
        if (strips >= 3072 && by > best_h) {
            best = v;
            best_h = by;
        }
        if (by < shortest_h) {
            shortest = v;
            shortest_h = by;
        }
    }
    return best >= 0 ? best : shortest;
}

// Thermal strip variant of a config: thermal_tile k >= 1 is variant k - 1,
// 0 the choice above for the domain alone.
int thermal_variant_of(const pb_config &c) {
    if (c.thermal_tile > 0) return c.thermal_tile - 1;
    return thermal_variant_for(c.precision, {{c.nx, c.ny_fluid + c.ny_solid}});
}

int max_tiles(int nx, int ny, bool flow) {
    int m = 0, nv = flow ? pb_flow_variants() : pb_thermal_variants();
    for (int v = 0; v < nv; ++v) {
        int bx, by;
        if (flow) pb_flow_tile_shape(v, &bx, &by); else pb_thermal_tile_shape(v, &bx, &by);
        m = std::max(m, ntiles_for(nx, ny, bx, by));
    }
    return m;
}

// Arena layout of one domain (offsets in bytes from the base).
struct Layout {
    size_t desc, dptr, f[2], rho[2], vx, vy, T[2], Tb, Tba, gb, gt, err, flux, sink, tflow, tth, total;
};

Layout layout_of(const pb_config &c) {
    Layout L{};
    const size_t pitch = align_up((size_t)c.nx, 64);
    const size_t nf = (size_t)c.ny_fluid * pitch, nt = (size_t)(c.ny_fluid + c.ny_solid) * pitch;
    const size_t es = c.precision == PB_FP32_DEV ? 4 : 8;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes, kAlign); return r; };
    L.desc = take(sizeof(PbDesc));
    L.dptr = take(sizeof(void *));
    L.f[0] = take(9 * nf * es);
    L.f[1] = take(9 * nf * es);
    L.rho[0] = take(nf * es);   // density stored like the populations: FP64 or FP32
    L.rho[1] = take(nf * es);
    L.vx = take(nf * es);   // velocity stored like the populations: FP64 or FP32
    L.vy = take(nf * es);
    L.T[0] = take(nt * 8);
    L.T[1] = take(nt * 8);
    L.Tb = take((size_t)c.nx * 8);
    L.Tba = take((size_t)c.nx * 8);
    L.gb = take((size_t)c.nx * 8);
    L.gt = take((size_t)c.nx * 8);
    L.err = take(sizeof(int32_t));
    L.flux = take(8 * sizeof(double));
    L.sink = take(64 * sizeof(double));
    L.tflow = take((size_t)max_tiles(c.nx, c.ny_fluid, true) * sizeof(PbTile));
    L.tth = take((size_t)max_tiles(c.nx, c.ny_fluid + c.ny_solid, false) * sizeof(PbTile));
    L.total = o;
    return L;
}

int validate(const pb_config *c) {
    if (!c) return fail(PB_EINVAL, "config is NULL");
    if (c->nx < 1 || c->ny_fluid < 1) return fail(PB_EINVAL, "nx and ny_fluid must be >= 1");
    if (c->nx > (1 << 20) || c->ny_fluid > (1 << 20) || c->ny_solid > (1 << 20))
        return fail(PB_EINVAL, "domain dimension above 2^20");
    {
        // the kernels address a domain's arrays with 32-bit element offsets:
        // nine population planes, and the thermal rows
        const uint64_t pitch = align_up((size_t)c->nx, 64);
        if (9ull * (uint64_t)c->ny_fluid * pitch >= (1ull << 32) ||
            (uint64_t)(c->ny_fluid + c->ny_solid) * pitch >= (1ull << 32))
            return fail(PB_EINVAL, "domain of %d x (%d + %d) nodes exceeds 32-bit element offsets "
                        "(9 * ny_fluid * pitch and (ny_fluid + ny_solid) * pitch must stay below 2^32)",
                        c->nx, c->ny_fluid, c->ny_solid);
    }
    if (c->precision != PB_FP64 && c->precision != PB_FP32_DEV) return fail(PB_EINVAL, "unknown precision %d", c->precision);
    if (c->flags & ~0x1Fu) return fail(PB_EINVAL, "unknown flag bits 0x%x", c->flags);
    const bool pery = (c->flags & PB_PERIODIC_Y) != 0;
    if (pery && c->ny_solid != 0) return fail(PB_EINVAL, "PB_PERIODIC_Y needs ny_solid == 0");
    if (!pery && c->ny_solid < 1) return fail(PB_EINVAL, "ny_solid must be >= 1 (row 0 is the Dirichlet heater bottom)");
    if (!(c->G < 0.0)) return fail(PB_EINVAL, "G must be negative (Eq. 12)");
    if (!(c->Tc > 0.0) || !(c->b > 0.0) || !(c->R > 0.0)) return fail(PB_EINVAL, "Tc, b and R must be positive");
    if (!(c->rho_L > c->rho_V) || !(c->rho_V > 0.0)) return fail(PB_EINVAL, "need rho_L > rho_V > 0");
    if (!(c->Cv > 0.0) || !(c->Cvchi > 0.0) || !(c->lambda_S > 0.0) || !(c->rho_S > 0.0) || !(c->C_S > 0.0))
        return fail(PB_EINVAL, "thermal properties must be positive");
    if (!(c->s_e > 0.0 && c->s_e < 2.0) || !(c->s_q > 0.0 && c->s_q < 2.0))
        return fail(PB_EINVAL, "relaxation rates must lie in (0, 2)");
    if (!(c->tau_L > 0.5) || !(c->tau_V > 0.5)) return fail(PB_EINVAL, "relaxation times must exceed 1/2");
    if (flow_variant_of(*c) < 0) return fail(PB_EINVAL, "no flow tile %dx%d", c->tile_x, c->tile_y);
    if (c->thermal_tile < 0 || c->thermal_tile > pb_thermal_variants())
        return fail(PB_EINVAL, "no thermal tile variant %d", c->thermal_tile);
    return PB_OK;
}

// Order tiles so that the hardware's round-robin placement of consecutive
// workgroups over the 8 XCDs gives each XCD a contiguous band of tiles (halo
// re-reads then hit that XCD's L2).
void xcd_order(std::vector<PbTile> &tiles) {
    const int n = (int)tiles.size(), X = 8;
    if (n < 2 * X) return;
    std::vector<PbTile> out(n);
    const int q = n / X, r = n % X;
    for (int b = 0; b < n; ++b) {
        const int j = b % X, s = b / X;
        const int off = j * q + std::min(j, r);
        out[b] = tiles[off + s];
    }
    tiles.swap(out);
}

void make_tiles(std::vector<PbTile> &out, int dom, int nx, int ny, int bx, int by) {
    for (int y0 = 0; y0 < ny; y0 += by)
        for (int x0 = 0; x0 < nx; x0 += bx) out.push_back(PbTile{dom, x0, y0, 0});
}

// Flow tiles of one domain for launches of (precision, variant).  Where the
// launch takes alternate tiles, the columns past the last full tile go to
// alternate tiles when that takes fewer of them than the partial tiles would
// (a partial tile computes as much as a full one); the list is never longer
// than make_tiles'.  Returns whether it added alternate tiles.
bool make_flow_tiles(std::vector<PbTile> &out, int dom, int nx, int ny, int prec, int variant) {
    int bx, by, ax, ay;
    pb_flow_tile_shape(variant, &bx, &by);
    const bool alt_ok = pb_flow_alt_shape(prec, variant, &ax, &ay) != 0;
    const int full = nx / bx * bx, r = nx - full;
    const bool alt = alt_ok && r > 0 &&
                     (int64_t)((r + ax - 1) / ax) * ((ny + ay - 1) / ay) < (int64_t)((ny + by - 1) / by);
    if (!alt) {
        make_tiles(out, dom, nx, ny, bx, by);
        return false;
    }
    make_tiles(out, dom, full, ny, bx, by);
    for (int y0 = 0; y0 < ny; y0 += ay)
        for (int x0 = full; x0 < nx; x0 += ax) out.push_back(PbTile{dom, x0, y0, 1});
    return true;
}

// A domain's share of an energy-strip work list: index, columns, thermal rows.
struct ThermalDom {
    int dom, nx, nr;
};

// Energy-strip work list of one or more domains (slots: wavefronts the chip
// holds at once, 256 CUs x 4 SIMDs x the sweep's waves per SIMD).  Strips of
// by rows; when there are more of them than slots, the top rows of every
// domain become 8-row strips (alt = 1), about 0.6 slots in all,
// shared out by area, and are placed last: the wavefronts that start last are
// then short and the launch ends with few idle slots (4096 x 2112 rows, FP32,
// 28-row strips: 91.5 -> 81.7 us).  With ordered set, each part is ordered for
// the XCDs on its own.
void make_thermal_tiles(std::vector<PbTile> &out, const std::vector<ThermalDom> &doms, int bx, int by, int slots,
                        bool ordered) {
    int64_t tall = 0, area = 0;
    for (const ThermalDom &t : doms) {
        const int64_t cols = (t.nx + bx - 1) / bx;
        tall += cols * ((t.nr + by - 1) / by);
        area += cols * t.nr;
    }
    const bool tail = by > 8 && tall > slots;
    std::vector<PbTile> big, small;
    for (const ThermalDom &t : doms) {
        int ytail = t.nr;
        if (tail) {
            const int trows = 8 * std::max(1, (int)(0.6 * slots * t.nr / (double)area + 0.5));
            ytail = std::max(0, (t.nr - trows) / by * by);
        }
        make_tiles(big, t.dom, t.nx, ytail, bx, by);
        for (int y0 = ytail; y0 < t.nr; y0 += 8)
            for (int x0 = 0; x0 < t.nx; x0 += bx) small.push_back(PbTile{t.dom, x0, y0, 1});
    }
    if (ordered) {
        xcd_order(big);
        xcd_order(small);
    }
    out.insert(out.end(), big.begin(), big.end());
    out.insert(out.end(), small.begin(), small.end());
}

// wavefront slots of the energy sweep: 3 waves per SIMD in FP32, 2 in FP64
int thermal_slots(int precision) { return 256 * 4 * (precision == PB_FP32_DEV ? 3 : 2); }

// Strip variant of one energy launch over these domains: the first one's,
// unless all leave the strips to the library (thermal_tile = 0); then strips
// chosen for all of them together (for one domain, its own size).
int launch_thermal_variant(const std::vector<const pb_config *> &cfgs) {
    bool auto_strips = true;
    std::vector<std::pair<int, int>> sizes;
    for (const pb_config *c : cfgs) {
        auto_strips = auto_strips && c->thermal_tile == 0;
        if (!(c->flags & PB_ISOTHERMAL)) sizes.push_back({c->nx, c->ny_fluid + c->ny_solid});
    }
    if (auto_strips && !sizes.empty()) return thermal_variant_for(cfgs[0]->precision, sizes);
    return thermal_variant_of(*cfgs[0]);
}

// Work list of one energy launch over these domains (isothermal ones left out)
void thermal_list(std::vector<PbTile> &tt, const std::vector<const pb_config *> &cfgs, int tvar, bool ordered) {
    int bx, by;
    pb_thermal_tile_shape(tvar, &bx, &by);
    std::vector<ThermalDom> tdoms;
    for (int j = 0; j < (int)cfgs.size(); ++j)
        if (!(cfgs[j]->flags & PB_ISOTHERMAL))
            tdoms.push_back(ThermalDom{j, cfgs[j]->nx, cfgs[j]->ny_fluid + cfgs[j]->ny_solid});
    make_thermal_tiles(tt, tdoms, bx, by, thermal_slots(cfgs[0]->precision), ordered);
}

}  // namespace

struct pb_domain {
    pb_config cfg{};
    hipStream_t stream = nullptr;
    char *base = nullptr;
    bool owns = false;
    Layout L{};
    PbDesc hd{};                 // host mirror of the device descriptor
    PbDesc *ddesc = nullptr;     // device descriptor
    PbDesc **dptr = nullptr;     // device array holding the one pointer ddesc
    int pitch = 0, nr = 0;
    int64_t t = 0;
    int par = 0;
    bool fields_set = false;
    int fvar = 0, tvar = 0;
    int flow_launch_var = 0;     // fvar, with PB_FLOW_ALT_TILES if its work list holds alternate tiles
    int nt_flow = 0, nt_th = 0;
    int device = 0;              // the GPU the domain lives on
    PbTile *dtiles_flow = nullptr, *dtiles_th = nullptr;
    std::vector<double> Tb, Tba, gb, gt;
    double *rd = nullptr;        // read-back staging of pb_read_fields (lazy)
    std::vector<hipEvent_t> prof_ev;   // events of pb_profile_steps, kept for reuse
};

struct pb_batch {
    std::vector<pb_domain *> doms;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    int prec = 0, fvar = 0, tvar = 0;
    int flow_launch_var = 0;     // fvar, with PB_FLOW_ALT_TILES if the flow work list holds alternate tiles
    int nt_flow = 0, nt_th = 0, grid_flow = 0, grid_th = 0;
    int spg = 0, persistent = 0;
    // device tables of the launches, one buffer: descriptor pointers, flow
    // tiles, energy strips; written from a pinned staging copy by an upload on
    // the batch stream, so they change in stream order.  Two staging copies
    // are used in turn: one is rewritten only after its previous upload (two
    // membership changes ago) has been read.
    char *dtab = nullptr, *htab[2] = {nullptr, nullptr};
    size_t tab_cap = 0, htab_cap[2] = {0, 0};
    int hslot = 0;
    PbDesc **dptrs = nullptr;
    PbTile *dtiles_flow = nullptr, *dtiles_th = nullptr;
    hipEvent_t ev_upload[2] = {nullptr, nullptr};   // after the last upload from each staging copy
    bool upload_pending[2] = {false, false};
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<char> graph_flux;   // steps of the captured graph that launch the flux sample
    // graphs and table buffers replaced by a membership change, released once
    // the work queued before the change (event `done`) has finished
    struct Retired {
        hipGraphExec_t exec;
        hipGraph_t graph;
        char *tab;
        hipEvent_t done;
    };
    std::vector<Retired> retired;
    hipEvent_t ev_batch = nullptr, ev_dom = nullptr;
    std::vector<hipStream_t> dom_streams;   // distinct member streams
};

namespace {

int upload_desc(pb_domain *d) {
    d->hd.t0 = d->t;
    d->hd.par0 = d->par;
    PB_HIP(hipMemcpyAsync(d->ddesc, &d->hd, sizeof(PbDesc), hipMemcpyHostToDevice, d->stream));
    PB_HIP(hipStreamSynchronize(d->stream));
    return PB_OK;
}

int upload_tiles(pb_domain *d) {
    std::vector<PbTile> tf, tt;
    const bool alt = make_flow_tiles(tf, 0, d->cfg.nx, d->cfg.ny_fluid, d->cfg.precision, d->fvar);
    d->flow_launch_var = d->fvar | (alt ? PB_FLOW_ALT_TILES : 0);
    thermal_list(tt, {&d->cfg}, d->tvar, true);
    xcd_order(tf);
    if ((int)tf.size() > max_tiles(d->cfg.nx, d->cfg.ny_fluid, true) || (int)tt.size() > max_tiles(d->cfg.nx, d->nr, false))
        return fail(PB_EINVAL, "work list longer than its table");
    d->nt_flow = (int)tf.size();
    d->nt_th = (int)tt.size();
    PB_HIP(hipMemcpyAsync(d->dtiles_flow, tf.data(), tf.size() * sizeof(PbTile), hipMemcpyHostToDevice, d->stream));
    PB_HIP(hipMemcpyAsync(d->dtiles_th, tt.data(), tt.size() * sizeof(PbTile), hipMemcpyHostToDevice, d->stream));
    PB_HIP(hipStreamSynchronize(d->stream));
    return PB_OK;
}

double bc_bottom(const pb_domain *d, int x, int64_t t) {
    if (!d->Tba.empty() && t >= d->hd.alt_t0 && t < d->hd.alt_t1) return d->Tba[x];
    return d->Tb.empty() ? d->hd.T_top : d->Tb[x];
}

// Host arrays hold dense rows of nx elements, device arrays rows pitch
// elements apart.  Every host transfer is one contiguous copy (a 2D copy
// between pageable host memory and the device moves row by row, minutes for
// a tall, narrow domain); where pitch != nx the rows are re-pitched on the
// device through tmp (rows x nx elements; unused when pitch == nx).
int upload_rows(pb_domain *d, void *dst, const void *src, int rows, int elem, void *tmp) {
    const size_t nx = (size_t)d->cfg.nx, bytes = (size_t)rows * nx * elem;
    if ((size_t)d->pitch == nx) {
        PB_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, d->stream));
        return PB_OK;
    }
    PB_HIP(hipMemcpyAsync(tmp, src, bytes, hipMemcpyHostToDevice, d->stream));
    PB_HIP(pb_launch_repitch(elem, dst, (size_t)d->pitch, tmp, nx, nx, (size_t)rows, d->stream));
    return PB_OK;
}

int download_rows(pb_domain *d, double *dst, const double *src, int rows, double *tmp) {
    const size_t nx = (size_t)d->cfg.nx, bytes = (size_t)rows * nx * sizeof(double);
    if ((size_t)d->pitch != nx) {
        PB_HIP(pb_launch_repitch(8, tmp, nx, src, (size_t)d->pitch, nx, (size_t)rows, d->stream));
        src = tmp;
    }
    PB_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, d->stream));
    return PB_OK;
}

// Device memory for the dense rows of an upload (rows x nx doubles); none
// when pitch == nx.  Freed when it goes out of scope, after the domain's
// stream (whose kernels read it) has drained, on error returns too.
struct UploadTmp {
    void *p = nullptr;
    hipStream_t s = nullptr;
    ~UploadTmp() {
        if (p) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(p);
        }
    }
    bool get(const pb_domain *d, int rows) {
        s = d->stream;
        if (d->pitch == d->cfg.nx) return true;
        return hipMalloc(&p, (size_t)rows * d->cfg.nx * sizeof(double)) == hipSuccess;
    }
};

int check_dom(const pb_domain *d) {
    if (!d) return fail(PB_EINVAL, "domain is NULL");
    return PB_OK;
}

int enqueue_steps(pb_domain *d, int64_t n) {
    const bool frozen = d->cfg.flags & PB_FROZEN_FLOW, iso = d->cfg.flags & PB_ISOTHERMAL;
    const bool sampling = !(d->cfg.flags & PB_PERIODIC_Y) && d->cfg.ny_solid >= 1 && d->hd.fl_tb > d->hd.fl_ta;
    const PbDesc *const *dp = (const PbDesc *const *)d->dptr;
    // the descriptor's kernel step index is an int; long runs are split
    const int64_t chunk = 1 << 30;
    while (n > 0) {
        const int m = (int)std::min<int64_t>(n, chunk);
        for (int k = 0; k < m; ++k) {
            if (!frozen) PB_HIP(pb_launch_flow(d->cfg.precision, PB_MODE_STEP, d->flow_launch_var, dp, d->dtiles_flow, d->nt_flow,
                                               d->nt_flow, k, d->stream));
            if (!iso) PB_HIP(pb_launch_thermal(d->cfg.precision, d->tvar, dp, d->dtiles_th, d->nt_th, d->nt_th, k, d->stream));
            const int64_t tk = d->t + k + 1;
            if (sampling && tk >= d->hd.fl_ta && tk < d->hd.fl_tb && (tk - d->hd.fl_ta) % d->hd.fl_every == 0)
                PB_HIP(pb_launch_flux(d->cfg.precision, dp, 1, k, d->stream));
        }
        PB_HIP(pb_launch_advance(d->dptr, 1, m, d->stream));
        d->t += m;
        d->par ^= (m & 1);
        n -= m;
    }
    d->hd.t0 = d->t;
    d->hd.par0 = d->par;
    return PB_OK;
}

}  // namespace

extern "C" {

int pb_version(void) { return PB_VERSION; }
const char *pb_last_error(void) { return g_err.c_str(); }

int pb_thermal_strip_rows(const pb_config *cfg, int *rows) {
    int rc = validate(cfg);
    if (rc) return rc;
    if (!rows) return fail(PB_EINVAL, "rows is NULL");
    int bx, by;
    pb_thermal_tile_shape(thermal_variant_of(*cfg), &bx, &by);
    *rows = by;
    return PB_OK;
}

int pb_flow_work_list(const pb_config *cfg, int32_t *out, int64_t cap, int64_t *count) {
    if (!count) return fail(PB_EINVAL, "count is NULL");
    int rc = validate(cfg);
    if (rc) return rc;
    const int fvar = flow_variant_of(*cfg);
    int bx, by, ax, ay;
    pb_flow_tile_shape(fvar, &bx, &by);
    pb_flow_alt_shape(cfg->precision, fvar, &ax, &ay);
    std::vector<PbTile> tf;
    make_flow_tiles(tf, 0, cfg->nx, cfg->ny_fluid, cfg->precision, fvar);
    *count = (int64_t)tf.size();
    if (out && cap < (int64_t)tf.size()) return fail(PB_EINVAL, "out holds %lld tiles, %lld needed", (long long)cap,
                                                     (long long)tf.size());
    if (out)
        for (size_t i = 0; i < tf.size(); ++i) {
            out[5 * i] = tf[i].x0;
            out[5 * i + 1] = tf[i].y0;
            out[5 * i + 2] = tf[i].alt ? ax : bx;
            out[5 * i + 3] = tf[i].alt ? ay : by;
            out[5 * i + 4] = tf[i].alt;
        }
    return PB_OK;
}

int pb_thermal_work_list(const pb_config *const *cfgs, int32_t n, int32_t *out, int64_t cap, int64_t *count) {
    if (!cfgs || n < 1) return fail(PB_EINVAL, "need at least one configuration");
    if (!count) return fail(PB_EINVAL, "count is NULL");
    std::vector<const pb_config *> v(n);
    for (int j = 0; j < n; ++j) {
        int rc = validate(cfgs[j]);
        if (rc) return rc;
        if (cfgs[j]->precision != cfgs[0]->precision) return fail(PB_EINVAL, "mixed precisions in one launch");
        v[j] = cfgs[j];
    }
    const int tvar = launch_thermal_variant(v);
    int bx, by;
    pb_thermal_tile_shape(tvar, &bx, &by);
    std::vector<PbTile> tt;
    thermal_list(tt, v, tvar, true);
    *count = (int64_t)tt.size();
    if (out && cap < (int64_t)tt.size()) return fail(PB_EINVAL, "out holds %lld strips, %lld needed", (long long)cap,
                                                     (long long)tt.size());
    if (out)
        for (size_t i = 0; i < tt.size(); ++i) {
            out[4 * i] = tt[i].dom;
            out[4 * i + 1] = tt[i].x0;
            out[4 * i + 2] = tt[i].y0;
            out[4 * i + 3] = tt[i].alt ? 8 : by;
        }
    return PB_OK;
}

int pb_domain_bytes(const pb_config *cfg, size_t *bytes) {
    int rc = validate(cfg);
    if (rc) return rc;
    if (!bytes) return fail(PB_EINVAL, "bytes is NULL");
    *bytes = layout_of(*cfg).total;
    return PB_OK;
}

int pb_create_domain(const pb_config *cfg, void *stream, void *dev_mem, size_t dev_bytes, pb_domain **out) {
    int rc = validate(cfg);
    if (rc) return rc;
    if (!out) return fail(PB_EINVAL, "out is NULL");
    *out = nullptr;
    pb_domain *d = new (std::nothrow) pb_domain();
    if (!d) return fail(PB_ENOMEM, "host allocation failed");
    d->cfg = *cfg;
    d->stream = (hipStream_t)stream;
    d->L = layout_of(*cfg);
    d->pitch = (int)align_up((size_t)cfg->nx, 64);
    d->nr = cfg->ny_fluid + cfg->ny_solid;
    d->fvar = flow_variant_of(*cfg);
    d->tvar = thermal_variant_of(*cfg);
    if (hipGetDevice(&d->device) != hipSuccess) {
        delete d;
        return fail(PB_EDEVICE, "no current device");
    }
    if (dev_mem) {
        if (dev_bytes < d->L.total) {
            delete d;
            return fail(PB_ENOMEM, "device buffer of %zu bytes, %zu needed", dev_bytes, d->L.total);
        }
        if ((uintptr_t)dev_mem % kAlign) {
            delete d;
            return fail(PB_EINVAL, "device buffer must be %zu-byte aligned", kAlign);
        }
        d->base = (char *)dev_mem;
    } else {
        if (hipMalloc((void **)&d->base, d->L.total) != hipSuccess) {
            delete d;
            return fail(PB_ENOMEM, "hipMalloc of %zu bytes failed", d->L.total);
        }
        d->owns = true;
    }
    const Layout &L = d->L;
    PbDesc &h = d->hd;
    memset(&h, 0, sizeof(h));
    h.nx = cfg->nx;
    h.nyf = cfg->ny_fluid;
    h.nys = cfg->ny_solid;
    h.nr = d->nr;
    h.pitch = d->pitch;
    h.flags = cfg->flags;
    for (int b = 0; b < 2; ++b) {
        h.f[b] = d->base + L.f[b];
        h.rho[b] = (void *)(d->base + L.rho[b]);
        h.T[b] = (double *)(d->base + L.T[b]);
    }
    h.vx = d->base + L.vx;
    h.vy = d->base + L.vy;
    h.Tb = (const double *)(d->base + L.Tb);
    h.Tb_alt = (const double *)(d->base + L.Tba);
    h.gbot = (const double *)(d->base + L.gb);
    h.gtop = (const double *)(d->base + L.gt);
    h.err = (int32_t *)(d->base + L.err);
    h.flux = (double *)(d->base + L.flux);
    h.sink = (double *)(d->base + L.sink);
    h.fl_every = 1;
    h.a = cfg->a;
    h.b = cfg->b;
    h.R = cfg->R;
    h.kappa = 0.37464 + 1.54226 * cfg->omega - 0.26992 * cfg->omega * cfg->omega;   // Eq. 13
    h.Tc = cfg->Tc;
    h.sqrtTc = std::sqrt(cfg->Tc);
    h.inv_sqrtTc = 1.0 / h.sqrtTc;
    h.G = cfg->G;
    h.invG = 1.0 / cfg->G;
    h.s_e = cfg->s_e;
    h.s_q = cfg->s_q;
    h.varpi = cfg->varpi;
    h.tau_V = cfg->tau_V;
    h.rho_V = cfg->rho_V;
    h.ktau = (cfg->tau_L - cfg->tau_V) / (cfg->rho_L - cfg->rho_V);                    // Eq. 5
    h.g = cfg->g;
    h.Cv = cfg->Cv;
    h.Cvchi = cfg->Cvchi;
    h.rho_S = cfg->rho_S;
    h.C_S = cfg->C_S;
    h.lambda_S = cfg->lambda_S;
    h.eos_s0 = 1.0 + h.kappa;
    h.eos_s1 = h.kappa * h.inv_sqrtTc;
    h.two_invG = 2.0 * h.invG;
    h.cw_k = 12.0 * cfg->varpi * cfg->s_e;
    h.hse = 1.0 - 0.5 * cfg->s_e;
    h.hsq = 1.0 - 0.5 * cfg->s_q;
    h.s2sign = (cfg->flags & PB_SBAR2_PLUS) ? 1.0 : -1.0;
    d->ddesc = (PbDesc *)(d->base + L.desc);
    d->dptr = (PbDesc **)(d->base + L.dptr);
    d->dtiles_flow = (PbTile *)(d->base + L.tflow);
    d->dtiles_th = (PbTile *)(d->base + L.tth);
    auto cleanup = [&](int code) {
        if (d->owns) (void)hipFree(d->base);
        delete d;
        return code;
    };
    // zero the whole state once (fields, boundary arrays, flags, accumulators)
    if (hipMemsetAsync(d->base, 0, L.total, d->stream) != hipSuccess) return cleanup(fail(PB_EDEVICE, "memset failed"));
    if (hipMemcpyAsync(d->dptr, &d->ddesc, sizeof(void *), hipMemcpyHostToDevice, d->stream) != hipSuccess)
        return cleanup(fail(PB_EDEVICE, "descriptor pointer upload failed"));
    if ((rc = upload_tiles(d))) return cleanup(rc);
    if ((rc = upload_desc(d))) return cleanup(rc);
    *out = d;
    return PB_OK;
}

void pb_destroy_domain(pb_domain *d) {
    if (!d) return;
    (void)hipStreamSynchronize(d->stream);
    for (hipEvent_t e : d->prof_ev) (void)hipEventDestroy(e);
    if (d->rd) (void)hipFree(d->rd);
    if (d->owns) (void)hipFree(d->base);
    delete d;
}

int pb_set_bc(pb_domain *d, const pb_bc *bc) {
    int rc = check_dom(d);
    if (rc) return rc;
    if (!bc) return fail(PB_EINVAL, "bc is NULL");
    const bool pery = d->cfg.flags & PB_PERIODIC_Y;
    if (!pery && !bc->T_bottom) return fail(PB_EINVAL, "T_bottom is required with walls");
    const int nx = d->cfg.nx;
    d->Tb.assign(nx, bc->T_top);
    if (bc->T_bottom) d->Tb.assign(bc->T_bottom, bc->T_bottom + nx);
    d->Tba.clear();
    if (bc->T_bottom_alt) d->Tba.assign(bc->T_bottom_alt, bc->T_bottom_alt + nx);
    d->gb.assign(nx, 0.0);
    d->gt.assign(nx, 0.0);
    if (bc->gamma_bottom) d->gb.assign(bc->gamma_bottom, bc->gamma_bottom + nx);
    if (bc->gamma_top) d->gt.assign(bc->gamma_top, bc->gamma_top + nx);
    const std::vector<double> &alt = d->Tba.empty() ? d->Tb : d->Tba;
    PB_HIP(hipStreamSynchronize(d->stream));
    PB_HIP(hipMemcpyAsync((void *)d->hd.Tb, d->Tb.data(), nx * 8, hipMemcpyHostToDevice, d->stream));
    PB_HIP(hipMemcpyAsync((void *)d->hd.Tb_alt, alt.data(), nx * 8, hipMemcpyHostToDevice, d->stream));
    PB_HIP(hipMemcpyAsync((void *)d->hd.gbot, d->gb.data(), nx * 8, hipMemcpyHostToDevice, d->stream));
    PB_HIP(hipMemcpyAsync((void *)d->hd.gtop, d->gt.data(), nx * 8, hipMemcpyHostToDevice, d->stream));
    d->hd.T_top = bc->T_top;
    d->hd.alt_t0 = bc->T_bottom_alt ? bc->alt_t0 : 0;
    d->hd.alt_t1 = bc->T_bottom_alt ? bc->alt_t1 : 0;
    return upload_desc(d);
}

int pb_set_fields(pb_domain *d, const double *rho, const double *T) {
    int rc = check_dom(d);
    if (rc) return rc;
    if (!rho || !T) return fail(PB_EINVAL, "rho and T are required");
    const int nx = d->cfg.nx, nyf = d->cfg.ny_fluid;
    double sum = 0.0;
    for (size_t i = 0; i < (size_t)nx * nyf; ++i) {
        if (!(rho[i] > 0.0) || !std::isfinite(rho[i])) return fail(PB_EINVAL, "rho must be positive and finite");
        sum += rho[i];
    }
    std::vector<double> Th(T, T + (size_t)nx * d->nr);
    if (!(d->cfg.flags & PB_PERIODIC_Y))
        for (int x = 0; x < nx; ++x) Th[x] = bc_bottom(d, x, 0);
    UploadTmp tmp;
    if (!tmp.get(d, d->nr)) return fail(PB_ENOMEM, "upload staging allocation failed");
    PB_HIP(hipStreamSynchronize(d->stream));
    d->t = 0;
    d->par = 0;
    d->hd.rho_bar = sum / ((double)nx * nyf);
    // the FP64 densities go through T[1] as dense rows (nr >= nyf rows of
    // pitch >= nx), which k_init reads before T is uploaded behind it on the
    // same stream
    PB_HIP(hipMemcpyAsync(d->hd.T[1], rho, (size_t)nyf * nx * sizeof(double), hipMemcpyHostToDevice, d->stream));
    PB_HIP(hipMemsetAsync(d->hd.err, 0, sizeof(int32_t), d->stream));
    if ((rc = upload_desc(d))) return rc;
    PB_HIP(pb_launch_init(d->cfg.precision, d->ddesc, d->hd.T[1], d->stream));
    for (int b = 0; b < 2; ++b)
        if ((rc = upload_rows(d, d->hd.T[b], Th.data(), d->nr, 8, tmp.p))) return rc;
    PB_HIP(hipStreamSynchronize(d->stream));
    d->fields_set = true;
    return PB_OK;
}

int pb_set_fields_full(pb_domain *d, const double *f, const double *T, int64_t t, double rho_bar) {
    int rc = check_dom(d);
    if (rc) return rc;
    if (!f || !T) return fail(PB_EINVAL, "f and T are required");
    if (d->cfg.flags & PB_FROZEN_FLOW) return fail(PB_EINVAL, "full state upload is not supported with PB_FROZEN_FLOW");
    if (t < 0) return fail(PB_EINVAL, "t must be >= 0");
    const int nx = d->cfg.nx, nyf = d->cfg.ny_fluid;
    const bool pery = d->cfg.flags & PB_PERIODIC_Y;
    const size_t np = (size_t)nx * nyf;
    // Undo the streaming: slot (i, y) is pulled by y + e_i as f_i, or, when
    // y + e_i is a wall, by y itself as f_opp(i) (bounce-back).
    std::vector<double> fs(9 * np), rref(np, 0.0);
    for (int y = 0; y < nyf; ++y)
        for (int x = 0; x < nx; ++x)
            for (int i = 0; i < 9; ++i) {
                const int xd = (x + kEXh[i] + nx) % nx;
                int yd = y + kEYh[i];
                double v;
                if (pery) yd = (yd + nyf) % nyf;
                if (yd >= 0 && yd < nyf) v = f[(size_t)i * np + (size_t)yd * nx + xd];
                else v = f[(size_t)kOPPh[i] * np + (size_t)y * nx + x];
                fs[(size_t)i * np + (size_t)y * nx + x] = v;
            }
    for (size_t n = 0; n < np; ++n) {
        double s = 0.0;
        for (int i = 0; i < 9; ++i) s += fs[(size_t)i * np + n];
        rref[n] = s;
    }
    UploadTmp tmp;
    if (!tmp.get(d, d->nr)) return fail(PB_ENOMEM, "upload staging allocation failed");
    PB_HIP(hipStreamSynchronize(d->stream));
    const int par = 0;
    if (d->cfg.precision == PB_FP64) {
        for (int i = 0; i < 9; ++i)
            if ((rc = upload_rows(d, (double *)d->hd.f[par] + (size_t)i * nyf * d->pitch, fs.data() + (size_t)i * np,
                                  nyf, 8, tmp.p)))
                return rc;
        if ((rc = upload_rows(d, d->hd.rho[par], rref.data(), nyf, 8, tmp.p))) return rc;
    } else {
        // deviations against the density as stored (FP32)
        std::vector<float> dev(9 * np), r32(np);
        for (size_t n = 0; n < np; ++n) r32[n] = (float)rref[n];
        for (int i = 0; i < 9; ++i)
            for (size_t n = 0; n < np; ++n)
                dev[(size_t)i * np + n] = (float)(fs[(size_t)i * np + n] - kWh[i] * (double)r32[n]);
        for (int i = 0; i < 9; ++i)
            if ((rc = upload_rows(d, (float *)d->hd.f[par] + (size_t)i * nyf * d->pitch, dev.data() + (size_t)i * np,
                                  nyf, 4, tmp.p)))
                return rc;
        if ((rc = upload_rows(d, d->hd.rho[par], r32.data(), nyf, 4, tmp.p))) return rc;
        PB_HIP(hipStreamSynchronize(d->stream));
    }
    for (int b = 0; b < 2; ++b)
        if ((rc = upload_rows(d, d->hd.T[b], T, d->nr, 8, tmp.p))) return rc;
    PB_HIP(hipMemsetAsync(d->hd.err, 0, sizeof(int32_t), d->stream));
    d->t = t;
    d->par = par;
    d->hd.rho_bar = rho_bar;
    if ((rc = upload_desc(d))) return rc;
    d->fields_set = true;
    return PB_OK;
}

int pb_step(pb_domain *d, int64_t n) {
    int rc = check_dom(d);
    if (rc) return rc;
    if (!d->fields_set) return fail(PB_ESTATE, "pb_set_fields was not called");
    if (n < 0) return fail(PB_EINVAL, "n must be >= 0");
    if (n == 0) return PB_OK;
    return enqueue_steps(d, n);
}

int pb_sync(pb_domain *d) {
    int rc = check_dom(d);
    if (rc) return rc;
    PB_HIP(hipStreamSynchronize(d->stream));
    int32_t e = 0;
    PB_HIP(hipMemcpy(&e, d->hd.err, sizeof(e), hipMemcpyDeviceToHost));
    if (e) return fail(PB_ENONFINITE, "non-finite value or negative psi radicand (t <= %lld)", (long long)d->t);
    return PB_OK;
}

}  // extern "C"

namespace {

// Doubles of read-back staging a domain needs: 12 dense [ny_fluid][nx]
// planes and T's nr = ny_fluid + ny_solid dense rows.
size_t read_stage_doubles(const pb_domain *d) {
    return (12 * (size_t)d->cfg.ny_fluid + (size_t)d->nr) * (size_t)d->cfg.nx;
}

// Read-back through FP64 staging at `stage` (read_stage_doubles(d)): dense
// [ny_fluid][nx] planes f_0..f_8, rho, v_x, v_y, which the flow kernel in
// read mode fills with f(t) rebuilt and rho(t), v(t), then T(t) re-pitched
// into dense rows behind them; each field goes to the host in one copy.
int read_through(pb_domain *d, double *stage, double *rho, double *ux, double *uy, double *T, double *f) {
    const int nyf = d->cfg.ny_fluid;
    const size_t nfd = (size_t)nyf * d->cfg.nx, bytes = nfd * sizeof(double);
    int rc;
    if (d->hd.rd_f != stage) {
        d->hd.rd_f = stage;
        d->hd.rd_rho = stage + 9 * nfd;
        d->hd.rd_vx = stage + 10 * nfd;
        d->hd.rd_vy = stage + 11 * nfd;
        if ((rc = upload_desc(d))) return rc;
    }
    if (rho || ux || uy || f) {
        PB_HIP(pb_launch_flow(d->cfg.precision, PB_MODE_READ, d->flow_launch_var, (const PbDesc *const *)d->dptr, d->dtiles_flow,
                              d->nt_flow, d->nt_flow, 0, d->stream));
    }
    if (rho) PB_HIP(hipMemcpyAsync(rho, d->hd.rd_rho, bytes, hipMemcpyDeviceToHost, d->stream));
    if (ux) PB_HIP(hipMemcpyAsync(ux, d->hd.rd_vx, bytes, hipMemcpyDeviceToHost, d->stream));
    if (uy) PB_HIP(hipMemcpyAsync(uy, d->hd.rd_vy, bytes, hipMemcpyDeviceToHost, d->stream));
    if (T && (rc = download_rows(d, T, d->hd.T[d->par], d->nr, stage + 12 * nfd))) return rc;
    if (f) PB_HIP(hipMemcpyAsync(f, d->hd.rd_f, 9 * bytes, hipMemcpyDeviceToHost, d->stream));
    PB_HIP(hipStreamSynchronize(d->stream));
    return PB_OK;
}

}  // namespace

extern "C" {

int pb_read_fields(pb_domain *d, double *rho, double *ux, double *uy, double *T, double *f) {
    int rc = check_dom(d);
    if (rc) return rc;
    if (!d->fields_set) return fail(PB_ESTATE, "pb_set_fields was not called");
    PB_HIP(hipStreamSynchronize(d->stream));
    if (!d->rd && hipMalloc((void **)&d->rd, read_stage_doubles(d) * sizeof(double)) != hipSuccess)
        return fail(PB_ENOMEM, "read staging allocation failed");
    return read_through(d, d->rd, rho, ux, uy, T, f);
}

int pb_read_fields_noalloc(pb_domain *d, double *rho, double *ux, double *uy, double *T, double *f) {
    int rc = check_dom(d);
    if (rc) return rc;
    if (!d->fields_set) return fail(PB_ESTATE, "pb_set_fields was not called");
    const size_t need = read_stage_doubles(d) * sizeof(double);
    if (need > PB_SCRATCH_BYTES)
        return fail(PB_EINVAL,
                    "read-back staging of %zu bytes exceeds the fixed %zu bytes ((13 * ny_fluid + ny_solid) * nx <= %zu)",
                    need, (size_t)PB_SCRATCH_BYTES, (size_t)PB_SCRATCH_BYTES / sizeof(double));
    int cur = 0;
    PB_HIP(hipGetDevice(&cur));
    if (cur != d->device) PB_HIP(hipSetDevice(d->device));
    void *stage = nullptr;
    size_t cap = 0;
    hipError_t e = pb_scratch_address(&stage, &cap);
    if (cur != d->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return fail(PB_EDEVICE, "staging address lookup failed: %s", hipGetErrorString(e));
    PB_HIP(hipStreamSynchronize(d->stream));
    return read_through(d, (double *)stage, rho, ux, uy, T, f);
}

int pb_flux_window(pb_domain *d, int64_t t_a, int64_t t_b, int32_t every) {
    int rc = check_dom(d);
    if (rc) return rc;
    if (every < 1) return fail(PB_EINVAL, "every must be >= 1");
    PB_HIP(hipStreamSynchronize(d->stream));
    const double zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    PB_HIP(hipMemcpyAsync(d->hd.flux, zero, sizeof(zero), hipMemcpyHostToDevice, d->stream));
    d->hd.fl_ta = t_a;
    d->hd.fl_tb = t_b;
    d->hd.fl_every = every;
    return upload_desc(d);
}

int pb_heat_flux(pb_domain *d, pb_flux *out) {
    int rc = check_dom(d);
    if (rc) return rc;
    if (!out) return fail(PB_EINVAL, "out is NULL");
    double v[8];
    PB_HIP(hipStreamSynchronize(d->stream));
    PB_HIP(hipMemcpy(v, d->hd.flux, sizeof(v), hipMemcpyDeviceToHost));
    const double n = v[6];
    out->q_bottom_inst = v[0];
    out->q_top_inst = v[1];
    out->T_w_inst = v[2];
    out->q_bottom_mean = n > 0 ? v[3] / n : 0.0;
    out->q_top_mean = n > 0 ? v[4] / n : 0.0;
    out->T_w_mean = n > 0 ? v[5] / n : 0.0;
    out->n_samples = (int64_t)n;
    return PB_OK;
}

int pb_profile_reserve(pb_domain *d, int64_t n) {
    int rc = check_dom(d);
    if (rc) return rc;
    if (n < 1 || n > (1 << 20)) return fail(PB_EINVAL, "n must be in [1, 2^20]");
    while (d->prof_ev.size() < 2 * (size_t)n + 1) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return fail(PB_EDEVICE, "event creation failed");
        d->prof_ev.push_back(e);
    }
    return PB_OK;
}

int pb_profile_steps(pb_domain *d, int64_t n, double *avg_ms) {
    int rc = check_dom(d);
    if (rc) return rc;
    if (!d->fields_set) return fail(PB_ESTATE, "pb_set_fields was not called");
    if (!avg_ms) return fail(PB_EINVAL, "avg_ms is NULL");
    if (n < 1 || n > (1 << 20)) return fail(PB_EINVAL, "n must be in [1, 2^20]");
    if ((rc = pb_profile_reserve(d, n))) return rc;
    const bool frozen = d->cfg.flags & PB_FROZEN_FLOW, iso = d->cfg.flags & PB_ISOTHERMAL;
    const bool sampling = !(d->cfg.flags & PB_PERIODIC_Y) && d->cfg.ny_solid >= 1 && d->hd.fl_tb > d->hd.fl_ta;
    const PbDesc *const *dp = (const PbDesc *const *)d->dptr;
    const int m = (int)n;
    // events e[2k] before the flow launch of step k, e[2k+1] between flow and
    // thermal, e[2k+2] after the thermal launch
    const std::vector<hipEvent_t> &ev = d->prof_ev;
    hipError_t err = hipSuccess;
    for (int k = 0; k < m && err == hipSuccess; ++k) {
        err = hipEventRecord(ev[2 * k], d->stream);
        if (err == hipSuccess && !frozen)
            err = pb_launch_flow(d->cfg.precision, PB_MODE_STEP, d->flow_launch_var, dp, d->dtiles_flow, d->nt_flow, d->nt_flow, k,
                                 d->stream);
        if (err == hipSuccess) err = hipEventRecord(ev[2 * k + 1], d->stream);
        if (err == hipSuccess && !iso) err = pb_launch_thermal(d->cfg.precision, d->tvar, dp, d->dtiles_th, d->nt_th, d->nt_th, k, d->stream);
        const int64_t tk = d->t + k + 1;
        if (err == hipSuccess && sampling && tk >= d->hd.fl_ta && tk < d->hd.fl_tb &&
            (tk - d->hd.fl_ta) % d->hd.fl_every == 0)
            err = pb_launch_flux(d->cfg.precision, dp, 1, k, d->stream);
    }
    if (err == hipSuccess) err = hipEventRecord(ev[2 * m], d->stream);
    if (err == hipSuccess) err = pb_launch_advance(d->dptr, 1, m, d->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(d->stream);
    if (err != hipSuccess) return fail(PB_EDEVICE, "profiled steps failed: %s", hipGetErrorString(err));
    d->t += m;
    d->par ^= (m & 1);
    d->hd.t0 = d->t;
    d->hd.par0 = d->par;
    double sf = 0.0, st = 0.0;
    float ms;
    for (int k = 0; k < m; ++k) {
        (void)hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]);
        sf += ms;
        (void)hipEventElapsedTime(&ms, ev[2 * k + 1], ev[2 * k + 2]);
        st += ms;
    }
    (void)hipEventElapsedTime(&ms, ev[0], ev[2 * m]);
    avg_ms[0] = sf / m;
    avg_ms[1] = st / m;
    avg_ms[2] = (double)ms / m;
    return PB_OK;
}

int64_t pb_time(const pb_domain *d) { return d ? d->t : -1; }
double pb_rho_bar(const pb_domain *d) { return d ? d->hd.rho_bar : 0.0; }

// ------------------------------------------------------------------ batches
namespace {

// Release what a membership change replaced, once the work queued before the
// change has finished (all = true: wait for it; used when the batch goes).
void batch_reap(pb_batch *b, bool all) {
    std::vector<pb_batch::Retired> keep;
    for (pb_batch::Retired &r : b->retired) {
        if (!all && hipEventQuery(r.done) != hipSuccess) {
            keep.push_back(r);
            continue;
        }
        if (all) (void)hipEventSynchronize(r.done);
        if (r.exec) (void)hipGraphExecDestroy(r.exec);
        if (r.graph) (void)hipGraphDestroy(r.graph);
        if (r.tab) (void)hipFree(r.tab);
        (void)hipEventDestroy(r.done);
    }
    b->retired.swap(keep);
}

// Retire the captured step graph and, if given, a table buffer: they stay
// alive until the work already queued on the batch stream has run.
int batch_retire(pb_batch *b, char *tab) {
    if (!b->gexec && !tab) return PB_OK;
    pb_batch::Retired r{b->gexec, b->graph, tab, nullptr};
    b->gexec = nullptr;
    b->graph = nullptr;
    if (hipEventCreateWithFlags(&r.done, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(r.done, b->stream) != hipSuccess) {
        // cannot order the release: wait for the batch instead
        (void)hipStreamSynchronize(b->stream);
        if (r.done) (void)hipEventDestroy(r.done);
        if (r.exec) (void)hipGraphExecDestroy(r.exec);
        if (r.graph) (void)hipGraphDestroy(r.graph);
        if (r.tab) (void)hipFree(r.tab);
        return PB_OK;
    }
    b->retired.push_back(r);
    return PB_OK;
}

// Work lists and descriptor table of the current members, uploaded on the
// batch stream (ordered after the steps already queued, which keep reading
// the previous contents); the captured step graph is dropped, to be captured
// again at the next graph-length step.  No member stream is synchronised.
int batch_rebuild(pb_batch *b) {
    const int n = (int)b->doms.size();
    std::vector<PbTile> tf, tt;
    std::vector<PbDesc *> ptrs(n);
    int prec = b->prec, fvar = b->fvar, tvar = b->tvar;
    bool flow_alt = false;
    if (n > 0) {
        prec = b->doms[0]->cfg.precision;
        fvar = b->doms[0]->fvar;
        std::vector<const pb_config *> cfgs(n);
        for (int j = 0; j < n; ++j) cfgs[j] = &b->doms[j]->cfg;
        tvar = launch_thermal_variant(cfgs);
        // a launch's work-list holds the tiles of the domains that take that
        // part of the step (frozen-flow domains skip the flow, isothermal ones
        // the energy equation, as when stepped alone)
        for (int j = 0; j < n; ++j) {
            if (!(b->doms[j]->cfg.flags & PB_FROZEN_FLOW))
                if (make_flow_tiles(tf, j, b->doms[j]->cfg.nx, b->doms[j]->cfg.ny_fluid, prec, fvar)) flow_alt = true;
            ptrs[j] = b->doms[j]->ddesc;
        }
        thermal_list(tt, cfgs, tvar, b->persistent == 0);
        if (b->persistent == 0) xcd_order(tf);
    }
    const size_t o_tf = align_up((size_t)std::max(n, 1) * sizeof(PbDesc *), kAlign);
    const size_t o_tt = o_tf + align_up(std::max<size_t>(1, tf.size()) * sizeof(PbTile), kAlign);
    const size_t total = o_tt + align_up(std::max<size_t>(1, tt.size()) * sizeof(PbTile), kAlign);
    // the staging copy is rewritten only after its previous upload has read it
    const int hs = b->hslot ^ 1;
    if (b->upload_pending[hs]) {
        PB_HIP(hipEventSynchronize(b->ev_upload[hs]));
        b->upload_pending[hs] = false;
    }
    if (total > b->htab_cap[hs]) {
        if (b->htab[hs]) PB_HIP(hipHostFree(b->htab[hs]));
        b->htab[hs] = nullptr;
        b->htab_cap[hs] = 0;
        if (hipHostMalloc((void **)&b->htab[hs], 2 * total, hipHostMallocDefault) != hipSuccess)
            return fail(PB_ENOMEM, "pinned staging of %zu bytes failed", 2 * total);
        b->htab_cap[hs] = 2 * total;
    }
    char *const stage = b->htab[hs];
    char *old_tab = nullptr;
    if (total > b->tab_cap) {
        char *t = nullptr;
        if (hipMalloc((void **)&t, 2 * total) != hipSuccess)
            return fail(PB_ENOMEM, "batch tables allocation of %zu bytes failed", 2 * total);
        old_tab = b->dtab;
        b->dtab = t;
        b->tab_cap = 2 * total;
    }
    memcpy(stage, ptrs.data(), (size_t)n * sizeof(PbDesc *));
    memcpy(stage + o_tf, tf.data(), tf.size() * sizeof(PbTile));
    memcpy(stage + o_tt, tt.data(), tt.size() * sizeof(PbTile));
    // what was captured or queued before reads the previous tables (and
    // buffer): retire them behind that work
    int rc = batch_retire(b, old_tab);
    if (rc) return rc;
    PB_HIP(hipMemcpyAsync(b->dtab, stage, total, hipMemcpyHostToDevice, b->stream));
    PB_HIP(hipEventRecord(b->ev_upload[hs], b->stream));
    b->upload_pending[hs] = true;
    b->hslot = hs;
    b->dptrs = (PbDesc **)b->dtab;
    b->dtiles_flow = (PbTile *)(b->dtab + o_tf);
    b->dtiles_th = (PbTile *)(b->dtab + o_tt);
    b->prec = prec;
    b->fvar = fvar;
    b->flow_launch_var = fvar | (flow_alt ? PB_FLOW_ALT_TILES : 0);
    b->tvar = tvar;
    b->nt_flow = (int)tf.size();
    b->nt_th = (int)tt.size();
    b->grid_flow = b->persistent > 0 ? std::min(b->nt_flow, b->persistent) : b->nt_flow;
    b->grid_th = b->persistent > 0 ? std::min(b->nt_th, b->persistent) : b->nt_th;
    b->dom_streams.clear();
    for (pb_domain *d : b->doms)
        if (std::find(b->dom_streams.begin(), b->dom_streams.end(), d->stream) == b->dom_streams.end())
            b->dom_streams.push_back(d->stream);
    batch_reap(b, false);
    return PB_OK;
}

int check_member(const pb_batch *b, const pb_domain *d) {
    if (!d) return fail(PB_EINVAL, "domain is NULL");
    if (!d->fields_set) return fail(PB_ESTATE, "domain has no fields");
    if (!b->doms.empty() && d->cfg.precision != b->doms[0]->cfg.precision)
        return fail(PB_EINVAL, "mixed precisions in one batch");
    if (std::find(b->doms.begin(), b->doms.end(), d) != b->doms.end()) return fail(PB_EINVAL, "domain listed twice");
    return PB_OK;
}

}  // namespace

int pb_batch_create(pb_domain *const *doms, int32_t n, int32_t steps_per_graph, int32_t persistent_blocks, void *stream,
                    pb_batch **out) {
    if (!out) return fail(PB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!doms || n < 1) return fail(PB_EINVAL, "need at least one domain");
    if (steps_per_graph < 0 || (steps_per_graph & 1)) return fail(PB_EINVAL, "steps_per_graph must be even and >= 0");
    if (persistent_blocks < 0) return fail(PB_EINVAL, "persistent_blocks must be >= 0");
    pb_batch *b = new (std::nothrow) pb_batch();
    if (!b) return fail(PB_ENOMEM, "host allocation failed");
    for (int j = 0; j < n; ++j) {
        int rc = check_member(b, doms[j]);
        if (rc) {
            delete b;
            return rc;
        }
        b->doms.push_back(doms[j]);
    }
    b->stream = (hipStream_t)stream;
    b->spg = steps_per_graph;
    b->persistent = persistent_blocks;
    // graphs cannot be captured on the legacy null stream: use an own stream,
    // ordered against the members' streams with events in pb_batch_step
    int rc = PB_OK;
    if (!b->stream) {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
            rc = fail(PB_EDEVICE, "stream creation failed");
        else
            b->owns_stream = true;
    }
    if (!rc && (hipEventCreateWithFlags(&b->ev_batch, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&b->ev_dom, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&b->ev_upload[0], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&b->ev_upload[1], hipEventDisableTiming) != hipSuccess))
        rc = fail(PB_EDEVICE, "event creation failed");
    if (!rc) rc = batch_rebuild(b);
    if (rc) {
        pb_batch_destroy(b);
        return rc;
    }
    *out = b;
    return PB_OK;
}

int pb_batch_add(pb_batch *b, pb_domain *d) {
    if (!b) return fail(PB_EINVAL, "batch is NULL");
    int rc = check_member(b, d);
    if (rc) return rc;
    b->doms.push_back(d);
    if ((rc = batch_rebuild(b))) {
        b->doms.pop_back();
        return rc;
    }
    return PB_OK;
}

int pb_batch_remove(pb_batch *b, pb_domain *d) {
    if (!b) return fail(PB_EINVAL, "batch is NULL");
    auto it = std::find(b->doms.begin(), b->doms.end(), d);
    if (!d || it == b->doms.end()) return fail(PB_EINVAL, "domain is not a member of the batch");
    const size_t at = (size_t)(it - b->doms.begin());
    b->doms.erase(it);
    int rc = batch_rebuild(b);
    if (rc) {
        b->doms.insert(b->doms.begin() + at, d);
        return rc;
    }
    return PB_OK;
}

int32_t pb_batch_size(const pb_batch *b) { return b ? (int32_t)b->doms.size() : -1; }

// Which of the next nsteps steps (step k ends at t + k + 1) some member
// samples for the heat flux.  The flux kernel checks each domain's window and
// period itself, so a launch where none samples only costs its dispatch; a
// missing one would lose samples.  For a captured graph (periodic = true)
// the steps must hold for every replay, which holds when the graph length is
// a multiple of each period; else every step launches.
static std::vector<char> batch_flux_steps(const pb_batch *b, int nsteps, bool periodic) {
    std::vector<char> need(nsteps, 0);
    for (const pb_domain *d : b->doms) {
        if (!(d->hd.fl_tb > d->hd.fl_ta && d->cfg.ny_solid >= 1)) continue;
        const int64_t e = std::max<int64_t>(1, d->hd.fl_every);
        if (periodic && nsteps % e != 0) return std::vector<char>(nsteps, 1);
        for (int k = 0; k < nsteps; ++k) {
            const int64_t r = (d->t + k + 1 - d->hd.fl_ta) % e;
            if (r == 0) need[k] = 1;
        }
    }
    return need;
}

static int batch_enqueue(pb_batch *b, int nsteps, const std::vector<char> &flux) {
    const PbDesc *const *dp = (const PbDesc *const *)b->dptrs;
    const int nd = (int)b->doms.size();
    for (int k = 0; k < nsteps; ++k) {
        if (b->nt_flow > 0)
            PB_HIP(pb_launch_flow(b->prec, PB_MODE_STEP, b->flow_launch_var, dp, b->dtiles_flow, b->nt_flow, b->grid_flow, k,
                                  b->stream));
        if (b->nt_th > 0)
            PB_HIP(pb_launch_thermal(b->prec, b->tvar, dp, b->dtiles_th, b->nt_th, b->grid_th, k, b->stream));
        if (flux[k]) PB_HIP(pb_launch_flux(b->prec, dp, nd, k, b->stream));
    }
    PB_HIP(pb_launch_advance(b->dptrs, nd, nsteps, b->stream));
    return PB_OK;
}

int pb_batch_step(pb_batch *b, int64_t n) {
    if (!b) return fail(PB_EINVAL, "batch is NULL");
    if (n < 0) return fail(PB_EINVAL, "n must be >= 0");
    if (b->doms.empty() || n == 0) return PB_OK;
    int rc;
    // the batch stream starts after the work already queued on member streams
    for (hipStream_t s : b->dom_streams) {
        if (s == b->stream) continue;
        PB_HIP(hipEventRecord(b->ev_dom, s));
        PB_HIP(hipStreamWaitEvent(b->stream, b->ev_dom, 0));
    }
    while (n > 0) {
        if (b->spg > 0 && n >= b->spg) {
            // a member's flux window or phase changed since the capture: capture again
            const std::vector<char> flux = batch_flux_steps(b, b->spg, true);
            if (b->gexec && flux != b->graph_flux) {
                if ((rc = batch_retire(b, nullptr))) return rc;
            }
            if (!b->gexec) {
                PB_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
                rc = batch_enqueue(b, b->spg, flux);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(b->stream, &g);
                if (rc) {
                    if (g) (void)hipGraphDestroy(g);
                    return rc;
                }
                if (e != hipSuccess) return fail(PB_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
                b->graph = g;
                b->graph_flux = flux;
                PB_HIP(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
            }
            PB_HIP(hipGraphLaunch(b->gexec, b->stream));
            for (pb_domain *d : b->doms) {
                d->t += b->spg;
                d->par ^= (b->spg & 1);
                d->hd.t0 = d->t;
                d->hd.par0 = d->par;
            }
            n -= b->spg;
        } else {
            const int m = (int)std::min<int64_t>(n, 1 << 20);
            if ((rc = batch_enqueue(b, m, batch_flux_steps(b, m, false)))) return rc;
            for (pb_domain *d : b->doms) {
                d->t += m;
                d->par ^= (m & 1);
                d->hd.t0 = d->t;
                d->hd.par0 = d->par;
            }
            n -= m;
        }
    }
    // later work on the members' streams (reads, syncs, steps) waits for the batch
    PB_HIP(hipEventRecord(b->ev_batch, b->stream));
    for (hipStream_t s : b->dom_streams)
        if (s != b->stream) PB_HIP(hipStreamWaitEvent(s, b->ev_batch, 0));
    return PB_OK;
}

void pb_batch_destroy(pb_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    batch_reap(b, true);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev_batch) (void)hipEventDestroy(b->ev_batch);
    if (b->ev_dom) (void)hipEventDestroy(b->ev_dom);
    for (int h = 0; h < 2; ++h)
        if (b->ev_upload[h]) (void)hipEventDestroy(b->ev_upload[h]);
    if (b->owns_stream) (void)hipStreamDestroy(b->stream);
    if (b->dtab) (void)hipFree(b->dtab);
    for (int h = 0; h < 2; ++h)
        if (b->htab[h]) (void)hipHostFree(b->htab[h]);
    delete b;
}

// --------------------------------------------------------- host EOS helpers
int pb_eos_critical_temperature(double a, double b, double R, double *Tc) {
    if (!Tc || !(a > 0) || !(b > 0) || !(R > 0)) return fail(PB_EINVAL, "need a, b, R > 0 and an output");
    // a = 0.45724 R^2 Tc^2 / Pc and b = 0.0778 R Tc / Pc  =>  a / b = (0.45724/0.0778) R Tc
    *Tc = (a / b) * 0.0778 / (0.45724 * R);
    return PB_OK;
}

// Maxwell pair by Newton iteration on (v_L, v_V): equal pressure and equal
// area (the integral of P dv between the two volumes equals P (v_V - v_L)),
// started from the roots of P = (P_max + P_min)/2 between the spinodals.
int pb_eos_coexistence(double a, double b, double R, double omega, double Tc, double T, double *rho_L, double *rho_V) {
    if (!rho_L || !rho_V) return fail(PB_EINVAL, "outputs are NULL");
    if (!(T > 0) || !(T < Tc) || !(a > 0) || !(b > 0) || !(R > 0)) return fail(PB_EINVAL, "need 0 < T < Tc and a, b, R > 0");
    const double kap = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
    const double s = 1.0 + kap * (1.0 - std::sqrt(T / Tc));
    const double A = a * s * s, r2 = std::sqrt(2.0);
    // in specific volume v = 1/rho: P = R T/(v - b) - A/(v^2 + 2 b v - b^2)
    auto P = [&](double v) { return R * T / (v - b) - A / (v * v + 2.0 * b * v - b * b); };
    auto dP = [&](double v) {
        const double q = v * v + 2.0 * b * v - b * b;
        return -R * T / ((v - b) * (v - b)) + A * (2.0 * v + 2.0 * b) / (q * q);
    };
    auto I = [&](double v) {   // antiderivative of P dv
        return R * T * std::log(v - b) - A / (2.0 * r2 * b) * std::log((v + b - r2 * b) / (v + b + r2 * b));
    };
    // spinodals: scan dP on a log grid of v
    const int N = 4000;
    double vmin_sp = 0, vmax_sp = 0;
    double prev = dP(b * 1.0001);
    bool got1 = false;
    for (int k = 1; k <= N; ++k) {
        const double v = b * std::exp(std::log(1.0001) + k * (std::log(1e4) / N));
        const double cur = dP(v);
        if (!got1 && prev < 0 && cur >= 0) { vmin_sp = v; got1 = true; }
        else if (got1 && prev > 0 && cur <= 0) { vmax_sp = v; break; }
        prev = cur;
    }
    if (!got1 || vmax_sp == 0) return fail(PB_EINVAL, "no two-phase region at this temperature");
    // vmin_sp: liquid spinodal (local minimum of P), vmax_sp: vapour spinodal (local maximum)
    const double pm = 0.5 * (std::max(P(vmin_sp), 0.0) + P(vmax_sp));
    auto root = [&](double lo, double hi) {   // P(v) = pm on a monotone bracket
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if ((P(mid) - pm) * (P(lo) - pm) > 0) lo = mid; else hi = mid;
        }
        return 0.5 * (lo + hi);
    };
    double vl = root(b * 1.0001, vmin_sp);
    double vv = root(vmax_sp, b * 1e5);
    for (int it = 0; it < 100; ++it) {
        const double F1 = P(vl) - P(vv);
        const double F2 = I(vv) - I(vl) - P(vl) * (vv - vl);
        const double J11 = dP(vl), J12 = -dP(vv);
        const double J21 = -dP(vl) * (vv - vl), J22 = P(vv) - P(vl);
        const double det = J11 * J22 - J12 * J21;
        if (det == 0.0) break;
        const double dl = (F1 * J22 - J12 * F2) / det, dv = (J11 * F2 - J21 * F1) / det;
        vl -= dl;
        vv -= dv;
        if (std::fabs(dl) < 1e-15 * vl && std::fabs(dv) < 1e-15 * vv) break;
    }
    if (!(vl > b) || !(vv > vl)) return fail(PB_EINVAL, "coexistence iteration failed");
    *rho_L = 1.0 / vl;
    *rho_V = 1.0 / vv;
    return PB_OK;
}

int pb_eos_latent_heat(double a, double b, double R, double omega, double Tc, double T, double *h_fg) {
    if (!h_fg) return fail(PB_EINVAL, "output is NULL");
    const double kap = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
    auto psat = [&](double TT, double *rl, double *rv) -> int {
        return pb_eos_coexistence(a, b, R, omega, Tc, TT, rl, rv);
    };
    auto pressure = [&](double TT, double r) {
        const double s = 1.0 + kap * (1.0 - std::sqrt(TT / Tc));
        return r * R * TT / (1.0 - b * r) - a * s * s * r * r / (1.0 + 2.0 * b * r - b * b * r * r);
    };
    double rl, rv, rl1, rv1, rl2, rv2;
    const double dT = 1e-5 * Tc;
    int rc;
    if ((rc = psat(T, &rl, &rv)) || (rc = psat(T + dT, &rl1, &rv1)) || (rc = psat(T - dT, &rl2, &rv2))) return rc;
    const double dPdT = (pressure(T + dT, rl1) - pressure(T - dT, rl2)) / (2.0 * dT);
    *h_fg = T * (1.0 / rv - 1.0 / rl) * dPdT;
    return PB_OK;
}

int pb_eos_psi(double a, double b, double R, double omega, double Tc, double G, double rho, double T, double *psi) {
    if (!psi || !(G < 0) || !(rho > 0) || !(T > 0) || !(Tc > 0) || !(rho * b < 1.0))
        return fail(PB_EINVAL, "need psi output, G < 0, 0 < rho < 1/b, T, Tc > 0");
    const double kap = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
    const double s = 1.0 + kap * (1.0 - std::sqrt(T / Tc));
    const double P = rho * R * T / (1.0 - b * rho) - a * s * s * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
    const double rad = 2.0 * (P - rho / 3.0) / G;
    if (!(rad >= 0.0)) return fail(PB_EINVAL, "negative psi radicand at rho = %g, T = %g", rho, T);
    *psi = std::sqrt(rad);
    return PB_OK;
}

}  // extern "C"
