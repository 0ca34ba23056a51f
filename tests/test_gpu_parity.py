"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances (max-norm relative error per field, err = max|X_gpu - X_orc| /
max|X_orc| over rho, T and f, and over u_x, u_y with the speed scale
max(|u_x|, |u_y|) as denominator): 1e-11 for FP64 storage and 2e-5 for
FP32-deviation storage, over a 200-step window; bit-identity where the
arithmetic per node is the same by construction (tile shape, batching,
checkpoint/resume in FP64).
"""
import numpy as np
import pytest

from paper_1911_10747_amd import workloads as W
from gpu_common import compare, gpu_domain, oracle_domain, pb_config, rel_err, run_pair
from helpers import params, pool_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")  # import at collection, outside per-test time limits

TOL = {0: 1e-11, 1: 2e-5}


def _report(name, errs):
    print(name, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)


@pytest.mark.parametrize("flag", ["varpi_fm_only", "sbar2_plus"])
@pytest.mark.parametrize("precision", [0, 1])
def test_printed_readings_of_eq9(flag, precision):
    """The two printed forms of Eq. 9 that this build reads otherwise, as
    flags on both sides: the varpi term with F_m of Eq. 11 alone
    (PB_VARPI_FM_ONLY) and with a + sign in row 2 (PB_SBAR2_PLUS).  The
    100x100 + 100x10 pool for 200 steps against the oracle with the same flag,
    and the flag changes the result (so it is in effect on both sides)."""
    P, d, bc, rho, T = pool_case(100, 100, 10, superheat=0.1, n_spots=4, seed=0, y0=40, **{flag: 1})
    g, o = run_pair(P, bc, rho, T, steps=200, precision=precision, window=(50, 201, 10))
    errs = compare(g, o)
    _report(f"{flag} prec={precision}", errs)
    assert all(v <= TOL[precision] for v in errs.values()), errs
    assert g["flux"]["q_bottom_mean"] == pytest.approx(o["flux"]["q_bottom_mean"], rel=TOL[precision] * 10)
    P0 = dict(P, **{flag: 0})
    o0 = oracle_domain(P0, bc, rho, T)
    o0.step(200)
    assert rel_err(o0.read()["f"], o["f"]) > 1e-6


@pytest.mark.parametrize("tile", [(0, 0), (64, 4)])
@pytest.mark.parametrize("precision", [0, 1])
def test_pool_boiling_100x100_200_steps(precision, tile):
    """Plain pool boiling, 100x100 fluid over a 100x10 heater, liquid below
    y = 40, heater bottom at Tsat + 0.1 Tc with 4 seeded +2% spots."""
    P, d, bc, rho, T = pool_case(100, 100, 10, superheat=0.1, n_spots=4, seed=0, y0=40)
    g, o = run_pair(P, bc, rho, T, steps=200, precision=precision, tile=tile, window=(50, 201, 10))
    errs = compare(g, o)
    _report(f"C0 prec={precision} tile={tile}", errs)
    assert all(v <= TOL[precision] for v in errs.values()), errs
    for k in ("q_bottom_mean", "q_top_mean", "T_w_mean", "q_bottom_inst"):
        assert g["flux"][k] == pytest.approx(o["flux"][k], rel=TOL[precision] * 10, abs=1e-15), k
    assert g["flux"]["n_samples"] == o["flux"]["n_samples"] == 16


@pytest.mark.parametrize("precision", [0, 1])
def test_ragged_domain_and_tile_shapes_are_bit_identical(precision):
    """77x45 fluid over 5 heater rows (ragged against every tile shape): the
    result matches the oracle and is bit-identical for every flow tile and
    every thermal variant (strip heights 8, 12, 16 and 20 have strips inside
    the fluid, which take the specialised path; 24, 28 and 36 have none)."""
    P, d, bc, rho, T = pool_case(77, 45, 5, superheat=0.2, n_spots=3, seed=7, y0=17)
    ref = None
    shapes = [(64, 4), (64, 8), (32, 8), (128, 4), (32, 16), (64, 16), (64, 4)]
    for i, tile in enumerate(shapes):
        g = gpu_domain(P, bc, rho, T, precision, tile=tile, thermal_tile=1 + i)
        g.step(120)
        g.sync()
        r = g.read()
        g.close()
        if ref is None:
            ref = r
            o = oracle_domain(P, bc, rho, T)
            o.step(120)
            errs = compare(r, o.read())
            _report(f"ragged precision={precision}", errs)
            assert all(v <= TOL[precision] for v in errs.values()), errs
        else:
            for k in ("rho", "ux", "uy", "T", "f"):
                np.testing.assert_array_equal(r[k], ref[k], err_msg=f"{k} differs for tile {tile}")


@pytest.mark.parametrize("nx", [67, 68, 69, 132])
def test_x_edge_tiles_around_the_wrap_limit(nx):
    """FP32 storage: tiles at the x edges and two rows from the walls take the
    LDS-decode path with x modulo nx when nx >= tile width + 4, else the
    general path.  Widths on both sides of that limit for 64- and 128-wide
    tiles, 80 steps: every tile shape matches the oracle and gives the same
    bits (the same node by either path)."""
    P, d, bc, rho, T = pool_case(nx, 40, 3, superheat=0.2, n_spots=3, seed=nx, y0=15)
    o = oracle_domain(P, bc, rho, T)
    o.step(80)
    orr = o.read()
    ref = None
    for tile in [(64, 8), (32, 8), (128, 4), (64, 16)]:
        g = gpu_domain(P, bc, rho, T, 1, tile=tile)
        g.step(80)
        g.sync()
        r = g.read()
        g.close()
        errs = compare(r, orr)
        _report(f"x-edge nx={nx} tile={tile}", errs)
        assert all(v <= TOL[1] for v in errs.values()), errs
        if ref is None:
            ref = r
        else:
            for k in ("rho", "ux", "uy", "T", "f"):
                np.testing.assert_array_equal(r[k], ref[k], err_msg=f"{k} differs for tile {tile}")


@pytest.mark.parametrize("precision,nx,nyf,nys", [(0, 3590, 1403, 56), (1, 4096, 1800, 64)])
def test_short_tail_strips_bit_identical(precision, nx, nyf, nys):
    """Domains with enough 28- or 36-row energy strips that the library ends
    the work list with 8-row strips (more than the 2048 / 3072 wavefront slots
    of the FP64 / FP32 sweep; ragged columns and a ragged top strip): 20 steps
    give the same bits as strips of 8 rows throughout (thermal_tile 6), which
    the ragged-domain test holds to the oracle."""
    from paper_1911_10747_amd import poolboil as pb
    P, d, bc, rho, T = pool_case(nx, nyf, nys, superheat=0.15, n_spots=nx // 64, seed=3, y0=int(0.4 * nyf))
    assert pb.thermal_strip_rows(pb_config(P, precision, (64, 8), 1)) == 28
    assert pb.thermal_strip_rows(pb_config(P, precision, (64, 8), 7)) == 36
    out = []
    for tt in (6, 1, 7):
        g = gpu_domain(P, bc, rho, T, precision, tile=(64, 8), thermal_tile=tt)
        g.step(20)
        g.sync()
        out.append(g.read(with_f=False))
        g.close()
    for k in ("rho", "ux", "uy", "T"):
        for j, tt in ((1, 1), (2, 7)):
            np.testing.assert_array_equal(out[j][k], out[0][k], err_msg=f"{k} differs for thermal_tile {tt}")


@pytest.mark.parametrize("tile,isothermal,precision", [((0, 0), 1, 0), ((32, 16), 1, 0), ((0, 0), 0, 0),
                                                       ((32, 16), 0, 0), ((0, 0), 0, 1)])
def test_periodic_drop(isothermal, tile, precision):
    """Fully periodic box with a drop (no walls, no heater): exercises the
    periodic wrap in y of streaming, forces and the thermal stencil."""
    nx, ny = 48, 40
    P, d = params(nx, ny, 0, periodic_y=1, isothermal=isothermal, g=0.0)
    rho = W.drop_rho(nx, ny, 9.0, d["rho_L"], d["rho_V"], width=3.0, cx=20.3, cy=17.6)
    T = W.perturbed(np.full((ny, nx), d["Tsat"]), 0.02, 11)
    bc = dict(T_top=d["Tsat"])
    g, o = run_pair(P, bc, rho, T, steps=200, precision=precision, tile=tile)
    errs = compare(g, o)
    _report(f"drop iso={isothermal} tile={tile} precision={precision}", errs)
    assert all(v <= TOL[precision] for v in errs.values()), errs


def test_frozen_flow_conduction():
    """Frozen flow (conduction only) through heater and liquid."""
    nx, nyf, nys = 5, 6, 5
    P, d = params(nx, nyf, nys, frozen_flow=1)
    Tb = W.spot_Tb(nx, d["Tsat"] + 0.1 * d["Tc"], 1, 2)
    bc = dict(T_top=d["Tsat"], Tb=Tb)
    rho = W.layered_rho(nx, nyf, 3, d["rho_L"], d["rho_V"])
    T = W.thermal_init(nx, nys, nyf, d["Tsat"], Tb)
    g, o = run_pair(P, bc, rho, T, steps=300, precision=0, window=(1, 301, 1))
    errs = compare(g, o)
    _report("frozen", errs)
    assert all(v <= 1e-11 for v in errs.values()), errs
    assert g["flux"]["q_bottom_mean"] == pytest.approx(o["flux"]["q_bottom_mean"], rel=1e-11)


@pytest.mark.parametrize("precision", [0, 1])
def test_steady_conduction_closed_form(precision):
    """Steady 1-D conduction through a heater under a thin frozen liquid layer,
    against the closed form: the same flux crosses every row link, so T is
    piecewise linear with link resistances 1/lambda_S in the heater, the
    harmonic mean at the interface and 1/lambda_L in the liquid and on the
    link to the T_sat row.  A steady field is where rounding T itself in FP32
    would act as a standing source; the FP32 energy equation works on FP64
    differences and FP32 increments, so its profile stays on the closed form."""
    nx, nyf, nys = 64, 4, 24
    P, d = params(nx, nyf, nys, frozen_flow=1)
    lamL, lamS = P["Cvchi"] * d["rho_L"], P["lambda_S"]
    Tb, Tt = d["Tsat"] + 0.1 * d["Tc"], d["Tsat"]
    g = gpu_domain(P, dict(T_top=Tt, Tb=np.full(nx, Tb)), np.full((nyf, nx), d["rho_L"]),
                   W.thermal_init(nx, nys, nyf, Tt, np.full(nx, Tb)), precision)
    n = 80000                     # about 45 e-folding times of the slowest mode
    g.step(n - 1)
    g.flux_window(n, n + 1, 1)
    g.step(1)
    res = [1 / lamS] * (nys - 1) + [(lamS + lamL) / (2 * lamS * lamL)] + [1 / lamL] * (nyf - 1) + [1 / lamL]
    q = (Tb - Tt) / sum(res)
    prof = Tb - q * np.concatenate([[0.0], np.cumsum(res)])[: nys + nyf]
    T = g.read(with_f=False)["T"]
    hf = g.heat_flux()
    g.close()
    errT = float(np.max(np.abs(T - prof[:, None])) / np.max(prof))
    errq = abs(hf["q_bottom_inst"] - q) / q
    print(f"steady conduction precision={precision}: T {errT:.2e}, q_bottom {errq:.2e}, "
          f"q_top {abs(hf['q_top_inst'] - q) / q:.2e}", flush=True)
    assert errT <= (1e-12 if precision == 0 else 1e-7)
    assert errq <= (1e-9 if precision == 0 else 1e-5)
    assert hf["q_top_inst"] == pytest.approx(q, rel=1e-9 if precision == 0 else 1e-5)


@pytest.mark.parametrize("tile", [(0, 0), (32, 16)])
@pytest.mark.parametrize("shape", [(1, 1, 3), (2, 3, 3), (3, 70, 4), (130, 2, 3), (2, 1, 1), (5, 4, 2)])
def test_degenerate_shapes(shape, tile):
    """Single column, one- and two-row fluid, tall-thin and wide-flat
    domains, one- and two-row heaters; heat flux sampled every step."""
    nx, nyf, nys = shape
    P, d, bc, rho, T = pool_case(nx, nyf, nys, superheat=0.15, n_spots=0, y0=max(1, nyf // 2))
    g, o = run_pair(P, bc, rho, T, steps=60, precision=0, tile=tile, window=(1, 61, 1))
    errs = compare(g, o)
    _report(f"shape {shape} tile={tile}", errs)
    assert all(v <= 1e-11 for v in errs.values()), errs
    assert g["flux"]["n_samples"] == o["flux"]["n_samples"] == 60
    for k in ("q_bottom_mean", "q_top_mean", "T_w_mean"):
        assert g["flux"][k] == pytest.approx(o["flux"][k], rel=1e-10, abs=1e-15), k


@pytest.mark.parametrize("precision", [0, 1])
def test_model_a_with_sinusoid_trigger(precision):
    """Model A of Section 4.1 (no heater: T_b is set on the Dirichlet row
    directly under the fluid, ny_solid = 1) with the Section 3.2 trigger
    T_b + 0.02 Tc sin(2 pi (x - l/4) / l) over a window of steps, then uniform
    T_b; the fluid is 2 l wide as in the paper's domain.  200 steps against
    the oracle; the heat flux is the link flux into the fluid."""
    nx, nyf, lam = 96, 64, 48.0
    P, d, bc, rho, T = pool_case(nx, nyf, 1, superheat=0.15, n_spots=0, y0=26)
    bc = dict(bc, Tb_alt=W.sinus_Tb(nx, bc["Tb"][0], 0.02 * d["Tc"], lam), t0=30, t1=150)
    g, o = run_pair(P, bc, rho, T, steps=200, precision=precision, window=(20, 201, 10))
    errs = compare(g, o)
    _report(f"model A prec={precision}", errs)
    assert all(v <= TOL[precision] for v in errs.values()), errs
    assert g["flux"]["n_samples"] == o["flux"]["n_samples"] == 19
    assert g["flux"]["q_bottom_mean"] == g["flux"]["q_top_mean"]
    for k in ("q_bottom_mean", "T_w_mean", "q_bottom_inst"):
        assert g["flux"][k] == pytest.approx(o["flux"][k], rel=TOL[precision] * 10, abs=1e-15), k


def test_bottom_window_and_zero_steps():
    """Section 3.2 trigger window on the heater bottom; step(0) is a no-op."""
    nx, nyf, nys = 40, 30, 4
    P, d, bc, rho, T = pool_case(nx, nyf, nys, superheat=0.1, n_spots=0)
    bc = dict(bc, Tb_alt=W.sinus_Tb(nx, bc["Tb"][0], 0.02 * d["Tc"], 20.0), t0=5, t1=25)
    g = gpu_domain(P, bc, rho, T)
    o = oracle_domain(P, bc, rho, T)
    g.step(0)
    for n in (3, 7, 20):
        g.step(n)
        o.step(n)
        errs = compare(g.read(), o.read())
        assert all(v <= 1e-11 for v in errs.values()), (n, errs)
    assert g.t == o.t == 30
    g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_profiled_steps_are_the_same_steps(precision):
    """pb_profile_steps runs real steps: stepping with HIP events around every
    launch (events reserved ahead, then reused by a second, longer call that
    creates the missing ones, with heat-flux samples inside) gives the same
    bits and the same time as plain stepping, and positive launch times."""
    P, d, bc, rho, T = pool_case(120, 60, 6, superheat=0.15, n_spots=3, seed=2)
    a = gpu_domain(P, bc, rho, T, precision=precision)
    b = gpu_domain(P, bc, rho, T, precision=precision)
    for dom in (a, b):
        dom.flux_window(1, 31, 3)
    a.step(30)
    b.profile_reserve(10)
    p1 = b.profile_steps(10)
    p2 = b.profile_steps(20)
    assert a.t == b.t == 30
    for p in (p1, p2):
        assert p["flow_ms"] > 0 and p["thermal_ms"] > 0 and p["step_ms"] >= p["flow_ms"]
    ra, rb = a.read(), b.read()
    for k in ("rho", "ux", "uy", "T", "f"):
        np.testing.assert_array_equal(ra[k], rb[k], err_msg=k)
    fa, fb = a.heat_flux(), b.heat_flux()
    assert fa["n_samples"] == fb["n_samples"] == 10
    assert fa["q_bottom_mean"] == fb["q_bottom_mean"]
    a.close()
    b.close()


def test_checkpoint_resume_fp64_bit_exact():
    """read f(t), T(t) and rho_bar, restore into a fresh domain, continue:
    identical to the uninterrupted run."""
    P, d, bc, rho, T = pool_case(50, 40, 5, superheat=0.2, n_spots=2, seed=4)
    a = gpu_domain(P, bc, rho, T)
    a.step(40)
    s = a.read()
    a.step(40)
    ra = a.read()
    b = gpu_domain(P, bc, rho, T)
    b.set_state(s["f"], s["T"], 40, a.rho_bar)
    b.step(40)
    rb = b.read()
    assert b.t == 80
    for k in ("rho", "ux", "uy", "T", "f"):
        np.testing.assert_array_equal(ra[k], rb[k], err_msg=k)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_alone_bit_exact(precision):
    """Three uneven domains stepped in shared launches (eager and replayed
    from a captured graph) equal each domain stepped alone, bit for bit."""
    from paper_1911_10747_amd import poolboil as pb
    cases = [pool_case(70, 50, 4, superheat=0.08, seed=1), pool_case(33, 20, 3, superheat=0.25, seed=2),
             pool_case(130, 64, 7, superheat=0.15, seed=3)]
    alone = []
    for P, d, bc, rho, T in cases:
        g = gpu_domain(P, bc, rho, T, precision)
        g.flux_window(10, 1000, 5)
        g.step(46)
        g.sync()
        alone.append((g.read(), g.heat_flux()))
        g.close()
    doms = []
    for P, d, bc, rho, T in cases:
        g = gpu_domain(P, bc, rho, T, precision)
        g.flux_window(10, 1000, 5)
        doms.append(g)
    batch = pb.Batch(doms, steps_per_graph=10)
    batch.step(3)     # eager
    batch.step(43)    # 4 graph replays + 3 eager
    for g in doms:
        g.sync()
    for g, (r0, f0) in zip(doms, alone):
        assert g.t == 46
        r = g.read()
        for k in ("rho", "ux", "uy", "T", "f"):
            np.testing.assert_array_equal(r[k], r0[k], err_msg=k)
        assert g.heat_flux() == f0
    batch.close()
    for g in doms:
        g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_of_auto_strip_domains_matches_alone(precision):
    """Six 1000x480 + 1000x24 domains that leave the energy strips to the
    library: alone each takes 8-row strips (18 x 63 strips), together the
    batch takes 16-row strips (3456 of them) and ends its work list with
    8-row strips (more strips than wavefront slots).  30 steps, bit for bit."""
    from paper_1911_10747_amd import poolboil as pb
    cases = [pool_case(1000, 480, 24, superheat=0.05 + 0.04 * i, n_spots=8, seed=20 + i, y0=190) for i in range(6)]
    assert pb.thermal_strip_rows(pb_config(cases[0][0], precision)) == 8
    alone = []
    for P, d, bc, rho, T in cases:
        g = gpu_domain(P, bc, rho, T, precision)
        g.step(30)
        g.sync()
        alone.append(g.read(with_f=False))
        g.close()
    doms = [gpu_domain(P, bc, rho, T, precision) for P, d, bc, rho, T in cases]
    batch = pb.Batch(doms, steps_per_graph=10)
    batch.step(30)
    for g, r0 in zip(doms, alone):
        g.sync()
        r = g.read(with_f=False)
        for k in ("rho", "ux", "uy", "T"):
            np.testing.assert_array_equal(r[k], r0[k], err_msg=k)
    batch.close()
    for g in doms:
        g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_membership_changes_bit_identical(precision):
    """Domains join and leave a running batch between steps (pb_batch_add,
    pb_batch_remove), each at a different time of its own, with graph
    replays and eager steps before and after every change, down to an empty
    batch: each domain equals the same domain stepped alone for its own number
    of steps, bit for bit, heat flux included.  A removed domain is read and
    destroyed right after its removal while the batch goes on."""
    from paper_1911_10747_amd import poolboil as pb
    cases = [pool_case(70, 50, 4, superheat=0.08, seed=1), pool_case(33, 20, 3, superheat=0.25, seed=2),
             pool_case(130, 64, 7, superheat=0.15, seed=3), pool_case(50, 40, 5, superheat=0.2, seed=4)]
    steps = [50, 91, 71, 28]
    alone = []
    for (P, d, bc, rho, T), n in zip(cases, steps):
        g = gpu_domain(P, bc, rho, T, precision)
        g.flux_window(10, 1000, 5)
        g.step(n)
        g.sync()
        alone.append((g.read(), g.heat_flux()))
        g.close()
    doms = []
    for P, d, bc, rho, T in cases:
        g = gpu_domain(P, bc, rho, T, precision)
        g.flux_window(10, 1000, 5)
        doms.append(g)
    A, B, C, D = doms
    got = {}

    def leave(k, dom):
        batch.remove(dom)
        got[k] = (dom.read(), dom.heat_flux(), dom.t)
        dom.close()

    batch = pb.Batch([A, B], steps_per_graph=10)
    batch.step(20)                     # two replays
    batch.add(C)
    assert len(batch) == 3
    batch.step(30)                     # captured again, three replays
    leave(0, A)
    batch.step(25)                     # two replays and five eager steps
    batch.add(D)
    batch.step(16)
    leave(1, B)
    leave(2, C)
    batch.step(12)
    leave(3, D)
    assert len(batch) == 0
    batch.step(5)                      # empty batch: nothing to do
    batch.close()
    for k, n in enumerate(steps):
        r, f, t = got[k]
        r0, f0 = alone[k]
        assert t == n, (k, t, n)
        for key in ("rho", "ux", "uy", "T", "f"):
            np.testing.assert_array_equal(r[key], r0[key], err_msg=f"domain {k}: {key}")
        assert f == f0, k
    with pytest.raises(pb.PbError):
        dup = gpu_domain(*cases[0][0:1], *cases[0][2:], precision)
        b2 = pb.Batch([dup], steps_per_graph=0)
        try:
            b2.add(dup)
        finally:
            b2.close()
            dup.close()


def test_batch_flux_windows_set_between_graph_replays():
    """Heat-flux windows opened on batch members after the batch has captured
    and replayed its step graph, with sampling periods that do (5) and do not
    (3) divide the graph length and different phases: every member's samples
    and means equal those of the same domain stepped alone."""
    from paper_1911_10747_amd import poolboil as pb
    cases = [pool_case(70, 50, 4, superheat=0.08, seed=1), pool_case(33, 20, 3, superheat=0.25, seed=2),
             pool_case(130, 64, 7, superheat=0.15, seed=3)]
    windows = [(23, 1000, 5), (31, 1000, 3), (27, 60, 5)]
    alone = []
    for (P, d, bc, rho, T), w in zip(cases, windows):
        g = gpu_domain(P, bc, rho, T, 1)
        g.step(20)
        g.flux_window(*w)
        g.step(55)
        g.sync()
        alone.append(g.heat_flux())
        g.close()
    doms = [gpu_domain(P, bc, rho, T, 1) for P, d, bc, rho, T in cases]
    batch = pb.Batch(doms, steps_per_graph=10)
    batch.step(20)                      # two replays of a graph with no flux sample
    for g, w in zip(doms, windows):
        g.flux_window(*w)
    batch.step(55)                      # captured again: five replays + 5 eager steps
    for g, f0 in zip(doms, alone):
        g.sync()
        f = g.heat_flux()
        print("flux", f["n_samples"], f0["n_samples"], flush=True)
        assert f["n_samples"] > 0
        assert f == f0
    batch.close()
    for g in doms:
        g.close()


@pytest.mark.parametrize("persistent", [1, 5, 64])
def test_persistent_batch_grid(persistent):
    """A capped (persistent) grid whose blocks loop over the tile work-list of
    several domains gives the same bits as one block per tile."""
    from paper_1911_10747_amd import poolboil as pb
    cases = [pool_case(70, 50, 4, superheat=0.08, seed=1), pool_case(33, 20, 3, superheat=0.25, seed=2)]
    ref = []
    for P, d, bc, rho, T in cases:
        g = gpu_domain(P, bc, rho, T, 1)
        g.step(24)
        ref.append(g.read())
        g.close()
    doms = [gpu_domain(P, bc, rho, T, 1) for P, d, bc, rho, T in cases]
    batch = pb.Batch(doms, steps_per_graph=8, persistent_blocks=persistent)
    batch.step(24)
    for g, r0 in zip(doms, ref):
        r = g.read()
        for k in ("rho", "ux", "uy", "T", "f"):
            np.testing.assert_array_equal(r[k], r0[k], err_msg=k)
        g.close()
    batch.close()


def test_checkpoint_resume_fp32_within_tolerance():
    """FP32-deviation restore re-encodes f(t) against the restored densities:
    identical to FP32 rounding, so the continued run stays within the FP32 bar."""
    P, d, bc, rho, T = pool_case(50, 40, 5, superheat=0.2, n_spots=2, seed=4)
    a = gpu_domain(P, bc, rho, T, 1)
    a.step(40)
    s = a.read()
    a.step(40)
    ra = a.read()
    b = gpu_domain(P, bc, rho, T, 1)
    b.set_state(s["f"], s["T"], 40, a.rho_bar)
    b.step(40)
    errs = compare(b.read(), ra)
    assert all(v <= 2e-5 for v in errs.values()), errs
    a.close()
    b.close()


def test_nonfinite_flag_is_sticky():
    """A density at the EOS pole region (rho b close to 1) makes the psi
    radicand negative: the step completes and pb_sync reports PB_ENONFINITE."""
    from paper_1911_10747_amd import poolboil as pb
    P, d, bc, rho, T = pool_case(20, 12, 3, n_spots=0)
    rho = rho.copy()
    rho[2, 5] = 10.0
    g = gpu_domain(P, bc, rho, T)
    g.step(2)
    with pytest.raises(pb.NonFiniteError):
        g.sync()
    g.set_fields(*pool_case(20, 12, 3, n_spots=0)[3:5])
    g.step(2)
    g.sync()
    g.close()
