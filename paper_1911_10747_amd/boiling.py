"""The paper's boiling curve (Section 4.3, Fig. 11) on its own set-up, run on
the GPU library.

Model B of Fig. 1: a 400 x 300 fluid over a 400 x 30 heater, liquid filling
the lower half of the pool (2 lambda_d x 0.75 lambda_d of each phase), the
printed g = 5e-5 and a = 3/49 (the value that reproduces the printed
Tc = 0.1094 and h_fg = 0.58; with a = 2/49 the vapour of a 300-row pool
cannot carry the hydrostatic head of the printed g), a 55 deg heater wall
with three nucleate spots of 105, 115 and 125 deg centred at x = 66, 200 and
356, and a constant heater-bottom temperature T_b for each superheat.

Reported per superheat: Ja (Eq. 37), Q'' (Eqs. 38-39: the time mean of the
dimensionless bottom heat flux over t_a <= t < t_b), the heater-top mean
temperature; and the CHF of Zuber's and Kandlikar's models (Eqs. 40-41) with
the surface tension measured by Laplace's law on the same parameters.  The
length and time scales l_0 and t_0 come from Eqs. 31-32 with that surface
tension.
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import workloads as W

from . import poolboil as pb
from . import presets
from . import wetting

A_PAPER = 3.0 / 49.0
NX, NYF, NYS = 400, 300, 30
SPOTS = ((66, 105.0), (200, 115.0), (356, 125.0))   # (centre x, contact angle)
SPOT_WIDTH = 10                                      # nodes; not printed in the paper
HEATER_ANGLE = 55.0


def paper_params():
    """Physical parameters of the paper's boiling runs (Section 3.1)."""
    return dict(W.BASE_PARAMS, a=A_PAPER, g=5e-5, varpi=W.VARPI_A_3_49)


def paper_derived(P=None):
    P = paper_params() if P is None else P
    return presets.derived(a=P["a"], b=P["b"], R=P["R"], omega=P["omega"], G=P["G"])


def latent_heat(P, d):
    return pb.latent_heat(P["a"], P["b"], P["R"], P["omega"], d.Tc, d.Tsat)


def scales(sigma, P, d):
    """l_0 (Eq. 31), t_0 (Eq. 32), lambda_d = 2 pi sqrt(3) l_0 (Eq. 29)."""
    l0 = math.sqrt(sigma / (P["g"] * (d.rho_L - d.rho_V)))
    return dict(l0=l0, t0=math.sqrt(l0 / P["g"]), lambda_d=2.0 * math.pi * math.sqrt(3.0) * l0)


def flux_scale(sigma, P, d, h_fg):
    """Q' = Q l_0 / (mu_L h_fg) (Eq. 39); mu_L = rho_L nu_L with nu_L from tau_L."""
    nu_l = (P["tau_L"] - 0.5) / 3.0
    return scales(sigma, P, d)["l0"] / (d.rho_L * nu_l * h_fg)


def chf_models(sigma, P, d, h_fg, theta_deg=HEATER_ANGLE):
    """Dimensionless CHF (Eq. 40 scaled by Eq. 39) of Zuber (K = 0.12 and
    0.157) and of Kandlikar (Eq. 41 at the heater's contact angle)."""
    base = d.rho_V * h_fg * (sigma * P["g"] * (d.rho_L - d.rho_V) / d.rho_V ** 2) ** 0.25
    c = math.cos(math.radians(theta_deg))
    k_kand = (1.0 + c) / 16.0 * (2.0 / math.pi + math.pi / 4.0 * (1.0 + c)) ** 0.5
    s = flux_scale(sigma, P, d, h_fg)
    return dict(zuber_012=0.12 * base * s, zuber_0157=0.157 * base * s, kandlikar=k_kand * base * s,
                K_kandlikar=k_kand)


def heater_gamma(nx, gammas, spots=SPOTS, width=SPOT_WIDTH):
    """Bottom-wall adhesion row: the heater angle everywhere, the spot angles
    on `width` columns around each spot centre (x scaled by nx / 400)."""
    row = np.full(nx, gammas[HEATER_ANGLE])
    for xc, th in spots:
        c = int(round(xc * nx / NX))
        for dx in range(-(width // 2), width - width // 2):
            row[(c + dx) % nx] = gammas[th]
    return row


def calibrated_gammas(P, d, **kw):
    """gamma for the heater and spot angles on these parameters (wetting.calibrate)."""
    angles = sorted({HEATER_ANGLE} | {th for _, th in SPOTS})
    g, _ = wetting.calibrate(np.array(angles), params=P, d=d, **kw)
    return dict(zip(angles, (float(v) for v in g)))


def job_inputs(superheat, gammas, nx=NX, nyf=NYF, nys=NYS, trigger="spots", P=None, d=None):
    """Parameters, boundary data and initial fields of one boiling-curve job:
    (params with nx, nyf, nys and every physical constant, bc keyword
    arguments of set_bc, rho [nyf][nx], T [nys + nyf][nx]).  Liquid in the
    lower half of the pool at the Maxwell density, T = T_sat except the
    heater bottom at T_sat + superheat Tc; the heater wall at 55 deg with the
    three spots (trigger "spots"), or a uniform 55 deg wall with the Section
    3.2 sinusoid on T_b for 3000 <= t < 15000 (trigger "fluctuation")."""
    P = paper_params() if P is None else P
    d = paper_derived(P) if d is None else d
    params = dict(P, nx=nx, nyf=nyf, nys=nys, Tc=d.Tc, rho_L=d.rho_L, rho_V=d.rho_V,
                  rho_S=W.RHO_S_OVER_RHO_L * d.rho_L)
    gam = heater_gamma(nx, gammas) if trigger == "spots" else np.full(nx, gammas[HEATER_ANGLE])
    Tb = np.full(nx, d.Tsat + superheat * d.Tc)
    bc = dict(T_top=d.Tsat, Tb=Tb, gamma_bot=gam, gamma_top=np.full(nx, -d.psi_V))
    if trigger == "fluctuation":
        bc.update(Tb_alt=W.sinus_Tb(nx, Tb[0], 0.02 * d.Tc, nx / 2.0), t0=3000, t1=15000)
    rho = W.layered_rho(nx, nyf, nyf // 2, d.rho_L, d.rho_V)
    return params, bc, rho, W.thermal_init(nx, nys, nyf, d.Tsat, Tb)


def run_curve(superheats, steps=42000, t_a=25000, every=10, precision=pb.PB_FP32_DEV, gammas=None, sigma=None,
              nx=NX, nyf=NYF, nys=NYS, trigger="spots", log=None, chunk=3000):
    """One job per superheat (units of Tc), all stepped in one batched launch
    from the same start; returns a dict with the per-job results and the
    scales used.  trigger "spots": the three nucleate spots on a 55 deg wall
    and a constant T_b (Fig. 11); "fluctuation": a uniform 55 deg wall and
    T_b + 0.02 Tc sin(2 pi (x - l/4) / l), l = nx / 2, for 3000 <= t < 15000
    (Section 3.2), then constant T_b.  A job whose run goes non-finite
    records the end of the first chunk of `chunk` steps after which that was
    seen (fail_by_t)."""
    if trigger not in ("spots", "fluctuation"):
        raise ValueError("trigger is 'spots' or 'fluctuation'")
    P = paper_params()
    d = paper_derived(P)
    h_fg = latent_heat(P, d)
    if gammas is None:
        gammas = calibrated_gammas(P, d)
    if sigma is None:
        sigma = wetting.surface_tension(params=P, d=d)[0]
    doms = []
    try:
        for sh in superheats:
            cp, bc, rho, T = job_inputs(sh, gammas, nx=nx, nyf=nyf, nys=nys, trigger=trigger, P=P, d=d)
            c = pb.make_config(nx=nx, ny_fluid=nyf, ny_solid=nys, precision=precision, flags=0,
                               **{k: v for k, v in cp.items() if k not in ("nx", "nyf", "nys")})
            dom = pb.Domain(c)
            dom.set_bc(**bc)
            dom.set_fields(rho, T)
            dom.flux_window(t_a, steps + 1, every)
            doms.append(dom)
        batch = pb.Batch(doms, steps_per_graph=500)
        t0 = time.time()
        fail_by = [None] * len(doms)   # end of the first chunk after which a job's non-finite flag was seen
        try:
            done = 0
            while done < steps:
                k = min(chunk, steps - done)
                batch.step(k)
                done += k
                for j, dom in enumerate(doms):
                    if fail_by[j] is None:
                        try:
                            dom.sync()
                        except pb.NonFiniteError:
                            fail_by[j] = done
                if log:
                    log(f"boiling curve: {done}/{steps} steps, {time.time() - t0:.1f} s")
        finally:
            batch.close()
        s = flux_scale(sigma, P, d, h_fg)
        jobs = []
        for sh, dom, fb in zip(superheats, doms, fail_by):
            rec = dict(superheat_Tc=float(sh), Ja=P["Cv"] * sh * d.Tc / h_fg, fail_by_t=fb)
            try:
                dom.sync()
                hf = dom.heat_flux()
                rec.update(Q=hf["q_bottom_mean"] * s, Q_top=hf["q_top_mean"] * s,
                           Tw_minus_Tsat_Tc=(hf["T_w_mean"] - d.Tsat) / d.Tc, samples=hf["n_samples"], error="")
            except pb.NonFiniteError as e:
                rec.update(Q=float("nan"), Q_top=float("nan"), Tw_minus_Tsat_Tc=float("nan"), samples=0,
                           error=str(e))
            jobs.append(rec)
        wall = time.time() - t0
    finally:
        for dom in doms:
            dom.close()
    sc = scales(sigma, P, d)
    return dict(jobs=jobs, sigma=sigma, h_fg=h_fg, l0=sc["l0"], t0=sc["t0"], lambda_d=sc["lambda_d"],
                flux_scale=s, chf=chf_models(sigma, P, d, h_fg), gammas_over_psiL={k: v / d.psi_L for k, v in
                                                                                  gammas.items()},
                steps=steps, t_a=t_a, every=every, precision=precision, trigger=trigger, wall_s=wall,
                node_updates=float(len(superheats)) * nx * (nyf + nys) * steps)


def berenson_nu(Tw_minus_Tsat, sigma, P, d, h_fg):
    """Space-averaged film-boiling Nusselt number of Berenson's model in the
    paper's form (Eq. 34), with h'_fg = h_fg + 0.5 C_V,V (T_w - T_sat),
    lambda_V = C_V chi rho_V and mu_V = rho_V nu_V."""
    lam_v = P["Cvchi"] * d.rho_V
    mu_v = d.rho_V * (P["tau_V"] - 0.5) / 3.0
    hp = h_fg + 0.5 * P["Cv"] * Tw_minus_Tsat
    g = P["g"]
    return (0.425 * 2.0 * math.sqrt(3.0) * math.pi
            * (g * d.rho_V * (d.rho_L - d.rho_V) * hp / (lam_v * mu_v * Tw_minus_Tsat)) ** 0.25
            * (sigma / (g * (d.rho_L - d.rho_V))) ** 0.375)


def film_boiling_nu(run, P=None, d=None):
    """Simulated space- and time-averaged Nu = h lambda_d / lambda_V with
    h = Q / (T_w - T_sat) (Section 3.2) for each job of a run_curve result,
    next to Berenson's value at the same wall superheat."""
    P = paper_params() if P is None else P
    d = paper_derived(P) if d is None else d
    lam_v = P["Cvchi"] * d.rho_V
    out = []
    for j in run["jobs"]:
        dTw = j["Tw_minus_Tsat_Tc"] * d.Tc
        q = j["Q"] / run["flux_scale"]
        nu = q / dTw * run["lambda_d"] / lam_v if dTw > 0 else float("nan")
        out.append(dict(Ja=j["Ja"], Nu=nu, Nu_berenson=berenson_nu(dTw, run["sigma"], P, d, run["h_fg"])
                        if dTw > 0 else float("nan")))
    return out


RECORD_SUPERHEATS = (0.03, 0.06, 0.09, 0.12, 0.15, 0.18, 0.21, 0.24, 0.27, 0.30, 0.33, 0.36, 0.40, 0.41, 0.45)
FILM_T_B_OVER_TC = 1.27     # Section 3.2: film boiling at T_b = 1.27 Tc


def record(superheats=RECORD_SUPERHEATS, log=None):
    """The boiling curve on the paper's set-up, as a record: the nucleate-spot
    curve in FP32-deviation and FP64 storage and the fluctuation-trigger curve
    in FP32-deviation storage, with the same calibrated wall adhesion and the
    surface tension of Laplace's law; the CHF point of each curve against
    Zuber (Eq. 40, K = 0.12) and Kandlikar (Eq. 41 at 55 deg), and the
    film-boiling Nusselt number at T_b = 1.27 Tc against Berenson (Eq. 34).
    The paper's own figures are carried as context."""
    P = paper_params()
    d = paper_derived(P)
    gammas = calibrated_gammas(P, d)
    sigma = wetting.surface_tension(params=P, d=d)[0]
    out = dict(set_up=dict(nx=NX, nyf=NYF, nys=NYS, a=P["a"], varpi=P["varpi"], g=P["g"], s_e=P["s_e"],
                           s_q=P["s_q"], heater_angle=HEATER_ANGLE, spots=[list(sp) for sp in SPOTS],
                           spot_width=SPOT_WIDTH, steps=42000, window=[25000, 42001, 10]),
               gammas_over_psiL={str(k): v / d.psi_L for k, v in gammas.items()}, sigma=sigma,
               paper=dict(chf_deviation_zuber=0.006, chf_deviation_kandlikar=0.099, Nu_film=54.01,
                          Nu_berenson=51.28, T_w_film_over_Tc=1.2660))
    film_sh = FILM_T_B_OVER_TC - 0.86
    for name, trig, prec in (("spots_fp32", "spots", pb.PB_FP32_DEV), ("fluctuation_fp32", "fluctuation", pb.PB_FP32_DEV),
                             ("spots_fp64", "spots", pb.PB_FP64)):
        r = run_curve(list(superheats), precision=prec, gammas=gammas, sigma=sigma, trigger=trig, log=log)
        r["film_boiling_nu"] = film_boiling_nu(r, P, d)
        fin = [j for j in r["jobs"] if not j["error"]]
        chf = max(fin, key=lambda j: j["Q"]) if fin else None
        summ = dict(finite=len(fin), jobs=len(r["jobs"]))
        if chf is not None:
            summ.update(chf_Q=chf["Q"], chf_Ja=chf["Ja"], zuber_012=r["chf"]["zuber_012"],
                        kandlikar=r["chf"]["kandlikar"], chf_over_zuber=chf["Q"] / r["chf"]["zuber_012"],
                        chf_over_kandlikar=chf["Q"] / r["chf"]["kandlikar"])
        for j, nu in zip(r["jobs"], r["film_boiling_nu"]):
            if abs(j["superheat_Tc"] - film_sh) < 1e-9 and not j["error"]:
                summ.update(film_T_w_over_Tc=0.86 + j["Tw_minus_Tsat_Tc"], film_Nu=nu["Nu"],
                            film_Nu_berenson=nu["Nu_berenson"])
        r["summary"] = summ
        out[name] = r
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--superheats", default="0.03,0.06,0.09,0.12,0.15,0.18,0.21,0.24,0.27,0.30,0.33,0.36,0.40,0.45",
                    help="heater-bottom superheats in units of Tc")
    ap.add_argument("--steps", type=int, default=42000)
    ap.add_argument("--t-a", type=int, default=25000)
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--trigger", choices=("spots", "fluctuation"), default="spots")
    ap.add_argument("--record", metavar="PATH", help="run the three curves of record() and write them to PATH")
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    if args.record:
        res = record(log=log)
        with open(args.record, "w") as fh:
            json.dump(res, fh, indent=1, default=float)
        for name in ("spots_fp32", "fluctuation_fp32", "spots_fp64"):
            print(name, json.dumps(res[name]["summary"]), file=sys.stderr)
        return
    sh = [float(v) for v in args.superheats.split(",")]
    res = run_curve(sh, steps=args.steps, t_a=args.t_a, precision=pb.PB_FP64 if args.fp64 else pb.PB_FP32_DEV,
                    trigger=args.trigger, log=log)
    res["film_boiling_nu"] = film_boiling_nu(res)
    for j in res["jobs"]:
        print(f"Ja {j['Ja']:.4f}  Q'' {j['Q']:.4f}  Q''(top) {j['Q_top']:.4f}  "
              f"(Tw-Tsat)/Tc {j['Tw_minus_Tsat_Tc']:.4f} {j['error']}", file=sys.stderr)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
