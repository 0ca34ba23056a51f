"""Shared test set-up: parameter sets whose derived constants (Tc, Maxwell
densities) come from the oracle's own thermodynamics, and the standard
pool-boiling initial state built from the seeded generators."""
import functools

import numpy as np

from paper_1911_10747_amd import workloads as W
from oracle import eos


@functools.lru_cache(maxsize=None)
def derived(a, b, R, omega, t_ratio=W.T_SAT_OVER_TC):
    Tc = eos.critical_temperature(a, b, R)
    Ts = t_ratio * Tc
    rl, rv, ps = eos.maxwell(Ts, a, b, R, omega, Tc)
    return dict(Tc=Tc, Tsat=Ts, rho_L=rl, rho_V=rv, P_sat=ps,
                psi_L=eos.psi(rl, Ts, a, b, R, omega, Tc), psi_V=eos.psi(rv, Ts, a, b, R, omega, Tc))


def params(nx, nyf, nys, **over):
    """Full parameter dict (oracle field names) plus the derived constants."""
    P = dict(W.BASE_PARAMS)
    P.update({k: v for k, v in over.items() if k in P})
    d = derived(P["a"], P["b"], P["R"], P["omega"])
    P.update(nx=nx, nyf=nyf, nys=nys, Tc=d["Tc"], rho_L=d["rho_L"], rho_V=d["rho_V"],
             rho_S=W.RHO_S_OVER_RHO_L * d["rho_L"])
    for k in ("periodic_y", "isothermal", "frozen_flow", "sbar2_plus", "varpi_fm_only"):
        P[k] = int(over.get(k, 0))
    for k, v in over.items():
        if k not in P:
            P[k] = v
    return P, d


def pool_case(nx, nyf, nys, superheat=0.1, n_spots=4, seed=0, y0=None, gamma_frac=0.7, **over):
    """Pool-boiling start: liquid below y0 at the Maxwell density, vapour above,
    T = Tsat everywhere except the heater bottom at Tsat + superheat*Tc with
    seeded +2% hot spots; heater-wall adhesion gamma = -gamma_frac * psi_L,
    vapour-neutral top wall gamma = -psi_V; gravity for the domain height."""
    over.setdefault("g", W.gravity_for_height(nyf))
    P, d = params(nx, nyf, nys, **over)
    y0 = int(round(0.4 * nyf)) if y0 is None else y0
    Tb = d["Tsat"] + superheat * d["Tc"]
    Tb_row = W.spot_Tb(nx, Tb, n_spots, seed) if n_spots > 0 else np.full(nx, Tb)
    gam = np.full(nx, -gamma_frac * d["psi_L"])
    bc = dict(T_top=d["Tsat"], Tb=Tb_row, gamma_bot=gam, gamma_top=np.full(nx, -d["psi_V"]))
    rho = W.layered_rho(nx, nyf, y0, d["rho_L"], d["rho_V"])
    T = W.thermal_init(nx, nys, nyf, d["Tsat"], Tb_row)
    return P, d, bc, rho, T


def c1_case(case, superheat):
    """The paper-scale long-run case of a stored record: `case` holds nx, nyf,
    nys, seed, y0, optionally the varpi it was written with, and n_spots (spot
    trigger) or, with trigger "fluctuation",
    a uniform T_b replaced by the seeded per-column T_b (1 + rel xi_x) for
    t0 <= t < t1 (the workload's +-1% fluctuation)."""
    fluct = case.get("trigger") == "fluctuation"
    over = {k: case[k] for k in ("varpi",) if k in case}
    P, d, bc, rho, T = pool_case(case["nx"], case["nyf"], case["nys"], superheat=superheat,
                                 n_spots=0 if fluct else case["n_spots"], seed=case["seed"], y0=case["y0"], **over)
    if fluct:
        bc.update(Tb_alt=W.fluct_Tb(case["nx"], bc["Tb"][0], case["seed"], rel=case["rel"]),
                  t0=case["t0"], t1=case["t1"])
    return P, d, bc, rho, T
