"""Writes longrun_c1_oracle.json: the FP64 oracle's time-mean wall heat flux
(Eq. 38 over steps 10000..20000, sampled every 10) for the paper-scale pool
(400x400 fluid over a 400x20 heater, liquid below y = 160, six seeded +2% hot
spots) at superheats 0.05 .. 0.25 Tc, 20000 steps each.  Calls only the
oracle (one process per superheat); about an hour on eight cores.

    python tests/golden/make_longrun_c1.py
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.join(os.path.dirname(HERE), ".."))

SUPERHEATS = [0.05, 0.10, 0.15, 0.20, 0.25]
CASE = dict(nx=400, nyf=400, nys=20, n_spots=6, seed=11, y0=160)
STEPS, WINDOW = 20000, (10000, 20001, 10)


def run(sh):
    from helpers import pool_case
    from oracle import orc
    P, d, bc, rho, T = pool_case(CASE["nx"], CASE["nyf"], CASE["nys"], superheat=sh, n_spots=CASE["n_spots"],
                                 seed=CASE["seed"], y0=CASE["y0"])
    o = orc.Domain(**P)
    o.set_bc(bc["T_top"], bc["Tb"], gamma_bot=bc["gamma_bot"], gamma_top=bc["gamma_top"])
    o.set_fields(rho, T)
    o.flux_window(*WINDOW)
    t0 = time.time()
    rc = o.step(STEPS)
    hf = o.heat_flux()
    return dict(superheat=sh, status=int(rc), seconds=round(time.time() - t0, 1), **hf)


def main():
    with mp.Pool(len(SUPERHEATS)) as pool:
        res = pool.map(run, SUPERHEATS)
    out = dict(case=CASE, steps=STEPS, window=list(WINDOW), results=res,
               note="FP64 oracle, Eq. 38 time means of Eq. 36 (q_bottom), the interface link flux (q_top) and the "
                    "heater-top temperature")
    with open(os.path.join(HERE, "longrun_c1_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
