"""Writes longrun_c1_oracle.json: the FP64 oracle's time-mean wall heat flux
(Eq. 38 over steps 10000..20000, sampled every 10) for the paper-scale pool
(400x400 fluid over a 400x20 heater, liquid below y = 160, six seeded +2% hot
spots) at superheats 0.05 .. 0.25 Tc, 20000 steps each; with `fluctuation`,
longrun_c1_fluct_oracle.json for the same pool with a uniform T_b replaced by
a seeded +-1% per-column fluctuation for 3000 <= t < 15000; with `draws`,
longrun_c1_draws_oracle.json for the hot-spot pool at three superheats drawn
uniformly from [0.05, 0.25] Tc (seed 2024).  The records were written with
varpi = 0.1 (Eq. 9), which each case names.  Calls only the oracle (one
process per superheat); about an hour on eight cores for five superheats.

    python tests/golden/make_longrun_c1.py [fluctuation | draws]
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
CASES = {
    "spots": (dict(nx=400, nyf=400, nys=20, n_spots=6, seed=11, y0=160, varpi=0.1), "longrun_c1_oracle.json"),
    "fluctuation": (dict(nx=400, nyf=400, nys=20, n_spots=0, seed=11, y0=160, trigger="fluctuation", rel=0.01,
                         t0=3000, t1=15000, varpi=0.1), "longrun_c1_fluct_oracle.json"),
    "draws": (dict(nx=400, nyf=400, nys=20, n_spots=6, seed=11, y0=160, varpi=0.1), "longrun_c1_draws_oracle.json"),
}


def drawn_superheats(n=3, seed=2024):
    import numpy as np
    rng = np.random.default_rng(seed)
    return sorted(round(float(s), 4) for s in rng.uniform(0.05, 0.25, n))
STEPS, WINDOW = 20000, (10000, 20001, 10)
CASE = CASES["spots"][0]


def run(sh):
    from helpers import c1_case
    from oracle import orc
    P, d, bc, rho, T = c1_case(CASE, sh)
    o = orc.Domain(**P)
    o.set_bc(**bc)
    o.set_fields(rho, T)
    o.flux_window(*WINDOW)
    t0 = time.time()
    rc = o.step(STEPS)
    hf = o.heat_flux()
    return dict(superheat=sh, status=int(rc), seconds=round(time.time() - t0, 1), **hf)


def main():
    global CASE
    trigger = sys.argv[1] if len(sys.argv) > 1 else "spots"
    CASE, name = CASES[trigger]
    superheats = drawn_superheats() if trigger == "draws" else SUPERHEATS
    with mp.Pool(len(superheats)) as pool:
        res = pool.map(run, superheats)
    out = dict(case=CASE, steps=STEPS, window=list(WINDOW), results=res,
               note="FP64 oracle, Eq. 38 time means of Eq. 36 (q_bottom), the interface link flux (q_top) and the "
                    "heater-top temperature")
    with open(os.path.join(HERE, name), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
