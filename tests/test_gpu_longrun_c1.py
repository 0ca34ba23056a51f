"""Long runs at paper scale, the long-run bar for FP32 storage: a 400x400
fluid over a 400x20 heater (liquid below y = 160, six seeded +2% hot spots)
at superheats 0.05 .. 0.25 Tc for 20000 steps.  Boiling is chaotic, so the
FP32-deviation GPU runs and the FP64 oracle are compared only through the
time-mean wall heat flux (Eq. 38 of Eq. 36, steps 10000..20000 every 10),
within 3% per superheat.  The oracle means are stored in
tests/golden/longrun_c1_oracle.json, written by make_longrun_c1.py beside it
(which runs the oracle and nothing else, about an hour on eight cores)."""
import json
import os

import numpy as np
import pytest

from gpu_common import gpu_domain
from helpers import pool_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "longrun_c1_oracle.json")


def _run(rec, precision):
    from paper_1911_10747_amd import poolboil as pb
    c = rec["case"]
    doms = []
    for r in rec["results"]:
        P, d, bc, rho, T = pool_case(c["nx"], c["nyf"], c["nys"], superheat=r["superheat"], n_spots=c["n_spots"],
                                     seed=c["seed"], y0=c["y0"])
        g = gpu_domain(P, bc, rho, T, precision)
        g.flux_window(*rec["window"])
        doms.append(g)
    batch = pb.Batch(doms, steps_per_graph=500)
    batch.step(rec["steps"])
    batch.close()
    out = []
    for g in doms:
        g.sync()
        out.append(g.heat_flux())
        g.close()
    return out


def test_c1_long_run_mean_heat_flux_within_3pct():
    if not os.path.exists(GOLDEN):
        pytest.skip("oracle means not written yet (tests/golden/make_longrun_c1.py)")
    rec = json.load(open(GOLDEN))
    gpu = _run(rec, 1)
    for r, h in zip(rec["results"], gpu):
        rel = abs(h["q_bottom_mean"] - r["q_bottom_mean"]) / abs(r["q_bottom_mean"])
        print(f"superheat {r['superheat']:.2f}: q_gpu_fp32 {h['q_bottom_mean']:.6e} q_oracle {r['q_bottom_mean']:.6e} "
              f"rel {rel:.2e}", flush=True)
        assert r["status"] == 0
        assert h["n_samples"] == r["n_samples"] == 1001
        assert rel <= 0.03
