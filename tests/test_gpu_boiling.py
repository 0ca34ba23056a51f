"""The boiling-curve driver on a reduced domain: jobs at several superheats
batched in one launch, both nucleation triggers, Q'' from the sampled bottom
flux with the Eq. 39 scale, and the FP32-deviation curve against the FP64 one
within the 3% heat-flux bar."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SMALL = dict(nx=100, nyf=75, nys=8, steps=4000, t_a=2000, every=10)
GAMMAS = {55.0: -0.7732, 105.0: -0.5296, 115.0: -0.4864, 125.0: -0.4455}   # times psi_L


@pytest.mark.parametrize("trigger", ["spots", "fluctuation"])
def test_small_curve_fp32_matches_fp64(trigger):
    from paper_1911_10747_amd import boiling, poolboil as pb
    P = boiling.paper_params()
    d = boiling.paper_derived(P)
    gam = {k: v * d.psi_L for k, v in GAMMAS.items()}
    runs = {}
    for prec in (pb.PB_FP64, pb.PB_FP32_DEV):
        runs[prec] = boiling.run_curve([0.2, 0.3], precision=prec, gammas=gam, sigma=0.079, trigger=trigger, **SMALL)
    r64, r32 = runs[pb.PB_FP64], runs[pb.PB_FP32_DEV]
    for j64, j32 in zip(r64["jobs"], r32["jobs"]):
        print(trigger, j64["Ja"], j64["Q"], j32["Q"], flush=True)
        assert not j64["error"] and not j32["error"]
        assert j64["samples"] == j32["samples"] == 201
        assert np.isfinite(j64["Q"]) and j64["Q"] > 0
        assert abs(j32["Q"] - j64["Q"]) <= 0.03 * abs(j64["Q"])
    assert r64["flux_scale"] == pytest.approx(r64["l0"] / (d.rho_L * 0.1 * r64["h_fg"]))
