"""Helpers for GPU parity tests: run the same seeded case through the HIP
library (C ABI) and the FP64 oracle and compare field by field."""
import numpy as np

FLAG_BITS = dict(periodic_y=0x1, isothermal=0x2, frozen_flow=0x4, sbar2_plus=0x8, varpi_fm_only=0x10)
CONFIG_KEYS = ["a", "b", "R", "omega", "Tc", "G", "s_e", "s_q", "varpi", "tau_L", "tau_V", "rho_L", "rho_V", "g",
               "Cv", "Cvchi", "rho_S", "C_S", "lambda_S"]


def pb_config(P, precision=0, tile=(0, 0), thermal_tile=0):
    from paper_1911_10747_amd import poolboil as pb
    flags = 0
    for k, bit in FLAG_BITS.items():
        if P.get(k, 0):
            flags |= bit
    kw = {k: P[k] for k in CONFIG_KEYS}
    return pb.make_config(nx=P["nx"], ny_fluid=P["nyf"], ny_solid=P["nys"], precision=precision, flags=flags,
                          tile_x=tile[0], tile_y=tile[1], thermal_tile=thermal_tile, **kw)


def gpu_domain(P, bc, rho, T, precision=0, tile=(0, 0), thermal_tile=0):
    from paper_1911_10747_amd import poolboil as pb
    dom = pb.Domain(pb_config(P, precision, tile, thermal_tile))
    dom.set_bc(**bc)
    dom.set_fields(rho, T)
    return dom


def oracle_domain(P, bc, rho, T):
    from oracle import orc
    dom = orc.Domain(**P)
    dom.set_bc(**bc)
    dom.set_fields(rho, T)
    return dom


def run_pair(P, bc, rho, T, steps, precision=0, tile=(0, 0), thermal_tile=0, window=None):
    """Step both sides; return (gpu fields, oracle fields) with heat flux."""
    g = gpu_domain(P, bc, rho, T, precision, tile, thermal_tile)
    o = oracle_domain(P, bc, rho, T)
    if window is not None:
        g.flux_window(*window)
        o.flux_window(*window)
    g.step(steps)
    g.sync()
    assert o.step(steps) == 0
    gr, orr = g.read(), o.read()
    gr["flux"], orr["flux"] = g.heat_flux(), o.heat_flux()
    gr["t"], orr["t"] = g.t, o.t
    g.close()
    return gr, orr


def rel_err(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def compare(g, o, keys=("rho", "ux", "uy", "T", "f")):
    """Max-norm relative error per field.  Velocity components are normalised
    by the speed scale max(|u_x|, |u_y|) of the oracle field: rounding noise
    in a component scales with the flow speed, not with that component's own
    maximum (which is near zero in nearly symmetric cases)."""
    out = {}
    uscale = max(np.max(np.abs(o["ux"])), np.max(np.abs(o["uy"])))
    for k in keys:
        if k in ("ux", "uy") and uscale > 0:
            out[k] = float(np.max(np.abs(g[k] - o[k])) / uscale)
        else:
            out[k] = rel_err(g[k], o[k])
    # the per-component form (each velocity component over its own maximum),
    # printed beside the bar for the record
    own = {k: rel_err(g[k], o[k]) for k in ("ux", "uy") if k in keys}
    print("per-component velocity errors", {k: f"{v:.2e}" for k, v in own.items()}, flush=True)
    return out
