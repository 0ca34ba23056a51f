"""The oracle's pins catch planted mistakes.

Each case copies oracle/orc_step.c, plants one mistake of the kind a careful
reading could still make (a swapped rate row of Eq. 3, reversed endpoints of
Eq. 5, a first-order Eq. 36, the printed sign of row 8 of Eq. 9, ...), builds
that copy and runs the named pins against it in a child process (through
ORC_LIB); at least one of them must fail.  The unmodified source must pass
the same pins.  CPU only: the mistakes live in a temporary copy of the
oracle, never in the HIP path.
"""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "orc_step.c")
PINS = "tests/test_oracle_pins.py::"

# (name, text in orc_step.c, replacement, pins expected to catch it)
MUTATIONS = [
    ("Eq. 3 s_e and s_q rows swapped",
     "s[0] = 1.0; s[1] = p->s_e; s[2] = p->s_e;\n    s[3] = 1.0; s[4] = p->s_q; s[5] = 1.0; s[6] = p->s_q;",
     "s[0] = 1.0; s[1] = p->s_q; s[2] = p->s_q;\n    s[3] = 1.0; s[4] = p->s_e; s[5] = 1.0; s[6] = p->s_e;",
     ["test_relaxation_rates_act_on_their_moments"]),
    ("Eq. 5 interpolation endpoints reversed",
     "double tau_v = p->tau_V + (rho - p->rho_V) / (p->rho_L - p->rho_V) * (p->tau_L - p->tau_V);",
     "double tau_v = p->tau_L + (rho - p->rho_V) / (p->rho_L - p->rho_V) * (p->tau_V - p->tau_L);",
     ["test_relaxation_rates_act_on_their_moments", "test_shear_wave_decays_with_printed_viscosity"]),
    ("Eq. 36 as a first-order difference",
     "double dTdy = (4.0 * d->T[NI(d, 1, x)] - d->T[NI(d, 2, x)] - 3.0 * d->T[NI(d, 0, x)]) / 2.0;",
     "double dTdy = d->T[NI(d, 1, x)] - d->T[NI(d, 0, x)];",
     ["test_eq36_second_order_on_quadratic_heater_profile"]),
    ("Eq. 9 varpi term with F_m alone by default",
     "if (!d->p.varpi_fm_only) { fwx += d->Fax[n]; fwy += d->Fay[n]; }",
     "if (0) { fwx += d->Fax[n]; fwy += d->Fay[n]; }",
     ["test_varpi_force_reading_rest_beside_neutral_wall", "test_rest_state_is_stationary"]),
    ("Eq. 9 row 8 with the printed minus sign",
     "S[8] = ux * Fy + uy * Fx;", "S[8] = ux * Fy - uy * Fx;",
     ["test_collision_reduces_to_bgk_with_guo_forcing"]),
    ("Eq. 9 varpi term missing from row 1",
     "S[1] = 6.0 * uF + 12.0 * p->varpi", "S[1] = 6.0 * uF + 0.0 * p->varpi",
     ["test_varpi_term_moment_rows", "test_flat_interface_coexistence"]),
    ("Eq. 10 velocity with the whole force",
     "d->ux[n] = (d->jx[n] + dt * d->Fx[n] / 2.0) / d->rho[n];",
     "d->ux[n] = (d->jx[n] + dt * d->Fx[n]) / d->rho[n];",
     ["test_forces_on_a_field_layered_in_x", "test_total_momentum_conserved_on_periodic_domain",
      "test_mirror_symmetry"]),
    ("Eq. 11 axis and diagonal weights swapped",
     "return i == 0 ? 0.0 : (i < 5 ? 1.0 / 3.0 : 1.0 / 12.0);",
     "return i == 0 ? 0.0 : (i < 5 ? 1.0 / 12.0 : 1.0 / 3.0);",
     ["test_forces_on_a_layered_field", "test_forces_on_a_field_layered_in_x"]),
    ("Eq. 13 attraction term with the wrong sign",
     "- p->a * phi * rho * rho / (1.0 + 2.0 * p->b * rho - p->b * p->b * rho * rho);",
     "+ p->a * phi * rho * rho / (1.0 + 2.0 * p->b * rho - p->b * p->b * rho * rho);",
     ["test_c_oracle_eos_and_dpdt"]),
    ("Eq. 15 buoyancy with the wrong sign",
     "double Fgx = 0.0, Fgy = (d->rho[n] - d->rho_bar) * (-p->g);",
     "double Fgx = 0.0, Fgy = (d->rho[n] - d->rho_bar) * (p->g);",
     ["test_forces_on_a_layered_field"]),
    ("Eq. 24 latent-heat term with the wrong sign",
     "- Tc0 / (rh * p->Cv) * orc_dpdt(p, rh, Tc0) * divv;",
     "+ Tc0 / (rh * p->Cv) * orc_dpdt(p, rh, Tc0) * divv;",
     ["test_latent_heat_term"]),
    ("Eq. 26 stage-2 weight 1 instead of 2",
     "for (size_t n = 0; n < nt; ++n) { d->acc[n] += 2.0 * d->K[n]; d->Ts[n] = d->T[n] + dt / 2.0 * d->K[n]; }",
     "for (size_t n = 0; n < nt; ++n) { d->acc[n] += 1.0 * d->K[n]; d->Ts[n] = d->T[n] + dt / 2.0 * d->K[n]; }",
     ["test_rk4_fourier_decay"]),
    ("Eq. 28 arithmetic instead of harmonic link mean",
     "lamh = 2.0 * lam0 * lamn / (lam0 + lamn);\n                    if (rn >= d->nys)",
     "lamh = 0.5 * (lam0 + lamn);\n                    if (rn >= d->nys)",
     ["test_steady_conduction_through_heater_and_liquid"]),
    ("Eq. 27 gradient with the force weights",
     "gx += w * Tn * EX[i]; gy += w * Tn * EY[i];",
     "gx += force_w(i) * Tn * EX[i]; gy += force_w(i) * Tn * EY[i];",
     ["test_thermal_stencils_on_fourier_modes"]),
    ("Eq. 8 bounce-back returning the wrong population",
     "else d->f[FI(d, i, y, x)] = d->fs[FI(d, OPP[i], y, x)];",
     "else d->f[FI(d, i, y, x)] = d->fs[FI(d, i, y, x)];",
     ["test_mass_conserved_with_walls_and_heater"]),
    ("Eq. 8 pull from the wrong side in x",
     "int xs = (x - EX[i] + d->nx) % d->nx;\n                int ys = y - EY[i];",
     "int xs = (x + EX[i] + d->nx) % d->nx;\n                int ys = y - EY[i];",
     ["test_total_momentum_conserved_on_periodic_domain", "test_mirror_symmetry"]),
]


def _run_pins(lib, tests):
    env = dict(os.environ, ORC_LIB=lib, PYTHONDONTWRITEBYTECODE="1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + [PINS + t for t in tests]
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def _build(src_text, tmp, name):
    from oracle import orc
    c = os.path.join(tmp, name + ".c")
    with open(c, "w") as fh:
        fh.write(src_text)
    return orc.build(force=True, src=c, out=os.path.join(tmp, name + ".so"))


def test_pins_catch_planted_mistakes():
    with open(SRC) as fh:
        src = fh.read()
    for name, old, new, _ in MUTATIONS:
        assert src.count(old) == 1, f"mutation site of '{name}' not found exactly once"
    all_pins = sorted({t for m in MUTATIONS for t in m[3]})
    with tempfile.TemporaryDirectory() as tmp:
        base = _build(src, tmp, "base")
        libs = [_build(src.replace(old, new), tmp, f"m{k}") for k, (_, old, new, _) in enumerate(MUTATIONS)]
        with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            ok = ex.submit(_run_pins, base, all_pins)
            runs = [ex.submit(_run_pins, lib, m[3]) for lib, m in zip(libs, MUTATIONS)]
            r0 = ok.result()
            assert r0.returncode == 0, "unmodified oracle fails its pins:\n" + r0.stdout[-3000:]
            missed = [m[0] for m, r in zip(MUTATIONS, runs) if r.result().returncode == 0]
    assert not missed, f"planted mistakes no pin caught: {missed}"
