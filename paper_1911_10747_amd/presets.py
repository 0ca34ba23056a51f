"""Configurations and seeded initial states for pool-boiling jobs.

Derived constants (Tc, Maxwell densities, psi at the liquid density) come from
the library's host EOS helpers; inputs (layouts, hot spots) from the seeded
generators in `workloads`.  Nothing here steps the method.
"""
from dataclasses import dataclass, field

import numpy as np

from . import workloads as W

from . import poolboil as pb


@dataclass
class Derived:
    Tc: float
    Tsat: float
    rho_L: float
    rho_V: float
    psi_L: float
    psi_V: float


def derived(a=None, b=None, R=None, omega=None, G=-1.0, t_ratio=W.T_SAT_OVER_TC):
    P = W.BASE_PARAMS
    a = P["a"] if a is None else a
    b = P["b"] if b is None else b
    R = P["R"] if R is None else R
    omega = P["omega"] if omega is None else omega
    Tc = pb.critical_temperature(a, b, R)
    Ts = t_ratio * Tc
    rl, rv = pb.coexistence(a, b, R, omega, Tc, Ts)
    return Derived(Tc, Ts, rl, rv, pb.eos_psi(a, b, R, omega, Tc, G, rl, Ts), pb.eos_psi(a, b, R, omega, Tc, G, rv, Ts))


# Wall adhesion gamma / psi_L for the contact angles the paper uses (55 deg on
# the heater, 105, 115 and 125 deg on its nucleate spots, Sections 3.1 and
# 4.1), found by wetting.calibrate: sessile drops of radius 32 on a 240 x 120
# fluid, isothermal at T_sat, g = 0, 20 000 FP64 steps.  tests/test_gpu_wetting
# recomputes the calibration and checks it to 1.5 deg.
CONTACT_ANGLE_GAMMA = {55.0: -0.7661, 105.0: -0.5366, 115.0: -0.4955, 125.0: -0.4570}


def gamma_for_angle(theta, d=None):
    """Adhesion gamma for a contact angle (degrees) between 55 and 125, by
    linear interpolation of CONTACT_ANGLE_GAMMA (theta(gamma) is close to
    linear there)."""
    d = derived() if d is None else d
    th = np.array(sorted(CONTACT_ANGLE_GAMMA))
    if not th[0] <= theta <= th[-1]:
        raise ValueError(f"contact angle {theta} outside the calibrated range {th[0]}..{th[-1]}")
    return float(np.interp(theta, th, [CONTACT_ANGLE_GAMMA[t] for t in th])) * d.psi_L


@dataclass
class JobSpec:
    """One boiling-curve job: a domain size, a heater-bottom superheat (units
    of Tc), a number of steps and a seed for the nucleate hot spots."""
    nx: int
    nyf: int
    nys: int
    superheat: float
    steps: int = 2000
    seed: int = 0
    precision: int = pb.PB_FP32_DEV
    spots_per_columns: int = 64      # one +2% hot spot per this many columns (at least one)
    liquid_fraction: float = 0.4     # liquid below this fraction of the fluid height
    gamma_frac: float = 0.7          # heater-wall adhesion gamma = -gamma_frac * psi_L (top wall: -psi_V)
    contact_angle: float = None      # if set (55..125 deg), the heater-wall gamma from CONTACT_ANGLE_GAMMA
    tile: tuple = (0, 0)
    thermal_tile: int = 0
    flux_every: int = 10
    overrides: dict = field(default_factory=dict)


def make_config(spec, d=None):
    d = derived() if d is None else d
    P = dict(W.BASE_PARAMS)
    P["g"] = W.gravity_for_height(spec.nyf)
    P.update({k: v for k, v in spec.overrides.items() if k in P})
    return pb.make_config(nx=spec.nx, ny_fluid=spec.nyf, ny_solid=spec.nys, precision=spec.precision, flags=0,
                          tile_x=spec.tile[0], tile_y=spec.tile[1], thermal_tile=spec.thermal_tile,
                          Tc=d.Tc, rho_L=d.rho_L, rho_V=d.rho_V, rho_S=W.RHO_S_OVER_RHO_L * d.rho_L, **P)


def initial_state(spec, d=None):
    """(bc kwargs, rho, T) of the standard pool-boiling start."""
    d = derived() if d is None else d
    Tb = d.Tsat + spec.superheat * d.Tc
    n_spots = max(1, spec.nx // spec.spots_per_columns)
    Tb_row = W.spot_Tb(spec.nx, Tb, n_spots, spec.seed)
    g_wall = -spec.gamma_frac * d.psi_L if spec.contact_angle is None else gamma_for_angle(spec.contact_angle, d)
    gam = np.full(spec.nx, g_wall)
    bc = dict(T_top=d.Tsat, Tb=Tb_row, gamma_bot=gam, gamma_top=np.full(spec.nx, -d.psi_V))
    rho = W.layered_rho(spec.nx, spec.nyf, int(round(spec.liquid_fraction * spec.nyf)), d.rho_L, d.rho_V)
    T = W.thermal_init(spec.nx, spec.nys, spec.nyf, d.Tsat, Tb_row)
    return bc, rho, T


def make_domain(spec, d=None, use_torch=True, stream=None, with_window=True):
    d = derived() if d is None else d
    dom = pb.Domain(make_config(spec, d), use_torch=use_torch, stream=stream)
    bc, rho, T = initial_state(spec, d)
    dom.set_bc(**bc)
    dom.set_fields(rho, T)
    if with_window and spec.nys >= 1:
        # Eq. 38 time mean over the second half of the run
        dom.flux_window(spec.steps // 2, spec.steps + 1, spec.flux_every)
    return dom
