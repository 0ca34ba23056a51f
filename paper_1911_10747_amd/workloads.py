"""Seeded synthetic inputs for the pool-boiling step: initial density and
temperature layouts, heater-bottom temperature arrays (nucleate hot spots,
seeded fluctuation), wall-adhesion arrays and job streams.

This module holds no arithmetic of the method itself: callers pass in every
physical number (coexistence densities, temperatures).  It is shared by the
tests, the benchmark and the serving front end so that the oracle and the HIP
path see byte-identical inputs.
"""
import math

import numpy as np

# Physical parameters as printed (Section 3.1) plus the readings for the values
# the paper leaves open (s_e, s_q, varpi, C_S, G).  nu_L = 0.1 -> tau_L = 0.8 and
# nu_V = 0.5/3 -> tau_V = 1.0 through Eq. 4.  varpi (Eq. 9, no value printed)
# is the value at which a flat, gravity-free liquid slab at T_sat = 0.86 Tc
# relaxes to the Maxwell densities of Eq. 13 (vapour within 0.03%, liquid
# within 0.001%): 0.1112 for a = 2/49, 0.1044 for a = 3/49 (VARPI_A_3_49).
BASE_PARAMS = dict(
    a=2.0 / 49.0, b=2.0 / 21.0, R=1.0, omega=0.344, G=-1.0,
    s_e=0.8, s_q=1.1, varpi=0.1112,
    tau_L=0.8, tau_V=1.0,
    g=5e-5,
    Cv=6.0, Cvchi=0.05, C_S=6.0, lambda_S=16.25,
)
VARPI_A_3_49 = 0.1044        # the same coexistence calibration for a = 3/49
T_SAT_OVER_TC = 0.86          # Section 3.1
RHO_S_OVER_RHO_L = 3.0        # Section 3.1
REF_FLUID_HEIGHT = 150        # rows up to which the printed g = 5e-5 is used (see gravity_for_height)


def gravity_for_height(nyf, g=BASE_PARAMS["g"]):
    """Gravity for a fluid domain of nyf rows: the printed g (Section 3.1)
    up to 150 rows, scaled by 150/nyf above, so that the hydrostatic head the
    buoyancy term (rho - rho_bar) g builds across the vapour column (60% of
    the height) stays near 0.6 P_sat.  With a head above P_sat the vapour
    cannot carry it: it rarefies to zero above the liquid and the run blows
    up (the FP64 oracle does so within ~1400 steps on a 395-row column)."""
    return float(g) * min(1.0, REF_FLUID_HEIGHT / float(nyf))


def layered_rho(nx, nyf, y0, rho_l, rho_v):
    """Liquid (rho_l) in fluid rows y < y0, vapour above: a sharp layer."""
    rho = np.full((nyf, nx), float(rho_v))
    rho[: int(y0), :] = float(rho_l)
    return rho


def thermal_init(nx, nys, nyf, T_sat, Tb_row=None):
    """T = T_sat on every thermal row; row 0 takes Tb_row if given."""
    T = np.full((nys + nyf, nx), float(T_sat))
    if Tb_row is not None and nys > 0:
        T[0, :] = np.asarray(Tb_row, dtype=np.float64)
    return T


def spot_positions(nx, n_spots, seed, width=3):
    """Distinct, non-overlapping seeded spot centres."""
    rng = np.random.default_rng(seed)
    n_slots = max(1, nx // (width + 1))
    n = min(n_spots, n_slots)
    slots = np.sort(rng.choice(n_slots, size=n, replace=False))
    return [int(s * (width + 1) + width // 2) for s in slots]


def spot_Tb(nx, Tb, n_spots, seed, rel=0.02, width=3):
    """Uniform heater-bottom temperature Tb with n_spots hot spots of `width`
    columns at Tb * (1 + rel)."""
    arr = np.full(nx, float(Tb))
    for c in spot_positions(nx, n_spots, seed, width):
        for dx in range(-(width // 2), width - width // 2):
            arr[(c + dx) % nx] = float(Tb) * (1.0 + rel)
    return arr


def fluct_Tb(nx, Tb, seed, rel=0.01):
    """Tb * (1 + rel * xi_x) with xi_x ~ U[-1, 1], one draw per column."""
    rng = np.random.default_rng(seed)
    return float(Tb) * (1.0 + rel * rng.uniform(-1.0, 1.0, size=nx))


def sinus_Tb(nx, Tb, amp, wavelength):
    """Tb + amp * sin(2 pi (x - wavelength/4) / wavelength) (Section 3.2 trigger)."""
    x = np.arange(nx, dtype=np.float64)
    return float(Tb) + float(amp) * np.sin(2.0 * math.pi * (x - wavelength / 4.0) / wavelength)


def drop_rho(nx, ny, radius, rho_in, rho_out, width=2.0, cx=None, cy=None):
    """Round drop (or bubble) with a tanh interface, centred in a periodic box."""
    cx = (nx - 1) / 2.0 if cx is None else cx
    cy = (ny - 1) / 2.0 if cy is None else cy
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return 0.5 * (rho_in + rho_out) - 0.5 * (rho_in - rho_out) * np.tanh(2.0 * (r - radius) / width)


def slab_rho(nx, ny, y_lo, y_hi, rho_in, rho_out, width=2.0):
    """Flat liquid slab between rows y_lo and y_hi with tanh interfaces."""
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    s = np.tanh(2.0 * (y - y_lo) / width) - np.tanh(2.0 * (y - y_hi) / width)
    return rho_out + 0.5 * (rho_in - rho_out) * s


def perturbed(arr, rel, seed):
    """arr * (1 + rel * xi), xi ~ U[-1, 1] elementwise."""
    rng = np.random.default_rng(seed)
    return np.asarray(arr, dtype=np.float64) * (1.0 + rel * rng.uniform(-1.0, 1.0, size=np.shape(arr)))


def log_uniform_int(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_jobs(seed=0, n=32, nx_range=(128, 1024), ny_range=(128, 512), superheat=(0.02, 0.30),
               steps=20000, heater_frac=1.0 / 20.0, min_heater=3):
    """Boiling-curve job mix: log-uniform fluid sizes, heater height a fixed
    fraction of the fluid height (at least min_heater rows), uniform
    superheat in units of Tc."""
    rng = np.random.default_rng(seed)
    jobs = []
    for k in range(n):
        nx = log_uniform_int(rng, *nx_range)
        ny = log_uniform_int(rng, *ny_range)
        jobs.append(dict(job=k, nx=nx, nyf=ny, nys=max(min_heater, int(round(ny * heater_frac))),
                         superheat=float(rng.uniform(*superheat)), steps=int(steps), seed=int(seed * 1000 + k)))
    return jobs


def job_stream(seed=0, n=64, rate_per_s=1.0, nx_range=(64, 2048), ny_range=(64, 1024),
               superheat=(0.02, 0.30), steps_range=(5000, 20000), heater_frac=1.0 / 20.0, min_heater=3):
    """Poisson arrival stream of boiling-curve jobs (arrival times in seconds)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for k in range(n):
        t += float(rng.exponential(1.0 / rate_per_s))
        nx = log_uniform_int(rng, *nx_range)
        ny = log_uniform_int(rng, *ny_range)
        jobs.append(dict(job=k, arrival=t, nx=nx, nyf=ny, nys=max(min_heater, int(round(ny * heater_frac))),
                         superheat=float(rng.uniform(*superheat)),
                         steps=int(rng.integers(steps_range[0], steps_range[1] + 1)), seed=int(seed * 1000 + k)))
    return jobs
