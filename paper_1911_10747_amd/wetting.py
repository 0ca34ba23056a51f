"""Wettability calibration: the contact angle a wall adhesion coefficient
gamma = G_w psi(rho_w) (Eq. 14) produces, measured on a sessile drop, and the
gamma that gives a wanted angle.  The paper sets the heater wall to
theta = 55 deg and its nucleate spots to 105, 115 and 125 deg through G_w
(Sections 3.1 and 4.1) without printing the coefficients, so they are found
here by running drops on the GPU library and measuring them.

Drops run isothermally at T_sat with no gravity; the measurement (a circle
fitted to the interface and cut with the wall plane) is host-side analysis of
the density field, not part of the step.
"""
import math

import numpy as np

from . import workloads as W

from . import poolboil as pb
from . import presets


def cap_contact_angle(rho, rho_l, rho_v, wall_y=-0.5, skip_rows=3):
    """Contact angle in degrees, measured through the liquid, of one liquid
    cap resting on the bottom wall of `rho` ([ny][nx], row 0 next to the
    wall).  Interface points are the rho = (rho_l + rho_v) / 2 crossings
    between adjacent nodes (linear interpolation, along rows and columns),
    kept when more than `skip_rows` rows above the wall; a circle is fitted to
    them by linear least squares (x^2 + y^2 + D x + E y + F = 0) and cut with
    the wall plane y = wall_y, which halfway bounce-back puts half a node below
    row 0: cos(theta) = (wall_y - y_centre) / radius.  Returns
    (theta, (x_centre, y_centre, radius))."""
    rho = np.asarray(rho, dtype=np.float64)
    mid = 0.5 * (rho_l + rho_v)
    pts = []
    a, b = rho[:-1, :] - mid, rho[1:, :] - mid           # between rows y and y + 1
    for y, x in zip(*np.nonzero((a > 0) != (b > 0))):
        pts.append((x, y + a[y, x] / (a[y, x] - b[y, x])))
    a, b = rho[:, :-1] - mid, rho[:, 1:] - mid           # between columns x and x + 1
    for y, x in zip(*np.nonzero((a > 0) != (b > 0))):
        pts.append((x + a[y, x] / (a[y, x] - b[y, x]), y))
    p = np.array(pts, dtype=np.float64).reshape(-1, 2)
    p = p[p[:, 1] > skip_rows]
    if len(p) < 8:
        raise ValueError("no liquid cap found in the density field")
    A = np.c_[p[:, 0], p[:, 1], np.ones(len(p))]
    D, E, F = np.linalg.lstsq(A, -(p[:, 0] ** 2 + p[:, 1] ** 2), rcond=None)[0]
    xc, yc = -0.5 * D, -0.5 * E
    r = math.sqrt(xc * xc + yc * yc - F)
    c = min(1.0, max(-1.0, (wall_y - yc) / r))
    return math.degrees(math.acos(c)), (xc, yc, r)


def _params_and_derived(params, d):
    P = dict(W.BASE_PARAMS if params is None else params)
    if d is None:
        d = presets.derived(a=P["a"], b=P["b"], R=P["R"], omega=P["omega"], G=P["G"])
    return P, d


def sessile_drop(nx, ny, radius, gamma, d=None, precision=pb.PB_FP64, tile=(0, 0), params=None):
    """(config, bc kwargs, rho, T) of a drop test: a half disk of liquid of
    the given radius on the middle of the bottom wall (Maxwell densities, tanh
    interface), T = T_sat and isothermal, g = 0; the bottom wall has adhesion
    gamma, the top wall -psi_V (neutral to vapour).  params: the physical
    parameters (default the workload set), d: their derived constants."""
    P, d = _params_and_derived(params, d)
    P["g"] = 0.0
    cfg = pb.make_config(nx=nx, ny_fluid=ny, ny_solid=1, precision=precision, flags=pb.PB_ISOTHERMAL,
                         tile_x=tile[0], tile_y=tile[1], Tc=d.Tc, rho_L=d.rho_L, rho_V=d.rho_V,
                         rho_S=W.RHO_S_OVER_RHO_L * d.rho_L, **P)
    rho = W.drop_rho(nx, ny, radius, d.rho_L, d.rho_V, width=3.0, cx=(nx - 1) / 2.0, cy=-0.5)
    T = W.thermal_init(nx, 1, ny, d.Tsat, np.full(nx, d.Tsat))
    bc = dict(T_top=d.Tsat, Tb=np.full(nx, d.Tsat), gamma_bot=np.full(nx, float(gamma)),
              gamma_top=np.full(nx, -d.psi_V))
    return cfg, bc, rho, T


def contact_angles(gammas, nx=240, ny=120, radius=32, steps=20000, precision=pb.PB_FP64, d=None,
                   steps_per_graph=500, params=None):
    """Equilibrium contact angle (degrees) for each bottom-wall gamma: one
    drop per gamma, all stepped together in one batched launch.  NaN where a
    drop's run went non-finite (the domain's sticky flag; the others are
    unaffected)."""
    P, d = _params_and_derived(params, d)
    doms = []
    try:
        for g in gammas:
            cfg, bc, rho, T = sessile_drop(nx, ny, radius, g, d, precision, params=P)
            dom = pb.Domain(cfg)
            dom.set_bc(**bc)
            dom.set_fields(rho, T)
            doms.append(dom)
        batch = pb.Batch(doms, steps_per_graph=steps_per_graph)
        try:
            batch.step(steps)
        finally:
            batch.close()
        out = []
        for dom in doms:
            try:
                dom.sync()
            except pb.NonFiniteError:
                out.append(float("nan"))
                continue
            out.append(cap_contact_angle(dom.read(with_f=False)["rho"], d.rho_L, d.rho_V)[0])
        return np.array(out)
    finally:
        for dom in doms:
            dom.close()


def calibrate(thetas, gamma_range=None, n_coarse=12, n_fine=8, d=None, params=None, **kw):
    """Bottom-wall gamma giving each wanted contact angle (degrees).  theta
    falls as gamma grows more negative (a more attractive wall), so one
    batched sweep over gamma_range brackets every target; a second sweep over
    each bracket refines it; the answer is the linear interpolation of
    theta(gamma) there.  The default range, -0.95 .. -0.3 psi_L, spans about
    20 to 180 degrees (the drop stays on the wall); at -psi_L the run goes
    non-finite and above about -0.3 psi_L the drop leaves the wall.  Returns
    (gammas, {"coarse": (g, theta), "fine": [(g, theta), ...]})."""
    P, d = _params_and_derived(params, d)
    kw["params"] = P
    lo, hi = (-0.95 * d.psi_L, -0.3 * d.psi_L) if gamma_range is None else gamma_range
    g0 = np.linspace(lo, hi, n_coarse)
    th0 = contact_angles(g0, d=d, **kw)
    out, fine = [], []
    for th in np.atleast_1d(thetas):
        k = _bracket(th0, th)
        g1 = np.linspace(g0[k], g0[k + 1], n_fine)
        th1 = contact_angles(g1, d=d, **kw)
        j = _bracket(th1, th)
        out.append(_interp(g1[j], g1[j + 1], th1[j], th1[j + 1], th))
        fine.append((g1, th1))
    return np.array(out), {"coarse": (g0, th0), "fine": fine}


def _bracket(thetas, th):
    for k in range(len(thetas) - 1):
        if (thetas[k] - th) * (thetas[k + 1] - th) <= 0.0:     # False with a NaN end
            return k
    raise ValueError(f"contact angle {th} outside the swept range {np.nanmin(thetas):.1f}..{np.nanmax(thetas):.1f}")


def _interp(g0, g1, t0, t1, th):
    return g0 if t1 == t0 else g0 + (g1 - g0) * (th - t0) / (t1 - t0)


def pressure(rho, T, P):
    """Pressure the pseudopotential model carries, rho c_s^2 + G psi^2 / 2
    with c = 1 (Eq. 12), which with psi from Eq. 12-13 is the EOS pressure."""
    psi = pb.eos_psi(P["a"], P["b"], P["R"], P["omega"], P["Tc"], P["G"], float(rho), float(T))
    return float(rho) / 3.0 + 0.5 * P["G"] * psi * psi


def surface_tension(radii=(12, 16, 20, 24, 28), n=128, steps=20000, precision=pb.PB_FP64, params=None, d=None,
                    steps_per_graph=500):
    """Surface tension by Laplace's law in 2-D, dp = sigma / R: static liquid
    drops of several radii in a periodic n x n box, isothermal at T_sat, g = 0,
    all in one batched launch.  dp = P(rho at the centre) - P(rho at the
    corner); R is the equimolar radius, from the liquid excess over the vapour
    (pi R^2 = sum(rho - rho_out) / (rho_in - rho_out)).  Returns
    (sigma, intercept, [(R, dp), ...]) of the least-squares line dp(1/R)."""
    P, d = _params_and_derived(params, d)
    P.update(g=0.0, Tc=d.Tc)
    cfg_kw = {k: v for k, v in P.items()}
    doms, out = [], []
    try:
        for r in radii:
            cfg = pb.make_config(nx=n, ny_fluid=n, ny_solid=0, precision=precision,
                                 flags=pb.PB_PERIODIC_Y | pb.PB_ISOTHERMAL, rho_L=d.rho_L, rho_V=d.rho_V,
                                 rho_S=W.RHO_S_OVER_RHO_L * d.rho_L, **cfg_kw)
            dom = pb.Domain(cfg)
            dom.set_bc(d.Tsat)
            dom.set_fields(W.drop_rho(n, n, r, d.rho_L, d.rho_V, width=3.0), np.full((n, n), d.Tsat))
            doms.append(dom)
        batch = pb.Batch(doms, steps_per_graph=steps_per_graph)
        try:
            batch.step(steps)
        finally:
            batch.close()
        for dom in doms:
            dom.sync()
            rho = dom.read(with_f=False)["rho"]
            c = n // 2
            r_in = float(rho[c - 1:c + 1, c - 1:c + 1].mean())
            r_out = float(rho[0, 0])
            R = math.sqrt(float(np.sum(rho - r_out)) / (r_in - r_out) / math.pi)
            out.append((R, pressure(r_in, d.Tsat, P) - pressure(r_out, d.Tsat, P)))
    finally:
        for dom in doms:
            dom.close()
    x = np.array([1.0 / R for R, _ in out])
    y = np.array([dp for _, dp in out])
    sigma, icpt = np.polyfit(x, y, 1)
    return float(sigma), float(icpt), out
