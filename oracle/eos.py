"""ORACLE -- test infrastructure only.

Plain FP64 thermodynamics of the Peng-Robinson equation of state used by the
hybrid phase-change LBM (arXiv:1911.10747, Section 2.1, Eq. 13, and the
Maxwell relation of Section 2.2, Eq. 19).  Pure Python floats; every routine
is a direct transcription of a definition or a bracketed root search, so a
reader can check it against the paper by eye.  Only tests, the smoke check and
the benchmark's CPU-baseline leg import this module.

Readings:
  * the critical temperature is taken from the paper's own relations
    a = 0.45724 R^2 Tc^2 / Pc and b = 0.0778 R Tc / Pc (Eq. 13 text), giving
    Tc = 0.0778 a / (0.45724 b R); the printed a = 2/49 and Tc = 0.1094 do not
    agree with each other (a = 3/49 reproduces 0.1094);
  * the coexistence densities are the Maxwell equal-area pair (Section 3.1);
  * the latent heat is T (s_V - s_L) with the entropy difference integrated
    from the Maxwell relation (dP/dT)_v along the isotherm (Eq. 19).
"""
import math


def kappa(omega):
    """Peng-Robinson kappa(omega) (Eq. 13)."""
    return 0.37464 + 1.54226 * omega - 0.26992 * omega * omega


def critical_temperature(a, b, R):
    """Tc from a = 0.45724 R^2 Tc^2/Pc and b = 0.0778 R Tc/Pc (Eq. 13 text)."""
    return 0.0778 * a / (0.45724 * b * R)


def phi(T, Tc, omega):
    """Temperature function of Eq. 13."""
    s = 1.0 + kappa(omega) * (1.0 - math.sqrt(T / Tc))
    return s * s


def pressure(rho, T, a, b, R, omega, Tc):
    """P_EOS(rho, T) of Eq. 13."""
    return (rho * R * T / (1.0 - b * rho)
            - a * phi(T, Tc, omega) * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho))


def dpdt(rho, T, a, b, R, omega, Tc):
    """(dP_EOS/dT) at constant rho, differentiated by hand from Eq. 13."""
    k = kappa(omega)
    s = 1.0 + k * (1.0 - math.sqrt(T / Tc))
    dphi = -k * s / math.sqrt(T * Tc)
    return rho * R / (1.0 - b * rho) - a * dphi * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho)


def psi(rho, T, a, b, R, omega, Tc, G=-1.0):
    """Pseudopotential of Eq. 12 with c = 1, c_s^2 = 1/3."""
    return math.sqrt(2.0 * (pressure(rho, T, a, b, R, omega, Tc) - rho / 3.0) / G)


def _pv_integral(v, T, a, b, R, omega, Tc):
    """Antiderivative of P with respect to specific volume v = 1/rho along an
    isotherm: R T ln(v-b) - a phi/(2 sqrt2 b) ln((v+b-sqrt2 b)/(v+b+sqrt2 b))."""
    r2 = math.sqrt(2.0)
    return (R * T * math.log(v - b)
            - a * phi(T, Tc, omega) / (2.0 * r2 * b)
            * math.log((v + b - r2 * b) / (v + b + r2 * b)))


def _bisect(fn, lo, hi, iters=200):
    flo = fn(lo)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        fm = fn(mid)
        if fm == 0.0:
            return mid
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
        if hi - lo <= 1e-16 * max(1.0, abs(mid)):
            break
    return 0.5 * (lo + hi)


def spinodals(T, a, b, R, omega, Tc, n=20000):
    """Local maximum (vapour spinodal) and local minimum (liquid spinodal) of
    P(rho) on (0, 1/b) at T < Tc, refined by bisection on a centred difference."""
    P = lambda r: pressure(r, T, a, b, R, omega, Tc)
    rmax = 1.0 / b
    grid = [rmax * (k + 0.5) / n for k in range(n)]
    vals = [P(r) for r in grid]
    i_max = next(k for k in range(1, n - 1) if vals[k] >= vals[k - 1] and vals[k] > vals[k + 1])
    i_min = next(k for k in range(i_max + 1, n - 1) if vals[k] <= vals[k - 1] and vals[k] < vals[k + 1])
    h = 1e-7
    dP = lambda r: P(r + h) - P(r - h)
    r1 = _bisect(dP, grid[i_max - 1], grid[i_max + 1])
    r2 = _bisect(dP, grid[i_min - 1], grid[i_min + 1])
    return r1, r2


def maxwell(T, a, b, R, omega, Tc):
    """Coexistence densities (rho_L, rho_V) and saturation pressure at T < Tc by
    the equal-area rule: P(v_L) = P(v_V) = P_s and the integral of P dv from v_L
    to v_V equals P_s (v_V - v_L).  Nested bisection on P_s."""
    P = lambda r: pressure(r, T, a, b, R, omega, Tc)
    rs1, rs2 = spinodals(T, a, b, R, omega, Tc)
    p_hi = P(rs1)
    p_lo = max(P(rs2), 1e-14)

    def roots(ps):
        rv = _bisect(lambda r: P(r) - ps, 1e-12, rs1)
        rl = _bisect(lambda r: P(r) - ps, rs2, (1.0 / b) * (1.0 - 1e-12))
        return rl, rv

    def area(ps):
        rl, rv = roots(ps)
        vl, vv = 1.0 / rl, 1.0 / rv
        integ = _pv_integral(vv, T, a, b, R, omega, Tc) - _pv_integral(vl, T, a, b, R, omega, Tc)
        return integ - ps * (vv - vl)

    ps = _bisect(area, p_lo, p_hi)
    rl, rv = roots(ps)
    return rl, rv, ps


def latent_heat(T, a, b, R, omega, Tc):
    """h_fg = T (s_V - s_L) with ds = (dP/dT)_v dv along the isotherm (Eq. 19).
    For Eq. 13 the integral of (dP/dT)_v over v is
    R ln(v-b) - a phi'(T)/(2 sqrt2 b) ln((v+b-sqrt2 b)/(v+b+sqrt2 b))."""
    rl, rv, _ = maxwell(T, a, b, R, omega, Tc)
    k = kappa(omega)
    s = 1.0 + k * (1.0 - math.sqrt(T / Tc))
    dphi = -k * s / math.sqrt(T * Tc)
    r2 = math.sqrt(2.0)

    def F(v):
        return R * math.log(v - b) - a * dphi / (2.0 * r2 * b) * math.log((v + b - r2 * b) / (v + b + r2 * b))

    return T * (F(1.0 / rv) - F(1.0 / rl))
