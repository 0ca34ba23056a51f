"""ORACLE -- test infrastructure only.

ctypes wrapper around the serial FP64 C oracle (oracle/orc_step.c) of one time
step of the hybrid pseudopotential phase-change LBM with conjugate heat
transfer (arXiv:1911.10747, Section 2).  Only tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It imports nothing from the product
package; the product never imports it.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "orc_step.c")
# ORC_LIB names another build of the same source (the mutation tests load a
# copy of the oracle with one planted mistake this way)
LIB = os.environ.get("ORC_LIB") or os.path.join(HERE, "liborc.so")


def build(force=True, src=SRC, out=None):
    """Compile the oracle with plain gcc, no fast-math, no FP contraction."""
    out = LIB if out is None else out
    if force or not os.path.exists(out):
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                               "-o", out, src, "-lm"])
    return out


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("nyf", C.c_int32), ("nys", C.c_int32),
        ("periodic_y", C.c_int32), ("isothermal", C.c_int32), ("frozen_flow", C.c_int32),
        ("sbar2_plus", C.c_int32), ("varpi_fm_only", C.c_int32),
        ("a", C.c_double), ("b", C.c_double), ("R", C.c_double), ("omega", C.c_double),
        ("Tc", C.c_double), ("G", C.c_double),
        ("s_e", C.c_double), ("s_q", C.c_double), ("varpi", C.c_double),
        ("tau_L", C.c_double), ("tau_V", C.c_double), ("rho_L", C.c_double), ("rho_V", C.c_double),
        ("g", C.c_double),
        ("Cv", C.c_double), ("Cvchi", C.c_double), ("rho_S", C.c_double), ("C_S", C.c_double),
        ("lambda_S", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        pp = C.POINTER(Params)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [pp]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_bc.argtypes = [C.c_void_p, C.c_double, dp, dp, C.c_int64, C.c_int64, dp, dp]
        L.orc_set_fields.argtypes = [C.c_void_p, dp, dp]
        L.orc_set_state.argtypes = [C.c_void_p, dp, dp, C.c_int64, C.c_double]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_step.restype = C.c_int
        L.orc_read.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
        L.orc_read_forces.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
        L.orc_flux_window.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int]
        L.orc_heat_flux.argtypes = [C.c_void_p, dp]
        L.orc_rho_bar.argtypes = [C.c_void_p]
        L.orc_rho_bar.restype = C.c_double
        L.orc_time.argtypes = [C.c_void_p]
        L.orc_time.restype = C.c_int64
        L.orc_error.argtypes = [C.c_void_p]
        L.orc_error.restype = C.c_int
        L.orc_pressure.argtypes = [pp, C.c_double, C.c_double]
        L.orc_pressure.restype = C.c_double
        L.orc_dpdt.argtypes = [pp, C.c_double, C.c_double]
        L.orc_dpdt.restype = C.c_double
        L.orc_psi.argtypes = [pp, C.c_double, C.c_double, dp]
        L.orc_psi.restype = C.c_double
        L.orc_collide_node.argtypes = [pp, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                       C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.orc_moment_matrix.argtypes = [dp]
        L.orc_thermal_rhs.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


PARAM_KEYS = [k for k, _ in Params._fields_]


def make_params(**kw):
    p = Params()
    for k in PARAM_KEYS:
        if k in kw:
            setattr(p, k, kw[k])
    return p


class Domain:
    """One oracle domain: fluid [nyf][nx] over a heater [nys][nx]; thermal
    rows 0..nys+nyf-1 with row 0 the heater bottom."""

    def __init__(self, **params):
        self.params = make_params(**params)
        self.nx, self.nyf, self.nys = self.params.nx, self.params.nyf, self.params.nys
        self.nr = self.nyf + self.nys
        self._h = lib().orc_create(C.byref(self.params))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and callable(lib):          # module globals are gone at interpreter exit
            lib().orc_destroy(h)
            self._h = None

    def set_bc(self, T_top, Tb=None, Tb_alt=None, t0=0, t1=0, gamma_bot=None, gamma_top=None):
        c = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        self._keep = [c(Tb), c(Tb_alt), c(gamma_bot), c(gamma_top)]
        lib().orc_set_bc(self._h, float(T_top), *[_ptr(a) for a in self._keep[:2]], int(t0), int(t1),
                         *[_ptr(a) for a in self._keep[2:]])

    def set_fields(self, rho, T):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.nyf, self.nx)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(self.nr, self.nx)
        lib().orc_set_fields(self._h, _ptr(rho), _ptr(T))

    def set_state(self, f, T, t, rho_bar):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(9, self.nyf, self.nx)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(self.nr, self.nx)
        lib().orc_set_state(self._h, _ptr(f), _ptr(T), int(t), float(rho_bar))

    def step(self, n=1):
        return lib().orc_step(self._h, int(n))

    @property
    def t(self):
        return lib().orc_time(self._h)

    @property
    def rho_bar(self):
        return lib().orc_rho_bar(self._h)

    @property
    def error(self):
        return lib().orc_error(self._h)

    def read(self):
        nf = (self.nyf, self.nx)
        rho, ux, uy = np.zeros(nf), np.zeros(nf), np.zeros(nf)
        T = np.zeros((self.nr, self.nx))
        f = np.zeros((9,) + nf)
        lib().orc_read(self._h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), _ptr(f))
        return dict(rho=rho, ux=ux, uy=uy, T=T, f=f)

    def read_forces(self):
        nf = (self.nyf, self.nx)
        out = [np.zeros(nf) for _ in range(5)]
        lib().orc_read_forces(self._h, *[_ptr(a) for a in out])
        return dict(zip(["Fmx", "Fmy", "Fx", "Fy", "psi"], out))

    def flux_window(self, ta, tb, every=1):
        lib().orc_flux_window(self._h, int(ta), int(tb), int(every))

    def heat_flux(self):
        out = np.zeros(7)
        lib().orc_heat_flux(self._h, _ptr(out))
        keys = ["q_bottom_inst", "q_top_inst", "T_w_inst", "q_bottom_mean", "q_top_mean", "T_w_mean", "n_samples"]
        return dict(zip(keys, out.tolist()))

    def thermal_rhs(self, Tst, rho, vx, vy):
        Tst = np.ascontiguousarray(Tst, dtype=np.float64).reshape(self.nr, self.nx)
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.nyf, self.nx)
        vx = np.ascontiguousarray(vx, dtype=np.float64).reshape(self.nyf, self.nx)
        vy = np.ascontiguousarray(vy, dtype=np.float64).reshape(self.nyf, self.nx)
        K = np.zeros((self.nr, self.nx))
        lib().orc_thermal_rhs(self._h, _ptr(Tst), _ptr(rho), _ptr(vx), _ptr(vy), _ptr(K))
        return K


def collide_node(params, f, rho, ux, uy, Fx, Fy, Fmx, Fmy, psi):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(9)
    lib().orc_collide_node(C.byref(params), _ptr(f), rho, ux, uy, Fx, Fy, Fmx, Fmy, psi, _ptr(out))
    return out


def moment_matrix():
    out = np.zeros(81)
    lib().orc_moment_matrix(_ptr(out))
    return out.reshape(9, 9)


def pressure(params, rho, T):
    return lib().orc_pressure(C.byref(params), rho, T)


def dpdt(params, rho, T):
    return lib().orc_dpdt(C.byref(params), rho, T)


def psi(params, rho, T):
    rad = C.c_double()
    v = lib().orc_psi(C.byref(params), rho, T, C.byref(rad))
    return v, rad.value
