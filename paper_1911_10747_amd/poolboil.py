"""Thin ctypes binding of the C ABI in include/poolboil.h.

Argument marshalling only: every step of the method runs in the HIP kernels of
libpoolboil.so.  PyTorch supplies device memory (a uint8 tensor whose pointer
is handed to pb_create_domain) and the stream (torch's current stream).  There
is no fallback path: if the library is missing, importing this module raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpoolboil.so")

PB_OK, PB_EINVAL, PB_ENOMEM, PB_EDEVICE, PB_ENONFINITE, PB_ESTATE = 0, -1, -2, -3, -4, -5
PB_FP64, PB_FP32_DEV = 0, 1
PB_PERIODIC_Y, PB_ISOTHERMAL, PB_FROZEN_FLOW, PB_SBAR2_PLUS, PB_VARPI_FM_ONLY = 0x1, 0x2, 0x4, 0x8, 0x10

EXPORTED = [
    "pb_domain_bytes", "pb_thermal_strip_rows", "pb_thermal_work_list", "pb_flow_work_list", "pb_create_domain", "pb_destroy_domain", "pb_set_bc", "pb_set_fields", "pb_set_fields_full",
    "pb_step", "pb_sync", "pb_read_fields", "pb_read_fields_noalloc", "pb_flux_window", "pb_heat_flux", "pb_profile_steps", "pb_profile_reserve", "pb_time",
    "pb_rho_bar",
    "pb_batch_create", "pb_batch_step", "pb_batch_destroy", "pb_batch_add", "pb_batch_remove", "pb_batch_size", "pb_eos_critical_temperature", "pb_eos_coexistence",
    "pb_eos_psi", "pb_eos_latent_heat", "pb_last_error", "pb_version",
]


class PbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"poolboil error {code}: {msg}")
        self.code = code


class NonFiniteError(PbError):
    pass


class Config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny_fluid", C.c_int32), ("ny_solid", C.c_int32),
        ("precision", C.c_int32), ("flags", C.c_uint32),
        ("tile_x", C.c_int32), ("tile_y", C.c_int32), ("thermal_tile", C.c_int32),
        ("a", C.c_double), ("b", C.c_double), ("R", C.c_double), ("omega", C.c_double), ("Tc", C.c_double),
        ("G", C.c_double), ("s_e", C.c_double), ("s_q", C.c_double), ("varpi", C.c_double),
        ("tau_L", C.c_double), ("tau_V", C.c_double), ("rho_L", C.c_double), ("rho_V", C.c_double),
        ("g", C.c_double), ("Cv", C.c_double), ("Cvchi", C.c_double),
        ("rho_S", C.c_double), ("C_S", C.c_double), ("lambda_S", C.c_double),
    ]


class BC(C.Structure):
    _fields_ = [
        ("T_top", C.c_double),
        ("T_bottom", C.POINTER(C.c_double)), ("T_bottom_alt", C.POINTER(C.c_double)),
        ("alt_t0", C.c_int64), ("alt_t1", C.c_int64),
        ("gamma_bottom", C.POINTER(C.c_double)), ("gamma_top", C.POINTER(C.c_double)),
    ]


class Flux(C.Structure):
    _fields_ = [
        ("q_bottom_inst", C.c_double), ("q_top_inst", C.c_double), ("T_w_inst", C.c_double),
        ("q_bottom_mean", C.c_double), ("q_top_mean", C.c_double), ("T_w_mean", C.c_double),
        ("n_samples", C.c_int64),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1911_10747_amd._build (no fallback exists)")
    # torch bundles its own HIP runtime under a different file name; loading it
    # first makes the library bind to that same runtime (one runtime per
    # process, so torch-allocated device memory is valid for the library)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, dp, i64, i32 = C.c_void_p, C.POINTER(C.c_double), C.c_int64, C.c_int32
    sig = {
        "pb_domain_bytes": ([C.POINTER(Config), C.POINTER(C.c_size_t)], C.c_int),
        "pb_thermal_strip_rows": ([C.POINTER(Config), C.POINTER(C.c_int)], C.c_int),
        "pb_thermal_work_list": ([C.POINTER(C.POINTER(Config)), C.c_int32, C.POINTER(C.c_int32), C.c_int64,
                                  C.POINTER(C.c_int64)], C.c_int),
        "pb_flow_work_list": ([C.POINTER(Config), C.POINTER(C.c_int32), C.c_int64, C.POINTER(C.c_int64)], C.c_int),
        "pb_create_domain": ([C.POINTER(Config), vp, vp, C.c_size_t, C.POINTER(vp)], C.c_int),
        "pb_destroy_domain": ([vp], None),
        "pb_set_bc": ([vp, C.POINTER(BC)], C.c_int),
        "pb_set_fields": ([vp, dp, dp], C.c_int),
        "pb_set_fields_full": ([vp, dp, dp, i64, C.c_double], C.c_int),
        "pb_step": ([vp, i64], C.c_int),
        "pb_sync": ([vp], C.c_int),
        "pb_read_fields": ([vp, dp, dp, dp, dp, dp], C.c_int),
        "pb_read_fields_noalloc": ([vp, dp, dp, dp, dp, dp], C.c_int),
        "pb_flux_window": ([vp, i64, i64, i32], C.c_int),
        "pb_heat_flux": ([vp, C.POINTER(Flux)], C.c_int),
        "pb_profile_steps": ([vp, i64, dp], C.c_int),
        "pb_profile_reserve": ([vp, i64], C.c_int),
        "pb_time": ([vp], i64),
        "pb_rho_bar": ([vp], C.c_double),
        "pb_batch_create": ([C.POINTER(vp), i32, i32, i32, vp, C.POINTER(vp)], C.c_int),
        "pb_batch_step": ([vp, i64], C.c_int),
        "pb_batch_destroy": ([vp], None),
        "pb_batch_add": ([vp, vp], C.c_int),
        "pb_batch_remove": ([vp, vp], C.c_int),
        "pb_batch_size": ([vp], i32),
        "pb_eos_critical_temperature": ([C.c_double, C.c_double, C.c_double, dp], C.c_int),
        "pb_eos_coexistence": ([C.c_double] * 6 + [dp, dp], C.c_int),
        "pb_eos_psi": ([C.c_double] * 8 + [dp], C.c_int),
        "pb_eos_latent_heat": ([C.c_double] * 6 + [dp], C.c_int),
        "pb_last_error": ([], C.c_char_p),
        "pb_version": ([], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def _check(rc):
    if rc != PB_OK:
        msg = lib.pb_last_error().decode()
        raise (NonFiniteError if rc == PB_ENONFINITE else PbError)(rc, msg)


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))


def make_config(**kw):
    """Config from keyword arguments (pb_config field names)."""
    c = Config()
    names = {f for f, _ in Config._fields_}
    for k, v in kw.items():
        if k not in names:
            raise KeyError(f"unknown config field {k}")
        setattr(c, k, v)
    return c


def domain_bytes(cfg):
    n = C.c_size_t()
    _check(lib.pb_domain_bytes(C.byref(cfg), C.byref(n)))
    return n.value


def thermal_strip_rows(cfg):
    n = C.c_int()
    _check(lib.pb_thermal_strip_rows(C.byref(cfg), C.byref(n)))
    return n.value


def thermal_work_list(cfgs):
    """The energy launch's strips for these configurations stepped together
    (one: alone), in launch order: int32 array of (domain, x0, y0, rows) rows."""
    import numpy as np
    cfgs = list(cfgs)
    arr = (C.POINTER(Config) * len(cfgs))(*[C.pointer(c) for c in cfgs])
    n = C.c_int64()
    _check(lib.pb_thermal_work_list(arr, len(cfgs), None, 0, C.byref(n)))
    out = np.zeros((n.value, 4), dtype=np.int32)
    _check(lib.pb_thermal_work_list(arr, len(cfgs), out.ctypes.data_as(C.POINTER(C.c_int32)), n.value, C.byref(n)))
    return out


def flow_work_list(cfg):
    """The flow launch's tiles of one domain: int32 array of (x0, y0, width,
    height, alt) rows."""
    import numpy as np
    n = C.c_int64()
    _check(lib.pb_flow_work_list(C.byref(cfg), None, 0, C.byref(n)))
    out = np.zeros((n.value, 5), dtype=np.int32)
    _check(lib.pb_flow_work_list(C.byref(cfg), out.ctypes.data_as(C.POINTER(C.c_int32)), n.value, C.byref(n)))
    return out


def critical_temperature(a, b, R):
    out = C.c_double()
    _check(lib.pb_eos_critical_temperature(a, b, R, C.byref(out)))
    return out.value


def coexistence(a, b, R, omega, Tc, T):
    rl, rv = C.c_double(), C.c_double()
    _check(lib.pb_eos_coexistence(a, b, R, omega, Tc, T, C.byref(rl), C.byref(rv)))
    return rl.value, rv.value


def eos_psi(a, b, R, omega, Tc, G, rho, T):
    out = C.c_double()
    _check(lib.pb_eos_psi(a, b, R, omega, Tc, G, rho, T, C.byref(out)))
    return out.value


def latent_heat(a, b, R, omega, Tc, T):
    out = C.c_double()
    _check(lib.pb_eos_latent_heat(a, b, R, omega, Tc, T, C.byref(out)))
    return out.value


def _torch_stream_and_memory(nbytes, use_torch):
    if not use_torch:
        return None, None, None
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible to torch")
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    return torch.cuda.current_stream().cuda_stream, buf.data_ptr(), buf


class Domain:
    """One boiling domain resident in HBM (see include/poolboil.h)."""

    def __init__(self, cfg, use_torch=True, stream=None):
        self.cfg = cfg
        self.nx, self.nyf, self.nys = cfg.nx, cfg.ny_fluid, cfg.ny_solid
        self.nr = self.nyf + self.nys
        self.nbytes = domain_bytes(cfg)
        st, mem, self._buf = _torch_stream_and_memory(self.nbytes, use_torch)
        if stream is not None:
            st = stream
        self.stream = st
        h = C.c_void_p()
        _check(lib.pb_create_domain(C.byref(cfg), st, mem, self.nbytes if mem else 0, C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib.pb_destroy_domain(self._h)
            self._h = None
            self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_bc(self, T_top, Tb=None, Tb_alt=None, t0=0, t1=0, gamma_bot=None, gamma_top=None):
        arrs = [None if a is None else _f64(a, (self.nx,)) for a in (Tb, Tb_alt, gamma_bot, gamma_top)]
        bc = BC(float(T_top), _dptr(arrs[0]), _dptr(arrs[1]), int(t0), int(t1), _dptr(arrs[2]), _dptr(arrs[3]))
        _check(lib.pb_set_bc(self._h, C.byref(bc)))

    def set_fields(self, rho, T):
        rho = _f64(rho, (self.nyf, self.nx))
        T = _f64(T, (self.nr, self.nx))
        _check(lib.pb_set_fields(self._h, _dptr(rho), _dptr(T)))

    def set_state(self, f, T, t, rho_bar):
        f = _f64(f, (9, self.nyf, self.nx))
        T = _f64(T, (self.nr, self.nx))
        _check(lib.pb_set_fields_full(self._h, _dptr(f), _dptr(T), int(t), float(rho_bar)))

    def step(self, n=1):
        _check(lib.pb_step(self._h, int(n)))

    def sync(self):
        _check(lib.pb_sync(self._h))

    def read(self, with_f=True, noalloc=False):
        """rho, ux, uy, T (and f) at the current time; noalloc: through the
        fixed per-GPU staging (pb_read_fields_noalloc)."""
        nf = (self.nyf, self.nx)
        rho, ux, uy = np.empty(nf), np.empty(nf), np.empty(nf)
        T = np.empty((self.nr, self.nx))
        f = np.empty((9,) + nf) if with_f else None
        fn = lib.pb_read_fields_noalloc if noalloc else lib.pb_read_fields
        _check(fn(self._h, _dptr(rho), _dptr(ux), _dptr(uy), _dptr(T), _dptr(f)))
        out = dict(rho=rho, ux=ux, uy=uy, T=T)
        if with_f:
            out["f"] = f
        return out

    def flux_window(self, ta, tb, every=1):
        _check(lib.pb_flux_window(self._h, int(ta), int(tb), int(every)))

    def heat_flux(self):
        fl = Flux()
        _check(lib.pb_heat_flux(self._h, C.byref(fl)))
        return {k: getattr(fl, k) for k, _ in Flux._fields_}

    def profile_steps(self, n):
        """n real steps with HIP events around each launch; mean ms of the
        flow kernel, the thermal kernel and the whole step."""
        out = (C.c_double * 3)()
        _check(lib.pb_profile_steps(self._h, int(n), out))
        return dict(flow_ms=out[0], thermal_ms=out[1], step_ms=out[2])

    def profile_reserve(self, n):
        """Create the events of profile_steps(n) now (they stay with the
        domain), so that a timed profile_steps creates none."""
        _check(lib.pb_profile_reserve(self._h, int(n)))

    @property
    def t(self):
        return lib.pb_time(self._h)

    @property
    def rho_bar(self):
        return lib.pb_rho_bar(self._h)


class Batch:
    """Lock-step stepping of several domains in shared launches."""

    def __init__(self, domains, steps_per_graph=0, persistent_blocks=0, stream=None):
        """stream None: the library steps the batch on a stream of its own,
        ordered after (and before) the members' own streams."""
        self.domains = list(domains)
        arr = (C.c_void_p * len(self.domains))(*[d.handle for d in self.domains])
        h = C.c_void_p()
        _check(lib.pb_batch_create(arr, len(self.domains), int(steps_per_graph), int(persistent_blocks), stream,
                                   C.byref(h)))
        self._h = h

    def step(self, n):
        _check(lib.pb_batch_step(self._h, int(n)))

    def add(self, domain):
        """Add a domain between steps (pb_batch_add)."""
        _check(lib.pb_batch_add(self._h, domain.handle))
        self.domains.append(domain)

    def remove(self, domain):
        """Take a domain out between steps (pb_batch_remove)."""
        _check(lib.pb_batch_remove(self._h, domain.handle))
        self.domains = [d for d in self.domains if d is not domain]

    def __len__(self):
        return int(lib.pb_batch_size(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib.pb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
