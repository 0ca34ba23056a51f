"""pb_read_fields_noalloc through the C ABI: the same outputs as
pb_read_fields, bit for bit, on two calls in a row (the second on a smaller
domain, so the fixed per-GPU staging holds a larger earlier read); a domain
whose staging would exceed the fixed array is refused before any device
work; reads through either entry point can alternate on one domain."""
import ctypes as C

import numpy as np
import pytest

from gpu_common import gpu_domain
from helpers import pool_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _read_abi(dom, noalloc):
    from paper_1911_10747_amd import poolboil as pb
    nf = (dom.nyf, dom.nx)
    out = dict(rho=np.empty(nf), ux=np.empty(nf), uy=np.empty(nf), T=np.empty((dom.nr, dom.nx)),
               f=np.empty((9,) + nf))
    ptr = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    fn = pb.lib.pb_read_fields_noalloc if noalloc else pb.lib.pb_read_fields
    rc = fn(dom.handle, ptr(out["rho"]), ptr(out["ux"]), ptr(out["uy"]), ptr(out["T"]), ptr(out["f"]))
    assert rc == pb.PB_OK, pb.lib.pb_last_error().decode()
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_read_matches_allocating_read(precision):
    from paper_1911_10747_amd import poolboil as pb
    for nx, nyf, nys, steps in ((300, 200, 10, 37), (70, 33, 4, 12)):
        print(f"noalloc read: {nx}x{nyf}+{nys} precision {precision}, {steps} steps", flush=True)
        P, d, bc, rho, T = pool_case(nx, nyf, nys, superheat=0.15, n_spots=3, seed=nx)
        dom = gpu_domain(P, bc, rho, T, precision)
        dom.step(steps)
        a = _read_abi(dom, noalloc=True)
        b = _read_abi(dom, noalloc=False)
        c = _read_abi(dom, noalloc=True)
        for k in ("rho", "ux", "uy", "T", "f"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)
            np.testing.assert_array_equal(c[k], b[k], err_msg=k)
        assert np.isfinite(a["f"]).all() and a["rho"].min() > 0
        dom.step(3)
        e = _read_abi(dom, noalloc=True)
        assert not np.array_equal(e["f"], a["f"])
        np.testing.assert_array_equal(e["T"], _read_abi(dom, noalloc=False)["T"])
        dom.close()


def test_noalloc_read_refuses_domains_beyond_the_fixed_staging():
    from paper_1911_10747_amd import poolboil as pb
    P, d, bc, rho, T = pool_case(1024, 700, 4, superheat=0.1, n_spots=0)
    dom = gpu_domain(P, bc, rho, T, 1)
    out = np.empty((700, 1024))
    rc = pb.lib.pb_read_fields_noalloc(dom.handle, out.ctypes.data_as(C.POINTER(C.c_double)), None, None, None, None)
    assert rc == pb.PB_EINVAL
    assert "exceeds" in pb.lib.pb_last_error().decode()
    assert dom.read(with_f=False)["rho"].shape == (700, 1024)
    dom.close()
