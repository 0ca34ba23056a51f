"""The contact-angle measurement used to calibrate the wall adhesion of
Eq. 14, checked on synthetic caps of known angle: a disk of radius R whose
centre sits R cos(theta) below the wall plane (half a node under row 0), with
a tanh interface of the width the drops develop."""
import math

import numpy as np
import pytest


def synthetic_cap(theta_deg, R=35.0, nx=240, ny=120, rl=6.5, rv=0.38, width=3.0):
    yc = -0.5 - R * math.cos(math.radians(theta_deg))
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.hypot(x - (nx - 1) / 2.0, y - yc)
    return 0.5 * (rl + rv) - 0.5 * (rl - rv) * np.tanh(2.0 * (r - R) / width), yc


@pytest.mark.parametrize("theta", [35.0, 55.0, 90.0, 105.0, 125.0, 145.0])
def test_angle_of_synthetic_caps(theta):
    from paper_1911_10747_amd import wetting
    rho, yc = synthetic_cap(theta)
    th, (xc, ycf, r) = wetting.cap_contact_angle(rho, 6.5, 0.38)
    assert th == pytest.approx(theta, abs=0.5)
    assert xc == pytest.approx(119.5, abs=0.05)
    assert ycf == pytest.approx(yc, abs=0.3)
    assert r == pytest.approx(35.0, abs=0.3)


def test_no_cap_raises():
    from paper_1911_10747_amd import wetting
    with pytest.raises(ValueError):
        wetting.cap_contact_angle(np.full((40, 60), 0.38), 6.5, 0.38)


def test_jobspec_contact_angle_sets_the_calibrated_gamma():
    from paper_1911_10747_amd import presets
    d = presets.derived()
    spec = presets.JobSpec(nx=32, nyf=20, nys=3, superheat=0.1, contact_angle=55.0)
    bc, rho, T = presets.initial_state(spec, d)
    assert np.all(bc["gamma_bot"] == presets.CONTACT_ANGLE_GAMMA[55.0] * d.psi_L)
    spec = presets.JobSpec(nx=32, nyf=20, nys=3, superheat=0.1)
    assert np.all(presets.initial_state(spec, d)[0]["gamma_bot"] == -0.7 * d.psi_L)
    with pytest.raises(ValueError):
        presets.gamma_for_angle(40.0, d)
