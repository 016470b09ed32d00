"""Pin of the oracle's contact-angle measurement (the paper does not state
how its angles of Sec. III C were measured; the reading here: the
(rho_l + rho_v)/2 isoline in the central x-z and y-z planes, a circle fit to
its points more than 3 lattice units above the wall plane z = 0.5, and
cos(theta) = (0.5 - z_c)/R).  Synthetic sessile caps with a known angle: a
tanh profile of width 5 (the paper's initial-interface form, Eqs.
(34)-(35)) around a sphere whose centre sits at z_c = 0.5 - R cos(theta), so
that the sphere meets the wall plane at theta.  The isoline of such a field
is the sphere itself, so the measurement must return theta; a wrong sign of
cos, a wrong wall plane or a point set cut at the wrong height moves it by
degrees."""
import math

import numpy as np
import pytest

from oracle import eos, phys

A, B, R = eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"]
RL, RV = eos.maxwell(A, B, R, eos.temperature(0.7))


def cap(shape, theta_deg, radius, width=5.0, z_wall=0.5):
    nz, ny, nx = shape
    zc = z_wall - radius * math.cos(math.radians(theta_deg))
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r0 = np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - zc) ** 2)
    rho = 0.5 * (RL + RV) - 0.5 * (RL - RV) * np.tanh(2 * (r0 - radius) / width)
    rho[0] = RV  # the solid plane (ignored by the measurement)
    return rho


def volume_matched_radius(theta_deg, r_hemisphere=30.0):
    """Radius of the spherical cap with contact angle theta that holds the
    liquid of a hemisphere of radius 30 (the initial droplet of Sec. III C):
    V = pi R^3 (2 - 3 cos theta + cos^3 theta) / 3."""
    c = math.cos(math.radians(theta_deg))
    v = 2.0 / 3.0 * math.pi * r_hemisphere ** 3
    return (3 * v / (math.pi * (2 - 3 * c + c ** 3))) ** (1.0 / 3.0)


@pytest.mark.parametrize("theta", [30.0, 33.5, 60.0, 89.9, 90.0, 120.0, 150.0, 153.4])
def test_contact_angle_of_volume_matched_caps(theta):
    Rc = volume_matched_radius(theta)
    th, zc, Rf = phys.contact_angle(cap((64, 160, 160), theta, Rc), RL, RV)
    assert abs(th - theta) < 0.5, (theta, th, Rc, Rf)
    assert abs(Rf - Rc) < 0.05 * Rc


@pytest.mark.parametrize("theta", [30.0, 60.0, 90.0, 120.0, 150.0])
def test_contact_angle_of_radius_30_caps(theta):
    # caps of the initial droplet's radius (at 30 degrees only the top unit of
    # the cap lies above the fit's cut-off, 3 units over the wall plane)
    th, zc, Rf = phys.contact_angle(cap((64, 128, 128), theta, 30.0), RL, RV)
    assert abs(th - theta) < 0.5, (theta, th)


def test_contact_angle_reads_the_bottom_wall_and_its_sign():
    # a hydrophobic cap (150 deg) and a hydrophilic one (30 deg) of equal
    # volume: the measured angles straddle 90 degrees in the right order, and
    # the fitted centre lies below the wall plane for the hydrophilic cap
    lo = phys.contact_angle(cap((64, 160, 160), 30.0, volume_matched_radius(30.0)), RL, RV)
    hi = phys.contact_angle(cap((64, 160, 160), 150.0, volume_matched_radius(150.0)), RL, RV)
    assert lo[0] < 90.0 < hi[0]
    assert lo[1] < 0.5 < hi[1]
