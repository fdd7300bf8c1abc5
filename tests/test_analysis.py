"""The contact-angle measurement recovers the geometry of synthetic density
fields built from known circles (tanh profiles), independently of any
lattice Boltzmann run."""
import numpy as np
import pytest

from paper_1908_04443_amd import analysis as A

RG, RL = 0.38, 6.5


def _cap(shape, center, r, width=3.0):
    ny, nx = shape
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    d = np.hypot(x - center[0], y - center[1])
    return 0.5 * (RL + RG) - 0.5 * (RL - RG) * np.tanh(2.0 * (d - r) / width)


def test_fit_circle_exact_points():
    t = np.linspace(0.2, 2.5, 40)
    pts = np.stack([3.0 + 7.5 * np.cos(t), -2.0 + 7.5 * np.sin(t)], axis=1)
    cx, cy, r = A.fit_circle(pts)
    assert abs(cx - 3.0) < 1e-9 and abs(cy + 2.0) < 1e-9 and abs(r - 7.5) < 1e-9


def test_angle_between_circles_limits():
    assert abs(A.angle_between_circles(3.0, 4.0, 5.0) - 90.0) < 1e-9
    assert abs(A.angle_between_circles(3.0, 4.0, 7.0) - 180.0) < 1e-6
    assert abs(A.angle_between_circles(3.0, 4.0, 1.0) - 0.0) < 1e-6


@pytest.mark.parametrize("theta", [35.0, 90.0, 125.0])
def test_flat_wall_angle_of_synthetic_cap(theta):
    ny, nx, r, wall_y = 90, 160, 28.0, 3.5
    cy = wall_y - r * np.cos(np.radians(theta))
    rho = _cap((ny, nx), (80.0, cy), r)
    solid = np.zeros((ny, nx), np.uint8)
    solid[0:4, :] = 1
    rho[solid == 1] = 0.0
    th, _ = A.contact_angle_flat(rho, solid, wall_y, RG, RL)
    assert abs(th - theta) < 1.0


@pytest.mark.parametrize("theta", [40.0, 90.0, 130.0])
def test_cylinder_angle_of_synthetic_droplet(theta):
    ny, nx, Rn, r = 260, 240, 40, 30.0
    c = (120.0, 110.0)
    Rw = Rn + 0.5
    # centre distance that makes the two circles meet at theta
    d = np.sqrt(r * r + Rw * Rw - 2.0 * r * Rw * np.cos(np.radians(theta)))
    rho = _cap((ny, nx), (c[0], c[1] + d), r)
    y, x = np.mgrid[0:ny, 0:nx]
    solid = (((x - c[0]) ** 2 + (y - c[1]) ** 2) <= Rn * Rn).astype(np.uint8)
    rho[solid == 1] = 0.0
    th, _ = A.contact_angle_cylinder(rho, solid, c, Rn, RG, RL)
    assert abs(th - theta) < 1.0


def test_fit_sphere_exact_points():
    rng = np.random.default_rng(3)
    v = rng.normal(size=(200, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    pts = np.array([1.0, -2.0, 0.5]) + 9.0 * v
    cx, cy, cz, r = A.fit_sphere(pts)
    assert max(abs(cx - 1.0), abs(cy + 2.0), abs(cz - 0.5), abs(r - 9.0)) < 1e-9


@pytest.mark.parametrize("theta", [50.0, 120.0])
def test_sphere_angle_of_synthetic_droplet(theta):
    n, Rn, r = 96, 20, 16.0
    c = (48.0, 48.0, 40.0)
    Rw = Rn + 0.5
    d = np.sqrt(r * r + Rw * Rw - 2.0 * r * Rw * np.cos(np.radians(theta)))
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(float)
    dd = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2] - d) ** 2)
    rho = 0.5 * (RL + RG) - 0.5 * (RL - RG) * np.tanh(2.0 * (dd - r) / 3.0)
    solid = (((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) <= Rn * Rn).astype(np.uint8)
    rho[solid == 1] = 0.0
    th, _ = A.contact_angle_sphere(rho, solid, c, Rn, RG, RL)
    assert abs(th - theta) < 1.0
