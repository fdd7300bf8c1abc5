"""Synthetic workloads of the benchmark and the parity tests.

Each builder returns geometry, initial density and per-node wetting
parameters for a lattice; thermodynamic constants (T, rho_g, rho_l) are
passed in by the caller so that the same builder can feed the GPU library
(constants from its EOS helpers) or the oracle (constants from the oracle).

  c0_cylinder    D2Q9 128^2 FP64: cylinder R = 24 at the centre, droplet
                 r = 20 (tanh width 3) tangent on top, +-1e-6 noise (seed 0),
                 improved virtual density at PHI_C0_60
  c1_porous      D2Q9 2048^2 FP32: 400 non-overlapping periodic cylinders,
                 radii U[8, 32] (dart throwing, seed 1), one prescribed
                 angle per cylinder U[30, 150] deg, 50/50 liquid/gas blobs
  c2_sphere      D3Q19 256^3 FP32: sphere R = 40 at the centre, droplet
                 r = 30 tangent on top, standard case (phi = 1)
  c3_cases       96 D2Q9 cases, n ~ U{128..768}, one cylinder each
  c4_adjoint     D2Q9 256^2: cylinder R = 40, droplet r = 32 on top
"""
import numpy as np

from . import inputs as I

# Prescribed angle -> (phi, drho) of the improved virtual-density scheme for
# the Carnahan-Starling fluid at 0.75 Tc (tau = 1, sigma = 0.1071): static
# angles of droplets on a flat wall measured with the CPU oracle
# (tests/golden/calibrate_angles.py, angle_calibration_cs075.json).  Angles
# below the standard case (phi = 1, drho = 0: 84.66 deg) use phi > 1, above
# it drho > 0 (Sec. III B); 20 and 160 deg extend the end segments.
ANGLE_TABLE_CS075 = {
    "theta": [20.0, 30.0, 45.0, 60.0, 75.0, 84.66, 90.0, 105.0, 120.0, 135.0, 150.0, 160.0],
    "phi": [1.9097, 1.7636, 1.5401, 1.3001, 1.1013, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0],
    "drho": [0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.00421, 0.01596, 0.02799, 0.03774, 0.04608, 0.05139],
}

# sigma of Eq. 7 per (EOS, T/Tc, lattice), from the flat-slab calibration in
# tests/golden/calibrate_sigma.py (gas density of a slab = Maxwell value).
SIGMA = {("cs", 0.75, 9): 0.1071, ("pr", 0.86, 9): 0.1115, ("cs", 0.8, 19): 0.1067}


# phi of the improved scheme for the 60 deg target on the 128^2 cylinder
# (R = 24), measured on that cylinder with the CPU oracle
# (tests/golden/calibrate_c0.py, c0_calibration.json).  The flat-wall table
# gives 1.3001, which settles at 51.1 deg there.  The settled angle is not
# continuous in phi on this staircase: 63.6 deg at phi = 1.2212, 57.3 deg
# at 1.2326 (the contact line rests on the next stair step), so 60 deg
# itself is not reached; 1.2326 is the closest settled angle below it.
PHI_C0_60 = 1.2326


def c0_cylinder(rho_g, rho_l, phi=None, drho=None, n=128, R=24, r0=20, noise=1e-6, seed=0):
    shape = (n, n)
    solid = I.disk_mask(shape, (n // 2, n // 2), R)
    rho = I.droplet_rho(shape, (n // 2, n // 2 + R + r0), r0, rho_g, rho_l, width=3.0, solid=solid)
    if noise:
        rho = I.add_noise(rho, noise, seed, solid=solid)
    if phi is None:
        phi, drho = PHI_C0_60, 0.0
    return dict(shape=shape, solid=solid, rho=rho,
                phi=np.full(shape, float(phi)), drho=np.full(shape, float(drho)))


def c1_porous(rho_g, rho_l, n=2048, count=400, rmin=8.0, rmax=32.0, seed=1):
    cyl = I.poisson_disk_cylinders(n, count, rmin, rmax, seed)
    solid, label = I.cylinders_mask(n, cyl)
    theta = I.uniform(seed, 40, count, 30.0, 150.0)
    ph, dr = I.angle_to_params(theta, ANGLE_TABLE_CS075)
    phi, drho = I.param_field(label, ph, dr)
    rho = I.blob_rho((n, n), seed, rho_g, rho_l, solid=solid)
    return dict(shape=(n, n), solid=solid, rho=rho, phi=phi, drho=drho, theta=theta, cyl=cyl)


def c2_sphere(rho_g, rho_l, n=256, R=40, r0=30, phi=1.0, drho=0.0):
    shape = (n, n, n)
    c = n // 2
    solid = I.disk_mask(shape, (c, c, c), R)
    rho = I.droplet_rho(shape, (c, c, c + R + r0), r0, rho_g, rho_l, width=3.0, solid=solid)
    return dict(shape=shape, solid=solid, rho=rho,
                phi=np.full(shape, float(phi)), drho=np.full(shape, float(drho)))


def c3_cases(rho_g, rho_l, count=96, seed0=1000, nmin=128, nmax=768):
    cases = []
    for i in range(count):
        s = seed0 + i
        u = I.uniform(s, 50, 4)
        n = int(nmin + np.floor(u[0] * (nmax - nmin + 1)))
        R = int(round((0.1 + 0.2 * u[1]) * n))
        r0 = (0.6 + 0.4 * u[2]) * R
        r0 = min(r0, (n - 8) / 2.0 - R)  # keep the droplet off the periodic image
        theta = 20.0 + 140.0 * u[3]
        ph, dr = I.angle_to_params(theta, ANGLE_TABLE_CS075)
        shape = (n, n)
        solid = I.disk_mask(shape, (n // 2, n // 2), R)
        rho = I.droplet_rho(shape, (n // 2, n // 2 + R + r0), r0, rho_g, rho_l, solid=solid)
        cases.append(dict(shape=shape, solid=solid, rho=rho, phi=np.full(shape, float(ph)),
                          drho=np.full(shape, float(dr)), theta=theta, n=n, R=R, r0=r0))
    return cases


def c4_adjoint(rho_g, rho_l, n=256, R=40, r0=32):
    shape = (n, n)
    solid = I.disk_mask(shape, (n // 2, n // 2), R)
    rho = I.droplet_rho(shape, (n // 2, n // 2 + R + r0), r0, rho_g, rho_l, solid=solid)
    return dict(shape=shape, solid=solid, rho=rho, phi=np.ones(shape), drho=np.zeros(shape))


def c4_target_params(solid, n, seed=4):
    """Per-node angle 90 + 50 g(beta) deg (beta: polar angle about the
    centre, g a seeded smooth 4-mode profile with max |g| = 1) mapped to
    (phi, drho) by the calibration table."""
    coef = I.smooth_angle_profile(seed)
    ys, xs = np.mgrid[0:n, 0:n]
    beta = np.arctan2(ys - n // 2, xs - n // 2)
    theta = 90.0 + 50.0 * I.eval_angle_profile(coef, beta.ravel()).reshape(n, n)
    ph, dr = I.angle_to_params(theta, ANGLE_TABLE_CS075)
    return np.where(solid != 0, ph, 1.0), np.where(solid != 0, dr, 0.0)
