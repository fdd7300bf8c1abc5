"""Physics pins of the CPU oracle: results the paper and the mathematics fix
for whole simulations, not single formulas.

* Coexistence (Sec. II A, Eq. 6 with the Eq. 7 sigma term): a flat slab
  relaxes to the Maxwell-construction densities of the EOS.  Only the gas
  side is tuned through sigma; the liquid side is an independent check.
* Laplace law: the pressure jump across a free droplet or bubble is
  gamma / R with one surface tension for droplets and bubbles.
* Static contact angle on a flat wall with the improved virtual-density
  scheme (Eqs. 16-17): the standard case phi = 1 gives about 90 deg
  (Sec. III B), phi > 1 lowers and drho > 0 raises the angle, to the
  values of Fig. 5 within the tolerance stated below.
* Poiseuille flow between plates (Sec. IV B): analytic profile with the
  improved scheme, thick mass-transfer layer with the constant one.

Pressures are the EOS pressures of the bulk densities (in the bulk the
pseudopotential model reproduces p_EOS, Eq. 6).
"""
import numpy as np
import pytest

from cases import SIGMA_CAL, SIGMA_CS075, SIGMA_PR086
from paper_1908_04443_amd import analysis as A
from paper_1908_04443_amd import inputs as I

pytestmark = pytest.mark.slow


def _slab(O, key):
    cal = SIGMA_CAL[key]
    nx, ny = cal["slab"]
    kw = dict(eos=O.EOS_PR, a=2.0 / 49.0, b=2.0 / 21.0) if key.startswith("pr") else {}
    Tr = 0.86 if key.startswith("pr") else 0.75
    p = O.make_params(nx=nx, ny=ny, T_ratio=Tr, sigma=cal["sigma"], **kw)
    solid = np.zeros((ny, nx), np.uint8)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    H = 0.5 * (np.tanh((y - ny / 4) / 2.0) - np.tanh((y - 3 * ny / 4) / 2.0))
    f = O.run(p, solid, O.init_eq(p, solid, p.rho_g + (p.rho_l - p.rho_g) * H), cal["steps"])
    rho, _, _ = O.fields(p, solid, f)
    return p, rho


@pytest.mark.parametrize("key", ["cs_0.75", "pr_0.86"])
def test_slab_coexistence_matches_maxwell(oracle_mod, key):
    p, rho = _slab(oracle_mod, key)
    # gas side: set by the sigma calibration (stored value rounded to 1e-4)
    assert abs(rho.min() / p.rho_g - 1.0) < 5e-3
    # liquid side: not tuned; sigma only moves it by parts in 1e4
    assert abs(rho.max() / p.rho_l - 1.0) < 1e-3


def _free_drop(O, n, r0, bubble, steps=8000):
    p = O.make_params(nx=n, ny=n, T_ratio=0.75, sigma=SIGMA_CS075)
    solid = np.zeros((n, n), np.uint8)
    c = (n / 2.0, n / 2.0)
    rho = I.droplet_rho((n, n), c, r0, p.rho_g, p.rho_l)
    if bubble:
        rho = p.rho_g + p.rho_l - rho
    f = O.run(p, solid, O.init_eq(p, solid, rho), steps)
    r, _, _ = O.fields(p, solid, f)
    r = r.reshape(n, n)
    cx, cy, R = A.fit_circle(A.interface_points(r, A.droplet_level(p.rho_g, p.rho_l)))
    inner, outer = A.bulk_densities(r, c, R - 6.0, R + 10.0)
    dp = O.eos_p(p, inner) - O.eos_p(p, outer)
    return R, dp  # p_in - p_out > 0 for droplets and bubbles alike


def test_laplace_law_droplets_and_bubble(oracle_mod):
    """dp = gamma / R: a linear fit of dp against 1/R over R = 8..18 has a
    small intercept, dp * R is constant to within the finite-interface-width
    drift (about 6 % over this range), and a bubble of the same radius has
    a positive jump of the same size.  With interfaces a few nodes wide the
    effective tension depends on the sign of the curvature (a Tolman-type
    correction of order width / R, about 8 % each way at R = 15), so the
    bubble is held to 20 %."""
    n = 64
    pts = [_free_drop(oracle_mod, n, r0, False) for r0 in (9.0, 12.0, 15.0, 18.0)]
    R = np.array([q[0] for q in pts])
    dp = np.array([q[1] for q in pts])
    assert np.all(dp > 0)
    gamma, c0 = np.polyfit(1.0 / R, dp, 1)
    fit = gamma / R + c0
    r2 = 1.0 - ((dp - fit) ** 2).sum() / ((dp - dp.mean()) ** 2).sum()
    assert r2 > 0.995
    assert abs(c0) < 0.15 * dp.min()
    g = dp * R
    assert g.max() / g.min() - 1.0 < 0.10
    Rb, dpb = _free_drop(oracle_mod, n, 15.0, True)
    assert dpb > 0
    assert abs(dpb * Rb / (dp[2] * R[2]) - 1.0) < 0.20


def _flat_angle(O, phi, drho, steps):
    nx, ny, r0 = 160, 80, 25.0
    tau = [1.0] * 9
    tau[7] = tau[8] = 0.95  # nu = 0.15, as in Sec. IV A
    p = O.make_params(nx=nx, ny=ny, eos=O.EOS_PR, a=2.0 / 49.0, b=2.0 / 21.0, T_ratio=0.86,
                      sigma=SIGMA_PR086, tau=tau, scheme=O.IVD)
    solid = np.zeros((ny, nx), np.uint8)
    solid[0:4, :] = 1  # wall rows; the surface is at y = 3.5 (halfway bounce-back)
    rho = I.droplet_rho((ny, nx), (nx / 2.0, 4.0 + 0.6 * r0), r0, p.rho_g, p.rho_l, solid=solid)
    nw = len(O.wall_nodes(p, solid))
    ph, dr = np.full(nw, phi), np.full(nw, drho)
    f = O.run(p, solid, O.init_eq(p, solid, rho), steps, ph, dr)
    r, _, _ = O.fields(p, solid, f, ph, dr)
    th, _ = A.contact_angle_flat(r.reshape(ny, nx), solid, 3.5, p.rho_g, p.rho_l,
                                 select=lambda x, y: y < ny - 4)
    return th


def test_flat_wall_contact_angles_improved_virtual_density(oracle_mod):
    """PR at 0.86 Tc, nu = 0.15 (Sec. IV A), droplet r = 25 on a flat wall.
    phi = 1 is the standard case (about 90 deg, Sec. III B); phi = 1.4 and
    drho = 0.5 are the parameters of Fig. 5(a) and 5(c) (34 and 125 deg on
    the cylinder).  The flat-wall angles must fall within 8 deg of those
    values: the paper reads its angles off images, does not state sigma or
    the non-viscous relaxation times, and the flat and curved walls differ
    in staircase detail."""
    th1 = _flat_angle(oracle_mod, 1.0, 0.0, 6000)
    th_lo = _flat_angle(oracle_mod, 1.4, 0.0, 12000)
    th_hi = _flat_angle(oracle_mod, 1.0, 0.5, 6000)
    print(f"flat-wall angles: phi=1 {th1:.2f}  phi=1.4 {th_lo:.2f}  drho=0.5 {th_hi:.2f}")
    assert abs(th1 - 90.0) < 5.0
    assert abs(th_lo - 34.0) < 8.0
    assert abs(th_hi - 125.0) < 8.0
    assert th_lo < th1 < th_hi


def _poiseuille_error(O, scheme, phi=1.0, drho=0.0, rho_w=0.0, steps=30000):
    """Liquid-filled channel between two plates L = 80 apart (Sec. IV B):
    PR at 0.86 Tc, nu = 1/6 (tau = 1), body force F_b = 1e-5 along x,
    periodic in x.  The plates are single solid rows, so with halfway
    bounce-back they sit at y = 0.5 and y = 80.5.  Returns the paper's
    relative error E_r = sum |u - u_a| / sum |u_a| against
    u_a(y) = F_b L^2 / (2 mu) [(y/L) - (y/L)^2], mu = rho_l nu."""
    nx, L = 4, 80
    ny = L + 2
    p = O.make_params(nx=nx, ny=ny, eos=O.EOS_PR, a=2.0 / 49.0, b=2.0 / 21.0, T_ratio=0.86,
                      sigma=SIGMA_PR086, tau=1.0, body_force=(1e-5, 0.0, 0.0),
                      scheme=O.IVD if scheme == "ivd" else O.VD, rho_w=rho_w)
    solid = np.zeros((ny, nx), np.uint8)
    solid[0, :] = 1
    solid[ny - 1, :] = 1
    nw = len(O.wall_nodes(p, solid))
    ph, dr = np.full(nw, phi), np.full(nw, drho)
    rho = np.where(solid == 0, p.rho_l, 0.0)
    f = O.run(p, solid, O.init_eq(p, solid, rho), steps, ph, dr)
    _, u, _ = O.fields(p, solid, f, ph, dr)
    ux = u.reshape(2, ny, nx)[0, 1:ny - 1, 0]
    y = np.arange(1, ny - 1) - 0.5
    ua = 1e-5 * L * L / (2.0 * p.rho_l / 6.0) * ((y / L) - (y / L) ** 2)
    return float(np.abs(ux - ua).sum() / np.abs(ua).sum())


def test_poiseuille_between_plates(oracle_mod):
    """Sec. IV B, Fig. 12: with the improved virtual density the velocity
    profile matches the analytic Poiseuille profile whatever the wall
    parameter (the paper reports no visible deviation); with the constant
    virtual density close to the gas density a thick mass-transfer layer
    forms at the plates and the profile deviates (relative errors of 7.7 %
    and 22.9 % reported at about 113 and 158 deg).  Here rho_w = 1.5 (about 120 deg on the
    cylinder of Fig. 4c)."""
    O = oracle_mod
    e_ivd = _poiseuille_error(O, "ivd", phi=1.0)
    e_ivd_hi = _poiseuille_error(O, "ivd", drho=0.5)
    e_vd = _poiseuille_error(O, "vd", rho_w=1.5)
    print(f"Poiseuille E_r: IVD phi=1 {e_ivd:.4f}, IVD drho=0.5 {e_ivd_hi:.4f}, VD rho_w=1.5 {e_vd:.4f}")
    assert e_ivd < 2e-3
    assert e_ivd_hi < 1e-2
    assert e_vd > 0.05


def test_d3q19_slab_equals_d2q9_slab(oracle_mod):
    """A flat slab varies along one axis only, where the 3-D model must
    reduce to the 2-D one: the D3Q19 forcing read here (M G of the Guo
    force plus 114 sigma |F_m|^2 / (psi^2 (tau_e - 1/2)) on the energy row)
    reproduces the D2Q9 Eq. 7 density profile of the same slab.  This pins
    the 3-D sigma term against the printed 2-D one."""
    O = oracle_mod
    ny, steps, sig = 64, 4000, SIGMA_PR086
    kw = dict(eos=O.EOS_PR, a=2.0 / 49.0, b=2.0 / 21.0, T_ratio=0.86, sigma=sig, tau=1.0)
    p2 = O.make_params(nx=2, ny=ny, **kw)
    p3 = O.make_params(lattice=19, nx=2, ny=2, nz=ny, **kw)
    y = np.arange(ny, dtype=float)
    H = 0.5 * (np.tanh((y - ny / 4) / 2.0) - np.tanh((y - 3 * ny / 4) / 2.0))
    prof = p2.rho_g + (p2.rho_l - p2.rho_g) * H
    s2 = np.zeros((ny, 2), np.uint8)
    s3 = np.zeros((ny, 2, 2), np.uint8)
    r2, _, _ = O.fields(p2, s2, O.run(p2, s2, O.init_eq(p2, s2, np.repeat(prof[:, None], 2, 1)), steps))
    r3, _, _ = O.fields(p3, s3, O.run(p3, s3, O.init_eq(p3, s3, np.repeat(prof[:, None], 4, 1)
                                                              .reshape(ny, 2, 2)), steps))
    a = r2.reshape(ny, 2)[:, 0]
    b = r3.reshape(ny, 2, 2)[:, 0, 0]
    assert np.abs(a - b).max() < 1e-9 * p2.rho_l


def test_gf_flat_wall_neutral_angle_takes_the_node_above(oracle_mod):
    """Geometric formulation on a flat wall (Sec. III A): the solid normal of
    Eqs. 13-14 is the wall normal, and at theta_a = 90 deg both
    characteristic lines of Eq. 15 run along it, so each wall node takes the
    density of the fluid node directly above it."""
    O = oracle_mod
    nx, ny = 12, 10
    p = O.make_params(nx=nx, ny=ny, T_ratio=0.75, sigma=SIGMA_CS075, scheme=O.GF)
    solid = np.zeros((ny, nx), np.uint8)
    solid[0:4, :] = 1  # periodic in y: row 3 faces up, row 0 faces down
    rng = np.random.default_rng(2)
    rho0 = np.where(solid == 0, 0.05 + 0.25 * rng.random((ny, nx)), 0.0)
    walls = O.wall_nodes(p, solid)
    theta = np.full(len(walls), 90.0)
    f = O.init_eq(p, solid, rho0)
    rho, _, _ = O.fields(p, solid, f, theta, None)
    rho = rho.reshape(ny, nx)
    assert np.array_equal(walls, np.r_[np.arange(nx), np.arange(3 * nx, 4 * nx)])
    assert np.array_equal(rho[3, :], rho[4, :])
    assert np.array_equal(rho[0, :], rho[ny - 1, :])


def _flat_gf_angle(O, theta_a, steps=6000):
    nx, ny, r0 = 160, 80, 25.0
    tau = [1.0] * 9
    tau[7] = tau[8] = 0.95
    p = O.make_params(nx=nx, ny=ny, eos=O.EOS_PR, a=2.0 / 49.0, b=2.0 / 21.0, T_ratio=0.86,
                      sigma=SIGMA_PR086, tau=tau, scheme=O.GF)
    solid = np.zeros((ny, nx), np.uint8)
    solid[0:4, :] = 1
    rho = I.droplet_rho((ny, nx), (nx / 2.0, 4.0 + 0.6 * r0), r0, p.rho_g, p.rho_l, solid=solid)
    th = np.full(len(O.wall_nodes(p, solid)), theta_a)
    f = O.run(p, solid, O.init_eq(p, solid, rho), steps, th, None)
    r, _, _ = O.fields(p, solid, f, th, None)
    ang, _ = A.contact_angle_flat(r.reshape(ny, nx), solid, 3.5, p.rho_g, p.rho_l,
                                  select=lambda x, y: y < ny - 4)
    return ang


def test_gf_flat_wall_reproduces_prescribed_angle(oracle_mod):
    """The geometric formulation makes the interface meet the wall at the
    prescribed angle (Sec. III A); on a flat wall the measured angles of
    theta_a = 60, 90, 120 deg must be within 2 deg of them."""
    for th in (60.0, 90.0, 120.0):
        m = _flat_gf_angle(oracle_mod, th)
        print(f"GF flat wall: theta_a {th:.0f} -> measured {m:.2f}")
        assert abs(m - th) < 2.0
