"""Pins of the oracle's geometric formulation (Sec. III A, Eqs. 11, 13-15)
and a CPU comparison of the library's stencil builder with it.

The oracle finds each characteristic point D_k as the nearest positive
crossing of the ray from the wall node P along n_k with the four mesh lines
that bound the 3 x 3 block around P, and interpolates rho at D_k from its
position.  The library builds integer stencil codes by a different route
(it decides between the vertical and the horizontal line first).  These
tests pin the oracle to what the construction must satisfy, independently of
how it is coded, and compare the two constructions point by point:

- the normal of Eqs. 13-14 is exact on flat walls and close to radial on a
  staircase circle;
- every D_k lies on the boundary of the 3 x 3 block, on the ray turned by
  +-(90 deg - theta_a) from the normal, at the first crossing found by
  marching along the ray (brute force);
- a linear density field is interpolated exactly, and the max / min rule of
  Eq. 11 picks the right point;
- a ray through a corner of the block (a tie between a vertical and a
  horizontal line) lands on the corner node, so no tie rule is needed;
- the noise-free 128 x 128 cylinder / droplet case stays mirror-symmetric
  about x = N_x / 2 under the geometric formulation;
- the library's stencils (host query) hold the same nodes and weights as the
  oracle's points, for random geometries and angles.
"""
import numpy as np
import pytest

from paper_1908_04443_amd import inputs as I
from paper_1908_04443_amd import workloads as W

SNAP = 1e-12  # a stencil node closer than this to D is D itself


def _params(O, nx, ny):
    return O.make_params(nx=nx, ny=ny, T_ratio=0.75, sigma=0.105, scheme=O.GF)


def _random_geometry(nx, ny, seed):
    """Disks of seeded centres and radii, a rectangle (convex corners) and
    a notch cut into it (concave corners)."""
    rng = np.random.default_rng(seed)
    solid = np.zeros((ny, nx), np.uint8)
    for _ in range(5):
        c = (rng.uniform(0, nx), rng.uniform(0, ny))
        solid |= I.disk_mask((ny, nx), c, rng.uniform(2.5, 9.0))
    x0, y0 = int(rng.integers(2, nx // 2)), int(rng.integers(2, ny // 2))
    solid[y0:y0 + 9, x0:x0 + 13] = 1
    solid[y0 + 3:y0 + 6, x0 + 4:x0 + 7] = 0
    return solid


def _stencil_from_point(D):
    """Nodes of the bilinear stencil of D with weight >= SNAP."""
    i0, j0 = int(np.floor(D[0])), int(np.floor(D[1]))
    out = []
    for j in (j0, j0 + 1):
        for i in (i0, i0 + 1):
            w = (1.0 - abs(D[0] - i)) * (1.0 - abs(D[1] - j))
            if w >= SNAP:
                out.append(((i, j), w))
    return out


def _fluid_at(solid, P, off):
    ny, nx = solid.shape
    return solid[(P[1] + off[1]) % ny, (P[0] + off[0]) % nx] == 0


def test_gf_normal_flat_walls_and_circle(oracle_mod):
    O = oracle_mod
    nx, ny = 24, 20
    solid = np.zeros((ny, nx), np.uint8)
    solid[0:5, :] = 1  # periodic: row 4 faces +y, row 0 faces -y
    p = _params(O, nx, ny)
    walls = O.wall_nodes(p, solid)
    g = O.gf_points(p, solid, 90.0)
    wy = walls // nx
    # exact up to the rounding of the weighted sums
    assert np.allclose(g[wy == 4, 0], np.tile([0.0, 1.0], (nx, 1)), rtol=0, atol=1e-15)
    assert np.allclose(g[wy == 0, 0], np.tile([0.0, -1.0], (nx, 1)), rtol=0, atol=1e-15)
    # a 45-degree staircase: the normals lie on the lattice diagonals
    n = 40
    yy, xx = np.mgrid[0:n, 0:n]
    solid = ((np.abs(xx - 20) + np.abs(yy - 20)) <= 9).astype(np.uint8)
    p = _params(O, n, n)
    walls = O.wall_nodes(p, solid)
    g = O.gf_points(p, solid, 90.0)
    wy, wx = np.divmod(walls, n)
    edge = (np.abs(wx - 20) > 2) & (np.abs(wy - 20) > 2)
    diag = np.stack([np.sign(wx - 20), np.sign(wy - 20)], 1) / np.sqrt(2.0)
    assert np.allclose(g[edge, 0], diag[edge], rtol=0, atol=1e-15)
    # a staircase circle: node by node the normal of the discrete gradient
    # of the solid indicator departs from the radial direction by up to
    # about 20 degrees (the steps), but the departures cancel around the
    # circle, whose staircase has the lattice's symmetries
    n, R = 96, 17
    c = (48, 47)
    solid = I.disk_mask((n, n), c, R)
    p = _params(O, n, n)
    walls = O.wall_nodes(p, solid)
    g = O.gf_points(p, solid, 90.0)
    wy, wx = np.divmod(walls, n)
    radial = np.stack([wx - c[0], wy - c[1]], 1).astype(float)
    radial /= np.linalg.norm(radial, axis=1)[:, None]
    cosang = (g[:, 0] * radial).sum(1)
    signed = radial[:, 0] * g[:, 0, 1] - radial[:, 1] * g[:, 0, 0]
    ang = np.degrees(np.arccos(np.clip(cosang, -1, 1)))
    print(f"circle R = {R}: normal vs radial max {ang.max():.2f} deg, mean {ang.mean():.2f}")
    assert ang.max() < 25.0 and ang.mean() < 12.0
    assert abs(signed.sum()) < 1e-12


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gf_points_lie_on_the_rays_at_the_first_mesh_line(oracle_mod, seed):
    O = oracle_mod
    nx, ny = 56, 48
    solid = _random_geometry(nx, ny, seed)
    p = _params(O, nx, ny)
    walls = O.wall_nodes(p, solid)
    rng = np.random.default_rng(100 + seed)
    theta = rng.uniform(15.0, 165.0, len(walls))
    theta[::7] = 90.0
    g = O.gf_points(p, solid, theta)
    ok = np.isfinite(g[:, 0, 0])
    assert ok.mean() > 0.9
    n = g[ok, 0]
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-14)
    turn = 90.0 - theta[ok]
    for k, sign in ((1, 1.0), (2, -1.0)):
        D = g[ok, k]
        # on the boundary of the 3 x 3 block around the wall node
        assert np.allclose(np.abs(D).max(1), 1.0, atol=1e-12)
        # on the ray turned by +-(90 deg - theta_a) from the normal (Eq. 15)
        cross = n[:, 0] * D[:, 1] - n[:, 1] * D[:, 0]
        dot = (n * D).sum(1)
        assert np.allclose(np.degrees(np.arctan2(cross, dot)), sign * turn, atol=1e-9)
        # the first mesh line crossed: march along the ray in steps of 1e-4
        u = D / np.linalg.norm(D, axis=1)[:, None]
        t = np.arange(1, 30001) * 1e-4
        inside = np.abs(u[:, None, :] * t[None, :, None]).max(2) < 1.0
        t_first = t[np.argmin(inside, axis=1)]
        assert np.all(np.abs(t_first - np.linalg.norm(D, axis=1)) <= 1.01e-4)


@pytest.mark.parametrize("theta", [35.0, 90.0, 140.0])
def test_gf_linear_density_is_interpolated_exactly(oracle_mod, theta):
    """rho = a + b x + c y on the fluid nodes: a point whose two stencil
    nodes are fluid carries a + b x_D + c y_D, a point with one fluid node
    that node's density, and the wall node the max (theta_a <= 90 deg) or
    the min of its points (Eq. 11)."""
    O = oracle_mod
    nx, ny = 56, 48
    solid = _random_geometry(nx, ny, 7)
    p = _params(O, nx, ny)
    walls = O.wall_nodes(p, solid)
    g = O.gf_points(p, solid, theta)
    yy, xx = np.mgrid[0:ny, 0:nx]
    a, b, c = 0.12, 0.0013, -0.0021
    lin = a + b * xx + c * yy
    rho = np.where(solid == 0, lin, 0.0)
    f = O.init_eq(p, solid, rho)
    rw, _, _ = O.fields(p, solid, f, np.full(len(walls), theta), None)
    checked = 0
    for k, w in enumerate(walls):
        P = (w % nx, w // nx)
        if not (3 <= P[0] < nx - 3 and 3 <= P[1] < ny - 3) or not np.isfinite(g[k, 0, 0]):
            continue  # the linear field jumps across the periodic seam
        vals = []
        for D in (g[k, 1], g[k, 2]):
            st = [(o, wt) for o, wt in _stencil_from_point(D) if _fluid_at(solid, P, o)]
            if len(st) == 2 or (len(st) == 1 and len(_stencil_from_point(D)) == 1):
                vals.append(a + b * (P[0] + D[0]) + c * (P[1] + D[1]))
            elif len(st) == 1:
                o = st[0][0]
                vals.append(lin[P[1] + o[1], P[0] + o[0]])
        if len(vals) < 2:
            continue
        want = min(vals) if theta > 90.0 else max(vals)
        assert abs(rw[w] - want) <= 1e-14, (P, vals, rw[w])
        checked += 1
    assert checked > 100


def test_gf_corner_crossings_need_no_tie_rule(oracle_mod):
    """A 45-degree staircase at theta_a = 90 deg: the normals point along a
    diagonal of the lattice, so each ray meets a vertical and a horizontal
    line of the block at the same corner.  Whichever line is taken, D is the
    corner node; the oracle puts D on it to rounding and its stencil is that
    node alone."""
    O = oracle_mod
    n = 40
    yy, xx = np.mgrid[0:n, 0:n]
    solid = ((np.abs(xx - 20) + np.abs(yy - 20)) <= 9).astype(np.uint8)  # a diamond
    p = _params(O, n, n)
    walls = O.wall_nodes(p, solid)
    g = O.gf_points(p, solid, 90.0)
    wy, wx = np.divmod(walls, n)
    edge = (np.abs(wx - 20) + np.abs(wy - 20) == 9) & (wx != 20) & (wy != 20) & \
        (np.abs(wx - 20) > 2) & (np.abs(wy - 20) > 2)
    assert edge.sum() >= 16
    for k in np.flatnonzero(edge):
        corner = np.array([np.sign(wx[k] - 20), np.sign(wy[k] - 20)], float)
        for D in (g[k, 1], g[k, 2]):
            assert np.abs(D - corner).max() < 1e-12
            st = _stencil_from_point(D)
            assert len(st) == 1 and st[0][0] == tuple(int(v) for v in corner)


def _mirror(a, nx):
    return a[:, (nx - np.arange(nx)) % nx]


@pytest.mark.parametrize("theta", [60.0, 120.0])
def test_gf_mirror_symmetry_noise_free_cylinder(oracle_mod, theta):
    """The 128 x 128 cylinder (R = 24) with a droplet (r = 20) on top, no
    noise, is mirror-symmetric about x = N_x / 2 (the line of Fig. 7); the
    geometric formulation keeps it so (max / min, both points, the normal)."""
    O = oracle_mod
    n = 128
    p = _params(O, n, n)
    d = W.c0_cylinder(p.rho_g, p.rho_l, noise=0.0)
    solid = d["solid"]
    walls = O.wall_nodes(p, solid)
    th = np.full(len(walls), theta)
    f = O.run(p, solid, O.init_eq(p, solid, d["rho"]), 600, th, None)
    rho, u, _ = O.fields(p, solid, f, th, None)
    rho = rho.reshape(n, n)
    ux = u[0].reshape(n, n)
    e_rho = np.abs(rho - _mirror(rho, n)).max()
    e_u = np.abs(ux + _mirror(ux, n)).max()
    print(f"theta_a {theta}: mirror |rho| {e_rho:.2e}, |ux| {e_u:.2e}")
    assert e_rho <= 1e-13 and e_u <= 1e-13


def _lib_params(L, O, p):
    q = L.lbm_params()
    q.lattice, q.precision, q.nx, q.ny, q.nz, q.eos = 9, 8, p.nx, p.ny, 1, p.eos
    for i in range(19):
        q.tau[i] = p.tau[i]
    q.eos_a, q.eos_b, q.eos_R, q.eos_T, q.eos_omega = p.eos_a, p.eos_b, p.eos_R, p.eos_T, p.eos_omega
    q.G, q.sigma, q.rho_g, q.rho_l = p.G, p.sigma, p.rho_g, p.rho_l
    return q


@pytest.mark.parametrize("case", ["random1", "random2", "diamond90", "circle"])
def test_library_gf_stencils_match_oracle_points(oracle_mod, case):
    """Host query of the library's stencils against the oracle's points: the
    same fluid nodes with the same weights (1e-12) for every point of every
    wall node, and the same void points.  The two codes locate D by
    different constructions."""
    from paper_1908_04443_amd import lbm as L
    O = oracle_mod
    if case.startswith("random"):
        nx, ny = 56, 48
        solid = _random_geometry(nx, ny, 11 if case == "random1" else 12)
        rng = np.random.default_rng(3)
    elif case == "diamond90":
        nx = ny = 40
        yy, xx = np.mgrid[0:ny, 0:nx]
        solid = ((np.abs(xx - 20) + np.abs(yy - 20)) <= 9).astype(np.uint8)
        rng = None
    else:
        nx = ny = 96
        solid = I.disk_mask((ny, nx), (48, 47), 30)
        rng = np.random.default_rng(5)
    p = _params(O, nx, ny)
    walls = O.wall_nodes(p, solid)
    theta = np.full(len(walls), 90.0) if rng is None else rng.uniform(10.0, 170.0, len(walls))
    g = O.gf_points(p, solid, theta)
    nodes, wts = L.lbm_gf_stencils(_lib_params(L, O, p), solid, theta)
    assert len(nodes) == len(walls)
    voids = 0
    for k, w in enumerate(walls):
        P = (w % nx, w // nx)
        for j in range(2):
            lib_st = {tuple(nodes[k, j, i]): wts[k, j, i] for i in range(2) if wts[k, j, i] > 0}
            if not np.isfinite(g[k, 0, 0]):
                assert not lib_st
                continue
            st = [(o, wt) for o, wt in _stencil_from_point(g[k, 1 + j])
                  if _fluid_at(solid, P, o)]
            tot = sum(wt for _, wt in st)
            want = {o: wt / tot for o, wt in st}
            voids += not want
            assert set(lib_st) == set(want), (case, P, j, lib_st, want)
            for o in want:
                assert abs(lib_st[o] - want[o]) <= 1e-12
    print(f"{case}: {len(walls)} wall nodes, {voids} void points")
