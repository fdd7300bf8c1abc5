"""Host-side post-processing of density fields: liquid-gas interface points,
circle and sphere fits, static contact angles on flat, cylindrical and
spherical walls.

Plain numpy on arrays copied to the host; no lattice Boltzmann arithmetic.
Conventions: a 2-D field is indexed [y, x]; node (x, y) sits at integer
coordinates; with halfway bounce-back the solid surface lies half a lattice
spacing outside the last solid node, so a staircase cylinder of node radius
R (|x - c|^2 <= R^2) has its surface near R + 1/2.

The contact angle is measured through the liquid, as in Figs. 4-6 and 8 of
the paper (static droplets on a cylinder): the free part of the droplet
interface is fitted by a circle, and the angle follows from where that
circle meets the wall.
"""
import numpy as np


def interface_points(rho, level, solid=None, min_wall_dist=0.0, wall_dist=None):
    """Points where rho crosses `level`, by linear interpolation along the x
    and y lattice links between two fluid nodes (no wrap across the domain
    edge).  Points closer than `min_wall_dist` to the wall (per `wall_dist`,
    a callable of (x, y) arrays) are dropped.  Returns an (n, 2) array of
    (x, y)."""
    rho = np.asarray(rho, dtype=np.float64)
    ny, nx = rho.shape
    fluid = np.ones_like(rho, bool) if solid is None else (np.asarray(solid) == 0)
    pts = []
    d = rho - level
    # links along x
    a, b = d[:, :-1], d[:, 1:]
    ok = fluid[:, :-1] & fluid[:, 1:] & (a * b < 0)
    yy, xx = np.nonzero(ok)
    t = a[yy, xx] / (a[yy, xx] - b[yy, xx])
    pts.append(np.stack([xx + t, yy.astype(float)], axis=1))
    # links along y
    a, b = d[:-1, :], d[1:, :]
    ok = fluid[:-1, :] & fluid[1:, :] & (a * b < 0)
    yy, xx = np.nonzero(ok)
    t = a[yy, xx] / (a[yy, xx] - b[yy, xx])
    pts.append(np.stack([xx.astype(float), yy + t], axis=1))
    p = np.concatenate(pts, axis=0)
    if wall_dist is not None and min_wall_dist > 0 and len(p):
        p = p[wall_dist(p[:, 0], p[:, 1]) >= min_wall_dist]
    return p


def fit_circle(pts):
    """Algebraic least-squares circle through points (x, y): returns
    (cx, cy, r).  Solves x^2 + y^2 + D x + E y + F = 0 in the least-squares
    sense (Kasa fit); adequate for arcs spanning tens of degrees or more."""
    x, y = pts[:, 0], pts[:, 1]
    A = np.stack([x, y, np.ones_like(x)], axis=1)
    rhs = -(x * x + y * y)
    (D, E, F), *_ = np.linalg.lstsq(A, rhs, rcond=None)
    cx, cy = -D / 2.0, -E / 2.0
    return cx, cy, float(np.sqrt(cx * cx + cy * cy - F))


def angle_between_circles(r_drop, R_wall, dist):
    """Angle (degrees) at the intersection of a droplet circle (radius
    r_drop) and a convex wall circle (radius R_wall) whose centres are
    `dist` apart, measured inside the droplet and outside the wall: 180 for
    a droplet that only touches the wall from outside, 90 for orthogonal
    circles, 0 for a film."""
    c = (r_drop ** 2 + R_wall ** 2 - dist ** 2) / (2.0 * r_drop * R_wall)
    return float(np.degrees(np.arccos(np.clip(c, -1.0, 1.0))))


def droplet_level(rho_g, rho_l):
    return 0.5 * (rho_g + rho_l)


def contact_angle_cylinder(rho, solid, center, R_nodes, rho_g, rho_l, min_wall_dist=4.0,
                           level=None, select=None):
    """Static contact angle of a droplet on a cylinder of node radius
    R_nodes centred at `center` (x, y).  Interface points at least
    `min_wall_dist` from the wall surface (radius R_nodes + 1/2) are fitted
    by a circle.  `select(x, y)` may restrict the points to one droplet.
    Returns (theta_deg, fit) with fit = (cx, cy, r, npoints)."""
    Rw = R_nodes + 0.5
    cxw, cyw = center
    lev = droplet_level(rho_g, rho_l) if level is None else level

    def wall_dist(x, y):
        return np.hypot(x - cxw, y - cyw) - Rw

    p = interface_points(rho, lev, solid, min_wall_dist, wall_dist)
    if select is not None and len(p):
        p = p[select(p[:, 0], p[:, 1])]
    if len(p) < 8:
        raise ValueError("too few interface points for a circle fit")
    cx, cy, r = fit_circle(p)
    theta = angle_between_circles(r, Rw, float(np.hypot(cx - cxw, cy - cyw)))
    return theta, (cx, cy, r, len(p))


def contact_angle_flat(rho, solid, wall_y, rho_g, rho_l, min_wall_dist=4.0, level=None,
                       select=None):
    """Static contact angle of a droplet resting on a flat wall whose surface
    is the line y = wall_y (the liquid above it).  Returns (theta_deg, fit)."""
    lev = droplet_level(rho_g, rho_l) if level is None else level
    p = interface_points(rho, lev, solid, min_wall_dist, lambda x, y: y - wall_y)
    if select is not None and len(p):
        p = p[select(p[:, 0], p[:, 1])]
    if len(p) < 8:
        raise ValueError("too few interface points for a circle fit")
    cx, cy, r = fit_circle(p)
    c = np.clip((wall_y - cy) / r, -1.0, 1.0)
    return float(np.degrees(np.arccos(c))), (cx, cy, r, len(p))


def bulk_densities(rho, center, r_in, r_out_min):
    """Mean density inside radius r_in of `center` and beyond r_out_min
    (minimum-image distance on the periodic domain): the bulk liquid and
    gas densities around a free droplet."""
    ny, nx = rho.shape
    y, x = np.mgrid[0:ny, 0:nx]
    dx = np.abs(x - center[0])
    dy = np.abs(y - center[1])
    dx = np.minimum(dx, nx - dx)
    dy = np.minimum(dy, ny - dy)
    d = np.hypot(dx, dy)
    return float(rho[d <= r_in].mean()), float(rho[d >= r_out_min].mean())


def interface_points_3d(rho, level, solid=None):
    """3-D version of interface_points for a field indexed [z, y, x]:
    crossings of `level` along x, y and z links between two fluid nodes.
    Returns an (n, 3) array of (x, y, z)."""
    rho = np.asarray(rho, dtype=np.float64)
    fluid = np.ones_like(rho, bool) if solid is None else (np.asarray(solid) == 0)
    d = rho - level
    pts = []
    for axis in (2, 1, 0):  # x, y, z
        sl0 = [slice(None)] * 3
        sl1 = [slice(None)] * 3
        sl0[axis] = slice(None, -1)
        sl1[axis] = slice(1, None)
        a, b = d[tuple(sl0)], d[tuple(sl1)]
        ok = fluid[tuple(sl0)] & fluid[tuple(sl1)] & (a * b < 0)
        zz, yy, xx = np.nonzero(ok)
        t = a[zz, yy, xx] / (a[zz, yy, xx] - b[zz, yy, xx])
        c = np.stack([xx, yy, zz], axis=1).astype(float)
        c[:, 2 - axis] += t
        pts.append(c)
    return np.concatenate(pts, axis=0)


def fit_sphere(pts):
    """Algebraic least-squares sphere through (x, y, z) points: returns
    (cx, cy, cz, r)."""
    A = np.concatenate([pts, np.ones((len(pts), 1))], axis=1)
    rhs = -(pts ** 2).sum(axis=1)
    (D, E, F, G), *_ = np.linalg.lstsq(A, rhs, rcond=None)
    c = -0.5 * np.array([D, E, F])
    return float(c[0]), float(c[1]), float(c[2]), float(np.sqrt(c @ c - G))


def contact_angle_sphere(rho, solid, center, R_nodes, rho_g, rho_l, min_wall_dist=4.0,
                         level=None, select=None):
    """Static contact angle of a droplet on a sphere of node radius R_nodes
    centred at `center` (x, y, z), field indexed [z, y, x]: a sphere fitted
    to the droplet interface (points at least `min_wall_dist` from the wall
    surface of radius R_nodes + 1/2) meets the wall sphere at the angle of
    angle_between_circles.  Returns (theta_deg, (cx, cy, cz, r, npoints))."""
    Rw = R_nodes + 0.5
    lev = droplet_level(rho_g, rho_l) if level is None else level
    p = interface_points_3d(rho, lev, solid)
    c0 = np.asarray(center, dtype=float)
    p = p[np.linalg.norm(p - c0, axis=1) - Rw >= min_wall_dist]
    if select is not None and len(p):
        p = p[select(p[:, 0], p[:, 1], p[:, 2])]
    if len(p) < 16:
        raise ValueError("too few interface points for a sphere fit")
    cx, cy, cz, r = fit_sphere(p)
    dist = float(np.linalg.norm(np.array([cx, cy, cz]) - c0))
    return angle_between_circles(r, Rw, dist), (cx, cy, cz, r, len(p))
