"""Oracle windows: the CPU oracle steps a periodic crop of a large
lattice's initial state, and the nodes far enough from the crop's edge must
equal the GPU's full-lattice result.

One step of the method at node x reads populations no farther than 3 nodes
away (Chebyshev distance): streaming from x - e (1), the force there needs
psi of its neighbours (2), and a wall neighbour's virtual density needs the
density of its own fluid neighbours (3).  After K steps a node's state
depends only on the initial state within 3K nodes, so the crop's artificial
wrap reaches no node farther than 3K from its edge.
"""
import numpy as np

from cases import lib_params, oracle_params

TOL_RHO = 1e-4   # FP32 vs FP64 oracle, normwise relative on rho
TOL_U = 1e-3     # normwise relative on u


def gpu_run(L, op, solid, rho0, phi_f, drho_f, nsteps, precision=4, graph_steps=None):
    import torch
    p = lib_params(L, op, dict(precision=precision))
    s = L.Solver(p, max(int(solid.sum()), 1))
    s.set_geometry(solid)
    walls = s.wall_nodes()
    phi = torch.as_tensor(phi_f.ravel()[walls], dtype=s.dtype, device=s.device)
    drho = torch.as_tensor(drho_f.ravel()[walls], dtype=s.dtype, device=s.device)
    s.set_wetting(L.LBM_WET_IVD, 0.0, phi if len(walls) else None, drho if len(walls) else None)
    s.set_fields(rho0.ravel())
    if graph_steps:
        s.set_graph_steps(graph_steps)
    variant = s.variant
    rc0, d0 = s.diagnostics()
    s.step(nsteps)
    rc1, d1 = s.diagnostics()
    out = s.get_fields(rho=True, u=True)
    torch.cuda.synchronize()
    rho = out["rho"].double().cpu().numpy().reshape(solid.shape)
    u = out["u"].double().cpu().numpy().reshape((-1,) + solid.shape)
    s.close()
    assert rc0 == 0 and rc1 == 0
    return rho, u, variant, d0, d1


def crop(a, origin, size):
    """Periodic crop of the last len(origin) axes: origin in (z,) y, x order."""
    idx = [np.arange(o, o + size) % n for o, n in zip(origin, a.shape[-len(origin):])]
    return a[(Ellipsis,) + np.ix_(*idx)]


def oracle_window(O, case, solid, rho0, phi_f, drho_f, origin, size, nsteps):
    kw = dict(case, nx=size, ny=size)
    if case.get("lattice", 9) == 19:
        kw["nz"] = size
    op = oracle_params(O, kw)
    s_w = np.ascontiguousarray(crop(solid, origin, size))
    r_w = np.ascontiguousarray(crop(rho0, origin, size))
    walls = O.wall_nodes(op, s_w)
    phi = crop(phi_f, origin, size).ravel()[walls]
    drho = crop(drho_f, origin, size).ravel()[walls]
    f = O.run(op, s_w, O.init_eq(op, s_w, r_w), nsteps, phi, drho)
    rho, u, _ = O.fields(op, s_w, f, phi, drho)
    shape = s_w.shape
    return rho.reshape(shape), u.reshape((-1,) + shape)


def compare_windows(O, case, solid, rho0, phi_f, drho_f, rho_g, u_g, origins, size, nsteps):
    """rho: normwise relative per window.  u: max abs difference over all
    windows relative to the largest oracle speed in them (a window in a
    region at rest has no velocity scale of its own)."""
    m = 3 * nsteps + 1  # margin untouched by the crop's wrap
    core = slice(m, size - m)
    assert size - 2 * m >= 8
    worst_r = du = u_scale = 0.0
    for org in origins:
        rho_o, u_o = oracle_window(O, case, solid, rho0, phi_f, drho_f, org, size, nsteps)
        sl = (core,) * len(org)
        ro = rho_o[sl]
        rg = crop(rho_g, org, size)[sl]
        uo = u_o[(slice(None),) + sl]
        ug = crop(u_g, org, size)[(slice(None),) + sl]
        er = np.abs(rg - ro).max() / np.abs(ro).max()
        eu = np.abs(ug - uo).max()
        print(f"window {org}: rho {er:.2e}  |du| {eu:.2e}  (|u|max {np.abs(uo).max():.2e})",
              flush=True)
        worst_r, du = max(worst_r, er), max(du, eu)
        u_scale = max(u_scale, np.abs(uo).max())
    print(f"worst rho {worst_r:.2e}, worst u {du / u_scale:.2e} of {u_scale:.2e}", flush=True)
    assert u_scale > 1e-3  # the windows include moving fluid
    assert worst_r <= TOL_RHO
    assert du / u_scale <= TOL_U
