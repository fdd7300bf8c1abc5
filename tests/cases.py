"""Problem setups shared by the tests: the same seeded inputs are handed to
the CPU oracle and to the GPU library.

Model constants (temperature, coexistence densities) come from the oracle,
never from the GPU library.  Initial fields and geometries come from the
input generators, which hold no lattice Boltzmann arithmetic.
"""
import json
import os

import numpy as np

from paper_1908_04443_amd import inputs as I

SCHEMES = {"ivd": 0, "vd": 1, "sfi": 2, "gf": 3}
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
# flat-slab calibration of Eq. 7's sigma (tests/golden/calibrate_sigma.py)
SIGMA_CAL = json.load(open(os.path.join(GOLDEN, "sigma_calibration.json")))
SIGMA_CS075 = SIGMA_CAL["cs_0.75"]["sigma"]
SIGMA_PR086 = SIGMA_CAL["pr_0.86"]["sigma"]


def oracle_params(O, case):
    kw = {}
    if case.get("eos", "cs") == "pr":
        kw = dict(eos=O.EOS_PR, a=2.0 / 49.0, b=2.0 / 21.0)
    return O.make_params(
        lattice=case.get("lattice", 9), nx=case["nx"], ny=case["ny"], nz=case.get("nz", 1),
        tau=case.get("tau", 1.0), T_ratio=case.get("T_ratio", 0.75),
        sigma=case.get("sigma", SIGMA_CS075), body_force=case.get("body", (0.0, 0.0, 0.0)),
        scheme=SCHEMES[case.get("scheme", "ivd")], rho_w=case.get("rho_w", 0.0),
        G_w=case.get("G_w", 0.0), **kw)


def lib_params(L, op, case):
    """Library parameters equal to the oracle's (same T, rho_g, rho_l)."""
    p = L.lbm_params()
    p.lattice, p.precision = op.lattice, case.get("precision", 8)
    p.nx, p.ny, p.nz, p.eos = op.nx, op.ny, op.nz, op.eos
    for i in range(19):
        p.tau[i] = op.tau[i]
    p.eos_a, p.eos_b, p.eos_R, p.eos_T, p.eos_omega = op.eos_a, op.eos_b, op.eos_R, op.eos_T, op.eos_omega
    p.G, p.sigma = op.G, op.sigma
    for i in range(3):
        p.body_force[i] = op.body_force[i]
    p.rho_g, p.rho_l = op.rho_g, op.rho_l
    return p


def shape_of(case):
    if case.get("lattice", 9) == 9:
        return (case["ny"], case["nx"])
    return (case["nz"], case["ny"], case["nx"])


def geometry(case):
    shape = shape_of(case)
    g = case.get("geometry", ("none",))
    if g[0] == "none":
        return np.zeros(shape, np.uint8)
    if g[0] == "disk":  # cylinder (2-D) or sphere (3-D): ("disk", center, R)
        return I.disk_mask(shape, g[1], g[2])
    if g[0] == "channel":
        return I.channel_mask(case["nx"], case["ny"])
    if g[0] == "mask":
        return np.asarray(g[1], np.uint8).reshape(shape)
    raise ValueError(g)


def initial_rho(case, op, solid):
    shape = shape_of(case)
    init = case.get("init", ("droplet",))
    if init[0] == "droplet":  # ("droplet", center, r0)
        rho = I.droplet_rho(shape, init[1], init[2], op.rho_g, op.rho_l,
                            width=case.get("width", 3.0), solid=solid)
    elif init[0] == "blobs":
        rho = I.blob_rho(shape, case.get("seed", 0), op.rho_g, op.rho_l, solid=solid,
                         sigma=init[1] if len(init) > 1 else 16.0)
    elif init[0] == "uniform":
        rho = np.where(solid != 0, 0.0, init[1]) * np.ones(shape)
    else:
        raise ValueError(init)
    amp = case.get("noise", 0.0)
    if amp:
        rho = I.add_noise(rho, amp, case.get("seed", 0), solid=solid)
    return rho


def wall_param_fields(case, solid):
    """(phi, drho) on every node; each side gathers at its own wall nodes."""
    phi = np.full(solid.shape, float(case.get("phi", 1.0)))
    drho = np.full(solid.shape, float(case.get("drho", 0.0)))
    if "phi_field" in case:
        phi = case["phi_field"](solid)
    if "drho_field" in case:
        drho = case["drho_field"](solid)
    return phi, drho


class Setup:
    def __init__(self, O, case):
        self.case = case
        self.op = oracle_params(O, case)
        self.solid = geometry(case)
        self.rho0 = initial_rho(case, self.op, self.solid)
        self.phi_field, self.drho_field = wall_param_fields(case, self.solid)
        self.walls = O.wall_nodes(self.op, self.solid)
        self.phi = self.phi_field.ravel()[self.walls]
        self.drho = self.drho_field.ravel()[self.walls]
        self.f0 = O.init_eq(self.op, self.solid, self.rho0)


def run_gpu(L, setup, nsteps, precision=None, n_wall_max=None, want_f=False, variant=None):
    """Run the GPU library on a Setup; returns (rho, u, [f]) as numpy."""
    import torch
    case = dict(setup.case)
    if precision is not None:
        case["precision"] = precision
    p = lib_params(L, setup.op, case)
    nw = len(setup.walls)
    s = L.Solver(p, n_wall_max if n_wall_max is not None else max(nw, 1))
    s.set_geometry(setup.solid)
    walls = s.wall_nodes()
    dt = s.dtype
    phi = torch.as_tensor(setup.phi_field.ravel()[walls], dtype=dt, device=s.device)
    drho = torch.as_tensor(setup.drho_field.ravel()[walls], dtype=dt, device=s.device)
    sch = SCHEMES[case.get("scheme", "ivd")]
    scalar = {1: case.get("rho_w", 0.0), 2: case.get("G_w", 0.0),
              3: case.get("phi", 90.0)}.get(sch, 0.0)  # GF: phi carries theta_a (deg)
    s.set_wetting(sch, scalar, phi if nw else None, drho if nw else None)
    s.set_fields(setup.rho0.ravel())
    if variant is not None:
        s.variant = variant
    s.step(nsteps)
    out = s.get_fields(rho=True, u=True, f=want_f)
    torch.cuda.synchronize()
    res = {k: v.double().cpu().numpy() for k, v in out.items()}
    res["walls"] = walls
    res["solver"] = s
    return res
