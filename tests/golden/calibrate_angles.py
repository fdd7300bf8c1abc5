"""Calibrate the prescribed-angle table of the improved virtual-density
scheme (Eqs. 16-17) for the Carnahan-Starling fluid at 0.75 Tc (tau = 1,
sigma from the slab calibration) with the CPU oracle, and write
tests/golden/angle_calibration_cs075.json.

Sec. III B fixes only the direction of each parameter: phi > 1 (with
drho = 0) lowers the contact angle below the standard case phi = 1,
drho > 0 (with phi = 1) raises it.  The paper prints angles for its PR
fluid only, so the table for the CS fluid of the benchmark inputs is
measured: a droplet (r = 20, tanh width 3) on a flat wall of four solid
rows in a periodic 320 x 80 lattice, 15000 steps, angle from the circle
fit of the free interface (analysis.contact_angle_flat).  The table maps
target angles to parameters by linear interpolation of the measured
angle(parameter) curves, which are monotone.

Calls only the oracle.  Run: python tests/golden/calibrate_angles.py
(about 15 minutes on 8 cores); --table-only rebuilds the table from the
stored sweeps.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
from paper_1908_04443_amd import analysis as A  # noqa: E402
from paper_1908_04443_amd import inputs as I  # noqa: E402

NX, NY, R0, STEPS = 320, 80, 20.0, 15000
PHI = [1.0, 1.05, 1.1, 1.2, 1.3, 1.4, 1.5, 1.6, 1.8]
DRHO = [0.004, 0.008, 0.012, 0.016, 0.02, 0.025, 0.03, 0.04, 0.05]
TARGETS = [20.0, 30.0, 45.0, 60.0, 75.0, 90.0, 105.0, 120.0, 135.0, 150.0, 160.0]


def sigma_cs075():
    with open(os.path.join(HERE, "sigma_calibration.json")) as fh:
        return json.load(fh)["cs_0.75"]["sigma"]


def flat_angle(phi, drho, sigma):
    p = O.make_params(nx=NX, ny=NY, T_ratio=0.75, sigma=sigma, tau=1.0, scheme=O.IVD)
    solid = np.zeros((NY, NX), np.uint8)
    solid[0:4, :] = 1  # the wall surface sits at y = 3.5 (halfway bounce-back)
    rho = I.droplet_rho((NY, NX), (NX / 2.0, 4.0 + 0.6 * R0), R0, p.rho_g, p.rho_l, solid=solid)
    nw = len(O.wall_nodes(p, solid))
    ph, dr = np.full(nw, phi), np.full(nw, drho)
    f = O.run(p, solid, O.init_eq(p, solid, rho), STEPS, ph, dr)
    r, _, _ = O.fields(p, solid, f, ph, dr)
    th, _ = A.contact_angle_flat(r.reshape(NY, NX), solid, 3.5, p.rho_g, p.rho_l,
                                 select=lambda x, y: y < NY - 4)
    return th


def table(phi_th, drho_th):
    """Target angle -> (phi, drho): below the standard case interpolate phi
    (drho = 0), above it drho (phi = 1); outside the measured range the end
    segment is extended linearly."""
    def interp(t, th, par):
        th, par = np.asarray(th), np.asarray(par)
        order = np.argsort(th)
        th, par = th[order], par[order]
        if t <= th[0]:
            k = 0
        elif t >= th[-1]:
            k = len(th) - 2
        else:
            return float(np.interp(t, th, par))
        return float(par[k] + (t - th[k]) * (par[k + 1] - par[k]) / (th[k + 1] - th[k]))

    th90 = phi_th[0][1]  # the standard case phi = 1, drho = 0
    out = {"theta": [], "phi": [], "drho": []}
    for t in sorted(TARGETS + [round(th90, 2)]):
        if t <= th90:
            ph = interp(t, [a for _, a in phi_th], [v for v, _ in phi_th])
            out["theta"].append(t), out["phi"].append(round(max(ph, 1.0), 4)), out["drho"].append(0.0)
        else:
            dr = interp(t, [th90] + [a for _, a in drho_th], [0.0] + [v for v, _ in drho_th])
            out["theta"].append(t), out["phi"].append(1.0), out["drho"].append(round(max(dr, 0.0), 5))
    return out


def main():
    path = os.path.join(HERE, "angle_calibration_cs075.json")
    if "--table-only" in sys.argv:  # rebuild the table from the stored sweeps
        with open(path) as fh:
            out = json.load(fh)
        out["table"] = table([tuple(v) for v in out["phi_sweep"]],
                             [tuple(v) for v in out["drho_sweep"]])
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        print(json.dumps(out["table"]))
        return
    sigma = sigma_cs075()
    phi_th = []
    for ph in PHI:
        th = flat_angle(ph, 0.0, sigma)
        phi_th.append((ph, th))
        print(f"phi {ph:.3f}: {th:.2f} deg", flush=True)
    drho_th = []
    for dr in DRHO:
        th = flat_angle(1.0, dr, sigma)
        drho_th.append((dr, th))
        print(f"drho {dr:.4f}: {th:.2f} deg", flush=True)
    out = dict(fluid="CS a=1 b=4 R=1, T = 0.75 Tc", sigma=sigma, tau=1.0,
               lattice=[NX, NY], r0=R0, steps=STEPS,
               phi_sweep=[[v, a] for v, a in phi_th], drho_sweep=[[v, a] for v, a in drho_th],
               table=table(phi_th, drho_th))
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out["table"]))


if __name__ == "__main__":
    main()
