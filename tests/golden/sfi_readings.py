"""Which pseudopotential do the solid nodes carry under the solid-fluid
interaction scheme (Sec. II B, Eq. 8; Fig. 6)?

The paper prints the adhesive force of Eq. 8 (pre-sum factor rho(x)) and
the contact angles it gives on the cylinder of Sec. IV A (G_w = -0.6, 0.3,
1.2 -> about 38, 59, 119 deg), but not what psi the solid nodes hold in
the cohesive force of Eq. 5.  This script runs the oracle on the cylinder
case for each candidate and writes the measured angles to
sfi_readings.json:

  zero   no pseudopotential in the solid (the reading the library takes)
  ave    psi of the Eq. 17 mean of the solid node's fluid neighbours
  gas    psi(rho_g)
  liq    psi(rho_l)
  own    each fluid node sees its solid neighbours at its own psi

each with the pre-sum factor of Eq. 8 as printed, rho(x), and with psi(x)
(the variant of Raiskinmaki et al. that the introduction mentions), and
with the weights of the sum in Eq. 8 taken as those of Eq. 5 (1/3, 1/12)
or, with --weights lattice, as the lattice weights (1/9, 1/36).

Runs at half the paper's scale by default (150 x 175, R = 35, droplet
r = 25, 12000 steps); --full runs 300 x 350, R = 70, r = 50, 40000 steps.
Only the oracle and the angle measurement are used.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
from paper_1908_04443_amd import analysis as A  # noqa: E402
from paper_1908_04443_amd import inputs as I  # noqa: E402

READINGS = {"zero": 0, "ave": 1, "gas": 2, "liq": 3, "own": 4}
GW = (-0.6, 0.3, 1.2)
PRINTED = {-0.6: 38.0, 0.3: 59.0, 1.2: 119.0}


def run(reading, presum, G_w, scale, steps, sigma, lattice_weights=0):
    nx, ny = 300 // scale, 350 // scale
    R, r0 = 70 // scale, 50 // scale
    cc, dc = (nx // 2, 130 // scale), (nx // 2, 230 // scale)
    tau = [1.0] * 9
    tau[7] = tau[8] = 0.95  # nu = 0.15 (Sec. IV A)
    p = O.make_params(nx=nx, ny=ny, eos=O.EOS_PR, a=2.0 / 49.0, b=2.0 / 21.0, T_ratio=0.86,
                      sigma=sigma, tau=tau, scheme=O.SFI, G_w=G_w,
                      sfi_solid_psi=READINGS[reading], sfi_psi_presum=int(presum == "psi"),
                      sfi_lattice_weights=lattice_weights)
    solid = I.disk_mask((ny, nx), cc, R)
    rho0 = I.droplet_rho((ny, nx), dc, r0, p.rho_g, p.rho_l, solid=solid)
    f = O.init_eq(p, solid, rho0)
    out = dict(reading=reading, presum=presum, weights="lattice" if lattice_weights else "eq5",
               G_w=G_w, printed=PRINTED[G_w], nx=nx, ny=ny, steps=steps)
    try:
        f = O.run(p, solid, f, steps)
    except O.OracleError:
        out["result"] = "left the psi domain"
        return out
    rho, u, _ = O.fields(p, solid, f)
    rho = rho.reshape(ny, nx)
    fluid = solid == 0
    out["rho_min"], out["rho_max"] = float(rho[fluid].min()), float(rho[fluid].max())
    out["max_u"] = float(np.sqrt((u ** 2).sum(0)).reshape(ny, nx)[fluid].max())
    liquid = (rho > 0.5 * (p.rho_g + p.rho_l)) & fluid
    if liquid.sum() < 0.2 * np.pi * r0 * r0:
        out["result"] = "no droplet left on the cylinder"
        return out
    try:
        th, fit = A.contact_angle_cylinder(rho, solid, cc, R, p.rho_g, p.rho_l,
                                           select=lambda x, y: y > cc[1])
        out["theta"] = round(float(th), 2)
        out["result"] = "ok"
    except Exception as e:  # no interface to fit (wetting film, detached droplet)
        out["result"] = f"no angle: {type(e).__name__}"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--full", action="store_true")
    ap.add_argument("--readings", default=",".join(READINGS))
    ap.add_argument("--presum", default="rho,psi")
    ap.add_argument("--weights", default="eq5", choices=("eq5", "lattice"))
    ap.add_argument("--out", default=os.path.join(HERE, "sfi_readings.json"))
    args = ap.parse_args()
    sigma = json.load(open(os.path.join(HERE, "sigma_calibration.json")))["pr_0.86"]["sigma"]
    scale, steps = (1, 40000) if args.full else (2, 12000)
    rows = []
    for pre in args.presum.split(","):
        for rd in args.readings.split(","):
            for gw in GW:
                t0 = time.time()
                r = run(rd, pre, gw, scale, steps, sigma, int(args.weights == "lattice"))
                r["seconds"] = round(time.time() - t0, 1)
                print(json.dumps(r), flush=True)
                rows.append(r)
    json.dump(dict(scale=scale, steps=steps, sigma=sigma, rows=rows), open(args.out, "w"),
              indent=1)


if __name__ == "__main__":
    main()
