"""Calibrate the thermodynamic-consistency constant sigma of Eq. 7 with the
CPU oracle and write tests/golden/sigma_calibration.json.

The paper treats sigma as a free constant (Sec. II A, the sigma term of
Eq. 7) and does not print its value.  It is chosen here so that a flat
liquid slab in its own vapour relaxes to the Maxwell-construction gas
density of the equation of state: a secant iteration on the relative error
of the simulated gas density, each evaluation a 4 x 128 periodic slab run
for 20000 steps from a tanh profile between the Maxwell densities.

Calls only the oracle.  Run: python tests/golden/calibrate_sigma.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle as O  # noqa: E402

NX, NY, STEPS = 4, 128, 20000

CASES = {
    # key: (eos kwargs, T/Tc, tau, lattice)
    "cs_0.75": (dict(eos=0, a=1.0, b=4.0), 0.75, 1.0, 9),
    "pr_0.86": (dict(eos=1, a=2.0 / 49.0, b=2.0 / 21.0), 0.86, 1.0, 9),
    "cs_0.80_d3q19": (dict(eos=0, a=1.0, b=4.0), 0.80, 1.0, 19),
    "pr_0.86_d3q19": (dict(eos=1, a=2.0 / 49.0, b=2.0 / 21.0), 0.86, 1.0, 19),
}


def slab(eos_kw, T_ratio, tau, sigma, lattice=9):
    """The slab is normal to the last axis (y in 2-D, z in 3-D)."""
    if lattice == 9:
        p = O.make_params(nx=NX, ny=NY, T_ratio=T_ratio, sigma=sigma, tau=tau, **eos_kw)
        shape = (NY, NX)
    else:
        p = O.make_params(lattice=19, nx=NX, ny=NX, nz=NY, T_ratio=T_ratio, sigma=sigma,
                          tau=tau, **eos_kw)
        shape = (NY, NX, NX)
    solid = np.zeros(shape, np.uint8)
    y = np.arange(NY).reshape((NY,) + (1,) * (len(shape) - 1)) * np.ones(shape)
    H = 0.5 * (np.tanh((y - NY / 4) / 2.0) - np.tanh((y - 3 * NY / 4) / 2.0))
    rho0 = p.rho_g + (p.rho_l - p.rho_g) * H
    f = O.run(p, solid, O.init_eq(p, solid, rho0), STEPS)
    rho, _, _ = O.fields(p, solid, f)
    return rho.min() / p.rho_g - 1.0, rho.max() / p.rho_l - 1.0, p


def calibrate(eos_kw, T_ratio, tau, lattice, s0=0.09, s1=0.12, tol=2e-3):
    e0, _, _ = slab(eos_kw, T_ratio, tau, s0, lattice)
    e1, l1, p = slab(eos_kw, T_ratio, tau, s1, lattice)
    for _ in range(8):
        s2 = s1 - e1 * (s1 - s0) / (e1 - e0)
        s0, e0 = s1, e1
        s1 = s2
        e1, l1, p = slab(eos_kw, T_ratio, tau, s1, lattice)
        if abs(e1) < tol:
            break
    return dict(sigma=round(float(s1), 4), gas_rel_err=float(e1), liquid_rel_err=float(l1),
                rho_g=p.rho_g, rho_l=p.rho_l, T=p.eos_T, slab=[NX, NY], steps=STEPS, tau=tau,
                lattice=lattice)


def main():
    out = {}
    for key, (kw, Tr, tau, lat) in CASES.items():
        out[key] = calibrate(kw, Tr, tau, lat)
        print(key, out[key], flush=True)
    with open(os.path.join(HERE, "sigma_calibration.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
