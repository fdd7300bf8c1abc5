"""Population arrays above 4 GiB: the step kernels switch from 32-bit buffer
offsets to 64-bit addressing (and the D3Q19 sweep to its non-buffer
instantiation).  Checked against the oracle on windows of the large lattice
(windows.py), including windows whose nodes sit at the high end of the
arrays, where direction offsets a * N * sizeof(real) pass 4 GiB.
"""
import numpy as np
import pytest

from cases import SIGMA_CAL, SIGMA_CS075, oracle_params
from paper_1908_04443_amd import workloads as W
from windows import compare_windows, gpu_run

pytestmark = pytest.mark.gpu


def test_d2q9_fp32_12288_squared_tiled_porous_medium(oracle_mod, gpu_lib):
    """The 2048^2 porous workload tiled 6 x 6 (151 M nodes, 5.4 GB per
    population buffer), 20 steps, 5 windows of 160^2."""
    O, L = oracle_mod, gpu_lib
    n = 6 * 2048
    assert 9 * 4 * n * n > 2 ** 32
    case = dict(nx=n, ny=n, T_ratio=0.75, sigma=SIGMA_CS075, scheme="ivd")
    op = oracle_params(O, case)
    d = W.c1_porous(op.rho_g, op.rho_l)
    solid = np.tile(d["solid"], (6, 6))
    rho0 = np.tile(d["rho"], (6, 6))
    phi = np.tile(d["phi"], (6, 6))
    drho = np.tile(d["drho"], (6, 6))
    K, size = 20, 160
    rho_g, u_g, _, d0, d1 = gpu_run(L, op, solid, rho0, phi, drho, K)
    drift = abs(d1["mass"] - d0["mass"]) / d0["mass"]
    print(f"mass drift {drift:.2e}", flush=True)
    assert drift < 1e-6
    h, off = size // 2, 5 * 2048
    cx, cy, r = d["cyl"][0]
    centres = [(n - 40, n - 100),                          # last rows, across the x seam
               (off + int(cy), off + int(cx + r)),         # a cylinder surface, last tile
               (n - 1, 7),                                 # across both seams
               (6000, 9000), (11000, 3000)]
    origins = [(y - h, x - h) for y, x in centres]
    compare_windows(O, case, solid, rho0, phi, drho, rho_g, u_g, origins, size, K)


def test_d3q19_fp32_384_cubed_sphere(oracle_mod, gpu_lib):
    """Sphere R = 40 with a droplet r = 30 on top at 384^3 (56.6 M nodes,
    4.30 GB per population buffer), 4 steps, 5 windows of 48^3."""
    O, L = oracle_mod, gpu_lib
    n = 384
    assert 19 * 4 * n ** 3 > 2 ** 32
    case = dict(lattice=19, nx=n, ny=n, nz=n, T_ratio=0.8,
                sigma=SIGMA_CAL["cs_0.80_d3q19"]["sigma"], scheme="ivd")
    op = oracle_params(O, case)
    d = W.c2_sphere(op.rho_g, op.rho_l, n=n)
    K, size = 4, 48
    rho_g, u_g, _, d0, d1 = gpu_run(L, op, d["solid"], d["rho"], d["phi"], d["drho"], K)
    drift = abs(d1["mass"] - d0["mass"]) / d0["mass"]
    print(f"mass drift {drift:.2e}", flush=True)
    assert drift < 1e-6
    h, c = size // 2, n // 2
    # (z, y, x): droplet centre at z = c + 70, interface up to z = c + 100
    centres = [(c + 100, c, c),          # top of the droplet interface
               (c + 70, c, c + 30),      # side of the droplet interface
               (c + 44, c, c + 20),      # contact line
               (c, c, c + 40),           # sphere equator
               (n - 2, n - 3, 1)]        # across all three seams, gas at rest
    origins = [(z - h, y - h, x - h) for z, y, x in centres]
    compare_windows(O, case, d["solid"], d["rho"], d["phi"], d["drho"], rho_g, u_g,
                    origins, size, K)
