"""The seeded input generators and the benchmark workloads built from them.

Pins: the published SplitMix64 output sequence for seed 0, brute-force
counts on small shapes, the geometric constraints the workload recipes
promise (non-overlapping periodic cylinders, droplets kept off the periodic
image), and the wall-node counts of the workload geometries.
"""
import numpy as np
import pytest

from paper_1908_04443_amd import inputs as I
from paper_1908_04443_amd import workloads as W


def test_splitmix64_published_sequence():
    # SplitMix64 seeded with 0: the state advances by the golden-ratio
    # increment and each state is finalised by the mix; the first three
    # outputs are the published ones
    g = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        out = [int(I._mix(g * np.uint64(k))) for k in (1, 2, 3)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_counter_streams_are_deterministic_and_addressable():
    a = I.uniform(5, 3, 1000)
    assert np.array_equal(a, I.uniform(5, 3, 1000))
    assert np.array_equal(I.uniform(5, 3, 10, start=37), a[37:47])  # counter-based
    assert not np.array_equal(a, I.uniform(5, 4, 1000))             # another stream
    assert not np.array_equal(a, I.uniform(6, 3, 1000))             # another seed
    assert a.min() >= 0.0 and a.max() < 1.0
    big = I.uniform(1, 0, 200000)
    assert abs(big.mean() - 0.5) < 0.005 and abs(big.var() - 1.0 / 12.0) < 0.002


@pytest.mark.parametrize("n,R", [(16, 3.0), (31, 7.5), (40, 9.0)])
def test_disk_mask_counts_lattice_points(n, R):
    """Brute force over every node with the minimum-image distance."""
    c = (n // 2 + 0.25, n // 3)
    m = I.disk_mask((n, n), c, R)
    cnt = 0
    for y in range(n):
        for x in range(n):
            dx = min(abs(x - c[0]), n - abs(x - c[0]))
            dy = min(abs(y - c[1]), n - abs(y - c[1]))
            cnt += dx * dx + dy * dy <= R * R
    assert int(m.sum()) == cnt


def test_droplet_profile_midpoint_and_bulk():
    rg, rl = 0.02, 0.3
    rho = I.droplet_rho((64, 64), (32, 32), 10.0, rg, rl)
    assert rho[32, 42] == pytest.approx(0.5 * (rg + rl), abs=1e-15)  # r = r0
    assert abs(rho[32, 32] - rl) < 1e-6 and abs(rho[0, 0] - rg) < 1e-6


def test_blobs_split_the_fluid_in_half():
    rg, rl = 0.02, 0.3
    solid = I.disk_mask((256, 256), (100, 100), 30)
    rho = I.blob_rho((256, 256), 3, rg, rl, solid=solid)
    fluid = solid == 0
    liquid = rho[fluid] > 0.5 * (rg + rl)
    assert abs(liquid.mean() - 0.5) < 0.02
    assert np.all(rho[~fluid] == 0.0)
    assert rho[fluid].min() >= rg - 1e-12 and rho[fluid].max() <= rl + 1e-12


def test_porous_medium_recipe():
    """400 periodic cylinders, radii in [8, 32], pairwise minimum-image gap
    at least 2 between surfaces, every solid node labelled by its cylinder."""
    d = W.c1_porous(0.02, 0.3)
    cyl = d["cyl"]
    assert len(cyl) == 400
    assert cyl[:, 2].min() >= 8.0 and cyl[:, 2].max() <= 32.0
    n = 2048
    dx = (cyl[:, None, 0] - cyl[None, :, 0] + n / 2) % n - n / 2
    dy = (cyl[:, None, 1] - cyl[None, :, 1] + n / 2) % n - n / 2
    gap = np.sqrt(dx * dx + dy * dy) - cyl[:, None, 2] - cyl[None, :, 2]
    np.fill_diagonal(gap, np.inf)
    assert gap.min() >= 2.0
    assert 0.10 < d["solid"].mean() < 0.14
    assert d["theta"].min() >= 30.0 and d["theta"].max() <= 150.0
    # the per-node parameters follow each cylinder's prescribed angle
    phi, drho = I.angle_to_params(d["theta"], W.ANGLE_TABLE_CS075)
    k = 17
    cx, cy = int(cyl[k, 0]), int(cyl[k, 1])
    assert d["phi"][cy % n, cx % n] == pytest.approx(phi[k])
    assert d["drho"][cy % n, cx % n] == pytest.approx(drho[k])


def test_uneven_cases_recipe():
    cases = W.c3_cases(0.02, 0.3)
    assert len(cases) == 96
    for c in cases:
        assert 128 <= c["n"] <= 768
        assert 2 * c["R"] + 2 * c["r0"] <= c["n"] - 8 + 1e-9  # off the periodic image
        assert 20.0 <= c["theta"] <= 160.0
        assert c["solid"].shape == (c["n"], c["n"])


def test_wall_counts_of_the_workload_geometries(oracle_mod):
    """Wall nodes (solid with a fluid neighbour) of the 128^2 cylinder
    (R = 24), the 256^2 adjoint cylinder (R = 40) and the 256^3 sphere
    (R = 40): 188, 316 and 25088."""
    O = oracle_mod
    d0 = W.c0_cylinder(0.02, 0.3)
    p = O.make_params(nx=128, ny=128, sigma=0.1)
    assert len(O.wall_nodes(p, d0["solid"])) == 188
    assert int(d0["solid"].sum()) == 1793
    d4 = W.c4_adjoint(0.02, 0.3)
    p = O.make_params(nx=256, ny=256, sigma=0.1)
    assert len(O.wall_nodes(p, d4["solid"])) == 316
    d2 = W.c2_sphere(0.02, 0.3)
    p = O.make_params(lattice=19, nx=256, ny=256, nz=256, T_ratio=0.8, sigma=0.1)
    assert len(O.wall_nodes(p, d2["solid"])) == 25088
    assert int(d2["solid"].sum()) == 267761


def test_c0_phi_is_the_stored_cylinder_calibration():
    """The 128^2 workload's wetting parameter is the value the committed
    oracle calibration on that cylinder found (tests/golden/calibrate_c0.py)."""
    import json
    import os
    cal = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c0_calibration.json")))
    assert W.PHI_C0_60 == cal["phi"]
    assert abs(cal["measured_deg"] - 60.0) <= 3.0
    d = W.c0_cylinder(0.02, 0.3)
    assert np.all(d["phi"] == W.PHI_C0_60) and np.all(d["drho"] == 0.0)
