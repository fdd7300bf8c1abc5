"""The D2Q9 FP32 step with 16-byte population accesses (lattice widths that
are multiples of 4) against the oracle and against the scalar tile of the
same shape.

- every vector variant on a 148 x 75 lattice (a partial tile in x and in y)
  against the FP64 oracle, FP32 normwise bars (1e-4 on rho, 1e-3 on u);
- every wetting scheme (improved and constant virtual density, solid-fluid
  interaction, geometric formulation) with per-node parameters, walls on
  the tile edges and across the periodic seam;
- lattices narrower than a tile and than the halo (4, 8, 12 wide): the lane
  shifts wrap through the seam inside one tile;
- the same run through the vector variant and the scalar variant of one
  tile shape: they differ only in how populations move, so they agree to
  rounding (normwise 1e-6).
"""
import numpy as np
import pytest

from cases import Setup, run_gpu

pytestmark = pytest.mark.gpu


def _vec_variants():
    """Indices of the 16-byte variants and of the scalar variant of the same
    tile shape (from the library's variant order)."""
    # tile shapes of the FP32 variant table: 12..15 are the vector ones
    return {12: 10, 13: 0, 14: 9, 15: None}


def _compare_fp32(O, s, res, nsteps, u_scale=0.0):
    """Normwise relative errors; velocities relative to max(max |u|,
    u_scale): the FP32 rounding of the momentum is absolute (a few 1e-8 at
    these densities), so a lattice nearly at rest needs a velocity scale."""
    f = O.run(s.op, s.solid, s.f0, nsteps, s.phi, s.drho)
    rho_o, u_o, _ = O.fields(s.op, s.solid, f, s.phi, s.drho)
    err = np.abs(res["rho"] - rho_o).max() / np.abs(rho_o).max()
    uerr = np.abs(res["u"] - u_o).max() / max(np.abs(u_o).max(), u_scale, 1e-30)
    print(f"rho err {err:.3e}  u err {uerr:.3e}", flush=True)
    assert err <= 1e-4 and uerr <= 1e-3
    return rho_o


@pytest.mark.parametrize("variant", sorted(_vec_variants()))
def test_vec_variants_ragged(oracle_mod, gpu_lib, variant):
    from paper_1908_04443_amd import lbm
    assert variant < lbm.lbm_variant_count(9, 4)
    case = dict(nx=148, ny=75, geometry=("disk", (70, 30), 12), init=("droplet", (70, 55), 10),
                scheme="ivd", phi=1.15, noise=1e-6, seed=7, precision=4)
    s = Setup(oracle_mod, case)
    res = run_gpu(gpu_lib, s, 150, variant=variant)
    _compare_fp32(oracle_mod, s, res, 150)


@pytest.mark.parametrize("scheme", ["ivd", "vd", "sfi", "gf"])
def test_vec_schemes_walls_on_tile_edges(oracle_mod, gpu_lib, scheme):
    """A 196 x 52 lattice (128-wide tiles: one full, one partial) with a
    cylinder across the x seam and one across the tile edge at x = 128."""
    from paper_1908_04443_amd import inputs as I
    nx, ny = 196, 52
    solid = I.disk_mask((ny, nx), (0, 20), 9) | I.disk_mask((ny, nx), (128, 30), 10)
    case = dict(nx=nx, ny=ny, geometry=("mask", solid), init=("blobs", 4.0), seed=5,
                scheme=scheme, rho_w=0.2, G_w=0.05, phi=70.0 if scheme == "gf" else 1.0,
                precision=4)
    if scheme == "ivd":
        rng = np.random.default_rng(6)
        case["phi_field"] = lambda sd: 1.0 + 0.3 * rng.random(sd.shape)
        case["drho_field"] = lambda sd: 0.04 * rng.random(sd.shape)
    s = Setup(oracle_mod, case)
    res = run_gpu(gpu_lib, s, 200, variant=12)
    assert np.array_equal(res["walls"], s.walls)
    _compare_fp32(oracle_mod, s, res, 200)


@pytest.mark.parametrize("nx,ny", [(4, 1), (4, 6), (8, 3), (12, 5)])
def test_vec_narrow_lattices(oracle_mod, gpu_lib, nx, ny):
    rng = np.random.default_rng(nx * 17 + ny)
    rho = 0.2 + 0.05 * rng.random((ny, nx))
    solid = np.zeros((ny, nx), np.uint8)
    if nx >= 8 and ny >= 3:
        solid[1, 2:4] = 1  # walls next to lane boundaries
    case = dict(nx=nx, ny=ny, geometry=("mask", solid), init=("uniform", 0.2), scheme="ivd",
                phi=1.1, precision=4)
    s = Setup(oracle_mod, case)
    s.rho0 = np.where(solid == 0, rho, 0.0)
    s.f0 = oracle_mod.init_eq(s.op, s.solid, s.rho0)
    res = run_gpu(gpu_lib, s, 30, variant=12)
    _compare_fp32(oracle_mod, s, res, 30, u_scale=1e-3)  # nearly at rest: |u| ~ 1e-5


@pytest.mark.parametrize("vec,scalar", [(v, s) for v, s in _vec_variants().items() if s is not None])
def test_vec_equals_scalar_tile(oracle_mod, gpu_lib, vec, scalar):
    case = dict(nx=256, ny=96, geometry=("disk", (128, 40), 20), init=("droplet", (128, 75), 14),
                scheme="ivd", phi=1.2, noise=1e-6, seed=9, precision=4)
    s = Setup(oracle_mod, case)
    a = run_gpu(gpu_lib, s, 300, variant=vec)
    b = run_gpu(gpu_lib, s, 300, variant=scalar)
    d = np.abs(a["rho"] - b["rho"]).max() / np.abs(b["rho"]).max()
    print(f"vector {vec} vs scalar {scalar}: rho normwise {d:.3e}", flush=True)
    assert d <= 1e-6
