"""Call order, error codes and degenerate inputs of the C ABI on a device
context, and the degenerate lattices of the method against the oracle.

Error paths are forced from the host (bad arguments, wrong call order); no
test makes a kernel fail.
"""
import numpy as np
import pytest

from cases import Setup, run_gpu
from test_gpu_parity import _compare

pytestmark = pytest.mark.gpu


def _params(L, **kw):
    base = dict(lattice=9, precision=8, nx=16, ny=12, T_ratio=0.75, sigma=0.1)
    base.update(kw)
    return L.make_params(**base)


def _code(exc_info):
    return exc_info.value.code


def test_call_order_is_enforced(gpu_lib):
    import torch
    L = gpu_lib
    s = L.Solver(_params(L), 64)
    with pytest.raises(L.LBMError) as e:
        s.step(1)
    assert _code(e) == L.LBM_ESTATE
    with pytest.raises(L.LBMError) as e:
        s.set_wetting(L.LBM_WET_IVD, 0.0, None, None)
    assert _code(e) == L.LBM_ESTATE
    with pytest.raises(L.LBMError) as e:
        s.set_fields(np.full(s.N, 0.2))
    assert _code(e) == L.LBM_ESTATE
    solid = np.zeros((12, 16), np.uint8)
    solid[4:7, 5:9] = 1
    s.set_geometry(solid)
    with pytest.raises(L.LBMError) as e:
        s.step(1)  # no fields yet
    assert _code(e) == L.LBM_ESTATE
    with pytest.raises(L.LBMError) as e:
        s.get_fields()
    assert _code(e) == L.LBM_ESTATE
    s.set_fields(np.where(solid.ravel() != 0, 0.0, 0.2))
    s.step(3)
    out = s.get_fields()
    torch.cuda.synchronize()
    assert torch.isfinite(out["rho"]).all()
    s.close()


def test_geometry_rejections(gpu_lib):
    L = gpu_lib
    s = L.Solver(_params(L), 8)
    with pytest.raises(L.LBMError) as e:
        s.set_geometry(np.ones((12, 16), np.uint8))  # no fluid node
    assert _code(e) == L.LBM_EINVAL
    solid = np.zeros((12, 16), np.uint8)
    solid[2:9, 3:12] = 1  # 28 wall nodes > n_wall_max = 8
    with pytest.raises(L.LBMError) as e:
        s.set_geometry(solid)
    assert _code(e) == L.LBM_EINVAL
    s.close()


def test_wetting_and_field_rejections(gpu_lib):
    import torch
    L = gpu_lib
    p = _params(L)
    s = L.Solver(p, 64)
    solid = np.zeros((12, 16), np.uint8)
    solid[4:7, 5:9] = 1
    s.set_geometry(solid)
    nw = len(s.wall_nodes())
    phi = torch.ones(nw, dtype=s.dtype, device=s.device)
    phi[3] = 0.0
    with pytest.raises(L.LBMError) as e:
        s.set_wetting(L.LBM_WET_IVD, 0.0, phi, None)  # phi must be positive
    assert _code(e) == L.LBM_EINVAL
    for rho_w in (0.6, 0.0, -0.1):  # psi not real at 0.6 (CS, 0.75 Tc); not a density
        with pytest.raises(L.LBMError) as e:
            s.set_wetting(L.LBM_WET_VD, rho_w, None, None)
        assert _code(e) == L.LBM_EINVAL
    with pytest.raises(L.LBMError) as e:
        s.set_wetting(99, 0.0, None, None)
    assert _code(e) == L.LBM_EINVAL
    # a density where Eq. 6 has no real psi (CS at 0.75 Tc: rho in (0.482, 1)):
    # the step raises the device flag, the diagnostics report it, and every
    # later step refuses until new fields are set
    rho = np.where(solid.ravel() != 0, 0.0, 0.2)
    rho[0] = 0.6
    s.set_fields(rho)
    s.step(1)
    rc, d = s.diagnostics()
    assert rc == L.LBM_EDOMAIN and d["flag"] != 0
    with pytest.raises(L.LBMError) as e:
        s.step(1)
    assert _code(e) == L.LBM_EDOMAIN
    s.set_fields(np.where(solid.ravel() != 0, 0.0, 0.2))
    s.step(2)
    rc, d = s.diagnostics()
    assert rc == 0 and d["flag"] == 0
    s.close()


def test_no_walls_and_no_wall_capacity(oracle_mod, gpu_lib):
    """All-fluid lattice (a free droplet) with n_wall_max = 0."""
    case = dict(nx=40, ny=33, init=("droplet", (20, 16), 9), noise=1e-6, seed=2, precision=8)
    s = Setup(oracle_mod, case)
    assert len(s.walls) == 0
    res = run_gpu(gpu_lib, s, 200, n_wall_max=0)
    _compare(oracle_mod, s, res, 200, 1e-12, 1e-12)


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 7), (9, 1), (2, 2)])
def test_degenerate_d2q9_lattices(oracle_mod, gpu_lib, nx, ny):
    """Lattices thinner than the stencil: every neighbour is the node itself
    or wraps several times."""
    rng = np.random.default_rng(nx * 31 + ny)
    rho = 0.2 + 0.05 * rng.random((ny, nx))
    case = dict(nx=nx, ny=ny, init=("uniform", 0.2), precision=8)
    s = Setup(oracle_mod, case)
    s.rho0 = rho
    s.f0 = oracle_mod.init_eq(s.op, s.solid, rho)
    res = run_gpu(gpu_lib, s, 30)
    _compare(oracle_mod, s, res, 30, 1e-12, 1e-12)


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 1, 5), (1, 4, 2)])
def test_degenerate_d3q19_lattices(oracle_mod, gpu_lib, shape):
    nx, ny, nz = shape
    rng = np.random.default_rng(nx + 10 * ny + 100 * nz)
    rho = 0.05 + 0.02 * rng.random((nz, ny, nx))
    case = dict(lattice=19, nx=nx, ny=ny, nz=nz, T_ratio=0.8, sigma=0.0,
                init=("uniform", 0.05), precision=8)
    s = Setup(oracle_mod, case)
    s.rho0 = rho
    s.f0 = oracle_mod.init_eq(s.op, s.solid, rho)
    res = run_gpu(gpu_lib, s, 20)
    _compare(oracle_mod, s, res, 20, 1e-12, 1e-12)


def test_autotune_cache_file(gpu_lib, tmp_path, monkeypatch):
    """LBM_AUTOTUNE_CACHE: a tuned choice is appended as one line; a later
    call on the same problem takes the last matching line without timing;
    a line whose key only starts like this problem's does not match."""
    import torch
    L = gpu_lib
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("LBM_AUTOTUNE_CACHE", str(path))
    p = _params(L, precision=4, nx=40, ny=24)
    s = L.Solver(p, 64)
    solid = np.zeros((24, 40), np.uint8)
    solid[8:14, 10:18] = 1
    s.set_geometry(solid)
    s.set_wetting(L.LBM_WET_IVD, 0.0, None, None)
    s.set_fields(np.where(solid.ravel() != 0, 0.0, 0.2))
    best = s.autotune(steps=2)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and f"variant={best} " in lines[0]
    key = lines[0].split(" variant=")[0]
    nv = L.lbm_variant_count(9, 4)
    other = (best + 1) % nv
    with open(path, "a") as fh:
        fh.write(f"{key} variant={other} ms=0\n")
        fh.write(f"{key}0 variant={(best + 2) % nv} ms=0\n")  # longer key: no match
    assert s.autotune(steps=2) == other
    assert s.variant == other
    assert len(path.read_text().splitlines()) == 3  # nothing timed, nothing appended
    s.step(2)
    torch.cuda.synchronize()
    s.close()
    # another size has another key: timed and appended
    q = L.Solver(_params(L, precision=4, nx=41, ny=24), 64)
    solid2 = np.zeros((24, 41), np.uint8)
    solid2[8:14, 10:18] = 1
    q.set_geometry(solid2)
    q.set_wetting(L.LBM_WET_IVD, 0.0, None, None)
    q.set_fields(np.where(solid2.ravel() != 0, 0.0, 0.2))
    q.autotune(steps=2)
    assert len(path.read_text().splitlines()) == 4
    q.close()


@pytest.mark.parametrize("precision", [8, 4])
def test_d3q19_state_forms(gpu_lib, precision):
    """D3Q19 contexts keep their populations in pull form internally.  A
    state set from post-stream populations reads back bit for bit on fluid
    nodes and as 0 on solid ones; a checkpoint equals the state read back at
    its time; restoring a checkpoint replays the same steps bit for bit.  A
    wall plane on the periodic seam puts bounce-back slots across the wrap."""
    import torch
    L = gpu_lib
    nx, ny, nz = 20, 14, 11
    p = L.make_params(lattice=19, precision=precision, nx=nx, ny=ny, nz=nz, T_ratio=0.8,
                      sigma=0.1)
    s = L.Solver(p, 4096)
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[3:7, 4:9, 5:12] = 1
    solid[:, 0, :] = 1
    s.set_geometry(solid)
    s.set_wetting(L.LBM_WET_IVD, 0.0, None, None, phi0=1.1)
    xs = np.broadcast_to(np.arange(nx)[None, None, :], solid.shape)
    rho = np.where(solid != 0, 0.0, np.where(xs < 9, p.rho_l, p.rho_g)).ravel()
    s.set_fields(rho)
    s.step(5)
    f5 = s.get_fields(rho=False, u=False, f=True)["f"].clone()
    fluid = torch.as_tensor(solid.ravel() == 0, device=f5.device)
    assert torch.all(f5[:, ~fluid] == 0) and torch.isfinite(f5).all()
    # set_state: solid entries are ignored, fluid entries come back unchanged
    g = f5.clone()
    g[:, fluid] *= 1.0 + 1e-3 * torch.rand_like(g[:, fluid])
    g[:, ~fluid] = 7.0
    s.set_state(g)
    back = s.get_fields(rho=False, u=False, f=True)["f"]
    assert torch.equal(back[:, fluid], g[:, fluid])
    assert torch.all(back[:, ~fluid] == 0)
    # checkpoints are post-stream states; a restore replays bit for bit
    s.set_state(f5)
    T, K = 4, 2
    ck = s.ckpt_buffer(T, K).view(2, 19, -1)
    s.step_ckpt(T, K, ck)
    f9 = s.get_fields(rho=False, u=False, f=True)["f"].clone()
    assert torch.equal(ck[0], f5)
    s.set_state(ck[1])
    s.step(2)
    again = s.get_fields(rho=False, u=False, f=True)["f"]
    torch.cuda.synchronize()
    assert torch.equal(again, f9)
    s.close()
