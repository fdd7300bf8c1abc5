"""lbm_adjoint_noalloc (scratch in the library's static device array) against
lbm_adjoint (scratch in a caller workspace), through the C ABI.

Two calls in a row share the static array: the 256 x 256 FP32 cylinder
workload (T = 60, K = 20), then a smaller FP64 lattice (48 x 40, T = 30,
K = 7) whose layout reads the array at other offsets.  Each must give the
same gradients and dL/df(0) as the workspace entry point, bit for bit (the
kernels and their order are the same).  A request above the array's size is
refused with LBM_ENOMEM before anything is launched.
"""
import numpy as np
import pytest

from cases import Setup, lib_params

pytestmark = pytest.mark.gpu


def _cylinder_case(O, L, precision, n, ny, R, r0, T, K):
    import torch
    from paper_1908_04443_amd import inputs as I
    case = dict(nx=n, ny=ny, geometry=("disk", (n // 2, ny // 2), R),
                init=("droplet", (n // 2, ny // 2 + R + r0), r0), noise=1e-4, seed=21,
                sigma=0.105, precision=precision, scheme="ivd")
    s = Setup(O, case)
    sol = L.Solver(lib_params(L, s.op, case), len(s.walls))
    sol.set_geometry(s.solid)
    nw = len(s.walls)
    rng = np.random.default_rng(5)
    phi = torch.as_tensor(1.0 + 0.2 * rng.random(nw), dtype=sol.dtype, device="cuda")
    drho = torch.as_tensor(0.004 * rng.random(nw), dtype=sol.dtype, device="cuda")
    sol.set_wetting(0, 0.0, phi, drho)
    sol.set_fields(s.rho0.ravel())
    ckpt = sol.ckpt_buffer(T, K)
    sol.step_ckpt(T, K, ckpt)
    rho_T = sol.get_fields(rho=True, u=False)["rho"]
    fluid = torch.as_tensor(s.solid.ravel() == 0, device="cuda")
    seed = torch.where(fluid, 2.0 * (rho_T - 0.9 * rho_T.mean()), torch.zeros_like(rho_T))
    return sol, nw, seed.contiguous(), ckpt


def _both(L, sol, nw, seed, T, K, ckpt):
    import torch
    outs = []
    for entry in ("workspace", "static"):
        gp = torch.full((max(nw, 1),), float("nan"), dtype=sol.dtype, device="cuda")
        gd = torch.full_like(gp, float("nan"))
        lam0 = torch.full((sol.Q * sol.N,), float("nan"), dtype=sol.dtype, device="cuda")
        if entry == "workspace":
            work = torch.empty(L.lbm_adjoint_workspace_bytes(sol.ctx, K), dtype=torch.uint8,
                               device="cuda")
            L.lbm_adjoint(sol.ctx, 0, seed, T, K, ckpt, work, gp, gd, lam0)
        else:
            L.lbm_adjoint_noalloc(sol.ctx, 0, seed, T, K, ckpt, gp, gd, lam0)
        torch.cuda.synchronize()
        outs.append((gp[:nw].clone(), gd[:nw].clone(), lam0.clone()))
    return outs


def test_noalloc_adjoint_equals_workspace_adjoint(oracle_mod, gpu_lib):
    import torch
    O, L = oracle_mod, gpu_lib
    runs = [dict(precision=4, n=256, ny=256, R=40, r0=32, T=60, K=20),
            dict(precision=8, n=48, ny=40, R=8, r0=7, T=30, K=7)]
    for cfg in runs:
        print(f"case {cfg}", flush=True)
        sol, nw, seed, ckpt = _cylinder_case(O, L, **cfg)
        need = L.lbm_adjoint_workspace_bytes(sol.ctx, cfg["K"])
        assert need <= L.LBM_NOALLOC_SCRATCH_BYTES
        (wp, wd, wl), (sp, sd, sl) = _both(L, sol, nw, seed, cfg["T"], cfg["K"], ckpt)
        assert torch.isfinite(wp).all() and wp.abs().max() > 0
        assert torch.equal(wp, sp) and torch.equal(wd, sd) and torch.equal(wl, sl)
        sol.close()


def test_noalloc_adjoint_refuses_oversized_scratch(oracle_mod, gpu_lib):
    """256^2 FP32 with K = 50 needs about 124 MB of scratch, above the 64 MiB
    array: refused on the host, nothing launched."""
    import torch
    O, L = oracle_mod, gpu_lib
    sol, nw, seed, ckpt = _cylinder_case(O, L, precision=4, n=256, ny=256, R=40, r0=32, T=50,
                                         K=50)
    assert L.lbm_adjoint_workspace_bytes(sol.ctx, 50) > L.LBM_NOALLOC_SCRATCH_BYTES
    gp = torch.zeros(nw, dtype=sol.dtype, device="cuda")
    with pytest.raises(L.LBMError) as e:
        L.lbm_adjoint_noalloc(sol.ctx, 0, seed, 50, 50, ckpt, gp, None, None)
    assert e.value.code == L.LBM_ENOMEM
    assert "scratch" in str(e.value)
    sol.close()
