"""D3Q19 sweeps that form the next step's density themselves (the PSUM
variants): no density pass between steps, per-block partial sums closed by
a small pass.  Lattices that the variants' blocks tile exactly (otherwise
they run as the plain sweep of their shape, which test_every_d3q19_variant
covers).

- every PSUM variant against the oracle (FP64 1e-12, FP32 1e-4 normwise):
  blocks in every direction, and one block per axis, where each block is
  its own periodic neighbour;
- the same run through the PSUM variant and the plain sweep of its shape:
  they differ only in the order the density's terms are summed;
- graph replay equal bit for bit to plain launches, with field reads,
  diagnostics and host waits between replays;
- switching variants mid-run and setting a new state: the density the
  next step reads is always the current state's.
"""
import numpy as np
import pytest

from cases import Setup, run_gpu

pytestmark = pytest.mark.gpu


def _psum_variants(precision):
    """Indices of the PSUM variants and of the plain sweep of the same shape."""
    return {4: {10: 2, 11: 0, 12: 3, 13: 3}, 8: {4: 0}}[precision]


def _case(precision, nx=64, ny=16, nz=32, scheme="ivd"):
    return dict(lattice=19, nx=nx, ny=ny, nz=nz, T_ratio=0.8, sigma=0.1067,
                geometry=("disk", (nx // 2 - 3, ny // 2, nz // 2 - 6), 5),
                init=("droplet", (nx // 2 - 3, ny // 2, nz // 2 + 4), 5), scheme=scheme,
                phi=1.1, rho_w=0.2, G_w=0.02, noise=1e-6, seed=12, precision=precision)


def _compare(O, s, res, nsteps, precision):
    f = O.run(s.op, s.solid, s.f0, nsteps, s.phi, s.drho)
    rho_o, u_o, _ = O.fields(s.op, s.solid, f, s.phi, s.drho)
    if precision == 8:
        e, eu = np.abs(res["rho"] - rho_o).max(), np.abs(res["u"] - u_o).max()
        print(f"FP64 rho {e:.3e} u {eu:.3e}", flush=True)
        assert e <= 1e-12 and eu <= 1e-12
    else:
        e = np.abs(res["rho"] - rho_o).max() / np.abs(rho_o).max()
        eu = np.abs(res["u"] - u_o).max() / np.abs(u_o).max()
        print(f"FP32 rho {e:.3e} u {eu:.3e}", flush=True)
        assert e <= 1e-4 and eu <= 1e-3


@pytest.mark.parametrize("shape", [(64, 16, 32), (32, 8, 32), (96, 24, 64)])
@pytest.mark.parametrize("precision,variant",
                         [(4, v) for v in (10, 11, 12, 13)] + [(8, 4)])
def test_psum_variant_vs_oracle(oracle_mod, gpu_lib, precision, variant, shape):
    nx, ny, nz = shape
    if (precision, variant) in ((4, 12), (4, 13)) and nz % 32:
        pytest.skip("the blocks do not tile this lattice in z")
    s = Setup(oracle_mod, _case(precision, nx, ny, nz))
    res = run_gpu(gpu_lib, s, 24, variant=variant)
    _compare(oracle_mod, s, res, 24, precision)


@pytest.mark.parametrize("scheme", ["vd", "sfi"])
def test_psum_other_schemes(oracle_mod, gpu_lib, scheme):
    s = Setup(oracle_mod, _case(8, scheme=scheme))
    res = run_gpu(gpu_lib, s, 24, variant=4)
    _compare(oracle_mod, s, res, 24, 8)


@pytest.mark.parametrize("precision", [8, 4])
def test_psum_equals_plain_sweep(oracle_mod, gpu_lib, precision):
    s = Setup(oracle_mod, _case(precision))
    for v, plain in _psum_variants(precision).items():
        a = run_gpu(gpu_lib, s, 40, variant=v)
        b = run_gpu(gpu_lib, s, 40, variant=plain)
        d = np.abs(a["rho"] - b["rho"]).max() / np.abs(b["rho"]).max()
        print(f"PSUM {v} vs plain {plain}: {d:.3e}", flush=True)
        assert d <= (1e-13 if precision == 8 else 1e-6)


@pytest.mark.parametrize("precision", [8, 4])
def test_psum_graph_replay_bitwise(oracle_mod, gpu_lib, precision):
    import torch
    from cases import lib_params
    s = Setup(oracle_mod, _case(precision))
    variant = 10 if precision == 4 else 4

    def make(graph):
        p = lib_params(gpu_lib, s.op, s.case)
        sol = gpu_lib.Solver(p, len(s.walls))
        sol.set_geometry(s.solid)
        sol.set_wetting(0, 0.0, None, None, phi0=1.1, drho0=0.0)
        sol.set_fields(s.rho0.ravel())
        sol.variant = variant
        if graph:
            sol.set_graph_steps(6)
        return sol

    g, e = make(True), make(False)
    for chunk in (13, 6, 12, 1, 7):
        g.step(chunk)
        e.step(chunk)
        a = g.get_fields(rho=True, u=True, f=True)
        b = e.get_fields(rho=True, u=True, f=True)
        g.diagnostics()
        torch.cuda.synchronize()
        for k in ("rho", "u", "f"):
            assert torch.equal(a[k], b[k]), (chunk, k)
    g.close()
    e.close()


def test_psum_density_follows_the_state(oracle_mod, gpu_lib):
    """PSUM steps, a plain variant's steps, PSUM again, a new state set in
    between: against the oracle run over the same states."""
    import torch
    O = oracle_mod
    s = Setup(O, _case(8))
    res = run_gpu(gpu_lib, s, 0, want_f=True)
    sol = res["solver"]
    sol.variant = 4
    sol.step(5)
    sol.variant = 0
    sol.step(3)
    sol.variant = 3  # the brick
    sol.step(2)
    sol.variant = 4
    sol.step(4)
    f = O.run(s.op, s.solid, s.f0, 14, s.phi, s.drho)
    out = sol.get_fields(rho=True, u=False, f=True)
    rho_o, _, _ = O.fields(s.op, s.solid, f, s.phi, s.drho)
    assert np.abs(out["rho"].cpu().numpy() - rho_o).max() <= 1e-12
    # a new state mid-run: the next step must not reuse the old density
    f2 = O.run(s.op, s.solid, s.f0, 3, s.phi, s.drho)
    sol.set_state(torch.as_tensor(f2.ravel(), device="cuda"))
    sol.step(6)
    f3 = O.run(s.op, s.solid, f2, 6, s.phi, s.drho)
    rho3, _, _ = O.fields(s.op, s.solid, f3, s.phi, s.drho)
    assert np.abs(sol.get_fields(rho=True, u=False)["rho"].cpu().numpy() - rho3).max() <= 1e-12
    sol.close()
