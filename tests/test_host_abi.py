"""Host-side checks of the C ABI library that need no GPU: it loads, exports
every entry point its header declares, validates parameters, and its EOS
helpers agree with the oracle's independent thermodynamics."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1908_04443_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1908_04443_amd import build
        build.build()
    lbm.lib()
    return lbm


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported(L):
    syms = declared_symbols()
    assert len(syms) >= 18
    lib = C.CDLL(L.LIB_PATH)
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_header_constants_match_the_binding(L):
    """Every numeric #define of the header has the same value in the
    binding (shifts and plain integers)."""
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    defs = re.findall(r"#define\s+(LBM_[A-Z0-9_]+)\s+\(?\s*(\d+)u?\s*(?:<<\s*(\d+))?\s*\)?", txt)
    assert len(defs) >= 1
    for name, base, shift in defs:
        want = int(base) << int(shift or 0)
        assert getattr(L, name) == want, name


def test_status_strings(L):
    lib = L.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.lbm_status_string(code) not in (None, b"unknown status")
    assert lib.lbm_status_string(-99) == b"unknown status"


def _good(L, **kw):
    p = L.make_params(rho_g=0.0145, rho_l=0.333, T=0.07, **kw)
    return p


@pytest.mark.parametrize("field,value", [
    ("lattice", 7), ("precision", 2), ("nx", 0), ("ny", -3), ("nz", 2), ("eos", 5),
    ("eos_a", 0.0), ("eos_b", -1.0), ("eos_T", 0.0), ("G", 0.0), ("rho_g", 0.5),
    ("rho_g", -0.1),
])
def test_validate_rejects(L, field, value):
    p = _good(L)
    assert L.lbm_validate_params(p) == 0
    setattr(p, field, value)
    assert L.lbm_validate_params(p) == L.LBM_EINVAL
    assert L.lib().lbm_last_error() != b""
    assert L.lbm_workspace_bytes(p, 10) == 0


def test_validate_tau(L):
    p = _good(L)
    p.tau[8] = 0.5
    assert L.lbm_validate_params(p) == L.LBM_EINVAL
    # pxx and pxy (rows 7, 8) form one group: both must change together
    p.tau[8] = 0.51
    assert L.lbm_validate_params(p) == L.LBM_EINVAL
    assert b"moment group" in L.lib().lbm_last_error()
    p.tau[7] = 0.51
    assert L.lbm_validate_params(p) == 0
    p.tau[1], p.tau[2], p.tau[4], p.tau[6] = 1.1, 1.2, 0.9, 0.9
    assert L.lbm_validate_params(p) == 0
    # rows beyond Q are not used by D2Q9
    p.tau[12] = 0.1
    assert L.lbm_validate_params(p) == 0
    p3 = _good(L, lattice=19, nz=4)
    p3.tau[13] = 0.8  # one of the five viscous rows alone
    assert L.lbm_validate_params(p3) == L.LBM_EINVAL


def test_workspace_size(L):
    p = _good(L, nx=100, ny=60)
    a = L.lbm_workspace_bytes(p, 0)
    b = L.lbm_workspace_bytes(p, 1000)
    assert a > 2 * 9 * 100 * 60 * 4 and b > a and a % 256 == 0
    p.precision = 8
    assert L.lbm_workspace_bytes(p, 0) > a
    assert L.lbm_workspace_bytes(p, -1) == 0


def test_create_rejects_small_workspace_before_touching_device(L):
    p = _good(L, nx=32, ny=32)
    need = L.lbm_workspace_bytes(p, 10)
    ctx = C.c_void_p()
    fake = C.c_void_p(256)  # never dereferenced: the size check comes first
    rc = L.lib().lbm_create(C.byref(p), None, fake, need - 1, 10, C.byref(ctx))
    assert rc == L.LBM_ENOMEM and ctx.value is None
    rc = L.lib().lbm_create(C.byref(p), None, None, need, 10, C.byref(ctx))
    assert rc == L.LBM_ENOMEM
    p.nx = 0
    rc = L.lib().lbm_create(C.byref(p), None, fake, need, 10, C.byref(ctx))
    assert rc == L.LBM_EINVAL


def test_null_context_calls(L):
    lib = L.lib()
    assert lib.lbm_step(None, 1) == L.LBM_EINVAL
    assert lib.lbm_set_geometry(None, None) == L.LBM_EINVAL
    assert lib.lbm_get_fields(None, None, None, None) == L.LBM_EINVAL
    assert lib.lbm_set_wetting(None, 0, 0.0, None, None, 1.0, 0.0) == L.LBM_EINVAL
    assert lib.lbm_destroy(None) == 0
    assert lib.lbm_autotune_save_bytes(None) == 0


def test_batch_rows_take_whole_lines(L):
    """A multi-case context stores each case's rows a whole number of
    128-byte lines apart: a 33-wide FP32 case needs the room of a 64-wide
    one (every tile shape covers both with one tile column), a 65-wide one
    more."""
    p = _good(L, nx=1, ny=1)
    ws = lambda nx: L.lbm_batch_workspace_bytes(p, [nx, 40], [50, 50], [10, 10])
    assert ws(33) == ws(64) > 0
    assert ws(65) > ws(64)


def test_eos_helpers_match_oracle(L, oracle_mod):
    O = oracle_mod
    for eos, a, b in [(0, 1.0, 4.0), (1, 2 / 49, 2 / 21)]:
        Tc_l, rc_l = L.lbm_eos_critical(eos, a, b, 1.0)
        Tc_o, rc_o = O.critical(eos, a, b, 1.0)
        assert abs(Tc_l - Tc_o) <= 1e-10 * Tc_o
        for Tr in (0.7, 0.75, 0.8, 0.86):
            kw = dict(eos=eos, a=a, b=b)
            op = O.make_params(T_ratio=Tr, **kw)
            lp = L.make_params(T=op.eos_T, **kw)
            assert abs(lp.rho_g - op.rho_g) <= 1e-9 * op.rho_g
            assert abs(lp.rho_l - op.rho_l) <= 1e-9 * op.rho_l
            for r in (op.rho_g, 0.5 * (op.rho_g + op.rho_l), op.rho_l):
                rc, pe, ps = L.lbm_eos_eval(lp, r)
                assert rc == 0
                assert abs(pe - O.eos_p(op, r)) <= 1e-14 * max(1.0, abs(pe))
                assert abs(ps * ps - O.psi_arg(op, r)) <= 1e-13 * max(1.0, ps * ps)


def test_eos_domain(L):
    p = L.make_params(T_ratio=0.75)
    rc, pe, ps = L.lbm_eos_eval(p, 0.7)
    assert rc == L.LBM_EDOMAIN
    p.eos_T = 2.0  # supercritical: no coexistence
    g, l = C.c_double(), C.c_double()
    assert L.lib().lbm_eos_coexistence(C.byref(p), C.byref(g), C.byref(l)) == L.LBM_EINVAL


def test_c_program_links_against_the_library(L):
    """The plain C consumer of include/lbm.h (csrc/cabi_demo.c) is built with
    the library and resolves liblbm.so and the HIP runtime at load time."""
    import subprocess
    from paper_1908_04443_amd import build
    if not os.path.exists(build.DEMO):
        build.build()
    out = subprocess.run(["ldd", build.DEMO], capture_output=True, text=True, check=True).stdout
    assert "liblbm.so" in out and "libamdhip64" in out
    assert "not found" not in out


def test_validate_d3q19_grid_limits(L):
    """D3Q19 rows and slices index the launch grid: at most 65535 each."""
    p = _good(L, lattice=19, nx=8, ny=65535, nz=4)
    assert L.lbm_validate_params(p) == 0
    p = _good(L, lattice=19, nx=8, ny=65536, nz=4)
    assert L.lbm_validate_params(p) == L.LBM_EINVAL
    p = _good(L, lattice=19, nx=8, ny=4, nz=70000)
    assert L.lbm_validate_params(p) == L.LBM_EINVAL
    p = _good(L, nx=8, ny=70000)  # D2Q9 rows are not limited
    assert L.lbm_validate_params(p) == 0
