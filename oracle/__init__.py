"""ctypes binding of the CPU oracle (oracle/liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the package smoke check and
by the CPU-baseline leg of bench.py.  The product path never imports it.

All arrays are numpy float64 / uint8 host arrays.  Node index
n = x + nx*(y + ny*z); populations are f[a, n] (structure of arrays).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

EOS_CS, EOS_PR = 0, 1
IVD, VD, SFI, GF = 0, 1, 2, 3
OK, EINVAL, EDOMAIN = 0, -1, -3


class Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("nz", C.c_int32), ("tau", C.c_double * 19), ("eos", C.c_int32),
        ("eos_a", C.c_double), ("eos_b", C.c_double), ("eos_R", C.c_double),
        ("eos_T", C.c_double), ("eos_omega", C.c_double), ("G", C.c_double),
        ("sigma", C.c_double), ("body_force", C.c_double * 3),
        ("scheme", C.c_int32), ("rho_w", C.c_double), ("G_w", C.c_double),
        ("rho_g", C.c_double), ("rho_l", C.c_double), ("sfi_solid_psi", C.c_int32),
        ("sfi_psi_presum", C.c_int32), ("sfi_lattice_weights", C.c_int32),
    ]


class OracleError(RuntimeError):
    pass


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        u8 = C.POINTER(C.c_uint8)
        i64p = C.POINTER(C.c_int64)
        P = C.POINTER(Params)
        L.orc_eos_p.restype = C.c_double
        L.orc_eos_p.argtypes = [P, C.c_double]
        L.orc_psi_arg.restype = C.c_double
        L.orc_psi_arg.argtypes = [P, C.c_double]
        L.orc_critical.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double,
                                   C.c_double, dp, dp]
        L.orc_coexistence.argtypes = [P, dp, dp]
        L.orc_wall_nodes.restype = C.c_int64
        L.orc_wall_nodes.argtypes = [P, u8, i64p]
        L.orc_init_eq.argtypes = [P, u8, dp, dp, dp]
        L.orc_run.argtypes = [P, u8, dp, dp, dp, C.c_int64]
        L.orc_fields.argtypes = [P, u8, dp, dp, dp, dp, dp, dp]
        L.orc_loss.argtypes = [P, u8, dp, dp, dp, C.c_int64, dp, dp]
        L.orc_loss_grad_cs.argtypes = [P, u8, dp, dp, dp, C.c_int64, dp, C.c_int32,
                                       C.c_int64, C.c_double, dp, dp]
        L.orc_state_tangent_cs.argtypes = [P, u8, dp, dp, dp, dp, C.c_int64,
                                           C.c_double, dp, dp]
        L.orc_lattice.argtypes = [C.c_int32, C.POINTER(C.c_int32), dp, dp, dp, dp,
                                  C.POINTER(C.c_int32)]
        L.orc_source.argtypes = [P, dp, dp, dp, C.c_double, dp]
        L.orc_gf_points.argtypes = [P, u8, dp, dp]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _check(rc, what):
    if rc != OK:
        raise OracleError(f"{what} failed with code {rc}")


def make_params(lattice=9, nx=16, ny=16, nz=1, tau=1.0, eos=EOS_CS, a=1.0, b=4.0,
                R=1.0, T=None, T_ratio=0.75, omega=0.344, G=-1.0, sigma=0.0,
                body_force=(0.0, 0.0, 0.0), scheme=IVD, rho_w=0.0, G_w=0.0,
                rho_g=None, rho_l=None, sfi_solid_psi=0, sfi_psi_presum=0,
                sfi_lattice_weights=0):
    """Build a Params struct; T defaults to T_ratio * Tc and the limiter
    bounds to the Maxwell coexistence densities, both from the oracle."""
    p = Params()
    p.lattice, p.nx, p.ny, p.nz = lattice, nx, ny, nz
    taus = np.broadcast_to(np.asarray(tau, dtype=np.float64), (19,)) \
        if np.ndim(tau) == 0 else np.asarray(tau, dtype=np.float64)
    for i in range(19):
        p.tau[i] = float(taus[i]) if i < len(taus) else 1.0
    p.eos, p.eos_a, p.eos_b, p.eos_R, p.eos_omega = eos, a, b, R, omega
    if T is None:
        Tc, _ = critical(eos, a, b, R, omega)
        T = T_ratio * Tc
    p.eos_T = T
    p.G, p.sigma = G, sigma
    for i in range(3):
        p.body_force[i] = body_force[i]
    p.scheme, p.rho_w, p.G_w = scheme, rho_w, G_w
    p.sfi_solid_psi, p.sfi_psi_presum = sfi_solid_psi, sfi_psi_presum
    p.sfi_lattice_weights = sfi_lattice_weights
    if rho_g is None or rho_l is None:
        g, l = coexistence(p)
        rho_g = g if rho_g is None else rho_g
        rho_l = l if rho_l is None else rho_l
    p.rho_g, p.rho_l = rho_g, rho_l
    return p


def N_of(p):
    return p.nx * p.ny * p.nz


def Q_of(p):
    return 9 if p.lattice == 9 else 19


def D_of(p):
    return 2 if p.lattice == 9 else 3


def eos_p(p, rho):
    return lib().orc_eos_p(C.byref(p), float(rho))


def psi_arg(p, rho):
    return lib().orc_psi_arg(C.byref(p), float(rho))


def critical(eos, a, b, R, omega=0.344):
    Tc, rc = C.c_double(), C.c_double()
    _check(lib().orc_critical(eos, a, b, R, omega, C.byref(Tc), C.byref(rc)),
           "critical")
    return Tc.value, rc.value


def coexistence(p):
    g, l = C.c_double(), C.c_double()
    _check(lib().orc_coexistence(C.byref(p), C.byref(g), C.byref(l)), "coexistence")
    return g.value, l.value


def lattice(q):
    Q = q
    e = np.zeros((Q, 3), dtype=np.int32)
    t, w = np.zeros(Q), np.zeros(Q)
    M, Minv = np.zeros((Q, Q)), np.zeros((Q, Q))
    opp = np.zeros(Q, dtype=np.int32)
    _check(lib().orc_lattice(q, e.ctypes.data_as(C.POINTER(C.c_int32)), _dp(t), _dp(w),
                             _dp(M), _dp(Minv), opp.ctypes.data_as(C.POINTER(C.c_int32))),
           "lattice")
    return dict(e=e, t=t, w=w, M=M, Minv=Minv, opp=opp)


def source(p, u, F, Fm, psi):
    Q = Q_of(p)
    S = np.zeros(Q)
    u = np.ascontiguousarray(np.resize(np.asarray(u, np.float64), 3))
    F = np.ascontiguousarray(np.resize(np.asarray(F, np.float64), 3))
    Fm = np.ascontiguousarray(np.resize(np.asarray(Fm, np.float64), 3))
    _check(lib().orc_source(C.byref(p), _dp(u), _dp(F), _dp(Fm), float(psi), _dp(S)),
           "source")
    return S


def wall_nodes(p, solid):
    solid = np.ascontiguousarray(solid, dtype=np.uint8).ravel()
    n = lib().orc_wall_nodes(C.byref(p), _u8(solid), None)
    if n < 0:
        raise OracleError("wall_nodes")
    idx = np.zeros(max(n, 1), dtype=np.int64)
    lib().orc_wall_nodes(C.byref(p), _u8(solid),
                         idx.ctypes.data_as(C.POINTER(C.c_int64)))
    return idx[:n]


def init_eq(p, solid, rho0, u0=None):
    N, Q = N_of(p), Q_of(p)
    solid = np.ascontiguousarray(solid, dtype=np.uint8).ravel()
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64).ravel()
    u0 = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64).reshape(-1)
    f = np.zeros((Q, N))
    _check(lib().orc_init_eq(C.byref(p), _u8(solid), _dp(rho0), _dp(u0), _dp(f)),
           "init_eq")
    return f


def _wall_params(p, solid, phi, drho):
    nw = len(wall_nodes(p, solid))
    phi = np.ones(nw) if phi is None else np.broadcast_to(
        np.asarray(phi, np.float64), (nw,)).copy()
    drho = np.zeros(nw) if drho is None else np.broadcast_to(
        np.asarray(drho, np.float64), (nw,)).copy()
    if nw == 0:
        phi, drho = np.ones(1), np.zeros(1)
    return np.ascontiguousarray(phi), np.ascontiguousarray(drho)


def run(p, solid, f, nsteps, phi=None, drho=None):
    """Advance a copy of f by nsteps; returns the new f."""
    solid = np.ascontiguousarray(solid, dtype=np.uint8).ravel()
    phi, drho = _wall_params(p, solid, phi, drho)
    f = np.array(f, dtype=np.float64, copy=True, order="C")
    _check(lib().orc_run(C.byref(p), _u8(solid), _dp(phi), _dp(drho), _dp(f),
                         int(nsteps)), "run")
    return f


def fields(p, solid, f, phi=None, drho=None):
    """Density (wall nodes carry their virtual density), velocity and total
    force of the state f."""
    N, D = N_of(p), D_of(p)
    solid = np.ascontiguousarray(solid, dtype=np.uint8).ravel()
    phi, drho = _wall_params(p, solid, phi, drho)
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho, u, F = np.zeros(N), np.zeros((D, N)), np.zeros((D, N))
    _check(lib().orc_fields(C.byref(p), _u8(solid), _dp(phi), _dp(drho), _dp(f),
                            _dp(rho), _dp(u), _dp(F)), "fields")
    return rho, u, F


def loss(p, solid, f0, nsteps, target, phi=None, drho=None):
    solid = np.ascontiguousarray(solid, dtype=np.uint8).ravel()
    phi, drho = _wall_params(p, solid, phi, drho)
    f0 = np.ascontiguousarray(f0, dtype=np.float64)
    target = np.ascontiguousarray(target, dtype=np.float64).ravel()
    out = C.c_double()
    _check(lib().orc_loss(C.byref(p), _u8(solid), _dp(phi), _dp(drho), _dp(f0),
                          int(nsteps), _dp(target), C.byref(out)), "loss")
    return out.value


def loss_grad_cs(p, solid, f0, nsteps, target, which, k, phi=None, drho=None, h=1e-30):
    """d loss / d phi[k] (which=0) or d drho[k] (which=1) by complex step."""
    solid = np.ascontiguousarray(solid, dtype=np.uint8).ravel()
    phi, drho = _wall_params(p, solid, phi, drho)
    f0 = np.ascontiguousarray(f0, dtype=np.float64)
    target = np.ascontiguousarray(target, dtype=np.float64).ravel()
    L, dL = C.c_double(), C.c_double()
    _check(lib().orc_loss_grad_cs(C.byref(p), _u8(solid), _dp(phi), _dp(drho), _dp(f0),
                                  int(nsteps), _dp(target), int(which), int(k), float(h),
                                  C.byref(L), C.byref(dL)), "loss_grad_cs")
    return L.value, dL.value


def state_tangent_cs(p, solid, f0, df0, nsteps, phi=None, drho=None, h=1e-30):
    solid = np.ascontiguousarray(solid, dtype=np.uint8).ravel()
    phi, drho = _wall_params(p, solid, phi, drho)
    f0 = np.ascontiguousarray(f0, dtype=np.float64)
    df0 = np.ascontiguousarray(df0, dtype=np.float64)
    fo, dfo = np.zeros_like(f0), np.zeros_like(f0)
    _check(lib().orc_state_tangent_cs(C.byref(p), _u8(solid), _dp(phi), _dp(drho),
                                      _dp(f0), _dp(df0), int(nsteps), float(h),
                                      _dp(fo), _dp(dfo)), "state_tangent_cs")
    return fo, dfo


def gf_points(p, solid, theta_deg):
    """Geometric formulation at every wall node (wall order): an array of
    shape (n_wall, 3, 2) holding the unit solid normal n_s and the points
    D_1, D_2, relative to the node (NaN where no normal can be formed)."""
    solid = np.ascontiguousarray(solid, dtype=np.uint8).ravel()
    nw = len(wall_nodes(p, solid))
    theta = np.ascontiguousarray(np.broadcast_to(np.asarray(theta_deg, np.float64), (nw,)))
    out = np.zeros((max(nw, 1), 3, 2))
    _check(lib().orc_gf_points(C.byref(p), _u8(solid), _dp(theta), _dp(out)), "gf_points")
    return out[:nw]


def set_threads(n):
    lib().orc_set_threads(int(n))


def get_threads():
    return lib().orc_get_threads()
