"""Thin ctypes binding of the C ABI in include/lbm.h.

Argument marshalling only: every step of the method runs in the HIP kernels
of liblbm.so.  PyTorch provides device memory (the workspace and the field
tensors) and the stream.  There is no CPU fallback: if the library is not
built, loading fails with an error.

The functions carry the C names (lbm_create, lbm_set_geometry, ...); the
`Solver` class is a convenience wrapper that owns a workspace tensor.
"""
import ctypes as C
import os

import numpy as np
import torch  # must be imported before liblbm.so so both share one HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDOMAIN, LBM_ESTATE, LBM_EDEVICE = 0, -1, -2, -3, -4, -5
LBM_EOS_CS, LBM_EOS_PR = 0, 1
LBM_WET_IVD, LBM_WET_VD, LBM_WET_SFI, LBM_WET_GF = 0, 1, 2, 3


class lbm_params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("precision", C.c_int32), ("nx", C.c_int32),
        ("ny", C.c_int32), ("nz", C.c_int32), ("eos", C.c_int32),
        ("tau", C.c_double * 19), ("eos_a", C.c_double), ("eos_b", C.c_double),
        ("eos_R", C.c_double), ("eos_T", C.c_double), ("eos_omega", C.c_double),
        ("G", C.c_double), ("sigma", C.c_double), ("body_force", C.c_double * 3),
        ("rho_g", C.c_double), ("rho_l", C.c_double),
    ]


class lbm_diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("max_u", C.c_double), ("rho_min", C.c_double),
                ("rho_max", C.c_double), ("flag", C.c_int32), ("n_fluid", C.c_int32)]


class LBMError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


_lib = None


def lib():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1908_04443_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, P, i64, dp = C.c_void_p, C.POINTER(lbm_params), C.c_int64, C.POINTER(C.c_double)
        sig = {
            "lbm_version": (C.c_char_p, []),
            "lbm_status_string": (C.c_char_p, [C.c_int]),
            "lbm_last_error": (C.c_char_p, []),
            "lbm_validate_params": (C.c_int, [P]),
            "lbm_eos_critical": (C.c_int, [C.c_int32, C.c_double, C.c_double, C.c_double,
                                           C.c_double, dp, dp]),
            "lbm_eos_coexistence": (C.c_int, [P, dp, dp]),
            "lbm_eos_eval": (C.c_int, [P, C.c_double, dp, dp]),
            "lbm_workspace_bytes": (C.c_size_t, [P, i64]),
            "lbm_create": (C.c_int, [P, vp, vp, C.c_size_t, i64, C.POINTER(vp)]),
            "lbm_destroy": (C.c_int, [vp]),
            "lbm_set_geometry": (C.c_int, [vp, C.POINTER(C.c_uint8)]),
            "lbm_wall_nodes": (C.c_int, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
            "lbm_gf_stencils": (C.c_int, [P, C.POINTER(C.c_uint8), dp, C.c_double, i64,
                                          C.POINTER(C.c_int64), C.POINTER(C.c_int32), dp]),
            "lbm_set_wetting": (C.c_int, [vp, C.c_int32, C.c_double, vp, vp, C.c_double,
                                          C.c_double]),
            "lbm_set_fields": (C.c_int, [vp, vp, vp]),
            "lbm_set_state": (C.c_int, [vp, vp]),
            "lbm_step": (C.c_int, [vp, i64]),
            "lbm_step_timed": (C.c_int, [vp, i64, dp]),
            "lbm_get_fields": (C.c_int, [vp, vp, vp, vp]),
            "lbm_get_diagnostics": (C.c_int, [vp, C.POINTER(lbm_diag)]),
            "lbm_variant_count": (C.c_int, [C.c_int32, C.c_int32]),
            "lbm_set_variant": (C.c_int, [vp, C.c_int32]),
            "lbm_get_variant": (C.c_int, [vp, C.POINTER(C.c_int32)]),
            "lbm_autotune": (C.c_int, [vp, i64, vp, C.POINTER(C.c_int32), dp]),
            "lbm_autotune_save_bytes": (C.c_size_t, [vp]),
            "lbm_set_graph_steps": (C.c_int, [vp, i64]),
            "lbm_adjoint_workspace_bytes": (C.c_size_t, [vp, i64]),
            "lbm_step_ckpt": (C.c_int, [vp, i64, i64, vp]),
            "lbm_adjoint": (C.c_int, [vp, C.c_int32, vp, i64, i64, vp, vp, C.c_size_t, vp, vp,
                                      vp]),
            "lbm_adjoint_noalloc": (C.c_int, [vp, C.c_int32, vp, i64, i64, vp, vp, vp, vp]),
            "lbm_batch_workspace_bytes": (C.c_size_t, [P, C.c_int32, C.POINTER(C.c_int32),
                                                       C.POINTER(C.c_int32), C.POINTER(i64)]),
            "lbm_create_batch": (C.c_int, [P, C.c_int32, C.POINTER(C.c_int32),
                                           C.POINTER(C.c_int32), C.POINTER(i64), vp, vp,
                                           C.c_size_t, C.POINTER(vp)]),
            "lbm_batch_cases": (C.c_int, [vp, C.POINTER(C.c_int32)]),
            "lbm_set_geometry_case": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_uint8)]),
            "lbm_wall_nodes_case": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_int64),
                                              C.POINTER(C.c_int64)]),
            "lbm_set_wetting_case": (C.c_int, [vp, C.c_int32, vp, vp, C.c_double, C.c_double]),
            "lbm_set_fields_case": (C.c_int, [vp, C.c_int32, vp, vp]),
            "lbm_get_fields_case": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
            "lbm_get_diagnostics_case": (C.c_int, [vp, C.c_int32, C.POINTER(lbm_diag)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype, fn.argtypes = res, args
        _lib = L
    return _lib


def _check(rc, where):
    if rc != LBM_OK:
        msg = lib().lbm_last_error().decode()
        raise LBMError(rc, where, msg)
    return rc


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ------------------------------------------------------------- C-named calls
def lbm_version():
    return lib().lbm_version().decode()


def lbm_validate_params(p):
    return lib().lbm_validate_params(C.byref(p))


def lbm_eos_critical(eos, a, b, R, omega=0.344):
    Tc, rc = C.c_double(), C.c_double()
    _check(lib().lbm_eos_critical(eos, a, b, R, omega, C.byref(Tc), C.byref(rc)),
           "lbm_eos_critical")
    return Tc.value, rc.value


def lbm_eos_coexistence(p):
    g, l = C.c_double(), C.c_double()
    _check(lib().lbm_eos_coexistence(C.byref(p), C.byref(g), C.byref(l)), "lbm_eos_coexistence")
    return g.value, l.value


def lbm_eos_eval(p, rho):
    pe, ps = C.c_double(), C.c_double()
    rc = lib().lbm_eos_eval(C.byref(p), float(rho), C.byref(pe), C.byref(ps))
    return rc, pe.value, ps.value


def lbm_workspace_bytes(p, n_wall_max):
    return lib().lbm_workspace_bytes(C.byref(p), int(n_wall_max))


def lbm_create(p, stream, workspace, n_wall_max):
    ctx = C.c_void_p()
    _check(lib().lbm_create(C.byref(p), C.c_void_p(stream), _ptr(workspace),
                            workspace.numel() * workspace.element_size(), int(n_wall_max),
                            C.byref(ctx)), "lbm_create")
    return ctx


def lbm_destroy(ctx):
    return lib().lbm_destroy(ctx)


def lbm_set_geometry(ctx, solid):
    s = np.ascontiguousarray(np.asarray(solid, dtype=np.uint8).ravel())
    _check(lib().lbm_set_geometry(ctx, s.ctypes.data_as(C.POINTER(C.c_uint8))),
           "lbm_set_geometry")


def lbm_wall_nodes(ctx):
    n = C.c_int64()
    _check(lib().lbm_wall_nodes(ctx, None, C.byref(n)), "lbm_wall_nodes")
    idx = np.zeros(max(n.value, 1), dtype=np.int64)
    _check(lib().lbm_wall_nodes(ctx, idx.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(n)),
           "lbm_wall_nodes")
    return idx[:n.value]


def lbm_gf_stencils(params, solid, theta_deg=None, theta0=90.0):
    """Host query: the geometric-formulation stencils of every wall node.
    Returns (nodes, weights): int32 (n_wall, 2, 2, 2) offsets [wall, point,
    node, xy] and float64 (n_wall, 2, 2) weights [wall, point, node]."""
    solid = np.ascontiguousarray(solid, dtype=np.uint8).ravel()
    u8 = solid.ctypes.data_as(C.POINTER(C.c_uint8))
    n = C.c_int64()
    _check(lib().lbm_gf_stencils(C.byref(params), u8, None, float(theta0), 0, C.byref(n), None,
                                 None), "lbm_gf_stencils")
    nw = n.value
    th = None
    if theta_deg is not None:
        th = np.ascontiguousarray(np.broadcast_to(np.asarray(theta_deg, np.float64), (nw,)))
    nodes = np.zeros((max(nw, 1), 2, 2, 2), dtype=np.int32)
    wts = np.zeros((max(nw, 1), 2, 2))
    _check(lib().lbm_gf_stencils(C.byref(params), u8,
                                 None if th is None else th.ctypes.data_as(C.POINTER(C.c_double)),
                                 float(theta0), max(nw, 1), C.byref(n),
                                 nodes.ctypes.data_as(C.POINTER(C.c_int32)),
                                 wts.ctypes.data_as(C.POINTER(C.c_double))), "lbm_gf_stencils")
    return nodes[:nw], wts[:nw]


def lbm_set_wetting(ctx, scheme, scalar=0.0, phi=None, drho=None, phi0=1.0, drho0=0.0):
    _check(lib().lbm_set_wetting(ctx, int(scheme), float(scalar), _ptr(phi), _ptr(drho),
                                 float(phi0), float(drho0)), "lbm_set_wetting")


def lbm_set_fields(ctx, rho, u=None):
    _check(lib().lbm_set_fields(ctx, _ptr(rho), _ptr(u)), "lbm_set_fields")


def lbm_set_state(ctx, f):
    _check(lib().lbm_set_state(ctx, _ptr(f)), "lbm_set_state")


def lbm_step(ctx, nsteps):
    _check(lib().lbm_step(ctx, int(nsteps)), "lbm_step")


def lbm_step_timed(ctx, nsteps):
    ms = C.c_double()
    _check(lib().lbm_step_timed(ctx, int(nsteps), C.byref(ms)), "lbm_step_timed")
    return ms.value


def lbm_get_fields(ctx, rho=None, u=None, f=None):
    _check(lib().lbm_get_fields(ctx, _ptr(rho), _ptr(u), _ptr(f)), "lbm_get_fields")


def lbm_get_diagnostics(ctx):
    d = lbm_diag()
    rc = lib().lbm_get_diagnostics(ctx, C.byref(d))
    if rc not in (LBM_OK, LBM_EDOMAIN):
        _check(rc, "lbm_get_diagnostics")
    return rc, dict(mass=d.mass, max_u=d.max_u, rho_min=d.rho_min, rho_max=d.rho_max,
                    flag=d.flag, n_fluid=d.n_fluid)


def lbm_variant_count(lattice, precision):
    n = lib().lbm_variant_count(int(lattice), int(precision))
    if n < 0:
        _check(n, "lbm_variant_count")
    return n


def lbm_set_variant(ctx, variant):
    _check(lib().lbm_set_variant(ctx, int(variant)), "lbm_set_variant")


def lbm_get_variant(ctx):
    v = C.c_int32()
    _check(lib().lbm_get_variant(ctx, C.byref(v)), "lbm_get_variant")
    return v.value


def lbm_autotune_save_bytes(ctx):
    return lib().lbm_autotune_save_bytes(ctx)


def lbm_autotune(ctx, steps, save=None, nvariants=None):
    """Returns (best variant, per-variant ms list or None)."""
    best = C.c_int32()
    ms = (C.c_double * nvariants)() if nvariants else None
    _check(lib().lbm_autotune(ctx, int(steps), _ptr(save), C.byref(best), ms), "lbm_autotune")
    return best.value, (list(ms) if ms is not None else None)


def lbm_adjoint_workspace_bytes(ctx, K):
    return lib().lbm_adjoint_workspace_bytes(ctx, int(K))


def lbm_step_ckpt(ctx, T, K, ckpt):
    _check(lib().lbm_step_ckpt(ctx, int(T), int(K), _ptr(ckpt)), "lbm_step_ckpt")


def lbm_adjoint(ctx, seed_kind, seed, T, K, ckpt, work, grad_phi=None, grad_drho=None, lam0=None):
    _check(lib().lbm_adjoint(ctx, int(seed_kind), _ptr(seed), int(T), int(K), _ptr(ckpt),
                             _ptr(work), work.numel() * work.element_size(), _ptr(grad_phi),
                             _ptr(grad_drho), _ptr(lam0)), "lbm_adjoint")


def lbm_adjoint_noalloc(ctx, seed_kind, seed, T, K, ckpt, grad_phi=None, grad_drho=None,
                        lam0=None):
    _check(lib().lbm_adjoint_noalloc(ctx, int(seed_kind), _ptr(seed), int(T), int(K), _ptr(ckpt),
                                     _ptr(grad_phi), _ptr(grad_drho), _ptr(lam0)),
           "lbm_adjoint_noalloc")


LBM_NOALLOC_SCRATCH_BYTES = 64 << 20


def lbm_set_graph_steps(ctx, steps):
    _check(lib().lbm_set_graph_steps(ctx, int(steps)), "lbm_set_graph_steps")


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(C.POINTER(C.c_int64))


def lbm_batch_workspace_bytes(p, nx, ny, n_wall_max):
    ax, px = _i32(nx)
    ay, py = _i32(ny)
    aw, pw = _i64(n_wall_max)
    return lib().lbm_batch_workspace_bytes(C.byref(p), len(ax), px, py, pw)


def lbm_create_batch(p, nx, ny, n_wall_max, stream, workspace):
    ax, px = _i32(nx)
    ay, py = _i32(ny)
    aw, pw = _i64(n_wall_max)
    ctx = C.c_void_p()
    _check(lib().lbm_create_batch(C.byref(p), len(ax), px, py, pw, C.c_void_p(stream),
                                  _ptr(workspace), workspace.numel(), C.byref(ctx)),
           "lbm_create_batch")
    return ctx


def lbm_set_geometry_case(ctx, i, solid):
    s = np.ascontiguousarray(np.asarray(solid, dtype=np.uint8).ravel())
    _check(lib().lbm_set_geometry_case(ctx, int(i), s.ctypes.data_as(C.POINTER(C.c_uint8))),
           "lbm_set_geometry_case")


def lbm_wall_nodes_case(ctx, i):
    n = C.c_int64()
    _check(lib().lbm_wall_nodes_case(ctx, int(i), None, C.byref(n)), "lbm_wall_nodes_case")
    idx = np.zeros(max(n.value, 1), dtype=np.int64)
    _check(lib().lbm_wall_nodes_case(ctx, int(i), idx.ctypes.data_as(C.POINTER(C.c_int64)),
                                     C.byref(n)), "lbm_wall_nodes_case")
    return idx[:n.value]


def lbm_set_wetting_case(ctx, i, phi=None, drho=None, phi0=1.0, drho0=0.0):
    _check(lib().lbm_set_wetting_case(ctx, int(i), _ptr(phi), _ptr(drho), float(phi0),
                                      float(drho0)), "lbm_set_wetting_case")


def lbm_set_fields_case(ctx, i, rho, u=None):
    _check(lib().lbm_set_fields_case(ctx, int(i), _ptr(rho), _ptr(u)), "lbm_set_fields_case")


def lbm_get_fields_case(ctx, i, rho=None, u=None, f=None):
    _check(lib().lbm_get_fields_case(ctx, int(i), _ptr(rho), _ptr(u), _ptr(f)),
           "lbm_get_fields_case")


def lbm_get_diagnostics_case(ctx, i):
    d = lbm_diag()
    rc = lib().lbm_get_diagnostics_case(ctx, int(i), C.byref(d))
    if rc not in (LBM_OK, LBM_EDOMAIN):
        _check(rc, "lbm_get_diagnostics_case")
    return rc, dict(mass=d.mass, max_u=d.max_u, rho_min=d.rho_min, rho_max=d.rho_max,
                    flag=d.flag, n_fluid=d.n_fluid)


# ---------------------------------------------------------------- helpers
def make_params(lattice=9, precision=4, nx=64, ny=64, nz=1, tau=1.0, eos=LBM_EOS_CS,
                a=1.0, b=4.0, R=1.0, T=None, T_ratio=0.75, omega=0.344, G=-1.0, sigma=0.0,
                body_force=(0.0, 0.0, 0.0), rho_g=None, rho_l=None):
    """Parameter block; T defaults to T_ratio * Tc and the limiter bounds to
    the Maxwell coexistence densities, both from the library's EOS helpers."""
    p = lbm_params()
    p.lattice, p.precision, p.nx, p.ny, p.nz, p.eos = lattice, precision, nx, ny, nz, eos
    taus = np.full(19, float(tau)) if np.ndim(tau) == 0 else np.asarray(tau, float)
    for i in range(19):
        p.tau[i] = float(taus[i]) if i < len(taus) else 1.0
    p.eos_a, p.eos_b, p.eos_R, p.eos_omega = a, b, R, omega
    if T is None:
        Tc, _ = lbm_eos_critical(eos, a, b, R, omega)
        T = T_ratio * Tc
    p.eos_T = T
    p.G, p.sigma = G, sigma
    for i in range(3):
        p.body_force[i] = body_force[i]
    if rho_g is None or rho_l is None:
        p.rho_g, p.rho_l = 0.1, 1.0  # placeholders for the coexistence call
        g, l = lbm_eos_coexistence(p)
        rho_g = g if rho_g is None else rho_g
        rho_l = l if rho_l is None else rho_l
    p.rho_g, p.rho_l = rho_g, rho_l
    return p


class Solver:
    """One lattice on one GPU: owns the workspace tensor and the context."""

    def __init__(self, params, n_wall_max, device="cuda:0", stream=None):
        self.p = params
        self.device = torch.device(device)
        self.dtype = torch.float32 if params.precision == 4 else torch.float64
        self.N = params.nx * params.ny * params.nz
        self.Q = params.lattice
        self.D = 2 if params.lattice == 9 else 3
        nbytes = lbm_workspace_bytes(params, n_wall_max)
        if nbytes == 0:
            raise LBMError(LBM_EINVAL, "lbm_workspace_bytes", lib().lbm_last_error().decode())
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = lbm_create(params, self.stream.cuda_stream, self.ws, n_wall_max)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_geometry(self, solid):
        lbm_set_geometry(self.ctx, solid)
        # fluid-node mask on the device (the seed of the adjoint uses only
        # fluid entries; LBMRollout returns rho on fluid nodes only)
        self.fluid = torch.as_tensor(np.asarray(solid).ravel() == 0, device=self.device)

    def wall_nodes(self):
        return lbm_wall_nodes(self.ctx)

    def set_wetting(self, scheme, scalar=0.0, phi=None, drho=None, phi0=1.0, drho0=0.0):
        lbm_set_wetting(self.ctx, scheme, scalar, phi, drho, phi0, drho0)

    def set_fields(self, rho, u=None):
        rho = torch.as_tensor(rho, dtype=self.dtype, device=self.device).contiguous().view(-1)
        if u is not None:
            u = torch.as_tensor(u, dtype=self.dtype, device=self.device).contiguous().view(-1)
        lbm_set_fields(self.ctx, rho, u)
        self._keep = (rho, u)  # inputs stay alive until the stream consumed them

    def set_state(self, f):
        f = torch.as_tensor(f, dtype=self.dtype, device=self.device).contiguous()
        lbm_set_state(self.ctx, f)
        self._keep = (f,)

    def step(self, n):
        lbm_step(self.ctx, n)

    def step_timed(self, n):
        return lbm_step_timed(self.ctx, n)

    def get_fields(self, rho=True, u=True, f=False):
        r = torch.empty(self.N, dtype=self.dtype, device=self.device) if rho else None
        v = torch.empty(self.D * self.N, dtype=self.dtype, device=self.device) if u else None
        g = torch.empty(self.Q * self.N, dtype=self.dtype, device=self.device) if f else None
        lbm_get_fields(self.ctx, r, v, g)
        out = {}
        if rho:
            out["rho"] = r
        if u:
            out["u"] = v.view(self.D, self.N)
        if f:
            out["f"] = g.view(self.Q, self.N)
        return out

    def diagnostics(self):
        return lbm_get_diagnostics(self.ctx)

    def autotune(self, steps=20, report=False):
        """Pick the fastest step-kernel variant on this problem; the state is
        saved and restored around the trials."""
        save = torch.empty(lbm_autotune_save_bytes(self.ctx), dtype=torch.uint8, device=self.device)
        nv = lbm_variant_count(self.p.lattice, self.p.precision) if report else None
        best, ms = lbm_autotune(self.ctx, steps, save, nv)
        torch.cuda.synchronize(self.device)
        return (best, ms) if report else best

    @property
    def variant(self):
        return lbm_get_variant(self.ctx)

    @variant.setter
    def variant(self, v):
        lbm_set_variant(self.ctx, v)

    def set_graph_steps(self, steps):
        lbm_set_graph_steps(self.ctx, steps)

    # ---- checkpointed runs and the adjoint
    def ckpt_buffer(self, T, K):
        nseg = (int(T) + int(K) - 1) // int(K)
        return torch.empty(nseg * self.Q * self.N, dtype=self.dtype, device=self.device)

    def step_ckpt(self, T, K, ckpt):
        lbm_step_ckpt(self.ctx, T, K, ckpt)

    def adjoint(self, seed, T, K, ckpt, seed_kind=0, want_lam0=False):
        """Gradients of a loss on the state at time T: seed is dL/drho(T)
        (seed_kind 0) or dL/df(T) (seed_kind 1).  Returns (dL/dphi,
        dL/ddrho[, dL/df(0)])."""
        nw = len(self.wall_nodes())
        work = torch.empty(lbm_adjoint_workspace_bytes(self.ctx, K), dtype=torch.uint8,
                           device=self.device)
        gp = torch.empty(max(nw, 1), dtype=self.dtype, device=self.device)
        gd = torch.empty(max(nw, 1), dtype=self.dtype, device=self.device)
        lam0 = torch.empty(self.Q * self.N, dtype=self.dtype, device=self.device) if want_lam0 else None
        seed = torch.as_tensor(seed, dtype=self.dtype, device=self.device).contiguous().view(-1)
        lbm_adjoint(self.ctx, seed_kind, seed, T, K, ckpt, work, gp, gd, lam0)
        out = (gp[:nw], gd[:nw])
        if want_lam0:
            out = out + (lam0.view(self.Q, self.N),)
        return out


class LBMRollout(torch.autograd.Function):
    """rho(T) of a D2Q9 lattice as a differentiable function of the
    per-wall-node parameters (phi, drho) of the improved virtual-density
    scheme.  Forward: T steps from the initial density rho0 with
    checkpoints every K steps; returns rho(T) on the fluid nodes and 0 on
    every solid node (the wall nodes' virtual densities are left out, so
    any loss of the output is a function of the fluid state only).
    Backward: the hand-written discrete adjoint (checkpointed
    recomputation), seeded with dL/drho(T) on the fluid nodes, under the
    parameters of this forward (set again before the adjoint runs, in case
    the solver was used in between)."""

    @staticmethod
    def forward(ctx, phi, drho, solver, rho0, T, K):
        phi_d, drho_d = phi.detach().contiguous().clone(), drho.detach().contiguous().clone()
        solver.set_wetting(LBM_WET_IVD, 0.0, phi_d, drho_d)
        solver.set_fields(rho0)
        ckpt = solver.ckpt_buffer(T, K)
        solver.step_ckpt(T, K, ckpt)
        rho_T = solver.get_fields(rho=True, u=False)["rho"]
        rho_T = torch.where(solver.fluid, rho_T, torch.zeros_like(rho_T))
        ctx.solver, ctx.T, ctx.K, ctx.ckpt = solver, T, K, ckpt
        ctx.phi, ctx.drho = phi_d, drho_d
        return rho_T

    @staticmethod
    def backward(ctx, grad_rho):
        ctx.solver.set_wetting(LBM_WET_IVD, 0.0, ctx.phi, ctx.drho)
        gp, gd = ctx.solver.adjoint(grad_rho.contiguous(), ctx.T, ctx.K, ctx.ckpt)
        return gp, gd, None, None, None, None


class BatchSolver:
    """Many independent D2Q9 lattices advanced together (one launch per
    step, optionally replayed from a HIP graph)."""

    def __init__(self, params, sizes, n_wall_max, device="cuda:0", stream=None):
        self.p = params
        self.device = torch.device(device)
        self.dtype = torch.float32 if params.precision == 4 else torch.float64
        self.sizes = [(int(a), int(b)) for a, b in sizes]
        nx = [a for a, _ in self.sizes]
        ny = [b for _, b in self.sizes]
        nbytes = lbm_batch_workspace_bytes(params, nx, ny, n_wall_max)
        if nbytes == 0:
            raise LBMError(LBM_EINVAL, "lbm_batch_workspace_bytes", lib().lbm_last_error().decode())
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = lbm_create_batch(params, nx, ny, n_wall_max, self.stream.cuda_stream, self.ws)
        self._keep = []

    def close(self):
        if getattr(self, "ctx", None) is not None:
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.sizes)

    def set_geometry(self, i, solid):
        lbm_set_geometry_case(self.ctx, i, solid)

    def wall_nodes(self, i):
        return lbm_wall_nodes_case(self.ctx, i)

    def set_scheme(self, scheme, scalar=0.0, phi0=1.0, drho0=0.0):
        lbm_set_wetting(self.ctx, scheme, scalar, None, None, phi0, drho0)

    def set_wetting(self, i, phi=None, drho=None, phi0=1.0, drho0=0.0):
        lbm_set_wetting_case(self.ctx, i, phi, drho, phi0, drho0)

    def set_fields(self, i, rho, u=None):
        rho = torch.as_tensor(rho, dtype=self.dtype, device=self.device).contiguous().view(-1)
        if u is not None:
            u = torch.as_tensor(u, dtype=self.dtype, device=self.device).contiguous().view(-1)
        lbm_set_fields_case(self.ctx, i, rho, u)
        self._keep.append((rho, u))

    def step(self, n):
        lbm_step(self.ctx, n)

    def step_timed(self, n):
        return lbm_step_timed(self.ctx, n)

    def set_graph_steps(self, steps):
        lbm_set_graph_steps(self.ctx, steps)

    def get_fields(self, i, rho=True, u=True, f=False):
        nx, ny = self.sizes[i]
        N = nx * ny
        r = torch.empty(N, dtype=self.dtype, device=self.device) if rho else None
        v = torch.empty(2 * N, dtype=self.dtype, device=self.device) if u else None
        g = torch.empty(9 * N, dtype=self.dtype, device=self.device) if f else None
        lbm_get_fields_case(self.ctx, i, r, v, g)
        out = {}
        if rho:
            out["rho"] = r
        if u:
            out["u"] = v.view(2, N)
        if f:
            out["f"] = g.view(9, N)
        return out

    def diagnostics(self, i=None):
        if i is None:
            return lbm_get_diagnostics(self.ctx)
        return lbm_get_diagnostics_case(self.ctx, i)

    def autotune(self, steps=10, report=False):
        save = torch.empty(lbm_autotune_save_bytes(self.ctx), dtype=torch.uint8, device=self.device)
        nv = lbm_variant_count(9, self.p.precision) if report else None
        best, ms = lbm_autotune(self.ctx, steps, save, nv)
        torch.cuda.synchronize(self.device)
        return (best, ms) if report else best

    @property
    def variant(self):
        return lbm_get_variant(self.ctx)

    @variant.setter
    def variant(self, v):
        lbm_set_variant(self.ctx, v)
