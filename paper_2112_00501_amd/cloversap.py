"""Python binding of the cloversap C ABI (include/cloversap.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  torch provides device memory and streams.  The library must be
built (paper_2112_00501_amd/build.py); importing this module without it
raises, so no code path can fall back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcloversap.so")

F64, F32, F16, BF16 = 0, 1, 2, 3
PREC = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16}
SITE_BYTES = {F64: 192, F32: 96, F16: 52, BF16: 52}

CS_OK, CS_NOT_CONVERGED, CS_BREAKDOWN, CS_NONFINITE = 0, 1, 2, 3
CS_ANTIPERIODIC_T = 1


class CloverSapError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


class _Params(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_iter", C.c_int), ("n_cy", C.c_int), ("n_mr", C.c_int),
                ("tol", C.c_double), ("inner_prec", C.c_int), ("basis_prec", C.c_int),
                ("reliable_delta", C.c_double), ("rhs_tile", C.c_int), ("use_graph", C.c_int),
                ("block_solver", C.c_int), ("rhs_groups", C.c_int)]


class LaunchConfig(C.Structure):
    """Multi-right-hand-side launch shape (cs_launch_config)."""
    _fields_ = [("rhs_tile", C.c_int), ("persistent_wgs", C.c_int), ("lanes_per_site", C.c_int)]

    def __repr__(self):
        return (f"LaunchConfig(rhs_tile={self.rhs_tile}, persistent_wgs={self.persistent_wgs}, "
                f"lanes_per_site={self.lanes_per_site})")


class _MgParams(C.Structure):
    _fields_ = [("nv", C.c_int), ("n_cy_setup", C.c_int), ("n_mr", C.c_int), ("n_adapt", C.c_int),
                ("n_coarse", C.c_int), ("n_cy_post", C.c_int), ("tol_coarse", C.c_double),
                ("coarse_prec", C.c_int), ("transfer_prec", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("true_relres", C.c_double),
                ("seconds", C.c_double)]


_lib = None

EXPORTED = ["cs_last_error", "cs_strerror", "cs_lattice_create", "cs_lattice_destroy",
            "cs_lattice_volume", "cs_field_bytes", "cs_field_import", "cs_field_export",
            "cs_gauge_create", "cs_gauge_destroy", "cs_clover_create", "cs_clover_destroy",
            "cs_clover_export", "cs_clover_inverse_export", "cs_apply_D", "cs_apply_Ddag",
            "cs_apply_D_cfg", "cs_sap_smooth", "cs_sap_smooth_cfg", "cs_sap_smooth_jacobi", "cs_sap_smooth_eo",
            "cs_autotune", "cs_solver_params_default", "cs_gcr_solve", "cs_gcr_solve_dag",
            "cs_bicgstab_solve", "cs_mg_params_default", "cs_mg_create", "cs_mg_destroy",
            "cs_mg_export", "cs_mg_restrict", "cs_mg_prolong", "cs_mg_coarse_apply",
            "cs_mg_coarse_solve", "cs_mg_apply", "cs_gcr_solve_mg", "cs_bicgstab_solve_mg", "cs_force",
            "cs_force_noalloc",
            "cs_profile_enable",
            "cs_profile_query", "cs_profile_reset", "cs_device_copy", "cs_probe_link_product"]


def load_library(path: str = LIB_PATH):
    """Load libcloversap.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2112_00501_amd/build.py "
                           "(or __graft_entry__.build())")
    L = C.CDLL(path)
    P, I, D = C.c_void_p, C.c_int, C.c_double
    I4 = C.c_int * 4
    L.cs_last_error.restype = C.c_char_p
    L.cs_strerror.restype = C.c_char_p
    L.cs_strerror.argtypes = [I]
    L.cs_lattice_create.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int), I, C.POINTER(P)]
    L.cs_lattice_destroy.argtypes = [P]
    L.cs_lattice_volume.argtypes = [P]
    L.cs_lattice_volume.restype = C.c_longlong
    L.cs_field_bytes.argtypes = [P, I, I]
    L.cs_field_bytes.restype = C.c_size_t
    L.cs_field_import.argtypes = [P, I, P, P, I, P]
    L.cs_field_export.argtypes = [P, I, P, P, I, P]
    L.cs_gauge_create.argtypes = [P, P, P, C.POINTER(P)]
    L.cs_gauge_destroy.argtypes = [P]
    L.cs_clover_create.argtypes = [P, D, D, P, C.POINTER(P)]
    L.cs_clover_destroy.argtypes = [P]
    L.cs_clover_export.argtypes = [P, P, P]
    L.cs_clover_inverse_export.argtypes = [P, P, P]
    L.cs_apply_D.argtypes = [P, P, I, P, P, I, P]
    L.cs_apply_Ddag.argtypes = [P, P, I, P, P, I, P]
    L.cs_sap_smooth.argtypes = [P, P, I, P, P, I, I, I, I, P]
    L.cs_sap_smooth_cfg.argtypes = [P, P, I, P, P, I, I, I, I, C.POINTER(LaunchConfig), P]
    L.cs_sap_smooth_jacobi.argtypes = [P, P, I, P, P, I, I, I, I, C.POINTER(LaunchConfig), P]
    L.cs_sap_smooth_eo.argtypes = [P, P, I, P, P, I, I, I, I, C.POINTER(LaunchConfig), P]
    L.cs_apply_D_cfg.argtypes = [P, P, I, P, P, I, C.POINTER(LaunchConfig), P]
    L.cs_autotune.argtypes = [P, P, I, I, C.POINTER(LaunchConfig), C.POINTER(LaunchConfig), P]
    L.cs_solver_params_default.argtypes = [C.POINTER(_Params)]
    L.cs_solver_params_default.restype = None
    L.cs_gcr_solve.argtypes = [P, P, C.POINTER(_Params), P, P, I, C.POINTER(_Stats), P]
    L.cs_gcr_solve_dag.argtypes = [P, P, C.POINTER(_Params), P, P, I, C.POINTER(_Stats), P]
    L.cs_bicgstab_solve.argtypes = [P, P, C.POINTER(_Params), P, P, C.POINTER(_Stats), P]
    L.cs_mg_params_default.argtypes = [C.POINTER(_MgParams)]
    L.cs_mg_params_default.restype = None
    L.cs_mg_create.argtypes = [P, P, C.POINTER(_MgParams), P, P, C.POINTER(P)]
    L.cs_mg_destroy.argtypes = [P]
    L.cs_mg_export.argtypes = [P, P, P, P]
    L.cs_mg_restrict.argtypes = [P, P, P, P]
    L.cs_mg_prolong.argtypes = [P, P, P, P]
    L.cs_mg_coarse_apply.argtypes = [P, P, P, P]
    L.cs_mg_coarse_solve.argtypes = [P, P, P, I, D, P]
    L.cs_mg_apply.argtypes = [P, P, P, P]
    L.cs_gcr_solve_mg.argtypes = [P, P, P, C.POINTER(_Params), P, P, C.POINTER(_Stats), P]
    L.cs_bicgstab_solve_mg.argtypes = [P, P, P, C.POINTER(_Params), P, P, C.POINTER(_Stats), P]
    L.cs_force.argtypes = [P, P, P, P, P, P, P]
    L.cs_force_noalloc.argtypes = [P, P, P, P, P, P, P]
    L.cs_profile_enable.argtypes = [I]
    L.cs_profile_query.argtypes = [C.c_char_p, C.POINTER(C.c_longlong), C.POINTER(C.c_double)]
    L.cs_profile_reset.argtypes = []
    L.cs_device_copy.argtypes = [P, P, C.c_size_t, P]
    L.cs_probe_link_product.argtypes = [I, C.c_longlong, I, P, P, P, P]
    _lib = L
    return L


def _check(status, where, allow=()):
    if status != CS_OK and status not in allow:
        msg = _lib.cs_last_error().decode()
        raise CloverSapError(status, where, msg)
    return status


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _need(t: torch.Tensor, nbytes: int, what: str):
    """Refuse a device buffer smaller than the kernels will touch (the C ABI
    takes raw pointers and cannot check)."""
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise ValueError(f"{what}: buffer of {have} bytes, {nbytes} needed")
    return t


def _ptr(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


class Lattice:
    """Geometry with 4^4 blocks.  dims = (Lx, Ly, Lz, Lt); antiperiodic_t:
    fermion fields antiperiodic in time (default periodic)."""

    def __init__(self, dims, block=(4, 4, 4, 4), antiperiodic_t=False):
        L = load_library()
        self.dims = tuple(int(d) for d in dims)
        self.block = tuple(int(b) for b in block)
        self.antiperiodic_t = bool(antiperiodic_t)
        h = C.c_void_p()
        _check(L.cs_lattice_create((C.c_int * 4)(*self.dims), (C.c_int * 4)(*self.block),
                                   CS_ANTIPERIODIC_T if self.antiperiodic_t else 0, C.byref(h)),
               "cs_lattice_create")
        self.handle = h
        self.volume = int(L.cs_lattice_volume(h))

    def field_bytes(self, prec: int, nrhs: int = 1) -> int:
        return int(_lib.cs_field_bytes(self.handle, prec, nrhs))

    def new_field(self, prec: int, nrhs: int = 1, device="cuda") -> torch.Tensor:
        """Uninitialised internal-layout field (a uint8 tensor of the right size)."""
        return torch.empty(self.field_bytes(prec, nrhs), dtype=torch.uint8, device=device)

    def import_field(self, canonical: torch.Tensor, prec: int, out: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
        """canonical complex128 [nrhs][V][4][3] or [V][4][3] (GPU) -> internal field."""
        if canonical.dtype != torch.complex128:
            raise ValueError("canonical spinors are complex128")
        nrhs = canonical.numel() // (self.volume * 12)
        if nrhs * self.volume * 12 != canonical.numel():
            raise ValueError("canonical field has the wrong size")
        if out is None:
            out = self.new_field(prec, nrhs, canonical.device)
        _need(out, self.field_bytes(prec, nrhs), "import_field out")
        _check(_lib.cs_field_import(self.handle, prec, _ptr(out), _ptr(canonical), nrhs,
                                    _stream(stream)), "cs_field_import")
        return out

    def export_field(self, internal: torch.Tensor, prec: int, nrhs: int = 1,
                     stream=None) -> torch.Tensor:
        _need(internal, self.field_bytes(prec, nrhs), "export_field internal")
        shape = (self.volume, 4, 3) if nrhs == 1 else (nrhs, self.volume, 4, 3)
        out = torch.empty(shape, dtype=torch.complex128, device=internal.device)
        _check(_lib.cs_field_export(self.handle, prec, _ptr(out), _ptr(internal), nrhs,
                                    _stream(stream)), "cs_field_export")
        return out

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cs_lattice_destroy(self.handle)
            self.handle = None


class Gauge:
    """Links, compressed on the device.  U: complex128 [V][4][3][3] on the GPU."""

    def __init__(self, lat: Lattice, U: torch.Tensor, stream=None):
        if U.dtype != torch.complex128 or U.numel() != lat.volume * 36:
            raise ValueError("U must be complex128 [V][4][3][3]")
        self.lat = lat
        h = C.c_void_p()
        _check(_lib.cs_gauge_create(lat.handle, _ptr(U), _stream(stream), C.byref(h)),
               "cs_gauge_create")
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cs_gauge_destroy(self.handle)
            self.handle = None


class Clover:
    """C = 1 + T for (kappa, c_sw), built on the device from the gauge field."""

    def __init__(self, gauge: Gauge, kappa: float, csw: float, stream=None):
        self.gauge = gauge
        self.kappa, self.csw = float(kappa), float(csw)
        h = C.c_void_p()
        _check(_lib.cs_clover_create(gauge.handle, self.kappa, self.csw, _stream(stream),
                                     C.byref(h)), "cs_clover_create")
        self.handle = h

    def export(self, stream=None) -> torch.Tensor:
        lat = self.gauge.lat
        out = torch.empty((lat.volume, 12, 12), dtype=torch.complex128, device="cuda")
        _check(_lib.cs_clover_export(self.handle, _ptr(out), _stream(stream)), "cs_clover_export")
        return out

    def export_inverse(self, stream=None) -> torch.Tensor:
        """(1 + T)^-1 as complex128 [V][12][12] on the GPU."""
        lat = self.gauge.lat
        out = torch.empty((lat.volume, 12, 12), dtype=torch.complex128, device="cuda")
        _check(_lib.cs_clover_inverse_export(self.handle, _ptr(out), _stream(stream)),
               "cs_clover_inverse_export")
        return out

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cs_clover_destroy(self.handle)
            self.handle = None


class Operator:
    """The clover-Wilson operator D of one gauge field and (kappa, c_sw)."""

    def __init__(self, lat: Lattice, U: torch.Tensor, kappa: float, csw: float, stream=None):
        self.lat = lat
        self.gauge = Gauge(lat, U, stream)
        self.clover = Clover(self.gauge, kappa, csw, stream)

    def _fields(self, ts, prec, nrhs):
        for t in ts:
            _need(t, self.lat.field_bytes(prec, nrhs), "field")

    def apply_D(self, out, inp, prec, nrhs=1, stream=None):
        self._fields((out, inp), prec, nrhs)
        _check(_lib.cs_apply_D(self.gauge.handle, self.clover.handle, prec, _ptr(out), _ptr(inp),
                               nrhs, _stream(stream)), "cs_apply_D")
        return out

    def apply_D_cfg(self, out, inp, prec, nrhs, cfg: "LaunchConfig", stream=None):
        self._fields((out, inp), prec, nrhs)
        _check(_lib.cs_apply_D_cfg(self.gauge.handle, self.clover.handle, prec, _ptr(out), _ptr(inp),
                                   nrhs, C.byref(cfg), _stream(stream)), "cs_apply_D_cfg")
        return out

    def sap_smooth_cfg(self, x, b, prec, nrhs, cfg: "LaunchConfig", n_cy=2, n_mr=4,
                       x0_is_zero=True, stream=None):
        self._fields((x, b), prec, nrhs)
        _check(_lib.cs_sap_smooth_cfg(self.gauge.handle, self.clover.handle, prec, _ptr(x), _ptr(b),
                                      int(n_cy), int(n_mr), int(bool(x0_is_zero)), nrhs,
                                      C.byref(cfg), _stream(stream)), "cs_sap_smooth_cfg")
        return x

    def sap_smooth_jacobi(self, x, b, prec, n_cy=2, n_jac=4, x0_is_zero=True, nrhs=1, cfg=None,
                          stream=None):
        """SAP on C^-1 D with n_jac Jacobi steps per block (the QWS smoother form)."""
        self._fields((x, b), prec, nrhs)
        _check(_lib.cs_sap_smooth_jacobi(self.gauge.handle, self.clover.handle, prec, _ptr(x), _ptr(b),
                                         int(n_cy), int(n_jac), int(bool(x0_is_zero)), nrhs,
                                         None if cfg is None else C.byref(cfg), _stream(stream)),
               "cs_sap_smooth_jacobi")
        return x

    def sap_smooth_eo(self, x, b, prec, n_cy=2, n_mr=4, x0_is_zero=True, nrhs=1, cfg=None, stream=None):
        """SAP with even-odd preconditioned MR block solves."""
        self._fields((x, b), prec, nrhs)
        _check(_lib.cs_sap_smooth_eo(self.gauge.handle, self.clover.handle, prec, _ptr(x), _ptr(b),
                                     int(n_cy), int(n_mr), int(bool(x0_is_zero)), nrhs,
                                     None if cfg is None else C.byref(cfg), _stream(stream)), "cs_sap_smooth_eo")
        return x

    def autotune(self, prec, nrhs, stream=None):
        """Fastest (SAP, operator) launch shapes for nrhs right-hand sides."""
        a, b = LaunchConfig(), LaunchConfig()
        _check(_lib.cs_autotune(self.gauge.handle, self.clover.handle, prec, nrhs, C.byref(a),
                                C.byref(b), _stream(stream)), "cs_autotune")
        return a, b

    def apply_Ddag(self, out, inp, prec, nrhs=1, stream=None):
        self._fields((out, inp), prec, nrhs)
        _check(_lib.cs_apply_Ddag(self.gauge.handle, self.clover.handle, prec, _ptr(out),
                                  _ptr(inp), nrhs, _stream(stream)), "cs_apply_Ddag")
        return out

    def sap_smooth(self, x, b, prec, n_cy=2, n_mr=4, x0_is_zero=True, nrhs=1, stream=None):
        self._fields((x, b), prec, nrhs)
        _check(_lib.cs_sap_smooth(self.gauge.handle, self.clover.handle, prec, _ptr(x), _ptr(b),
                                  int(n_cy), int(n_mr), int(bool(x0_is_zero)), nrhs,
                                  _stream(stream)), "cs_sap_smooth")
        return x

    def gcr_solve(self, x, b, params: "SolverParams", nrhs=1, stream=None, allow_fail=False,
                  dagger=False):
        """x, b: CS_F64 internal fields.  Solves D x = b (D^dag x = b with
        dagger).  Returns (status, [stats per rhs])."""
        self._fields((x, b), F64, nrhs)
        p = params.to_c()
        stats = (_Stats * nrhs)()
        fn = _lib.cs_gcr_solve_dag if dagger else _lib.cs_gcr_solve
        st = fn(self.gauge.handle, self.clover.handle, C.byref(p), _ptr(x), _ptr(b), nrhs, stats,
                _stream(stream))
        if not allow_fail:
            _check(st, "cs_gcr_solve_dag" if dagger else "cs_gcr_solve")
        out = [dict(iters=s.iters, restarts=s.restarts, true_relres=s.true_relres,
                    seconds=s.seconds) for s in stats]
        return st, out

    def bicgstab_solve(self, x, b, params: "SolverParams", stream=None, allow_fail=False):
        """x, b: one CS_F64 internal field each.  Solves D x = b with BiCGStab
        (SAP on the right): flexible BiCGStab with FP64 vectors when
        params.basis_prec is F64, FP32 inner solves inside an FP64 Richardson
        iteration when it is F32.  Returns (status, stats)."""
        self._fields((x, b), F64, 1)
        p = params.to_c()
        st_ = _Stats()
        st = _lib.cs_bicgstab_solve(self.gauge.handle, self.clover.handle, C.byref(p), _ptr(x), _ptr(b),
                                    C.byref(st_), _stream(stream))
        if not allow_fail:
            _check(st, "cs_bicgstab_solve")
        return st, dict(iters=st_.iters, restarts=st_.restarts, true_relres=st_.true_relres,
                        seconds=st_.seconds)

    def force(self, x, y, want_lie=True, want_grad=False, stream=None):
        """Link gradient of L given x = D^-1 b and y = D^-dag dL/dx (CS_F64
        internal fields).  Returns (g_lie [V][4][8] float64 or None,
        grad_U [V][4][3][3] complex128 or None), on the GPU."""
        self._fields((x, y), F64, 1)
        V = self.lat.volume
        g = torch.empty((V, 4, 8), dtype=torch.float64, device="cuda") if want_lie else None
        G = torch.empty((V, 4, 3, 3), dtype=torch.complex128, device="cuda") if want_grad else None
        _check(_lib.cs_force(self.gauge.handle, self.clover.handle, _ptr(x), _ptr(y),
                             None if g is None else _ptr(g), None if G is None else _ptr(G),
                             _stream(stream)), "cs_force")
        return g, G

    def force_noalloc(self, x, y, g_lie=None, grad_U=None, stream=None):
        """cs_force with the library's fixed workspace (no device allocation
        by the library): writes into the caller's g_lie (float64 [V][4][8])
        and/or grad_U (complex128 [V][4][3][3]) device tensors."""
        self._fields((x, y), F64, 1)
        V = self.lat.volume
        if g_lie is not None:
            _need(g_lie, V * 4 * 8 * 8, "g_lie")
        if grad_U is not None:
            _need(grad_U, V * 4 * 9 * 16, "grad_U")
        _check(_lib.cs_force_noalloc(self.gauge.handle, self.clover.handle, _ptr(x), _ptr(y),
                                     None if g_lie is None else _ptr(g_lie),
                                     None if grad_U is None else _ptr(grad_U), _stream(stream)),
               "cs_force_noalloc")


@dataclass
class MgParams:
    nv: int = 8             # null vectors; nc = 2 nv coarse values per aggregate
    n_cy_setup: int = 4     # SAP cycles turning each random vector into a null-vector candidate
    n_mr: int = 4           # MR steps per block solve in every SAP use
    n_adapt: int = 1        # adaptive passes v <- M_MG v
    n_coarse: int = 50      # coarse BiCGStab iteration cap per application
    n_cy_post: int = 2      # SAP post-smoothing cycles per application
    tol_coarse: float = 0.05
    coarse_prec: int = F32   # D_c storage read by the coarse solve: F32 or F16
    transfer_prec: int = F32  # P storage read by restriction and prolongation: F32 or F16

    def to_c(self) -> _MgParams:
        return _MgParams(self.nv, self.n_cy_setup, self.n_mr, self.n_adapt, self.n_coarse,
                         self.n_cy_post, self.tol_coarse, self.coarse_prec, self.transfer_prec)


class Multigrid:
    """Two-level multigrid hierarchy of one operator (cs_mg).  etas: nv
    consecutive F32 internal fields of random vectors."""

    def __init__(self, op: "Operator", etas: torch.Tensor, params: MgParams | None = None, stream=None):
        self.op = op
        self.params = params or MgParams()
        _need(etas, op.lat.field_bytes(F32, self.params.nv), "etas")
        p = self.params.to_c()
        h = C.c_void_p()
        _check(_lib.cs_mg_create(op.gauge.handle, op.clover.handle, C.byref(p), _ptr(etas),
                                 _stream(stream), C.byref(h)), "cs_mg_create")
        self.handle = h
        self.nv = self.params.nv
        self.nc = 2 * self.nv
        self.nblk = op.lat.volume // 256

    def new_coarse(self) -> torch.Tensor:
        """A coarse vector: complex64 [nblk][nc] (float2 per entry)."""
        return torch.zeros((self.nblk, self.nc), dtype=torch.complex64, device="cuda")

    def export(self, stream=None):
        """(P as nv F32 internal fields, D_c complex64 [nblk][9][nc (column)][nc (row)])."""
        P = self.op.lat.new_field(F32, self.nv)
        Dc = torch.empty((self.nblk, 9, self.nc, self.nc), dtype=torch.complex64, device="cuda")
        _check(_lib.cs_mg_export(self.handle, _ptr(P), _ptr(Dc), _stream(stream)), "cs_mg_export")
        return P, Dc

    def _coarse_bytes(self):
        return self.nblk * self.nc * 8

    def restrict(self, r, rc=None, stream=None):
        rc = self.new_coarse() if rc is None else rc
        _need(r, self.op.lat.field_bytes(F32), "r")
        _need(rc, self._coarse_bytes(), "rc")
        _check(_lib.cs_mg_restrict(self.handle, _ptr(r), _ptr(rc), _stream(stream)), "cs_mg_restrict")
        return rc

    def prolong(self, ec, z=None, stream=None):
        z = self.op.lat.new_field(F32) if z is None else z
        _need(ec, self._coarse_bytes(), "ec")
        _need(z, self.op.lat.field_bytes(F32), "z")
        _check(_lib.cs_mg_prolong(self.handle, _ptr(ec), _ptr(z), _stream(stream)), "cs_mg_prolong")
        return z

    def coarse_apply(self, x, y=None, stream=None):
        y = self.new_coarse() if y is None else y
        _need(x, self._coarse_bytes(), "x")
        _need(y, self._coarse_bytes(), "y")
        _check(_lib.cs_mg_coarse_apply(self.handle, _ptr(x), _ptr(y), _stream(stream)), "cs_mg_coarse_apply")
        return y

    def coarse_solve(self, rc, n_iter, tol=0.0, ec=None, stream=None):
        ec = self.new_coarse() if ec is None else ec
        _need(rc, self._coarse_bytes(), "rc")
        _need(ec, self._coarse_bytes(), "ec")
        _check(_lib.cs_mg_coarse_solve(self.handle, _ptr(rc), _ptr(ec), int(n_iter), float(tol),
                                       _stream(stream)), "cs_mg_coarse_solve")
        return ec

    def apply(self, r, z=None, stream=None):
        """z = M_MG r (F32 internal fields)."""
        z = self.op.lat.new_field(F32) if z is None else z
        _need(z, self.op.lat.field_bytes(F32), "z")
        _need(r, self.op.lat.field_bytes(F32), "r")
        _check(_lib.cs_mg_apply(self.handle, _ptr(z), _ptr(r), _stream(stream)), "cs_mg_apply")
        return z

    def gcr_solve(self, x, b, params: "SolverParams", stream=None, allow_fail=False):
        """Flexible GCR on D x = b (CS_F64 internal fields) preconditioned by
        M_MG.  Returns (status, stats)."""
        p = params.to_c()
        st_ = _Stats()
        _need(x, self.op.lat.field_bytes(F64), "x")
        _need(b, self.op.lat.field_bytes(F64), "b")
        st = _lib.cs_gcr_solve_mg(self.op.gauge.handle, self.op.clover.handle, self.handle, C.byref(p),
                                  _ptr(x), _ptr(b), C.byref(st_), _stream(stream))
        if not allow_fail:
            _check(st, "cs_gcr_solve_mg")
        return st, dict(iters=st_.iters, restarts=st_.restarts, true_relres=st_.true_relres,
                        seconds=st_.seconds)

    def bicgstab_solve(self, x, b, params: "SolverParams", stream=None, allow_fail=False):
        """Flexible BiCGStab on D x = b (CS_F64 internal fields) with M_MG on
        the right (params.basis_prec F64), or FP32 BiCGStab with M_MG inside
        the FP64 Richardson iteration (F32).  Returns (status, stats)."""
        p = params.to_c()
        st_ = _Stats()
        _need(x, self.op.lat.field_bytes(F64), "x")
        _need(b, self.op.lat.field_bytes(F64), "b")
        st = _lib.cs_bicgstab_solve_mg(self.op.gauge.handle, self.op.clover.handle, self.handle, C.byref(p),
                                       _ptr(x), _ptr(b), C.byref(st_), _stream(stream))
        if not allow_fail:
            _check(st, "cs_bicgstab_solve_mg")
        return st, dict(iters=st_.iters, restarts=st_.restarts, true_relres=st_.true_relres,
                        seconds=st_.seconds)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cs_mg_destroy(self.handle)
            self.handle = None


@dataclass
class SolverParams:
    restart: int = 16
    max_iter: int = 2000
    n_cy: int = 2
    n_mr: int = 4
    tol: float = 1e-10
    inner_prec: int = F32
    basis_prec: int = F32
    reliable_delta: float = 1e-5
    rhs_tile: int = 0
    use_graph: bool = True
    block_solver: int = 0     # 0: MR on D_BB; 1: Jacobi on (C^-1 D)_BB; 2: even-odd preconditioned MR (n_mr steps)
    rhs_groups: int = 1       # > 1: the batch split into that many groups solved concurrently

    def to_c(self) -> _Params:
        return _Params(self.restart, self.max_iter, self.n_cy, self.n_mr, self.tol,
                       self.inner_prec, self.basis_prec, self.reliable_delta, self.rhs_tile,
                       int(bool(self.use_graph)), int(self.block_solver), int(self.rhs_groups))


def profile_enable(on: bool = True):
    load_library()
    _check(_lib.cs_profile_enable(int(on)), "cs_profile_enable")


def profile_reset():
    _check(_lib.cs_profile_reset(), "cs_profile_reset")


def device_copy(dst: torch.Tensor, src: torch.Tensor, stream=None):
    """dst = src by the library's plain streaming-copy kernel (the bandwidth
    reference of the field kernels); both contiguous device tensors."""
    nbytes = src.numel() * src.element_size()
    _need(dst, nbytes, "device_copy dst")
    load_library()
    _check(_lib.cs_device_copy(_ptr(dst), _ptr(src), nbytes, _stream(stream)), "cs_device_copy")


def probe_link_product(kind: int, U: torch.Tensor, H: torch.Tensor, V: torch.Tensor, reps: int, stream=None):
    """cs_probe_link_product: U float32 [n][9][2], H and V float32 [n][16][3][2]
    device tensors; kind 0 FP32 VALU, 1 bfloat16 MFMA."""
    n = U.shape[0]
    for t, per in ((U, 18), (H, 96), (V, 96)):
        if t.dtype != torch.float32:
            raise ValueError("probe tensors are float32")
        _need(t, n * per * 4, "probe tensor")
    load_library()
    _check(_lib.cs_probe_link_product(int(kind), int(n), int(reps), _ptr(U), _ptr(H), _ptr(V), _stream(stream)),
           "cs_probe_link_product")


def profile_query(name: str):
    n = C.c_longlong(0)
    ms = C.c_double(0)
    _check(_lib.cs_profile_query(name.encode(), C.byref(n), C.byref(ms)), "cs_profile_query")
    return int(n.value), float(ms.value)


class CloverSolve(torch.autograd.Function):
    """x = D(U)^{-1} b as a differentiable torch operation.

    forward(U, b, lat, kappa, csw, params, recompute): U complex128
    [V][4][3][3] (SU(3)), b complex128 [V][4][3], both on the GPU; returns x
    (complex128).
    backward: the adjoint solve y = D^{-dag} grad_x (D^dag = gamma5 D gamma5,
    same solver), grad_b = y, and grad_U from the force kernel: the
    tangent-space gradient 2 i (sum_a g_a T^a) U, exact for any SU(3)-valued
    parametrisation of U.
    recompute = False keeps the operator (links and clover term in the
    library) and the FP64 solution between forward and backward; recompute =
    True keeps only references to U and b and rebuilds the operator and
    solves D x = b again in the backward pass (the solve is deterministic, so
    the gradient is the same bit for bit), for when device memory is short.
    """

    @staticmethod
    def forward(ctx, U, b, lat, kappa, csw, params=None, recompute=False):
        params = params or SolverParams(inner_prec=F32, basis_prec=F32)
        op = Operator(lat, U.detach().contiguous(), kappa, csw)
        bd = lat.import_field(b.detach().contiguous(), F64)
        xd = lat.new_field(F64).zero_()
        op.gcr_solve(xd, bd, params)
        x = lat.export_field(xd, F64)
        ctx.lat, ctx.params, ctx.kappa, ctx.csw, ctx.recompute = lat, params, kappa, csw, recompute
        if recompute:
            ctx.save_for_backward(U, b)
            ctx.op = ctx.xd = None
            del op, xd, bd
        else:
            ctx.op, ctx.xd = op, xd
        return x

    @staticmethod
    def backward(ctx, grad_x):
        lat = ctx.lat
        if ctx.recompute:
            U, b = ctx.saved_tensors
            op = Operator(lat, U.detach().contiguous(), ctx.kappa, ctx.csw)
            bd = lat.import_field(b.detach().contiguous(), F64)
            xd = lat.new_field(F64).zero_()
            op.gcr_solve(xd, bd, ctx.params)
            del bd
        else:
            op, xd = ctx.op, ctx.xd
        gd = lat.import_field(grad_x.detach().contiguous().to(torch.complex128), F64)
        yd = lat.new_field(F64).zero_()
        op.gcr_solve(yd, gd, ctx.params, dagger=True)
        grad_b = lat.export_field(yd, F64) if ctx.needs_input_grad[1] else None
        grad_U = None
        if ctx.needs_input_grad[0]:
            _, grad_U = op.force(xd, yd, want_lie=False, want_grad=True)
        ctx.op = ctx.xd = None
        return grad_U, grad_b, None, None, None, None, None
