"""ctypes wrapper of the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the GPU library or its binding.

All arrays are numpy complex128 in the canonical layouts documented in
oracle.h (U[V][4][3][3], psi[V][4][3], T[V][12][12]).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def _host_tag() -> str:
    """Short tag of this host's CPU (model and feature flags), so that a
    -march=native build is only ever loaded on the kind of CPU it was built
    for."""
    import hashlib
    h = hashlib.sha1()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith(("model name", "flags")):
                    h.update(line.encode())
                    if line.startswith("flags"):
                        break
    except OSError:
        h.update(b"unknown")
    return h.hexdigest()[:10]


_LIB_NATIVE = os.path.join(_HERE, f"liboracle_native_{_host_tag()}.so")

# Plain ISO C11 (so no floating-point contraction and no reassociation): the
# arithmetic is exactly what the source says.  The default library is built
# for generic x86-64 so that it runs on any host it is copied to; the native
# build (-march=native, for timing the oracle on the host it runs on) gives
# the same results, since neither build contracts or reorders operations.
BUILD_FLAGS = ["-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared"]


def build(native: bool = False) -> str:
    """Compile the oracle library (plain gcc; no GPU code)."""
    out = _LIB_NATIVE if native else _LIB
    tmp = out + ".tmp"
    cmd = ["gcc"] + BUILD_FLAGS + (["-march=native"] if native else []) + [_SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_lib = None
_native = False


def use_native_build() -> None:
    """Load the -march=native build (built here on first use) instead of the
    generic one; must be called before the first oracle call."""
    global _native
    if _lib is not None and not _native:
        raise RuntimeError("the generic oracle library is already loaded")
    _native = True


def build_flags() -> str:
    return " ".join(["gcc"] + BUILD_FLAGS + (["-march=native"] if _native else []))


def lib():
    global _lib
    if _lib is None:
        path = _LIB_NATIVE if _native else _LIB
        hdr = os.path.join(os.path.dirname(_SRC), "oracle.h")
        if not os.path.exists(path) or os.path.getmtime(path) < max(os.path.getmtime(_SRC),
                                                                     os.path.getmtime(hdr)):
            build(native=_native)
        _lib = C.CDLL(path)
        _declare(_lib)
    return _lib


_P = C.c_void_p
_I4 = C.c_int * 4


def _declare(L):
    L.or_set_threads.argtypes = [C.c_int]
    L.or_get_threads.restype = C.c_int
    L.or_gamma.argtypes = [C.c_int, _P]
    L.or_sigma.argtypes = [C.c_int, C.c_int, _P]
    L.or_clover_site.argtypes = [_I4, _P, C.c_double, C.c_double, C.c_long, _P]
    L.or_clover_field.argtypes = [_I4, _P, C.c_double, C.c_double, _P]
    L.or_leaf_sum.argtypes = [_I4, _P, C.c_long, C.c_int, C.c_int, _P]
    L.or_apply_D.argtypes = [_I4, _P, _P, C.c_double, _P, _P]
    L.or_apply_Ddag.argtypes = [_I4, _P, _P, C.c_double, _P, _P]
    L.or_apply_D_sites.argtypes = [_I4, _P, C.c_double, C.c_double, _P, C.c_long, _P, _P]
    L.or_residual_norm.argtypes = [_I4, _P, C.c_double, C.c_double, _P, _P]
    L.or_residual_norm.restype = C.c_double
    L.or_num_blocks.argtypes = [_I4, _I4]
    L.or_num_blocks.restype = C.c_long
    L.or_block_colour.argtypes = [_I4, _I4, C.c_long]
    L.or_block_colour.restype = C.c_int
    L.or_block_of_site.argtypes = [_I4, _I4, C.c_long]
    L.or_block_of_site.restype = C.c_long
    L.or_apply_D_block.argtypes = [_I4, _I4, C.c_long, _P, _P, C.c_double, _P, _P]
    L.or_mr_block.argtypes = [_I4, _I4, C.c_long, _P, _P, C.c_double, C.c_int, _P, _P]
    L.or_sap.argtypes = [_I4, _I4, _P, _P, C.c_double, C.c_int, C.c_int, _P, _P]
    L.or_clover_inverse_field.argtypes = [_I4, _P, _P]
    L.or_jacobi_block.argtypes = [_I4, _I4, C.c_long, _P, _P, C.c_double, C.c_int, _P, _P]
    L.or_sap_jacobi.argtypes = [_I4, _I4, _P, _P, C.c_double, C.c_int, C.c_int, _P, _P]
    L.or_mr_eo_block.argtypes = [_I4, _I4, C.c_long, _P, _P, C.c_double, C.c_int, _P, _P]
    L.or_sap_eo.argtypes = [_I4, _I4, _P, _P, C.c_double, C.c_int, C.c_int, _P, _P]
    L.or_fgcr.argtypes = [_I4, _I4, _P, _P, C.c_double, C.c_int, C.c_int, C.c_int,
                          C.c_double, C.c_int, _P, _P, C.POINTER(C.c_int),
                          C.POINTER(C.c_double), _P]
    L.or_fgcr.restype = C.c_int
    L.or_fbicgstab.argtypes = [_I4, _I4, _P, _P, C.c_double, C.c_int, C.c_int, C.c_double,
                               C.c_int, C.c_double, _P, _P, C.POINTER(C.c_int),
                               C.POINTER(C.c_int), C.POINTER(C.c_double), _P]
    L.or_fbicgstab.restype = C.c_int
    L.or_richardson_bicgstab.argtypes = [_I4, _I4, _P, _P, C.c_double, C.c_int, C.c_int, C.c_double,
                                         C.c_int, C.c_double, _P, _P, C.POINTER(C.c_int),
                                         C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.or_richardson_bicgstab.restype = C.c_int
    L.or_force.argtypes = [_I4, _P, C.c_double, C.c_double, _P, _P, _P, _P]
    L.or_su3_generator.argtypes = [C.c_int, _P]


def _dims(d):
    return _I4(*[int(v) for v in d])


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return lib().or_get_threads()


def antiperiodic_t_links(dims, U) -> np.ndarray:
    """Links for the operator with antiperiodic boundary conditions in time.

    The paper states no boundary conditions; fermion fields are usually taken
    antiperiodic in time, psi(x + L_t e_t) = -psi(x).  In the operator this
    puts a factor -1 on the two hops that cross the time boundary: the
    forward hop out of the last time slice, which carries U_t(x), and the
    backward hop into it, which carries the same link as U_t(x)^dag.  Both
    are obtained by negating U_t(x) on the last time slice, so every oracle
    routine (operator, smoothers, solvers, force) given these links computes
    the antiperiodic case.  The clover term is unchanged, since every
    plaquette holds either none or two of the negated links; it is built from
    the original links (or, equally, from these).  The negated links have
    determinant -1, so they are input to the oracle only, never to the GPU
    library, which takes the boundary condition as a lattice flag."""
    out = np.array(U, dtype=np.complex128, copy=True)
    lx, ly, lz, lt = (int(d) for d in dims)
    last = slice((lt - 1) * lx * ly * lz, lt * lx * ly * lz)
    out[last, 3] *= -1.0
    return out


def gamma(mu: int) -> np.ndarray:
    g = np.zeros((4, 4), np.complex128)
    lib().or_gamma(mu, _ptr(g))
    return g


def sigma(mu: int, nu: int) -> np.ndarray:
    s = np.zeros((4, 4), np.complex128)
    lib().or_sigma(mu, nu, _ptr(s))
    return s


def su3_generator(a: int) -> np.ndarray:
    t = np.zeros((3, 3), np.complex128)
    lib().or_su3_generator(a, _ptr(t))
    return t


def volume(dims) -> int:
    return int(np.prod([int(v) for v in dims]))


def leaf_sum(dims, U, site, mu, nu) -> np.ndarray:
    U = _c128(U)
    q = np.zeros((3, 3), np.complex128)
    lib().or_leaf_sum(_dims(dims), _ptr(U), int(site), mu, nu, _ptr(q))
    return q


def clover_site(dims, U, kappa, csw, site) -> np.ndarray:
    U = _c128(U)
    t = np.zeros((12, 12), np.complex128)
    lib().or_clover_site(_dims(dims), _ptr(U), float(kappa), float(csw), int(site), _ptr(t))
    return t


def clover_field(dims, U, kappa, csw) -> np.ndarray:
    U = _c128(U)
    t = np.zeros((volume(dims), 12, 12), np.complex128)
    lib().or_clover_field(_dims(dims), _ptr(U), float(kappa), float(csw), _ptr(t))
    return t


def apply_D(dims, U, T, kappa, psi) -> np.ndarray:
    U, psi = _c128(U), _c128(psi)
    T = None if T is None else _c128(T)
    out = np.empty_like(psi)
    lib().or_apply_D(_dims(dims), _ptr(U), _ptr(T), float(kappa), _ptr(psi), _ptr(out))
    return out


def apply_Ddag(dims, U, T, kappa, psi) -> np.ndarray:
    U, psi = _c128(U), _c128(psi)
    T = None if T is None else _c128(T)
    out = np.empty_like(psi)
    lib().or_apply_Ddag(_dims(dims), _ptr(U), _ptr(T), float(kappa), _ptr(psi), _ptr(out))
    return out


def apply_D_sites(dims, U, kappa, csw, psi, sites) -> np.ndarray:
    U, psi = _c128(U), _c128(psi)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(sites), 4, 3), np.complex128)
    lib().or_apply_D_sites(_dims(dims), _ptr(U), float(kappa), float(csw), _ptr(psi),
                           len(sites), _ptr(sites), _ptr(out))
    return out


def residual_norm(dims, U, kappa, csw, b, x) -> float:
    U, b, x = _c128(U), _c128(b), _c128(x)
    return lib().or_residual_norm(_dims(dims), _ptr(U), float(kappa), float(csw),
                                  _ptr(b), _ptr(x))


def num_blocks(dims, bdim) -> int:
    return lib().or_num_blocks(_dims(dims), _dims(bdim))


def block_colour(dims, bdim, blk) -> int:
    return lib().or_block_colour(_dims(dims), _dims(bdim), int(blk))


def block_of_site(dims, bdim, site) -> int:
    return lib().or_block_of_site(_dims(dims), _dims(bdim), int(site))


def apply_D_block(dims, bdim, blk, U, T, kappa, psi) -> np.ndarray:
    U, psi = _c128(U), _c128(psi)
    T = None if T is None else _c128(T)
    out = np.zeros_like(psi)
    lib().or_apply_D_block(_dims(dims), _dims(bdim), int(blk), _ptr(U), _ptr(T),
                           float(kappa), _ptr(psi), _ptr(out))
    return out


def mr_block(dims, bdim, blk, U, T, kappa, n_mr, r) -> np.ndarray:
    U, r = _c128(U), _c128(r)
    T = None if T is None else _c128(T)
    delta = np.zeros_like(r)
    lib().or_mr_block(_dims(dims), _dims(bdim), int(blk), _ptr(U), _ptr(T), float(kappa),
                      int(n_mr), _ptr(r), _ptr(delta))
    return delta


def sap(dims, bdim, U, T, kappa, n_cy, n_mr, b, x0=None) -> np.ndarray:
    U, b = _c128(U), _c128(b)
    T = None if T is None else _c128(T)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    lib().or_sap(_dims(dims), _dims(bdim), _ptr(U), _ptr(T), float(kappa), int(n_cy),
                 int(n_mr), _ptr(b), _ptr(x))
    return x


def clover_inverse_field(dims, T) -> np.ndarray:
    """(1 + T(x))^-1 for every site, [V][12][12]."""
    T = None if T is None else _c128(T)
    out = np.zeros((volume(dims), 12, 12), np.complex128)
    lib().or_clover_inverse_field(_dims(dims), _ptr(T), _ptr(out))
    return out


def jacobi_block(dims, bdim, blk, U, T, kappa, n_jac, r) -> np.ndarray:
    """Jacobi block solve of (C^-1 D)_BB delta = C^-1 r_B for one block."""
    U, r = _c128(U), _c128(r)
    T = None if T is None else _c128(T)
    delta = np.zeros_like(r)
    lib().or_jacobi_block(_dims(dims), _dims(bdim), int(blk), _ptr(U), _ptr(T), float(kappa), int(n_jac),
                          _ptr(r), _ptr(delta))
    return delta


def sap_jacobi(dims, bdim, U, T, kappa, n_cy, n_jac, b, x0=None) -> np.ndarray:
    U, b = _c128(U), _c128(b)
    T = None if T is None else _c128(T)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    lib().or_sap_jacobi(_dims(dims), _dims(bdim), _ptr(U), _ptr(T), float(kappa), int(n_cy), int(n_jac),
                        _ptr(b), _ptr(x))
    return x


def mr_eo_block(dims, bdim, blk, U, T, kappa, n_mr, r) -> np.ndarray:
    """Even-odd preconditioned MR solve of D_BB delta = r_B for one block."""
    U, r = _c128(U), _c128(r)
    T = None if T is None else _c128(T)
    delta = np.zeros_like(r)
    lib().or_mr_eo_block(_dims(dims), _dims(bdim), int(blk), _ptr(U), _ptr(T), float(kappa), int(n_mr),
                         _ptr(r), _ptr(delta))
    return delta


def sap_eo(dims, bdim, U, T, kappa, n_cy, n_mr, b, x0=None) -> np.ndarray:
    """SAP with even-odd preconditioned MR block solves."""
    U, b = _c128(U), _c128(b)
    T = None if T is None else _c128(T)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    lib().or_sap_eo(_dims(dims), _dims(bdim), _ptr(U), _ptr(T), float(kappa), int(n_cy), int(n_mr),
                    _ptr(b), _ptr(x))
    return x


def fgcr(dims, bdim, U, T, kappa, b, n_cy=2, n_mr=4, restart=16, tol=1e-10,
         max_iter=2000, x0=None):
    """Returns (x, status, iterations, true_relres, history)."""
    U, b = _c128(U), _c128(b)
    T = None if T is None else _c128(T)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    it = C.c_int(0)
    rel = C.c_double(0)
    hist = np.zeros(max_iter + 1, np.float64)
    st = lib().or_fgcr(_dims(dims), _dims(bdim), _ptr(U), _ptr(T), float(kappa), int(n_cy),
                       int(n_mr), int(restart), float(tol), int(max_iter), _ptr(b), _ptr(x),
                       C.byref(it), C.byref(rel), _ptr(hist))
    return x, st, it.value, rel.value, hist[: it.value + 1].copy()


def fbicgstab(dims, bdim, U, T, kappa, b, n_cy=2, n_mr=4, tol=1e-10, max_iter=2000,
              delta=0.0, x0=None):
    """Flexible BiCGStab with the SAP preconditioner.  Returns (x, status,
    iterations, restarts, true_relres, history)."""
    U, b = _c128(U), _c128(b)
    T = None if T is None else _c128(T)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    it, rs = C.c_int(0), C.c_int(0)
    rel = C.c_double(0)
    hist = np.zeros(max_iter + 1, np.float64)
    st = lib().or_fbicgstab(_dims(dims), _dims(bdim), _ptr(U), _ptr(T), float(kappa), int(n_cy),
                            int(n_mr), float(tol), int(max_iter), float(delta), _ptr(b), _ptr(x),
                            C.byref(it), C.byref(rs), C.byref(rel), _ptr(hist))
    return x, st, it.value, rs.value, rel.value, hist[: it.value + 1].copy()


def richardson_bicgstab(dims, bdim, U, T, kappa, b, n_cy=2, n_mr=4, tol=1e-10, max_iter=2000,
                        inner_tol=1e-5, x0=None):
    """Richardson iteration around inner BiCGStab solves.  Returns (x, status,
    inner iterations, outer steps, true_relres)."""
    U, b = _c128(U), _c128(b)
    T = None if T is None else _c128(T)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    it, outer = C.c_int(0), C.c_int(0)
    rel = C.c_double(0)
    st = lib().or_richardson_bicgstab(_dims(dims), _dims(bdim), _ptr(U), _ptr(T), float(kappa), int(n_cy),
                                      int(n_mr), float(tol), int(max_iter), float(inner_tol), _ptr(b),
                                      _ptr(x), C.byref(it), C.byref(outer), C.byref(rel))
    return x, st, it.value, outer.value, rel.value


def force(dims, U, kappa, csw, x, y, parts=("hop", "clov")):
    """Gradient g[V][4][8] of Re(eta^dag D^-1 b); returns (g_hop, g_clov)."""
    U, x, y = _c128(U), _c128(x), _c128(y)
    V = volume(dims)
    gh = np.zeros((V, 4, 8)) if "hop" in parts else None
    gc = np.zeros((V, 4, 8)) if "clov" in parts else None
    lib().or_force(_dims(dims), _ptr(U), float(kappa), float(csw), _ptr(x), _ptr(y),
                   _ptr(gh), _ptr(gc))
    return gh, gc
