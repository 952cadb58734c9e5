"""Seeded synthetic inputs: gauge fields, sources and gauge transformations.

The paper benchmarks on real gauge configurations (its sets A, B and C in
Section 4) that are not available here.  These generators stand in for them
with fields of the same shapes built from a fixed recipe, so that the CPU
oracle and the GPU library can be fed identical inputs.

This module holds input generation only: none of the operator, smoother or
solver arithmetic lives here, and it imports neither the oracle nor the HIP
library.

Canonical layouts (complex128, C order, site index x fastest):
  gauge   U[V][mu][a][b]       mu = 0..3 for x, y, z, t; (a, b) = (row, col)
  spinor  psi[V][spin][colour] 4 spins x 3 colours
  batch   psi[nrhs][V][4][3]

Recipe for the links (one reading of an unspecified generator):
  per site (x fastest), then per direction, nine N(0,1) draws from
  numpy PCG64(seed): d0, d1, d2, then (Re, Im) of the (0,1), (0,2) and (1,2)
  entries.  H is Hermitian with diagonal d - mean(d) (traceless) and the drawn
  upper off-diagonal entries.  U = GS(exp(i eps H)), where GS orthonormalises
  rows 0 and 1 and sets row 2 = conj(row0 x row1), so det U = 1 exactly and
  the third row is a function of the first two.
"""
from __future__ import annotations

import numpy as np

try:  # torch's batched CPU matmul is much faster than numpy's for 3x3 stacks
    import torch as _torch
except Exception:  # pragma: no cover - torch is always present in this image
    _torch = None

DRAWS_PER_LINK = 9


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def _matmul(a, b):
    if _torch is not None:
        return _torch.matmul(_torch.from_numpy(a), _torch.from_numpy(b)).numpy()
    return a @ b


def expm_i_herm(h: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*h) for a stack of Hermitian 3x3 matrices.

    Scaling and squaring with a degree-20 Taylor polynomial: the scaled
    argument has norm below 0.5, so the truncation error is far below double
    rounding.
    """
    a = np.ascontiguousarray(1j * eps * h)
    if a.size == 0:
        return a.copy()
    nrm = float(np.abs(a).sum(axis=2).max())
    k = 0
    while nrm / (2.0 ** k) > 0.5:
        k += 1
    a = a / (2.0 ** k)
    res = np.broadcast_to(np.eye(3, dtype=np.complex128), a.shape).copy()
    term = res.copy()
    for n in range(1, 21):
        term = _matmul(term, a) / n
        res = res + term
    for _ in range(k):
        res = _matmul(res, res)
    return res


def gram_schmidt_su3(m: np.ndarray) -> np.ndarray:
    """Row Gram-Schmidt onto SU(3): rows 0, 1 orthonormalised, row 2 = conj(r0 x r1)."""
    out = np.empty_like(m)
    r0 = m[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = m[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    out[..., 0, :] = r0
    out[..., 1, :] = r1
    out[..., 2, :] = np.conj(np.cross(r0, r1))
    return out


def hermitian_from_draws(r: np.ndarray) -> np.ndarray:
    """Traceless Hermitian 3x3 from rows of nine draws (recipe above)."""
    n = r.shape[0]
    d = r[:, 0:3] - r[:, 0:3].mean(axis=1, keepdims=True)
    h = np.zeros((n, 3, 3), dtype=np.complex128)
    for i in range(3):
        h[:, i, i] = d[:, i]
    for j, (a, b) in enumerate(((0, 1), (0, 2), (1, 2))):
        z = r[:, 3 + 2 * j] + 1j * r[:, 4 + 2 * j]
        h[:, a, b] = z
        h[:, b, a] = np.conj(z)
    return h


def gauge_field(dims, eps: float, seed: int, chunk: int = 1 << 17) -> np.ndarray:
    """Random SU(3) links U = GS(exp(i eps H)); complex128 [V][4][3][3]."""
    v = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((v, 4, 3, 3), dtype=np.complex128)
    for s0 in range(0, v, chunk):
        s1 = min(v, s0 + chunk)
        n = (s1 - s0) * 4
        r = rng.standard_normal((n, DRAWS_PER_LINK))
        u = gram_schmidt_su3(expm_i_herm(hermitian_from_draws(r), eps))
        out[s0:s1] = u.reshape(s1 - s0, 4, 3, 3)
    return out


def unit_gauge(dims) -> np.ndarray:
    v = volume(dims)
    out = np.zeros((v, 4, 3, 3), dtype=np.complex128)
    out[:, :, 0, 0] = out[:, :, 1, 1] = out[:, :, 2, 2] = 1.0
    return out


def source(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Gaussian source, Re and Im ~ N(0,1) per component in canonical order.

    Returns [V][4][3] complex128, or [nrhs][V][4][3] when nrhs is given
    (the right-hand-side index outermost in the draw order).
    """
    v = volume(dims)
    n = 1 if nrhs is None else int(nrhs)
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.standard_normal((n, v, 4, 3, 2))
    out = r[..., 0] + 1j * r[..., 1]
    return out[0] if nrhs is None else out


def random_su3(n: int, seed: int) -> np.ndarray:
    """n SU(3) matrices: GS of complex Gaussian 3x3 matrices."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.standard_normal((n, 3, 3, 2))
    return gram_schmidt_su3(r[..., 0] + 1j * r[..., 1])


def gauge_transform(dims, seed: int) -> np.ndarray:
    """One random SU(3) matrix per site: Omega[V][3][3]."""
    return random_su3(volume(dims), seed)


# Configurations the benchmarks and tests use (lattice, eps, kappa, c_sw, seeds).
CONFIGS = {
    "plain_fp64_8x8x8x8": dict(dims=(8, 8, 8, 8), eps=0.3, kappa=0.13, csw=1.0,
                               gauge_seed=1001, src_seed=2001),
    "mixed_16x16x16x32": dict(dims=(16, 16, 16, 32), eps=0.3, kappa=0.1355, csw=1.0,
                              gauge_seed=1002, src_seed=2002, mg_eta_seed=4002),
    "lowprec_32x32x32x64": dict(dims=(32, 32, 32, 64), eps=0.25, kappa=0.1370, csw=1.1,
                                gauge_seed=1003, src_seed=2003, mg_eta_seed=4003),
    "lowprec_sub_16x16x16x16": dict(dims=(16, 16, 16, 16), eps=0.25, kappa=0.1370, csw=1.1,
                                    gauge_seed=1013, src_seed=2013),
    "multirhs_24x24x24x48": dict(dims=(24, 24, 24, 48), eps=0.3, kappa=0.1355, csw=1.0,
                                 gauge_seed=1004, src_seed=2004),
    "grad_32x32x32x64": dict(dims=(32, 32, 32, 64), eps=0.3, kappa=0.1355, csw=1.0,
                             gauge_seed=1005, src_seed=2005, eta_seed=3005),
    "grad_fd_4x4x4x4": dict(dims=(4, 4, 4, 4), eps=0.3, kappa=0.1355, csw=1.0,
                            gauge_seed=1015, src_seed=2015, eta_seed=3015),
    "grad_8x8x8x8": dict(dims=(8, 8, 8, 8), eps=0.3, kappa=0.1355, csw=1.0,
                         gauge_seed=1025, src_seed=2025, eta_seed=3025),
    "mg_8x8x8x8": dict(dims=(8, 8, 8, 8), eps=0.3, kappa=0.1355, csw=1.0,
                       gauge_seed=1006, src_seed=2006, mg_eta_seed=4006),
}
