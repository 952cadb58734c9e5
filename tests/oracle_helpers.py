"""Helpers for the oracle pins: dense assembly of the oracle's D on tiny lattices
and gamma-matrix utilities written independently of the oracle's code."""
import numpy as np

import oracle


def dense_D(dims, U, T, kappa):
    """Dense matrix of the oracle's D, column j = D e_j (canonical ordering)."""
    V = int(np.prod(dims))
    n = 12 * V
    M = np.empty((n, n), np.complex128)
    e = np.zeros((V, 4, 3), np.complex128)
    flat = e.reshape(-1)
    for j in range(n):
        flat[j] = 1.0
        M[:, j] = oracle.apply_D(dims, U, T, kappa, e).reshape(-1)
        flat[j] = 0.0
    return M


def g5_apply(psi):
    sign = np.array([1, 1, -1, -1], dtype=np.float64)
    return psi * sign[None, :, None]


def site_index(dims, c):
    x, y, z, t = c
    return x + dims[0] * (y + dims[1] * (z + dims[2] * t))


def coords(dims, V):
    s = np.arange(V)
    x = s % dims[0]
    y = (s // dims[0]) % dims[1]
    z = (s // (dims[0] * dims[1])) % dims[2]
    t = s // (dims[0] * dims[1] * dims[2])
    return np.stack([x, y, z, t], axis=1)


def block_sites(dims, bdim, blk):
    """Canonical site indices of block blk (block coordinates x fastest)."""
    nb = [dims[m] // bdim[m] for m in range(4)]
    bc = [blk % nb[0], (blk // nb[0]) % nb[1], (blk // (nb[0] * nb[1])) % nb[2],
          blk // (nb[0] * nb[1] * nb[2])]
    out = []
    for lt in range(bdim[3]):
        for lz in range(bdim[2]):
            for ly in range(bdim[1]):
                for lx in range(bdim[0]):
                    out.append(site_index(dims, (bc[0] * bdim[0] + lx, bc[1] * bdim[1] + ly,
                                                 bc[2] * bdim[2] + lz, bc[3] * bdim[3] + lt)))
    return np.array(out)


def dof_indices(sites):
    return (np.asarray(sites)[:, None] * 12 + np.arange(12)[None, :]).reshape(-1)


def gauge_transform_links(dims, U, Om):
    """U'_mu(x) = Om(x) U_mu(x) Om(x+mu)^dag."""
    V = int(np.prod(dims))
    c = coords(dims, V)
    out = np.empty_like(U)
    for mu in range(4):
        cp = c.copy()
        cp[:, mu] = (cp[:, mu] + 1) % dims[mu]
        sp = cp[:, 0] + dims[0] * (cp[:, 1] + dims[1] * (cp[:, 2] + dims[2] * cp[:, 3]))
        out[:, mu] = Om @ U[:, mu] @ np.conj(np.transpose(Om[sp], (0, 2, 1)))
    return out


def gauge_transform_spinor(Om, psi):
    return np.einsum("vab,vsb->vsa", Om, psi)
