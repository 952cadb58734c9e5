"""Two-level multigrid pieces of the paper's Section 3 in plain numpy on top of
the FP64 C oracle.

TEST INFRASTRUCTURE ONLY (like the rest of this package).

Definitions (aggregates are the 4^4 SAP blocks; every coarse site carries
2 Nv degrees of freedom, index c = chi * Nv + i):
* null vectors: v_i = M_SAP eta_i, the smoother applied to random vectors
  eta_i from x = 0, then n_adapt adaptive passes v_i <- M_MG v_i with P and
  the coarse operator rebuilt after every pass;
* local orthonormalisation: for every aggregate a and chirality chi
  (spins 0, 1 / spins 2, 3), modified Gram-Schmidt of the restrictions of
  v_0 .. v_{Nv-1} in that order gives the columns p_{a,chi,i};
* restriction r_c = P^dag r, prolongation e = P e_c;
* coarse operator D_c = P^dag D P (Galerkin);
* coarse solver: BiCGStab on D_c from zero, at most n_coarse iterations,
  stopping once the recursive residual is below tol_coarse times |r_c|;
* the multigrid preconditioner: z = P (coarse solve of P^dag r), then
  n_cy_post SAP cycles on D z = r started from z (post-smoothing);
* outer solvers with a callable preconditioner: flexible GCR and the
  paper's flexible BiCGStab.
P is kept as Nv full-lattice fields: field i holds p_{a,chi,i} on every
aggregate a and chirality chi (aggregates and chiralities occupy disjoint
components)."""
from __future__ import annotations

import numpy as np

from . import apply_D, block_of_site, sap

CHI = (slice(0, 2), slice(2, 4))  # spin ranges of the two chiralities


def aggregates(dims, bdim):
    """Site lists of the aggregates, indexed by block number."""
    V = int(np.prod(dims))
    owner = np.array([block_of_site(dims, bdim, s) for s in range(V)])
    nagg = int(owner.max()) + 1
    return [np.nonzero(owner == a)[0] for a in range(nagg)]


def build_prolongator(vecs, aggs):
    """Local orthonormalisation of vecs [Nv][V][4][3]: returns P with the same shape."""
    P = np.array(vecs, dtype=np.complex128, copy=True)
    Nv = P.shape[0]
    for sites in aggs:
        for chi in CHI:
            for i in range(Nv):
                pi = P[i][sites, chi, :]
                for j in range(i):
                    pj = P[j][sites, chi, :]
                    pi = pi - np.vdot(pj, pi) * pj
                nrm = np.linalg.norm(pi)
                P[i][sites, chi, :] = pi / nrm if nrm > 0 else 0.0
    return P


def restrict(P, aggs, r):
    """r_c[a][chi * Nv + i] = <p_{a,chi,i}, r> over the aggregate."""
    Nv = P.shape[0]
    rc = np.zeros((len(aggs), 2 * Nv), np.complex128)
    for a, sites in enumerate(aggs):
        for c, chi in enumerate(CHI):
            for i in range(Nv):
                rc[a, c * Nv + i] = np.vdot(P[i][sites, chi, :], r[sites, chi, :])
    return rc


def prolong(P, aggs, ec):
    Nv = P.shape[0]
    e = np.zeros(P.shape[1:], np.complex128)
    for a, sites in enumerate(aggs):
        for c, chi in enumerate(CHI):
            for i in range(Nv):
                e[sites, chi, :] += ec[a, c * Nv + i] * P[i][sites, chi, :]
    return e


def coarse_operator(dims, U, T, kappa, P, aggs):
    """Dense D_c = P^dag D P, [nagg * 2Nv][nagg * 2Nv] (coarse index a * 2Nv + c)."""
    Nv = P.shape[0]
    nc = len(aggs) * 2 * Nv
    Dc = np.zeros((nc, nc), np.complex128)
    for b, sites in enumerate(aggs):
        for c, chi in enumerate(CHI):
            for j in range(Nv):
                col = np.zeros(P.shape[1:], np.complex128)
                col[sites, chi, :] = P[j][sites, chi, :]
                Dc[:, b * 2 * Nv + c * Nv + j] = restrict(P, aggs, apply_D(dims, U, T, kappa, col)).reshape(-1)
    return Dc


def coarse_bicgstab(Dc, rc, n_iter, tol=0.0):
    """BiCGStab on Dc x = rc from x = 0: at most n_iter iterations, fewer when
    |r| <= tol |rc| or when <rh, r> = 0, <rh, v> = 0 or omega = 0."""
    stop = tol * np.linalg.norm(rc)
    x = np.zeros_like(rc)
    r = rc.copy()
    rh = r.copy()
    p = np.zeros_like(r)
    v = np.zeros_like(r)
    rho = alpha = omega = 1.0 + 0j
    for _ in range(n_iter):
        rho_new = np.vdot(rh, r)
        if rho_new == 0:
            break
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = Dc @ p
        rv = np.vdot(rh, v)
        if rv == 0:
            break
        alpha = rho_new / rv
        s = r - alpha * v
        t = Dc @ s
        tt = np.vdot(t, t).real
        omega = np.vdot(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
        if omega == 0 or np.linalg.norm(r) <= stop:
            break
    return x


def mg_apply(dims, bdim, U, T, kappa, P, aggs, Dc, r, n_coarse, n_cy_post, n_mr, tol_coarse=0.05):
    """z = SAP^{n_cy_post}(D z = r, from P (coarse solve of P^dag r))."""
    ec = coarse_bicgstab(Dc, restrict(P, aggs, r).reshape(-1), n_coarse, tol_coarse).reshape(len(aggs), -1)
    z0 = prolong(P, aggs, ec)
    return sap(dims, bdim, U, T, kappa, n_cy_post, n_mr, r, x0=z0) if n_cy_post > 0 else z0


def setup(dims, bdim, U, T, kappa, etas, n_cy_setup=2, n_mr=4, n_adapt=0, n_coarse=50, n_cy_post=2,
          tol_coarse=0.05):
    """Null vectors, P and D_c after the initial and n_adapt adaptive passes."""
    aggs = aggregates(dims, bdim)
    vecs = [sap(dims, bdim, U, T, kappa, n_cy_setup, n_mr, eta) for eta in etas]
    P = build_prolongator(vecs, aggs)
    Dc = coarse_operator(dims, U, T, kappa, P, aggs)
    for _ in range(n_adapt):
        vecs = [mg_apply(dims, bdim, U, T, kappa, P, aggs, Dc, v, n_coarse, n_cy_post, n_mr, tol_coarse)
                for v in vecs]
        P = build_prolongator(vecs, aggs)
        Dc = coarse_operator(dims, U, T, kappa, P, aggs)
    return P, Dc, aggs, vecs


def fgcr(matvec, precond, b, restart=16, tol=1e-10, max_iter=500):
    """Flexible GCR(restart) with a callable preconditioner (modified
    Gram-Schmidt, true residual at every restart), FP64.  Returns (x,
    iterations, true relative residual)."""
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    it = 0
    while True:
        r = b - matvec(x)
        rel = np.linalg.norm(r) / bn
        if rel <= tol or it >= max_iter:
            return x, it, rel
        Z, W, c = [], [], []
        R = np.zeros((restart, restart), np.complex128)
        for k in range(restart):
            z = precond(r)
            w = matvec(z)
            for j in range(k):
                R[j, k] = np.vdot(W[j], w)
                w = w - R[j, k] * W[j]
            R[k, k] = np.linalg.norm(w)
            w = w / R[k, k]
            ck = np.vdot(w, r)
            r = r - ck * w
            Z.append(z)
            W.append(w)
            c.append(ck)
            it += 1
            if np.linalg.norm(r) <= tol * bn or it >= max_iter:
                break
        kk = len(c)
        gam = np.linalg.solve(np.triu(R[:kk, :kk]), np.array(c))
        for k in range(kk):
            x = x + gam[k] * Z[k]


def fbicgstab(matvec, precond, b, tol=1e-10, max_iter=500, delta=0.0):
    """Flexible BiCGStab with a callable right preconditioner (the paper's
    outer solver around the multigrid preconditioner, Section 3), FP64.  The
    true residual b - D x is recomputed, and the iteration restarted from x
    with rh = r, whenever the recursive residual meets tol, falls below
    delta times the last true residual, or the iteration breaks down
    (<rh, v> = 0 or omega = 0); a restart without a smaller true residual is
    a breakdown (status 2).  Returns (x, status, iterations, restarts,
    true relative residual)."""
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bn == 0:
        return x, 0, 0, 0, 0.0
    it = restarts = 0
    last_true = 0.0
    while True:
        r = b - matvec(x)
        rt = np.linalg.norm(r)
        rel = rt / bn
        if rel <= tol:
            return x, 0, it, restarts, rel
        if it >= max_iter:
            return x, 1, it, restarts, rel
        if it > 0 and not rt < last_true:
            return x, 2, it, restarts, rel
        if it > 0:
            restarts += 1
        last_true = rt
        rh = r.copy()
        p = np.zeros_like(r)
        v = np.zeros_like(r)
        rho = alpha = omega = 1.0 + 0j
        while it < max_iter:
            rho_new = np.vdot(rh, r)
            beta = (rho_new / rho) * (alpha / omega)
            p = r + beta * (p - omega * v)
            ph = precond(p)
            v = matvec(ph)
            rv = np.vdot(rh, v)
            if rv == 0:
                break
            alpha = rho_new / rv
            s = r - alpha * v
            sh = precond(s)
            t = matvec(sh)
            tt = np.vdot(t, t).real
            omega = np.vdot(t, s) / tt if tt > 0 else 0.0
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            rho = rho_new
            it += 1
            rr = np.linalg.norm(r)
            if rr <= tol * bn or omega == 0 or (delta > 0 and rr < delta * last_true):
                break
