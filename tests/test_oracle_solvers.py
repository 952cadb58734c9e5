"""Oracle pins for the MR block solve, the multiplicative red/black SAP
smoother (paper Section 2 and Section 3: fixed-count block solves applied
alternately to the two colours of domains) and flexible GCR.

Pins: exact-block SAP equals red/black block Gauss-Seidel built from a dense
matrix; MR is monotone and has a one-step closed form; FGCR matches a dense
LU solve; SAP and GCR are gauge covariant.
"""
import numpy as np
import pytest

import oracle
from paper_2112_00501_amd import synth
from tests.oracle_helpers import (block_sites, coords, dense_D, dof_indices, gauge_transform_links,
                                  gauge_transform_spinor)

DIMS, BDIM = (4, 4, 4, 4), (2, 2, 2, 2)
KAPPA, CSW = 0.13, 1.0


@pytest.fixture(scope="module")
def system():
    U = synth.gauge_field(DIMS, 0.3, 21)
    T = oracle.clover_field(DIMS, U, KAPPA, CSW)
    M = dense_D(DIMS, U, T, KAPPA)
    return U, T, M


@pytest.fixture(scope="module")
def cond2(system):
    sv = np.linalg.svd(system[2], compute_uv=False)
    return sv[0] / sv[-1]


def _colour_blocks(colour):
    nblk = oracle.num_blocks(DIMS, BDIM)
    return [b for b in range(nblk) if oracle.block_colour(DIMS, BDIM, b) == colour]


def _K(M, colour, v):
    """Apply the sum over blocks of one colour of the exact Dirichlet-block inverse."""
    out = np.zeros_like(v)
    for blk in _colour_blocks(colour):
        idx = dof_indices(block_sites(DIMS, BDIM, blk))
        out[idx] = np.linalg.solve(M[np.ix_(idx, idx)], v[idx])
    return out


def test_block_colouring_is_a_checkerboard():
    dims, bdim = (4, 4, 4, 8), (2, 2, 2, 4)
    nblk = oracle.num_blocks(dims, bdim)
    assert nblk == 16
    cols = [oracle.block_colour(dims, bdim, b) for b in range(nblk)]
    assert sum(cols) == 8
    # every hop that leaves a block lands in a block of the other colour
    V = int(np.prod(dims))
    for s in range(0, V, 7):
        b0 = oracle.block_of_site(dims, bdim, s)
        c = np.array(np.unravel_index(s, dims[::-1])[::-1])
        for mu in range(4):
            for step in (1, -1):
                cc = c.copy()
                cc[mu] = (cc[mu] + step) % dims[mu]
                s2 = cc[0] + dims[0] * (cc[1] + dims[1] * (cc[2] + dims[2] * cc[3]))
                b1 = oracle.block_of_site(dims, bdim, s2)
                if b1 != b0:
                    assert cols[b1] != cols[b0]


def test_mr_one_step_closed_form_and_monotone(system):
    U, T, M = system
    r = synth.source(DIMS, 31)
    blk = 3
    idx = dof_indices(block_sites(DIMS, BDIM, blk))
    Mb = M[np.ix_(idx, idx)]
    rb = r.reshape(-1)[idx]
    q = Mb @ rb
    alpha = np.vdot(q, rb) / np.vdot(q, q)
    d1 = oracle.mr_block(DIMS, BDIM, blk, U, T, KAPPA, 1, r).reshape(-1)[idx]
    assert np.abs(d1 - alpha * rb).max() < 1e-14
    res = [np.linalg.norm(rb)]
    for n in range(1, 9):
        d = oracle.mr_block(DIMS, BDIM, blk, U, T, KAPPA, n, r).reshape(-1)[idx]
        res.append(np.linalg.norm(rb - Mb @ d))
    assert all(res[i + 1] <= res[i] * (1 + 1e-14) for i in range(len(res) - 1))
    assert res[-1] < 0.2 * res[0]
    # many steps converge to the exact block solve
    d = oracle.mr_block(DIMS, BDIM, blk, U, T, KAPPA, 300, r).reshape(-1)[idx]
    assert np.linalg.norm(d - np.linalg.solve(Mb, rb)) < 1e-11 * np.linalg.norm(rb)


def test_mr_exact_in_one_step_at_kappa_zero():
    U = synth.gauge_field(DIMS, 0.3, 22)
    T = oracle.clover_field(DIMS, U, 0.0, CSW)
    r = synth.source(DIMS, 32)
    d = oracle.mr_block(DIMS, BDIM, 0, U, T, 0.0, 1, r)
    idx = dof_indices(block_sites(DIMS, BDIM, 0))
    assert np.abs(d.reshape(-1)[idx] - r.reshape(-1)[idx]).max() < 1e-15


def test_exact_block_sap_is_block_gauss_seidel(system):
    U, T, M = system
    b = synth.source(DIMS, 33)
    bf = b.reshape(-1)
    # one cycle from x = 0: M1 = K0 + K1 - K1 D K0
    x1 = oracle.sap(DIMS, BDIM, U, T, KAPPA, 1, 300, b).reshape(-1)
    k0b = _K(M, 0, bf)
    ref1 = k0b + _K(M, 1, bf) - _K(M, 1, M @ k0b)
    assert np.linalg.norm(x1 - ref1) < 1e-10 * np.linalg.norm(ref1)
    # two cycles from a nonzero x0: error propagator [(1 - K1 D)(1 - K0 D)]^2
    x0 = synth.source(DIMS, 34)
    x2 = oracle.sap(DIMS, BDIM, U, T, KAPPA, 2, 300, b, x0=x0).reshape(-1)
    xs = np.linalg.solve(M, bf)
    e = x0.reshape(-1) - xs
    for _ in range(2):
        e = e - _K(M, 0, M @ e)
        e = e - _K(M, 1, M @ e)
    ref2 = xs + e
    assert np.linalg.norm(x2 - ref2) < 1e-10 * np.linalg.norm(ref2)


def test_sap_with_mr_reduces_residual_and_is_homogeneous(system):
    U, T, M = system
    b = synth.source(DIMS, 35)
    x = oracle.sap(DIMS, BDIM, U, T, KAPPA, 2, 4, b)
    r = b.reshape(-1) - M @ x.reshape(-1)
    assert np.linalg.norm(r) < 0.3 * np.linalg.norm(b)
    # MR is homogeneous of degree one in the right-hand side
    x3 = oracle.sap(DIMS, BDIM, U, T, KAPPA, 2, 4, (2.5 - 1j) * b)
    assert np.abs(x3 - (2.5 - 1j) * x).max() < 1e-13 * np.abs(x).max()


@pytest.mark.parametrize("n_cy", [0, 2])
def test_fgcr_matches_dense_lu(system, cond2, n_cy):
    U, T, M = system
    b = synth.source(DIMS, 36)
    x_lu = np.linalg.solve(M, b.reshape(-1))
    x, st, it, rel, hist = oracle.fgcr(DIMS, BDIM, U, T, KAPPA, b, n_cy=n_cy, n_mr=4,
                                       restart=16, tol=1e-10)
    assert st == 0 and rel <= 1e-10
    assert np.linalg.norm(x.reshape(-1) - x_lu) <= cond2 * 1e-10 * np.linalg.norm(x_lu)
    assert np.linalg.norm(b.reshape(-1) - M @ x.reshape(-1)) <= 1e-10 * np.linalg.norm(b)
    # the recursive residual is non-increasing within a restart cycle
    h = hist
    for i in range(1, min(len(h) - 1, 16)):
        assert h[i + 1] <= h[i] * (1 + 1e-12)
    if n_cy:
        assert it < 30


def test_fgcr_restart_and_warm_start(system):
    U, T, M = system
    b = synth.source(DIMS, 37)
    x, st, it, rel, _ = oracle.fgcr(DIMS, BDIM, U, T, KAPPA, b, n_cy=2, restart=3, tol=1e-10)
    assert st == 0 and rel <= 1e-10
    xa, st, it_a, rel_a, _ = oracle.fgcr(DIMS, BDIM, U, T, KAPPA, b, tol=1e-5)
    assert st == 0 and rel_a <= 1e-5
    xb, st, it_b, rel_b, _ = oracle.fgcr(DIMS, BDIM, U, T, KAPPA, b, tol=1e-10, x0=xa)
    assert st == 0 and rel_b <= 1e-10
    assert np.linalg.norm(b.reshape(-1) - M @ xb.reshape(-1)) <= 1e-10 * np.linalg.norm(b)


def test_fgcr_zero_rhs_and_iteration_cap(system):
    U, T, M = system
    z = np.zeros((int(np.prod(DIMS)), 4, 3), complex)
    x, st, it, rel, _ = oracle.fgcr(DIMS, BDIM, U, T, KAPPA, z, x0=synth.source(DIMS, 1))
    assert st == 0 and it == 0 and np.abs(x).max() == 0
    b = synth.source(DIMS, 38)
    x, st, it, rel, _ = oracle.fgcr(DIMS, BDIM, U, T, KAPPA, b, max_iter=2, n_cy=0)
    assert st == 1 and it == 2 and rel > 1e-10


def test_sap_and_gcr_gauge_covariant(system):
    U, T, M = system
    Om = synth.gauge_transform(DIMS, 4003)
    Ug = gauge_transform_links(DIMS, U, Om)
    Tg = oracle.clover_field(DIMS, Ug, KAPPA, CSW)
    b = synth.source(DIMS, 39)
    bg = gauge_transform_spinor(Om, b)
    x = oracle.sap(DIMS, BDIM, U, T, KAPPA, 2, 4, b)
    xg = oracle.sap(DIMS, BDIM, Ug, Tg, KAPPA, 2, 4, bg)
    assert np.abs(xg - gauge_transform_spinor(Om, x)).max() < 1e-12
    s, st, it, _, _ = oracle.fgcr(DIMS, BDIM, U, T, KAPPA, b)
    sg, stg, itg, _, _ = oracle.fgcr(DIMS, BDIM, Ug, Tg, KAPPA, bg)
    assert it == itg
    assert np.abs(sg - gauge_transform_spinor(Om, s)).max() < 1e-9


# ---- flexible BiCGStab (the paper's outer solver, Section 3)

@pytest.mark.parametrize("n_cy", [0, 2])
def test_fbicgstab_matches_dense_lu(system, cond2, n_cy):
    U, T, M = system
    b = synth.source(DIMS, 41)
    x_lu = np.linalg.solve(M, b.reshape(-1))
    x, st, it, rs, rel, hist = oracle.fbicgstab(DIMS, BDIM, U, T, KAPPA, b, n_cy=n_cy, tol=1e-10)
    assert st == 0 and rel <= 1e-10
    assert np.linalg.norm(x.reshape(-1) - x_lu) <= cond2 * 1e-10 * np.linalg.norm(x_lu)
    assert np.linalg.norm(b.reshape(-1) - M @ x.reshape(-1)) <= 1e-10 * np.linalg.norm(b)
    if n_cy:  # the preconditioner pays: fewer iterations than without
        _, _, it0, _, _, _ = oracle.fbicgstab(DIMS, BDIM, U, T, KAPPA, b, n_cy=0, tol=1e-10)
        assert it < it0


def test_fbicgstab_recursive_residual_is_the_true_one(system):
    """Stopped by the iteration cap, the recursive residual of the last
    iteration must equal b - D x of the returned x: the x and r recurrences
    use the same alpha, omega, p-hat, s-hat."""
    U, T, M = system
    b = synth.source(DIMS, 42)
    for n_cy in (0, 2):
        x, st, it, rs, rel, hist = oracle.fbicgstab(DIMS, BDIM, U, T, KAPPA, b, n_cy=n_cy,
                                                    max_iter=3, tol=1e-14)
        assert st == 1 and it == 3 and rs == 0
        true = np.linalg.norm(b.reshape(-1) - M @ x.reshape(-1)) / np.linalg.norm(b)
        assert abs(rel - true) <= 1e-12 * true
        assert abs(hist[-1] - true) <= 1e-9 * true


def test_fbicgstab_exact_in_one_step_at_kappa_zero():
    U = synth.gauge_field(DIMS, 0.3, 23)
    T = oracle.clover_field(DIMS, U, 0.0, CSW)
    b = synth.source(DIMS, 43)
    x, st, it, rs, rel, _ = oracle.fbicgstab(DIMS, BDIM, U, T, 0.0, b, n_cy=0, tol=1e-12)
    assert st == 0 and it == 1 and rel == 0.0
    assert np.abs(x - b).max() < 1e-15


def test_fbicgstab_reliable_restarts_zero_rhs_and_covariance(system):
    U, T, M = system
    b = synth.source(DIMS, 44)
    x, st, it, rs, rel, _ = oracle.fbicgstab(DIMS, BDIM, U, T, KAPPA, b, n_cy=2, tol=1e-10, delta=1e-3)
    assert st == 0 and rel <= 1e-10 and rs >= 2
    z = np.zeros_like(b)
    x0, st0, it0, _, _, _ = oracle.fbicgstab(DIMS, BDIM, U, T, KAPPA, z, x0=b)
    assert st0 == 0 and it0 == 0 and np.abs(x0).max() == 0
    Om = synth.gauge_transform(DIMS, 4004)
    Ug = gauge_transform_links(DIMS, U, Om)
    Tg = oracle.clover_field(DIMS, Ug, KAPPA, CSW)
    s, _, its, _, _, _ = oracle.fbicgstab(DIMS, BDIM, U, T, KAPPA, b, n_cy=2)
    sg, _, itg, _, _, _ = oracle.fbicgstab(DIMS, BDIM, Ug, Tg, KAPPA, gauge_transform_spinor(Om, b), n_cy=2)
    assert its == itg
    assert np.abs(sg - gauge_transform_spinor(Om, s)).max() < 1e-9


def test_richardson_bicgstab_matches_dense_lu(system, cond2):
    """The QWS scheme (Section 2): FP64 Richardson around inner BiCGStab
    solves reaches the dense solution; with an inner tolerance at the outer
    one a single Richardson step suffices."""
    U, T, M = system
    b = synth.source(DIMS, 45)
    x_lu = np.linalg.solve(M, b.reshape(-1))
    x, st, it, outer, rel = oracle.richardson_bicgstab(DIMS, BDIM, U, T, KAPPA, b, inner_tol=1e-4)
    assert st == 0 and rel <= 1e-10 and outer >= 2
    assert np.linalg.norm(x.reshape(-1) - x_lu) <= cond2 * 1e-10 * np.linalg.norm(x_lu)
    x1, st1, it1, outer1, rel1 = oracle.richardson_bicgstab(DIMS, BDIM, U, T, KAPPA, b, inner_tol=1e-12)
    assert st1 == 0 and outer1 == 1 and rel1 <= 1e-10


# ---- QWS smoother form: SAP on A = C^-1 D with Jacobi block solves (Section 2)

def test_clover_inverse_is_the_inverse(system):
    U, T, M = system
    Ci = oracle.clover_inverse_field(DIMS, T)
    eye = np.eye(12)
    err = max(np.abs(Ci[s] @ (eye + T[s]) - eye).max() for s in range(0, T.shape[0], 5))
    assert err < 1e-13
    # the inverse of a Hermitian matrix is Hermitian
    assert max(np.abs(Ci[s] - Ci[s].conj().T).max() for s in range(0, T.shape[0], 5)) < 1e-13


def test_jacobi_sap_exact_block_limit_equals_mr_sap_limit():
    """With converged block solves, SAP on A = C^-1 D equals SAP on D: C is
    site diagonal, so (A_BB)^-1 C^-1 = (D_BB)^-1 and both are red/black block
    Gauss-Seidel of D.  kappa is small enough for the block Jacobi iteration
    to converge."""
    kappa = 0.06
    U = synth.gauge_field(DIMS, 0.3, 24)
    T = oracle.clover_field(DIMS, U, kappa, CSW)
    b = synth.source(DIMS, 46)
    x0 = synth.source(DIMS, 47)
    xj = oracle.sap_jacobi(DIMS, BDIM, U, T, kappa, 2, 200, b, x0=x0)
    xm = oracle.sap(DIMS, BDIM, U, T, kappa, 2, 200, b, x0=x0)
    assert np.linalg.norm(xj - xm) < 1e-11 * np.linalg.norm(xm)


def test_jacobi_sap_one_step_closed_form_and_kappa_zero(system):
    U, T, M = system
    Ci = oracle.clover_inverse_field(DIMS, T)
    b = synth.source(DIMS, 48)
    # one Jacobi step per block, one cycle from x = 0: colour-0 blocks get
    # C^-1 b, colour-1 blocks C^-1 (b - D x0) with x0 the colour-0 result
    x = oracle.sap_jacobi(DIMS, BDIM, U, T, KAPPA, 1, 1, b)
    col = np.array([oracle.block_colour(DIMS, BDIM, oracle.block_of_site(DIMS, BDIM, s))
                    for s in range(b.shape[0])])
    x0 = np.einsum("sij,sj->si", Ci, b.reshape(-1, 12)) * (col == 0)[:, None]
    r = b.reshape(-1) - M @ x0.reshape(-1)
    x1 = np.einsum("sij,sj->si", Ci, r.reshape(-1, 12))
    ref = np.where((col == 0)[:, None], x0, x1)
    assert np.abs(x.reshape(-1, 12) - ref).max() < 1e-13 * np.abs(ref).max()
    # kappa = 0: D = C, so any number of cycles gives x = C^-1 b
    T0 = oracle.clover_field(DIMS, U, 0.0, CSW)
    x = oracle.sap_jacobi(DIMS, BDIM, U, T0, 0.0, 2, 3, b)
    C0 = oracle.clover_inverse_field(DIMS, T0)
    assert np.abs(x.reshape(-1, 12) - np.einsum("sij,sj->si", C0, b.reshape(-1, 12))).max() < 1e-14


def test_jacobi_sap_gauge_covariant(system):
    U, T, M = system
    Om = synth.gauge_transform(DIMS, 4005)
    Ug = gauge_transform_links(DIMS, U, Om)
    Tg = oracle.clover_field(DIMS, Ug, KAPPA, CSW)
    b = synth.source(DIMS, 49)
    x = oracle.sap_jacobi(DIMS, BDIM, U, T, KAPPA, 2, 3, b)
    xg = oracle.sap_jacobi(DIMS, BDIM, Ug, Tg, KAPPA, 2, 3, gauge_transform_spinor(Om, b))
    assert np.abs(xg - gauge_transform_spinor(Om, x)).max() < 1e-12


def _eo_split(blk):
    sites = block_sites(DIMS, BDIM, blk)
    par = coords(DIMS, int(np.prod(DIMS)))[sites].sum(axis=1) % 2
    return dof_indices(sites[par == 0]), dof_indices(sites[par == 1])


def test_eo_block_mr_one_step_against_the_dense_schur_complement(system):
    """One even-odd MR step, built from dense blocks of D: S = D_ee - D_eo
    D_oo^-1 D_oe, rhat = r_e - D_eo D_oo^-1 r_o, delta_e = alpha rhat with
    alpha = <S rhat, rhat> / |S rhat|^2, delta_o = D_oo^-1 (r_o - D_oe delta_e)."""
    U, T, M = system
    r = synth.source(DIMS, 41)
    blk = 5
    ie, io = _eo_split(blk)
    Dee, Deo = M[np.ix_(ie, ie)], M[np.ix_(ie, io)]
    Doe, Doo = M[np.ix_(io, ie)], M[np.ix_(io, io)]
    assert np.abs(Dee - np.diag(np.diag(Dee))).max() > 0  # clover couples spins and colours on a site
    rf = r.reshape(-1)
    S = Dee - Deo @ np.linalg.solve(Doo, Doe)
    rhat = rf[ie] - Deo @ np.linalg.solve(Doo, rf[io])
    q = S @ rhat
    de = np.vdot(q, rhat) / np.vdot(q, q) * rhat
    do = np.linalg.solve(Doo, rf[io] - Doe @ de)
    got = oracle.mr_eo_block(DIMS, BDIM, blk, U, T, KAPPA, 1, r).reshape(-1)
    assert np.abs(got[ie] - de).max() < 1e-13 and np.abs(got[io] - do).max() < 1e-13
    # outside the block nothing is written
    rest = np.setdiff1d(np.arange(rf.size), np.concatenate([ie, io]))
    assert np.abs(got[rest]).max() == 0.0


def test_eo_block_mr_converges_to_the_block_solve_and_beats_plain_mr(system):
    U, T, M = system
    r = synth.source(DIMS, 42)
    blk = 2
    ie, io = _eo_split(blk)
    idx = np.sort(np.concatenate([ie, io]))
    exact = np.linalg.solve(M[np.ix_(idx, idx)], r.reshape(-1)[idx])
    got = oracle.mr_eo_block(DIMS, BDIM, blk, U, T, KAPPA, 60, r).reshape(-1)[idx]
    assert np.linalg.norm(got - exact) < 1e-10 * np.linalg.norm(exact)
    # at equal step counts the Schur-complement iteration is closer to the block solve
    for n in (2, 4):
        e_eo = np.linalg.norm(oracle.mr_eo_block(DIMS, BDIM, blk, U, T, KAPPA, n, r).reshape(-1)[idx] - exact)
        e_mr = np.linalg.norm(oracle.mr_block(DIMS, BDIM, blk, U, T, KAPPA, n, r).reshape(-1)[idx] - exact)
        assert e_eo < e_mr


def test_eo_sap_exact_block_limit_equals_mr_sap_limit(system):
    """With enough steps both block solvers are exact, so even-odd SAP and
    MR-SAP reach the same red/black block Gauss-Seidel result; the even-odd
    smoother is gauge covariant."""
    U, T, M = system
    b = synth.source(DIMS, 43)
    x_eo = oracle.sap_eo(DIMS, BDIM, U, T, KAPPA, 2, 60, b)
    x_mr = oracle.sap(DIMS, BDIM, U, T, KAPPA, 2, 200, b)
    assert np.linalg.norm(x_eo - x_mr) < 1e-9 * np.linalg.norm(x_mr)
    g = synth.gauge_transform(DIMS, 44)
    Ug = gauge_transform_links(DIMS, U, g)
    Tg = oracle.clover_field(DIMS, Ug, KAPPA, CSW)
    x1 = oracle.sap_eo(DIMS, BDIM, U, T, KAPPA, 2, 4, b)
    x2 = oracle.sap_eo(DIMS, BDIM, Ug, Tg, KAPPA, 2, 4, gauge_transform_spinor(g, b))
    assert np.linalg.norm(x2 - gauge_transform_spinor(g, x1)) < 1e-12 * np.linalg.norm(x1)


def test_jacobi_block_equals_dense_jacobi_iteration(system):
    """The QWS block solve (paper Section 2: a fixed number of Jacobi steps on
    a domain of A = C^-1 D) against the same iteration written with dense
    numpy matrices: rho = C_B^-1 r_B with C_B^-1 from numpy.linalg.inv of the
    12 x 12 site matrices 1 + T, A_BB = C_B^-1 (D restricted to the block's
    rows and columns), delta_0 = 0 and delta += rho - A_BB delta.  A dropped
    C^-1 in rho, a wrong sign or a hop leaking over the block's faces each
    fail it."""
    U, T, M = system
    r = synth.source(DIMS, 51)
    eye = np.eye(12)
    for blk in (0, 5):
        sites = block_sites(DIMS, BDIM, blk)
        idx = dof_indices(sites)
        Cinv = np.zeros((idx.size, idx.size), np.complex128)
        for i, s in enumerate(sites):
            Cinv[12 * i:12 * i + 12, 12 * i:12 * i + 12] = np.linalg.inv(eye + T[s])
        A = Cinv @ M[np.ix_(idx, idx)]
        rho = Cinv @ r.reshape(-1)[idx]
        for n_jac in (1, 2, 5):
            ref = np.zeros_like(rho)
            for _ in range(n_jac):
                ref = ref + rho - A @ ref
            got = oracle.jacobi_block(DIMS, BDIM, blk, U, T, KAPPA, n_jac, r)
            assert np.abs(got.reshape(-1)[idx] - ref).max() < 1e-13 * np.abs(ref).max()
            # nothing outside the block is written
            rest = np.setdiff1d(np.arange(got.size), idx)
            assert np.abs(got.reshape(-1)[rest]).max() == 0.0


def test_jacobi_block_is_the_first_colour_of_a_jacobi_sap_cycle(system):
    """From x = 0 the colour-0 half-sweep of the Jacobi smoother solves every
    colour-0 block with r_B = b_B, and the colour-1 half-sweep leaves those
    blocks alone: after one cycle they hold the single-block solve."""
    U, T, M = system
    b = synth.source(DIMS, 52)
    x = oracle.sap_jacobi(DIMS, BDIM, U, T, KAPPA, 1, 3, b)
    for blk in _colour_blocks(0)[:3]:
        idx = dof_indices(block_sites(DIMS, BDIM, blk))
        d = oracle.jacobi_block(DIMS, BDIM, blk, U, T, KAPPA, 3, b)
        assert np.abs(x.reshape(-1)[idx] - d.reshape(-1)[idx]).max() < 1e-14 * np.abs(d).max()
