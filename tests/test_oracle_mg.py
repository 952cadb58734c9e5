"""Pins of the oracle's two-level multigrid pieces (paper Section 3: null
vectors from the smoother, aggregation with local orthonormalisation,
restriction / prolongation, Galerkin coarse operator, BiCGStab coarse solver,
SAP post-smoothing)."""
import numpy as np
import pytest

import oracle
from oracle import mg
from paper_2112_00501_amd import synth
from tests.oracle_helpers import dense_D

DIMS, BDIM = (4, 4, 4, 4), (2, 2, 2, 2)
# a lighter quark than the solver tests: the coarse space pays where SAP
# alone slows down (paper Section 4: the multigrid solver wins for light
# quarks)
KAPPA, CSW, NV = 0.145, 1.0, 8


@pytest.fixture(scope="module")
def system():
    U = synth.gauge_field(DIMS, 0.3, 51)
    T = oracle.clover_field(DIMS, U, KAPPA, CSW)
    M = dense_D(DIMS, U, T, KAPPA)
    etas = [synth.source(DIMS, 5100 + i) for i in range(NV)]
    P, Dc, aggs, vecs = mg.setup(DIMS, BDIM, U, T, KAPPA, etas, n_cy_setup=4, n_mr=4, n_adapt=1)
    return U, T, M, P, Dc, aggs, vecs


def _dense_P(P, aggs):
    cols = []
    for sites in aggs:
        for chi in mg.CHI:
            for i in range(P.shape[0]):
                col = np.zeros(P.shape[1:], np.complex128)
                col[sites, chi, :] = P[i][sites, chi, :]
                cols.append(col.reshape(-1))
    return np.stack(cols, axis=1)


def test_prolongator_orthonormal_and_spans_the_null_vectors(system):
    U, T, M, P, Dc, aggs, vecs = system
    Pd = _dense_P(P, aggs)
    assert np.abs(Pd.conj().T @ Pd - np.eye(Pd.shape[1])).max() < 1e-13
    for v in vecs:  # each null vector lies in the span of the columns
        back = mg.prolong(P, aggs, mg.restrict(P, aggs, v))
        assert np.linalg.norm(back - v) < 1e-12 * np.linalg.norm(v)


def test_coarse_operator_is_galerkin_and_gamma5_hermitian(system):
    U, T, M, P, Dc, aggs, vecs = system
    Pd = _dense_P(P, aggs)
    assert np.abs(Dc - Pd.conj().T @ M @ Pd).max() < 1e-12 * np.abs(Dc).max()
    # P preserves chirality, so gamma5-hermiticity of D carries over with
    # Gamma5 = +1 on chirality-0 and -1 on chirality-1 coarse components
    g5 = np.tile(np.repeat([1.0, -1.0], NV), len(aggs))
    assert np.abs(g5[:, None] * Dc * g5[None, :] - Dc.conj().T).max() < 1e-12 * np.abs(Dc).max()


def test_coarse_grid_correction_is_exact_on_the_coarse_space(system):
    U, T, M, P, Dc, aggs, vecs = system
    rng = np.random.default_rng(3)
    ec = rng.standard_normal(Dc.shape[0]) + 1j * rng.standard_normal(Dc.shape[0])
    e = mg.prolong(P, aggs, ec.reshape(len(aggs), -1))
    rc = mg.restrict(P, aggs, oracle.apply_D(DIMS, U, T, KAPPA, e)).reshape(-1)
    back = mg.prolong(P, aggs, np.linalg.solve(Dc, rc).reshape(len(aggs), -1))
    assert np.linalg.norm(back - e) < 1e-11 * np.linalg.norm(e)


def test_coarse_bicgstab_converges_to_the_dense_solution(system):
    U, T, M, P, Dc, aggs, vecs = system
    rng = np.random.default_rng(4)
    rc = rng.standard_normal(Dc.shape[0]) + 1j * rng.standard_normal(Dc.shape[0])
    x = mg.coarse_bicgstab(Dc, rc, 200, tol=1e-12)
    assert np.linalg.norm(Dc @ x - rc) < 1e-10 * np.linalg.norm(rc)
    x2 = mg.coarse_bicgstab(Dc, rc, 2)  # a few iterations already reduce the residual
    assert np.linalg.norm(Dc @ x2 - rc) < np.linalg.norm(rc)
    x3 = mg.coarse_bicgstab(Dc, rc, 200, tol=0.05)  # the tolerance stops early
    assert np.linalg.norm(Dc @ x3 - rc) < 0.1 * np.linalg.norm(rc)


def test_mg_preconditioned_fgcr_solves_and_beats_sap(system):
    U, T, M, P, Dc, aggs, vecs = system
    b = synth.source(DIMS, 52)
    mv = lambda v: oracle.apply_D(DIMS, U, T, KAPPA, v)
    x_lu = np.linalg.solve(M, b.reshape(-1))
    pre_mg = lambda r: mg.mg_apply(DIMS, BDIM, U, T, KAPPA, P, aggs, Dc, r, 50, 2, 4)
    pre_sap = lambda r: oracle.sap(DIMS, BDIM, U, T, KAPPA, 2, 4, r)
    x, it_mg, rel = mg.fgcr(mv, pre_mg, b)
    _, it_sap, _ = mg.fgcr(mv, pre_sap, b)
    print(f"FGCR iterations: multigrid {it_mg}, SAP {it_sap}")
    assert rel <= 1e-10
    assert np.linalg.norm(x.reshape(-1) - x_lu) < 1e-8 * np.linalg.norm(x_lu)
    assert it_mg < it_sap


def test_adaptive_pass_improves_the_coarse_space(system):
    """Without the adaptive pass the same multigrid is weaker: the adaptive
    setup is what makes the coarse space pay."""
    U, T, M, P, Dc, aggs, vecs = system
    etas = [synth.source(DIMS, 5100 + i) for i in range(NV)]
    P0, Dc0, aggs0, _ = mg.setup(DIMS, BDIM, U, T, KAPPA, etas, n_cy_setup=4, n_mr=4, n_adapt=0)
    b = synth.source(DIMS, 53)
    mv = lambda v: oracle.apply_D(DIMS, U, T, KAPPA, v)
    _, it0, _ = mg.fgcr(mv, lambda r: mg.mg_apply(DIMS, BDIM, U, T, KAPPA, P0, aggs0, Dc0, r, 50, 2, 4), b)
    _, it1, _ = mg.fgcr(mv, lambda r: mg.mg_apply(DIMS, BDIM, U, T, KAPPA, P, aggs, Dc, r, 50, 2, 4), b)
    print(f"FGCR iterations: initial setup {it0}, one adaptive pass {it1}")
    assert it1 < it0


def test_flexible_bicgstab_with_a_callable_preconditioner(system):
    """The numpy flexible BiCGStab taking any preconditioner equals the plain-C
    oracle's SAP-preconditioned one when handed the same SAP (an independent
    implementation of the same recurrences), reaches the dense solution, and
    with M_MG needs fewer iterations than with SAP."""
    U, T, M, P, Dc, aggs, vecs = system
    b = synth.source(DIMS, 57)
    mv = lambda v: oracle.apply_D(DIMS, U, T, KAPPA, v)  # noqa: E731
    sap = lambda r: oracle.sap(DIMS, BDIM, U, T, KAPPA, 2, 4, r)  # noqa: E731
    x, st, it, rs, rel = mg.fbicgstab(mv, sap, b, tol=1e-10, delta=1e-5)
    xc, stc, itc, rsc, relc, _ = oracle.fbicgstab(DIMS, BDIM, U, T, KAPPA, b, n_cy=2, n_mr=4, tol=1e-10,
                                                 delta=1e-5)
    assert st == 0 and stc == 0 and it == itc and rs == rsc
    assert np.linalg.norm(x - xc) <= 1e-12 * np.linalg.norm(xc)
    xd = np.linalg.solve(M, b.reshape(-1)).reshape(b.shape)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    mgp = lambda r: mg.mg_apply(DIMS, BDIM, U, T, KAPPA, P, aggs, Dc, r, 50, 2, 4)  # noqa: E731
    x2, st2, it2, _, rel2 = mg.fbicgstab(mv, mgp, b, tol=1e-10, delta=1e-5)
    assert st2 == 0 and rel2 <= 1e-10 and it2 < it
    assert np.linalg.norm(x2 - xd) <= 1e-8 * np.linalg.norm(xd)
