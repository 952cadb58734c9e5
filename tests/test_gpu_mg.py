"""GPU two-level multigrid (paper Section 3) against the oracle's numpy
multigrid, through the C ABI, on an 8^4 lattice: 16 aggregates of 4^4 sites,
two aggregates per direction, so that the +mu and -mu neighbours of an
aggregate coincide and the 9-point stencil has to keep their faces apart.

The GPU hierarchy is FP32 (coarse reductions FP64) and the oracle FP64, so
the comparisons are relative norms with bounds set by FP32 rounding (unit
roundoff 6e-8) grown through the SAP cycles, the Gram-Schmidt steps and, for
the coarse solve, the BiCGStab recursion.  Coarse solves in parity cases run
a fixed number of iterations (tol_coarse = 0), so that both sides stop at the
same step."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from oracle import mg
from paper_2112_00501_amd import cloversap as cs
from paper_2112_00501_amd import synth
from tests.gpu_helpers import Case, rel

pytestmark = pytest.mark.gpu

DIMS, BDIM = (8, 8, 8, 8), (4, 4, 4, 4)
KAPPA, CSW, NV = 0.14, 1.0, 8
N_COARSE = 20
TOL_P = 1e-5       # P, D_c and the transfer operators (observed ~4e-7)
TOL_SOLVE = 1e-4   # after the BiCGStab recursion and the post-smoothing (observed ~4e-7)


def _nb(d):
    return [x // 4 for x in d]


def dense_from_stencil(Dc, dims):
    """The 9-point stencil float2[nblk][9][col][row] as a dense matrix with
    coarse index a * nc + c (the documented layout, summed over faces)."""
    Dc = Dc.cpu().numpy().astype(np.complex128)
    nblk, _, nc, _ = Dc.shape
    NB = _nb(dims)
    M = np.zeros((nblk * nc, nblk * nc), np.complex128)
    for a in range(nblk):
        bc = [a % NB[0], (a // NB[0]) % NB[1], (a // (NB[0] * NB[1])) % NB[2], a // (NB[0] * NB[1] * NB[2])]
        for d in range(9):
            nbc = list(bc)
            if d > 0:
                mu, step = (d - 1) // 2, (+1 if d % 2 == 1 else -1)
                nbc[mu] = (nbc[mu] + step) % NB[mu]
            n = nbc[0] + NB[0] * (nbc[1] + NB[1] * (nbc[2] + NB[2] * nbc[3]))
            M[a * nc:(a + 1) * nc, n * nc:(n + 1) * nc] += Dc[a, d].T
    return M


def _coarse(x):
    return torch.from_numpy(np.ascontiguousarray(x).astype(np.complex64)).cuda()


@pytest.fixture(scope="module")
def sys8():
    c = Case(DIMS, 0.3, KAPPA, CSW, 61)
    etas = [synth.source(DIMS, 6100 + i) for i in range(NV)]
    etas_d = c.lat.import_field(torch.from_numpy(np.stack(etas)).cuda(), cs.F32)
    torch.cuda.synchronize()
    return c, etas, etas_d


def _params(n_adapt):
    return cs.MgParams(nv=NV, n_cy_setup=4, n_mr=4, n_adapt=n_adapt, n_coarse=N_COARSE, n_cy_post=2,
                       tol_coarse=0.0)


@pytest.fixture(scope="module")
def plain(sys8):
    c, etas, etas_d = sys8
    m = cs.Multigrid(c.op, etas_d, _params(0))
    P, Dc, aggs, _ = mg.setup(DIMS, BDIM, c.U, c.T, KAPPA, etas, n_cy_setup=4, n_mr=4, n_adapt=0)
    torch.cuda.synchronize()
    return c, m, P, Dc, aggs


def _export(c, m):
    P, Dc = m.export()
    Pc = c.lat.export_field(P, cs.F32, m.nv)
    torch.cuda.synchronize()
    return Pc.cpu().numpy().reshape(m.nv, -1, 4, 3), dense_from_stencil(Dc, DIMS)


def test_prolongator_matches_oracle(plain):
    c, m, P_or, Dc_or, aggs = plain
    P, _ = _export(c, m)
    err = rel(P, P_or)
    # orthonormal per aggregate and chirality in FP32
    cols = []
    for sites in aggs:
        for chi in mg.CHI:
            for i in range(NV):
                col = np.zeros(P.shape[1:], np.complex128)
                col[sites, chi, :] = P[i][sites, chi, :]
                cols.append(col.reshape(-1))
    Pd = np.stack(cols, axis=1)
    G = Pd.conj().T @ Pd
    print(f"|P - P_oracle| / |P_oracle| = {err:.2e}; max |P^dag P - 1| = {np.abs(G - np.eye(len(G))).max():.2e}")
    assert err <= TOL_P
    assert np.abs(G - np.eye(len(G))).max() <= 1e-5


def test_coarse_operator_matches_oracle(plain):
    c, m, P_or, Dc_or, aggs = plain
    _, Dc = _export(c, m)
    err = rel(Dc, Dc_or)
    g5 = np.tile(np.repeat([1.0, -1.0], NV), len(aggs))
    herm = np.abs(g5[:, None] * Dc * g5[None, :] - Dc.conj().T).max() / np.abs(Dc).max()
    print(f"|D_c - D_c oracle| / |D_c oracle| = {err:.2e}; gamma5-hermiticity defect {herm:.2e}")
    assert err <= TOL_P
    assert herm <= 1e-5


def test_transfer_and_coarse_apply_match_oracle(plain):
    c, m, P_or, Dc_or, aggs = plain
    r = synth.source(DIMS, 6200)
    rc = m.restrict(c.to_dev(r, cs.F32)).cpu().numpy()
    rc_or = mg.restrict(P_or, aggs, r)
    rng = np.random.default_rng(6201)
    ec = rng.standard_normal(rc_or.shape) + 1j * rng.standard_normal(rc_or.shape)
    z = c.to_host(m.prolong(_coarse(ec)), cs.F32)
    z_or = mg.prolong(P_or, aggs, ec)
    y = m.coarse_apply(_coarse(ec)).cpu().numpy().reshape(-1)
    y_or = Dc_or @ ec.reshape(-1)
    e = (rel(rc, rc_or), rel(z, z_or), rel(y, y_or))
    print("restrict / prolong / coarse apply: %.2e %.2e %.2e" % e)
    assert max(e) <= TOL_P


def test_coarse_solve_matches_oracle(plain):
    c, m, P_or, Dc_or, aggs = plain
    rng = np.random.default_rng(6300)
    n = Dc_or.shape[0]
    rc = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    rcd = _coarse(rc.reshape(len(aggs), -1))
    for it in (1, 5, N_COARSE):
        ec = m.coarse_solve(rcd, it, 0.0).cpu().numpy().reshape(-1)
        ec_or = mg.coarse_bicgstab(Dc_or, rc, it)
        print(f"{it} iterations: rel diff {rel(ec, ec_or):.2e}")
        assert rel(ec, ec_or) <= TOL_SOLVE
    # the tolerance stops the iteration (judged with the oracle's D_c)
    ec = m.coarse_solve(rcd, 500, 0.05).cpu().numpy().reshape(-1)
    res = np.linalg.norm(Dc_or @ ec - rc) / np.linalg.norm(rc)
    ec_or = mg.coarse_bicgstab(Dc_or, rc, 500, 0.05)
    print(f"tol 0.05: residual {res:.3e}, oracle {np.linalg.norm(Dc_or @ ec_or - rc) / np.linalg.norm(rc):.3e}")
    assert res <= 0.05 * (1 + TOL_SOLVE)
    assert rel(ec, ec_or) <= TOL_SOLVE
    # degenerate cases: zero right-hand side and no iterations give zero
    assert float(m.coarse_solve(torch.zeros_like(rcd), 10, 0.0).abs().max()) == 0.0
    assert float(m.coarse_solve(rcd, 0, 0.0).abs().max()) == 0.0


def test_mg_apply_matches_oracle(plain):
    c, m, P_or, Dc_or, aggs = plain
    r = synth.source(DIMS, 6400)
    z = c.to_host(m.apply(c.to_dev(r, cs.F32)), cs.F32)
    z_or = mg.mg_apply(DIMS, BDIM, c.U, c.T, KAPPA, P_or, aggs, Dc_or, r, N_COARSE, 2, 4, tol_coarse=0.0)
    print(f"M_MG r: rel diff {rel(z, z_or):.2e}")
    assert rel(z, z_or) <= TOL_SOLVE


def test_adaptive_setup_matches_oracle(sys8):
    c, etas, etas_d = sys8
    m = cs.Multigrid(c.op, etas_d, _params(1))
    P_or, Dc_or, aggs, _ = mg.setup(DIMS, BDIM, c.U, c.T, KAPPA, etas, n_cy_setup=4, n_mr=4, n_adapt=1,
                                    n_coarse=N_COARSE, n_cy_post=2, tol_coarse=0.0)
    P, Dc = _export(c, m)
    print(f"adaptive pass: P rel diff {rel(P, P_or):.2e}, D_c rel diff {rel(Dc, Dc_or):.2e}")
    assert rel(P, P_or) <= TOL_SOLVE
    assert rel(Dc, Dc_or) <= TOL_SOLVE


def test_mg_gcr_solve_reaches_fp64_residual(sys8):
    """FGCR preconditioned by M_MG: the true FP64 residual reaches 1e-10, in
    about as many iterations as the oracle's FP64 FGCR with its own M_MG."""
    c, etas, etas_d = sys8
    prm = cs.MgParams(nv=NV, n_cy_setup=4, n_mr=4, n_adapt=1, n_coarse=50, n_cy_post=2, tol_coarse=0.05)
    m = cs.Multigrid(c.op, etas_d, prm)
    b = synth.source(DIMS, 6500)
    xd = c.lat.new_field(cs.F64).zero_()
    st, stats = m.gcr_solve(xd, c.to_dev(b, cs.F64), cs.SolverParams(inner_prec=cs.F32, tol=1e-10))
    x = c.to_host(xd, cs.F64)
    relres = oracle.residual_norm(c.dims, c.U, c.kappa, c.csw, b, x) / np.linalg.norm(b)
    P, Dc, aggs, _ = mg.setup(DIMS, BDIM, c.U, c.T, KAPPA, etas, n_cy_setup=4, n_mr=4, n_adapt=1)
    mv = lambda v: oracle.apply_D(DIMS, c.U, c.T, KAPPA, v)  # noqa: E731
    _, it_or, _ = mg.fgcr(mv, lambda r: mg.mg_apply(DIMS, BDIM, c.U, c.T, KAPPA, P, aggs, Dc, r, 50, 2, 4),
                          b, 16, 1e-10, 300)
    print(f"MG-FGCR: gpu iters {stats['iters']} relres {relres:.2e}; oracle iters {it_or}")
    assert st == 0 and relres <= 1e-10 * (1 + 1e-6)
    assert abs(stats["iters"] - it_or) <= max(2, it_or // 10)


def test_mg_gcr_graph_replay_equals_eager(plain):
    c, m, _, _, _ = plain
    b = c.to_dev(synth.source(DIMS, 6600), cs.F64)
    outs = []
    for use_graph in (False, True, True):
        x = c.lat.new_field(cs.F64).zero_()
        m.gcr_solve(x, b, cs.SolverParams(inner_prec=cs.F32, tol=1e-10, use_graph=use_graph))
        torch.cuda.synchronize()
        outs.append(x)
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_mg_argument_errors(sys8, plain):
    c, etas, etas_d = sys8
    m = plain[1]
    big = c.lat.new_field(cs.F32, 33).zero_()  # large enough that the library itself must refuse nv = 33
    for bad in (dict(nv=0), dict(nv=33), dict(n_cy_setup=0), dict(n_coarse=0), dict(tol_coarse=-1.0)):
        p = _params(0)
        for k, v in bad.items():
            setattr(p, k, v)
        with pytest.raises(cs.CloverSapError):
            cs.Multigrid(c.op, big, p)
    with pytest.raises(ValueError):  # the binding refuses too small a buffer of random vectors
        cs.Multigrid(c.op, c.lat.new_field(cs.F32, 1), _params(0))
    b = c.to_dev(synth.source(DIMS, 1), cs.F64)
    x = c.lat.new_field(cs.F64).zero_()
    with pytest.raises(cs.CloverSapError):  # the hierarchy is FP32
        m.gcr_solve(x, b, cs.SolverParams(inner_prec=cs.F16))
    other = Case(DIMS, 0.3, KAPPA, CSW, 62, oracle_T=False)
    prm = cs.SolverParams().to_c()
    st = cs._lib.cs_gcr_solve_mg(other.op.gauge.handle, other.op.clover.handle, m.handle, ctypes.byref(prm),
                                 cs._ptr(x), cs._ptr(b), None, cs._stream(None))
    assert st != 0  # the hierarchy was built for another operator


def test_fp16_coarse_matrices(sys8, plain):
    """FP16 storage of D_c for the coarse solve: the coarse product agrees
    with the oracle's FP64 D_c to the FP16 rounding of the entries (unit
    roundoff 4.9e-4), and MG-FGCR still reaches 1e-10 in about as many
    iterations as with FP32 storage."""
    c, etas, etas_d = sys8
    _, m32, P_or, Dc_or, aggs = plain
    m = cs.Multigrid(c.op, etas_d, cs.MgParams(**{**_params(0).__dict__, "coarse_prec": cs.F16}))
    rng = np.random.default_rng(6700)
    ec = rng.standard_normal((len(aggs), 2 * NV)) + 1j * rng.standard_normal((len(aggs), 2 * NV))
    y = m.coarse_apply(_coarse(ec)).cpu().numpy().reshape(-1)
    err = rel(y, Dc_or @ ec.reshape(-1))
    print(f"FP16 coarse product: rel diff {err:.2e}")
    assert err <= 1e-3
    b = c.to_dev(synth.source(DIMS, 6800), cs.F64)
    its = []
    for mm in (m32, m):
        x = c.lat.new_field(cs.F64).zero_()
        st, stats = mm.gcr_solve(x, b, cs.SolverParams(inner_prec=cs.F32, tol=1e-10))
        relres = oracle.residual_norm(c.dims, c.U, c.kappa, c.csw, synth.source(DIMS, 6800),
                                      c.to_host(x, cs.F64)) / np.linalg.norm(synth.source(DIMS, 6800))
        assert st == 0 and relres <= 1e-10 * (1 + 1e-6)
        its.append(stats["iters"])
    print(f"MG-FGCR iterations FP32 / FP16 coarse matrices: {its}")
    assert its[1] <= its[0] + 2


def test_graphs_follow_a_recreated_hierarchy(sys8):
    """A hierarchy destroyed and another created (possibly at the same
    addresses) must not replay graphs captured for the first: graph-replayed
    and eager solves with the second agree bit for bit."""
    import gc
    c, etas, etas_d = sys8
    b = c.to_dev(synth.source(DIMS, 6900), cs.F64)
    m1 = cs.Multigrid(c.op, etas_d, _params(0))
    x = c.lat.new_field(cs.F64).zero_()
    m1.gcr_solve(x, b, cs.SolverParams(inner_prec=cs.F32, tol=1e-10))
    torch.cuda.synchronize()
    del m1
    gc.collect()
    etas2 = c.lat.import_field(torch.from_numpy(np.stack([synth.source(DIMS, 7100 + i) for i in range(NV)])).cuda(),
                               cs.F32)
    m2 = cs.Multigrid(c.op, etas2, cs.MgParams(**{**_params(1).__dict__, "coarse_prec": cs.F16}))
    outs = []
    for use_graph in (True, False):
        x = c.lat.new_field(cs.F64).zero_()
        st, stats = m2.gcr_solve(x, b, cs.SolverParams(inner_prec=cs.F32, tol=1e-10, use_graph=use_graph))
        torch.cuda.synchronize()
        outs.append((x, stats["iters"]))
    print(f"iterations graph / eager: {outs[0][1]} / {outs[1][1]}")
    assert outs[0][1] == outs[1][1] and torch.equal(outs[0][0], outs[1][0])


@pytest.mark.parametrize("vec", [cs.F64, cs.F32])
def test_mg_bicgstab_reaches_fp64_residual(sys8, vec):
    """The paper's method: flexible BiCGStab around M_MG (FP64 vectors), and
    FP32 BiCGStab with M_MG inside the FP64 Richardson iteration; both reach
    1e-10 by the oracle's residual, the first in about as many iterations as
    the oracle's flexible BiCGStab around its own M_MG; graph replay equals
    the eager path bit for bit."""
    c, etas, etas_d = sys8
    prm = cs.MgParams(nv=NV, n_cy_setup=4, n_mr=4, n_adapt=1, n_coarse=50, n_cy_post=2, tol_coarse=0.05)
    m = cs.Multigrid(c.op, etas_d, prm)
    b = synth.source(DIMS, 7200)
    bd = c.to_dev(b, cs.F64)
    outs = []
    for use_graph in (True, False):
        xd = c.lat.new_field(cs.F64).zero_()
        st, stats = m.bicgstab_solve(xd, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=vec, tol=1e-10,
                                                             reliable_delta=1e-5, use_graph=use_graph))
        torch.cuda.synchronize()
        outs.append((xd, stats))
    assert torch.equal(outs[0][0], outs[1][0]) and outs[0][1]["iters"] == outs[1][1]["iters"]
    xd, stats = outs[0]
    relres = oracle.residual_norm(c.dims, c.U, c.kappa, c.csw, b, c.to_host(xd, cs.F64)) / np.linalg.norm(b)
    msg = f"MG-BiCGStab vec={vec}: gpu iters {stats['iters']} restarts {stats['restarts']} relres {relres:.2e}"
    if vec == cs.F64:
        P, Dc, aggs, _ = mg.setup(DIMS, BDIM, c.U, c.T, KAPPA, etas, n_cy_setup=4, n_mr=4, n_adapt=1)
        mv = lambda v: oracle.apply_D(DIMS, c.U, c.T, KAPPA, v)  # noqa: E731
        pre = lambda r: mg.mg_apply(DIMS, BDIM, c.U, c.T, KAPPA, P, aggs, Dc, r, 50, 2, 4)  # noqa: E731
        _, st_or, it_or, _, _ = mg.fbicgstab(mv, pre, b, tol=1e-10, delta=1e-5)
        msg += f"; oracle iters {it_or}"
        assert st_or == 0 and abs(stats["iters"] - it_or) <= max(2, it_or // 10)
    print(msg)
    assert relres <= 1e-10 * (1 + 1e-6)


def test_fp16_prolongator_transfers(sys8, plain):
    """FP16 storage of P for restriction and prolongation (one FP32 scale per
    site): both agree with the oracle's FP64 transfers to the FP16 rounding of
    P (unit roundoff 4.9e-4), and MG-FGCR with FP16 transfers and FP16 coarse
    matrices reaches 1e-10 in about as many iterations as the FP32 hierarchy."""
    c, etas, etas_d = sys8
    _, m32, P_or, Dc_or, aggs = plain
    m = cs.Multigrid(c.op, etas_d, cs.MgParams(**{**_params(0).__dict__, "transfer_prec": cs.F16,
                                                 "coarse_prec": cs.F16}))
    r = synth.source(DIMS, 7300)
    rc = m.restrict(c.to_dev(r, cs.F32)).cpu().numpy()
    rng = np.random.default_rng(7301)
    ec = rng.standard_normal(rc.shape) + 1j * rng.standard_normal(rc.shape)
    z = c.to_host(m.prolong(_coarse(ec)), cs.F32)
    e = (rel(rc, mg.restrict(P_or, aggs, r)), rel(z, mg.prolong(P_or, aggs, ec)))
    print("FP16 transfers: restrict / prolong rel diff %.2e %.2e" % e)
    assert max(e) <= 1e-3
    b = synth.source(DIMS, 7302)
    its = []
    for mm in (m32, m):
        x = c.lat.new_field(cs.F64).zero_()
        st, stats = mm.gcr_solve(x, c.to_dev(b, cs.F64), cs.SolverParams(inner_prec=cs.F32, tol=1e-10))
        relres = oracle.residual_norm(c.dims, c.U, c.kappa, c.csw, b, c.to_host(x, cs.F64)) / np.linalg.norm(b)
        assert st == 0 and relres <= 1e-10 * (1 + 1e-6)
        its.append(stats["iters"])
    print(f"MG-FGCR iterations FP32 / FP16 storage: {its}")
    assert its[1] <= its[0] + 2


@pytest.mark.parametrize("nv", [1, 3, 32])
def test_unusual_null_vector_counts(sys8, nv):
    """The index arithmetic that depends on nc = 2 nv (lane split of the
    coarse product, the assembly's row rounds, the transfers): one null
    vector, an odd count, and the largest count (nc = 64, one full wave of
    rows) against the oracle."""
    c, _, _ = sys8
    etas = [synth.source(DIMS, 7500 + i) for i in range(nv)]
    etas_d = c.lat.import_field(torch.from_numpy(np.stack(etas)).cuda(), cs.F32)
    m = cs.Multigrid(c.op, etas_d, cs.MgParams(nv=nv, n_cy_setup=2, n_mr=4, n_adapt=0, n_coarse=10,
                                               n_cy_post=1, tol_coarse=0.0))
    P_or, Dc_or, aggs, _ = mg.setup(DIMS, BDIM, c.U, c.T, KAPPA, etas, n_cy_setup=2, n_mr=4, n_adapt=0)
    P, Dc = _export(c, m)
    rng = np.random.default_rng(7600 + nv)
    rc = rng.standard_normal(Dc_or.shape[0]) + 1j * rng.standard_normal(Dc_or.shape[0])
    ec = m.coarse_solve(_coarse(rc.reshape(len(aggs), -1)), 10, 0.0).cpu().numpy().reshape(-1)
    r = synth.source(DIMS, 7601)
    z = c.to_host(m.apply(c.to_dev(r, cs.F32)), cs.F32)
    z_or = mg.mg_apply(DIMS, BDIM, c.U, c.T, KAPPA, P_or, aggs, Dc_or, r, 10, 1, 4, tol_coarse=0.0)
    e = (rel(P, P_or), rel(Dc, Dc_or), rel(ec, mg.coarse_bicgstab(Dc_or, rc, 10)), rel(z, z_or))
    print(f"nv={nv}: P %.2e D_c %.2e coarse solve %.2e M_MG %.2e" % e)
    assert e[0] <= TOL_P and e[1] <= TOL_P and e[2] <= TOL_SOLVE and e[3] <= TOL_SOLVE


def test_noncubic_lattice_stencil():
    """8 x 8 x 16 x 8: four aggregates along z, so the +z and -z neighbours
    are different aggregates while the other directions wrap onto the same
    one; D_c, the coarse product and M_MG against the oracle."""
    dims, nv = (8, 8, 16, 8), 4
    c = Case(dims, 0.3, KAPPA, CSW, 63)
    etas = [synth.source(dims, 7700 + i) for i in range(nv)]
    etas_d = c.lat.import_field(torch.from_numpy(np.stack(etas)).cuda(), cs.F32)
    m = cs.Multigrid(c.op, etas_d, cs.MgParams(nv=nv, n_cy_setup=2, n_mr=4, n_adapt=0, n_coarse=10, n_cy_post=1,
                                               tol_coarse=0.0))
    P_or, Dc_or, aggs, _ = mg.setup(dims, BDIM, c.U, c.T, KAPPA, etas, n_cy_setup=2, n_mr=4, n_adapt=0)
    _, Dc = m.export()
    Dc = dense_from_stencil(Dc, dims)
    rng = np.random.default_rng(7800)
    ec = rng.standard_normal((len(aggs), 2 * nv)) + 1j * rng.standard_normal((len(aggs), 2 * nv))
    y = m.coarse_apply(_coarse(ec)).cpu().numpy().reshape(-1)
    r = synth.source(dims, 7801)
    z = c.to_host(m.apply(c.to_dev(r, cs.F32)), cs.F32)
    z_or = mg.mg_apply(dims, BDIM, c.U, c.T, KAPPA, P_or, aggs, Dc_or, r, 10, 1, 4, tol_coarse=0.0)
    e = (rel(Dc, Dc_or), rel(y, Dc_or @ ec.reshape(-1)), rel(z, z_or))
    print("8x8x16x8: D_c %.2e coarse product %.2e M_MG %.2e" % e)
    assert e[0] <= TOL_P and e[1] <= TOL_P and e[2] <= TOL_SOLVE
