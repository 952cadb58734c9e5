"""Multi-right-hand-side path: tiled SAP and operator launches (links and
clover read once per tile), persistent launches, the autotuner, the batched
lock-step FGCR and its HIP-graph replay.  Every column must reproduce the
single-right-hand-side result bit for bit (same arithmetic, same reduction
order)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2112_00501_amd import cloversap as cs
from paper_2112_00501_amd import synth
from tests.gpu_helpers import Case

pytestmark = pytest.mark.gpu

NRHS = 6


@pytest.fixture(scope="module")
def case():
    return Case((8, 8, 8, 16), 0.3, 0.1355, 1.0, 1004, oracle_T=False)


CFGS = [(1, 0), (4, 0), (6, 0), (4, 16), (1, 7), (12, 0)]


@pytest.mark.parametrize("prec,lanes", [(cs.F32, 1), (cs.F32, 2), (cs.F64, 1), (cs.F16, 1), (cs.F16, 2)])
@pytest.mark.parametrize("tile,pers", CFGS)
def test_tiled_sap_and_dslash_equal_untiled(case, prec, lanes, tile, pers):
    c = case
    bs = synth.source(c.dims, 7, nrhs=NRHS)
    bd = c.to_dev(bs, prec)
    cfg = cs.LaunchConfig(tile, pers, lanes)
    # operator
    ref = c.lat.new_field(prec, NRHS)
    c.op.apply_D(ref, bd, prec, nrhs=NRHS)
    got = c.lat.new_field(prec, NRHS)
    c.op.apply_D_cfg(got, bd, prec, NRHS, cfg)
    torch.cuda.synchronize()
    assert torch.equal(ref, got)
    # smoother, from zero and from a start vector
    for x0z in (True, False):
        x0 = c.to_dev(0.1 * synth.source(c.dims, 8, nrhs=NRHS), prec)
        xr = x0.clone()
        xg = x0.clone()
        c.op.sap_smooth_cfg(xr, bd, prec, NRHS, cs.LaunchConfig(1, 0, lanes), x0_is_zero=x0z)
        c.op.sap_smooth_cfg(xg, bd, prec, NRHS, cfg, x0_is_zero=x0z)
        torch.cuda.synchronize()
        assert torch.equal(xr, xg)


def test_autotune_returns_valid_shapes(case):
    sap, d = case.op.autotune(cs.F32, NRHS)
    print("autotuned", sap, d)
    assert sap.rhs_tile in (1, 4) and d.rhs_tile in (1, 4)
    assert sap.persistent_wgs >= 0 and d.persistent_wgs >= 0


# rd = 1e-3 restarts every few iterations, so columns often stop while the
# next iteration is already queued for the batch but not for the lone solve
@pytest.mark.parametrize("inner,basis,rd", [(cs.F32, cs.F32, 1e-5), (cs.F64, cs.F64, 1e-5),
                                            (cs.F32, cs.F32, 1e-3), (cs.F32, cs.F16, 1e-3),
                                            (cs.F32, cs.BF16, 1e-3)])
def test_batched_gcr_columns_equal_single_solves(case, inner, basis, rd):
    c = case
    bs = synth.source(c.dims, 9, nrhs=NRHS)
    bs[2] = 0.0  # a zero right-hand side is solved by x = 0 without iterations
    p_batch = cs.SolverParams(inner_prec=inner, basis_prec=basis, reliable_delta=rd, rhs_tile=4, use_graph=False)
    bd = c.to_dev(bs, cs.F64)
    xd = c.lat.new_field(cs.F64, NRHS).zero_()
    st, stats = c.op.gcr_solve(xd, bd, p_batch, nrhs=NRHS)
    xb = c.to_host(xd, cs.F64, NRHS)
    assert st == 0 and stats[2]["iters"] == 0 and np.abs(xb[2]).max() == 0
    for r in (0, 3, 5):
        x1 = c.lat.new_field(cs.F64).zero_()
        st1, s1 = c.op.gcr_solve(x1, c.to_dev(bs[r], cs.F64),
                                 cs.SolverParams(inner_prec=inner, basis_prec=basis, reliable_delta=rd,
                                                 use_graph=False))
        assert s1[0]["iters"] == stats[r]["iters"]
        assert np.array_equal(c.to_host(x1, cs.F64), xb[r])
        rel = oracle.residual_norm(c.dims, c.U, c.kappa, c.csw, bs[r], xb[r]) / np.linalg.norm(bs[r])
        assert rel <= 1e-10


@pytest.mark.parametrize("groups,use_graph,basis", [(2, False, cs.F32), (3, True, cs.F32), (4, True, cs.F16),
                                                     (9, False, cs.F32)])
def test_concurrent_groups_equal_single_solves(case, groups, use_graph, basis):
    """rhs_groups > 1: contiguous groups solved as their own batches on
    their own workspaces, streams and host threads; every column still
    equals its single-right-hand-side solve bit for bit (groups above nrhs
    fall back to one right-hand side per group)."""
    c = case
    n = 5
    bs = synth.source(c.dims, 13, nrhs=n)
    rd = 1e-3 if basis == cs.F16 else 1e-5
    bd = c.to_dev(bs, cs.F64)
    xd = c.lat.new_field(cs.F64, n).zero_()
    st, stats = c.op.gcr_solve(xd, bd, cs.SolverParams(basis_prec=basis, reliable_delta=rd, rhs_tile=2,
                                                       use_graph=use_graph, rhs_groups=groups), nrhs=n)
    assert st == 0
    xb = c.to_host(xd, cs.F64, n)
    for r in range(n):
        x1 = c.lat.new_field(cs.F64).zero_()
        st1, s1 = c.op.gcr_solve(x1, c.to_dev(bs[r], cs.F64),
                                 cs.SolverParams(basis_prec=basis, reliable_delta=rd, use_graph=False))
        assert s1[0]["iters"] == stats[r]["iters"], r
        assert np.array_equal(c.to_host(x1, cs.F64), xb[r]), r


def test_concurrent_groups_adjoint(case):
    c = case
    bs = synth.source(c.dims, 14, nrhs=4)
    bd = c.to_dev(bs, cs.F64)
    yd = c.lat.new_field(cs.F64, 4).zero_()
    c.op.gcr_solve(yd, bd, cs.SolverParams(rhs_groups=2), nrhs=4, dagger=True)
    y = c.to_host(yd, cs.F64, 4)
    T = oracle.clover_field(c.dims, c.U, c.kappa, c.csw)
    for r in range(4):
        res = oracle.apply_Ddag(c.dims, c.U, T, c.kappa, y[r]) - bs[r]
        assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(bs[r])
    with pytest.raises(cs.CloverSapError):
        c.op.gcr_solve(yd, bd, cs.SolverParams(rhs_groups=-1), nrhs=4)


@pytest.mark.parametrize("use_graph", [False, True])
def test_columns_stopping_at_different_iterations(case, use_graph):
    """Columns with start vectors of different quality stop at different
    iterations.  The solver queues iteration k + 1 before it reads the
    residuals of iteration k, so a column that stops at k still runs k + 1
    once; that must leave its solution untouched: every column equals its
    single solve bit for bit."""
    c = case
    bs = synth.source(c.dims, 21, nrhs=4)
    x0 = np.zeros_like(bs)
    for r, tol in ((1, 1e-3), (2, 1e-6)):  # columns 0 and 3 start from zero
        x1 = c.lat.new_field(cs.F64).zero_()
        c.op.gcr_solve(x1, c.to_dev(bs[r], cs.F64), cs.SolverParams(tol=tol, use_graph=False))
        x0[r] = c.to_host(x1, cs.F64)
    xd = c.to_dev(x0, cs.F64)
    st, stats = c.op.gcr_solve(xd, c.to_dev(bs, cs.F64), cs.SolverParams(rhs_tile=4, use_graph=use_graph),
                               nrhs=4)
    xb = c.to_host(xd, cs.F64, 4)
    its = [s["iters"] for s in stats]
    assert st == 0 and len(set(its)) >= 3, its
    for r in range(4):
        x1 = c.to_dev(x0[r], cs.F64)
        st1, s1 = c.op.gcr_solve(x1, c.to_dev(bs[r], cs.F64), cs.SolverParams(use_graph=use_graph))
        assert st1 == 0 and s1[0]["iters"] == its[r], (r, s1[0]["iters"], its)
        assert np.array_equal(c.to_host(x1, cs.F64), xb[r]), r
        rel = oracle.residual_norm(c.dims, c.U, c.kappa, c.csw, bs[r], xb[r]) / np.linalg.norm(bs[r])
        assert rel <= 1e-10


def test_graph_replay_equals_eager(case):
    c = case
    bs = synth.source(c.dims, 10, nrhs=NRHS)
    bd = c.to_dev(bs, cs.F64)
    eager = c.lat.new_field(cs.F64, NRHS).zero_()
    c.op.gcr_solve(eager, bd, cs.SolverParams(rhs_tile=4, use_graph=False), nrhs=NRHS)
    for rep in range(3):
        xg = c.lat.new_field(cs.F64, NRHS).zero_()
        c.op.gcr_solve(xg, bd, cs.SolverParams(rhs_tile=4, use_graph=True), nrhs=NRHS)
        torch.cuda.synchronize()
        assert torch.equal(xg, eager), rep
        # eager work between replays
        tmp = c.lat.new_field(cs.F32, NRHS)
        c.op.sap_smooth(tmp, c.to_dev(bs, cs.F32), cs.F32, nrhs=NRHS)
        torch.cuda.synchronize()
    # single right-hand side through graphs too
    x1 = c.lat.new_field(cs.F64).zero_()
    x2 = c.lat.new_field(cs.F64).zero_()
    b1 = c.to_dev(bs[1], cs.F64)
    c.op.gcr_solve(x1, b1, cs.SolverParams(use_graph=False))
    c.op.gcr_solve(x2, b1, cs.SolverParams(use_graph=True))
    c.op.gcr_solve(x2.zero_(), b1, cs.SolverParams(use_graph=True))
    torch.cuda.synchronize()
    assert torch.equal(x1, x2)
    # and with a 16-bit basis (the operator writes w_k into it directly)
    p16 = dict(basis_prec=cs.F16, reliable_delta=1e-3)
    c.op.gcr_solve(x1.zero_(), b1, cs.SolverParams(use_graph=False, **p16))
    c.op.gcr_solve(x2.zero_(), b1, cs.SolverParams(use_graph=True, **p16))
    c.op.gcr_solve(x2.zero_(), b1, cs.SolverParams(use_graph=True, **p16))
    torch.cuda.synchronize()
    assert torch.equal(x1, x2)
    # the batch with a 16-bit basis (the tiled operator writes it directly)
    eager16 = c.lat.new_field(cs.F64, NRHS).zero_()
    c.op.gcr_solve(eager16, bd, cs.SolverParams(rhs_tile=4, use_graph=False, **p16), nrhs=NRHS)
    for rep in range(2):
        xg = c.lat.new_field(cs.F64, NRHS).zero_()
        c.op.gcr_solve(xg, bd, cs.SolverParams(rhs_tile=4, use_graph=True, **p16), nrhs=NRHS)
        torch.cuda.synchronize()
        assert torch.equal(xg, eager16), rep


def test_batched_adjoint_solve(case):
    c = case
    bs = synth.source(c.dims, 12, nrhs=3)
    bd = c.to_dev(bs, cs.F64)
    yd = c.lat.new_field(cs.F64, 3).zero_()
    c.op.gcr_solve(yd, bd, cs.SolverParams(rhs_tile=0), nrhs=3, dagger=True)
    y = c.to_host(yd, cs.F64, 3)
    T = oracle.clover_field(c.dims, c.U, c.kappa, c.csw)
    for r in range(3):
        res = oracle.apply_Ddag(c.dims, c.U, T, c.kappa, y[r]) - bs[r]
        assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(bs[r])
