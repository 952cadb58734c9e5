"""GPU flexible BiCGStab (the paper's outer solver, Section 3) against the
FP64 oracle's flexible BiCGStab, through the C ABI: with FP64 everywhere the
two follow the same iterations; with FP32/FP16/BF16 smoothing the FP64 outer
iteration still reaches a true residual of 1e-10 (Section 2), checked with the
oracle's own operator."""
import numpy as np
import pytest
import torch

import oracle
from paper_2112_00501_amd import cloversap as cs
from paper_2112_00501_amd import synth
from tests.gpu_helpers import Case

pytestmark = pytest.mark.gpu

BDIM = (4, 4, 4, 4)


@pytest.fixture(scope="module")
def cfg1():
    return Case((8, 8, 8, 8), 0.3, 0.13, 1.0, 1001)


def _solve(c, b, inner, vec=cs.F64, **kw):
    p = cs.SolverParams(inner_prec=inner, basis_prec=vec, **kw)
    bd = c.to_dev(b, cs.F64)
    xd = c.lat.new_field(cs.F64).zero_()
    st, stats = c.op.bicgstab_solve(xd, bd, p, allow_fail=True)
    return st, stats, c.to_host(xd, cs.F64)


@pytest.mark.parametrize("n_cy", [0, 2])
def test_fp64_bicgstab_follows_oracle(cfg1, n_cy):
    c = cfg1
    b = synth.source(c.dims, 2001)
    xr, st_r, it_r, rs_r, rel_r, _ = oracle.fbicgstab(c.dims, BDIM, c.U, c.T, c.kappa, b, n_cy=n_cy,
                                                      tol=1e-10, delta=1e-5)
    st, stats, x = _solve(c, b, cs.F64, n_cy=n_cy, tol=1e-10, reliable_delta=1e-5)
    rel = oracle.residual_norm(c.dims, c.U, c.kappa, c.csw, b, x) / np.linalg.norm(b)
    print(f"n_cy={n_cy} oracle iters={it_r} restarts={rs_r}; gpu iters={stats['iters']} "
          f"restarts={stats['restarts']} relres={rel:.3e}")
    assert st == 0 and st_r == 0
    assert abs(stats["iters"] - it_r) <= 1
    assert rel <= 1e-10
    assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xr)


@pytest.mark.parametrize("inner", [cs.F32, cs.F16, cs.BF16])
def test_mixed_bicgstab_reaches_fp64_residual(cfg1, inner):
    for c, seed in ((cfg1, 2001), (Case((16, 16, 16, 32), 0.3, 0.1355, 1.0, 1002, oracle_T=False), 2002)):
        b = synth.source(c.dims, seed)
        st, stats, x = _solve(c, b, inner, tol=1e-10)
        rel = oracle.residual_norm(c.dims, c.U, c.kappa, c.csw, b, x) / np.linalg.norm(b)
        print(f"{c.dims} inner={inner} iters={stats['iters']} restarts={stats['restarts']} "
              f"gpu relres={stats['true_relres']:.3e} oracle relres={rel:.3e}")
        assert st == 0
        assert rel <= 1e-10 * (1 + 1e-6)


def test_bicgstab_zero_rhs_warm_start_and_cap(cfg1):
    c = cfg1
    p = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F64, tol=1e-10)
    # zero right-hand side: x = 0 without iterations, whatever x held
    xd = c.to_dev(synth.source(c.dims, 5), cs.F64)
    st, stats = c.op.bicgstab_solve(xd, c.lat.new_field(cs.F64).zero_(), p)
    assert st == 0 and stats["iters"] == 0 and float(xd.view(torch.float64).abs().max()) == 0.0
    # warm start from a 1e-4 solution needs fewer iterations than from zero
    b = synth.source(c.dims, 6)
    bd = c.to_dev(b, cs.F64)
    x1 = c.lat.new_field(cs.F64).zero_()
    st, s1 = c.op.bicgstab_solve(x1, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F64, tol=1e-4))
    x2 = x1.clone()
    st, s2 = c.op.bicgstab_solve(x2, bd, p)
    x3 = c.lat.new_field(cs.F64).zero_()
    st, s3 = c.op.bicgstab_solve(x3, bd, p)
    assert st == 0 and s2["iters"] < s3["iters"]
    rel = oracle.residual_norm(c.dims, c.U, c.kappa, c.csw, b, c.to_host(x2, cs.F64)) / np.linalg.norm(b)
    assert rel <= 1e-10 * (1 + 1e-6)
    # iteration cap
    x4 = c.lat.new_field(cs.F64).zero_()
    st, s4 = c.op.bicgstab_solve(x4, bd, cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F64, max_iter=2),
                                 allow_fail=True)
    assert st == 1 and s4["iters"] == 2 and s4["true_relres"] > 1e-10


def test_bicgstab_graph_replay_equals_eager(cfg1):
    c = cfg1
    b = c.to_dev(synth.source(c.dims, 7), cs.F64)
    outs = []
    for vec in (cs.F64, cs.F32):
        outs = []
        for use_graph in (False, True, True):
            x = c.lat.new_field(cs.F64).zero_()
            c.op.bicgstab_solve(x, b, cs.SolverParams(inner_prec=cs.F32, basis_prec=vec, use_graph=use_graph))
            torch.cuda.synchronize()
            outs.append(x)
        assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


@pytest.mark.parametrize("inner", [cs.F32, cs.F16, cs.BF16])
def test_single_precision_richardson_form(cfg1, inner):
    """FP32 BiCGStab vectors inside an FP64 Richardson iteration (the QWS
    scheme, paper Section 2): the true residual still reaches 1e-10, in about
    as many Richardson steps as the oracle's FP64 version of the scheme."""
    for c, seed in ((cfg1, 2001), (Case((16, 16, 16, 32), 0.3, 0.1355, 1.0, 1002, oracle_T=False), 2002)):
        b = synth.source(c.dims, seed)
        st, stats, x = _solve(c, b, inner, vec=cs.F32, tol=1e-10, reliable_delta=1e-5)
        rel = oracle.residual_norm(c.dims, c.U, c.kappa, c.csw, b, x) / np.linalg.norm(b)
        print(f"{c.dims} inner={inner} iters={stats['iters']} richardson steps={stats['restarts'] + 1} "
              f"oracle relres={rel:.3e}")
        assert st == 0
        assert rel <= 1e-10 * (1 + 1e-6)
        if c is cfg1:
            _, st_r, it_r, outer_r, _ = oracle.richardson_bicgstab(c.dims, BDIM, c.U, c.T, c.kappa, b,
                                                                   inner_tol=1e-5)
            print(f"  oracle: iters={it_r} richardson steps={outer_r}")
            assert st_r == 0 and abs(stats["restarts"] + 1 - outer_r) <= 1


@pytest.mark.parametrize("block_solver", [1, 2])
@pytest.mark.parametrize("solver", ["gcr", "bicgstab_sp"])
def test_solves_with_the_jacobi_smoother(cfg1, solver, block_solver):
    """The smoother variants — the QWS form (SAP on C^-1 D, Jacobi block
    solves) and SAP with even-odd preconditioned MR — as the preconditioner
    of the FP64 outer solvers: the true residual reaches 1e-10."""
    for c, seed in ((cfg1, 2001), (Case((16, 16, 16, 32), 0.3, 0.1355, 1.0, 1002, oracle_T=False), 2002)):
        b = synth.source(c.dims, seed)
        p = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32, n_cy=2, n_mr=4, tol=1e-10,
                            block_solver=block_solver)
        bd = c.to_dev(b, cs.F64)
        xd = c.lat.new_field(cs.F64).zero_()
        if solver == "gcr":
            st, stats = c.op.gcr_solve(xd, bd, p)
            stats = stats[0]
        else:
            st, stats = c.op.bicgstab_solve(xd, bd, p)
        x = c.to_host(xd, cs.F64)
        rel = oracle.residual_norm(c.dims, c.U, c.kappa, c.csw, b, x) / np.linalg.norm(b)
        print(f"{c.dims} {solver} block solver {block_solver} iters={stats['iters']} oracle relres={rel:.3e}")
        assert st == 0
        assert rel <= 1e-10 * (1 + 1e-6)
