"""GPU link gradient (the differentiation growth line on the operator of the
paper's Eq. (1), Section 2): force kernel against the oracle's literal
leaf-by-leaf derivative, against central finite differences of GPU solves,
and through torch.autograd."""
import numpy as np
import pytest
import torch

import oracle
from paper_2112_00501_amd import cloversap as cs
from paper_2112_00501_amd import synth
from tests.gpu_helpers import Case, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def grad8():
    c = synth.CONFIGS["grad_8x8x8x8"]
    return Case(c["dims"], c["eps"], c["kappa"], c["csw"], c["gauge_seed"])


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_force_matches_oracle(grad8, csw):
    c = grad8
    x = synth.source(c.dims, 11)
    y = synth.source(c.dims, 12)
    lat = c.lat
    op = cs.Operator(lat, torch.from_numpy(c.U).cuda(), c.kappa, csw)
    g, G = op.force(c.to_dev(x, cs.F64), c.to_dev(y, cs.F64), want_lie=True, want_grad=True)
    torch.cuda.synchronize()
    gh, gc = oracle.force(c.dims, c.U, c.kappa, csw, x, y)
    ref = gh + gc
    err = rel(g.cpu().numpy(), ref)
    print(f"csw={csw} force rel.err={err:.3e}")
    assert err < 1e-12
    # G = 2 i (sum_a g_a T^a) U
    gens = np.stack([oracle.su3_generator(a) for a in range(8)])
    P = np.einsum("vma,aij->vmij", ref, gens)
    Gref = 2j * np.einsum("vmij,vmjk->vmik", P, c.U)
    assert rel(G.cpu().numpy(), Gref) < 1e-12


def _loss(dims, U, kappa, csw, b, eta):
    lat = cs.Lattice(dims)
    op = cs.Operator(lat, torch.from_numpy(U).cuda(), kappa, csw)
    bd = lat.import_field(torch.from_numpy(b).cuda(), cs.F64)
    xd = lat.new_field(cs.F64).zero_()
    op.gcr_solve(xd, bd, cs.SolverParams(inner_prec=cs.F64, basis_prec=cs.F64, tol=1e-13,
                                         max_iter=1000))
    x = lat.export_field(xd, cs.F64).cpu().numpy()
    return np.vdot(eta, x).real


def test_gradient_matches_central_differences_8x8x8x8(grad8):
    c = grad8
    b, eta = synth.source(c.dims, 2025), synth.source(c.dims, 3025)
    U = c.U
    Ut = torch.from_numpy(U).cuda().requires_grad_(True)
    bt = torch.from_numpy(b).cuda().requires_grad_(True)
    params = cs.SolverParams(inner_prec=cs.F64, basis_prec=cs.F64, tol=1e-13, max_iter=1000)
    x = cs.CloverSolve.apply(Ut, bt, c.lat, c.kappa, c.csw, params)
    L = (torch.conj(torch.from_numpy(eta).cuda()) * x).sum().real
    L.backward()
    G = Ut.grad.cpu().numpy()
    rng = np.random.default_rng(5)
    gens = np.stack([oracle.su3_generator(a) for a in range(8)])
    X = rng.standard_normal((c.lat.volume, 4, 8))
    Xm = np.einsum("vma,aij->vmij", X, gens)
    h = 1e-5
    Up = np.einsum("vmij,vmjk->vmik", synth.expm_i_herm(Xm.reshape(-1, 3, 3), h).reshape(Xm.shape), U)
    Um = np.einsum("vmij,vmjk->vmik", synth.expm_i_herm(Xm.reshape(-1, 3, 3), -h).reshape(Xm.shape), U)
    fd = (_loss(c.dims, Up, c.kappa, c.csw, b, eta) - _loss(c.dims, Um, c.kappa, c.csw, b, eta)) / (2 * h)
    # dL = Re tr(G^dag dU) with dU = i X U
    an = np.real(np.einsum("vmij,vmij->", np.conj(G), 1j * np.einsum("vmij,vmjk->vmik", Xm, U)))
    print(f"FD {fd:.12e} analytic {an:.12e} rel {abs(fd - an) / abs(an):.2e}")
    assert abs(fd - an) <= 1e-6 * abs(an)
    # grad_b = D^-dag eta
    y = bt.grad.cpu().numpy()
    T = oracle.clover_field(c.dims, U, c.kappa, c.csw)
    assert rel(oracle.apply_Ddag(c.dims, U, T, c.kappa, y), eta) < 1e-12


def test_force_against_oracle_gradient_of_solutions(grad8):
    """The oracle's gradient of L (its own FP64 solves) equals the GPU's."""
    c = grad8
    b, eta = synth.source(c.dims, 2025), synth.source(c.dims, 3025)
    bdim = (4, 4, 4, 4)
    xo, *_ = oracle.fgcr(c.dims, bdim, c.U, c.T, c.kappa, b, tol=1e-12)
    s = np.array([1, 1, -1, -1])[None, :, None]
    yo, *_ = oracle.fgcr(c.dims, bdim, c.U, c.T, c.kappa, s * eta, tol=1e-12)
    yo = s * yo
    gh, gc = oracle.force(c.dims, c.U, c.kappa, c.csw, xo, yo)
    bd = c.to_dev(b, cs.F64)
    ed = c.to_dev(eta, cs.F64)
    xd = c.lat.new_field(cs.F64).zero_()
    yd = c.lat.new_field(cs.F64).zero_()
    p = cs.SolverParams(inner_prec=cs.F32, basis_prec=cs.F32, tol=1e-12)
    c.op.gcr_solve(xd, bd, p)
    c.op.gcr_solve(yd, ed, p, dagger=True)
    g, _ = c.op.force(xd, yd)
    torch.cuda.synchronize()
    err = rel(g.cpu().numpy(), gh + gc)
    print(f"gradient vs oracle rel.err={err:.3e}")
    assert err < 1e-9


def test_recomputed_forward_gives_the_same_gradient(grad8):
    """CloverSolve with recompute=True keeps only U and b between the passes
    and solves D x = b again in the backward pass: the gradients equal those
    of the stored-solution form bit for bit."""
    c = grad8
    b, eta = synth.source(c.dims, 2026), synth.source(c.dims, 3026)
    etat = torch.from_numpy(eta).cuda()
    grads = []
    for recompute in (False, True):
        Ut = torch.from_numpy(c.U).cuda().requires_grad_(True)
        bt = torch.from_numpy(b).cuda().requires_grad_(True)
        x = cs.CloverSolve.apply(Ut, bt, c.lat, c.kappa, c.csw, cs.SolverParams(), recompute)
        L = (torch.conj(etat) * x).sum().real
        L.backward()
        torch.cuda.synchronize()
        grads.append((x.detach().cpu().numpy(), Ut.grad.cpu().numpy(), bt.grad.cpu().numpy()))
    for a, r in zip(grads[0], grads[1]):
        assert np.array_equal(a, r)
