"""Oracle pins for the gradient of L = Re(eta^dag D^{-1} b) with respect to the
gauge links (the differentiation growth line built on the operator of the
paper's Eq. (1), Section 2).

The gradient is taken in left Lie-algebra coordinates, U -> exp(i w T^a) U,
T^a = lambda^a / 2.  It is pinned against central finite differences of L
(h = 1e-5, tight FP64 solves), first with c_sw = 0 (hopping term only) and
then with the clover term, and against gauge covariance of the projected
force.
"""
import numpy as np
import pytest

import oracle
from paper_2112_00501_amd import synth
from tests.oracle_helpers import gauge_transform_links, gauge_transform_spinor

DIMS, BDIM = (4, 4, 4, 4), (2, 2, 2, 2)
KAPPA = 0.1355
H = 1e-5


def _solve(U, T, rhs):
    x, st, it, rel, _ = oracle.fgcr(DIMS, BDIM, U, T, KAPPA, rhs, n_cy=2, n_mr=4,
                                    restart=16, tol=1e-13, max_iter=500)
    assert st == 0, rel
    return x


def _loss(U, csw, b, eta):
    T = oracle.clover_field(DIMS, U, KAPPA, csw)
    return np.vdot(eta, _solve(U, T, b)).real


def _gradient(U, csw, b, eta):
    T = oracle.clover_field(DIMS, U, KAPPA, csw)
    x = _solve(U, T, b)
    # D^dag = g5 D g5, so y = D^{-dag} eta = g5 D^{-1} g5 eta
    s = np.array([1, 1, -1, -1])[None, :, None]
    y = s * _solve(U, T, s * eta)
    gh, gc = oracle.force(DIMS, U, KAPPA, csw, x, y)
    return gh, gc, x, y


def _perturb(U, X, h):
    """U_mu(x) -> exp(i h X_mu(x)) U_mu(x), X = sum_a X^a T^a."""
    gens = np.stack([oracle.su3_generator(a) for a in range(8)])
    Xm = np.einsum("vma,aij->vmij", X, gens)
    E = synth.expm_i_herm(Xm.reshape(-1, 3, 3), h).reshape(Xm.shape)
    return np.einsum("vmij,vmjk->vmik", E, U)


@pytest.fixture(scope="module")
def inputs():
    U = synth.gauge_field(DIMS, 0.3, 1015)
    b = synth.source(DIMS, 2015)
    eta = synth.source(DIMS, 3015)
    return U, b, eta


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_gradient_matches_central_differences(inputs, csw):
    U, b, eta = inputs
    gh, gc, _, _ = _gradient(U, csw, b, eta)
    g = gh + gc
    if csw == 0.0:
        assert np.abs(gc).max() == 0
    rng = np.random.default_rng(17)
    # a random direction over all links at once
    X = rng.standard_normal(g.shape)
    fd = (_loss(_perturb(U, X, H), csw, b, eta) - _loss(_perturb(U, X, -H), csw, b, eta)) / (2 * H)
    an = np.sum(g * X)
    assert abs(fd - an) <= 1e-6 * abs(an)
    # single links and generators, including the largest components
    flat = np.argsort(np.abs(g).ravel())[::-1]
    picks = list(flat[:3]) + list(rng.choice(g.size, 3, replace=False))
    for k in picks:
        X = np.zeros(g.size)
        X[k] = 1.0
        X = X.reshape(g.shape)
        fd = (_loss(_perturb(U, X, H), csw, b, eta) - _loss(_perturb(U, X, -H), csw, b, eta)) / (2 * H)
        assert abs(fd - g.ravel()[k]) <= 1e-6 * np.abs(g).max()


def test_clover_part_scales_linearly_in_csw(inputs):
    U, b, eta = inputs
    T = oracle.clover_field(DIMS, U, KAPPA, 1.0)
    x = _solve(U, T, b)
    y = synth.source(DIMS, 5)
    _, gc1 = oracle.force(DIMS, U, KAPPA, 1.0, x, y, parts=("clov",))
    _, gc2 = oracle.force(DIMS, U, KAPPA, 2.5, x, y, parts=("clov",))
    assert np.allclose(gc2, 2.5 * gc1, atol=1e-13)


def test_projected_force_is_gauge_covariant(inputs):
    U, b, eta = inputs
    csw = 1.0
    gh, gc, x, y = _gradient(U, csw, b, eta)
    Om = synth.gauge_transform(DIMS, 4011)
    Ug = gauge_transform_links(DIMS, U, Om)
    xg, yg = gauge_transform_spinor(Om, x), gauge_transform_spinor(Om, y)
    ghg, gcg = oracle.force(DIMS, Ug, KAPPA, csw, xg, yg)
    gens = np.stack([oracle.su3_generator(a) for a in range(8)])
    P = np.einsum("vma,aij->vmij", gh + gc, gens)
    Pg = np.einsum("vma,aij->vmij", ghg + gcg, gens)
    # left derivative: P'_mu(x) = Om(x) P_mu(x) Om(x)^dag
    ref = np.einsum("vab,vmbc,vdc->vmad", Om, P, np.conj(Om))
    assert np.abs(Pg - ref).max() < 1e-12 * np.abs(P).max()


def test_every_link_against_central_differences():
    """Every link and generator of a 4^4 lattice (1024 links x 8), c_sw = 1:
    the oracle's force against central differences (h = 1e-5) of the loss
    L = Re(eta^dag D^-1 b), with L evaluated exactly by dense linear
    algebra.  D is assembled densely from the oracle's operator and inverted
    once.  A link change alters D only on the 14 sites whose clover leaves
    contain the link (which include the link's two hop rows), so the changed
    loss follows from the Woodbury identity on that 168 x 168 block:
    L' - L = -Re(y_S^dag (1 + Delta Dinv_SS)^-1 Delta x_S), x = D^-1 b,
    y = D^-dag eta.  The difference is formed directly, so nothing cancels.
    Delta is written here with numpy: the changed clover blocks come from
    the oracle's per-site clover term, and the two hop blocks
    -kappa (1 -/+ gamma_mu) (x) dU are built from explicit gamma matrices."""
    import scipy.linalg

    from tests.oracle_helpers import coords, dense_D, dof_indices
    from tests.test_oracle_operator import GAMMA

    csw = 1.0
    U = synth.gauge_field(DIMS, 0.3, 1015)
    b, eta = synth.source(DIMS, 2015), synth.source(DIMS, 3015)
    T = oracle.clover_field(DIMS, U, KAPPA, csw)
    M = dense_D(DIMS, U, T, KAPPA)
    Minv = np.linalg.inv(M)
    x = Minv @ b.reshape(-1)
    y = Minv.conj().T @ eta.reshape(-1)
    gh, gc = oracle.force(DIMS, U, KAPPA, csw, x.reshape(b.shape), y.reshape(b.shape))
    g = gh + gc

    V = int(np.prod(DIMS))
    c = coords(DIMS, V)

    def site(cc):
        cc = np.mod(cc, DIMS)
        return int(cc[0] + DIMS[0] * (cc[1] + DIMS[1] * (cc[2] + DIMS[2] * cc[3])))

    E = {(a, sgn): scipy.linalg.expm(1j * sgn * H * oracle.su3_generator(a)) for a in range(8) for sgn in (1, -1)}
    eye4 = np.eye(4)
    fd = np.zeros_like(g)
    for s in range(V):
        for mu in range(4):
            e_mu = np.eye(4, dtype=int)[mu]
            sp = site(c[s] + e_mu)
            S = {s, sp}
            for nu in range(4):
                if nu == mu:
                    continue
                e_nu = np.eye(4, dtype=int)[nu]
                for step in (1, -1):
                    S |= {site(c[s] + step * e_nu), site(c[s] + e_mu + step * e_nu)}
            S = sorted(S)
            assert len(S) == 14
            pos = {z: i for i, z in enumerate(S)}
            idx = dof_indices(S)
            Dinv_SS = Minv[np.ix_(idx, idx)]
            xS, yS = x[idx], y[idx]
            k = idx.size
            dl = {}
            for (a, sgn), Ea in E.items():
                Up = U.copy()
                Up[s, mu] = Ea @ U[s, mu]
                dU = Up[s, mu] - U[s, mu]
                Delta = np.zeros((k, k), np.complex128)
                for z in S:
                    i = 12 * pos[z]
                    Delta[i:i + 12, i:i + 12] = oracle.clover_site(DIMS, Up, KAPPA, csw, z) - T[z]
                i, j = 12 * pos[s], 12 * pos[sp]
                Delta[i:i + 12, j:j + 12] += -KAPPA * np.kron(eye4 - GAMMA[mu], dU)
                Delta[j:j + 12, i:i + 12] += -KAPPA * np.kron(eye4 + GAMMA[mu], dU.conj().T)
                zv = np.linalg.solve(np.eye(k) + Delta @ Dinv_SS, Delta @ xS)
                dl[(a, sgn)] = -np.vdot(yS, zv).real
            for a in range(8):
                fd[s, mu, a] = (dl[(a, 1)] - dl[(a, -1)]) / (2 * H)
    err = np.linalg.norm(fd - g) / np.linalg.norm(g)
    err_max = np.abs(fd - g).max() / np.abs(g).max()
    print(f"every link: |fd - g| / |g| = {err:.3e}, max |fd - g| / max |g| = {err_max:.3e}")
    assert err <= 1e-6 and err_max <= 1e-6
