"""Pins of the oracle's discrete operators against what the paper and the
mathematics fix (Section 2.2 of the paper): backward-difference gradient, the
divergence as its negative adjoint, the Gershgorin bound, the shrink operator,
the closed-form primal update and the dual update."""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_default_parameters_are_the_papers(oracle_mod):
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        k = json.load(fh)
    p = oracle_mod.Params()
    assert p.eps == k["eps"] and p.xi == k["xi"] and p.zeta == k["zeta"]
    assert p.delta == k["delta"]


@pytest.mark.parametrize("nr,nt,dx,dt", [(5, 7, 0.3, 0.1), (1, 9, 1.0, 0.25), (6, 1, 0.5, 1.0)])
def test_grad_of_linear_field(oracle_mod, nr, nt, dx, dt):
    # phi = a x + b t: backward differences give (a, b) except the zero first row/col
    a, b = 1.7, -0.6
    x = np.arange(nr)[:, None] * dx
    t = np.arange(nt)[None, :] * dt
    gx, gt = oracle_mod.grad(a * x + b * t + 0 * x * t, dx, dt)
    ex = np.full((nr, nt), a)
    ex[0, :] = 0.0
    et = np.full((nr, nt), b)
    et[:, 0] = 0.0
    np.testing.assert_allclose(gx, ex, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gt, et, rtol=1e-12, atol=1e-12)


def test_grad_is_backward_difference(oracle_mod):
    # phi = x^2 (receiver axis) and t^3 (time axis): a backward difference at i is
    # ((i dx)^2 - ((i-1) dx)^2)/dx = (2i - 1) dx; forward or central would differ
    nr, nt, dx, dt = 6, 5, 0.5, 0.2
    i = np.arange(nr)[:, None]
    j = np.arange(nt)[None, :]
    phi = (i * dx) ** 2 + (j * dt) ** 3
    gx, gt = oracle_mod.grad(phi, dx, dt)
    ex = np.where(i > 0, (2 * i - 1) * dx, 0.0) + 0 * j
    et = np.where(j > 0, ((j * dt) ** 3 - ((j - 1) * dt) ** 3) / dt, 0.0) + 0 * i
    np.testing.assert_allclose(gx, ex, rtol=1e-12)
    np.testing.assert_allclose(gt, et, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("nr,nt", [(5, 7), (1, 11), (9, 1), (13, 17)])
def test_adjoint_identity(oracle_mod, seed, nr, nt):
    # <u, grad phi> = -<div u, phi> (Section 2.2) for random fields
    rng = np.random.default_rng(seed)
    dx, dt = 0.3, 0.07
    ux, ut, phi = rng.normal(size=(3, nr, nt))
    gx, gt = oracle_mod.grad(phi, dx, dt)
    d = oracle_mod.div(ux, ut, dx, dt)
    lhs = np.sum(ux * gx + ut * gt)
    rhs = -np.sum(d * phi)
    scale = np.sum(np.abs(ux * gx) + np.abs(ut * gt))
    assert abs(lhs - rhs) <= 1e-13 * scale


def test_div_is_forward_difference_in_interior(oracle_mod):
    # away from the last row/column the divergence is the printed forward difference
    rng = np.random.default_rng(3)
    nr, nt, dx, dt = 7, 9, 0.4, 0.3
    ux, ut = rng.normal(size=(2, nr, nt))
    d = oracle_mod.div(ux, ut, dx, dt)
    fwd = (ux[2:, 1:-1] - ux[1:-1, 1:-1]) / dx + (ut[1:-1, 2:] - ut[1:-1, 1:-1]) / dt
    np.testing.assert_allclose(d[1:-1, 1:-1], fwd, rtol=1e-12, atol=1e-12)


def test_div_conserves_mass(oracle_mod):
    # the column sums of -grad^T vanish: sum(div u) = 0 for every u, so div u + s = 0
    # is solvable exactly when sum(s) = 0 (the mass balance of Section 2.1)
    rng = np.random.default_rng(4)
    for nr, nt in [(5, 7), (1, 8), (12, 3)]:
        ux, ut = rng.normal(size=(2, nr, nt))
        d = oracle_mod.div(ux, ut, 0.2, 0.9)
        assert abs(d.sum()) <= 1e-12 * np.abs(d).sum()


def _operator_matrix(oracle_mod, nr, nt, dx, dt):
    n = nr * nt
    L = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        gx, gt = oracle_mod.grad(e.reshape(nr, nt), dx, dt)
        L[:, c] = -oracle_mod.div(gx, gt, dx, dt).reshape(-1)
    return L


@pytest.mark.parametrize("nr,nt,dx,dt", [(5, 7, 0.3, 0.1), (12, 12, 1.0, 1.0), (3, 20, 0.5, 0.05)])
def test_gershgorin_bound(oracle_mod, nr, nt, dx, dt):
    # lambda_max(-div grad) <= 4/dx^2 + 4/dt^2 (Section 2.2), and the operator is
    # the symmetric positive semidefinite Neumann Laplacian with constants in its kernel
    L = _operator_matrix(oracle_mod, nr, nt, dx, dt)
    np.testing.assert_allclose(L, L.T, atol=1e-9 * np.abs(L).max())
    w = np.linalg.eigvalsh(L)
    bound = oracle_mod.lambda_bound(nr, nt, dx, dt)
    assert bound == pytest.approx(4 / dx**2 + 4 / dt**2)
    assert w.max() <= bound * (1 + 1e-12)
    assert w.max() >= 0.5 * bound
    assert abs(w.min()) <= 1e-9 * w.max()
    assert np.sum(np.abs(w) <= 1e-9 * w.max()) == 1  # only constants in the kernel


def test_gershgorin_bound_is_tight_for_large_grids(oracle_mod):
    # the 1D Neumann Laplacian's top eigenvalue (4/dt^2) sin^2(pi (n-1) / (2n)) -> 4/dt^2
    n, dt = 64, 0.1
    L = _operator_matrix(oracle_mod, 1, n, 1.0, dt)
    w = np.linalg.eigvalsh(L)
    exact = 4 / dt**2 * np.sin(np.pi * (n - 1) / (2 * n)) ** 2
    assert w.max() == pytest.approx(exact, rel=1e-10)


def test_shrink_definition(oracle_mod):
    # shrink(x, y) = (1 - y/|x|) x for |x| >= y, else 0 (Section 2.2)
    assert oracle_mod.shrink(3.0, 1.0) == pytest.approx(2.0)
    assert oracle_mod.shrink(-3.0, 1.0) == pytest.approx(-2.0)
    assert oracle_mod.shrink(0.5, 1.0) == 0.0
    assert oracle_mod.shrink(-0.999, 1.0) == 0.0
    assert oracle_mod.shrink(1.0, 1.0) == 0.0
    assert oracle_mod.shrink(0.0, 0.0) == 0.0


def _golden_min(fun, lo, hi, iters=200):
    gr = (np.sqrt(5) - 1) / 2
    a, b = lo, hi
    c, d = b - gr * (b - a), a + gr * (b - a)
    for _ in range(iters):
        if fun(c) < fun(d):
            b = d
        else:
            a = c
        c, d = b - gr * (b - a), a + gr * (b - a)
    return 0.5 * (a + b)


@pytest.mark.parametrize("u0,g,alpha,eps", [(0.3, 2.0, 0.4, 1e-4), (-1.0, 0.5, 0.2, 0.3),
                                            (0.05, -0.1, 0.5, 1e-4), (2.0, -9.0, 0.1, 1.0),
                                            (0.0, 0.2, 1.0, 0.0)])
def test_prox_minimises_the_primal_subproblem(oracle_mod, u0, g, alpha, eps):
    # u^{k+1} = argmin |u| + eps/2 u^2 - g u + (u - u^k)^2 / (2 alpha) per component
    # (the primal subproblem after the adjoint identity, Section 2.2)
    def obj(u):
        return abs(u) + 0.5 * eps * u * u - g * u + (u - u0) ** 2 / (2 * alpha)
    ref = _golden_min(obj, -50.0, 50.0)
    got = oracle_mod.prox(u0, g, alpha, eps)
    # a golden-section search locates a smooth minimum only to ~sqrt(machine eps);
    # the objective value is the sharp check
    assert got == pytest.approx(ref, abs=1e-6)
    assert obj(got) <= obj(ref) + 1e-14 * (1 + abs(obj(ref)))


def test_dual_update_maximises_the_dual_subproblem(oracle_mod):
    # one iteration of plain PDHG (fixed steps, theta = 1): phi^1 must maximise
    # <phi, div ubar + s> - ||phi - phi^0||^2 / (2 beta) with ubar = 2 u^1 - u^0,
    # u^1 the primal update from (u^0, phi^0)
    rng = np.random.default_rng(7)
    nr, nt, dx, dt = 4, 6, 0.5, 0.25
    s = rng.normal(size=(nr, nt))
    s -= s.mean()
    ux0, ut0, phi0 = 0.1 * rng.normal(size=(3, nr, nt))
    p = oracle_mod.Params(ls_mode=oracle_mod.LS_FIXED, max_iter=1, check_every=1,
                          tol_res=0.0, delta=3.0)
    alpha = 1.0 / np.sqrt(p.delta * oracle_mod.lambda_bound(nr, nt, dx, dt))
    beta = p.delta * alpha
    r = oracle_mod.solve(s, dx, dt, p, u0=(ux0, ut0), phi0=phi0)
    assert r.iters == 1
    gx, gt = oracle_mod.grad(phi0, dx, dt)
    ux1 = np.vectorize(lambda u, g: oracle_mod.prox(u, g, alpha, p.eps))(ux0, gx)
    ut1 = np.vectorize(lambda u, g: oracle_mod.prox(u, g, alpha, p.eps))(ut0, gt)
    np.testing.assert_allclose(r.ux, ux1, rtol=1e-12, atol=1e-15)
    d = oracle_mod.div(2 * ux1 - ux0, 2 * ut1 - ut0, dx, dt) + s
    for c in range(nr * nt):
        i, j = divmod(c, nt)
        def neg(v):
            return -(v * d[i, j] - (v - phi0[i, j]) ** 2 / (2 * beta))
        best = _golden_min(neg, phi0[i, j] - 1e3, phi0[i, j] + 1e3)
        assert r.phi[i, j] == pytest.approx(best, abs=1e-5 * (1 + abs(best)))
        assert neg(r.phi[i, j]) <= neg(best) + 1e-14 * (1 + abs(neg(best)))
