"""The oracle's optimum certified by duality at sizes the Kantorovich LP cannot reach.

Any potential whose neighbour differences are at most the grid step gives a lower
bound dx dt <phi, s> on W1 (the dual Kantorovich form of Section 2.1; the Beckmann
dual of Section 2.2 has the same constraint), and the flux plus a transport of its
residual gives an upper bound.  ``certificate`` computes both from the oracle's
outputs with its own divergence and Lipschitz projection, so the bracket depends on
nothing the oracle computes except the two fields it checks.
"""
import itertools

import numpy as np
import pytest

from certificate import divergence, lip_below, residual_flux, transport_bounds
from synth import config1_pairs, config2_gather, random_small_pair
from test_oracle_solver import FIXED_BUDGET, closed_form_1d, kantorovich_lp


def test_lip_below_is_the_inf_convolution_with_the_l1_cone():
    rng = np.random.default_rng(7)
    nr, nt, dx, dt = 5, 7, 0.3, 0.2
    phi = rng.normal(size=(nr, nt))
    got = lip_below(phi, dx, dt)
    ref = np.empty_like(phi)
    for i, j in itertools.product(range(nr), range(nt)):
        ref[i, j] = min(phi[a, b] + dx * abs(a - i) + dt * abs(b - j)
                        for a, b in itertools.product(range(nr), range(nt)))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)
    assert np.all(got <= phi)
    assert np.all(np.abs(np.diff(got, axis=0)) <= dx * (1 + 1e-12))
    assert np.all(np.abs(np.diff(got, axis=1)) <= dt * (1 + 1e-12))


def test_lip_below_keeps_a_feasible_potential():
    nr, nt, dx, dt = 9, 13, 0.05, 0.02
    i, j = np.meshgrid(np.arange(nr), np.arange(nt), indexing="ij")
    phi = 0.9 * i * dx - 0.6 * j * dt + 3.0
    np.testing.assert_array_equal(lip_below(phi, dx, dt), phi)


def test_certificate_divergence_is_minus_the_gradient_transpose():
    rng = np.random.default_rng(8)
    nr, nt, dx, dt = 6, 11, 0.4, 0.15
    ux, ut, phi = rng.normal(size=(3, nr, nt))
    gx = np.zeros((nr, nt))
    gt = np.zeros((nr, nt))
    gx[1:] = np.diff(phi, axis=0) / dx       # backward differences, zero on the first row
    gt[:, 1:] = np.diff(phi, axis=1) / dt
    ux[0] = 0.0                              # components the gradient never reaches
    ut[:, 0] = 0.0
    d = divergence(ux, ut, dx, dt)
    assert abs((d * phi).sum() + (gx * ux + gt * ut).sum()) <= 1e-12 * np.abs(d * phi).sum()
    assert abs(d.sum()) <= 1e-12 * np.abs(d).sum()


@pytest.mark.parametrize("nr,nt", [(6, 9), (1, 12), (10, 1)])
def test_residual_flux_cancels_the_residual(nr, nt):
    rng = np.random.default_rng(9)
    r = rng.normal(size=(nr, nt))
    r -= r.mean()
    vx, vt = residual_flux(r, 0.3, 0.07)
    np.testing.assert_allclose(divergence(vx, vt, 0.3, 0.07), -r, rtol=0, atol=1e-13)
    assert not vx[0].any() and not vt[:, 0].any()        # only edges the gradient reaches


@pytest.mark.parametrize("nr,nt,dx,dt,seed", [(4, 5, 0.3, 0.1, 1), (8, 8, 0.2, 0.7, 3),
                                               (7, 5, 0.05, 0.08, 6)])
def test_bounds_bracket_the_kantorovich_lp(oracle_mod, nr, nt, dx, dt, seed):
    g = random_small_pair(nr, nt, seed, dx=dx, dt=dt)
    s, _, _, _ = oracle_mod.decompose(g.pcal, g.pobs, g.dx, g.dt)
    lp = kantorovich_lp(s, g.dx, g.dt, oracle_mod.cell_measure(nr, nt, g.dx, g.dt))
    # early in a solve the bracket is wide but valid; after a long fixed budget at
    # eps = 0 (the unregularised problem, whose optimum the LP is) it closes
    r = oracle_mod.solve(s, g.dx, g.dt, oracle_mod.Params(tol_res=1e-6, max_iter=200000))
    lo, w, hi = transport_bounds(s, r.ux, r.ut, r.phi, g.dx, g.dt)
    assert lo <= lp * (1 + 1e-12) and lp <= hi * (1 + 1e-12)
    r = oracle_mod.solve(s, g.dx, g.dt, FIXED_BUDGET(eps=0.0))
    lo, w, hi = transport_bounds(s, r.ux, r.ut, r.phi, g.dx, g.dt)
    assert lo <= lp * (1 + 1e-12) and lp <= hi * (1 + 1e-12)
    assert hi - lo <= 1e-8 * lp


def test_bounds_bracket_the_1d_closed_form(oracle_mod):
    g = config1_pairs([90])[0]
    s, _, _, _ = oracle_mod.decompose(g.pcal, g.pobs, g.dx, g.dt)
    _, W, _ = closed_form_1d(s, g.dt, 1e-4)
    r = oracle_mod.solve(s, g.dx, g.dt, oracle_mod.Params(tol_res=1e-6, max_iter=400000))
    lo, w, hi = transport_bounds(s, r.ux, r.ut, r.phi, g.dx, g.dt)
    assert lo <= W * (1 + 1e-12) <= hi * (1 + 2e-12)
    # the flux is fixed by the source in 1D and converges first; the potential lags
    # (it is pinned only on the flux support), which leaves the lower side looser
    assert hi - W <= 1e-4 * W
    assert W - lo <= 2e-3 * W


def test_oracle_optimum_certified_on_a_40x400_gather(oracle_mod):
    # 16,000 cells: far past the LP, the solve to a 1e-6 residual is within 2e-5 of
    # the certified bracket, and the reported transport lies inside it
    g = config2_gather(nr=40, nt=400, f_peak=6.0, dtype=np.float64)
    s, _, _, _ = oracle_mod.decompose(g.pcal, g.pobs, g.dx, g.dt)
    r = oracle_mod.solve(s, g.dx, g.dt, oracle_mod.Params(tol_res=1e-6, max_iter=400000))
    assert r.status == oracle_mod.CONVERGED
    lo, w, hi = transport_bounds(s, r.ux, r.ut, r.phi, g.dx, g.dt)
    assert w == pytest.approx(r.transport, rel=1e-12)
    assert lo <= r.transport <= hi
    assert (hi - lo) / hi <= 5e-5
    # a potential of the wrong sign collapses the lower bound; a flux that moves only
    # half the mass reports a transport below it
    lo_neg, _, _ = transport_bounds(s, r.ux, r.ut, -r.phi, g.dx, g.dt)
    assert lo_neg < 0.5 * lo
    _, w_half, _ = transport_bounds(s, 0.5 * r.ux, 0.5 * r.ut, r.phi, g.dx, g.dt)
    assert w_half < 0.6 * lo



@pytest.mark.parametrize("axis", [0, 1])
def test_reflection_maps_the_iteration_onto_itself(oracle_mod, axis):
    # With div = -grad^T, reversing a gather along either axis maps the discrete
    # problem onto itself (the flux changes sign and moves to the mirrored edge, the
    # potential is mirrored), so Algorithm 1 takes the same steps and reaches the same
    # transport, up to the order of the sums.  The boundary rows of the divergence as
    # printed would break this symmetry.
    g = random_small_pair(16, 120, 31)
    out = []
    for pc, po in ((g.pcal, g.pobs), (np.flip(g.pcal, axis).copy(), np.flip(g.pobs, axis).copy())):
        s, _, _, _ = oracle_mod.decompose(pc, po, g.dx, g.dt)
        r = oracle_mod.solve(s, g.dx, g.dt, oracle_mod.Params(tol_res=1e-6, max_iter=400000))
        assert r.status == oracle_mod.CONVERGED
        out.append((r, transport_bounds(s, r.ux, r.ut, r.phi, g.dx, g.dt)))
    (r0, (lo0, w0, hi0)), (r1, (lo1, w1, hi1)) = out
    assert r1.iters == r0.iters and r1.ls_trials == r0.ls_trials
    assert r1.transport == pytest.approx(r0.transport, rel=1e-10)
    assert max(lo0, lo1) <= min(hi0, hi1)              # and the brackets agree
    np.testing.assert_allclose(np.flip(r1.phi, axis), r0.phi, rtol=0,
                               atol=1e-9 * np.abs(r0.phi).max())


def test_transport_is_homogeneous_in_the_data_at_zero_eps(oracle_mod):
    # W1(c s) = c W1(s): at eps = 0 the optimum scales with the data (the iteration
    # does not: the shrink threshold is alpha whatever the scale)
    g = config2_gather(nr=16, nt=120, f_peak=4.0, dtype=np.float64)
    s, _, _, _ = oracle_mod.decompose(g.pcal, g.pobs, g.dx, g.dt)
    vals = []
    for c in (1.0, 8.0):
        r = oracle_mod.solve(c * s, g.dx, g.dt, oracle_mod.Params(eps=0.0, tol_res=1e-6, max_iter=400000))
        assert r.status == oracle_mod.CONVERGED
        lo, w, hi = transport_bounds(c * s, r.ux, r.ut, r.phi, g.dx, g.dt)
        assert lo <= w * (1 + 1e-12) and (hi - lo) / hi <= 2e-3
        vals.append(w / c)
    assert vals[1] == pytest.approx(vals[0], rel=2e-5)
