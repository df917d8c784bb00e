"""Pins of the oracle's grid transfer for the multi-grid strategy (the closing remark
of Section 2.2; Section 3.3 resamples each shot and interpolates the solution back):
block-mean restriction and bilinear prolongation on the staggered grid.

Fixed independently of the oracle: restriction conserves the sum of a field over
every whole block and keeps constants; prolongation keeps constants, is the
identity for unit factors, reproduces linear fields at every fine point whose
coarse coordinate is inside the coarse grid (at the staggering of each field), puts
zero flux on the boundary edges; and a warm start from a coarse solution does not
change the optimum the fine solve reaches.
"""
import numpy as np
import pytest

from synth import config2_gather, random_small_pair


def test_restriction_block_means(oracle_mod):
    rng = np.random.default_rng(3)
    f = rng.normal(size=(12, 30))
    c = oracle_mod.restrict(f, 3, 5)
    assert c.shape == (4, 6)
    # every block is whole: the coarse sum times the block size is the fine sum
    assert c.sum() * 15 == pytest.approx(f.sum(), rel=1e-13, abs=1e-12)
    np.testing.assert_allclose(c, f.reshape(4, 3, 6, 5).mean(axis=(1, 3)), rtol=1e-14, atol=1e-15)
    # ragged last blocks average what they hold
    g = rng.normal(size=(7, 11))
    cg = oracle_mod.restrict(g, 3, 4)
    assert cg.shape == (3, 3)
    assert cg[2, 2] == pytest.approx(g[6, 8:].mean(), rel=1e-14)
    assert cg[0, 2] == pytest.approx(g[0:3, 8:].mean(), rel=1e-14)
    np.testing.assert_array_equal(oracle_mod.restrict(np.full((7, 11), 2.5), 3, 4), np.full((3, 3), 2.5))
    np.testing.assert_array_equal(oracle_mod.restrict(g, 1, 1), g)


def test_prolongation_identity_and_constants(oracle_mod):
    rng = np.random.default_rng(4)
    ux, ut, ph = rng.normal(size=(3, 6, 9))
    fx, ftm, fp = oracle_mod.prolong(ux, ut, ph, 6, 9, 1, 1)
    np.testing.assert_array_equal(fp, ph)
    # unit factors: every interior edge keeps its value; the edges before the first
    # receiver and the first sample are boundary edges and carry no flux
    np.testing.assert_array_equal(fx[1:], ux[1:])
    np.testing.assert_array_equal(ftm[:, 1:], ut[:, 1:])
    assert not fx[0].any() and not ftm[:, 0].any()
    one = np.ones((3, 4))
    _, _, p1 = oracle_mod.prolong(one, one, 3.0 * one, 7, 13, 3, 4)
    np.testing.assert_allclose(p1, 3.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("fr,ft", [(2, 4), (3, 2), (1, 4)])
def test_prolongation_reproduces_linear_fields(oracle_mod, fr, ft):
    nrc, ntc = 6, 7
    nr, nt = nrc * fr, ntc * ft
    I, J = np.meshgrid(np.arange(nrc), np.arange(ntc), indexing="ij")
    i, j = np.meshgrid(np.arange(nr), np.arange(nt), indexing="ij")
    a, b, c0 = 0.7, -0.3, 2.0
    # phi at cell centres: fine point (i, j) sits at ((i - (fr-1)/2)/fr, (j - (ft-1)/2)/ft)
    xr, xt = (i - 0.5 * (fr - 1)) / fr, (j - 0.5 * (ft - 1)) / ft
    inside = (xr >= 0) & (xr <= nrc - 1) & (xt >= 0) & (xt <= ntc - 1)
    # u^x on receiver edges (edge I at coordinate I; the boundary edges 0 and nrc
    # carry zero flux, so only coordinates in [1, nrc - 1] see the linear field)
    ux_c = a * I + b * J + c0
    ex = i / fr
    in_x = (ex >= 1) & (ex <= nrc - 1) & (xt >= 0) & (xt <= ntc - 1)
    ut_c = a * I + b * J + c0
    et = j / ft
    in_t = (xr >= 0) & (xr <= nrc - 1) & (et >= 1) & (et <= ntc - 1)
    fx, ftm, fp = oracle_mod.prolong(ux_c, ut_c, a * I + b * J + c0, nr, nt, fr, ft)
    np.testing.assert_allclose(fp[inside], (a * xr + b * xt + c0)[inside], rtol=0, atol=1e-13)
    np.testing.assert_allclose(fx[in_x], (a * ex + b * xt + c0)[in_x], rtol=0, atol=1e-13)
    np.testing.assert_allclose(ftm[in_t], (a * xr + b * et + c0)[in_t], rtol=0, atol=1e-13)
    # the flux fades to zero at the boundary edges
    assert not fx[0].any() and not ftm[:, 0].any()
    assert inside.sum() > 0.5 * nr * nt or fr == 1 or ft == 1


def test_coarse_warm_start_keeps_the_optimum(oracle_mod):
    # the coarse solution only changes where the fine iteration starts: the fine
    # solve reaches the same EMD as from a cold start
    g = config2_gather(nr=24, nt=240, f_peak=4.0, dtype=np.float64)
    fr, ft = 1, 4
    s, _, _, _ = oracle_mod.decompose(g.pcal, g.pobs, g.dx, g.dt)
    pc_c, po_c = oracle_mod.restrict(g.pcal, fr, ft), oracle_mod.restrict(g.pobs, fr, ft)
    s_c, _, _, _ = oracle_mod.decompose(pc_c, po_c, g.dx * fr, g.dt * ft)
    p = oracle_mod.Params(tol_res=1e-6, max_iter=400000)
    rc = oracle_mod.solve(s_c, g.dx * fr, g.dt * ft, p)
    assert rc.status == oracle_mod.CONVERGED
    ux, ut, ph = oracle_mod.prolong(rc.ux, rc.ut, rc.phi, g.nr, g.nt, fr, ft)
    cold = oracle_mod.solve(s, g.dx, g.dt, p)
    warm = oracle_mod.solve(s, g.dx, g.dt, p, u0=(ux, ut), phi0=ph)
    assert cold.status == warm.status == oracle_mod.CONVERGED
    assert warm.emd == pytest.approx(cold.emd, rel=1e-5)
    # and the coarse EMD already approximates the fine one (same grid scale)
    assert rc.emd == pytest.approx(cold.emd, rel=0.1)


def test_transfer_of_a_single_trace(oracle_mod):
    # nr = 1: no receiver edges, so u^x stays zero; time keeps its staggering
    g = random_small_pair(1, 40, 9)
    c = oracle_mod.restrict(g.pcal, 1, 4)
    assert c.shape == (1, 10)
    ux, ut, ph = oracle_mod.prolong(np.ones((1, 10)), np.ones((1, 10)), np.ones((1, 10)), 1, 40, 1, 4)
    assert not ux.any()
    np.testing.assert_allclose(ph, 1.0, rtol=0, atol=1e-15)
    assert ut[0, 0] == 0.0 and ut[0, 4] == 1.0
