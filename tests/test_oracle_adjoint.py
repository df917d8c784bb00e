"""Pins of the oracle's adjoint source (Section 2.3 of the paper: the derivative of
the misfit with respect to Pcal is the dual potential phi), chained through the
mass normalisation.  The reference is the derivative of the exact 1D optimum
(differentiable away from the zeros of the cumulative source), taken by central
finite differences, so a wrong sign, a missing mean removal or a wrong unit-mass
chain term in the oracle fails it."""
import numpy as np
import pytest

from synth import config1_pairs


def exact_emd_1d(pcal, pobs, dt, eps, mode):
    """Exact misfit of a single trace after the chosen normalisation (Section 2.1)."""
    pcal = np.asarray(pcal, np.float64).reshape(-1)
    pobs = np.asarray(pobs, np.float64).reshape(-1)
    if mode == "balance":
        s = (pcal - pobs) - (pcal - pobs).mean()
    elif mode == "unit":
        f = np.maximum(pcal, 0) + np.maximum(-pobs, 0)
        g = np.maximum(pobs, 0) + np.maximum(-pcal, 0)
        s = f / (dt * f.sum()) - g / (dt * g.sum())
    else:
        s = pcal - pobs
    S = np.cumsum(s)[:-1]
    return dt * dt * np.abs(S).sum() + 0.5 * eps * dt ** 3 * (S * S).sum()


def _smooth_pair(nt):
    # two positive traces whose mass sits left (Pcal) and right (Pobs): the
    # cumulative source never vanishes inside the trace, so the exact misfit is
    # differentiable there and the potential is unique up to a constant
    t = np.linspace(0.0, 1.0, nt)
    pcal = 0.3 + np.exp(-((t - 0.3) / 0.12) ** 2) + 0.2 * np.sin(7 * t) ** 2
    pobs = 0.3 + np.exp(-((t - 0.7) / 0.12) ** 2) + 0.2 * np.sin(7 * (1 - t)) ** 2
    pobs *= pcal.sum() / pobs.sum()
    return pcal[None, :], pobs[None, :], 1.0 / (nt - 1)


@pytest.mark.parametrize("mode,mm", [("balance", 0), ("unit", 1), ("none", 2)])
def test_adjoint_matches_derivative_of_exact_optimum(oracle_mod, mode, mm):
    pcal, pobs, dt = _smooth_pair(80)
    p = oracle_mod.Params(tol_res=1e-9, max_iter=3000000, mass_tol=1e-9)
    r, mass = oracle_mod.misfit(pcal, pobs, 1.0, dt, mass_mode=mm, params=p)
    assert r.status == oracle_mod.CONVERGED
    assert r.emd == pytest.approx(exact_emd_1d(pcal, pobs, dt, 1e-4, mode), rel=1e-7)
    psi = oracle_mod.adjoint(r.phi, pcal, pobs, mass, 1.0, dt, mass_mode=mm)[0]
    rng = np.random.default_rng(5)
    h = 1e-7
    for _ in range(4):
        d = rng.normal(size=pcal.shape[1])
        if mode == "none":
            d -= d.mean()  # stay on the balanced set where the problem is feasible
        fp = exact_emd_1d(pcal[0] + h * d, pobs[0], dt, 1e-4, mode)
        fm = exact_emd_1d(pcal[0] - h * d, pobs[0], dt, 1e-4, mode)
        fd = (fp - fm) / (2 * h)
        assert float(psi @ d) == pytest.approx(fd, rel=2e-4, abs=1e-9)


def test_adjoint_of_shifted_ricker_pair(oracle_mod):
    # the 1D shift study (Section 3.1): where the cumulative source is bounded away
    # from zero the adjoint agrees with the derivative of the exact optimum; where it
    # vanishes the misfit has a kink and the potential is not unique there
    g = config1_pairs([40], nt=120, dt=1.0 / 119, centre=0.45)[0]
    r, mass = oracle_mod.misfit(g.pcal, g.pobs, g.dx, g.dt,
                                params=oracle_mod.Params(tol_res=1e-8, max_iter=3000000))
    assert r.status == oracle_mod.CONVERGED
    psi = oracle_mod.adjoint(r.phi, g.pcal, g.pobs, mass, g.dx, g.dt)[0]
    s = (g.pcal[0] - g.pobs[0]) - (g.pcal[0] - g.pobs[0]).mean()
    S = np.cumsum(s)[:-1]
    # potential differences on the flux support: dt sign(u)(1 + eps|u|), u = -dt S
    sup = np.abs(S) > 1e-3 * np.abs(S).max()
    expect = g.dt * np.sign(-S[sup]) * (1 + 1e-4 * g.dt * np.abs(S[sup]))
    np.testing.assert_allclose(np.diff(r.phi[0])[sup], expect, rtol=1e-4)
    # the adjoint is envelope-like (Section 3.1): one sign change per lobe boundary
    assert abs(psi.sum()) <= 1e-12 * np.abs(psi).sum()


def test_adjoint_scaling_and_modes(oracle_mod):
    rng = np.random.default_rng(2)
    nr, nt, dx, dt = 3, 5, 0.5, 0.25
    phi = rng.normal(size=(nr, nt))
    pc = rng.normal(size=(nr, nt))
    po = rng.normal(size=(nr, nt))
    _, _, _, mass = oracle_mod.decompose(pc, po, dx, dt)
    b = oracle_mod.adjoint(phi, pc, po, mass, dx, dt, oracle_mod.MASS_BALANCE, gbar=2.0)
    # balance: the adjoint is orthogonal to constants (a uniform change of Pcal is
    # removed by the balancing), and linear in the upstream gradient
    assert abs(b.sum()) <= 1e-12 * np.abs(b).sum()
    b1 = oracle_mod.adjoint(phi, pc, po, mass, dx, dt, oracle_mod.MASS_BALANCE, gbar=1.0)
    np.testing.assert_allclose(b, 2.0 * b1, rtol=1e-14)
    # adding a constant to phi changes nothing in balance mode (phi is defined up to
    # a constant)
    b2 = oracle_mod.adjoint(phi + 3.0, pc, po, mass, dx, dt, oracle_mod.MASS_BALANCE)
    np.testing.assert_allclose(b2, b1, atol=1e-13)
    n = oracle_mod.adjoint(phi, pc, po, mass, dx, dt, oracle_mod.MASS_NONE)
    np.testing.assert_allclose(n, dx * dt * phi, rtol=1e-14)
    # unit: invariant to adding a constant to phi as well (both sides carry unit mass)
    u1 = oracle_mod.adjoint(phi, pc, po, mass, dx, dt, oracle_mod.MASS_UNIT)
    u2 = oracle_mod.adjoint(phi + 3.0, pc, po, mass, dx, dt, oracle_mod.MASS_UNIT)
    np.testing.assert_allclose(u2, u1, atol=1e-12)
