"""Residual history (the optional per-check record of the stop-rule residual,
Algorithm 1's stopping test in Section 2.2), through the C ABI: each recorded
residual against the oracle's residual after the same number of iterations, the
ring's wrap-around, the stop rule it documents, and that checkpoint/resume and the
autotuner keep it consistent."""
import dataclasses

import numpy as np
import pytest

import oracle
from gpu_util import log, make_plan, oracle_params
from synth import random_small_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU machines too
    pytest.skip("no GPU", allow_module_level=True)

import paper_1808_07284_amd as E  # noqa: E402


def small_batch(dtype):
    gs = [random_small_pair(13, 301, 1), random_small_pair(5, 9, 2), random_small_pair(3, 250, 4)]
    z = gs[1]
    gs.append(type(z)(z.pcal.copy(), z.pcal.copy(), z.dx, z.dt, "zero source"))
    return [type(g)(g.pcal.astype(dtype), g.pobs.astype(dtype), g.dx, g.dt, g.label) for g in gs]


def _solve(plan, pcal, pobs):
    s, mass = E.emd_decompose(plan, pcal, pobs)
    emd, phi, _, info = E.emd_pdhg_solve(plan, s, mass=mass)
    torch.cuda.synchronize()
    return E.info_numpy(info)


@pytest.mark.parametrize("ls", [E.LS_L2, E.LS_L1])
def test_history_matches_the_oracle_at_every_check(ls):
    # FP64: the residual recorded at check c is the oracle's relative residual after
    # c * check_every iterations (the same decisions, reductions in another order)
    gs = small_batch(np.float64)
    ce, checks = 10, 12
    p = E.SolverParams(precision=E.F64, max_iter=ce * checks, tol_res=0.0, check_every=ce, ls_mode=ls)
    plan, pcal, pobs, desc = make_plan(gs, p)
    buf = plan.set_history(checks)
    info = _solve(plan, pcal, pobs)
    hist = E.residual_history(plan, info)
    h = buf.cpu().numpy()
    for k, g in enumerate(gs):
        if g.label == "zero source":
            assert info["status"][k] == E.GATHER_STATUS.index("ZERO_SOURCE")
            assert hist[k].size == 0 and np.isnan(h[k]).all()  # never iterated: nothing written
            continue
        assert info["iters"][k] == ce * checks and hist[k].size == checks
        s, _, _, _ = oracle.decompose(g.pcal, g.pobs, g.dx, g.dt)
        ref = [oracle.solve(s, g.dx, g.dt, oracle_params(p, max_iter=ce * c, check_every=ce)).rel_res
               for c in range(1, checks + 1)]
        log(f"  ls={ls} gather {k} {g.label}: gpu {hist[k][[0, -1]]} oracle {np.array(ref)[[0, -1]]}")
        np.testing.assert_allclose(hist[k], ref, rtol=1e-7)
        # the last check is the solve's final residual (the same double)
        assert hist[k][-1] == info["rel_res"][k]
    plan.close()


def test_ring_keeps_the_last_checks_and_the_stop_rule():
    gs = small_batch(np.float32)
    ce, checks = 10, 12
    p = E.SolverParams(precision=E.F32, max_iter=ce * checks, tol_res=0.0, check_every=ce)
    plan, pcal, pobs, desc = make_plan(gs, p)
    plan.set_history(checks)
    full = E.residual_history(plan, _solve(plan, pcal, pobs))
    plan.set_history(5)
    info = _solve(plan, pcal, pobs)
    last = E.residual_history(plan, info)
    for k in range(len(gs)):
        np.testing.assert_array_equal(last[k], full[k][-5:])  # solves are bitwise repeatable
    # free-running to the stop rule: a gather stops at its first check at or below tol
    tol = 1e-3
    plan.set_params(dataclasses.replace(p, tol_res=tol, max_iter=100000))
    plan.set_history(100000 // ce)
    info = _solve(plan, pcal, pobs)
    hist = E.residual_history(plan, info)
    for k, g in enumerate(gs):
        if info["status"][k] != E.GATHER_STATUS.index("CONVERGED"):
            continue
        log(f"  gather {k} {g.label}: {info['iters'][k]} iterations, {hist[k].size} checks, "
            f"last {hist[k][-3:]}")
        assert hist[k].size == info["iters"][k] // ce
        assert hist[k][-1] <= tol and (hist[k][:-1] > tol).all()
    assert (info["status"][:3] == E.GATHER_STATUS.index("CONVERGED")).all()
    plan.set_history(0)
    with pytest.raises(RuntimeError):
        E.residual_history(plan, info)
    plan.close()


def test_history_through_autotune_and_resume():
    gs = small_batch(np.float32)
    ce, K = 10, 60
    p2 = E.SolverParams(precision=E.F32, max_iter=2 * K, tol_res=0.0, check_every=ce)
    p1 = dataclasses.replace(p2, max_iter=K)
    plan, pcal, pobs, desc = make_plan(gs, p2)
    s, mass = E.emd_decompose(plan, pcal, pobs)
    buf = plan.set_history(2 * K // ce)
    plan.autotune(s, sweeps=8)
    torch.cuda.synchronize()
    assert np.isnan(buf.cpu().numpy()).all()  # the timing solves record nothing
    _, _, _, i_ref = E.emd_pdhg_solve(plan, s, mass=mass)
    ref = E.residual_history(plan, i_ref)
    # K iterations, checkpoint, resume to 2K: the same history as one solve of 2K
    plan.set_history(2 * K // ce)
    plan.set_params(p1)
    u = plan.empty(2)
    _, phi, _, _ = E.emd_pdhg_solve(plan, s, u=u, mass=mass)
    state = E.solver_state(plan)
    plan.set_params(p2)
    _, phi, u, i2 = E.emd_pdhg_solve_resume(plan, s, state, u, phi, mass=mass)
    torch.cuda.synchronize()
    got = E.residual_history(plan, i2)
    for k in range(len(gs)):
        np.testing.assert_array_equal(got[k], ref[k])
    assert all(got[k].size == 2 * K // ce for k in range(3))
    plan.close()
