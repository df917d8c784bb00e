"""Plain PDHG with fixed steps, two iterations per sweep (iters_per_sweep = 2): one
HBM pass per two iterations of the primal and dual updates of Section 2.2.

* against the one-iteration sweep with the same fixed steps: the fields are computed
  with the same operands and operations, so they must be bitwise equal, for any
  iteration count (odd counts end with a single-iteration sweep) and any tiling;
* against the oracle's plain PDHG (FP64): identical statuses and iteration counts,
  EMD and fields to 1e-9;
* checkpoint/resume mixes the two forms: a one-iteration solve to an odd count
  resumed by the two-iteration form equals the one-iteration solve to the end.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from gpu_util import log, make_plan, oracle_params, rel_l2, to_precision, unpack
from synth import config1_pairs, config2_gather, config3_batch, random_small_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1808_07284_amd as E  # noqa: E402


def _batch(dtype):
    gs = [config2_gather(nr=40, nt=530, f_peak=3.0, dtype=np.float64), random_small_pair(13, 301, 1),
          random_small_pair(5, 9, 2), config1_pairs([60], nt=257, dt=1.0 / 256)[0],
          random_small_pair(7, 1, 3), random_small_pair(3, 250, 4), random_small_pair(2, 700, 8)]
    return to_precision(gs, dtype)


def _run(plan, s, mass, **kw):
    u = plan.empty(2)
    emd, phi, u, info = E.emd_pdhg_solve(plan, s, u=u, mass=mass, **kw)
    torch.cuda.synchronize()
    return emd.cpu().numpy(), phi.cpu().numpy(), u.cpu().numpy(), E.info_numpy(info)


@pytest.mark.parametrize("precision,ips,K", [(E.F32, 2, 300), (E.F32, 2, 301), (E.F64, 2, 300), (E.F64, 2, 301),
                                             (E.F32, 3, 300), (E.F32, 3, 301), (E.F32, 3, 302)])
def test_two_iterations_per_sweep_equal_one_iteration_per_sweep(precision, ips, K):
    # ips iterations per sweep (2, or 3 in FP32); a count that is not a multiple of ips
    # ends with a shorter sweep
    dtype = np.float64 if precision == E.F64 else np.float32
    gs = _batch(dtype)
    ce = ips * (K // ips + 1)  # a multiple of ips past K: no stop-rule check
    p1 = E.SolverParams(precision=precision, ls_mode=E.LS_FIXED, max_iter=K, tol_res=0.0, check_every=ce)
    p2 = dataclasses.replace(p1, iters_per_sweep=ips)
    out = {}
    s = None
    for rows in (16, 1, 3):
        for tag, p in (("one", p1), ("two", p2)):
            plan, pcal, pobs, desc = make_plan(gs, p, rows=rows)
            if s is None:
                # one source for every tiling: the decompose's FP64 sums are taken per
                # tile, so in FP64 the mean it removes differs in the last bit
                s, mass = E.emd_decompose(plan, pcal, pobs)
            out[tag, rows] = _run(plan, s, mass)
            out[tag, rows, "sweeps"] = plan.query()["last_sweeps"]
            plan.close()
    ref = out["one", 16]
    log(f"  precision={precision} ips={ips} K={K}: sweeps one/multi {out['one', 16, 'sweeps']}/"
        f"{out['two', 16, 'sweeps']}")
    for rows in (16, 1, 3):
        emd, phi, u, info = out["two", rows]
        # the multi-iteration sweeps form every row with the calls and operands of
        # the one-iteration sweep (the two-iteration one marching even strips down
        # and odd strips up): any tiling gives its bits, which are those of the
        # one-iteration sweep
        np.testing.assert_array_equal(phi, ref[1], err_msg=f"two, rows {rows}")
        np.testing.assert_array_equal(u, ref[2], err_msg=f"two, rows {rows}")
        np.testing.assert_array_equal(info["iters"], ref[3]["iters"])
        np.testing.assert_array_equal(info["status"], ref[3]["status"])
        # the sums are taken in another order, and the two-iteration sweep forms the
        # final residual directly (the one-iteration sweep from the previous residual
        # plus the divergence of the flux change)
        np.testing.assert_allclose(emd, ref[0], rtol=1e-13 if precision == E.F64 else 1e-6)
        np.testing.assert_allclose(info["rel_res"], ref[3]["rel_res"], rtol=1e-9 if precision == E.F64 else 2e-3)
        # and the one-iteration sweep gives the same bits under every tiling
        np.testing.assert_array_equal(out["one", rows][1], ref[1])
        np.testing.assert_array_equal(out["one", rows][2], ref[2])
    # about 1/ips as many sweeps (each solve rounds its sweeps up to whole chunks)
    assert out["two", 16, "sweeps"] <= out["one", 16, "sweeps"] // ips + 4


@pytest.mark.parametrize("tol", [0.0, 1e-4])
def test_two_iterations_per_sweep_match_the_oracle(tol):
    # (three iterations per sweep run in FP32 only; they are held to the one-iteration
    # sweep bitwise above, which is held to the oracle in the parity tests)
    gs = _batch(np.float64)
    K = 300 if tol == 0.0 else 20000
    p = E.SolverParams(precision=E.F64, ls_mode=E.LS_FIXED, iters_per_sweep=2, max_iter=K, tol_res=tol,
                       check_every=K if tol == 0.0 else 10)
    plan, pcal, pobs, desc = make_plan(gs, p, rows=8)
    s, mass = E.emd_decompose(plan, pcal, pobs)
    emd, phi, u, info = _run(plan, s, mass)
    phis, us = unpack(phi, desc), unpack(u, desc, 2)
    for k, g in enumerate(gs):
        so, _, _, _ = oracle.decompose(g.pcal, g.pobs, g.dx, g.dt)
        r = oracle.solve(so, g.dx, g.dt, oracle_params(p))
        log(f"  gather {k} {g.label}: gpu {info[k]['status']} {info[k]['iters']} {emd[k]:.12e}  "
            f"oracle {r.status} {r.iters} {r.emd:.12e}")
        assert info[k]["status"] == r.status
        assert info[k]["iters"] == r.iters
        if r.status == oracle.ZERO_SOURCE:
            continue
        assert emd[k] == pytest.approx(r.emd, rel=1e-9)
        assert info[k]["rel_res"] == pytest.approx(r.rel_res, rel=1e-7)
        assert rel_l2(phis[k], r.phi) <= 1e-9
        un = np.sqrt(np.sum(r.ux ** 2) + np.sum(r.ut ** 2))
        assert np.linalg.norm(us[k][0] - r.ux) <= 1e-9 * un
        assert np.linalg.norm(us[k][1] - r.ut) <= 1e-9 * un
    if tol > 0:
        assert (info["status"] == E.GATHER_STATUS.index("CONVERGED")).sum() >= 3
    plan.close()


@pytest.mark.parametrize("ips", [2, 3])
def test_resume_from_an_odd_count_with_two_iterations_per_sweep(ips):
    # 151 iterations one per sweep, then ips per sweep to 400: the first resumed sweep
    # realigns the count, the last one ends at 400
    gs = _batch(np.float32)
    K1, K2 = 151, 400
    p1 = E.SolverParams(precision=E.F32, ls_mode=E.LS_FIXED, max_iter=K2, tol_res=0.0, check_every=K2)
    plan, pcal, pobs, desc = make_plan(gs, p1)
    s, mass = E.emd_decompose(plan, pcal, pobs)
    ref = _run(plan, s, mass)
    plan.set_params(dataclasses.replace(p1, max_iter=K1, check_every=K1))
    u = plan.empty(2)
    _, phi, u, _ = E.emd_pdhg_solve(plan, s, u=u, mass=mass)
    state = E.solver_state(plan)
    plan.set_params(dataclasses.replace(p1, iters_per_sweep=ips, check_every=ips * (K2 // ips + 1)))
    emd, phi, u, info = E.emd_pdhg_solve_resume(plan, s, state, u, phi, mass=mass)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(phi.cpu().numpy(), ref[1])
    np.testing.assert_array_equal(u.cpu().numpy(), ref[2])
    np.testing.assert_array_equal(E.info_numpy(info)["iters"], ref[3]["iters"])
    plan.close()


def test_two_iterations_per_sweep_on_the_benchmark_batch():
    # full size: 40 iterations of the 64-gather batch, bitwise the fields of the
    # one-iteration sweep, two per sweep on the default tiles and three per sweep on
    # the benchmark's 24-row tiles (40 = 13 x 3 + 1: the last sweep runs one)
    gs = config3_batch()
    p1 = E.SolverParams(precision=E.F32, ls_mode=E.LS_FIXED, max_iter=40, tol_res=0.0, check_every=42)
    res = []
    s = None
    for p, rows in ((p1, 0), (dataclasses.replace(p1, iters_per_sweep=2), 0),
                    (dataclasses.replace(p1, iters_per_sweep=3), 24)):
        plan, pcal, pobs, desc = make_plan(gs, p)
        if rows:
            plan.set_tiling(rows)
        if s is None:
            # one source for every tiling (the decompose's FP64 sums are taken per tile)
            s, mass = E.emd_decompose(plan, pcal, pobs)
        res.append(_run(plan, s, mass))
        plan.close()
        del pcal, pobs
    for r in res[1:]:
        np.testing.assert_array_equal(r[1], res[0][1])
        np.testing.assert_array_equal(r[2], res[0][2])
        np.testing.assert_allclose(r[0], res[0][0], rtol=1e-6)


def test_two_iterations_per_sweep_rejected_with_a_linesearch():
    gs = _batch(np.float32)[:2]
    with pytest.raises(E.EMDError):
        make_plan(gs, E.SolverParams(iters_per_sweep=2))
    with pytest.raises(E.EMDError):
        make_plan(gs, E.SolverParams(ls_mode=E.LS_FIXED, iters_per_sweep=2, check_every=5))
