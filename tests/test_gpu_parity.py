"""GPU parity: the HIP library, called through its C ABI, against the FP64 oracle on
the same seeded inputs.

Tolerances:
* FP64 path: the same algorithm in the same precision, reductions in another
  order -> EMD and fields within 1e-9 (relative), identical iteration and
  backtracking counts.
* FP32 path: relative EMD error <= 1e-5 and mean-removed relative L2 error of phi
  <= 1e-4 against the FP64 oracle, both with the oracle's step schedule replayed
  (arithmetic parity) and free-running to the stop rule (accuracy parity).
* decompose / adjoint on identical inputs: FP32 within a few ulps (1e-6 relative),
  FP64 within 1e-12.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from gpu_util import centred, log, make_plan, oracle_params, rel_l2, to_precision, unpack
from synth import config1_pairs, config2_gather, random_small_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU machines too
    pytest.skip("no GPU", allow_module_level=True)

import paper_1808_07284_amd as E  # noqa: E402


def ragged_batch(dtype):
    """Gathers spanning several tiles in both directions plus ragged and degenerate
    shapes: 1 receiver, 1 sample, fewer rows than a tile, nt not a multiple of 4."""
    gs = [
        config2_gather(nr=40, nt=530, f_peak=3.0, dtype=np.float64),   # 3 time tiles, 5 strips
        random_small_pair(13, 301, 1),
        random_small_pair(5, 9, 2),
        config1_pairs([60], nt=257, dt=1.0 / 256)[0],                   # single trace
        random_small_pair(7, 1, 3),                                     # single sample per trace
        random_small_pair(3, 250, 4),
    ]
    return to_precision(gs, dtype)


def oracle_batch(gathers, op, mass_mode=oracle.MASS_BALANCE, trace=False):
    res = []
    for g in gathers:
        s, _, _, mass = oracle.decompose(g.pcal, g.pobs, g.dx, g.dt, mass_mode)
        r = oracle.solve(s, g.dx, g.dt, op, trace=trace)
        res.append((r, mass))
    return res


@pytest.mark.parametrize("precision", [E.F32, E.F64])
@pytest.mark.parametrize("mode", [E.MASS_BALANCE, E.MASS_UNIT, E.MASS_NONE])
def test_decompose_matches_oracle(precision, mode):
    dtype = np.float64 if precision == E.F64 else np.float32
    gs = ragged_batch(dtype)
    p = E.SolverParams(precision=precision, mass_mode=mode)
    log(f"decompose precision={precision} mode={mode}")
    plan, pcal, pobs, desc = make_plan(gs, p, rows=8)
    f = plan.empty()
    g = plan.empty()
    s, mass = E.emd_decompose(plan, pcal, pobs, f_out=f, g_out=g)
    torch.cuda.synchronize()
    s_h, f_h, g_h = (unpack(t.cpu().numpy(), desc) for t in (s, f, g))
    mass_h = mass.cpu().numpy()
    tol = 1e-12 if precision == E.F64 else 1e-6
    for k, gg in enumerate(gs):
        so, fo, go, mo = oracle.decompose(gg.pcal, gg.pobs, gg.dx, gg.dt, mode)
        np.testing.assert_allclose(mass_h[k][:2], mo[:2], rtol=tol, atol=1e-300)
        # the mean of Pcal - Pobs cancels: bound its error by the size of the terms
        dscale = np.abs(gg.pcal.astype(np.float64) - gg.pobs).mean()
        assert abs(mass_h[k][2] - mo[2]) <= 1e-13 * dscale
        scale = np.abs(so).max() if np.abs(so).max() > 0 else 1.0
        np.testing.assert_allclose(s_h[k], so, rtol=0, atol=tol * scale * 4)
        np.testing.assert_allclose(f_h[k], fo, rtol=tol)
        np.testing.assert_allclose(g_h[k], go, rtol=tol)
    plan.close()


def _solve(plan, pcal, pobs, **kw):
    s, mass = E.emd_decompose(plan, pcal, pobs)
    u = plan.empty(2)
    emd, phi, u, info = E.emd_pdhg_solve(plan, s, u=u, mass=mass, **kw)
    torch.cuda.synchronize()
    return emd.cpu().numpy(), phi.cpu().numpy(), u.cpu().numpy(), E.info_numpy(info), mass


@pytest.mark.parametrize("rows,ls", [(8, E.LS_L2), (32, E.LS_L2), (8, E.LS_L1), (32, E.LS_L1)])
def test_f64_fixed_iterations_match_oracle(rows, ls):
    gs = ragged_batch(np.float64)
    p = E.SolverParams(precision=E.F64, max_iter=300, tol_res=0.0, check_every=300, ls_mode=ls)
    log(f"f64 fixed K=300 rows={rows} ls_mode={ls}")
    plan, pcal, pobs, desc = make_plan(gs, p, rows=rows)
    emd, phi, u, info, _ = _solve(plan, pcal, pobs)
    ref = oracle_batch(gs, oracle_params(p))
    phis = unpack(phi, desc)
    us = unpack(u, desc, 2)
    for k, (r, _) in enumerate(ref):
        log(f"  gather {k} {gs[k].label}: gpu {info[k]['status']} {info[k]['iters']} "
            f"{info[k]['ls_trials']} {emd[k]:.12e}  oracle {r.status} {r.iters} {r.ls_trials} {r.emd:.12e}")
        assert info[k]["status"] == r.status
        assert info[k]["iters"] == r.iters
        if r.status == oracle.ZERO_SOURCE:
            continue
        assert info[k]["ls_trials"] == r.ls_trials
        assert emd[k] == pytest.approx(r.emd, rel=1e-9)
        assert info[k]["rel_res"] == pytest.approx(r.rel_res, rel=1e-7)
        assert rel_l2(phis[k], r.phi) <= 1e-9
        assert rel_l2(us[k][0], r.ux) <= 1e-9 or np.abs(r.ux).max() == 0
        assert rel_l2(us[k][1], r.ut) <= 1e-9
    plan.close()


@pytest.mark.parametrize("rows,tol", [(8, 0.0), (32, 0.0), (16, 1e-4)])
def test_f64_fixed_step_pdhg_matches_oracle(rows, tol):
    # plain PDHG with the fixed steps alpha_1, beta_1 = delta alpha_1 and theta = 1
    # (the primal and dual updates of Section 2.2 before the linesearch): no
    # backtracking, so iterates, counts and the stop rule depend on the arithmetic only
    gs = ragged_batch(np.float64)
    K = 300 if tol == 0.0 else 20000
    p = E.SolverParams(precision=E.F64, max_iter=K, tol_res=tol, check_every=K if tol == 0.0 else 10,
                       ls_mode=E.LS_FIXED)
    log(f"f64 fixed step rows={rows} tol={tol} max_iter={K}")
    plan, pcal, pobs, desc = make_plan(gs, p, rows=rows)
    emd, phi, u, info, _ = _solve(plan, pcal, pobs)
    ref = oracle_batch(gs, oracle_params(p), trace=True)
    phis = unpack(phi, desc)
    us = unpack(u, desc, 2)
    for k, (r, _) in enumerate(ref):
        log(f"  gather {k} {gs[k].label}: gpu {info[k]['status']} {info[k]['iters']} {emd[k]:.12e}  "
            f"oracle {r.status} {r.iters} {r.emd:.12e}")
        assert info[k]["status"] == r.status
        assert info[k]["iters"] == r.iters
        if r.status == oracle.ZERO_SOURCE:
            continue
        assert info[k]["ls_trials"] == 0 and r.ls_trials == 0
        # every accepted step is alpha_1
        assert np.all(r.alpha_trace == r.alpha_trace[0]) and info[k]["alpha"] == r.alpha_trace[0]
        assert emd[k] == pytest.approx(r.emd, rel=1e-9)
        assert info[k]["rel_res"] == pytest.approx(r.rel_res, rel=1e-7)
        assert rel_l2(phis[k], r.phi) <= 1e-9
        assert rel_l2(us[k][0], r.ux) <= 1e-9 or np.abs(r.ux).max() == 0
        assert rel_l2(us[k][1], r.ut) <= 1e-9 or np.abs(r.ut).max() == 0
    if tol > 0:
        assert any(r.status == oracle.CONVERGED for r, _ in ref)
    plan.close()


def _warm_start_point(g, step=0.05, iters=150):
    """The oracle's iterate after `iters` iterations on a neighbouring problem: Pcal
    moved by `step` towards Pobs, as between two evaluations of an FWI loop."""
    pc = g.pcal.astype(np.float64) + step * (g.pobs.astype(np.float64) - g.pcal)
    s0, _, _, _ = oracle.decompose(pc, g.pobs, g.dx, g.dt)
    r0 = oracle.solve(s0, g.dx, g.dt, oracle.Params(max_iter=iters, tol_res=0.0, check_every=iters))
    return r0.ux, r0.ut, r0.phi


@pytest.mark.parametrize("ls,tol", [(E.LS_L2, 0.0), (E.LS_L1, 0.0), (E.LS_FIXED, 0.0), (E.LS_L2, 1e-5)])
def test_f64_warm_start_matches_oracle(ls, tol):
    # warm start (Section 3.3 evaluates the misfit three times per FWI iteration, each
    # time near the previous problem): the same start flux and potential go into the
    # library and into the oracle, and both must take the same steps from there
    gs = ragged_batch(np.float64)
    K = 300 if tol == 0.0 else 20000
    p = E.SolverParams(precision=E.F64, max_iter=K, tol_res=tol, check_every=K if tol == 0.0 else 10,
                       ls_mode=ls)
    log(f"f64 warm start ls_mode={ls} tol={tol}")
    plan, pcal, pobs, desc = make_plan(gs, p, rows=8)
    starts = [_warm_start_point(g) for g in gs]
    u0 = plan.empty(2)
    phi0 = plan.empty()
    n = plan.batch_len
    u0_h = np.zeros(2 * n)
    phi0_h = np.zeros(n)
    for (nr, nt, _, _, off), (ux, ut, ph) in zip(desc, starts):
        u0_h[off:off + nr * nt] = ux.reshape(-1)
        u0_h[n + off:n + off + nr * nt] = ut.reshape(-1)
        phi0_h[off:off + nr * nt] = ph.reshape(-1)
    u0.copy_(torch.from_numpy(u0_h.reshape(2, n)))
    phi0.copy_(torch.from_numpy(phi0_h))
    s, mass = E.emd_decompose(plan, pcal, pobs)
    emd, phi, u, info = E.emd_pdhg_solve(plan, s, phi=phi0, u=u0, warm_start=True, mass=mass)
    torch.cuda.synchronize()
    emd, info = emd.cpu().numpy(), E.info_numpy(info)
    phis, us = unpack(phi.cpu().numpy(), desc), unpack(u.cpu().numpy(), desc, 2)
    for k, g in enumerate(gs):
        so, _, _, _ = oracle.decompose(g.pcal, g.pobs, g.dx, g.dt)
        r = oracle.solve(so, g.dx, g.dt, oracle_params(p), u0=starts[k][:2], phi0=starts[k][2])
        log(f"  gather {k} {g.label}: gpu {info[k]['status']} {info[k]['iters']} {info[k]['ls_trials']} "
            f"{emd[k]:.12e}  oracle {r.status} {r.iters} {r.ls_trials} {r.emd:.12e}")
        assert info[k]["status"] == r.status
        assert info[k]["iters"] == r.iters
        if r.status == oracle.ZERO_SOURCE:
            continue
        assert info[k]["ls_trials"] == r.ls_trials
        assert emd[k] == pytest.approx(r.emd, rel=1e-9)
        assert info[k]["rel_res"] == pytest.approx(r.rel_res, rel=1e-7)
        assert rel_l2(phis[k], r.phi) <= 1e-9
        # each flux component relative to the whole flux: after thousands of
        # iterations the last-bit differences of the reduction order show on a
        # component ~1e3 times smaller than the other (u^x of the 40 x 530 gather)
        un = np.sqrt(np.sum(r.ux ** 2) + np.sum(r.ut ** 2))
        assert np.linalg.norm(us[k][0] - r.ux) <= 1e-9 * un
        assert np.linalg.norm(us[k][1] - r.ut) <= 1e-9 * un
    plan.close()


@pytest.mark.parametrize("max_trials", [40, 10])
def test_l1_backtracking_past_one_sweep_of_candidates(max_trials):
    # a first step of 1e-2 (50 to 3000 times the safe one on these grids) makes the
    # first linesearch backtrack 7 to 13 times: more candidates than one sweep sums,
    # so evaluation sweeps run; with 10 trials allowed some gathers fail there
    gs = ragged_batch(np.float64)
    p = E.SolverParams(precision=E.F64, max_iter=60, tol_res=0.0, check_every=60, ls_mode=E.LS_L1,
                       alpha1=1e-2, max_ls_trials=max_trials)
    log(f"l1 linesearch, alpha1=1e-2, max_ls_trials={max_trials}")
    plan, pcal, pobs, desc = make_plan(gs, p)
    emd, phi, u, info, _ = _solve(plan, pcal, pobs)
    ref = oracle_batch(gs, oracle_params(p), trace=True)
    phis = unpack(phi, desc)
    us = unpack(u, desc, 2)
    first = []
    for k, (r, _) in enumerate(ref):
        if r.iters:
            # backtracking trials of the first linesearch: alpha_2 = 1e-2 sqrt(2) xi^m
            first.append(int(round(np.log(r.alpha_trace[0] / (1e-2 * np.sqrt(2.0))) / np.log(0.5))))
        log(f"  gather {k} {gs[k].label}: gpu {info[k]['status']} {info[k]['iters']} {info[k]['ls_trials']} "
            f"{emd[k]:.12e}  oracle {r.status} {r.iters} {r.ls_trials} {r.emd:.12e}")
        assert info[k]["status"] == r.status
        assert info[k]["iters"] == r.iters
        if r.status == oracle.ZERO_SOURCE:
            continue
        assert info[k]["ls_trials"] == r.ls_trials
        assert emd[k] == pytest.approx(r.emd, rel=1e-9, abs=1e-300)
        assert info[k]["rel_res"] == pytest.approx(r.rel_res, rel=1e-7)
        assert rel_l2(phis[k], r.phi) <= 1e-9
        assert rel_l2(us[k][0], r.ux) <= 1e-9 or np.abs(r.ux).max() == 0
        assert rel_l2(us[k][1], r.ut) <= 1e-9 or np.abs(r.ut).max() == 0
    failed = [k for k, (r, _) in enumerate(ref) if r.status == oracle.LS_FAIL]
    log(f"  first-linesearch trials {first}, failed {failed}")
    # more than 6 trials (a failure at 10 needed more than 10) needs evaluation sweeps
    assert any(f > 6 for f in first) or failed
    assert bool(failed) == (max_trials == 10)
    plan.close()


@pytest.mark.parametrize("precision", [E.F32, E.F64])
def test_replayed_schedule_matches_oracle(precision):
    dtype = np.float64 if precision == E.F64 else np.float32
    gs = ragged_batch(dtype)
    K = 400
    p = E.SolverParams(precision=precision, max_iter=K, tol_res=0.0, check_every=K)
    ref = oracle_batch(gs, oracle_params(p), trace=True)
    alpha = np.zeros((len(gs), K))
    for k, (r, _) in enumerate(ref):
        alpha[k, :len(r.alpha_trace)] = r.alpha_trace
    log(f"replay precision={precision} K={K}")
    plan, pcal, pobs, desc = make_plan(gs, p, rows=16)
    s, mass = E.emd_decompose(plan, pcal, pobs)
    u = plan.empty(2)
    emd, phi, u, info = E.emd_pdhg_solve_replay(plan, s, torch.from_numpy(alpha).cuda(), u=u)
    torch.cuda.synchronize()
    emd, phi, info = emd.cpu().numpy(), unpack(phi.cpu().numpy(), desc), E.info_numpy(info)
    tol_e, tol_p = (1e-11, 1e-9) if precision == E.F64 else (1e-5, 1e-4)
    for k, (r, _) in enumerate(ref):
        log(f"  gather {k}: gpu {emd[k]:.10e} oracle {r.emd:.10e} "
            f"phi err {rel_l2(centred(phi[k]), centred(r.phi)) if r.emd > 0 else 0:.2e}")
        assert info[k]["iters"] == r.iters
        if r.status == oracle.ZERO_SOURCE:
            assert emd[k] == 0.0
            continue
        assert emd[k] == pytest.approx(r.emd, rel=tol_e)
        # The FP32 potential is claimed to 1e-4 on gathers of 100 cells or more.  On
        # the 5 x 9 and 7 x 1 grids the steps are ~1e2-1e3 times those of seismic size
        # and phi moves by beta times the FP32 rounding of the stored flux's residual
        # every iteration, so it drifts further; those two keep the EMD bound here and
        # the 1e-9 potential bound in FP64.
        if precision == E.F64 or gs[k].cells >= 100:
            assert rel_l2(centred(phi[k]), centred(r.phi)) <= tol_p
    plan.close()


@pytest.mark.parametrize("ls", [E.LS_L2, E.LS_L1])
def test_f32_reaches_the_oracle_optimum(ls):
    # accuracy parity: the oracle runs to a 1e-8 residual (within ~1e-7 of the
    # optimum here); the FP32 solve, free-running with its own linesearch, runs twice
    # as many iterations and must land within 1e-5 of that EMD.  (The residual stop
    # rule certifies feasibility only: a 1e-6 residual can leave the EMD 1e-3 high
    # on spiky data, so the budget, not the residual, is what is compared here.)
    gs = to_precision([config2_gather(nr=24, nt=120, f_peak=2.0, dtype=np.float64),
                       random_small_pair(8, 40, 5), random_small_pair(16, 16, 6),
                       config1_pairs([-80], nt=160, dt=1.0 / 159)[0]], np.float32)
    ref = oracle_batch(gs, oracle.Params(tol_res=1e-8, max_iter=2000000, ls_mode=ls))
    K = 2 * max(r.iters for r, _ in ref)
    p = E.SolverParams(precision=E.F32, tol_res=0.0, max_iter=K, check_every=K, ls_mode=ls)
    log(f"f32 to the optimum, K={K}, ls_mode={ls}")
    plan, pcal, pobs, desc = make_plan(gs, p)
    emd, phi, u, info, _ = _solve(plan, pcal, pobs)
    for k, (r, _) in enumerate(ref):
        log(f"  gather {k}: gpu it={info[k]['iters']} res={info[k]['rel_res']:.1e} emd={emd[k]:.10e} "
            f"oracle it={r.iters} emd={r.emd:.10e} rel={abs(emd[k] - r.emd) / r.emd:.2e}")
        assert info[k]["iters"] == K
        assert abs(emd[k] - r.emd) <= 1e-5 * r.emd
    plan.close()


def test_f32_stop_rule_reaches_tolerance():
    # the stop rule itself: every gather stops CONVERGED with the residual it reports,
    # and the reported residual and EMD are those of the returned flux (recomputed
    # here by the oracle's own operators in FP64)
    gs = to_precision([config2_gather(nr=30, nt=200, f_peak=2.5, dtype=np.float64),
                       random_small_pair(12, 50, 7)], np.float32)
    p = E.SolverParams(precision=E.F32, tol_res=1e-5, max_iter=200000)
    plan, pcal, pobs, desc = make_plan(gs, p)
    log("f32 stop rule 1e-5")
    emd, phi, u, info, _ = _solve(plan, pcal, pobs)
    us = unpack(u, desc, 2)
    phis = unpack(phi, desc)
    for k, g in enumerate(gs):
        s, _, _, _ = oracle.decompose(g.pcal, g.pobs, g.dx, g.dt)
        assert E.GATHER_STATUS[info[k]["status"]] == "CONVERGED"
        assert info[k]["iters"] % p.check_every == 0
        ux, ut = (c.astype(np.float64) for c in us[k])
        res = np.linalg.norm(oracle.div(ux, ut, g.dx, g.dt) + s) / np.linalg.norm(s)
        assert res <= 1.05e-5
        assert info[k]["rel_res"] == pytest.approx(res, rel=1e-3, abs=2e-7)
        # the objective of the returned flux and the Lagrangian value at the returned
        # pair (the EMD estimate), both recomputed by the oracle
        lag, primal = oracle.lagrangian_value(s, ux, ut, phis[k], g.dx, g.dt)
        assert info[k]["primal"] == pytest.approx(primal, rel=1e-6)
        assert emd[k] == pytest.approx(lag, rel=1e-6) and info[k]["emd"] == emd[k]
    plan.close()


@pytest.mark.parametrize("precision", [E.F32, E.F64])
@pytest.mark.parametrize("mode", [E.MASS_BALANCE, E.MASS_UNIT, E.MASS_NONE])
def test_adjoint_matches_oracle_on_same_phi(precision, mode):
    dtype = np.float64 if precision == E.F64 else np.float32
    gs = ragged_batch(dtype)
    p = E.SolverParams(precision=precision, mass_mode=mode, max_iter=50, tol_res=0.0,
                       check_every=50, mass_tol=1.0)
    log(f"adjoint precision={precision} mode={mode}")
    plan, pcal, pobs, desc = make_plan(gs, p, rows=8)
    s, mass = E.emd_decompose(plan, pcal, pobs)
    emd, phi, _, _ = E.emd_pdhg_solve(plan, s, mass=mass)
    gbar = torch.linspace(0.5, 2.0, len(gs), dtype=torch.float64, device=plan.device)
    psi = E.emd_adjoint_source(plan, phi, pcal, pobs, mass, gbar=gbar)
    torch.cuda.synchronize()
    phis = unpack(phi.cpu().numpy(), desc)
    psis = unpack(psi.cpu().numpy(), desc)
    mass_h = mass.cpu().numpy()
    tol = 1e-12 if precision == E.F64 else 2e-6
    for k, g in enumerate(gs):
        ref = oracle.adjoint(phis[k].astype(np.float64), g.pcal, g.pobs, mass_h[k], g.dx, g.dt,
                             mode, gbar=float(gbar[k]))
        scale = max(np.abs(ref).max(), 1e-300)
        np.testing.assert_allclose(psis[k], ref, rtol=0, atol=tol * scale * 4)
    plan.close()


@pytest.mark.parametrize("precision", [E.F32, E.F64])
def test_lsd_matches_oracle(precision):
    dtype = np.float64 if precision == E.F64 else np.float32
    gs = ragged_batch(dtype)
    p = E.SolverParams(precision=precision)
    plan, pcal, pobs, desc = make_plan(gs, p)
    gbar = torch.linspace(-1.5, 2.0, len(gs), dtype=torch.float64)
    value, psi = E.lsd_misfit(plan, pcal, pobs, gbar=gbar)
    value_only, none = E.lsd_misfit(plan, pcal, pobs, with_adjoint=False)
    torch.cuda.synchronize()
    assert none is None
    value, value_only = value.cpu().numpy(), value_only.cpu().numpy()
    psis = unpack(psi.cpu().numpy(), desc)
    for k, g in enumerate(gs):
        f, grad = oracle.lsd(g.pcal, g.pobs, g.dx, g.dt)
        # FP64 sums of the same differences in another order
        assert value[k] == pytest.approx(f, rel=1e-13)
        assert value_only[k] == value[k]
        want = grad * float(gbar[k])
        # FP32 output: the rounding of the FP64 value; values far below the field's
        # peak may fall into (or below) the subnormal range
        np.testing.assert_allclose(psis[k], want, rtol=1e-15 if precision == E.F64 else 1.2e-7,
                                   atol=1e-300 if precision == E.F64 else 1e-30 * np.abs(want).max())
    plan.close()


def test_statuses_of_degenerate_gathers():
    base = random_small_pair(6, 20, 9)
    q = np.round(base.pcal * 1024) / 1024
    nan = base.pcal.copy()
    nan[2, 3] = np.nan
    gs = [type(base)(q + 0.25, q.copy(), base.dx, base.dt, "offset"),
          type(base)(nan, base.pobs, base.dx, base.dt, "nan"),
          base]
    gs = to_precision(gs, np.float64)
    p = E.SolverParams(precision=E.F64, max_iter=5, check_every=5, tol_res=0.0)
    log("statuses")
    plan, pcal, pobs, desc = make_plan(gs, p)
    emd, phi, u, info, _ = _solve(plan, pcal, pobs)
    st = [E.GATHER_STATUS[i] for i in info["status"]]
    assert st == ["ZERO_SOURCE", "NONFINITE", "MAX_ITER"]
    assert emd[0] == 0.0 and info["iters"][2] == 5
    assert np.all(unpack(phi, desc)[0] == 0)
    plan.close()
    # mass mode none with unequal masses, and a failing linesearch
    g2 = to_precision([random_small_pair(6, 20, 9, balanced=False)], np.float64)
    p = E.SolverParams(precision=E.F64, mass_mode=E.MASS_NONE, max_iter=5)
    plan, pcal, pobs, desc = make_plan(g2, p)
    emd, _, _, info, _ = _solve(plan, pcal, pobs)
    assert E.GATHER_STATUS[info["status"][0]] == "MASS_IMBALANCE" and np.isnan(emd[0])
    plan.close()
    p = E.SolverParams(precision=E.F64, zeta=1e-12, max_ls_trials=5, max_iter=50)
    plan, pcal, pobs, desc = make_plan(to_precision([base], np.float64), p)
    emd, _, _, info, _ = _solve(plan, pcal, pobs)
    r, _ = oracle.misfit(base.pcal, base.pobs, base.dx, base.dt,
                         params=oracle_params(p))
    assert E.GATHER_STATUS[info["status"][0]] == "LS_FAIL" and r.status == oracle.LS_FAIL
    assert info["iters"][0] == r.iters
    plan.close()


def test_replay_fields_are_independent_of_tiling():
    # with the step schedule fixed, every field value is a per-cell computation, so
    # any tiling must give bitwise identical iterates (catches halo and ordering races)
    gs = ragged_batch(np.float32)
    K = 120
    alpha = np.zeros((len(gs), K))
    for k, g in enumerate(gs):
        lam = oracle.lambda_bound(g.nr, g.nt, g.dx, g.dt)
        alpha[k] = 1.0 / np.sqrt(1e5 * lam) * 1.3 ** np.minimum(np.arange(K), 20)
    p = E.SolverParams(precision=E.F32, max_iter=K, tol_res=0.0, check_every=K)
    outs = []
    # uniform heights, then a different height per gather
    for rows in (1, 3, 16, 64, [5, 2, 7, 1, 3, 12]):
        log(f"tiling rows={rows}")
        if isinstance(rows, list):
            plan, pcal, pobs, desc = make_plan(gs, p)
            plan.set_gather_tiling(rows)
            assert plan.gather_tiling() == rows
        else:
            plan, pcal, pobs, desc = make_plan(gs, p, rows=rows)
        s, mass = E.emd_decompose(plan, pcal, pobs)
        u = plan.empty(2)
        emd, phi, u, info = E.emd_pdhg_solve_replay(plan, s, torch.from_numpy(alpha).cuda(), u=u)
        torch.cuda.synchronize()
        outs.append((phi.cpu().numpy(), u.cpu().numpy()))
        plan.close()
    for o in outs[1:]:
        np.testing.assert_array_equal(o[0], outs[0][0])
        np.testing.assert_array_equal(o[1], outs[0][1])


def test_autotuned_tiling_is_valid_and_reusable():
    # the autotuner picks a height per size bucket; a plan given the same heights
    # reproduces a solve bitwise, and the result agrees with the default tiling
    from synth import config3_batch
    gs = config3_batch()[:12]
    p = E.SolverParams(precision=E.F32, max_iter=300, tol_res=0.0, check_every=300)
    plan, pcal, pobs, desc = make_plan(gs, p)
    s, mass = E.emd_decompose(plan, pcal, pobs)
    rows = plan.autotune(s, sweeps=8)
    log(f"  autotuned heights {rows}")
    assert set(rows) <= {8, 12, 16}
    nts = np.array([g.nt for g in gs])
    nrs = np.array([g.nr for g in gs])
    tert = lambda v: (v >= np.sort(v)[len(v) // 3]).astype(int) + (v >= np.sort(v)[2 * len(v) // 3])
    bucket = 3 * tert(nts) + tert(nrs)
    for b in set(bucket.tolist()):
        assert len({rows[k] for k in np.flatnonzero(bucket == b)}) == 1
    assert plan.params.ls_mode == E.LS_L2
    e1, phi1, _, i1 = E.emd_pdhg_solve(plan, s, mass=mass)
    plan2, _, _, _ = make_plan(gs, p)
    plan2.set_gather_tiling(rows)
    e2, phi2, _, i2 = E.emd_pdhg_solve(plan2, s, mass=mass)
    plan3, _, _, _ = make_plan(gs, p)
    e3, _, _, _ = E.emd_pdhg_solve(plan3, s, mass=mass)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(e1.cpu().numpy(), e2.cpu().numpy())
    np.testing.assert_array_equal(phi1.cpu().numpy(), phi2.cpu().numpy())
    np.testing.assert_allclose(e1.cpu().numpy(), e3.cpu().numpy(), rtol=1e-5)
    for pl in (plan, plan2, plan3):
        pl.close()


def test_autotune_cache_hit_skips_the_timing(tmp_path, monkeypatch):
    # the first plan times the heights and stores them under its key; a second plan of
    # the same batch finds them in the cache (EMD_AUTOTUNE_CACHE) and times nothing
    from synth import config3_batch
    from paper_1808_07284_amd import _lib as L
    gs = config3_batch()[:6]
    p = E.SolverParams(precision=E.F32)
    path = tmp_path / "tiles.json"
    monkeypatch.setenv("EMD_AUTOTUNE_CACHE", str(path))
    plan, pcal, pobs, desc = make_plan(gs, p)
    s, _ = E.emd_decompose(plan, pcal, pobs)
    rows = plan.autotune(s, sweeps=8)
    import json
    entries = json.loads(path.read_text())
    assert list(entries.values()) == [rows]
    plan2, _, _, _ = make_plan(gs, p)
    calls = []
    lib = L.load()
    real = lib.emd_plan_autotune
    monkeypatch.setattr(lib, "emd_plan_autotune", lambda *a: calls.append(a) or real(*a))
    assert plan2.autotune(s, sweeps=8) == rows
    assert calls == [] and plan2.gather_tiling() == rows
    plan.close()
    plan2.close()


@pytest.mark.parametrize("ls", [E.LS_L2, E.LS_L1])
def test_checkpoint_resume_is_bitwise(ls):
    # a solve of K iterations, checkpointed (solver state + its u, phi) and resumed to
    # 2K, reproduces a single solve of 2K iterations bitwise
    gs = ragged_batch(np.float32)
    K = 150
    p2 = E.SolverParams(precision=E.F32, max_iter=2 * K, tol_res=0.0, check_every=2 * K, ls_mode=ls)
    p1 = E.SolverParams(precision=E.F32, max_iter=K, tol_res=0.0, check_every=K, ls_mode=ls)
    plan, pcal, pobs, desc = make_plan(gs, p2)
    with pytest.raises(E.EMDError):
        E.solver_state(plan)  # nothing solved yet
    s, mass = E.emd_decompose(plan, pcal, pobs)
    u_ref = plan.empty(2)
    e_ref, phi_ref, _, i_ref = E.emd_pdhg_solve(plan, s, u=u_ref, mass=mass)
    torch.cuda.synchronize()
    e_ref, phi_ref, u_ref, i_ref = (e_ref.cpu().numpy(), phi_ref.cpu().numpy(), u_ref.cpu().numpy(),
                                    E.info_numpy(i_ref))
    plan.set_params(p1)
    u = plan.empty(2)
    _, phi, _, _ = E.emd_pdhg_solve(plan, s, u=u, mass=mass)
    state = E.solver_state(plan)
    assert [state[k].iters for k in range(len(gs))] == [K] * len(gs)
    plan.set_params(p2)
    e2, phi, u, i2 = E.emd_pdhg_solve_resume(plan, s, state, u, phi, mass=mass)
    torch.cuda.synchronize()
    i2 = E.info_numpy(i2)
    log(f"  ls_mode={ls}: 2K iterations {i_ref['iters'].tolist()} resumed {i2['iters'].tolist()}, "
        f"trials {i_ref['ls_trials'].tolist()} / {i2['ls_trials'].tolist()}")
    np.testing.assert_array_equal(e2.cpu().numpy(), e_ref)
    np.testing.assert_array_equal(phi.cpu().numpy(), phi_ref)
    np.testing.assert_array_equal(u.cpu().numpy(), u_ref)
    for f in ("status", "iters", "ls_trials", "rel_res", "emd", "transport", "alpha", "primal"):
        np.testing.assert_array_equal(i2[f], i_ref[f])
    plan.close()


@pytest.mark.parametrize("ls", [E.LS_L2, E.LS_L1])
def test_resume_keeps_finished_gathers_and_continues_the_rest(ls):
    # with the stop rule on, a checkpoint taken when some gathers have converged and
    # others have not: resumed (twice, in two legs) it reproduces the uninterrupted
    # solve bitwise -- the converged gathers are not iterated again
    gs = ragged_batch(np.float32)
    z = gs[1]
    gs.append(type(z)(z.pcal.copy(), z.pcal.copy(), z.dx, z.dt, "zero source"))
    N = 4000
    pN = E.SolverParams(precision=E.F32, max_iter=N, tol_res=1e-4, ls_mode=ls)
    plan, pcal, pobs, desc = make_plan(gs, pN)
    s, mass = E.emd_decompose(plan, pcal, pobs)
    u_ref = plan.empty(2)
    e_ref, phi_ref, _, i_ref = E.emd_pdhg_solve(plan, s, u=u_ref, mass=mass)
    torch.cuda.synchronize()
    e_ref, phi_ref, u_ref, i_ref = (e_ref.cpu().numpy(), phi_ref.cpu().numpy(), u_ref.cpu().numpy(),
                                    E.info_numpy(i_ref))
    conv = i_ref["iters"][i_ref["status"] == E.GATHER_STATUS.index("CONVERGED")]
    assert len(set(conv.tolist())) >= 2
    K1 = int(np.sort(conv)[len(conv) // 2])          # some gathers finish before, some after
    K2 = (K1 + int(conv.max())) // 2
    u = plan.empty(2)
    plan.set_params(dataclasses.replace(pN, max_iter=K1))
    _, phi, _, i1 = E.emd_pdhg_solve(plan, s, u=u, mass=mass)
    st1 = E.info_numpy(i1)["status"]
    assert (st1 == E.GATHER_STATUS.index("CONVERGED")).any() and (st1 == E.GATHER_STATUS.index("MAX_ITER")).any()
    for kmax in (K2, N):
        state = E.solver_state(plan)
        plan.set_params(dataclasses.replace(pN, max_iter=kmax))
        e2, phi, u, i2 = E.emd_pdhg_solve_resume(plan, s, state, u, phi, mass=mass)
    torch.cuda.synchronize()
    i2 = E.info_numpy(i2)
    log(f"  ls_mode={ls}: legs to {K1}, {K2}, {N}; iterations {i_ref['iters'].tolist()} "
        f"resumed {i2['iters'].tolist()}, statuses {i2['status'].tolist()}")
    np.testing.assert_array_equal(e2.cpu().numpy(), e_ref)
    np.testing.assert_array_equal(phi.cpu().numpy(), phi_ref)
    np.testing.assert_array_equal(u.cpu().numpy(), u_ref)
    for f in ("status", "iters", "ls_trials", "rel_res", "emd", "transport", "alpha", "primal"):
        np.testing.assert_array_equal(i2[f], i_ref[f])
    plan.close()


def test_repeat_solves_are_bitwise_deterministic():
    gs = ragged_batch(np.float32)
    p = E.SolverParams(precision=E.F32, max_iter=200, tol_res=0.0, check_every=200)
    plan, pcal, pobs, desc = make_plan(gs, p)
    a = _solve(plan, pcal, pobs)
    b = _solve(plan, pcal, pobs)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])
    plan.close()


def test_narrowed_tile_table_gives_bitwise_identical_results():
    # gathers that converge at different iterations plus one with nothing to solve;
    # with a status read every two sweeps the sweep's tile table is narrowed to the
    # running gathers several times, with one chunk of sweeps never
    gs = ragged_batch(np.float32)
    z = gs[1]
    gs.append(type(z)(z.pcal.copy(), z.pcal.copy(), z.dx, z.dt, "zero source"))
    res = {}
    for spsync in (4096, 2):
        p = E.SolverParams(precision=E.F32, max_iter=4000, tol_res=1e-4, sweeps_per_sync=spsync)
        plan, pcal, pobs, desc = make_plan(gs, p)
        res[spsync] = _solve(plan, pcal, pobs)
        res[spsync, "rebuilds"] = plan.query()["last_table_rebuilds"]
        if spsync == 2:
            # a second solve on the same plan starts from stale state buffers
            again = _solve(plan, pcal, pobs)
            for k in range(3):
                np.testing.assert_array_equal(again[k], res[2][k])
            np.testing.assert_array_equal(again[3], res[2][3])
        plan.close()
    info = res[2][3]
    log(f"  iterations {info['iters'].tolist()}, statuses {info['status'].tolist()}, "
        f"rebuilds {res[4096, 'rebuilds']} / {res[2, 'rebuilds']}")
    assert res[4096, "rebuilds"] == 0 and res[2, "rebuilds"] >= 1
    assert len(set(info["iters"][info["status"] == 1].tolist())) >= 2
    assert info["status"][-1] == E.GATHER_STATUS.index("ZERO_SOURCE")
    for k in range(3):
        np.testing.assert_array_equal(res[2][k], res[4096][k])
    np.testing.assert_array_equal(res[2][3], res[4096][3])


def test_autograd_backward_is_the_adjoint_source():
    gs = to_precision([random_small_pair(10, 64, 21), random_small_pair(6, 30, 22)], np.float32)
    p = E.SolverParams(precision=E.F32, max_iter=100, tol_res=0.0, check_every=100)
    plan, pcal, pobs, desc = make_plan(gs, p)
    x = pcal.clone().requires_grad_(True)
    e = E.emd_misfit(x, pobs, plan)
    w = torch.tensor([0.7, -1.3], dtype=torch.float64, device=plan.device)
    (e * w).sum().backward()
    s, mass = E.emd_decompose(plan, pcal, pobs)
    _, phi, _, _ = E.emd_pdhg_solve(plan, s, mass=mass)
    psi = E.emd_adjoint_source(plan, phi, pcal, pobs, mass, gbar=w)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(x.grad.cpu().numpy(), psi.cpu().numpy())
    plan.close()
