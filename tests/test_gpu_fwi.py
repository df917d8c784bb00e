"""The misfit inside an FWI loop: warm starts across successive evaluations of one
batch, and the time-axis weighting T of the EMD grid (the T = 0.1, 1, 10 study of
the paper's Marmousi example)."""
import numpy as np
import pytest

from gpu_util import log, make_plan, unpack
from synth import Gather, config1_pairs, config2_gather

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1808_07284_amd as E  # noqa: E402


def closed_form_1d(s, dt, eps=1e-4):
    S = np.cumsum(np.asarray(s, np.float64).reshape(-1))[:-1]
    return dt * dt * np.abs(S).sum() + 0.5 * eps * dt ** 3 * (S * S).sum()


def test_warm_start_across_fwi_evaluations():
    # an FWI loop evaluates the misfit of a slowly changing predicted batch: starting
    # each solve from the previous flux and potential cuts the iterations (here by
    # about half; by 3-7x on other data), and lands on the same EMD to the stop
    # rule's accuracy
    gs = [config2_gather(seed=s, nr=60, nt=300, f_peak=2.0) for s in (21, 22, 23)]
    p = E.SolverParams(precision=E.F32, tol_res=1e-5, max_iter=2000000)
    plan, pcal, pobs, desc = make_plan(gs, p)
    warm = E.WarmStart(plan)
    for k, step in enumerate((0.0, 0.02, 0.05, 0.05)):
        pcal = pcal + step * (pobs - pcal)
        x = pcal.clone().requires_grad_(True)
        e_w = E.emd_misfit(x, pobs, plan, warm)
        e_w.sum().backward()
        torch.cuda.synchronize()
        q_w = plan.query()["last_cell_updates"]
        psi_w = x.grad.clone()
        e_c = E.emd_misfit(pcal, pobs, plan)
        torch.cuda.synchronize()
        q_c = plan.query()["last_cell_updates"]
        rel = (e_w.detach() - e_c).abs() / e_c
        log(f"  evaluation {k}: cell updates warm {q_w} cold {q_c}, EMD rel diff {float(rel.max()):.1e}")
        assert float(rel.max()) <= 1e-3
        assert torch.isfinite(psi_w).all()
        if k == 0:
            assert q_w == q_c
        else:
            assert q_w * 1.5 <= q_c
    plan.close()


def test_time_weighting_in_1d_matches_the_closed_form():
    # the EMD grid's time extent T sets dt = T / (nt - 1): with the samples fixed the
    # 1D optimum scales as T^2 W + eps/2 T^3 Q, which the closed form gives exactly
    base = config1_pairs([40], nt=200, dt=1.0 / 199, f_peak=3.0, centre=0.45)[0]
    gs = [Gather(base.pcal, base.pobs, dx=1.0, dt=T / 199, label=f"T={T}") for T in (0.1, 1.0, 10.0)]
    p = E.SolverParams(precision=E.F64, tol_res=1e-7, max_iter=4000000, sweeps_per_sync=4096)
    plan, pcal, pobs, desc = make_plan(gs, p)
    s, mass = E.emd_decompose(plan, pcal, pobs)
    emd, phi, u, info = E.emd_pdhg_solve(plan, s, mass=mass)
    torch.cuda.synchronize()
    emd = emd.cpu().numpy()
    inf = E.info_numpy(info)
    s_h = unpack(s.cpu().numpy(), desc)
    for k, g in enumerate(gs):
        ref = closed_form_1d(s_h[k], g.dt)
        log(f"  {g.label}: emd {emd[k]:.10e} closed form {ref:.10e} it={inf['iters'][k]} "
            f"{E.GATHER_STATUS[inf['status'][k]]}")
        assert E.GATHER_STATUS[inf["status"][k]] == "CONVERGED"
        assert emd[k] == pytest.approx(ref, rel=1e-6)
    plan.close()


def test_time_weighting_moves_transport_to_the_receiver_axis():
    # with X = 1 fixed, a larger T makes time moves dearer: the optimal flux moves more
    # mass across receivers (the adjoint source grows more continuous along that axis,
    # as the paper observes for T = 0.1, 1, 10) and less along time.  Amounts in grid
    # steps: sum |u^x| / dx (mass x receiver steps) and sum |u^t| / dt (mass x time
    # steps); the second cannot grow with T (the optimal value is concave in the time
    # cost and this is its slope), the first grows here by orders of magnitude
    base = config2_gather(seed=7, nr=40, nt=200, f_peak=2.0)
    gs = [Gather(base.pcal, base.pobs, dx=1.0 / 39, dt=T / 199, label=f"T={T}") for T in (0.1, 1.0, 10.0)]
    p = E.SolverParams(precision=E.F32, tol_res=1e-5, max_iter=2000000)
    plan, pcal, pobs, desc = make_plan(gs, p)
    s, mass = E.emd_decompose(plan, pcal, pobs)
    u = plan.empty(2)
    emd, phi, u, info = E.emd_pdhg_solve(plan, s, u=u, mass=mass)
    torch.cuda.synchronize()
    us = unpack(u.cpu().numpy(), desc, 2)
    xs, ts = [], []
    for k, g in enumerate(gs):
        xs.append(np.abs(us[k][0].astype(np.float64)).sum() / g.dx)
        ts.append(np.abs(us[k][1].astype(np.float64)).sum() / g.dt)
        log(f"  {g.label}: EMD {float(emd[k]):.6e}, transport along receivers {xs[-1]:.4e}, "
            f"along time {ts[-1]:.4e} (grid steps x mass)")
    assert xs[0] < xs[1] < xs[2]
    assert ts[1] <= ts[0] * 1.01 and ts[2] < ts[1]
    e = emd.cpu().numpy()
    assert e[0] < e[1] < e[2]
    plan.close()


def test_two_plans_on_two_streams_from_two_threads():
    # shots handled as separate plans, each on its own stream and host thread (the
    # plans share no state; a call releases the interpreter while it runs): the
    # concurrent solves give bitwise the results of solving the plans one after the
    # other
    import threading
    from synth import random_small_pair
    sets = [[config2_gather(seed=31, nr=40, nt=300, f_peak=3.0), random_small_pair(9, 120, 32)],
            [config2_gather(seed=33, nr=30, nt=400, f_peak=3.0), random_small_pair(5, 77, 34)]]
    p = E.SolverParams(precision=E.F32, tol_res=1e-5, max_iter=200000)
    plans = [make_plan(gs, p) for gs in sets]

    def solve(k, out, stream=None):
        plan, pcal, pobs, _ = plans[k]
        ctx = torch.cuda.stream(stream) if stream is not None else torch.cuda.stream(torch.cuda.current_stream())
        with ctx:
            s, mass = E.emd_decompose(plan, pcal, pobs)
            emd, phi, u, info = E.emd_pdhg_solve(plan, s, u=plan.empty(2), mass=mass)
            torch.cuda.current_stream().synchronize()
            out[k] = (emd.cpu().numpy(), phi.cpu().numpy(), u.cpu().numpy(), E.info_numpy(info))

    seq = {}
    for k in range(2):
        solve(k, seq)
    torch.cuda.synchronize()
    par = {}
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    threads = [threading.Thread(target=solve, args=(k, par, streams[k])) for k in range(2)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
        assert not th.is_alive()
    torch.cuda.synchronize()
    for k in range(2):
        for a, b in zip(seq[k][:3], par[k][:3]):
            np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(seq[k][3], par[k][3])
    log(f"  iterations {[seq[k][3]['iters'].tolist() for k in range(2)]}")
    for plan, *_ in plans:
        plan.close()
