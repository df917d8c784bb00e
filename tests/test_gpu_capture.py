"""The fixed-budget solve (sweeps_per_sync = 0): every sweep on the caller's stream,
nothing read back, so a caller can capture a misfit evaluation into a HIP graph.
Its results are bitwise those of the chunked solve, eagerly and replayed."""
import dataclasses

import numpy as np
import pytest

from gpu_util import log, make_plan, to_precision
from synth import config1_pairs, config2_gather, random_small_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1808_07284_amd as E  # noqa: E402


def _batch():
    gs = [config2_gather(nr=40, nt=530, f_peak=3.0, dtype=np.float64), random_small_pair(13, 301, 1),
          random_small_pair(5, 9, 2), config1_pairs([60], nt=257, dt=1.0 / 256)[0],
          random_small_pair(7, 1, 3), random_small_pair(3, 250, 4)]
    z = gs[1]
    gs.append(type(z)(z.pcal.copy(), z.pcal.copy(), z.dx, z.dt, "zero source"))
    return to_precision(gs, np.float32)


def _out(plan):
    return {"phi": plan.empty(), "u": plan.empty(2),
            "emd": torch.empty(plan.ngather, dtype=torch.float64, device=plan.device),
            "info": torch.empty(plan.ngather * E.INFO_DTYPE.itemsize, dtype=torch.uint8, device=plan.device)}


def _solve(plan, s, mass, o):
    E.emd_pdhg_solve(plan, s, phi=o["phi"], u=o["u"], mass=mass, emd_out=o["emd"], info_out=o["info"])


def _host(o):
    return {k: v.cpu().numpy().copy() for k, v in o.items()}


def _same(a, b):
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("ls", [E.LS_L2, E.LS_L1])
def test_fixed_budget_solve_matches_the_chunked_solve_and_replays_from_a_graph(ls):
    gs = _batch()
    # a stop rule that some gathers meet before the budget and others do not
    p = E.SolverParams(precision=E.F32, tol_res=1e-4, max_iter=900, ls_mode=ls)
    plan, pcal, pobs, desc = make_plan(gs, p)
    s, mass = E.emd_decompose(plan, pcal, pobs)
    o = _out(plan)
    _solve(plan, s, mass, o)
    torch.cuda.synchronize()
    ref = _host(o)
    q_ref = plan.query()
    info = E.info_numpy(o["info"])
    log(f"  ls_mode={ls}: statuses {info['status'].tolist()} iterations {info['iters'].tolist()}")
    assert {1, 2} <= set(info["status"].tolist())       # converged and capped gathers
    plan.set_params(dataclasses.replace(p, sweeps_per_sync=0))
    # eager fixed-budget call
    for v in o.values():
        v.zero_()
    _solve(plan, s, mass, o)
    torch.cuda.synchronize()
    _same(_host(o), ref)
    q = plan.query()
    assert q["last_cell_updates"] == q_ref["last_cell_updates"]
    state = E.solver_state(plan)
    assert [state[k].iters for k in range(len(gs))] == info["iters"].tolist()
    # captured into a graph by the caller, replayed with eager work in between
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        _solve(plan, s, mass, o)
    other = torch.randn(1 << 20, device=plan.device)
    for r in range(3):
        for v in o.values():
            v.fill_(7)
        other.mul_(1.5).add_(1.0)                         # the program's own work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        _same(_host(o), ref)
        log(f"  replay {r}: bitwise equal to the chunked solve")
    assert plan.query()["last_cell_updates"] == q_ref["last_cell_updates"]
    del graph
    plan.close()
