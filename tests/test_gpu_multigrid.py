"""GPU parity of the grid transfer (emd_restrict, emd_prolong) with the oracle, and
the coarse-to-fine solve (Multigrid) against the cold solve, through the C ABI."""
import numpy as np
import pytest

import oracle
from certificate import transport_bounds
from gpu_util import log, make_plan, to_precision, unpack
from synth import config1_pairs, config2_gather, random_small_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1808_07284_amd as E  # noqa: E402


def ragged(dtype):
    gs = [
        config2_gather(nr=40, nt=530, f_peak=3.0, dtype=np.float64),
        random_small_pair(13, 301, 1),
        random_small_pair(5, 9, 2),
        config1_pairs([60], nt=257, dt=1.0 / 256)[0],
        random_small_pair(7, 1, 3),
        random_small_pair(3, 250, 4),
    ]
    return to_precision(gs, dtype)


def _plans(gs, precision, fr, ft, **kw):
    p = E.SolverParams(precision=precision, **kw)
    fine, pcal, pobs, desc = make_plan(gs, p)
    cd, n = E.coarse_descs(desc, fr, ft)
    coarse = E.Plan(cd, n, p)
    return fine, coarse, pcal, pobs, desc, cd


@pytest.mark.parametrize("precision", [E.F32, E.F64])
@pytest.mark.parametrize("fr,ft", [(2, 4), (3, 2), (1, 4), (1, 1)])
def test_restrict_matches_oracle(precision, fr, ft):
    dtype = np.float64 if precision == E.F64 else np.float32
    gs = ragged(dtype)
    fine, coarse, pcal, pobs, desc, cd = _plans(gs, precision, fr, ft)
    out = E.restrict(fine, coarse, fr, ft, pcal)
    torch.cuda.synchronize()
    got = unpack(out.cpu().numpy(), cd)
    for g, c in zip(gs, got):
        ref = oracle.restrict(g.pcal.astype(np.float64), fr, ft)
        assert c.shape == ref.shape
        if precision == E.F64:
            np.testing.assert_array_equal(c, ref)     # same sums in the same order
        else:
            # one rounding to FP32 (subnormal results round on the subnormal grid)
            np.testing.assert_allclose(c, ref, rtol=2 ** -23, atol=2e-38)
    fine.close()
    coarse.close()


@pytest.mark.parametrize("precision", [E.F32, E.F64])
@pytest.mark.parametrize("fr,ft", [(2, 4), (3, 2), (1, 4), (1, 1)])
def test_prolong_matches_oracle(precision, fr, ft):
    dtype = np.float64 if precision == E.F64 else np.float32
    gs = ragged(dtype)
    fine, coarse, pcal, pobs, desc, cd = _plans(gs, precision, fr, ft)
    rng = np.random.default_rng(17)
    n_c = coarse.batch_len
    u_c_h = rng.normal(size=(2, n_c)).astype(dtype)
    phi_c_h = rng.normal(size=n_c).astype(dtype)
    u_c = torch.from_numpy(u_c_h).to(coarse.device)
    phi_c = torch.from_numpy(phi_c_h).to(coarse.device)
    u_f, phi_f = E.prolong(coarse, fine, fr, ft, u_c, phi_c)
    torch.cuda.synchronize()
    us = unpack(u_f.cpu().numpy(), desc, 2)
    phis = unpack(phi_f.cpu().numpy(), desc)
    ucs = unpack(u_c_h, cd, 2)
    phics = unpack(phi_c_h, cd)
    for k, g in enumerate(gs):
        rx, rt, rp = oracle.prolong(ucs[k][0], ucs[k][1], phics[k], g.nr, g.nt, fr, ft)
        if precision == E.F64:
            for got, ref in ((us[k][0], rx), (us[k][1], rt), (phis[k], rp)):
                np.testing.assert_array_equal(got, ref)
        else:
            for got, ref in ((us[k][0], rx), (us[k][1], rt), (phis[k], rp)):
                np.testing.assert_allclose(got, ref, rtol=0, atol=4e-7 * max(1.0, np.abs(ref).max()))
    # phi only: u is neither read nor written
    L = E._lib
    phi_only = fine.empty()
    with torch.cuda.device(fine.device):
        L.check(L.load().emd_prolong(coarse.handle, fine.handle, fr, ft, None, phi_c.data_ptr(), None,
                                     phi_only.data_ptr(), None))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(phi_only.cpu().numpy(), phi_f.cpu().numpy())
    fine.close()
    coarse.close()


@pytest.mark.parametrize("precision", [E.F32, E.F64])
@pytest.mark.parametrize("fr,ft", [(1, 2), (2, 3)])
def test_prolong_wide_gather_and_single_outputs(precision, fr, ft):
    # a 20 x 5000 gather has more 16-row by 256-sample pieces (20 x 2) than the launch
    # has blocks per gather (its 20 rows), so blocks take several pieces in turn; the
    # u-only and phi-only calls give the fields of the call with both outputs
    dtype = np.float64 if precision == E.F64 else np.float32
    gs = to_precision([random_small_pair(20, 5000, 31), random_small_pair(9, 300, 32)], dtype)
    fine, coarse, pcal, pobs, desc, cd = _plans(gs, precision, fr, ft)
    rng = np.random.default_rng(23)
    n_c = coarse.batch_len
    u_c_h = rng.normal(size=(2, n_c)).astype(dtype)
    phi_c_h = rng.normal(size=n_c).astype(dtype)
    u_c = torch.from_numpy(u_c_h).to(coarse.device)
    phi_c = torch.from_numpy(phi_c_h).to(coarse.device)
    u_f, phi_f = E.prolong(coarse, fine, fr, ft, u_c, phi_c)
    L = E._lib
    u_only, phi_only = fine.empty(2), fine.empty()
    with torch.cuda.device(fine.device):
        L.check(L.load().emd_prolong(coarse.handle, fine.handle, fr, ft, u_c.data_ptr(), None,
                                     u_only.data_ptr(), None, None))
        L.check(L.load().emd_prolong(coarse.handle, fine.handle, fr, ft, None, phi_c.data_ptr(), None,
                                     phi_only.data_ptr(), None))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u_only.cpu().numpy(), u_f.cpu().numpy())
    np.testing.assert_array_equal(phi_only.cpu().numpy(), phi_f.cpu().numpy())
    us = unpack(u_f.cpu().numpy(), desc, 2)
    phis = unpack(phi_f.cpu().numpy(), desc)
    ucs = unpack(u_c_h, cd, 2)
    phics = unpack(phi_c_h, cd)
    for k, g in enumerate(gs):
        rx, rt, rp = oracle.prolong(ucs[k][0], ucs[k][1], phics[k], g.nr, g.nt, fr, ft)
        for got, ref in ((us[k][0], rx), (us[k][1], rt), (phis[k], rp)):
            if precision == E.F64:
                np.testing.assert_array_equal(got, ref)
            else:
                np.testing.assert_allclose(got, ref, rtol=0, atol=4e-7 * max(1.0, np.abs(ref).max()))
    fine.close()
    coarse.close()


def test_transfer_rejects_mismatched_plans():
    gs = ragged(np.float32)
    fine, coarse, pcal, pobs, desc, cd = _plans(gs, E.F32, 2, 4)
    with pytest.raises(E.EMDError, match="ceil"):
        E.restrict(fine, coarse, 2, 3, pcal)              # sizes do not match (2, 3)
    with pytest.raises(E.EMDError, match="fr and ft"):
        E.restrict(fine, coarse, 0, 4, pcal)
    other = E.Plan(cd, coarse.batch_len, E.SolverParams(precision=E.F64))
    with pytest.raises(E.EMDError, match="precision"):
        L = E._lib
        L.check(L.load().emd_restrict(fine.handle, other.handle, 2, 4, pcal.data_ptr(),
                                      other.empty().data_ptr(), None))
    fewer = E.Plan(cd[:-1], coarse.batch_len, E.SolverParams(precision=E.F32))
    with pytest.raises(E.EMDError, match="numbers of gathers"):
        E.restrict(fine, fewer, 2, 4, pcal)
    for pl in (fine, coarse, other, fewer):
        pl.close()


@pytest.mark.parametrize("coarse_ips", [0, 2])
@pytest.mark.parametrize("factors", [((1, 2),), ((2, 2), (1, 2))])
def test_multigrid_solve_reaches_the_cold_optimum(factors, coarse_ips):
    # FP64: the coarse levels only change where the fine solve starts (also when they
    # are solved by fixed-step PDHG, two iterations per sweep).  The stop rule
    # certifies feasibility, not optimality (on tiny random grids a 1e-6 residual can
    # leave the transport ~0.5 % above the optimum), so the two solves are compared
    # through their duality brackets: both bracket the same optimum, and their EMDs
    # differ by no more than the brackets allow
    gs = ragged(np.float64)
    p = E.SolverParams(precision=E.F64, tol_res=1e-6, max_iter=400000)
    plan, pcal, pobs, desc = make_plan(gs, p)
    mg = E.Multigrid(plan, factors, coarse_iters_per_sweep=coarse_ips)
    emd_w, phi_w, u_w, info_w, mass = mg.solve(pcal, pobs)
    s, mass = E.emd_decompose(plan, pcal, pobs)
    emd_c, phi_c, u_c, info_c = E.emd_pdhg_solve(plan, s, u=plan.empty(2), mass=mass)
    torch.cuda.synchronize()
    iw, ic = E.info_numpy(info_w), E.info_numpy(info_c)
    coarse_iters = [E.info_numpy(i)["iters"].tolist() for i in mg.last_info]
    log(f"  factors {factors}: coarse iterations {coarse_iters}, fine {iw['iters'].tolist()} "
        f"(cold {ic['iters'].tolist()})")
    assert np.all(iw["status"] == E.GATHER_STATUS.index("CONVERGED"))
    assert np.all(ic["status"] == E.GATHER_STATUS.index("CONVERGED"))
    ew, ec = emd_w.cpu().numpy(), emd_c.cpu().numpy()
    sol = {}
    for name, u, phi in (("warm", u_w, phi_w), ("cold", u_c, phi_c)):
        sol[name] = (unpack(u.cpu().numpy(), desc, 2), unpack(phi.cpu().numpy(), desc))
    for k, g in enumerate(gs):
        sk, _, _, _ = oracle.decompose(g.pcal, g.pobs, g.dx, g.dt)
        br = {}
        for name, (us, phis) in sol.items():
            lo, w, hi = transport_bounds(sk, us[k][0], us[k][1], phis[k], g.dx, g.dt)
            assert lo - (hi - w) <= w <= hi
            br[name] = (lo, w, hi)
        assert max(br["warm"][0], br["cold"][0]) <= min(br["warm"][2], br["cold"][2])
        allow = sum((hi - lo) / hi for lo, _, hi in br.values())
        assert abs(ew[k] / ec[k] - 1) <= allow + 1e-6, k
    mg.close()
    plan.close()


def test_multigrid_through_autograd():
    # seismic-like gathers, where the EMD at the 1e-5 residual is within ~1e-5 of the
    # optimum from any start (on random grids the stop rule is looser, see above)
    gs = to_precision([config2_gather(nr=20, nt=300, f_peak=4.0, dtype=np.float64),
                       config1_pairs([60], nt=257, dt=1.0 / 256)[0]], np.float32)
    p = E.SolverParams(precision=E.F32, tol_res=1e-5, max_iter=100000)
    plan, pcal, pobs, desc = make_plan(gs, p)
    mg = E.Multigrid(plan, ((1, 2),))
    x = pcal.clone().requires_grad_(True)
    emd = E.emd_misfit(x, pobs, plan, multigrid=mg)
    emd.sum().backward()
    s, mass = E.emd_decompose(plan, pcal, pobs)
    emd_c, _, _, _ = E.emd_pdhg_solve(plan, s, mass=mass)
    torch.cuda.synchronize()
    np.testing.assert_allclose(emd.detach().cpu().numpy(), emd_c.cpu().numpy(), rtol=2e-4)
    assert torch.isfinite(x.grad).all() and x.grad.abs().sum() > 0
    mg.close()
    plan.close()


def test_multigrid_with_mass_mode_none():
    # the fine problem as printed (no mass balancing, masses equal by construction);
    # the coarse level balances its block means and still supplies a usable start
    gs = to_precision([config2_gather(nr=20, nt=301, f_peak=4.0, dtype=np.float64)], np.float32)
    p = E.SolverParams(precision=E.F32, tol_res=1e-5, max_iter=100000, mass_mode=E.MASS_NONE,
                       mass_tol=1e-3)
    plan, pcal, pobs, desc = make_plan(gs, p)
    mg = E.Multigrid(plan, ((1, 4),))
    assert mg.levels[0][0].params.mass_mode == E.MASS_BALANCE
    emd_w, _, _, info_w, _ = mg.solve(pcal, pobs)
    s, mass = E.emd_decompose(plan, pcal, pobs)
    emd_c, _, _, info_c = E.emd_pdhg_solve(plan, s, mass=mass)
    torch.cuda.synchronize()
    iw, ic = E.info_numpy(info_w), E.info_numpy(info_c)
    log(f"  mass mode none: statuses {iw['status'].tolist()} / {ic['status'].tolist()}, "
        f"fine iterations {iw['iters'].tolist()} (cold {ic['iters'].tolist()})")
    np.testing.assert_array_equal(iw["status"], ic["status"])
    if ic["status"][0] == E.GATHER_STATUS.index("CONVERGED"):
        np.testing.assert_allclose(emd_w.cpu().numpy(), emd_c.cpu().numpy(), rtol=2e-4)
    mg.close()
    plan.close()


def test_fwi_loop_multigrid_then_warm_start():
    # the first evaluation of a batch starts from the coarse grid, later ones from the
    # previous evaluation's (u, phi) without touching the coarse level
    gs = to_precision([config2_gather(nr=24, nt=400, f_peak=4.0, dtype=np.float64),
                       config2_gather(seed=5, nr=16, nt=300, f_peak=4.0, dtype=np.float64)], np.float32)
    p = E.SolverParams(precision=E.F32, tol_res=1e-5, max_iter=100000)
    plan, pcal, pobs, desc = make_plan(gs, p)
    mg = E.Multigrid(plan, ((1, 2),))
    coarse = mg.levels[0][0]
    warm = E.WarmStart(plan)
    fine_cost, coarse_cost = [], []
    for step in range(3):
        x = (pcal * (1.0 - 0.02 * step)).contiguous().requires_grad_(True)
        emd = E.emd_misfit(x, pobs, plan, warm, mg)
        emd.sum().backward()
        torch.cuda.synchronize()
        fine_cost.append(plan.query()["last_cell_updates"])
        coarse_cost.append(coarse.query()["last_cell_updates"])
        assert torch.isfinite(emd).all() and torch.isfinite(x.grad).all() and warm.valid
    log(f"  fine cell updates {fine_cost}, coarse level's last solve {coarse_cost}")
    assert coarse_cost[0] > 0
    assert coarse_cost[1] == coarse_cost[0] and coarse_cost[2] == coarse_cost[0]   # not re-solved
    # for reference (not asserted): a cold solve of the last model; whether the warm
    # start is cheaper depends on the model step (for this 2 % rescaling of the
    # amplitudes it is not)
    s, mass = E.emd_decompose(plan, (pcal * 0.96).contiguous(), pobs)
    E.emd_pdhg_solve(plan, s, mass=mass)
    torch.cuda.synchronize()
    log(f"  cold solve of the last model: {plan.query()['last_cell_updates']}")
    mg.close()
    plan.close()


def test_multigrid_coarse_level_settings():
    # the coarse plans' stop rule is the fine one's times coarse_tol_factor and their
    # tiles are coarse_rows high; each level then stops at its own rule
    gs = to_precision([config2_gather(nr=24, nt=400, f_peak=4.0, dtype=np.float64),
                       config2_gather(seed=5, nr=16, nt=300, f_peak=4.0, dtype=np.float64)], np.float32)
    p = E.SolverParams(precision=E.F32, tol_res=1e-5, max_iter=100000)
    plan, pcal, pobs, desc = make_plan(gs, p)
    with pytest.raises(ValueError):
        E.Multigrid(plan, ((1, 2),), coarse_tol_factor=0.0)
    with pytest.raises(ValueError, match="one tile height per level"):
        E.Multigrid(plan, ((1, 2), (1, 2)), coarse_rows=[8])
    plain = E.Multigrid(plan, ((1, 2),), coarse_rows=None)
    q16 = plain.levels[0][0].query()
    assert q16["rows_per_tile"] == 16
    assert plain.levels[0][0].params.tol_res == p.tol_res
    plain.close()
    per_level = E.Multigrid(plan, ((1, 2), (1, 2)), coarse_rows=[12, 4])
    assert [cp.query()["rows_per_tile"] for cp, _, _ in per_level.levels] == [12, 4]
    per_level.close()
    # fixed-step coarse levels: plain PDHG, three iterations per sweep, the stop rule
    # every nine, the library's default tile height; the fine plan keeps its method
    with pytest.raises(ValueError, match="coarse_iters_per_sweep"):
        E.Multigrid(plan, ((1, 2),), coarse_iters_per_sweep=4)
    fx = E.Multigrid(plan, ((1, 2), (1, 2)), coarse_iters_per_sweep=3)
    for cp, _, _ in fx.levels:
        assert (cp.params.ls_mode, cp.params.iters_per_sweep, cp.params.check_every) == (E.LS_FIXED, 3, 9)
        assert cp.query()["rows_per_tile"] == 16
    assert plan.params.ls_mode == p.ls_mode
    emd_x, _, _, info_x, _ = fx.solve(pcal, pobs)
    emd_x = emd_x.clone()
    ls = E.Multigrid(plan, ((1, 2), (1, 2)))
    ref_emd, _, _, _, _ = ls.solve(pcal, pobs)
    torch.cuda.synchronize()
    ls.close()
    ix = E.info_numpy(info_x)
    assert np.all(ix["status"] == E.GATHER_STATUS.index("CONVERGED"))
    for li in fx.last_info:
        assert np.all(E.info_numpy(li)["rel_res"] <= 1e-5)
    # seismic-like gathers: at the 1e-5 rule the EMD hardly depends on the start
    np.testing.assert_allclose(emd_x.cpu().numpy(), ref_emd.cpu().numpy(), rtol=2e-4)
    fx.close()
    mg = E.Multigrid(plan, ((1, 2), (1, 2)), coarse_tol_factor=1.5)
    for cp, _, _ in mg.levels:
        assert cp.params.tol_res == pytest.approx(1.5e-5, rel=1e-15)
        assert cp.query()["rows_per_tile"] == 8
    # the shorter tiles' extra partial-sum slots are accounted for (the table itself is
    # padded to eight runs of whole blocks, so on gathers this small it keeps its length)
    q8 = mg.levels[0][0].query()
    assert q8["tiles"] >= q16["tiles"] and q8["workspace_bytes"] > q16["workspace_bytes"]
    emd, _, _, info, _ = mg.solve(pcal, pobs)
    torch.cuda.synchronize()
    conv = E.GATHER_STATUS.index("CONVERGED")
    for li in mg.last_info:
        ci = E.info_numpy(li)
        assert np.all(ci["status"] == conv) and np.all(ci["rel_res"] <= 1.5e-5)
    fi = E.info_numpy(info)
    log(f"  coarse iterations {[E.info_numpy(li)['iters'].tolist() for li in mg.last_info]}, "
        f"fine {fi['iters'].tolist()}, fine residuals {fi['rel_res'].tolist()}")
    assert np.all(fi["status"] == conv) and np.all(fi["rel_res"] <= 1e-5)
    assert torch.isfinite(emd).all()
    mg.close()
    plan.close()
