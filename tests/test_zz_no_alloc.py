"""The allocation-free decompose (emd_decompose_noalloc) against emd_decompose on a
plan: same inputs, two calls in a row on the library's static scratch array, the
first with the largest batch it takes (64 gathers), the second with a smaller one."""
import numpy as np
import pytest

from gpu_util import log, make_plan, to_precision
from synth import config1_pairs, config2_gather, config3_batch, pack_batch, random_small_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1808_07284_amd as E  # noqa: E402


def _small_batch():
    return [config2_gather(nr=40, nt=530, f_peak=3.0, dtype=np.float64), random_small_pair(13, 301, 1),
            random_small_pair(5, 9, 2), config1_pairs([60], nt=257, dt=1.0 / 256)[0],
            random_small_pair(7, 1, 3), random_small_pair(3, 250, 4, balanced=False)]


def _check(gs, precision, mode):
    dtype = np.float64 if precision == E.F64 else np.float32
    gs = to_precision(gs, dtype)
    p = E.SolverParams(precision=precision, mass_mode=mode)
    plan, pcal, pobs, desc = make_plan(gs, p)
    f_ref, g_ref = plan.empty(), plan.empty()
    s_ref, m_ref = E.emd_decompose(plan, pcal, pobs, f_out=f_ref, g_out=g_ref)
    s = torch.full_like(s_ref, float("nan"))
    f, g = torch.full_like(s_ref, float("nan")), torch.full_like(s_ref, float("nan"))
    m = torch.full((len(gs), 3), float("nan"), dtype=torch.float64, device=plan.device)
    E.emd_decompose_noalloc(desc, pcal, pobs, s, m, precision=precision, mass_mode=mode, f_out=f, g_out=g)
    torch.cuda.synchronize()
    s_ref, m_ref, s, m = s_ref.cpu().numpy(), m_ref.cpu().numpy(), s.cpu().numpy(), m.cpu().numpy()
    # f and g are elementwise: identical; the FP64 sums are taken in another order
    np.testing.assert_array_equal(f.cpu().numpy(), f_ref.cpu().numpy())
    np.testing.assert_array_equal(g.cpu().numpy(), g_ref.cpu().numpy())
    np.testing.assert_allclose(m[:, :2], m_ref[:, :2], rtol=1e-12, atol=0)
    tol = 1e-12 if precision == E.F64 else 1e-6
    for k, (nr, nt, _, _, off) in enumerate(desc):
        d = gs[k].pcal.astype(np.float64) - gs[k].pobs
        assert abs(m[k, 2] - m_ref[k, 2]) <= 1e-13 * np.abs(d).mean()
        a, b = s[off:off + nr * nt], s_ref[off:off + nr * nt]
        scale = max(np.abs(b).max(), 1e-300)
        np.testing.assert_allclose(a, b, rtol=0, atol=tol * scale * 4)
    plan.close()
    return len(gs)


@pytest.mark.parametrize("precision", [E.F32, E.F64])
@pytest.mark.parametrize("mode", [E.MASS_BALANCE, E.MASS_UNIT, E.MASS_NONE])
def test_noalloc_decompose_matches_the_plan_decompose(precision, mode):
    # call 1: the 64-gather benchmark batch (the most gathers the scratch array
    # holds); call 2: six ragged gathers, on the scratch the first call left behind
    big = config3_batch()
    log(f"noalloc decompose precision={precision} mode={mode}: 64 gathers, then 6")
    assert _check(big, precision, mode) == E.api.NOALLOC_MAX_GATHERS
    assert _check(_small_batch(), precision, mode) == 6


def test_noalloc_decompose_rejects_more_gathers_than_its_scratch_holds():
    gs = to_precision([random_small_pair(3, 8, k) for k in range(65)], np.float32)
    pcal, pobs, desc = pack_batch(gs, np.float32)
    pc = torch.from_numpy(pcal).cuda()
    po = torch.from_numpy(pobs).cuda()
    s = torch.empty_like(pc)
    m = torch.empty(65, 3, dtype=torch.float64, device=pc.device)
    with pytest.raises(E.EMDError, match="static scratch"):
        E.emd_decompose_noalloc(desc, pc, po, s, m)
    # 64 of them pass
    E.emd_decompose_noalloc(desc[:64], pc, po, s, m)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(m[:64].cpu().numpy()))
