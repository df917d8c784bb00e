"""Host-side logic of the Python binding: every per-gather buffer handed to a kernel
(masses, EMD values, solve records, step schedules, upstream gradients) must be a
contiguous tensor of the expected type on the plan's device and large enough, or the
binding raises before anything reaches the library; and the residual-history ring is
unrolled into check order."""
from types import SimpleNamespace

import numpy as np
import pytest
import torch

import paper_1808_07284_amd.api as A


def _plan(device="cpu", ngather=3):
    return SimpleNamespace(device=torch.device(device), ngather=ngather)


def test_buffer_on_another_device_is_rejected():
    plan = _plan("cuda")
    with pytest.raises(ValueError, match="mass"):
        A._check_buf(plan, torch.zeros(9, dtype=torch.float64), "mass", torch.float64, 9)


def test_buffer_type_size_and_layout():
    plan = _plan()
    A._check_buf(plan, None, "emd_out", torch.float64, 3)  # optional
    A._check_buf(plan, torch.zeros(3, 3, dtype=torch.float64), "mass", torch.float64, 9)
    with pytest.raises(ValueError, match="float64"):
        A._check_buf(plan, torch.zeros(9, dtype=torch.float32), "mass", torch.float64, 9)
    with pytest.raises(ValueError, match="at least 9"):
        A._check_buf(plan, torch.zeros(8, dtype=torch.float64), "mass", torch.float64, 9)
    with pytest.raises(ValueError, match="contiguous"):
        A._check_buf(plan, torch.zeros(3, 6, dtype=torch.float64)[:, ::2], "mass", torch.float64, 9)


def test_solve_outputs():
    plan = _plan()
    ok_info = torch.zeros(3 * A.INFO_DTYPE.itemsize, dtype=torch.uint8)
    A._check_outputs(plan, torch.zeros(3, 3, dtype=torch.float64), torch.zeros(3, dtype=torch.float64), ok_info)
    with pytest.raises(ValueError, match="info_out"):
        A._check_outputs(plan, None, None, ok_info[:-1])
    with pytest.raises(ValueError, match="emd_out"):
        A._check_outputs(plan, None, torch.zeros(3, dtype=torch.float32), None)


def test_upstream_gradients_are_one_per_gather():
    plan = _plan()
    assert A._gbar(plan, None) is None
    g = A._gbar(plan, torch.tensor([1.0, 2.0, 3.0], dtype=torch.float32))
    assert g.dtype == torch.float64 and g.tolist() == [1.0, 2.0, 3.0]
    with pytest.raises(ValueError, match="gbar"):
        A._gbar(plan, torch.ones(2))


def test_residual_history_unrolls_the_ring():
    # checks c = 1..n land in slot (c - 1) % capacity; the unrolled history lists the
    # last min(n, capacity) checks in iteration order
    cap, ce = 4, 10
    rec = np.zeros(3, dtype=A.INFO_DTYPE)
    rec["iters"] = [70, 30, 0]  # 7 checks (wrapped), 3 checks, none
    ring = np.full((3, cap), np.nan)
    for g, n in enumerate((7, 3, 0)):
        for c in range(1, n + 1):
            ring[g, (c - 1) % cap] = 100 * g + c
    plan = SimpleNamespace(ngather=3, params=SimpleNamespace(check_every=ce), _hist=torch.from_numpy(ring))
    h = A.residual_history(plan, rec)
    assert h[0].tolist() == [4, 5, 6, 7]
    assert h[1].tolist() == [101, 102, 103]
    assert h[2].size == 0
    with pytest.raises(RuntimeError):
        A.residual_history(SimpleNamespace(ngather=1, params=plan.params, _hist=None), rec[:1])


def test_multigrid_arguments_are_checked_before_any_plan_is_built():
    # every bad setting raises before a coarse plan (and so the library) is touched
    fine = SimpleNamespace(params=A.SolverParams(), descs=[(8, 40, 1.0, 0.01, 0)], device=torch.device("cpu"))
    with pytest.raises(ValueError, match="coarse_tol_factor"):
        A.Multigrid(fine, ((1, 2),), coarse_tol_factor=0.0)
    with pytest.raises(ValueError, match="coarse_iters_per_sweep"):
        A.Multigrid(fine, ((1, 2),), coarse_iters_per_sweep=1)
    with pytest.raises(ValueError, match="coarse_rows must be"):
        A.Multigrid(fine, ((1, 2),), coarse_rows="tall")
    with pytest.raises(ValueError, match="one tile height per level"):
        A.Multigrid(fine, ((1, 2), (1, 2)), coarse_rows=[8, 8, 8])
