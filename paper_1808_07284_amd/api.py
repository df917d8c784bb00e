"""Python binding of the C ABI (argument marshalling only; every step runs in the
HIP kernels of libemd_mi355x.so).

Tensors are torch device tensors holding a batch in the ABI layout: gather g is a
dense [nr][nt] block at element ``offset`` of a flat buffer (see ``pack_batch`` in
the synthetic-data package for one way to build it).  Work is enqueued on torch's
current stream of the tensors' device.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import hashlib
import json
import os
from dataclasses import dataclass, fields
from typing import Sequence

import numpy as np
import torch

from . import _lib as L

INFO_DTYPE = np.dtype([("status", "<i4"), ("iters", "<i4"), ("ls_trials", "<i4"), ("pad", "<i4"),
                       ("rel_res", "<f8"), ("emd", "<f8"), ("transport", "<f8"), ("alpha", "<f8"),
                       ("primal", "<f8")])


@dataclass
class SolverParams:
    """Mirror of emd_params; the defaults are the paper's constants (Section 2.2:
    eps = 1e-4; Algorithm 1: xi = 0.5, zeta = 0.99, delta = 1e5)."""
    eps: float = 1e-4
    xi: float = 0.5
    zeta: float = 0.99
    delta: float = 1e5
    alpha1: float = 0.0
    alpha_max_factor: float = 1e6
    tol_res: float = 1e-5
    mass_tol: float = 1e-6
    max_iter: int = 100000
    check_every: int = 10
    max_ls_trials: int = 40
    ls_mode: int = L.LS_L2
    mass_mode: int = L.MASS_BALANCE
    precision: int = L.F32
    sweeps_per_sync: int = 64
    iters_per_sweep: int = 1

    def to_c(self) -> L.Params:
        p = L.Params()
        for f in fields(self):
            setattr(p, f.name, getattr(self, f.name))
        return p

    @classmethod
    def library_default(cls) -> "SolverParams":
        p = L.Params()
        L.check(L.load().emd_params_default(C.byref(p)))
        return cls(**{f.name: getattr(p, f.name) for f in fields(cls)})

    @property
    def dtype(self) -> torch.dtype:
        return torch.float64 if self.precision == L.F64 else torch.float32


# revision of the autotuner's candidate heights and timing rule: a cached choice made
# by another revision is not reused
AUTOTUNE_REVISION = 2


def autotune_key(arch: str, rocm: str | None, precision: int, sizes) -> str:
    """Cache key of a tile-height choice: device architecture, ROCm version, precision,
    the (nr, nt) of every gather in batch order and the autotuner's revision."""
    h = hashlib.sha256(json.dumps([[int(a), int(b)] for a, b in sizes]).encode()).hexdigest()[:24]
    return (f"{arch}|rocm {rocm}|{'f64' if precision == L.F64 else 'f32'}|{len(sizes)} gathers|{h}"
            f"|tuner {AUTOTUNE_REVISION}")


def _read_cache(path: str) -> dict:
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """An emd_plan: workspace and tiling for one batch of gathers.

    descs: sequence of (nr, nt, dx, dt, offset); batch_len: elements per batch buffer."""

    def __init__(self, descs, batch_len: int, params: SolverParams | None = None,
                 device: int | torch.device | None = None):
        self.params = params or SolverParams()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        arr = (L.GatherDesc * len(descs))()
        for k, (nr, nt, dx, dt, off) in enumerate(descs):
            arr[k] = L.GatherDesc(int(nr), int(nt), float(dx), float(dt), int(off))
        self.descs = [tuple(d) for d in descs]
        self.ngather = len(descs)
        self.batch_len = int(batch_len)
        self._h = C.c_void_p()
        lib = L.load()
        with torch.cuda.device(self.device):
            L.check(lib.emd_plan_create(arr, self.ngather, self.batch_len,
                                        C.byref(self.params.to_c()), C.byref(self._h)))

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("plan is closed")
        return self._h

    def close(self):
        if self._h:
            L.load().emd_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: SolverParams):
        with torch.cuda.device(self.device):
            L.check(L.load().emd_plan_set_params(self.handle, C.byref(params.to_c())))
        self.params = params

    def set_tiling(self, rows_per_tile: int):
        with torch.cuda.device(self.device):
            L.check(L.load().emd_plan_set_tiling(self.handle, int(rows_per_tile)))

    def set_gather_tiling(self, rows):
        """Tile height (receiver rows per wavefront tile) of each gather."""
        arr = (C.c_int32 * self.ngather)(*[int(r) for r in rows])
        with torch.cuda.device(self.device):
            L.check(L.load().emd_plan_set_gather_tiling(self.handle, arr))

    def gather_tiling(self) -> list:
        arr = (C.c_int32 * self.ngather)()
        L.check(L.load().emd_plan_get_gather_tiling(self.handle, arr))
        return list(arr)

    def autotune(self, s, sweeps: int = 0, cache: str | None = None) -> list:
        """Pick tile heights per size bucket by timing short fixed-step solves from the
        source s (the workspace is overwritten; the parameters are kept).  Returns the
        chosen per-gather heights.

        cache: a JSON file (default: the EMD_AUTOTUNE_CACHE environment variable, none if
        unset) of earlier choices keyed by device architecture, ROCm version, precision
        and the batch's gather sizes; a hit applies the stored heights without timing."""
        self._check(s, "s")
        path = cache if cache is not None else os.environ.get("EMD_AUTOTUNE_CACHE")
        key = None
        if path:
            props = torch.cuda.get_device_properties(self.device)
            key = autotune_key(getattr(props, "gcnArchName", props.name), torch.version.hip,
                               self.params.precision, [(d[0], d[1]) for d in self.descs])
            entries = _read_cache(path)
            rows = entries.get(key)
            if rows is not None and len(rows) == self.ngather:
                self.set_gather_tiling(rows)
                return self.gather_tiling()
        with torch.cuda.device(self.device):
            L.check(L.load().emd_plan_autotune(self.handle, _ptr(s), int(sweeps), _stream(self.device)))
        rows = self.gather_tiling()
        if path:
            entries = _read_cache(path)
            entries[key] = rows
            tmp = f"{path}.{os.getpid()}.tmp"
            with open(tmp, "w") as fh:
                json.dump(entries, fh)
            os.replace(tmp, path)
        return rows

    def set_history(self, capacity: int):
        """Record every gather's relative residual at each stop-rule check of later
        solves in a ring of the last `capacity` checks (0 turns it off).  Returns the
        float64 [ngather, capacity] device buffer (filled with NaN), or None; read it
        with residual_history()."""
        buf = None
        if capacity > 0:
            buf = torch.full((self.ngather, int(capacity)), float("nan"), dtype=torch.float64,
                             device=self.device)
        with torch.cuda.device(self.device):
            L.check(L.load().emd_plan_set_history(self.handle, _ptr(buf), int(capacity) if buf is not None else 0))
        self._hist = buf  # the library writes into it: keep it alive with the plan
        return buf

    def query(self) -> dict:
        s = L.PlanStats()
        L.check(L.load().emd_plan_query(self.handle, C.byref(s)))
        return {f[0]: getattr(s, f[0]) for f in L.PlanStats._fields_}

    def empty(self, *lead) -> torch.Tensor:
        return torch.zeros(*lead, self.batch_len, dtype=self.params.dtype, device=self.device)

    def _check(self, t, name, lead=()):
        if t is None:
            return
        if t.device != self.device or t.dtype != self.params.dtype or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous {self.params.dtype} tensor on "
                             f"{self.device}, got {t.dtype} on {t.device}")
        if t.numel() != int(np.prod(lead, dtype=np.int64)) * self.batch_len:
            raise ValueError(f"{name}: expected {lead + (self.batch_len,)} elements")


def _check_buf(plan: Plan, t, name: str, dtype: torch.dtype, numel: int):
    """A per-gather buffer the kernels read or write (masses, EMD values, solve info,
    step schedules): a contiguous tensor of `dtype` on the plan's device holding at
    least `numel` elements (None passes: the argument is optional)."""
    if t is None:
        return
    if t.device != plan.device or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {dtype} tensor on {plan.device}, "
                         f"got {t.dtype} on {t.device}")
    if t.numel() < numel:
        raise ValueError(f"{name}: expected at least {numel} elements, got {t.numel()}")


def _check_outputs(plan: Plan, mass, emd_out, info_out):
    _check_buf(plan, mass, "mass", torch.float64, 3 * plan.ngather)
    _check_buf(plan, emd_out, "emd_out", torch.float64, plan.ngather)
    _check_buf(plan, info_out, "info_out", torch.uint8, plan.ngather * INFO_DTYPE.itemsize)


def _gbar(plan: Plan, gbar):
    """Upstream gradients per gather as a float64 device vector (None: all 1)."""
    if gbar is None:
        return None
    gbar = gbar.to(device=plan.device, dtype=torch.float64).contiguous()
    if gbar.numel() != plan.ngather:
        raise ValueError(f"gbar: expected {plan.ngather} values, got {gbar.numel()}")
    return gbar


def emd_decompose(plan: Plan, pcal, pobs, s_out=None, f_out=None, g_out=None, mass_out=None):
    """Mainini recombination and mass normalisation (Section 2.1).
    Returns (s, mass) with mass[g] = (M_f, M_g, mean(Pcal - Pobs))."""
    s_out = plan.empty() if s_out is None else s_out
    mass_out = (torch.empty(plan.ngather, 3, dtype=torch.float64, device=plan.device)
                if mass_out is None else mass_out)
    for t, n in ((pcal, "pcal"), (pobs, "pobs"), (s_out, "s_out"), (f_out, "f_out"), (g_out, "g_out")):
        plan._check(t, n)
    _check_buf(plan, mass_out, "mass_out", torch.float64, 3 * plan.ngather)
    with torch.cuda.device(plan.device):
        L.check(L.load().emd_decompose(plan.handle, _ptr(pcal), _ptr(pobs), _ptr(s_out), _ptr(f_out),
                                       _ptr(g_out), _ptr(mass_out), _stream(plan.device)))
    return s_out, mass_out


NOALLOC_MAX_GATHERS = 64


def emd_decompose_noalloc(descs, pcal, pobs, s_out, mass_out, precision=L.F32,
                          mass_mode=L.MASS_BALANCE, f_out=None, g_out=None):
    """emd_decompose without a plan (the library allocates nothing; at most 64
    gathers): descs as for Plan, every buffer caller-owned on the current device.
    Returns (s_out, mass_out)."""
    dtype = torch.float64 if precision == L.F64 else torch.float32
    dev = pcal.device
    need = max(int(off) + int(nr) * int(nt) for nr, nt, _, _, off in descs)
    for t_, n in ((pcal, "pcal"), (pobs, "pobs"), (s_out, "s_out"), (f_out, "f_out"), (g_out, "g_out")):
        if t_ is None:
            continue
        if t_.device != dev or t_.dtype != dtype or not t_.is_contiguous() or t_.numel() < need:
            raise ValueError(f"{n}: expected a contiguous {dtype} tensor on {dev} of at least {need} elements")
    if (mass_out.device != dev or mass_out.dtype != torch.float64 or not mass_out.is_contiguous()
            or mass_out.numel() < 3 * len(descs)):
        raise ValueError(f"mass_out: expected a contiguous float64 tensor of {3 * len(descs)} elements on {dev}")
    arr = (L.GatherDesc * len(descs))()
    for k, (nr, nt, dx, dt, off) in enumerate(descs):
        arr[k] = L.GatherDesc(int(nr), int(nt), float(dx), float(dt), int(off))
    with torch.cuda.device(dev):
        L.check(L.load().emd_decompose_noalloc(arr, len(descs), int(precision), int(mass_mode), _ptr(pcal),
                                               _ptr(pobs), _ptr(s_out), _ptr(f_out), _ptr(g_out),
                                               _ptr(mass_out), _stream(dev)))
    return s_out, mass_out


def emd_pdhg_solve(plan: Plan, s, phi=None, u=None, warm_start=False, mass=None, emd_out=None,
                   info_out=None):
    """PDHG with linesearch for every gather (Algorithm 1).
    Returns (emd [ngather] float64, phi, u or None, info uint8 [ngather * INFO_DTYPE.itemsize])."""
    phi = plan.empty() if phi is None else phi
    emd_out = (torch.empty(plan.ngather, dtype=torch.float64, device=plan.device)
               if emd_out is None else emd_out)
    info_out = (torch.empty(plan.ngather * INFO_DTYPE.itemsize, dtype=torch.uint8, device=plan.device)
                if info_out is None else info_out)
    plan._check(s, "s")
    plan._check(phi, "phi")
    plan._check(u, "u", (2,))
    _check_outputs(plan, mass, emd_out, info_out)
    with torch.cuda.device(plan.device):
        L.check(L.load().emd_pdhg_solve(plan.handle, _ptr(s), _ptr(u), _ptr(phi), int(bool(warm_start)),
                                        _ptr(mass), _ptr(emd_out), _ptr(info_out),
                                        _stream(plan.device)))
    return emd_out, phi, u, info_out


def emd_pdhg_solve_replay(plan: Plan, s, alpha, phi=None, u=None, warm_start=False, emd_out=None,
                          info_out=None):
    """The solve with the accepted steps alpha [ngather, ld] (float64) replayed."""
    phi = plan.empty() if phi is None else phi
    emd_out = (torch.empty(plan.ngather, dtype=torch.float64, device=plan.device)
               if emd_out is None else emd_out)
    info_out = (torch.empty(plan.ngather * INFO_DTYPE.itemsize, dtype=torch.uint8, device=plan.device)
                if info_out is None else info_out)
    if alpha.dtype != torch.float64 or alpha.dim() != 2 or alpha.shape[0] != plan.ngather:
        raise ValueError("alpha must be a float64 [ngather, ld] tensor")
    alpha = alpha.contiguous()
    _check_buf(plan, alpha, "alpha", torch.float64, alpha.numel())
    plan._check(s, "s")
    plan._check(phi, "phi")
    plan._check(u, "u", (2,))
    _check_outputs(plan, None, emd_out, info_out)
    with torch.cuda.device(plan.device):
        L.check(L.load().emd_pdhg_solve_replay(plan.handle, _ptr(s), _ptr(u), _ptr(phi),
                                               int(bool(warm_start)), _ptr(alpha),
                                               int(alpha.shape[1]), _ptr(emd_out), _ptr(info_out),
                                               _stream(plan.device)))
    return emd_out, phi, u, info_out


def solver_state(plan: Plan):
    """Checkpoint of the plan's last solve: per gather the last accepted step alpha,
    theta, the iteration count and backtracking trials (with that solve's u and phi)."""
    arr = (L.GatherState * plan.ngather)()
    L.check(L.load().emd_solver_state(plan.handle, arr))
    return arr


def emd_pdhg_solve_resume(plan: Plan, s, state, u, phi, mass=None, emd_out=None, info_out=None):
    """Continue a solve from a checkpoint (solver_state plus the u, phi it returned);
    u and phi are updated in place.  K iterations resumed to 2K reproduce a single
    solve of 2K bitwise."""
    emd_out = (torch.empty(plan.ngather, dtype=torch.float64, device=plan.device)
               if emd_out is None else emd_out)
    info_out = (torch.empty(plan.ngather * INFO_DTYPE.itemsize, dtype=torch.uint8, device=plan.device)
                if info_out is None else info_out)
    plan._check(s, "s")
    plan._check(phi, "phi")
    plan._check(u, "u", (2,))
    _check_outputs(plan, mass, emd_out, info_out)
    if len(state) != plan.ngather:
        raise ValueError(f"state: expected {plan.ngather} gather states, got {len(state)}")
    with torch.cuda.device(plan.device):
        L.check(L.load().emd_pdhg_solve_resume(plan.handle, _ptr(s), _ptr(u), _ptr(phi), state, _ptr(mass),
                                               _ptr(emd_out), _ptr(info_out), _stream(plan.device)))
    return emd_out, phi, u, info_out


def emd_adjoint_source(plan: Plan, phi, pcal=None, pobs=None, mass=None, gbar=None, psi_out=None):
    """Adjoint source psi = d EMD / d Pcal (Section 2.3), scaled by gbar [ngather]."""
    psi_out = plan.empty() if psi_out is None else psi_out
    for t, n in ((phi, "phi"), (pcal, "pcal"), (pobs, "pobs"), (psi_out, "psi_out")):
        plan._check(t, n)
    _check_buf(plan, mass, "mass", torch.float64, 3 * plan.ngather)
    gbar = _gbar(plan, gbar)
    with torch.cuda.device(plan.device):
        L.check(L.load().emd_adjoint_source(plan.handle, _ptr(phi), _ptr(pcal), _ptr(pobs), _ptr(mass),
                                            _ptr(gbar), _ptr(psi_out), _stream(plan.device)))
    return psi_out


def lsd_misfit(plan: Plan, pcal, pobs, gbar=None, value_out=None, psi_out=None, with_adjoint=True):
    """Least-squares misfit 1/2 dx dt sum (Pcal - Pobs)^2 per gather (Section 2.1) and its
    adjoint source gbar dx dt (Pcal - Pobs) (Section 2.3).  Returns (value [ngather] float64,
    psi or None)."""
    if with_adjoint and psi_out is None:
        psi_out = plan.empty()
    for t, n in ((pcal, "pcal"), (pobs, "pobs"), (psi_out, "psi_out")):
        plan._check(t, n)
    value_out = (torch.empty(plan.ngather, dtype=torch.float64, device=plan.device)
                 if value_out is None else value_out)
    _check_buf(plan, value_out, "value_out", torch.float64, plan.ngather)
    gbar = _gbar(plan, gbar)
    with torch.cuda.device(plan.device):
        L.check(L.load().emd_lsd_misfit(plan.handle, _ptr(pcal), _ptr(pobs), _ptr(gbar), _ptr(value_out),
                                        _ptr(psi_out), _stream(plan.device)))
    return value_out, psi_out


def coarse_descs(descs, fr: int, ft: int):
    """Descriptors of the coarse grid that groups fr receivers by ft samples: sizes
    ceil(nr/fr) x ceil(nt/ft), spacings fr dx and ft dt, gathers packed back to back.
    Returns (descs, batch_len)."""
    out, off = [], 0
    for nr, nt, dx, dt, _ in descs:
        nrc, ntc = -(-int(nr) // fr), -(-int(nt) // ft)
        out.append((nrc, ntc, float(dx) * fr, float(dt) * ft, off))
        off += nrc * ntc
    return out, off


def restrict(fine: Plan, coarse: Plan, fr: int, ft: int, x, out=None):
    """Block means of a fine batch field on the coarse plan's grid (emd_restrict)."""
    fine._check(x, "x")
    out = coarse.empty() if out is None else out
    coarse._check(out, "out")
    with torch.cuda.device(fine.device):
        L.check(L.load().emd_restrict(fine.handle, coarse.handle, int(fr), int(ft), _ptr(x), _ptr(out),
                                      _stream(fine.device)))
    return out


def prolong(coarse: Plan, fine: Plan, fr: int, ft: int, u_c, phi_c, u_out=None, phi_out=None):
    """Bilinear prolongation of a coarse (u, phi) to the fine plan's grid, each field
    on its own staggering (emd_prolong).  Returns (u, phi)."""
    coarse._check(u_c, "u_c", (2,))
    coarse._check(phi_c, "phi_c")
    u_out = fine.empty(2) if u_out is None else u_out
    phi_out = fine.empty() if phi_out is None else phi_out
    fine._check(u_out, "u_out", (2,))
    fine._check(phi_out, "phi_out")
    with torch.cuda.device(fine.device):
        L.check(L.load().emd_prolong(coarse.handle, fine.handle, int(fr), int(ft), _ptr(u_c), _ptr(phi_c),
                                     _ptr(u_out), _ptr(phi_out), _stream(fine.device)))
    return u_out, phi_out


class Multigrid:
    """Coarse-to-fine solve (the multi-grid strategy of Section 2.2; Section 3.3
    resamples each shot and interpolates the coarse solution back).  `factors` lists,
    from the fine plan down, how each coarser level groups the receivers and samples
    of the level above it.  The data are restricted level by level (block means),
    the coarsest level is solved cold, and each solution, prolonged bilinearly
    (u and phi), starts the solve of the next finer level; the fine solve itself is
    left to the caller, who warm-starts it from (u, phi) written by start().  The
    coarse plans are built once, with the fine plan's parameters unless given; a
    coarse level never uses mass mode `none` (block means over the ragged last
    blocks shift the two masses slightly, and a coarse level only supplies a start),
    it balances the masses instead.  `coarse_rows` is the tile height of the coarse
    plans, one height for all or one per level in the order of `factors` (None: the
    library's default; "auto": 8 rows, or the default 16 for fixed-step levels): a
    coarse batch is a few times smaller than the fine one, so more of its sweeps run
    with only its slowest gathers left, and there a shorter tile gives more,
    shorter-lived waves.  `coarse_tol_factor` scales the coarse levels' stop rule
    (tol_res) against the one of their parameters: a coarse level only supplies a
    start, which the fine solve then takes to its own rule.  `coarse_iters_per_sweep`
    = K (2 or 3) solves the coarse levels by plain PDHG with the fixed steps of
    Section 2.2, K iterations per pass over the fields (stop rule checked every 3K
    iterations), whatever method the fine plan uses: a cheaper start."""

    def __init__(self, plan: Plan, factors=((1, 4),), params: SolverParams | None = None,
                 coarse_rows: int | Sequence[int] | str | None = "auto", coarse_tol_factor: float = 1.0,
                 coarse_iters_per_sweep: int = 0):
        self.fine = plan
        self.levels = []  # (coarse plan, fr, ft), finest first
        prm = params or plan.params
        if prm.mass_mode == L.MASS_NONE:
            prm = dataclasses.replace(prm, mass_mode=L.MASS_BALANCE)
        if not coarse_tol_factor > 0:
            raise ValueError("coarse_tol_factor must be > 0")
        prm = dataclasses.replace(prm, tol_res=prm.tol_res * float(coarse_tol_factor))
        k = int(coarse_iters_per_sweep)
        if k:
            if k not in (2, 3):
                raise ValueError("coarse_iters_per_sweep must be 0, 2 or 3")
            prm = dataclasses.replace(prm, ls_mode=L.LS_FIXED, iters_per_sweep=k, check_every=3 * k)
        if isinstance(coarse_rows, str):
            if coarse_rows != "auto":
                raise ValueError('coarse_rows must be a height, a list of heights, None or "auto"')
            coarse_rows = None if k else 8
        descs = plan.descs
        factors = list(factors)
        if coarse_rows is None or isinstance(coarse_rows, int):
            rows = [coarse_rows] * len(factors)
        else:
            rows = list(coarse_rows)
            if len(rows) != len(factors):
                raise ValueError("coarse_rows needs one tile height per level")
        for (fr, ft), r in zip(factors, rows):
            cd, n = coarse_descs(descs, int(fr), int(ft))
            cp = Plan(cd, n, prm, device=plan.device)
            if r:
                cp.set_tiling(int(r))
            self.levels.append((cp, int(fr), int(ft)))
            descs = cd
        self.last_info = []  # per level, coarsest first: the solve info of the last start()

    def close(self):
        for cp, _, _ in self.levels:
            cp.close()

    def start(self, pcal, pobs, u, phi):
        """Solve the coarse levels for (pcal, pobs) and write the prolonged start of the
        fine solve into u ([2, N]) and phi ([N])."""
        data, finer = [], self.fine
        pc, po = pcal, pobs
        for cp, fr, ft in self.levels:
            pc, po = restrict(finer, cp, fr, ft, pc), restrict(finer, cp, fr, ft, po)
            data.append((pc, po))
            finer = cp
        u_l = phi_l = None
        self.last_info = []
        for lvl in range(len(self.levels) - 1, -1, -1):
            cp, fr, ft = self.levels[lvl]
            s, mass = emd_decompose(cp, *data[lvl])
            warm = u_l is not None
            u_c = u_l if warm else cp.empty(2)
            phi_c = phi_l if warm else cp.empty()
            _, phi_c, u_c, info = emd_pdhg_solve(cp, s, phi=phi_c, u=u_c, warm_start=warm, mass=mass)
            self.last_info.append(info)
            finer = self.fine if lvl == 0 else self.levels[lvl - 1][0]
            if lvl == 0:
                prolong(cp, finer, fr, ft, u_c, phi_c, u, phi)
            else:
                u_l, phi_l = prolong(cp, finer, fr, ft, u_c, phi_c)
        return u, phi

    def solve(self, pcal, pobs, emd_out=None, info_out=None):
        """decompose -> coarse levels -> fine solve warm-started from them.
        Returns (emd, phi, u, info, mass) of the fine plan."""
        s, mass = emd_decompose(self.fine, pcal, pobs)
        u, phi = self.fine.empty(2), self.fine.empty()
        self.start(pcal, pobs, u, phi)
        emd, phi, u, info = emd_pdhg_solve(self.fine, s, phi=phi, u=u, warm_start=True, mass=mass,
                                           emd_out=emd_out, info_out=info_out)
        return emd, phi, u, info, mass


def residual_history(plan: Plan, info) -> list:
    """Per gather, the relative residuals of the last solve's stop-rule checks in
    iteration order (the ring of Plan.set_history unrolled; at most its capacity,
    the latest checks).  info: that solve's info records."""
    hist = getattr(plan, "_hist", None)
    if hist is None:
        raise RuntimeError("the plan records no residual history (Plan.set_history)")
    rec = info_numpy(info) if isinstance(info, torch.Tensor) else info
    h = hist.cpu().numpy()
    cap = h.shape[1]
    out = []
    for g in range(plan.ngather):
        n = int(rec["iters"][g]) // plan.params.check_every
        first = max(n - cap, 0)
        out.append(np.array([h[g, c % cap] for c in range(first, n)]))
    return out


@dataclass
class Resolved:
    """Outcome of resolve_failed: the merged per-gather EMD and solve records, the
    indices of the gathers solved again, and the FP64 plan of those gathers with its
    potential and masses (for emd_adjoint_source on them)."""
    emd: torch.Tensor
    info: np.ndarray
    indices: list
    plan: "Plan | None" = None
    phi: "torch.Tensor | None" = None
    mass: "torch.Tensor | None" = None


FAILED = ("MAX_ITER", "LS_FAIL", "NONFINITE")


def resolve_failed(plan: Plan, pcal, pobs, emd, info, statuses=FAILED,
                   params: SolverParams | None = None) -> Resolved:
    """Solve again, in FP64 throughout, the gathers of a solve whose status is one of
    `statuses` (by name; by default those that stopped without meeting the stop rule).
    FP32 fields cannot take the residual much below 1e-7, and their rounding can stall
    the linesearch; the FP64 solve has neither limit.  The gathers are packed into a
    plan of their own (params: the batch plan's, in FP64, unless given) and solved by
    the same kernels; their EMD values and records replace those of the batch solve.
    Gathers with other statuses (converged, zero source, mass imbalance) keep theirs."""
    rec = (info_numpy(info) if isinstance(info, torch.Tensor) else np.asarray(info)).copy()
    codes = [L.GATHER_STATUS.index(n) for n in statuses]
    idx = [g for g in range(plan.ngather) if int(rec["status"][g]) in codes]
    out = emd.detach().clone()
    if not idx:
        return Resolved(out, rec, idx)
    descs, off = [], 0
    for g in idx:
        nr, nt, dx, dt, _ = plan.descs[g]
        descs.append((nr, nt, dx, dt, off))
        off += int(nr) * int(nt)
    prm = dataclasses.replace(params or plan.params, precision=L.F64)
    sub = Plan(descs, off, prm, device=plan.device)

    def pack(x):
        plan._check(x, "pcal/pobs")
        parts = []
        for g in idx:
            nr, nt, _, _, o = plan.descs[g]
            parts.append(x.detach()[int(o):int(o) + int(nr) * int(nt)])
        return torch.cat(parts).to(torch.float64).contiguous()

    s, mass = emd_decompose(sub, pack(pcal), pack(pobs))
    e, phi, _, inf = emd_pdhg_solve(sub, s, mass=mass)
    r = info_numpy(inf)
    out[idx] = e.to(out.dtype)
    for k, g in enumerate(idx):
        rec[g] = r[k]
    return Resolved(out, rec, idx, sub, phi, mass)


def info_numpy(info: torch.Tensor) -> np.ndarray:
    """Per-gather emd_solve_info records as a numpy structured array."""
    return np.frombuffer(info.cpu().numpy().tobytes(), dtype=INFO_DTYPE)


class WarmStart:
    """Solver state carried between misfit evaluations of one batch (the evaluations
    of an FWI loop): the flux u and potential phi of the last solve.  Each solve
    starts from them and overwrites them; the first one starts cold."""

    def __init__(self, plan: Plan):
        self.u = plan.empty(2)
        self.phi = plan.empty()
        self.valid = False

    def reset(self):
        self.valid = False


class EMDMisfit(torch.autograd.Function):
    """EMD misfit of a batch: forward = decompose + PDHG solve, returning the EMD of
    every gather; backward = the hand-written adjoint-source kernel (the dual
    potential chained through the normalisation, Section 2.3).  No gradient flows
    to the observed data."""

    @staticmethod
    def forward(ctx, pcal, pobs, plan: Plan, warm: WarmStart | None = None,
                multigrid: "Multigrid | None" = None):
        s, mass = emd_decompose(plan, pcal, pobs)
        if warm is None and multigrid is None:
            emd, phi, _, info = emd_pdhg_solve(plan, s, mass=mass)
        else:
            u0 = warm.u if warm is not None else plan.empty(2)
            phi0 = warm.phi if warm is not None else plan.empty()
            started = warm is not None and warm.valid
            if not started and multigrid is not None:
                multigrid.start(pcal, pobs, u0, phi0)
                started = True
            emd, phi, _, info = emd_pdhg_solve(plan, s, phi=phi0, u=u0, warm_start=started, mass=mass)
            if warm is not None:
                warm.valid = True
                phi = phi.clone()  # the state moves on with the next evaluation
        ctx.plan = plan
        ctx.info = info
        ctx.save_for_backward(phi, pcal, pobs, mass)
        return emd.clone()

    @staticmethod
    def backward(ctx, grad_out):
        phi, pcal, pobs, mass = ctx.saved_tensors
        psi = emd_adjoint_source(ctx.plan, phi, pcal, pobs, mass, gbar=grad_out)
        return psi, None, None, None, None


def emd_misfit(pcal, pobs, plan: Plan, warm: WarmStart | None = None,
               multigrid: Multigrid | None = None):
    """EMD of every gather of the batch, differentiable with respect to pcal.  With a
    WarmStart, the solve starts from the previous evaluation's flux and potential;
    with a Multigrid (and no previous evaluation), from its coarse solution."""
    return EMDMisfit.apply(pcal, pobs, plan, warm, multigrid)
