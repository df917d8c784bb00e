"""Seeded synthetic seismograms with the shape class of the paper's workloads.

Every generator returns ``Gather`` objects: signed arrays ``pcal`` (predicted) and
``pobs`` (observed) of shape ``[nr, nt]`` (receiver-major, time contiguous, the
paper's (i, j) = (receiver, time) indexing of Section 2.2) plus the spacings of the
EMD grid ``dx`` (receiver axis) and ``dt`` (time axis).

Recipes (the paper's experiments use gathers of 10^2-10^3 receivers by 10^3-10^4
samples; its data sets are not available here, so these stand in for them):

* config 1 -- 41 single-trace pairs, nt = 1000, dt = 1 ms: a 10 Hz Ricker wavelet
  centred at 0.4 s (observed) against the same wavelet shifted by -200..+200 ms in
  10 ms steps (predicted).  The 1D shift study of Section 3.1.
* config 2 -- one split-spread gather, nr = 400 (10 m), nt = 2000 (2 ms), six
  hyperbolic 12 Hz Ricker events t(h) = sqrt(t0^2 + h^2/v^2) with a ~ U(-1, 1),
  t0 ~ U(0.2, 2.5) s (sorted) and v = 1500 + 2500 (t0 - 0.2)/2.3 m/s; the predicted
  gather uses 0.9 v.  Seed 2.
* config 3 -- 64 gathers, nt ~ U{1500..3000}, nr ~ U{200..500}, U{4..8} events,
  otherwise as config 2.  Seed 3.
* config 4 -- 32 gathers of nt = 2000 by nr = 300, as config 2.  Seed 4.
* config 5 -- 16 gathers of nt = 4000 (2 ms) by nr = 1600 (12.5 m), ten events as
  config 2 plus a linear direct arrival t = |h|/1500 s of amplitude 1; the predicted
  gather uses 0.85 v.  Seed 5.

For configs 2-5 the EMD grid is the unit square (T = X = 1, the paper's practice in
Sections 3.2 and 3.4): dt = 1/(nt - 1), dx = 1/(nr - 1).  The physical spacings only
place the events.  Config 1 uses dt = 1e-3 on a single trace.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Gather:
    pcal: np.ndarray  # [nr, nt] predicted, signed
    pobs: np.ndarray  # [nr, nt] observed, signed
    dx: float         # EMD grid spacing along receivers
    dt: float         # EMD grid spacing along time
    label: str = ""

    @property
    def nr(self) -> int:
        return int(self.pcal.shape[0])

    @property
    def nt(self) -> int:
        return int(self.pcal.shape[1])

    @property
    def cells(self) -> int:
        return self.nr * self.nt


def ricker(t: np.ndarray, f: float) -> np.ndarray:
    """Ricker wavelet of peak frequency ``f``: (1 - 2 pi^2 f^2 t^2) exp(-pi^2 f^2 t^2)."""
    a = (np.pi * f * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def _add_events(out: np.ndarray, dt: float, taus: np.ndarray, amp: float, f: float) -> None:
    """Add amp * ricker(t - tau_i) to every trace i, evaluated on a window of
    |t - tau| <= 2.2/f (outside it the wavelet is below 1e-20)."""
    nr, nt = out.shape
    w = int(np.ceil(2.2 / (f * dt)))
    k = np.arange(-w, w + 1)
    c = np.floor(taus / dt).astype(np.int64)
    j = c[:, None] + k[None, :]                      # [nr, 2w+1]
    valid = (j >= 0) & (j < nt)
    tj = j.astype(np.float64) * dt
    val = amp * ricker(tj - taus[:, None], f)
    rows = np.broadcast_to(np.arange(nr)[:, None], j.shape)
    np.add.at(out, (rows[valid], j[valid]), val[valid])


def hyperbolic_gather(nr: int, nt: int, dt_phys: float, dx_phys: float,
                      amps, t0s, vels, f_peak: float, vel_scale: float,
                      direct_amp: float | None = None, direct_vel: float = 1500.0,
                      dtype=np.float32, label: str = "") -> Gather:
    """A split-spread shot gather (source at the centre receiver) of hyperbolic events.

    The observed gather uses the velocities ``vels``; the predicted one uses
    ``vel_scale * vels`` (and ``vel_scale * direct_vel`` for the direct arrival)."""
    h = (np.arange(nr, dtype=np.float64) - 0.5 * (nr - 1)) * dx_phys
    pobs = np.zeros((nr, nt), np.float64)
    pcal = np.zeros((nr, nt), np.float64)
    for a, t0, v in zip(amps, t0s, vels):
        _add_events(pobs, dt_phys, np.sqrt(t0 * t0 + (h / v) ** 2), a, f_peak)
        vc = v * vel_scale
        _add_events(pcal, dt_phys, np.sqrt(t0 * t0 + (h / vc) ** 2), a, f_peak)
    if direct_amp is not None:
        _add_events(pobs, dt_phys, np.abs(h) / direct_vel, direct_amp, f_peak)
        _add_events(pcal, dt_phys, np.abs(h) / (direct_vel * vel_scale), direct_amp, f_peak)
    return Gather(pcal.astype(dtype), pobs.astype(dtype),
                  dx=1.0 / (nr - 1) if nr > 1 else 1.0,
                  dt=1.0 / (nt - 1) if nt > 1 else 1.0, label=label)


def _events(rng: np.random.Generator, n: int):
    amps = rng.uniform(-1.0, 1.0, n)
    t0s = np.sort(rng.uniform(0.2, 2.5, n))
    vels = 1500.0 + 2500.0 * (t0s - 0.2) / 2.3
    return amps, t0s, vels


def config1_pairs(shifts_ms=None, nt: int = 1000, dt: float = 1e-3, f_peak: float = 10.0,
                  centre: float = 0.4) -> list[Gather]:
    """Single-trace Ricker pairs: observed centred at ``centre``, predicted shifted by
    each entry of ``shifts_ms`` (default -200..+200 ms in 10 ms steps)."""
    if shifts_ms is None:
        shifts_ms = np.arange(-200, 201, 10)
    t = np.arange(nt, dtype=np.float64) * dt
    pobs = ricker(t - centre, f_peak)
    out = []
    for sh in shifts_ms:
        pcal = ricker(t - centre - 1e-3 * float(sh), f_peak)
        out.append(Gather(pcal[None, :].copy(), pobs[None, :].copy(), dx=1.0, dt=dt,
                          label=f"shift{int(sh):+d}ms"))
    return out


def config2_gather(seed: int = 2, nr: int = 400, nt: int = 2000, n_events: int = 6,
                   dtype=np.float32, f_peak: float = 12.0) -> Gather:
    """Config 2; other sizes keep its 4 s by 4 km extent (dt = 4/nt s, dx = 4000/nr m),
    so a reduced gather is a coarser sampling of the same wavefield (lower
    ``f_peak`` keeps coarse samplings from aliasing)."""
    rng = np.random.default_rng(seed)
    a, t0, v = _events(rng, n_events)
    return hyperbolic_gather(nr, nt, 4.0 / nt, 4000.0 / nr, a, t0, v, f_peak, 0.9, dtype=dtype,
                             label=f"c2_{nr}x{nt}")


def config3_batch(seed: int = 3, n: int = 64, dtype=np.float32) -> list[Gather]:
    rng = np.random.default_rng(seed)
    out = []
    for g in range(n):
        nt = int(rng.integers(1500, 3001))
        nr = int(rng.integers(200, 501))
        ne = int(rng.integers(4, 9))
        a, t0, v = _events(rng, ne)
        out.append(hyperbolic_gather(nr, nt, 2e-3, 10.0, a, t0, v, 12.0, 0.9, dtype=dtype,
                                     label=f"c3_{g}_{nr}x{nt}"))
    return out


def config4_batch(seed: int = 4, n: int = 32, nr: int = 300, nt: int = 2000,
                  dtype=np.float32) -> list[Gather]:
    rng = np.random.default_rng(seed)
    out = []
    for g in range(n):
        a, t0, v = _events(rng, 6)
        out.append(hyperbolic_gather(nr, nt, 2e-3, 10.0, a, t0, v, 12.0, 0.9, dtype=dtype,
                                     label=f"c4_{g}"))
    return out


def config5_batch(seed: int = 5, n: int = 16, nr: int = 1600, nt: int = 4000,
                  dtype=np.float32) -> list[Gather]:
    rng = np.random.default_rng(seed)
    out = []
    for g in range(n):
        a, t0, v = _events(rng, 10)
        out.append(hyperbolic_gather(nr, nt, 2e-3, 12.5, a, t0, v, 12.0, 0.85,
                                     direct_amp=1.0, dtype=dtype, label=f"c5_{g}"))
    return out


def random_small_pair(nr: int, nt: int, seed: int, dx: float | None = None,
                      dt: float | None = None, density: float = 0.3,
                      balanced: bool = True, dtype=np.float64) -> Gather:
    """Small signed random gathers (sparse spikes) for the tiny-grid checks.

    With ``balanced`` the observed gather is shifted by a constant so that both have
    the same total signed mass, the paper's assumption in Section 2.1."""
    rng = np.random.default_rng(seed)
    pcal = rng.normal(size=(nr, nt)) * (rng.random((nr, nt)) < density)
    pobs = rng.normal(size=(nr, nt)) * (rng.random((nr, nt)) < density)
    if balanced:
        pobs = pobs + (pcal.sum() - pobs.sum()) / (nr * nt)
    return Gather(pcal.astype(dtype), pobs.astype(dtype),
                  dx=dx if dx is not None else (1.0 / (nr - 1) if nr > 1 else 1.0),
                  dt=dt if dt is not None else (1.0 / (nt - 1) if nt > 1 else 1.0),
                  label=f"rand{nr}x{nt}s{seed}")


def blob_pair(nr: int, nt: int, shift_r: int, shift_t: int, seed: int = 0,
              size: tuple[int, int] = (3, 4), dx: float = 0.5, dt: float = 0.25,
              dtype=np.float64) -> Gather:
    """A non-negative blob (observed) and the same blob moved by (shift_r, shift_t)
    whole cells (predicted); both stay inside the grid."""
    rng = np.random.default_rng(seed)
    br, bt = size
    blob = rng.uniform(0.2, 1.0, size)
    r0 = max(0, -shift_r) + 1 if nr > br + abs(shift_r) + 1 else max(0, -shift_r)
    t0 = max(0, -shift_t) + 1 if nt > bt + abs(shift_t) + 1 else max(0, -shift_t)
    if r0 + br + max(shift_r, 0) > nr or t0 + bt + max(shift_t, 0) > nt:
        raise ValueError("blob and its shift do not fit the grid")
    pobs = np.zeros((nr, nt))
    pcal = np.zeros((nr, nt))
    pobs[r0:r0 + br, t0:t0 + bt] = blob
    pcal[r0 + shift_r:r0 + shift_r + br, t0 + shift_t:t0 + shift_t + bt] = blob
    return Gather(pcal.astype(dtype), pobs.astype(dtype), dx=dx, dt=dt,
                  label=f"blob{shift_r},{shift_t}")


def pack_batch(gathers, dtype=np.float32):
    """Concatenate gathers back to back (each dense [nr][nt]) into flat arrays.

    Returns (pcal, pobs, desc) where desc is a list of (nr, nt, dx, dt, offset)."""
    offs = []
    o = 0
    for g in gathers:
        offs.append(o)
        o += g.cells
    pcal = np.empty(o, dtype)
    pobs = np.empty(o, dtype)
    desc = []
    for g, off in zip(gathers, offs):
        pcal[off:off + g.cells] = g.pcal.reshape(-1)
        pobs[off:off + g.cells] = g.pobs.reshape(-1)
        desc.append((g.nr, g.nt, float(g.dx), float(g.dt), off))
    return pcal, pobs, desc
