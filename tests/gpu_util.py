"""Helpers for the GPU parity tests: run the same seeded batch through the HIP
library (via its C ABI binding) and through the oracle, gather by gather."""
from __future__ import annotations

import sys

import numpy as np

import oracle
from synth import pack_batch


def log(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def to_precision(gathers, dtype):
    """Round the inputs to the GPU precision; the oracle then sees the same values."""
    out = []
    for g in gathers:
        g2 = type(g)(g.pcal.astype(dtype), g.pobs.astype(dtype), g.dx, g.dt, g.label)
        out.append(g2)
    return out


def make_plan(gathers, params, rows=None):
    import torch
    import paper_1808_07284_amd as E
    dtype = np.float64 if params.precision == E.F64 else np.float32
    pcal, pobs, desc = pack_batch(gathers, dtype)
    plan = E.Plan(desc, len(pcal), params)
    if rows is not None:
        plan.set_tiling(rows)
    dev = plan.device
    return plan, torch.from_numpy(pcal).to(dev), torch.from_numpy(pobs).to(dev), desc


def unpack(buf, desc, comps=1):
    """Split a batch buffer (numpy) into per-gather [nr, nt] arrays."""
    buf = np.asarray(buf).reshape(-1)
    n = buf.size // comps
    out = []
    for nr, nt, _, _, off in desc:
        if comps == 1:
            out.append(buf[off:off + nr * nt].reshape(nr, nt))
        else:
            out.append(tuple(buf[c * n + off:c * n + off + nr * nt].reshape(nr, nt) for c in range(comps)))
    return out


def oracle_params(gp, **over):
    p = oracle.Params(eps=gp.eps, xi=gp.xi, zeta=gp.zeta, delta=gp.delta, alpha1=gp.alpha1,
                      alpha_max_factor=gp.alpha_max_factor, tol_res=gp.tol_res,
                      mass_tol=gp.mass_tol, max_iter=gp.max_iter, check_every=gp.check_every,
                      max_ls_trials=gp.max_ls_trials, ls_mode=gp.ls_mode)
    for k, v in over.items():
        setattr(p, k, v)
    return p


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.linalg.norm(a - b)
    n = np.linalg.norm(b)
    return d / n if n > 0 else d


def centred(a):
    a = np.asarray(a, np.float64)
    return a - a.mean()
