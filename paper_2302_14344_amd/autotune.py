"""Schedule autotuner for the rigid step.

The library offers interchangeable forms of the per-step work (the iteration kernel with
a thread per slot row or a lane team per interface, long rows split over lanes or not; the
factorisation size classes run concurrently on forked streams or one after another).  Which is faster depends on the
scene shapes, so the tuner times each candidate on the caller's own problem: from a copy
of the state and of the kept warm-start values it runs a few untimed steps and then a few
timed ones (HIP events on the problem's stream), keeps the fastest and leaves the state
and the warm-start values as it found them.  Results are cached per problem signature.
"""
from __future__ import annotations

import itertools

import torch

from . import _lib as L

CANDIDATES = {
    "team_kernel": (0, 1, 2),
    "factor_streams": (1, 0),
    "split_rows": (2, 1, 0),
}
_CACHE: dict = {}


def candidates():
    """Every distinct schedule (row splitting, within the default workgroup or growing it,
    applies to the thread-per-slot-row form only; a form the problem does not admit is
    skipped when it is applied)."""
    out = []
    for values in itertools.product(*CANDIDATES.values()):
        cfg = dict(zip(CANDIDATES.keys(), values))
        if cfg["team_kernel"] and cfg["split_rows"] != 1:
            continue
        out.append(cfg)
    return out


def _signature(prob):
    s = prob.sizes
    return (s.n_sub, s.n_if, s.n_scene, s.n_slot, s.max_dof, s.max_slot_scene, str(prob.dtype))


def _apply(prob, cfg):
    """Applies a schedule; False (and nothing changed) if the problem does not admit its
    iteration-kernel form."""
    lib = L.lib()
    if lib.subadmm_set_option(prob._h, L.OPT_TEAM_KERNEL, int(cfg["team_kernel"])) != 0:
        return False
    L.check(lib.subadmm_set_option(prob._h, L.OPT_FACTOR_STREAMS, int(cfg["factor_streams"])), prob._h)
    L.check(lib.subadmm_set_option(prob._h, L.OPT_SPLIT_ROWS, int(cfg["split_rows"])), prob._h)
    return True


def tune_rigid(prob, pos, rot, vel, omega, max_iters=1000, tol=1e-6, warm="prev", warmup=3, steps=10,
               use_cache=True):
    """Times every candidate schedule on ``prob`` from the given state and applies the
    fastest.  Returns (chosen config, {config key: ms per step})."""
    key = _signature(prob)
    if use_cache and key in _CACHE:
        _apply(prob, _CACHE[key][0])
        return _CACHE[key]
    z0, u0 = prob.get_warm()
    z0, u0 = z0.clone(), u0.clone()
    state0 = [t.clone() for t in (pos, rot, vel, omega)]
    times = {}
    best = None
    for cfg in candidates():
        if not _apply(prob, cfg):
            continue
        st = [t.clone() for t in state0]
        prob.set_warm(z0, u0)
        for _ in range(warmup):
            prob.rigid_step(*st, max_iters=max_iters, tol=tol, warm=warm)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(prob.stream)
        for _ in range(steps):
            prob.rigid_step(*st, max_iters=max_iters, tol=tol, warm=warm)
        ev1.record(prob.stream)
        torch.cuda.synchronize(prob.device)
        ms = ev0.elapsed_time(ev1) / steps
        times[tuple(sorted(cfg.items()))] = ms
        if best is None or ms < best[1]:
            best = (cfg, ms)
    _apply(prob, best[0])
    prob.set_warm(z0, u0)
    prob.reset_totals()
    torch.cuda.synchronize(prob.device)
    _CACHE[key] = (best[0], times)
    return best[0], times


FEM_CANDIDATES = {"fem_resident": (1, 0)}


def tune_fem(prob, pos, vel, max_iters=5000, tol=1e-6, warm="prev", warmup=1, steps=3, use_cache=True):
    """The FEM step's iteration form: block operators held in registers and LDS for the
    whole step (when every block's operator fits) or read from device memory in every
    iteration.  Timed like ``tune_rigid`` from copies of the state and warm-start values,
    which are restored; the fastest is applied.  Returns (chosen config, {key: ms per step})."""
    key = ("fem",) + _signature(prob)
    lib = L.lib()
    if use_cache and key in _CACHE:
        L.check(lib.subadmm_set_option(prob._h, L.OPT_FEM_RESIDENT, int(_CACHE[key][0]["fem_resident"])), prob._h)
        return _CACHE[key]
    z0, u0 = prob.get_warm()
    z0, u0 = z0.clone(), u0.clone()
    state0 = [t.clone() for t in (pos, vel)]
    times = {}
    best = None
    for res in FEM_CANDIDATES["fem_resident"]:
        cfg = {"fem_resident": res}
        L.check(lib.subadmm_set_option(prob._h, L.OPT_FEM_RESIDENT, res), prob._h)
        st = [t.clone() for t in state0]
        prob.set_warm(z0, u0)
        for _ in range(warmup):
            prob.fem_step(*st, max_iters=max_iters, tol=tol, warm=warm)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(prob.stream)
        for _ in range(steps):
            prob.fem_step(*st, max_iters=max_iters, tol=tol, warm=warm)
        ev1.record(prob.stream)
        torch.cuda.synchronize(prob.device)
        ms = ev0.elapsed_time(ev1) / steps
        times[tuple(sorted(cfg.items()))] = ms
        if best is None or ms < best[1]:
            best = (cfg, ms)
    L.check(lib.subadmm_set_option(prob._h, L.OPT_FEM_RESIDENT, int(best[0]["fem_resident"])), prob._h)
    prob.set_warm(z0, u0)
    prob.reset_totals()
    torch.cuda.synchronize(prob.device)
    _CACHE[key] = (best[0], times)
    return best[0], times
