"""Fixed-iteration evaluation of the paper (Sec. IV-C, Table I): whole steps at a set number
of ADMM iterations (no tolerance stop), reported as the average time per step and the
accuracy index, the mean over the steps of -log10 of the per-step constraint error (the
error computed on the GPU by ``subadmm_constraint_error`` over the interfaces with a
feasibility law: equality residuals, Fischer-Burmeister for contacts and hard rows, the
friction law's fixed-point residual).  The residual of the soft couplings (Eq. 3), force laws
with no feasible set, is reported beside it as its own index.

Both the rigid model (``pr.rigid_step``) and the FEM model (``pr.fem_step``) are driven;
the state tensors are updated in place.  The timed pass and the measured pass start from
the same state and warm start (saved and restored), so they run the same trajectory."""
from __future__ import annotations

import time

import numpy as np
import torch

from . import _lib as L


def _step(pr, kind, state, iters, v_hat=None, lam=None, graph=False):
    if kind == "rigid":
        pr.rigid_step(*state, max_iters=iters, tol=0.0, warm="prev", v_hat=v_hat, lam=lam, graph=graph)
    else:
        pr.fem_step(*state, max_iters=iters, tol=0.0, warm="prev", v_hat=v_hat, lam=lam)


def _snapshot(pr, state):
    return [t.clone() for t in state], [w.clone() for w in pr.get_warm()]


def _restore(pr, state, snap):
    for t, s in zip(state, snap[0]):
        t.copy_(s)
    pr.set_warm(*snap[1])


def run(pr, kind, state, iters, n_steps, warmup=2, graph=True):
    """``warmup`` untimed steps, then ``n_steps`` timed steps at ``iters`` iterations (HIP
    events on the library's stream), then the same steps again from the same state with the
    constraint error of each.  Returns a dict with ms_per_step, the per-step, per-scene
    errors and the accuracy index (mean of -log10 over steps and scenes)."""
    if kind not in ("rigid", "fem"):
        raise ValueError("kind is 'rigid' or 'fem'")
    graph = graph and kind == "rigid"
    for _ in range(warmup):
        _step(pr, kind, state, iters, graph=graph)
    torch.cuda.synchronize()
    snap = _snapshot(pr, state)
    if graph:
        # capture outside the timed region
        _step(pr, kind, state, iters, graph=True)
        torch.cuda.synchronize()
        _restore(pr, state, snap)
        torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(pr.stream)
    t0 = time.perf_counter()
    for _ in range(n_steps):
        _step(pr, kind, state, iters, graph=graph)
    ev1.record(pr.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    _restore(pr, state, snap)
    torch.cuda.synchronize()
    sz = pr.sizes
    vh, lam = pr.empty(sz.n_dof), pr.empty(sz.n_rows)
    errs, soft = [], []
    for _ in range(n_steps):
        _step(pr, kind, state, iters, v_hat=vh, lam=lam)
        errs.append(pr.constraint_error(vh, lam, kinds=L.ERR_LAWS))
        soft.append(pr.constraint_error(vh, lam, kinds=L.ERR_SOFT))
    errs, soft = np.array(errs), np.array(soft)
    out = {"iters": int(iters), "steps": int(n_steps), "ms_per_step": ms / n_steps,
           "wall_ms_per_step": 1e3 * wall / n_steps, "errors": errs, "aa": accuracy_index(errs),
           "soft_residuals": soft}
    if soft.max() > 0:
        out["aa_soft"] = accuracy_index(soft)
    return out


def accuracy_index(errors):
    """Mean of -log10 of the errors (larger is more accurate)."""
    e = np.maximum(np.asarray(errors, dtype=np.float64), 1e-300)
    return float(np.mean(-np.log10(e)))


def linear_fit(x, y):
    """Least-squares line y = a + b x with its coefficient of determination."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    b, a = np.polyfit(x, y, 1)
    res = y - (a + b * x)
    tot = y - y.mean()
    r2 = 1.0 - float(res @ res) / float(tot @ tot) if float(tot @ tot) > 0 else 1.0
    return {"intercept": float(a), "slope": float(b), "r2": r2}
