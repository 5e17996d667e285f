"""Accuracy measure of the paper's evaluation (Sec. IV: constraint error per step, with the
Fischer-Burmeister function for contacts, reported as the average of -log(error)), written
from its definition on the CPU.  Test infrastructure: used by tests and by the benchmark's
baseline leg only.

Reading (the paper names the measure, not its formula): per interface j with constraint
value c_j = sum_i J_i,j v_hat_i + e_j and the scalar metric w_j = sum_i 1/beta_i of the
z-update (which brings forces to velocity units),
  equality          r_j = |c_j|
  hard inequality   r_j = |FB(c_j, w_j lambda_j)| (per row)
  soft (Eq. 3)      r_j = w_j |lambda_j + k_j (e_j + alpha_j (c_j - e_j))|
  contact (Eq. 5)   r_j^2 = FB(c_n, w lambda_n)^2 + |w lambda_t - P(w lambda_t - c_t)|^2, P the
                    projection onto the disc of radius mu w lambda_n (the friction law's
                    fixed-point residual)
with FB(a, b) = a + b - sqrt(a^2 + b^2), zero exactly when a >= 0, b >= 0, a b = 0.  The scene's
error is sqrt(sum_j r_j^2); the accuracy index of a run is the mean over its steps of
-log10(error).  The index of the evaluation is taken over the interfaces with a feasibility
law (equality, hard inequality, contact): a soft coupling is a force law with no feasible set
to violate, so its residual (the distance of the iterate from Eq. 3) is reported beside it.
"""
from __future__ import annotations

import numpy as np


def fb(a, b):
    return a + b - np.sqrt(a * a + b * b)


def _layout(sub_ndof, if_dim, if_nsub, if_sub):
    n = np.asarray(sub_ndof, np.int64)
    ns = len(n)
    nc = np.zeros(ns, np.int64)
    for j in range(len(if_dim)):
        for m in range(int(if_nsub[j])):
            nc[if_sub[j][m]] += int(if_dim[j])
    joff = np.concatenate([[0], np.cumsum(nc * n)])
    doff = np.concatenate([[0], np.cumsum(n)])
    eoff = np.concatenate([[0], np.cumsum(if_dim)])
    fill = np.zeros(ns, np.int64)
    slot = {}
    for j in range(len(if_dim)):
        for m in range(int(if_nsub[j])):
            i = if_sub[j][m]
            slot[(j, m)] = int(fill[i])
            fill[i] += int(if_dim[j])
    return n, nc, joff, doff, eoff, slot


def constraint_error(topo, J, e, v_hat, lam, beta, kinds=(0, 1, 2, 3)):
    """Per-scene constraint error of a step's (v_hat, lambda) with the assembled J, e (dense
    layout) and the penalties beta, over the interfaces whose kind is in ``kinds``.
    ``topo``: sub_ndof, sub_scene, if_kind, if_dim, if_nsub, if_sub, if_mu, and if_k,
    if_alpha for soft interfaces."""
    if_sub = np.asarray(topo.if_sub).reshape(len(topo.if_dim), -1)
    n, nc, joff, doff, eoff, slot = _layout(topo.sub_ndof, topo.if_dim, topo.if_nsub, if_sub)
    sub_scene = np.asarray(topo.sub_scene)
    n_scene = int(sub_scene.max()) + 1
    acc = np.zeros(n_scene)
    if_k = getattr(topo, "if_k", None)
    if_alpha = getattr(topo, "if_alpha", None)
    for j in range(len(topo.if_dim)):
        if int(topo.if_kind[j]) not in kinds:
            continue
        d = int(topo.if_dim[j])
        c = np.array(e[eoff[j]:eoff[j] + d], dtype=np.float64)
        w = 0.0
        for m in range(int(topo.if_nsub[j])):
            i = int(if_sub[j, m])
            Ji = np.asarray(J[joff[i]:joff[i + 1]]).reshape(nc[i], n[i])
            c = c + Ji[slot[(j, m)]:slot[(j, m)] + d] @ np.asarray(v_hat[doff[i]:doff[i + 1]])
            w += 1.0 / float(beta[i])
        lj = np.asarray(lam[eoff[j]:eoff[j] + d], dtype=np.float64)
        kind = int(topo.if_kind[j])
        if kind == 0:
            r2 = float(c @ c)
        elif kind == 2:
            r2 = float(np.sum(fb(c, w * lj) ** 2))
        elif kind == 3:
            k, al = float(if_k[j]), float(if_alpha[j])
            ev = np.asarray(e[eoff[j]:eoff[j] + d], dtype=np.float64)
            res = w * (lj + k * (ev + al * (c - ev)))
            r2 = float(res @ res)
        else:
            mu = float(topo.if_mu[j])
            rn = fb(c[0], w * lj[0])
            q = w * lj[1:] - c[1:]
            rad = mu * w * max(lj[0], 0.0)
            nq = float(np.linalg.norm(q))
            proj = q if nq <= rad else (q * (rad / nq) if nq > 0 else q)
            rt = w * lj[1:] - proj
            r2 = float(rn * rn + rt @ rt)
        acc[sub_scene[if_sub[j, 0]]] += r2
    return np.sqrt(acc)


def accuracy_index(errors):
    """Mean of -log10 over the per-step errors (the larger, the more accurate)."""
    e = np.maximum(np.asarray(errors, dtype=np.float64), 1e-300)
    return float(np.mean(-np.log10(e)))
