"""FP64 oracle of the learned warm start: per-interface features, the initial (z^0, u^0)
built from a network output, and the training targets.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper leaves the initial
(z^0, u^0) of Algorithm 1 open; the learned start is this project's own extension and
these functions define it.  Quantities are in velocity units: a constraint force lambda
is divided by the interface's z-metric weight w_hat = 1 / sum_{i in S_j} beta_i^-1, the
weight with which Eq. (18) combines the members' proposals (beta z = y + lambda).

Classes: 0 = contact interfaces (dim 3, one member), 1 = equality interfaces of
dimension 5 (revolute joints, one or two members); every other interface keeps the
previous step's values.  Row layouts:
  contact (12): e_n, c (3), lambda_prev / w_hat (3), z_prev (3), log w_hat, mu
  joint (27):   e (5), c (5), lambda_prev / w_hat (5), z_prev member 0 (5),
                z_prev member 1 (5, zeros for one member), log w_hat, |S_j| - 1
  output contact (6): delta lambda / w_hat (3), delta z (3)
  output joint (15):  delta lambda / w_hat (5), delta z member 0 (5), member 1 (5)
with c = sum_i J_i,j v_i the constraint velocity at the start-of-step velocity and
(z_prev, u_prev = -lambda_prev) the previous step's final slot values.

Slot layout (shared convention of the solver's inputs and outputs): subsystem i lists,
for each interface j that contains it in ascending j, d_j rows; subsystems are
concatenated in index order.
"""
from __future__ import annotations

import numpy as np

CONTACT_IN, CONTACT_OUT, JOINT_IN, JOINT_OUT = 12, 6, 27, 15
KIND_EQUALITY, KIND_CONTACT = 0, 1


def interface_classes(if_kind, if_dim, if_nsub):
    """(class per interface (-1 none), row within the class, class sizes)."""
    cls = np.full(len(if_kind), -1, np.int64)
    row = np.full(len(if_kind), -1, np.int64)
    count = [0, 0]
    for j in range(len(if_kind)):
        c = -1
        if if_kind[j] == KIND_CONTACT and if_nsub[j] == 1:
            c = 0
        elif if_kind[j] == KIND_EQUALITY and if_dim[j] == 5:
            c = 1
        if c >= 0:
            cls[j] = c
            row[j] = count[c]
            count[c] += 1
    return cls, row, tuple(count)


def slots(sub_ndof, if_dim, if_nsub, if_sub):
    """Offsets: dof per subsystem, slot per subsystem, first slot of each member, e row."""
    if_sub = np.asarray(if_sub).reshape(-1, 2)
    nc = np.zeros(len(sub_ndof), np.int64)
    local = np.zeros((len(if_dim), 2), np.int64)
    for j in range(len(if_dim)):
        for m in range(int(if_nsub[j])):
            i = int(if_sub[j, m])
            local[j, m] = nc[i]
            nc[i] += int(if_dim[j])
    dof = np.concatenate([[0], np.cumsum(sub_ndof)]).astype(np.int64)
    slot = np.concatenate([[0], np.cumsum(nc)]).astype(np.int64)
    first = np.full((len(if_dim), 2), -1, np.int64)
    for j in range(len(if_dim)):
        for m in range(int(if_nsub[j])):
            first[j, m] = slot[int(if_sub[j, m])] + local[j, m]
    erow = np.concatenate([[0], np.cumsum(if_dim)]).astype(np.int64)
    return dof, slot, first, erow, nc


def dof_velocity(sc, vel=None, omega=None):
    """Velocity vector of the rigid batch: per body (v world, omega body) at its DOF block."""
    vel = np.asarray(sc.vel if vel is None else vel, np.float64).reshape(-1, 3)
    omega = np.asarray(sc.omega if omega is None else omega, np.float64).reshape(-1, 3)
    dof = np.concatenate([[0], np.cumsum(sc.sub_ndof)]).astype(np.int64)
    v = np.zeros(int(dof[-1]))
    for k in range(sc.n_bodies):
        o = dof[int(sc.body_sub[k])] + 6 * int(sc.body_local[k])
        v[o:o + 3] = vel[k]
        v[o + 3:o + 6] = omega[k]
    return v


class _Topo:
    def __init__(self, t):
        self.sub_ndof = np.asarray(t.sub_ndof)
        self.if_kind, self.if_dim, self.if_nsub = np.asarray(t.if_kind), np.asarray(t.if_dim), np.asarray(t.if_nsub)
        self.if_sub = np.asarray(t.if_sub).reshape(-1, 2)
        self.if_mu = np.asarray(t.if_mu, np.float64)
        self.cls, self.row, self.count = interface_classes(self.if_kind, self.if_dim, self.if_nsub)
        self.dof, self.slot, self.first, self.erow, self.nc = slots(self.sub_ndof, self.if_dim, self.if_nsub,
                                                                    self.if_sub)
        joff = [0]
        for i in range(len(self.sub_ndof)):
            joff.append(joff[-1] + int(self.nc[i]) * int(self.sub_ndof[i]))
        self.joff = np.asarray(joff, np.int64)

    def members(self, j):
        return [(int(self.if_sub[j, m]), int(self.first[j, m])) for m in range(int(self.if_nsub[j]))]

    def w_hat(self, beta, j):
        return 1.0 / sum(1.0 / float(beta[i]) for i, _ in self.members(j))

    def slot_row(self, J, i, g):
        """Row of J_i for global slot row g of subsystem i."""
        n = int(self.sub_ndof[i])
        loc = g - int(self.slot[i])
        return J[self.joff[i] + loc * n: self.joff[i] + (loc + 1) * n]


def features(topo, J, e, beta, v, z_prev, u_prev):
    """Feature rows (xc, xj) of the two classes, FP64."""
    t = _Topo(topo)
    J, e, beta, v = (np.asarray(a, np.float64) for a in (J, e, beta, v))
    z_prev, u_prev = np.asarray(z_prev, np.float64), np.asarray(u_prev, np.float64)
    xc = np.zeros((t.count[0], CONTACT_IN))
    xj = np.zeros((t.count[1], JOINT_IN))
    for j in range(len(t.if_kind)):
        c = t.cls[j]
        if c < 0:
            continue
        d = int(t.if_dim[j])
        mem = t.members(j)
        wh = t.w_hat(beta, j)
        cvel = np.zeros(d)
        for i, g in mem:
            vi = v[t.dof[i]:t.dof[i + 1]]
            for k in range(d):
                cvel[k] += t.slot_row(J, i, g + k) @ vi
        g0 = mem[0][1]
        lam_prev = -u_prev[g0:g0 + d]
        ej = e[t.erow[j]:t.erow[j] + d]
        if c == 0:
            x = xc[t.row[j]]
            x[0] = ej[0]
            x[1:4] = cvel
            x[4:7] = lam_prev / wh
            x[7:10] = z_prev[g0:g0 + 3]
            x[10] = np.log(wh)
            x[11] = t.if_mu[j]
        else:
            x = xj[t.row[j]]
            x[0:5] = ej
            x[5:10] = cvel
            x[10:15] = lam_prev / wh
            x[15:20] = z_prev[g0:g0 + 5]
            if len(mem) == 2:
                g1 = mem[1][1]
                x[20:25] = z_prev[g1:g1 + 5]
            x[25] = np.log(wh)
            x[26] = len(mem) - 1
    return xc, xj


def apply(topo, beta, z_prev, u_prev, yc, yj):
    """Initial (z^0, u^0): for an interface of a class with a finite output row,
    lambda^0 = lambda_prev + w_hat * (delta lambda / w_hat), u^0 = -lambda^0 on every member
    slot and z^0 = z_prev + delta z per member; elsewhere the previous values."""
    t = _Topo(topo)
    z0 = np.array(z_prev, np.float64, copy=True)
    u0 = np.array(u_prev, np.float64, copy=True)
    for j in range(len(t.if_kind)):
        c = t.cls[j]
        if c < 0:
            continue
        y = (yc if c == 0 else yj)
        if y is None:
            continue
        y = np.asarray(y[t.row[j]], np.float64)
        if not np.all(np.isfinite(y)):
            continue
        d = int(t.if_dim[j])
        mem = t.members(j)
        wh = t.w_hat(beta, j)
        lam0 = -np.asarray(u_prev[mem[0][1]:mem[0][1] + d], np.float64) + wh * y[:d]
        for m, (_, g) in enumerate(mem):
            u0[g:g + d] = -lam0
            z0[g:g + d] = z_prev[g:g + d] + y[d + m * d: d + (m + 1) * d]
    return z0, u0


def targets(topo, beta, z_prev, u_prev, z_fin, u_fin, conv, sub_scene):
    """Targets (tc, tj) and loss weights (wc, wj): the output rows that ``apply`` turns
    into the final values, weighted by the ADMM metric sum_i beta_i |dz_i|^2 +
    beta_i^-1 |du_i|^2 (w_hat on the lambda / w_hat entries, beta_i on member i's z
    entries), zero weight for absent members and unconverged scenes."""
    t = _Topo(topo)
    out = {"tc": np.zeros((t.count[0], CONTACT_OUT)), "tj": np.zeros((t.count[1], JOINT_OUT)),
           "wc": np.zeros((t.count[0], CONTACT_OUT)), "wj": np.zeros((t.count[1], JOINT_OUT))}
    for j in range(len(t.if_kind)):
        c = t.cls[j]
        if c < 0:
            continue
        d = int(t.if_dim[j])
        mem = t.members(j)
        wh = t.w_hat(beta, j)
        ok = bool(conv[int(sub_scene[mem[0][0]])])
        y = out["tc" if c == 0 else "tj"][t.row[j]]
        w = out["wc" if c == 0 else "wj"][t.row[j]]
        g0 = mem[0][1]
        y[:d] = (np.asarray(u_prev[g0:g0 + d]) - np.asarray(u_fin[g0:g0 + d])) / wh
        w[:d] = wh if ok else 0.0
        for m, (i, g) in enumerate(mem):
            y[d + m * d: d + (m + 1) * d] = np.asarray(z_fin[g:g + d]) - np.asarray(z_prev[g:g + d])
            w[d + m * d: d + (m + 1) * d] = float(beta[i]) if ok else 0.0
    return out
