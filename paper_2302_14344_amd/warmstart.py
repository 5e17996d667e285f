"""Learned warm start: data generation, training and evaluation on the GPU.

The data come from plain ADMM runs (previous-step warm start) of the library itself with
recording switched on; every network product runs in the library's BF16 matrix-core
kernels (``Mlp.forward/backward/adam``).  Host-side work is limited to bookkeeping:
minibatch row indices (drawn with numpy, gathered on the device by the library), the input and output normalisation constants (means and
standard deviations of the recorded data) and folding the output scale into the last
layer's FP32 master parameters.

Network per class: ReLU perceptron (widths in -> 256 -> 256 -> 256 -> out), inputs
normalised in FP32 before the BF16 rounding (``Mlp.set_input_affine``), outputs
de-normalised by the last layer.  Loss: the ADMM metric of the recorded weights,
sum_i beta_i |z - z*|^2 + beta_i^-1 |u - u*|^2, with every output column scaled to unit
variance and the weights to unit mean.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from .solver import Mlp, Problem, rigid_state_tensors

HIDDEN = (256, 256, 256)
CLASS_IO = ((L.CONTACT_IN, L.CONTACT_OUT), (L.JOINT_IN, L.JOINT_OUT))


@dataclass
class Samples:
    """Recorded rows of one interface class (device FP32)."""
    x: list = field(default_factory=list)
    t: list = field(default_factory=list)
    w: list = field(default_factory=list)

    def cat(self):
        return torch.cat(self.x), torch.cat(self.t), torch.cat(self.w)


def collect(sc, steps, dtype=torch.float32, max_iters=1000, tol=1e-6, every=1, device="cuda"):
    """Run ``steps`` plain-ADMM steps (previous-step warm start) of the rigid batch ``sc``
    from its stored state, recording features, targets and weights every ``every`` steps.
    Rows of unconverged scenes carry zero weight.  Returns (Samples contact, Samples joint)."""
    prob = Problem.from_rigid(sc, dtype=dtype, device=device)
    st = rigid_state_tensors(sc, dtype=dtype, device=device)
    rec = prob.set_recording(True)
    out = (Samples(), Samples())
    for k in range(steps):
        prob.rigid_step(*st, max_iters=max_iters, tol=tol, warm="prev")
        if k % every == 0:
            for c, key in enumerate(("c", "j")):
                if rec["x" + key].shape[0]:
                    out[c].x.append(rec["x" + key].clone())
                    out[c].t.append(rec["t" + key].clone())
                    out[c].w.append(rec["w" + key].clone())
    prob.set_recording(False)
    torch.cuda.synchronize(prob.device)
    return out


def _moments(a, w=None):
    a = a.detach().double().cpu().numpy()
    if w is None:
        mu, sd = a.mean(0), a.std(0)
    else:
        w = w.detach().double().cpu().numpy()
        ws = np.maximum(w.sum(0), 1e-300)
        mu = (w * a).sum(0) / ws
        sd = np.sqrt((w * (a - mu) ** 2).sum(0) / ws)
    return mu, sd


def _init_params(widths, rng):
    parts = []
    for k in range(len(widths) - 1):
        parts.append(rng.standard_normal(widths[k + 1] * widths[k]) * np.sqrt(2.0 / widths[k]))
        parts.append(np.zeros(widths[k + 1]))
    return np.concatenate(parts)


@dataclass
class Trained:
    widths: list
    params: np.ndarray      # FP32 parameters with the output scale folded in
    scale: np.ndarray       # input normalisation x * scale + shift
    shift: np.ndarray
    losses: list

    def network(self, max_batch, device="cuda"):
        net = Mlp(self.widths, max(int(max_batch), 1), device=device)
        net.set_params(self.params)
        net.set_input_affine(self.scale, self.shift)
        return net


def fit(samples, cls, iters=3000, batch=4096, lr=1e-3, seed=0, hidden=HIDDEN, device="cuda", log_every=0):
    """Train the class-``cls`` network on recorded samples with the library's kernels.

    Targets are scaled per column to unit (weighted) variance; the ADMM-metric weights
    are scaled by the same factors squared and then to unit mean, so the loss is the
    metric up to one constant.  Learning rate: ``lr`` with cosine decay to lr/20."""
    x, t, w = samples.cat()
    # rows with a recorded target (host bookkeeping; the arrays go back to the device once)
    wk = w.detach().cpu().numpy()
    keep = np.nonzero(wk.sum(1) > 0)[0]
    dev = x.device
    x = torch.as_tensor(x.detach().cpu().numpy()[keep], device=dev).contiguous()
    t = torch.as_tensor(t.detach().cpu().numpy()[keep], device=dev).contiguous()
    w = torch.as_tensor(wk[keep], device=dev).contiguous()
    n = x.shape[0]
    if n == 0:
        raise ValueError("no converged samples to train on")
    nin, nout = CLASS_IO[cls]
    widths = [nin, *hidden, nout]
    mux, sdx = _moments(x)
    sdx = np.where(sdx > 1e-8 * np.maximum(np.abs(mux), 1.0), sdx, 1.0)
    mut, sdt = _moments(t, w)
    sdt = np.where(sdt > 0, sdt, 1.0)
    # scaled targets and weights (host): tn = (t - mut) / sdt, wn = w sdt^2 / mean
    th = t.double().cpu().numpy()
    wh = w.double().cpu().numpy() * sdt ** 2
    wh /= wh[wh > 0].mean()
    tn = torch.as_tensor((th - mut) / sdt, dtype=torch.float32, device=x.device).contiguous()
    wn = torch.as_tensor(wh, dtype=torch.float32, device=x.device).contiguous()
    rng = np.random.default_rng(seed)
    net = Mlp(widths, min(batch, n), device=device)
    net.set_params(_init_params(widths, rng))
    scale, shift = 1.0 / sdx, -mux / sdx
    net.set_input_affine(scale, shift)
    bsz = min(batch, n)
    # minibatch rows drawn on the host (numpy), 256 iterations' worth per upload, and gathered
    # on the device by the library
    x = x.float().contiguous()
    xb = torch.empty((bsz, x.shape[1]), dtype=torch.float32, device=x.device)
    tb = torch.empty((bsz, tn.shape[1]), dtype=torch.float32, device=x.device)
    wb = torch.empty((bsz, wn.shape[1]), dtype=torch.float32, device=x.device)
    chunk = 256
    losses = []
    for it in range(1, iters + 1):
        if (it - 1) % chunk == 0:
            rows = min(chunk, iters - it + 1)
            idx_all = torch.as_tensor(rng.integers(0, n, (rows, bsz), dtype=np.int32), device=x.device)
        idx = idx_all[(it - 1) % chunk]
        net.gather_rows(x, idx, xb)
        net.gather_rows(tn, idx, tb)
        net.gather_rows(wn, idx, wb)
        net.forward(xb)
        loss, _ = net.backward(tb, wb)
        a = lr * (0.05 + 0.95 * 0.5 * (1 + np.cos(np.pi * (it - 1) / iters)))
        net.adam(a, it)
        if log_every and it % log_every == 0:
            losses.append((it, float(loss.item()) / bsz))
    p = net.get_params().double().cpu().numpy()
    # fold the output scaling into the last layer: y = sdt * (W h + b) + mut
    nW = widths[-1] * widths[-2]
    off = len(p) - nW - widths[-1]
    W = p[off:off + nW].reshape(widths[-1], widths[-2]) * sdt[:, None]
    b = p[off + nW:] * sdt + mut
    p[off:off + nW] = W.reshape(-1)
    p[off + nW:] = b
    return Trained(widths, p.astype(np.float32), scale.astype(np.float32), shift.astype(np.float32), losses)


def attach(prob, trained, device="cuda"):
    """Networks for a problem's classes (trained: (contact, joint), entries may be None)."""
    counts = prob.warm_class_counts()
    nets = []
    for c, tr in enumerate(trained):
        if tr is None or counts[c] == 0:
            nets.append(None)
            continue
        net = tr.network(counts[c], device=device)
        prob.set_warm_model(c, net)
        nets.append(net)
    return nets


def evaluate(sc, steps, warm, trained=None, dtype=torch.float32, max_iters=1000, tol=1e-6, warmup=0,
             device="cuda"):
    """Run ``warmup + steps`` steps of ``sc`` from its stored state with the given warm
    start and report, over the last ``steps``: mean iterations per scene-step (both runs
    of a fallback counted), scene-steps that fell back, unconverged scene-steps and
    wall-clock steps per second."""
    prob = Problem.from_rigid(sc, dtype=dtype, device=device)
    st = rigid_state_tensors(sc, dtype=dtype, device=device)
    if warm == "learned":
        attach(prob, trained, device=device)
    for _ in range(warmup):
        prob.rigid_step(*st, max_iters=max_iters, tol=tol, warm=warm)
    torch.cuda.synchronize(prob.device)
    prob.reset_totals()
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.rigid_step(*st, max_iters=max_iters, tol=tol, warm=warm)
    torch.cuda.synchronize(prob.device)
    dt = time.perf_counter() - t0
    s = prob.stats()
    n = prob.sizes.n_scene * steps
    return {"iters_per_scene_step": float(s["iters_total"].sum()) / n,
            "fallback_frac": float(s["fallback_total"].sum()) / n,
            # a learned-start run that stops at max_iters is counted once more by its fallback
            "unconverged_frac": float(s["unconverged_total"].sum() - s["fallback_total"].sum()) / n,
            "steps_per_s": steps / dt, "state": st}
