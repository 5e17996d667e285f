"""GPU deformable-body path (co-rotated FEM blocks) against the FP64 oracle.

Tolerances as in the solver parity tests: FP64 1e-9 relative to the largest reference
entry (velocity floor g t, force floor the body's weight); FP32 1e-5 with the same
floors.  Assembly in FP64 agrees to rounding (1e-12 relative).  The iteration is compared
after a fixed number of iterations and under the stopping rule from identical inputs.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2302_14344_amd import scenes as S

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _solver():
    from paper_2302_14344_amd.solver import Problem, fem_state_tensors
    return Problem, fem_state_tensors


def _perturbed(fs, seed, amp=0.02):
    """A deformed, moving state: node displacements U[-amp, amp] h (shared by coincident
    copies through the lattice jitter seed) and velocities N(0, 0.05) m/s."""
    rng = np.random.default_rng(seed)
    h = fs.meta["h"]
    pos = fs.pos + rng.uniform(-amp, amp, fs.pos.shape) * h
    vel = rng.normal(0, 0.05, fs.pos.shape)
    return fs.with_state(pos, vel)


def _round32(fs):
    r = lambda a: np.asarray(a, np.float32).astype(np.float64)
    return fs.with_state(r(fs.pos), r(fs.vel))


CASES = {
    "2x2x2": dict(blocks=(2, 2, 2), nodes_per_block=5),
    "two-bodies": dict(blocks=(2, 1, 1), nodes_per_block=4, n_bodies=2),
}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("case", list(CASES))
def test_fem_assemble_parity(case, dtype):
    print(f"case {case} {dtype}", flush=True)
    Problem, fst = _solver()
    fs = _perturbed(S.fem_scene(seed=S.config_seed(3, 10), **CASES[case]), 1)
    if dtype == torch.float32:
        fs = _round32(fs)
    pr = Problem.from_fem(fs, dtype=dtype)
    pos, vel = fst(fs, dtype=dtype)
    A, b, J, e = (_np(t) for t in pr.fem_assemble(pos, vel))
    rA, rb, rJ, re = O.fem_assemble(fs)
    tol = 1e-12 if dtype == torch.float64 else 2e-7
    for g, r, nm in ((A, rA, "A"), (b, rb, "b"), (J, rJ, "J"), (e, re, "e")):
        np.testing.assert_allclose(g, r, atol=tol * max(1.0, np.abs(r).max()), err_msg=nm)


def _scene_floor(fs):
    return fs.gravity * fs.dt, fs.gravity * fs.density * 1e-6


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("mode", ["fixed", "converged"])
def test_fem_step_fp64_parity(case, mode):
    """FP64 whole step (assembly, FP64 factorisation, cooperative iteration, v_hat and
    state update) against the oracle from the same deformed state and warm start."""
    print(f"case {case} {mode}", flush=True)
    Problem, fst = _solver()
    fs = _perturbed(S.fem_scene(seed=S.config_seed(3, 11), **CASES[case]), 2)
    (p1, v1), r0 = O.fem_step(fs, max_iters=300, tol=0.0, n_threads=8)
    fs1 = fs.with_state(p1, v1)
    iters, tol = (60, 0.0) if mode == "fixed" else (20000, 1e-7)
    _, ref = O.fem_step(fs1, max_iters=iters, tol=tol, z0=r0.z, u0=r0.u, n_threads=8)
    pr = Problem.from_fem(fs, dtype=torch.float64)
    pos, vel = fst(fs1, dtype=torch.float64)
    pr.set_warm(pr.tensor(r0.z), pr.tensor(r0.u))
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    pr.fem_step(pos, vel, max_iters=iters, tol=tol, warm="prev", v_hat=vh, lam=lam)
    s = pr.stats()
    print(f"  iterations gpu {s['iters']} ref {ref.iters}", flush=True)
    if mode == "fixed":
        assert (s["iters"] == iters).all()
    else:
        assert (s["converged"] == ref.converged).all() and np.abs(s["iters"] - ref.iters).max() <= 2
    vf, lf = _scene_floor(fs)
    np.testing.assert_allclose(_np(vh), ref.v_hat, atol=1e-9 * max(vf, np.abs(ref.v_hat).max()))
    np.testing.assert_allclose(_np(lam), ref.lam, atol=1e-9 * max(lf, np.abs(ref.lam).max()))
    new_pos, new_vel = O.fem_advance(fs1, ref.v_hat)
    np.testing.assert_allclose(_np(pos), new_pos.reshape(-1), atol=1e-12)
    np.testing.assert_allclose(_np(vel), new_vel.reshape(-1), atol=1e-9 * max(vf, np.abs(new_vel).max()))
    z, u = pr.get_warm()
    np.testing.assert_allclose(_np(z), ref.z, atol=1e-9 * max(vf, np.abs(ref.z).max()))


def test_fem_step_fp32_parity():
    """FP32 iteration with the FP64 factorisation against the FP64 oracle after a fixed
    number of iterations, from identical (FP32-rounded) inputs."""
    Problem, fst = _solver()
    fs = _round32(_perturbed(S.fem_scene(seed=S.config_seed(3, 12), **CASES["2x2x2"]), 3))
    _, ref = O.fem_step(fs, max_iters=40, tol=0.0, n_threads=8)
    pr = Problem.from_fem(fs, dtype=torch.float32)
    pos, vel = fst(fs, dtype=torch.float32)
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    pr.fem_step(pos, vel, max_iters=40, tol=0.0, warm="cold", v_hat=vh, lam=lam)
    vf, lf = _scene_floor(fs)
    ev = np.abs(_np(vh) - ref.v_hat).max() / max(vf, np.abs(ref.v_hat).max())
    el = np.abs(_np(lam) - ref.lam).max() / max(lf, np.abs(ref.lam).max())
    print(f"  fp32 errors: v {ev:.3e} lambda {el:.3e}", flush=True)
    assert ev <= 1e-5 and el <= 1e-5


def test_fem_full_block_lattice_first_iterations():
    """The full 40^3-node lattice in 512 blocks of 375 DOF (FP32, the benchmark's launch
    configuration) against the oracle after 3 iterations from rest."""
    Problem, fst = _solver()
    fs = S.fem_scene()
    fs = _round32(fs)
    _, ref = O.fem_step(fs, max_iters=3, tol=0.0, n_threads=16)
    pr = Problem.from_fem(fs, dtype=torch.float32)
    pos, vel = fst(fs, dtype=torch.float32)
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    pr.fem_step(pos, vel, max_iters=3, tol=0.0, warm="cold", v_hat=vh, lam=lam)
    vf, lf = _scene_floor(fs)
    ev = np.abs(_np(vh) - ref.v_hat).max() / max(vf, np.abs(ref.v_hat).max())
    el = np.abs(_np(lam) - ref.lam).max() / max(lf, np.abs(ref.lam).max())
    print(f"  full lattice fp32 errors: v {ev:.3e} lambda {el:.3e}", flush=True)
    assert ev <= 1e-5 and el <= 1e-5


def test_fem_determinism_bitwise():
    Problem, fst = _solver()
    fs = _perturbed(S.fem_scene(seed=S.config_seed(3, 13), **CASES["2x2x2"]), 4)
    outs = []
    for _ in range(2):
        pr = Problem.from_fem(fs, dtype=torch.float32)
        pos, vel = fst(fs, dtype=torch.float32)
        vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
        pr.fem_step(pos, vel, max_iters=200, tol=1e-6, warm="cold", v_hat=vh, lam=lam)
        outs.append((_np(vh), _np(lam), _np(pos), pr.stats()["iters"]))
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("scene", ["2x2x2", "lattice"])
def test_fem_resident_form_matches_streamed(scene):
    """The resident iteration (operators in registers and LDS for the whole step) and the
    streamed one (operators read from device memory every iteration) form the same
    products in the same order: bitwise-equal results, same iteration counts."""
    Problem, fst = _solver()
    if scene == "lattice":
        fs = _perturbed(S.fem_scene(), 5, amp=0.005)
        iters, tol = 40, 0.0
    else:
        fs = _perturbed(S.fem_scene(seed=S.config_seed(3, 14), **CASES["2x2x2"]), 6)
        iters, tol = 400, 1e-6
    outs, forms = [], []
    for resident in (True, False):
        pr = Problem.from_fem(fs, dtype=torch.float32)
        pr.set_fem_resident(resident)
        pos, vel = fst(fs, dtype=torch.float32)
        vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
        for _ in range(2):
            pr.fem_step(pos, vel, max_iters=iters, tol=tol, warm="prev", v_hat=vh, lam=lam)
        forms.append(pr.fem_loop_form())
        outs.append((_np(vh), _np(lam), _np(pos), _np(vel), pr.stats()["iters"]))
    print(f"  {scene}: forms {forms}", flush=True)
    assert forms[0] > 0 and forms[1] == 0
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fem_large_blocks_parity(dtype):
    """Blocks of 6 x 6 x 6 nodes (648 DOF, up to ~460 constrained DOFs: more tile rows than
    the fixed-size operator schedules hold, so the run-time-indexed form runs) against the
    oracle after a fixed number of iterations, and the factorisation of such blocks."""
    Problem, fst = _solver()
    fs = _perturbed(S.fem_scene(seed=S.config_seed(3, 15), blocks=(2, 2, 2), nodes_per_block=6), 7)
    if dtype == torch.float32:
        fs = _round32(fs)
    _, ref = O.fem_step(fs, max_iters=30, tol=0.0, n_threads=8)
    pr = Problem.from_fem(fs, dtype=dtype)
    pos, vel = fst(fs, dtype=dtype)
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    pr.fem_step(pos, vel, max_iters=30, tol=0.0, warm="cold", v_hat=vh, lam=lam)
    assert pr.fem_loop_form() == 0
    vf, lf = _scene_floor(fs)
    ev = np.abs(_np(vh) - ref.v_hat).max() / max(vf, np.abs(ref.v_hat).max())
    el = np.abs(_np(lam) - ref.lam).max() / max(lf, np.abs(ref.lam).max())
    print(f"  {dtype}: v {ev:.3e} lambda {el:.3e}", flush=True)
    tol = 1e-9 if dtype == torch.float64 else 1e-5
    assert ev <= tol and el <= tol
