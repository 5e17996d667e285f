"""The rigid step replayed from a HIP graph gives bit for bit the results of the same
steps run eagerly: every replay is checked, with unrelated eager GPU work and
synchronisations between the replays, and a change of arguments captures again."""
import numpy as np
import pytest
import torch

from paper_2302_14344_amd import scenes as S

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _pair(sc, dtype):
    from paper_2302_14344_amd.solver import Problem, rigid_state_tensors
    out = []
    for _ in range(2):
        pr = Problem.from_rigid(sc, dtype=dtype)
        st = rigid_state_tensors(sc, dtype=dtype)
        vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
        out.append((pr, st, vh, lam))
    return out


def _constant_nets(pr):
    from paper_2302_14344_amd.solver import Mlp
    nc, nj = pr.warm_class_counts()
    nets = []
    rng = np.random.default_rng(3)
    for c, (nin, nout, n) in enumerate(((12, 6, nc), (27, 15, nj))):
        net = Mlp([nin, nout], max(n, 1))
        net.set_params(np.concatenate([np.zeros(nin * nout), rng.normal(0, 0.01, nout)]))
        pr.set_warm_model(c, net)
        nets.append(net)
    return nets


@pytest.mark.parametrize("case", ["legged-fp32", "chain-fp64", "legged-learned"])
def test_graph_replays_match_eager_steps(case):
    print(f"case {case}", flush=True)
    if case == "chain-fp64":
        sc, dtype, kw = S.chain_scene(S.config_seed(1)), torch.float64, dict(max_iters=200, tol=1e-8)
    else:
        sc, dtype, kw = S.legged_scenes(64, seed=S.config_seed(2, 21)), torch.float32, dict(max_iters=1000, tol=1e-6)
    warm = "learned" if case == "legged-learned" else "prev"
    (p1, s1, v1, l1), (p2, s2, v2, l2) = _pair(sc, dtype)
    nets = (_constant_nets(p1), _constant_nets(p2)) if warm == "learned" else None
    noise = torch.randn(1 << 20, device="cuda")
    for k in range(8):
        dt = sc.dt if k < 5 else 0.5 * sc.dt  # the change of dt captures a new graph
        p1.rigid_step(*s1, dt=dt, warm=warm, v_hat=v1, lam=l1, **kw)
        p2.rigid_step(*s2, dt=dt, warm=warm, v_hat=v2, lam=l2, graph=True, **kw)
        torch.cuda.synchronize()
        for a, b in zip((*s1, v1, l1), (*s2, v2, l2)):
            np.testing.assert_array_equal(_np(a), _np(b))
        np.testing.assert_array_equal(p1.stats()["iters"], p2.stats()["iters"])
        # unrelated eager work between replays
        noise.mul_(1.0001).add_(noise.sum() * 0.0)
        torch.cuda.synchronize()
    p1.check()
    p2.check()
    del nets
