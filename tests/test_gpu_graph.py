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


def test_graph_recaptures_after_configuration_changes():
    """Options, attached networks and a network's input normalisation are captured into the
    graph's launches; after each change the next graph step must equal an eager step
    (a replay of the old graph would run the old contact model, kernel form or network)."""
    from paper_2302_14344_amd.solver import Mlp
    sc = S.legged_scenes(64, seed=S.config_seed(2, 22))
    kw = dict(max_iters=1000, tol=1e-6)
    (p1, s1, v1, l1), (p2, s2, v2, l2) = _pair(sc, torch.float32)
    nc, nj = p1.warm_class_counts()
    rng = np.random.default_rng(5)

    def nets_for(seed):
        r = np.random.default_rng(seed)
        out = []
        for nin, nout, n in ((12, 6, nc), (27, 15, nj)):
            params = np.concatenate([r.normal(0, 0.02, nin * nout), r.normal(0, 0.01, nout)])
            pair = []
            for _ in range(2):
                net = Mlp([nin, nout], max(n, 1))
                net.set_params(params)
                pair.append(net)
            out.append(pair)
        return out

    def attach(nets):
        for c in (0, 1):
            p1.set_warm_model(c, nets[c][0])
            p2.set_warm_model(c, nets[c][1])

    def step(warm, what):
        print(f"graph step after: {what}", flush=True)
        p1.rigid_step(*s1, warm=warm, v_hat=v1, lam=l1, **kw)
        p2.rigid_step(*s2, warm=warm, v_hat=v2, lam=l2, graph=True, **kw)
        torch.cuda.synchronize()
        for a, b in zip((*s1, v1, l1), (*s2, v2, l2)):
            np.testing.assert_array_equal(_np(a), _np(b), err_msg=what)
        np.testing.assert_array_equal(p1.stats()["iters"], p2.stats()["iters"], err_msg=what)

    step("prev", "first capture")
    step("prev", "replay")
    for pr in (p1, p2):
        pr.set_contact_model(relaxed=True)
    step("prev", "contact model relaxed")
    for pr in (p1, p2):
        pr.set_contact_model(relaxed=False)
        pr.set_split_rows(True)
    step("prev", "exact contacts, split rows")
    a = nets_for(11)
    attach(a)
    step("learned", "networks A")
    step("learned", "networks A, replay")
    b = nets_for(12)
    attach(b)
    step("learned", "networks B swapped in")
    scale = rng.uniform(0.5, 2.0, 12).astype(np.float32)
    shift = rng.normal(0, 0.1, 12).astype(np.float32)
    for net in b[0]:
        net.set_input_affine(scale, shift)
    step("learned", "contact network input affine set")
    for pr in (p1, p2):
        pr.set_learned_budget(7)
    step("learned", "learned budget 7")
    p1.check()
    p2.check()
    del a, b


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_fem_graph_replays_match_eager_steps(dtype):
    """The FEM step (construction, factorisation, the resident iteration, v_hat and state
    update) replayed from a HIP graph equals the eager steps bit for bit, with eager GPU work
    between the replays, and a change of max_iters captures again."""
    from paper_2302_14344_amd.solver import Problem, fem_state_tensors
    fs = S.fem_scene(seed=S.config_seed(3, 11), blocks=(2, 2, 2), nodes_per_block=4)
    pa, pb = Problem.from_fem(fs, dtype=dtype), Problem.from_fem(fs, dtype=dtype)
    sa, sb = fem_state_tensors(fs, dtype=dtype), fem_state_tensors(fs, dtype=dtype)
    la, lb = pa.empty(pa.sizes.n_rows), pb.empty(pb.sizes.n_rows)
    junk = torch.zeros(1 << 16, device="cuda")
    for k, iters in enumerate((300, 300, 300, 120, 120)):
        print(f"FEM {dtype} step {k}, max_iters {iters}", flush=True)
        pa.fem_step(*sa, max_iters=iters, lam=la)
        pb.fem_step(*sb, max_iters=iters, lam=lb, graph=True)
        junk.add_(1.0)
        torch.cuda.synchronize()
        for x, y in zip((*sa, la), (*sb, lb)):
            np.testing.assert_array_equal(_np(x), _np(y))
        np.testing.assert_array_equal(pa.stats()["iters"], pb.stats()["iters"])
    pa.check()
    pb.check()
