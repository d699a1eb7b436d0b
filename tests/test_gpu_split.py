"""GPU parity of the two-sided split (ADELIA_SPLIT; the two-phase decomposition with two
partitions on one GPU): the objective and the exact gradient with the block chain swept from
both ends at once and the separator block with the tip as the reduced system, against the dense
oracle (f: rel 1e-10, gradient: rel 1e-8) and against the unsplit sweep.  Cases: univariate and
three-field models with several 64-wide panels and ragged tails, halves of equal and unequal
length, the shortest chain that splits (three blocks), and the refusal below it."""
import numpy as np
import pytest
import torch

import oracle
from workloads import make_model, named_config

pytestmark = pytest.mark.gpu

CASES = [("uni_8x8_nt8", 0), ("uni_6x5_nt5", 2), ("coreg3_4x4_nt4", 0), ("uni_12x12_nt6", 4),
         ("coreg3_9x7_nt4", 6), ("coreg3_12x10_nt3", 7)]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return "cuda:0"


def rel_inf(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


_models = {}


def _model(name, seed):
    from paper_2605_06392_amd.inla import InlaModel
    if (name, seed) not in _models:
        spec = named_config(name, seed=seed)
        _models[(name, seed)] = (spec, InlaModel(spec, device=_dev()))
    return _models[(name, seed)]


@pytest.mark.parametrize("name,seed", CASES)
def test_split_objective_and_gradient_match_oracle(name, seed):
    spec, m = _model(name, seed)
    print(f"split {name} seed {seed} nt {spec.nt}", flush=True)
    th = torch.tensor(spec.theta)
    fo, io = m.objective(th[None], split=True)
    f, g, info = m.grad(th, split=True)
    torch.cuda.synchronize()
    ref = oracle.gradient(spec, spec.theta)
    assert int(io.item()) == 0 and int(info.item()) == 0
    assert abs(fo.item() - ref["f"]) <= 1e-10 * abs(ref["f"])
    assert abs(f.item() - ref["f"]) <= 1e-10 * abs(ref["f"])
    assert rel_inf(g.cpu().numpy(), ref["grad"]) <= 1e-8
    # and the unsplit sweep, up to rounding
    f1, g1, _ = m.grad(th)
    torch.cuda.synchronize()
    assert abs(f.item() - f1.item()) <= 1e-12 * abs(f1.item())
    assert rel_inf(g.cpu().numpy(), g1.cpu().numpy()) <= 1e-10


def test_split_shortest_chain_and_refusal():
    from paper_2605_06392_amd._lib import AdeliaError
    from paper_2605_06392_amd.inla import InlaModel
    dev = _dev()
    spec = make_model(1, 7, 6, 3, 3, 9, 41)  # three blocks: one per half and the separator
    m = InlaModel(spec, device=dev)
    f, g, info = m.grad(torch.tensor(spec.theta), split=True)
    torch.cuda.synchronize()
    ref = oracle.gradient(spec, spec.theta)
    assert int(info.item()) == 0
    assert abs(f.item() - ref["f"]) <= 1e-10 * abs(ref["f"])
    assert rel_inf(g.cpu().numpy(), ref["grad"]) <= 1e-8
    spec2 = make_model(1, 7, 6, 2, 3, 9, 42)
    m2 = InlaModel(spec2, device=dev)
    assert m2.workspace_bytes(1, 4) == 0
    with pytest.raises((AdeliaError, ValueError)):
        m2.grad(torch.tensor(spec2.theta), split=True)


def test_split_repeatable_and_graph_replay():
    spec, m = _model("uni_12x12_nt6", 4)
    th = torch.tensor(spec.theta, device="cuda:0")
    f = torch.empty(1, dtype=torch.float64, device="cuda:0")
    g = torch.empty(spec.d, dtype=torch.float64, device="cuda:0")
    info = torch.empty(1, dtype=torch.int32, device="cuda:0")
    m.grad(th, f=f, g=g, info=info, split=True)
    torch.cuda.synchronize()
    f0, g0 = f.item(), g.cpu().numpy().copy()
    m.grad(th, f=f, g=g, info=info, split=True)
    torch.cuda.synchronize()
    assert f.item() == f0 and np.array_equal(g.cpu().numpy(), g0)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        m.grad(th, f=f, g=g, info=info, split=True)
    rng = np.random.default_rng(3)
    for _ in range(3):
        pt = spec.theta + 0.2 * rng.standard_normal(spec.d)
        th.copy_(torch.tensor(pt))
        graph.replay()
        torch.cuda.synchronize()
        fr, gr = f.item(), g.cpu().numpy().copy()
        fe, ge, _ = m.grad(torch.tensor(pt), split=True)
        torch.cuda.synchronize()
        assert fr == fe.item() and np.array_equal(gr, ge.cpu().numpy())
        ref = oracle.gradient(spec, pt)
        assert rel_inf(gr, ref["grad"]) <= 1e-8
