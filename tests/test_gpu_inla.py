"""GPU parity of the INLA objective and its exact gradient against the dense CPU oracle.

Tolerances: f within rel 1e-10, grad within rel 1e-8 (infinity norm) of the oracle; AD vs GPU
central differences (h = 1e-4) within rel 1e-5.  Inputs are the seeded synthetic models of
workloads.spde at sizes the dense oracle finishes in seconds (several 64-wide tiles, ragged
tails, k = 1 and k = 3 fields).
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from workloads import make_model, named_config

pytestmark = pytest.mark.gpu

CASES = [("uni_8x8_nt8", 0), ("uni_8x8_nt8", 1), ("uni_6x5_nt5", 2), ("coreg3_4x4_nt4", 0),
         ("uni_9x7_nt4", 3), ("uni_12x12_nt6", 4), ("coreg3_5x4_nt3", 5),
         ("coreg3_9x7_nt4", 6), ("coreg3_12x10_nt3", 7)]

_models = {}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return "cuda:0"


def gpu_model(name, seed):
    from paper_2605_06392_amd.inla import InlaModel
    key = (name, seed)
    if key not in _models:
        spec = named_config(name, seed=seed)
        _models[key] = (spec, InlaModel(spec, device=_dev()))
    return _models[key]


def rel_inf(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


@pytest.mark.parametrize("name,seed", CASES)
def test_objective_matches_oracle(name, seed):
    spec, m = gpu_model(name, seed)
    f, info = m.objective(torch.tensor(spec.theta)[None])
    torch.cuda.synchronize()
    ref = oracle.objective(spec, spec.theta)["f"]
    assert int(info.item()) == 0
    assert abs(f.item() - ref) <= 1e-10 * abs(ref)


@pytest.mark.parametrize("name,seed", CASES)
def test_gradient_matches_oracle(name, seed):
    spec, m = gpu_model(name, seed)
    f, g, info = m.grad(torch.tensor(spec.theta))
    torch.cuda.synchronize()
    ref = oracle.gradient(spec, spec.theta)
    assert int(info.item()) == 0
    assert abs(f.item() - ref["f"]) <= 1e-10 * abs(ref["f"])
    assert rel_inf(g.cpu().numpy(), ref["grad"]) <= 1e-8


def test_batched_objective_matches_pointwise():
    spec, m = gpu_model("coreg3_4x4_nt4", 0)
    rng = np.random.default_rng(3)
    th = 0.5 * rng.standard_normal((5, spec.d))
    f, info = m.objective(torch.tensor(th))
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    for p in range(5):
        ref = oracle.objective(spec, th[p])["f"]
        assert abs(f[p].item() - ref) <= 1e-10 * abs(ref)
    f1, _ = m.objective(torch.tensor(th[2])[None])
    torch.cuda.synchronize()
    assert f1.item() == f[2].item()  # the batch position does not change the bits


@pytest.mark.parametrize("name,seed", [("uni_8x8_nt8", 0), ("coreg3_4x4_nt4", 1)])
def test_ad_vs_gpu_fd(name, seed):
    spec, m = gpu_model(name, seed)
    _, g, _ = m.grad(torch.tensor(spec.theta))
    f_fd, g_fd, info = m.fd_grad(torch.tensor(spec.theta), h=1e-4)
    f_sub, g_sub, _ = m.fd_grad(torch.tensor(spec.theta), h=1e-4, max_batch=3)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    assert rel_inf(g_fd.cpu().numpy(), g.cpu().numpy()) <= 1e-5
    assert np.array_equal(g_sub.cpu().numpy(), g_fd.cpu().numpy())
    ref_fd, _ = oracle.fd_gradient(spec, spec.theta, h=1e-4)
    assert rel_inf(g_fd.cpu().numpy(), ref_fd) <= 1e-7


def test_autograd_function():
    from paper_2605_06392_amd.inla import InlaObjective
    spec, m = gpu_model("uni_8x8_nt8", 1)
    theta = torch.tensor(spec.theta, device="cuda:0", requires_grad=True)
    f = InlaObjective.apply(theta, m)
    f.backward()
    torch.cuda.synchronize()
    ref = oracle.gradient(spec, spec.theta)
    assert abs(f.item() - ref["f"]) <= 1e-10 * abs(ref["f"])
    assert rel_inf(theta.grad.cpu().numpy(), ref["grad"]) <= 1e-8
    # an intervening forward on another point forces the backward to recompute the factors
    theta2 = torch.tensor(spec.theta, device="cuda:0", requires_grad=True)
    f2 = InlaObjective.apply(theta2 * 1.0, m)
    other = torch.tensor(spec.theta[::-1].copy(), device="cuda:0", requires_grad=True)
    InlaObjective.apply(other, m)
    (3.0 * f2).backward()
    torch.cuda.synchronize()
    assert rel_inf(theta2.grad.cpu().numpy(), 3.0 * ref["grad"]) <= 1e-8


def test_golden_values():
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")
    gold = json.load(open(path))
    for key, val in gold.items():
        name, seed = key.split(":")
        spec, m = gpu_model(name, int(seed))
        assert np.allclose(spec.theta, val["theta"])
        f, g, _ = m.grad(torch.tensor(spec.theta))
        torch.cuda.synchronize()
        assert abs(f.item() - val["f"]) <= 1e-10 * abs(val["f"])
        assert rel_inf(g.cpu().numpy(), val["grad"]) <= 1e-8


# k = 2 and k = 4 coregionalised fields (d = 9 and 22): every field pair of the sub-diagonal
# blocks, whose coefficients the selected inversion rebuilds from theta for W_t = B_t G^T G,
# and b = 80 spanning a full and a ragged 64-wide panel
@pytest.mark.parametrize("k,nx,ny,nt,a,obs", [(2, 6, 5, 4, 3, 8), (4, 4, 3, 3, 2, 6),
                                              (4, 5, 4, 3, 3, 8)])
def test_two_and_four_fields_match_oracle(k, nx, ny, nt, a, obs):
    from paper_2605_06392_amd.inla import InlaModel
    spec = make_model(k, nx, ny, nt, a, obs, seed=21)
    m = InlaModel(spec, device=_dev())
    print(f"k={k} b={k * nx * ny} n={nt} a={a} d={spec.d}", flush=True)
    ref = oracle.gradient(spec, spec.theta)
    for carry in (False, True):
        f, g, info = m.grad(torch.tensor(spec.theta), carry=carry)
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        assert abs(f.item() - ref["f"]) <= 1e-10 * abs(ref["f"]), carry
        assert rel_inf(g.cpu().numpy(), ref["grad"]) <= 1e-8, carry


@pytest.mark.parametrize("k", [1, 3])
def test_no_observations_gives_prior(k):
    from paper_2605_06392_amd.inla import InlaModel
    spec = make_model(k, 4, 3, 3, 2, 0, seed=11)
    m = InlaModel(spec, device=_dev())
    f, g, info = m.grad(torch.tensor(spec.theta))
    torch.cuda.synchronize()
    s2 = spec.sigma_prior ** 2
    logp = np.sum(-spec.theta ** 2 / (2 * s2)) - 0.5 * spec.d * np.log(2 * np.pi * s2)
    assert abs(f.item() - logp) <= 1e-10 * abs(logp)
    assert np.allclose(g.cpu().numpy(), -spec.theta / s2, rtol=1e-9, atol=1e-9)


def test_repeat_runs_bitwise_identical():
    spec, m = gpu_model("uni_12x12_nt6", 4)
    outs = []
    for _ in range(3):
        f, g, _ = m.grad(torch.tensor(spec.theta))
        torch.cuda.synchronize()
        outs.append((f.item(), g.cpu().numpy().copy()))
    for f, g in outs[1:]:
        assert f == outs[0][0] and np.array_equal(g, outs[0][1])


def test_graph_replay_matches_eager():
    """A captured gradient replays to the eager result, with eager work on the same workspace
    between replays."""
    spec, m = gpu_model("uni_12x12_nt6", 4)
    theta = torch.tensor(spec.theta, device="cuda:0")
    f = torch.empty(1, dtype=torch.float64, device="cuda:0")
    g = torch.empty(spec.d, dtype=torch.float64, device="cuda:0")
    info = torch.empty(1, dtype=torch.int32, device="cuda:0")
    m.grad(theta, f=f, g=g, info=info)
    torch.cuda.synchronize()
    f_ref, g_ref = f.item(), g.cpu().numpy().copy()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        m.grad(theta, f=f, g=g, info=info)
    other = torch.tensor(spec.theta[::-1].copy(), device="cuda:0")
    for _ in range(3):
        f.zero_()
        g.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert f.item() == f_ref and np.array_equal(g.cpu().numpy(), g_ref)
        m.grad(other)  # eager work on the same workspace in between
        torch.cuda.synchronize()


@pytest.mark.parametrize("name,seed", [("uni_8x8_nt8", 0), ("coreg3_4x4_nt4", 0)])
def test_gradient_phases_match_oracle(name, seed):
    spec, m = gpu_model(name, seed)
    t = m.grad_terms(torch.tensor(spec.theta))
    ref = oracle.gradient(spec, spec.theta)
    ev = oracle.objective(spec, spec.theta)
    scale = np.abs(ref["grad"]).max()
    for key in ("phaseA", "phaseB", "phaseC", "dloglik", "dlogprior", "grad"):
        assert np.abs(t[key] - ref[key]).max() <= 1e-8 * max(scale, np.abs(ref[key]).max()), key
    assert abs(t["logdet_p"] - ev["logdet_p"]) <= 1e-11 * abs(ev["logdet_p"])
    assert abs(t["logdet_c"] - ev["logdet_c"]) <= 1e-11 * abs(ev["logdet_c"])
    nb = spec.nt * spec.b
    assert abs(t["trZT"] - np.trace(ref["Zc"][nb:, nb:])) <= 1e-10 * abs(t["trZT"])


def test_large_batches_split_panels_match_oracle():
    """Batches whose panel workgroups outnumber the CUs factor each panel's diagonal tile once
    per chain and solve its rows with a GEMM: objectives of 150 points and gradients of 60
    points (300 and 120 chains) against the oracle at a few points and against one-point
    evaluations everywhere."""
    spec, m = gpu_model("uni_8x8_nt8", 0)
    rng = np.random.default_rng(17)
    pts = spec.theta + 0.2 * rng.standard_normal((150, spec.d))
    f, info = m.objective(torch.tensor(pts))
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    f = f.cpu().numpy()
    for p in (0, 77, 149):
        ref = oracle.objective(spec, pts[p])["f"]
        assert abs(f[p] - ref) <= 1e-10 * abs(ref)
    for p in range(0, 150, 10):
        f1, _ = m.objective(torch.tensor(pts[p])[None])
        assert abs(f[p] - f1.item()) <= 1e-12 * abs(f1.item())
    gp = pts[:60]
    fg, g, info = m.grad_batched(torch.tensor(gp))
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    g = g.cpu().numpy()
    for p in (0, 31, 59):
        ref = oracle.gradient(spec, gp[p])
        assert np.abs(g[p] - ref["grad"]).max() <= 1e-8 * np.abs(ref["grad"]).max()
    for p in range(0, 60, 6):
        _, g1, _ = m.grad(torch.tensor(gp[p]))
        g1 = g1.cpu().numpy()
        assert np.abs(g[p] - g1).max() <= 1e-10 * np.abs(g1).max()


@pytest.mark.parametrize("name,seed", [("uni_8x8_nt8", 0), ("uni_9x7_nt4", 3), ("coreg3_4x4_nt4", 0),
                                       ("coreg3_9x7_nt4", 6)])
def test_carry_only_gradient_matches_oracle_and_stored(name, seed):
    """The carry-only memory mode (factors rebuilt block by block in the backward pass from the
    stored Schur-updated diagonal blocks) against the oracle and against the stored-factor
    gradient, phase by phase."""
    spec, m = gpu_model(name, seed)
    t_c = m.grad_terms(torch.tensor(spec.theta), carry=True)
    t_s = m.grad_terms(torch.tensor(spec.theta))
    assert t_c["info"] == 0
    ref = oracle.gradient(spec, spec.theta)
    assert abs(t_c["f"] - ref["f"]) <= 1e-10 * abs(ref["f"])
    assert rel_inf(t_c["grad"], ref["grad"]) <= 1e-8
    scale = np.abs(t_s["grad"]).max()
    for key in ("phaseA", "phaseB", "phaseC", "dloglik", "grad"):
        assert np.abs(t_c[key] - t_s[key]).max() <= 1e-12 * scale, key
    f, g, info = m.grad(torch.tensor(spec.theta), carry=True)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert np.abs(g.cpu().numpy() - t_s["grad"]).max() <= 1e-12 * scale


def test_carry_only_workspace_is_smaller():
    from paper_2605_06392_amd.inla import MODE_GRAD, MODE_GRAD_CARRY
    spec, m = gpu_model("uni_12x12_nt6", 4)
    stored = m.workspace_bytes(1, MODE_GRAD)
    carry = m.workspace_bytes(1, MODE_GRAD_CARRY)
    assert 0 < carry < stored


def test_saved_factors_are_consumed_once():
    """A reverse pass reusing saved factors consumes them: a second backward of the same f
    recomputes (same gradient), a gradient on another point in between forces a recompute, and a
    second raw REUSE call on the workspace is rejected with ADELIA_E_STATE."""
    from paper_2605_06392_amd.inla import InlaObjective
    spec, m = gpu_model("uni_8x8_nt8", 1)
    ref = oracle.gradient(spec, spec.theta)
    theta = torch.tensor(spec.theta, device="cuda:0", requires_grad=True)
    f = InlaObjective.apply(theta, m)
    f.backward(retain_graph=True)
    g1 = theta.grad.cpu().numpy().copy()
    theta.grad = None
    f.backward()
    g2 = theta.grad.cpu().numpy().copy()
    assert rel_inf(g1, ref["grad"]) <= 1e-8 and rel_inf(g2, ref["grad"]) <= 1e-8
    theta3 = torch.tensor(spec.theta, device="cuda:0", requires_grad=True)
    f3 = InlaObjective.apply(theta3, m)
    m.grad(torch.tensor(spec.theta[::-1].copy()))  # same workspace, another point
    f3.backward()
    assert rel_inf(theta3.grad.cpu().numpy(), ref["grad"]) <= 1e-8
    m.forward_saved(torch.tensor(spec.theta))
    m.grad(torch.tensor(spec.theta), reuse=True)
    from paper_2605_06392_amd._lib import AdeliaError
    with pytest.raises(AdeliaError, match="-104"):
        m.grad(torch.tensor(spec.theta), reuse=True)
    torch.cuda.synchronize()


def test_carry_only_graph_replay_matches_eager():
    """A captured carry-only gradient (three streams in its reverse pass) replays to the eager
    result, with other work on the model in between."""
    spec, m = gpu_model("uni_12x12_nt6", 4)
    theta = torch.tensor(spec.theta, device="cuda:0")
    f = torch.empty(1, dtype=torch.float64, device="cuda:0")
    g = torch.empty(spec.d, dtype=torch.float64, device="cuda:0")
    info = torch.empty(1, dtype=torch.int32, device="cuda:0")
    m.grad(theta, f=f, g=g, info=info, carry=True)
    torch.cuda.synchronize()
    f_ref, g_ref = f.item(), g.cpu().numpy().copy()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        m.grad(theta, f=f, g=g, info=info, carry=True)
    other = torch.tensor(spec.theta[::-1].copy(), device="cuda:0")
    for _ in range(3):
        f.zero_()
        g.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert f.item() == f_ref and np.array_equal(g.cpu().numpy(), g_ref)
        m.grad(other, carry=True)
        m.grad(other)
        torch.cuda.synchronize()


def test_batch_runner_replays_batched_evaluations():
    """BatchRunner: graph-captured batched objectives and gradients equal the eager batched
    calls on new points at every call."""
    import paper_2605_06392_amd as adelia
    spec, m = gpu_model("uni_8x8_nt8", 0)
    rng = np.random.default_rng(5)
    obj = adelia.BatchRunner(m, 5, "objective")
    grd = adelia.BatchRunner(m, 3, "grad")
    for _ in range(3):
        pts = spec.theta + 0.1 * rng.standard_normal((5, spec.d))
        f, info = obj(pts)
        f = f.cpu().numpy().copy()
        fe, _ = m.objective(torch.tensor(pts))
        assert (info.cpu().numpy() == 0).all()
        assert np.array_equal(f, fe.cpu().numpy())
        f3, g3, info3 = grd(pts[:3])
        g3 = g3.cpu().numpy().copy()
        _, ge, _ = m.grad_batched(torch.tensor(pts[:3]))
        assert (info3.cpu().numpy() == 0).all()
        assert np.array_equal(g3, ge.cpu().numpy())
    f0, g0, _ = adelia.fd_grad(m, torch.tensor(spec.theta), h=1e-4)
    assert np.isfinite(g0.cpu().numpy()).all()


def test_lookahead_stream_schedule_matches_oracle():
    """Objectives and gradients of 16 points of uni_12x12_nt6 in one pass: 32 chains with 6
    panel workgroups each (192 <= 256 CUs, so no split panels; 384 > 256, so no fused steps) run
    each panel's trailing update on the look-ahead stream, the schedule of a single b = 2700
    gradient.  Against the oracle at three points, and bitwise repeatable."""
    spec, m = gpu_model("uni_12x12_nt6", 4)
    rng = np.random.default_rng(23)
    pts = spec.theta + 0.2 * rng.standard_normal((16, spec.d))
    fo, info_o = m.objective(torch.tensor(pts))
    f, g, info = m.grad_batched(torch.tensor(pts))
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all() and (info_o.cpu().numpy() == 0).all()
    f, g, fo = f.cpu().numpy().copy(), g.cpu().numpy().copy(), fo.cpu().numpy().copy()
    for p in (0, 7, 15):
        ref = oracle.gradient(spec, pts[p])
        assert abs(f[p] - ref["f"]) <= 1e-10 * abs(ref["f"]), p
        assert abs(fo[p] - ref["f"]) <= 1e-10 * abs(ref["f"]), p
        assert rel_inf(g[p], ref["grad"]) <= 1e-8, p
    f2, g2, _ = m.grad_batched(torch.tensor(pts))
    torch.cuda.synchronize()
    assert np.array_equal(f2.cpu().numpy(), f) and np.array_equal(g2.cpu().numpy(), g)


def test_nan_theta_reports_failure():
    """A NaN hyperparameter makes every pivot NaN: the pivot check reports the first column
    (info = 1) for the objective, the gradient and every FD stencil point, and the call itself
    still returns 0 (numerical failure is asynchronous)."""
    spec, m = gpu_model("uni_8x8_nt8", 0)
    th = spec.theta.copy()
    th[1] = np.nan
    _, info = m.objective(torch.tensor(th)[None])
    _, _, ginfo = m.grad(torch.tensor(th))
    _, _, finfo = m.fd_grad(torch.tensor(th), h=1e-4)
    torch.cuda.synchronize()
    assert int(info.item()) == 1
    assert int(ginfo.item()) == 1
    assert (finfo.cpu().numpy() == 1).all()
    # the model is unharmed: the next evaluation is correct
    f, _ = m.objective(torch.tensor(spec.theta)[None])
    torch.cuda.synchronize()
    ref = oracle.objective(spec, spec.theta)["f"]
    assert abs(f.item() - ref) <= 1e-10 * abs(ref)


def test_double_backward_raises():
    """The hand-written reverse pass is not itself differentiable: asking for a second-order
    derivative through it raises instead of returning a wrong one."""
    from paper_2605_06392_amd.inla import InlaObjective
    spec, m = gpu_model("uni_8x8_nt8", 0)
    theta = torch.tensor(spec.theta, device="cuda:0", requires_grad=True)
    f = InlaObjective.apply(theta, m)
    # with a constant output gradient the result carries no graph at all: there is nothing to
    # differentiate, so no second derivative can come back silently
    (g,) = torch.autograd.grad(f, theta, create_graph=True)
    ref = oracle.gradient(spec, spec.theta)
    assert rel_inf(g.detach().cpu().numpy(), ref["grad"]) <= 1e-8
    assert not g.requires_grad
    # with an output gradient that itself requires grad, differentiating again raises
    f = InlaObjective.apply(theta, m)
    seed = torch.ones((), dtype=torch.float64, device="cuda:0", requires_grad=True)
    (g,) = torch.autograd.grad(f, theta, grad_outputs=seed, create_graph=True)
    assert rel_inf(g.detach().cpu().numpy(), ref["grad"]) <= 1e-8
    with pytest.raises(RuntimeError, match="twice"):
        g.sum().backward()


def test_batch_runner_replay_keeps_saved_factors():
    """A one-point gradient runner replayed between InlaObjective.forward and backward works in
    its own workspace: the backward still reuses the factors of its own forward pass and gives
    the oracle's gradient."""
    import paper_2605_06392_amd as adelia
    from paper_2605_06392_amd.inla import InlaObjective
    spec, m = gpu_model("uni_8x8_nt8", 1)
    runner = adelia.BatchRunner(m, 1, "grad")
    other = spec.theta[::-1].copy()
    runner(other[None])  # captures
    theta = torch.tensor(spec.theta, device="cuda:0", requires_grad=True)
    f = InlaObjective.apply(theta, m)
    token = m.saved_token
    _, g_other, _ = runner(other[None])  # replay on another point
    assert m.saved_token == token
    f.backward()
    torch.cuda.synchronize()
    ref = oracle.gradient(spec, spec.theta)
    assert rel_inf(theta.grad.cpu().numpy(), ref["grad"]) <= 1e-8
    ref_o = oracle.gradient(spec, other)
    assert rel_inf(g_other[0].cpu().numpy(), ref_o["grad"]) <= 1e-8


def test_long_pattern_rows_match_oracle():
    """A mesh whose stiffness matrix couples node 0 with twelve distant nodes (each pair adds the
    positive semidefinite eps (e_0 - e_j)(e_0 - e_j)^T) has a pattern row of more than 16
    entries, longer than the banded W_t kernel holds in registers, so W_t = B_t G_t^T G_t goes
    through the LDS-batched kernel, per block and for all blocks at once (split).  f and the
    gradient match the oracle on the same matrices."""
    import dataclasses
    import scipy.sparse as sp
    from paper_2605_06392_amd.inla import InlaModel
    dev = _dev()
    spec = make_model(1, 8, 6, 5, 3, 9, 31)
    ns = spec.nx * spec.ny
    g1 = spec.g1.tolil()
    eps = 0.05
    for j in range(ns - 12, ns):
        g1[0, 0] += eps
        g1[j, j] += eps
        g1[0, j] -= eps
        g1[j, 0] -= eps
    spec = dataclasses.replace(spec, g1=sp.csr_matrix(g1))
    union = (abs(spec.c0) + abs(spec.g1) + abs(spec.g2)).tocsr()
    assert np.diff(union.indptr).max() > 16
    m = InlaModel(spec, device=dev)
    th = torch.tensor(spec.theta)
    ref = oracle.gradient(spec, spec.theta)
    for split in (False, True):
        f, g, info = m.grad(th, split=split)
        torch.cuda.synchronize()
        assert int(info.item()) == 0, split
        assert abs(f.item() - ref["f"]) <= 1e-10 * abs(ref["f"]), split
        assert rel_inf(g.cpu().numpy(), ref["grad"]) <= 1e-8, split


@pytest.mark.parametrize("k,nx,ny,nt,obs,seed", [(1, 6, 5, 5, 6, 51), (3, 4, 3, 4, 4, 52)])
def test_no_fixed_effects_match_oracle(k, nx, ny, nt, obs, seed):
    """a = 0: the arrow holds only the right-hand-side row (no V, no Z_C products, an empty
    tip), for the plain sweep, the two-sided split and the carry-only mode."""
    from paper_2605_06392_amd.inla import InlaModel
    spec = make_model(k, nx, ny, nt, 0, obs, seed=seed)
    m = InlaModel(spec, device=_dev())
    ref = oracle.gradient(spec, spec.theta)
    th = torch.tensor(spec.theta)
    for kw in ({}, {"split": True}, {"carry": True}):
        f, g, info = m.grad(th, **kw)
        torch.cuda.synchronize()
        assert int(info.item()) == 0, kw
        assert abs(f.item() - ref["f"]) <= 1e-10 * abs(ref["f"]), kw
        assert rel_inf(g.cpu().numpy(), ref["grad"]) <= 1e-8, kw
        fo, io = m.objective(th[None], **kw) if "carry" not in kw else m.objective(th[None])
        torch.cuda.synchronize()
        assert int(io.item()) == 0, kw
        assert abs(fo.item() - ref["f"]) <= 1e-10 * abs(ref["f"]), kw


def test_many_fixed_effects_match_oracle():
    """a = 10 > 8 arrow rows: V_t = L_Ct G_t and Z_Ct go through the tile GEMM instead of the
    short-product kernel (plain sweep, split, carry-only)."""
    from paper_2605_06392_amd.inla import InlaModel
    spec = make_model(1, 6, 5, 5, 10, 12, seed=53)
    m = InlaModel(spec, device=_dev())
    ref = oracle.gradient(spec, spec.theta)
    th = torch.tensor(spec.theta)
    for kw in ({}, {"split": True}, {"carry": True}):
        f, g, info = m.grad(th, **kw)
        torch.cuda.synchronize()
        assert int(info.item()) == 0, kw
        assert abs(f.item() - ref["f"]) <= 1e-10 * abs(ref["f"]), kw
        assert rel_inf(g.cpu().numpy(), ref["grad"]) <= 1e-8, kw
