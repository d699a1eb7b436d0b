"""GPU parity of the posterior Hessian (Sec. III-D, Eq. 12: central differences of exact
gradients over 2d+1 points) and of its finite-difference baseline (second-order central
differences of f over 2d^2+1 points) against the dense CPU oracle.

Tolerances follow from the parity bars of the quantities differenced: each gradient is within
rel 1e-8 of the oracle's, so a column of Eq. 12 is within 2 * 1e-8 * max|g| / 2h; each
objective value is within rel 1e-10, so a second difference is within 4 * 1e-10 * max|f| / h^2.
Inputs: the seeded synthetic models of workloads.spde (k = 1 with d = 4, k = 3 with d = 15,
ragged tiles), h = 5e-3 as in the paper.
"""
import numpy as np
import pytest
import torch

import oracle
from workloads import named_config

pytestmark = pytest.mark.gpu

H_STEP = 5e-3
CASES = [("uni_8x8_nt8", 0), ("uni_9x7_nt4", 3), ("coreg3_4x4_nt4", 0)]

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


@pytest.mark.parametrize("name,seed", [("uni_8x8_nt8", 1), ("coreg3_4x4_nt4", 2)])
def test_batched_gradients_match_oracle_and_pointwise(name, seed):
    """inla_grad_batched over several points (all chains in the same launches) against the
    oracle and against one-point gradients."""
    spec, m = gpu_model(name, seed)
    rng = np.random.default_rng(seed)
    pts = [spec.theta, spec.theta + 0.1 * rng.standard_normal(spec.d),
           spec.theta - 0.05 * rng.standard_normal(spec.d)]
    f, g, info = m.grad_batched(torch.tensor(np.stack(pts)))
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    f, g = f.cpu().numpy(), g.cpu().numpy()
    for p, t in enumerate(pts):
        ref = oracle.gradient(spec, t)
        assert abs(f[p] - ref["f"]) <= 1e-10 * abs(ref["f"])
        assert np.abs(g[p] - ref["grad"]).max() <= 1e-8 * np.abs(ref["grad"]).max()
        f1, g1, _ = m.grad(torch.tensor(t))
        torch.cuda.synchronize()
        assert abs(f[p] - f1.item()) <= 1e-12 * abs(f1.item())
        g1 = g1.cpu().numpy()
        assert np.abs(g[p] - g1).max() <= 1e-10 * np.abs(g1).max()


@pytest.mark.parametrize("name,seed", CASES)
@pytest.mark.parametrize("max_batch", [1, 4, None])
def test_hessian_of_gradients_matches_oracle(name, seed, max_batch):
    spec, m = gpu_model(name, seed)
    f, g, H, info = m.hessian(torch.tensor(spec.theta), h=H_STEP, max_batch=max_batch)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all() and info.numel() == 2 * spec.d + 1
    H_ref, g_ref, f_ref = oracle.hessian_fd_of_grad(spec, spec.theta, h=H_STEP)
    assert abs(f.item() - f_ref) <= 1e-10 * abs(f_ref)
    assert np.abs(g.cpu().numpy() - g_ref).max() <= 1e-8 * np.abs(g_ref).max()
    # gradients at the stencil points are of the size of the centre's plus h |H|
    gmax = np.abs(g_ref).max() + H_STEP * np.abs(H_ref).max()
    bound = 2 * 1e-8 * gmax / (2 * H_STEP)
    assert np.abs(H.cpu().numpy() - H_ref).max() <= bound


@pytest.mark.parametrize("name,seed", CASES)
@pytest.mark.parametrize("max_batch", [None, 7])
def test_fd_hessian_matches_oracle(name, seed, max_batch):
    spec, m = gpu_model(name, seed)
    f, H, info = m.fd_hessian(torch.tensor(spec.theta), h=H_STEP, max_batch=max_batch)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all() and info.numel() == 2 * spec.d ** 2 + 1
    H_ref, f_ref = oracle.fd_hessian(spec, spec.theta, h=H_STEP)
    assert abs(f.item() - f_ref) <= 1e-10 * abs(f_ref)
    Hn = H.cpu().numpy()
    assert np.array_equal(Hn, Hn.T)
    bound = 4 * 1e-10 * 2 * abs(f_ref) / H_STEP ** 2
    assert np.abs(Hn - H_ref).max() <= bound


def test_hessian_symmetric_and_agrees_with_fd_hessian():
    """Two GPU routes (exact gradients vs f alone) agree to their O(h^2) truncation, and the
    Hessian of Eq. 12 is symmetric to the same order."""
    spec, m = gpu_model("uni_12x12_nt6", 4)
    _, _, H, info = m.hessian(torch.tensor(spec.theta), h=H_STEP)
    _, Hf, info_f = m.fd_hessian(torch.tensor(spec.theta), h=H_STEP)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all() and (info_f.cpu().numpy() == 0).all()
    H, Hf = H.cpu().numpy(), Hf.cpu().numpy()
    scale = np.abs(H).max()
    assert np.abs(H - H.T).max() <= 1e-5 * scale
    assert np.abs(H - Hf).max() <= 1e-5 * scale


def test_hessian_graph_replay_matches_eager():
    """The whole Hessian (2d+1 gradients) captured in one graph replays to the eager result,
    with eager work on the same workspace between replays."""
    spec, m = gpu_model("uni_8x8_nt8", 0)
    d = spec.d
    theta = torch.tensor(spec.theta, device="cuda:0")
    f = torch.empty(1, dtype=torch.float64, device="cuda:0")
    g = torch.empty(d, dtype=torch.float64, device="cuda:0")
    H = torch.empty((d, d), dtype=torch.float64, device="cuda:0")
    info = torch.empty(2 * d + 1, dtype=torch.int32, device="cuda:0")
    m.hessian(theta, max_batch=3, f=f, g=g, H=H, info=info)
    torch.cuda.synchronize()
    ref = (f.item(), g.cpu().numpy().copy(), H.cpu().numpy().copy())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        m.hessian(theta, max_batch=3, f=f, g=g, H=H, info=info)
    other = torch.tensor(spec.theta[::-1].copy(), device="cuda:0")
    for _ in range(3):
        H.zero_()
        g.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert f.item() == ref[0] and np.array_equal(g.cpu().numpy(), ref[1])
        assert np.array_equal(H.cpu().numpy(), ref[2])
        m.grad(other)
        torch.cuda.synchronize()


def test_entry_points_reject_bad_arguments():
    """Argument checks of the Hessian, batched-gradient and carry-only entry points (each
    returns before anything is enqueued)."""
    import ctypes as C
    from paper_2605_06392_amd._lib import lib
    from paper_2605_06392_amd.inla import (CARRY_ONLY, MODE_GRAD, MODE_OBJECTIVE,
                                           REUSE_FACTORS)
    spec, m = gpu_model("uni_8x8_nt8", 0)
    d = spec.d
    dev = "cuda:0"
    th = torch.tensor(spec.theta, device=dev)
    f = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(d, dtype=torch.float64, device=dev)
    H = torch.empty((d, d), dtype=torch.float64, device=dev)
    info = torch.empty(2 * d * d + 1, dtype=torch.int32, device=dev)
    ws, nb = m.workspace(1, MODE_GRAD)
    wso, nbo = m.workspace(1, MODE_OBJECTIVE)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def p(t):
        return C.c_void_p(t.data_ptr())

    L = lib()
    assert L.inla_hessian(m._h, p(th), 0.0, 1, p(f), p(g), p(H), p(info), ws, nb, s) == -3
    assert L.inla_hessian(m._h, p(th), 5e-3, 0, p(f), p(g), p(H), p(info), ws, nb, s) == -4
    assert L.inla_hessian(m._h, p(th), 5e-3, 1, p(f), p(g), p(H), p(info), ws, 256, s) == -101
    assert L.inla_fd_hessian(m._h, p(th), -1.0, 1, p(f), p(H), p(info), wso, nbo, s) == -3
    assert L.inla_grad(m._h, p(th), p(f), p(g), p(info), ws, nb, REUSE_FACTORS | CARRY_ONLY,
                       s) == -8
    assert L.inla_grad_batched(m._h, p(th), 0, p(f), p(g), p(info), ws, nb, s) == -3
    assert L.inla_workspace_bytes(m._h, 1, 7) == 0
    assert L.inla_workspace_bytes(m._h, 1, 2) < L.inla_workspace_bytes(m._h, 1, 1)
    torch.cuda.synchronize()


def test_capture_of_very_long_call_is_refused_before_enqueueing():
    """Capturing a call whose estimated launch count passes the library's capture bound (here an
    FD Hessian of 451 points one at a time, about 3.4e5 launches) returns ADELIA_E_UNSUPPORTED
    before anything is enqueued; the model keeps working eagerly afterwards."""
    from paper_2605_06392_amd._lib import AdeliaError
    from paper_2605_06392_amd.inla import InlaModel, MODE_OBJECTIVE
    spec = named_config("coreg3_20x20_nt32", seed=0)
    m = InlaModel(spec, device="cuda:0")
    theta = torch.tensor(spec.theta, device="cuda:0")
    d = spec.d
    f = torch.empty(1, dtype=torch.float64, device="cuda:0")
    H = torch.empty((d, d), dtype=torch.float64, device="cuda:0")
    info = torch.empty(2 * d * d + 1, dtype=torch.int32, device="cuda:0")
    m.workspace(1, MODE_OBJECTIVE)  # allocated outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with pytest.raises(AdeliaError, match="-103"):
        with torch.cuda.graph(graph):
            m.fd_hessian(theta, h=5e-3, max_batch=1, f=f, H=H, info=info)
    torch.cuda.synchronize()
    fo, io = m.objective(theta[None])
    torch.cuda.synchronize()
    assert int(io.item()) == 0 and np.isfinite(fo.item())
    del m
    torch.cuda.empty_cache()
