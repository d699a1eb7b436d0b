"""GPU parity of the GEMM launches whose last round of tiles is split along K (a launch whose
tiles take just over a whole number of rounds of the device's resident GEMM workgroups runs the
whole rounds as usual and the rest in K chunks over the idle workgroups, summed in a fixed
order).  Each case asserts through the event profiler that split launches ran, then checks the
result against the dense CPU oracle (f: rel 1e-10, gradient: rel 1e-8 in the inf-norm).

Cases, on the 512 workgroup slots of an MI355X (256 CUs, two GEMM workgroups each):
- a two-sided split gradient at b = 1024 (four chains): the Schur update (153 lower tiles per
  chain, 612 in all) and the Z_D update (136 per chain, 544) split;
- batched gradients at b = 256: 18 points (36 chains) split the Schur update (540 tiles) and
  the Z_B product (576); 26 points split the Z_D update (520).  Every point is also checked
  against its own single-point gradient, whose launches fit one round (rel 1e-10).

Inputs: seeded synthetic univariate SPDE models (workloads.make_model) on 32 x 32 (b = 1024,
n = 4, a = 6, 200 observations per step) and 16 x 16 grids (b = 256, n = 3, a = 2, 64 per step).
"""
import numpy as np
import pytest
import torch

import oracle
from workloads import make_model

pytestmark = pytest.mark.gpu

SPLIT = "gemm_f64:split_last_round"


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if torch.cuda.get_device_properties(0).multi_processor_count != 256:
        pytest.skip("the cases are sized for 256 CUs")
    return "cuda:0"


def rel_inf(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def test_split_gradient_at_block_size_1024_matches_oracle():
    from paper_2605_06392_amd import bta
    from paper_2605_06392_amd.inla import InlaModel
    dev = _dev()
    spec = make_model(1, 32, 32, 4, 6, 200, 3)
    m = InlaModel(spec, device=dev)
    theta = torch.tensor(spec.theta, device=dev)
    with bta.profile() as P:
        f, g, info = m.grad(theta, split=True)
    assert P.stats.get(SPLIT, {}).get("launches", 0) >= 2, P.stats.keys()
    f, g = f.item(), g.cpu().numpy().copy()
    assert info.item() == 0
    ref = oracle.gradient(spec, spec.theta)
    assert abs(f - ref["f"]) <= 1e-10 * abs(ref["f"])
    assert rel_inf(g, ref["grad"]) <= 1e-8, (g, ref["grad"])
    # bitwise repeatable
    f2, g2, _ = m.grad(theta, split=True)
    assert f2.item() == f and np.array_equal(g2.cpu().numpy(), g)


@pytest.mark.parametrize("points", [18, 26])
def test_batched_gradients_with_split_rounds_match_oracle(points):
    from paper_2605_06392_amd import bta
    from paper_2605_06392_amd.inla import InlaModel
    dev = _dev()
    spec = make_model(1, 16, 16, 3, 2, 64, 7)
    m = InlaModel(spec, device=dev)
    rng = np.random.default_rng(points)
    th = spec.theta + 0.1 * rng.standard_normal((points, spec.d))
    with bta.profile() as P:
        f, g, info = m.grad_batched(torch.tensor(th, device=dev))
    assert P.stats.get(SPLIT, {}).get("launches", 0) >= 1, P.stats.keys()
    f, g = f.cpu().numpy().copy(), g.cpu().numpy().copy()
    assert (info.cpu().numpy() == 0).all()
    for i in (0, points // 2, points - 1):
        ref = oracle.gradient(spec, th[i])
        assert abs(f[i] - ref["f"]) <= 1e-10 * abs(ref["f"]), i
        assert rel_inf(g[i], ref["grad"]) <= 1e-8, i
    for i in range(points):
        f1, g1, _ = m.grad(torch.tensor(th[i], device=dev))
        assert abs(f[i] - f1.item()) <= 1e-12 * abs(f1.item()), i
        assert rel_inf(g[i], g1.cpu().numpy()) <= 1e-10, i
