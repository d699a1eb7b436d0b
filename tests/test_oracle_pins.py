"""Pins for the dense oracle: each check compares it with something other than itself.

* brute-force (Leibniz) determinants on tiny inputs,
* closed-form spectral log-determinants of the prior (cosine eigenbasis of the grid Laplacian,
  continuant recurrence for the per-mode temporal tridiagonals),
* complex-step derivatives (analytic to rounding) of the prior precision and of the objective
  evaluated through LU instead of Cholesky,
* exact special cases (no observations; the theta1 scale identity; theta1 + tau identity),
* the coregional weights of Eq. 9 written directly from the paper,
* BTA selected-inverse identities.
"""
import itertools

import numpy as np
import pytest

import oracle
from workloads import make_model, named_config, neumann_second_difference
from workloads.bta import random_bta

from tests import spectral


def leibniz_det(M):
    n = M.shape[0]
    total = 0.0
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        prod = 1.0
        for i in range(n):
            prod *= M[i, perm[i]]
        total += (-1) ** inv * prod
    return total


def continuant_logdet(diag, off):
    return spectral.continuant_logdet(diag, off)


def spectral_field_logdet(model, rng_par, tmp_par):
    return spectral.field_logdet(model, rng_par, tmp_par)


def tiny_model(seed=3, a=1, obs=2):
    return make_model(1, 2, 1, 2, a, obs, seed)


# --------------------------------------------------------------------------------------------

def test_generator_deterministic():
    m1 = named_config("uni_6x5_nt5", seed=5)
    m2 = named_config("uni_6x5_nt5", seed=5)
    for f in ("obs_node", "obs_w", "X", "y", "theta"):
        assert np.array_equal(getattr(m1, f), getattr(m2, f))
    m3 = named_config("uni_6x5_nt5", seed=6)
    assert not np.array_equal(m1.y, m3.y)


def test_leibniz_logdets_tiny():
    m = tiny_model()
    assert m.N <= 7
    ev = oracle.objective(m, m.theta)
    assert np.isclose(ev["logdet_p"], np.log(leibniz_det(ev["Qp"])), rtol=1e-13, atol=1e-13)
    assert np.isclose(ev["logdet_c"], np.log(leibniz_det(ev["Qc"])), rtol=1e-13, atol=1e-13)


def test_bta_pattern_of_prior():
    m = named_config("uni_6x5_nt5", seed=1)
    Qp = oracle.prior_precision(m, m.theta)
    b = m.b
    for i in range(m.nt - 2):
        assert np.all(Qp[(i + 2) * b:(i + 3) * b, i * b:(i + 1) * b] == 0.0)
    assert np.all(Qp[:m.nt * b, m.nt * b:] == 0.0)  # prior has no arrow
    assert np.array_equal(Qp, Qp.T)


@pytest.mark.parametrize("name,seed", [("uni_6x5_nt5", 0), ("uni_8x8_nt8", 1), ("uni_9x7_nt4", 2)])
def test_prior_logdet_spectral_univariate(name, seed):
    m = named_config(name, seed=seed)
    th = m.theta
    ld = oracle.objective(m, th)["logdet_p"]
    ref = m.ns * m.nt * th[0] + spectral_field_logdet(m, th[1], th[2]) + m.a * np.log(m.tip_prec)
    assert np.isclose(ld, ref, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("name,seed", [("coreg3_4x4_nt4", 0), ("coreg3_5x4_nt3", 4)])
def test_prior_logdet_spectral_coreg(name, seed):
    m = named_config(name, seed=seed)
    th = m.theta
    lay = oracle.theta_layout(m)
    ld = oracle.objective(m, th)["logdet_p"]
    ref = sum(spectral_field_logdet(m, th[lay["range"][j]], th[lay["temporal"][j]]) for j in range(m.k))
    ref += m.ns * m.nt * sum(th[i] for i in lay["prec"])  # -2 nt ns log|Lambda|
    ref += m.a * np.log(m.tip_prec)
    assert np.isclose(ld, ref, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("name", ["uni_6x5_nt5", "coreg3_4x4_nt4"])
def test_jacobian_complex_step(name):
    m = named_config(name, seed=2)
    J = oracle.prior_precision_jacobian(m, m.theta)
    h = 1e-30
    for k in range(m.d):
        th = m.theta.astype(complex)
        th[k] += 1j * h
        cs = oracle.prior_precision(m, th).imag / h
        scale = max(np.abs(cs).max(), 1.0)
        assert np.abs(J[k] - cs).max() <= 1e-13 * scale, k


@pytest.mark.parametrize("name,seed", [("uni_6x5_nt5", 0), ("coreg3_4x4_nt4", 1), ("uni_9x7_nt4", 3)])
def test_gradient_complex_step(name, seed):
    m = named_config(name, seed=seed)
    g = oracle.gradient(m, m.theta)["grad"]
    h = 1e-30
    cs = np.zeros(m.d)
    for k in range(m.d):
        th = m.theta.astype(complex)
        th[k] += 1j * h
        cs[k] = oracle.objective(m, th, factor="lu")["f"].imag / h
    assert np.abs(g - cs).max() <= 1e-11 * np.abs(cs).max()


def test_gradient_central_differences():
    m = named_config("uni_6x5_nt5", seed=7)
    g = oracle.gradient(m, m.theta)["grad"]
    fd, f0 = oracle.fd_gradient(m, m.theta, h=1e-4)
    assert np.isclose(f0, oracle.objective(m, m.theta)["f"])
    assert np.abs(g - fd).max() <= 1e-6 * np.abs(g).max()


@pytest.mark.parametrize("k", [1, 3])
def test_no_observations_reduces_to_prior(k):
    m = make_model(k, 4, 3, 3, 2, 0, seed=11)
    assert m.n_obs == 0
    out = oracle.gradient(m, m.theta)
    s2 = m.sigma_prior ** 2
    logp = np.sum(-m.theta ** 2 / (2 * s2)) - 0.5 * m.d * np.log(2 * np.pi * s2)
    assert np.isclose(out["f"], logp, rtol=1e-12, atol=1e-12)
    assert np.allclose(out["grad"], -m.theta / s2, rtol=1e-10, atol=1e-10)


def test_theta1_scale_identity():
    m = named_config("uni_8x8_nt8", seed=0)
    out = oracle.gradient(m, m.theta)
    # dQ_x/dtheta1 = Q_x, so 1/2 tr(Qp^-1 dQp/dtheta1) = ns*nt/2 exactly
    assert np.isclose(out["phaseC"][0], 0.5 * m.ns * m.nt, rtol=1e-12)


def test_theta1_plus_tau_identity():
    m = named_config("uni_6x5_nt5", seed=3)
    out = oracle.gradient(m, m.theta)
    nb = m.nt * m.b
    ZT = out["Zc"][nb:, nb:]
    lhs = -2.0 * (out["phaseA"][0] + out["phaseA"][3])
    assert np.isclose(lhs, m.N - m.tip_prec * np.trace(ZT), rtol=1e-12)


def test_coreg_lambda_scaling_identities():
    # Scaling every entry of Lambda by c (prec -> prec - 2 log c, lambda_ij -> c lambda_ij)
    # scales the latent prior by c^-2, so the direction (prec: 1, lambda_ij: -lambda_ij/2)
    # of dQp is Qp's latent part; with the tau derivatives it gives Qc - blkdiag(0, tip I).
    # |Qp| depends on the diagonal of Lambda only, so Phase C has no coupling terms.
    m = named_config("coreg3_9x7_nt4", seed=2)
    out = oracle.gradient(m, m.theta)
    lay = oracle.theta_layout(m)
    nb = m.nt * m.b
    ZT = out["Zc"][nb:, nb:]
    A, C = out["phaseA"], out["phaseC"]
    comb = (sum(A[i] for i in lay["prec"]) + sum(A[i] for i in lay["tau"])
            - 0.5 * sum(m.theta[i] * A[i] for i in lay["lambda"]))
    assert np.isclose(-2.0 * comb, m.N - m.tip_prec * np.trace(ZT), rtol=1e-12)
    assert np.isclose(sum(C[i] for i in lay["prec"]), 0.5 * m.nt * m.b, rtol=1e-12)
    for i in lay["lambda"]:
        assert abs(C[i]) <= 1e-12 * m.nt * m.b


def test_mode_stationarity():
    m = named_config("coreg3_4x4_nt4", seed=5)
    ev = oracle.objective(m, m.theta)
    A, x = ev["A"], ev["x"]
    grad_x = ev["Qp"] @ x - A.T @ (ev["tau_obs"] * (m.y - A @ x))
    assert np.abs(grad_x).max() <= 1e-10 * np.abs(ev["r"]).max()


def test_scalar_model_closed_form():
    # one node, one time step, one covariate, one observation: everything is 2x2
    m = make_model(1, 1, 1, 1, 1, 1, seed=9)
    t1, t2, t3, t4 = m.theta
    k2 = np.exp(2 * t2)
    g1 = 0.1
    K1, K2 = k2 + g1, k2 * k2 + 2 * k2 * g1 + g1 * g1
    q = np.exp(t1) * (1.0 * K2 + np.exp(t3) * 0.0 * K1 + 2.0)  # M0=1, M1=L1(1)=0, M2=2
    w, xr, y = m.obs_w[0].sum(), m.X[0, 0], m.y[0]
    tau = np.exp(t4)
    Qp = np.array([[q, 0.0], [0.0, m.tip_prec]])
    av = np.array([w, xr])
    Qc = Qp + tau * np.outer(av, av)
    det_p = q * m.tip_prec
    det_c = Qc[0, 0] * Qc[1, 1] - Qc[0, 1] ** 2
    inv_c = np.array([[Qc[1, 1], -Qc[0, 1]], [-Qc[1, 0], Qc[0, 0]]]) / det_c
    x = inv_c @ (tau * y * av)
    res = y - av @ x
    s2 = 0.25
    f = (0.5 * np.log(det_p) - 0.5 * np.log(det_c) - 0.5 * x @ Qp @ x
         + 0.5 * t4 - 0.5 * tau * res ** 2 - 0.5 * np.log(2 * np.pi)
         + np.sum(-m.theta ** 2 / (2 * s2)) - 2 * np.log(2 * np.pi * s2))
    assert np.isclose(oracle.objective(m, m.theta)["f"], f, rtol=1e-13)


def test_coreg_matches_eq9_weights():
    m = named_config("coreg3_4x4_nt4", seed=8)
    th = m.theta
    lay = oracle.theta_layout(m)
    Qp = oracle.prior_precision(m, th)
    k, ns, nt, b = m.k, m.ns, m.nt, m.b
    Lam = np.zeros((k, k))
    for j in range(k):
        Lam[j, j] = np.exp(-0.5 * th[lay["prec"][j]])
    Lam[1, 0], Lam[2, 0], Lam[2, 1] = th[lay["lambda"]]
    Li = np.linalg.inv(Lam)
    c0, g1, g2 = m.c0.toarray(), m.g1.toarray(), m.g2.toarray()
    M0 = oracle.temporal_dense(m.m0)
    M1 = oracle.temporal_dense(m.m1)
    M2 = oracle.temporal_dense(m.m2)
    ref = np.zeros((nt * b, nt * b))
    for mm in range(k):
        kk2 = np.exp(2 * th[lay["range"][mm]])
        K1 = kk2 * c0 + g1
        K2 = kk2 ** 2 * c0 + 2 * kk2 * g1 + g2
        e3 = np.exp(th[lay["temporal"][mm]])
        for t in range(nt):
            for s in range(nt):
                blk = M0[t, s] * K2 + e3 * M1[t, s] * K1 + M2[t, s] * c0
                for i in range(k):
                    for j in range(k):
                        W = Li[mm, i] * Li[mm, j]  # Eq. 9 coregional weight
                        ref[t * b + i * ns:t * b + (i + 1) * ns, s * b + j * ns:s * b + (j + 1) * ns] += W * blk
    assert np.allclose(Qp[:nt * b, :nt * b], ref, rtol=1e-13, atol=1e-12)


def test_coreg_k1_equals_univariate():
    mu = make_model(1, 4, 3, 3, 2, 3, seed=12)
    mc = make_model(1, 4, 3, 3, 2, 3, seed=12, kind="coreg")
    # univariate [scale, range, temporal, tau]  <->  coreg(1) [range, temporal, prec, tau]
    th_u = mu.theta
    th_c = np.array([th_u[1], th_u[2], th_u[0], th_u[3]])
    gu = oracle.gradient(mu, th_u)
    gc = oracle.gradient(mc, th_c)
    assert np.isclose(gu["f"], gc["f"], rtol=1e-13)
    assert np.allclose(gu["grad"][[1, 2, 0, 3]], gc["grad"], rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("n,b,a", [(4, 5, 2), (1, 6, 3), (3, 4, 0), (5, 3, 1)])
def test_selected_inverse_identities(n, b, a):
    blk = random_bta(n, b, a, seed=n * 100 + b * 10 + a)
    Q = oracle.bta_dense(blk["D"], blk["B"], blk["C"], blk["T"])
    Z = oracle.selected_inverse(Q, n, b, a)
    D, B, C, T = blk["D"], blk["B"], blk["C"], blk["T"]
    for i in range(n):
        acc = D[i] @ Z["D"][i]
        if i > 0:
            acc += B[i - 1] @ Z["B"][i - 1].T
        if i < n - 1:
            acc += B[i].T @ Z["B"][i]
        if a:
            acc += C[i].T @ Z["C"][i]
        assert np.allclose(acc, np.eye(b), atol=1e-12)
        assert np.allclose(Z["D"][i], Z["D"][i].T, atol=1e-14)
    if a:
        acc = T @ Z["T"] + sum(C[i] @ Z["C"][i].T for i in range(n))
        assert np.allclose(acc, np.eye(a), atol=1e-12)


def test_bta_cholesky_no_fill_and_leibniz():
    blk = random_bta(2, 2, 1, seed=4)
    Q = oracle.bta_dense(blk["D"], blk["B"], blk["C"], blk["T"])
    ch = oracle.dense_cholesky(Q, blk["rhs"])
    assert np.isclose(ch["logdet"], np.log(leibniz_det(Q)), rtol=1e-13)
    assert np.allclose(Q @ ch["x"], blk["rhs"], atol=1e-12)
    big = random_bta(4, 3, 2, seed=5)
    Qb = oracle.bta_dense(big["D"], big["B"], big["C"], big["T"])
    L = oracle.dense_cholesky(Qb)["L"]
    for i in range(2):  # no fill two blocks below the diagonal
        assert np.all(np.abs(L[(i + 2) * 3:(i + 3) * 3, i * 3:(i + 1) * 3]) < 1e-15)


def test_neumann_second_difference():
    d, o = neumann_second_difference(4)
    assert np.array_equal(d, [1, 2, 2, 1]) and np.array_equal(o, [-1, -1, -1])


# ---- posterior Hessian (Sec. III-D, Eq. 12) and its FD baseline ----------------------------

def test_hessian_from_gradients_column_orientation_and_scale():
    # a linear gradient field g(t) = J t + c (J not symmetric): Eq. 12 returns J exactly, column
    # j being the difference along e_j; a transposed or mis-scaled difference fails
    rng = np.random.default_rng(4)
    d = 5
    J = rng.standard_normal((d, d))
    c = rng.standard_normal(d)
    t0 = rng.standard_normal(d)
    H, g0 = oracle.hessian_from_gradients(lambda t: J @ t + c, t0, 5e-3)
    assert np.allclose(g0, J @ t0 + c, rtol=0, atol=1e-14)
    assert np.abs(H - J).max() <= 1e-12


def test_difference_hessians_on_a_quartic_closed_form():
    # f = sum t_i^4 / 12 + t_0^2 t_1^2 / 4.  Central differences of the exact gradient give
    # t_i^2 + h^2/3 (+ the coupling terms), second differences of f give t_i^2 + h^2/6; the
    # mixed second difference of t_0^2 t_1^2 / 4 is t_0 t_1 exactly.
    h = 5e-3
    t0 = np.array([0.7, -0.4, 0.3])

    def f(t):
        return np.sum(t ** 4) / 12 + t[0] ** 2 * t[1] ** 2 / 4

    def g(t):
        out = t ** 3 / 3
        out[0] += t[0] * t[1] ** 2 / 2
        out[1] += t[0] ** 2 * t[1] / 2
        return out

    exact = np.diag(t0 ** 2)
    exact[0, 0] += t0[1] ** 2 / 2
    exact[1, 1] += t0[0] ** 2 / 2
    exact[0, 1] = exact[1, 0] = t0[0] * t0[1]
    Hg, _ = oracle.hessian_from_gradients(g, t0, h)
    Hf, f0 = oracle.second_differences(f, t0, h)
    assert np.isclose(f0, f(t0), rtol=1e-15)
    assert np.abs(Hg - (exact + np.eye(3) * h * h / 3)).max() <= 1e-12
    assert np.abs(Hf - (exact + np.eye(3) * h * h / 6)).max() <= 1e-9


@pytest.mark.parametrize("k", [1, 3])
def test_hessian_without_observations_is_prior_curvature(k):
    # no observations: f = log p(theta), whose Hessian is -I / sigma^2
    m = make_model(k, 4, 3, 3, 2, 0, seed=11)
    s2 = m.sigma_prior ** 2
    H, g, f = oracle.hessian_fd_of_grad(m, m.theta, h=5e-3)
    assert np.abs(H + np.eye(m.d) / s2).max() <= 1e-9
    assert np.allclose(g, -m.theta / s2, rtol=1e-10, atol=1e-10)
    Hf, f0 = oracle.fd_hessian(m, m.theta, h=5e-3)
    assert np.isclose(f0, f, rtol=1e-13)
    assert np.abs(Hf + np.eye(m.d) / s2).max() <= 1e-6


def test_hessian_of_gradients_agrees_with_second_differences():
    # two independent routes to the same Hessian (exact gradients vs f alone) agree to their
    # O(h^2) truncation, and Eq. 12's H is symmetric to the same order
    m = named_config("uni_6x5_nt5", seed=7)
    H, _, _ = oracle.hessian_fd_of_grad(m, m.theta, h=5e-3)
    Hf, _ = oracle.fd_hessian(m, m.theta, h=5e-3)
    scale = np.abs(H).max()
    assert np.abs(H - Hf).max() <= 1e-5 * scale
    assert np.abs(H - H.T).max() <= 1e-5 * scale


@pytest.mark.parametrize("k,nx,ny,nt,a,obs", [(1, 6, 5, 4, 3, 7), (3, 5, 4, 3, 6, 4),
                                              (2, 1, 6, 3, 2, 5), (1, 7, 1, 2, 0, 6)])
def test_observation_matrix_interpolates_linear_fields(k, nx, ny, nt, a, obs):
    """Bilinear interpolation reproduces a linear field exactly: placing alpha*ix + beta*iy +
    gamma on the nodes of time block t and field m, row r of A returns alpha*u + beta*v + gamma
    at the observation's location for the observations of (t, m) and 0 for all others; the
    covariates sit on the fixed-effect columns.  A wrong time or field offset, a swapped weight or
    a transposed node id fails this."""
    spec = make_model(k, nx, ny, nt, a, obs, seed=4)
    A = oracle.observation_matrix(spec)
    uv = spec.extra["obs_uv"]
    assert A.shape == (spec.n_obs, spec.N)
    ns, b, nb = spec.ns, spec.b, spec.nt * spec.b
    ix, iy = np.arange(ns) % nx, np.arange(ns) // nx
    alpha, beta, gamma = 0.37, -1.21, 2.5
    lin = alpha * ix + beta * iy + gamma
    for t in range(nt):
        for m in range(k):
            x = np.zeros(spec.N)
            x[t * b + m * ns:t * b + (m + 1) * ns] = lin
            sel = (spec.obs_t == t) & (spec.obs_field == m)
            expect = np.where(sel, alpha * uv[:, 0] + beta * uv[:, 1] + gamma, 0.0)
            assert np.allclose(A @ x, expect, rtol=0, atol=1e-12)
    for r in range(spec.n_obs):
        lo = spec.obs_t[r] * b + spec.obs_field[r] * ns
        nzc = np.nonzero(A[r, :nb])[0]
        assert nzc.size > 0 and nzc.min() >= lo and nzc.max() < lo + ns
        assert abs(A[r, :nb].sum() - 1.0) <= 1e-14
    assert np.array_equal(A[:, nb:], spec.X)
