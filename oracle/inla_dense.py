"""Dense CPU oracle for the INLA objective f(theta) and its gradient (test infrastructure).

This is the slow, obviously-correct reference the HIP path is checked against.  Every matrix
is assembled densely (N x N), every factorisation is a textbook LAPACK call, and the
gradient uses dense inverses.  Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may import it.

What is computed (paper references are to sections, equations and tables):

* The objective, Sec. II-A, Eq. 1:
      f = 1/2 log|Qp| - 1/2 log|Qc| - 1/2 x*^T Qp x* + log l(y | x*, theta) + log p(theta)
  with ``Qc = Qp + sum_m tau_m A_m^T A_m`` and ``x* = Qc^-1 r``, ``r = sum_m tau_m A_m^T y_m``
  (Sec. II-A).  Readings where the paper is silent (listed in the design notes):
    - Gaussian likelihood: ``log l = sum_m [n_m/2 log tau_m - tau_m/2 |y_m - A_m x*|^2]
      - n_y/2 log(2 pi)``, with ``tau_m = exp(theta_tau_m)``;
    - prior ``theta_k ~ N(0, sigma^2)`` independently, ``sigma = 0.5``, including its
      normalising constant;
    - the ``-N/2 log(2 pi)`` terms of the prior and of the Gaussian approximation cancel and
      are left out; ``log p(y)`` is left out;
    - ``Qp = blkdiag(Q_x, tip_prec * I_a)`` (fixed effects with a vague Gaussian prior).
* The prior precision (Sec. II-A, Kronecker assembly; Sec. III-B, Eq. 9 for k fields):
    - univariate, theta = [log scale, range, temporal, log tau]:
          Q_x = e^t1 [ M0 (x) K2 + e^t3 M1 (x) K1 + M2 (x) c0 ],
          K1 = e^(2 t2) c0 + g1,   K2 = e^(4 t2) c0 + 2 e^(2 t2) g1 + g2;
    - coregional, theta = [range(k), temporal(k), prec(k), lambda(k(k-1)/2), log tau(k)]:
      x_t = (Lambda (x) I) u_t with independent fields u_m ~ N(0, Q_m^-1),
          Q_m = M0 (x) K2(r_m) + e^(t_m) M1 (x) K1(r_m) + M2 (x) c0,
      Lambda lower triangular, Lambda_mm = exp(-p_m/2), strictly-lower entries = lambda
      (row-major).  Q_x is the precision of x, i.e. S Q_u S^T with S = I (x) Lambda^-T (x) I.
* The gradient, Sec. III-A, Eq. 5 (x* held fixed by the envelope argument) with the trace
  identity d log|Q| = tr(Q^-1 dQ):
      g_k = 1/2 tr(Qp^-1 dQp) - 1/2 tr(Qc^-1 dQc) - 1/2 x*^T dQp x* + d log l + d log p.
  ``dQp/dtheta_k`` is assembled analytically.  This formula is pinned in the tests against
  the complex-step derivative of ``objective(..., factor="lu")`` and against central
  differences.
* Central differences, Sec. II-D, Eq. 2, with 2d+1 evaluations.
* The posterior Hessian, Sec. III-D, Eq. 12: column j is the central difference of the exact
  gradient along e_j (2d+1 gradient evaluations), not symmetrised; and the FD baseline it
  replaces, second-order central differences of f over 2d^2+1 points (Sec. II-D).
* The selected inverse (Sec. III-A, Phase A): the dense inverse read at the BTA pattern.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = [
    "dense_bases", "temporal_dense", "theta_layout", "prior_precision",
    "prior_precision_jacobian", "observation_matrix", "obs_tau", "objective", "gradient",
    "fd_gradient", "hessian_from_gradients", "hessian_fd_of_grad", "second_differences",
    "fd_hessian", "bta_dense", "bta_split", "dense_cholesky", "selected_inverse",
]


def temporal_dense(tri, dtype=float):
    """Dense nt x nt matrix from (diagonal, sub-diagonal)."""
    diag, off = tri
    m = np.diag(np.asarray(diag, dtype=dtype))
    if len(off):
        m = m + np.diag(np.asarray(off, dtype=dtype), -1) + np.diag(np.asarray(off, dtype=dtype), 1)
    return m


def dense_bases(model):
    return model.c0.toarray(), model.g1.toarray(), model.g2.toarray()


def theta_layout(model):
    """Index groups of theta.  Univariate: scale, range, temporal, tau.  Coregional:
    range(k), temporal(k), prec(k), lambda(k(k-1)/2), tau(k)."""
    k = model.k
    if model.kind == "univariate":
        return {"scale": [0], "range": [1], "temporal": [2], "tau": [3], "lambda": []}
    nl = k * (k - 1) // 2
    return {
        "range": list(range(0, k)),
        "temporal": list(range(k, 2 * k)),
        "prec": list(range(2 * k, 3 * k)),
        "lambda": list(range(3 * k, 3 * k + nl)),
        "tau": list(range(3 * k + nl, 4 * k + nl)),
    }


def _field_precision(model, rng_par, tmp_par, dtype):
    """Q_m = M0 (x) K2 + e^tmp M1 (x) K1 + M2 (x) c0 and its two partial derivatives."""
    c0, g1, g2 = dense_bases(model)
    M0 = temporal_dense(model.m0, dtype)
    M1 = temporal_dense(model.m1, dtype)
    M2 = temporal_dense(model.m2, dtype)
    k2 = np.exp(2 * rng_par)
    e3 = np.exp(tmp_par)
    K1 = k2 * c0 + g1
    K2 = k2 * k2 * c0 + 2 * k2 * g1 + g2
    Q = np.kron(M0, K2) + e3 * np.kron(M1, K1) + np.kron(M2, c0)
    dK1 = 2 * k2 * c0
    dK2 = 4 * k2 * k2 * c0 + 4 * k2 * g1
    dQ_range = np.kron(M0, dK2) + e3 * np.kron(M1, dK1)
    dQ_temporal = e3 * np.kron(M1, K1)
    return Q, dQ_range, dQ_temporal


def _lambda(model, theta):
    k = model.k
    lay = theta_layout(model)
    L = np.zeros((k, k), dtype=np.asarray(theta).dtype)
    for m in range(k):
        L[m, m] = np.exp(-0.5 * theta[lay["prec"][m]])
    idx = 0
    for i in range(1, k):
        for j in range(i):
            L[i, j] = theta[lay["lambda"][idx]]
            idx += 1
    return L


def _field_index(model, m):
    """Positions of field m's latent entries (time-major, then node) in the global order."""
    ns, b = model.ns, model.b
    t = np.arange(model.nt)[:, None]
    p = np.arange(ns)[None, :]
    return (t * b + m * ns + p).reshape(-1)


def prior_precision(model, theta):
    """Dense N x N prior precision Qp(theta); complex theta is allowed (complex step)."""
    theta = np.asarray(theta)
    dtype = np.result_type(theta.dtype, float)
    N, a = model.N, model.a
    Qp = np.zeros((N, N), dtype=dtype)
    nb = model.nt * model.b
    if model.kind == "univariate":
        Q, _, _ = _field_precision(model, theta[1], theta[2], dtype)
        Qp[:nb, :nb] = np.exp(theta[0]) * Q
    else:
        lay = theta_layout(model)
        Qu = np.zeros((nb, nb), dtype=dtype)
        for m in range(model.k):
            Q, _, _ = _field_precision(model, theta[lay["range"][m]], theta[lay["temporal"][m]], dtype)
            idx = _field_index(model, m)
            Qu[np.ix_(idx, idx)] += Q
        Linv = np.linalg.inv(_lambda(model, theta))
        S = np.kron(np.eye(model.nt), np.kron(Linv.T, np.eye(model.ns)))
        Qp[:nb, :nb] = S @ Qu @ S.T
    Qp[nb:, nb:] = model.tip_prec * np.eye(a)
    return Qp


def prior_precision_jacobian(model, theta):
    """Analytic dQp/dtheta_k, k = 0..d-1, as a (d, N, N) array."""
    theta = np.asarray(theta, dtype=float)
    d, N = model.d, model.N
    nb = model.nt * model.b
    J = np.zeros((d, N, N))
    if model.kind == "univariate":
        Q, dQr, dQt = _field_precision(model, theta[1], theta[2], float)
        e1 = np.exp(theta[0])
        J[0, :nb, :nb] = e1 * Q
        J[1, :nb, :nb] = e1 * dQr
        J[2, :nb, :nb] = e1 * dQt
        return J
    lay = theta_layout(model)
    k = model.k
    Qu = np.zeros((nb, nb))
    dQu = {}
    for m in range(k):
        Q, dQr, dQt = _field_precision(model, theta[lay["range"][m]], theta[lay["temporal"][m]], float)
        idx = _field_index(model, m)
        Qu[np.ix_(idx, idx)] += Q
        for key, val in ((lay["range"][m], dQr), (lay["temporal"][m], dQt)):
            tmp = np.zeros((nb, nb))
            tmp[np.ix_(idx, idx)] = val
            dQu[key] = tmp
    Lam = _lambda(model, theta)
    Linv = np.linalg.inv(Lam)
    I_t, I_s = np.eye(model.nt), np.eye(model.ns)
    S = np.kron(I_t, np.kron(Linv.T, I_s))
    for key, val in dQu.items():
        J[key, :nb, :nb] = S @ val @ S.T
    # coupling parameters act through Lambda: d(Lambda^-1) = -Lambda^-1 dLambda Lambda^-1
    for m in range(k):
        dLam = np.zeros((k, k))
        dLam[m, m] = -0.5 * np.exp(-0.5 * theta[lay["prec"][m]])
        dLinv = -Linv @ dLam @ Linv
        dS = np.kron(I_t, np.kron(dLinv.T, I_s))
        J[lay["prec"][m], :nb, :nb] = dS @ Qu @ S.T + S @ Qu @ dS.T
    idx = 0
    for i in range(1, k):
        for j in range(i):
            dLam = np.zeros((k, k))
            dLam[i, j] = 1.0
            dLinv = -Linv @ dLam @ Linv
            dS = np.kron(I_t, np.kron(dLinv.T, I_s))
            J[lay["lambda"][idx], :nb, :nb] = dS @ Qu @ S.T + S @ Qu @ dS.T
            idx += 1
    return J


def observation_matrix(model):
    """Dense A (n_obs x N): bilinear weights on the observation's time block and field,
    covariates on the fixed-effect columns."""
    n_obs, N = model.n_obs, model.N
    A = np.zeros((n_obs, N))
    nb = model.nt * model.b
    for r in range(n_obs):
        base = model.obs_t[r] * model.b + model.obs_field[r] * model.ns
        for e in range(4):
            A[r, base + model.obs_node[r, e]] += model.obs_w[r, e]
        A[r, nb:] = model.X[r]
    return A


def obs_tau(model, theta):
    """Observation precision tau_m = exp(theta_tau_m) for every observation (and per field)."""
    lay = theta_layout(model)
    tau_field = np.exp(np.asarray([theta[i] for i in lay["tau"]]))
    return tau_field[model.obs_field], tau_field


def _logdet(Q, factor):
    if factor == "cholesky":
        L = np.linalg.cholesky(Q)
        return 2.0 * np.sum(np.log(np.diag(L)))
    sign, logabs = np.linalg.slogdet(Q)
    return logabs + np.log(sign)


def objective(model, theta, factor="cholesky"):
    """f(theta) by Eq. 1 from dense matrices.  ``factor="lu"`` uses LU determinants and
    solves so that complex theta gives a complex-step derivative."""
    theta = np.asarray(theta)
    Qp = prior_precision(model, theta)
    A = observation_matrix(model)
    tau_r, tau_f = obs_tau(model, theta)
    Qc = Qp + A.T @ (tau_r[:, None] * A)
    r = A.T @ (tau_r * model.y)
    ld_p = _logdet(Qp, factor)
    ld_c = _logdet(Qc, factor)
    if factor == "cholesky":
        x = sla.cho_solve(sla.cho_factor(Qc, lower=True), r)
    else:
        x = np.linalg.solve(Qc, r)
    quad = x @ Qp @ x
    res = model.y - A @ x
    lay = theta_layout(model)
    loglik = -0.5 * model.n_obs * np.log(2 * np.pi)
    for m in range(len(lay["tau"])):
        sel = model.obs_field == m
        loglik = loglik + 0.5 * np.count_nonzero(sel) * theta[lay["tau"][m]] \
            - 0.5 * tau_f[m] * np.sum(res[sel] ** 2)
    s2 = model.sigma_prior ** 2
    logprior = np.sum(-theta ** 2 / (2 * s2)) - 0.5 * model.d * np.log(2 * np.pi * s2)
    f = 0.5 * ld_p - 0.5 * ld_c - 0.5 * quad + loglik + logprior
    return {"f": f, "logdet_p": ld_p, "logdet_c": ld_c, "x": x, "quad": quad,
            "loglik": loglik, "logprior": logprior, "Qp": Qp, "Qc": Qc, "A": A,
            "tau_obs": tau_r, "tau_field": tau_f, "r": r}


def gradient(model, theta):
    """Exact gradient of f (Eq. 5) with dense inverses; returns the phases separately."""
    theta = np.asarray(theta, dtype=float)
    ev = objective(model, theta)
    Qp, Qc, A, x = ev["Qp"], ev["Qc"], ev["A"], ev["x"]
    N = model.N
    I = np.eye(N)
    Zp = sla.cho_solve(sla.cho_factor(Qp, lower=True), I)
    Zc = sla.cho_solve(sla.cho_factor(Qc, lower=True), I)
    J = prior_precision_jacobian(model, theta)
    lay = theta_layout(model)
    tau_f = ev["tau_field"]
    res = model.y - A @ x
    d = model.d
    phaseA = np.zeros(d)
    phaseB = np.zeros(d)
    phaseC = np.zeros(d)
    dlik = np.zeros(d)
    for k in range(d):
        dQc = J[k].copy()
        if k in lay["tau"]:
            m = lay["tau"].index(k)
            sel = model.obs_field == m
            Am = A[sel]
            dQc += tau_f[m] * Am.T @ Am
            dlik[k] = 0.5 * np.count_nonzero(sel) - 0.5 * tau_f[m] * np.sum(res[sel] ** 2)
        phaseA[k] = -0.5 * np.sum(Zc * dQc)
        phaseB[k] = -0.5 * x @ J[k] @ x
        phaseC[k] = 0.5 * np.sum(Zp * J[k])
    dprior = -theta / model.sigma_prior ** 2
    g = phaseA + phaseB + phaseC + dlik + dprior
    return {"grad": g, "f": ev["f"], "phaseA": phaseA, "phaseB": phaseB, "phaseC": phaseC,
            "dloglik": dlik, "dlogprior": dprior, "Zc": Zc, "Zp": Zp, "x": x}


def fd_gradient(model, theta, h=1e-3):
    """Central differences (Eq. 2): 2d+1 objective evaluations (the centre gives f)."""
    theta = np.asarray(theta, dtype=float)
    f0 = objective(model, theta)["f"]
    g = np.zeros(model.d)
    for j in range(model.d):
        e = np.zeros(model.d)
        e[j] = h
        g[j] = (objective(model, theta + e)["f"] - objective(model, theta - e)["f"]) / (2 * h)
    return g, f0


def hessian_from_gradients(grad_fun, theta, h):
    """Eq. 12 for any gradient routine: H[:, j] = (g(theta + h e_j) - g(theta - h e_j)) / (2h).
    Returns (H, g(theta)); H is returned as the equation defines it (not symmetrised)."""
    theta = np.asarray(theta, dtype=float)
    d = theta.size
    g0 = np.asarray(grad_fun(theta), dtype=float)
    H = np.zeros((d, d))
    for j in range(d):
        e = np.zeros(d)
        e[j] = h
        H[:, j] = (np.asarray(grad_fun(theta + e)) - np.asarray(grad_fun(theta - e))) / (2 * h)
    return H, g0


def hessian_fd_of_grad(model, theta, h=5e-3):
    """Sec. III-D, Eq. 12 with the exact gradient (Eq. 5): 2d+1 gradient evaluations, the centre
    one giving f and the gradient at theta.  Returns (H, g, f)."""
    theta = np.asarray(theta, dtype=float)
    H, g0 = hessian_from_gradients(lambda t: gradient(model, t)["grad"], theta, h)
    return H, g0, objective(model, theta)["f"]


def second_differences(fun, theta, h):
    """Second-order central differences of a scalar function over 2d^2+1 points:
    H_jj = (f(+e_j) - 2 f(0) + f(-e_j)) / h^2 and, for j != k,
    H_jk = (f(+e_j+e_k) - f(+e_j-e_k) - f(-e_j+e_k) + f(-e_j-e_k)) / (4 h^2), steps of size h.
    Returns (H, f(theta))."""
    theta = np.asarray(theta, dtype=float)
    d = theta.size
    E = np.eye(d) * h
    f0 = float(fun(theta))
    H = np.zeros((d, d))
    for j in range(d):
        H[j, j] = (fun(theta + E[j]) - 2.0 * f0 + fun(theta - E[j])) / h ** 2
        for k in range(j + 1, d):
            v = (fun(theta + E[j] + E[k]) - fun(theta + E[j] - E[k])
                 - fun(theta - E[j] + E[k]) + fun(theta - E[j] - E[k])) / (4.0 * h ** 2)
            H[j, k] = H[k, j] = v
    return H, f0


def fd_hessian(model, theta, h=5e-3):
    """The FD Hessian that Eq. 12 replaces (Sec. II-D): 2d^2+1 objective evaluations."""
    return second_differences(lambda t: objective(model, t)["f"], theta, h)


# ---- BTA helpers (Sec. II-B layout) -------------------------------------------------------

def bta_dense(D, B, C, T):
    """Dense symmetric N x N matrix from BTA blocks: D (n,b,b), B (n-1,b,b) sub-diagonal
    blocks [Q]_{i+1,i}, C (n,a,b) arrow blocks [Q]_{T,i}, T (a,a)."""
    n, b = D.shape[0], D.shape[1]
    a = T.shape[0]
    N = n * b + a
    Q = np.zeros((N, N))
    for i in range(n):
        Q[i * b:(i + 1) * b, i * b:(i + 1) * b] = D[i]
        if i < n - 1:
            Q[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = B[i]
            Q[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = B[i].T
        if a:
            Q[n * b:, i * b:(i + 1) * b] = C[i]
            Q[i * b:(i + 1) * b, n * b:] = C[i].T
    if a:
        Q[n * b:, n * b:] = T
    return Q


def bta_split(M, n, b, a):
    """Read a dense N x N matrix at the BTA pattern (lower blocks)."""
    D = np.stack([M[i * b:(i + 1) * b, i * b:(i + 1) * b] for i in range(n)])
    B = np.stack([M[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] for i in range(n - 1)]) \
        if n > 1 else np.zeros((0, b, b))
    C = np.stack([M[n * b:, i * b:(i + 1) * b] for i in range(n)])
    T = M[n * b:, n * b:]
    return {"D": D, "B": B, "C": C, "T": T}


def dense_cholesky(Q, rhs=None):
    """Dense lower Cholesky factor, log-determinant, and (optionally) z = L^-1 rhs and
    x = Q^-1 rhs."""
    L = np.linalg.cholesky(Q)
    out = {"L": L, "logdet": 2.0 * np.sum(np.log(np.diag(L)))}
    if rhs is not None:
        z = sla.solve_triangular(L, rhs, lower=True)
        out["z"] = z
        out["x"] = sla.solve_triangular(L.T, z, lower=False)
    return out


def selected_inverse(Q, n, b, a):
    """Blocks of the dense inverse at the BTA pattern (Sec. III-A, Phase A)."""
    Z = sla.cho_solve(sla.cho_factor(Q, lower=True), np.eye(Q.shape[0]))
    return bta_split(Z, n, b, a)
