"""Synthetic SPDE-type spatio-temporal models with a block-tridiagonal-arrowhead precision.

The models follow the paper's problem statement (Sec. II-A, Eq. 1; Sec. II-B for the BTA
layout; Sec. III-B, Eq. 9 for the coregional case).  The paper does not give its synthetic
generator, so the recipe here is our own and is stated in full:

* Space: an ``nx`` x ``ny`` grid, node id ``iy*nx + ix``.  ``L1(m)`` is the 1-D Neumann second
  difference (diagonal ``[1, 2, ..., 2, 1]``, off-diagonals ``-1``); the grid Laplacian is
  ``I_ny (x) L1(nx) + L1(ny) (x) I_nx``.  Base matrices: ``c0 = I``, ``g1 = Laplacian + 0.1 I``,
  ``g2 = g1 @ g1``.
* Time: ``M0 = I``, ``M1 = L1(nt)`` (random-walk structure), ``M2 = tridiag(-1, 2, -1)``.  All
  three are tridiagonal, so the precision stays block tridiagonal.
* Observations: ``obs_per_step`` per time step (per field for ``k > 1``) at uniform random
  locations in ``[0, nx-1] x [0, ny-1]`` with bilinear weights on the 4 surrounding nodes,
  and ``a`` N(0,1) covariates (for ``k > 1`` field ``m`` uses covariate columns ``2m, 2m+1``
  modulo ``a``).
* Data: ``y = A [x; beta] + eps`` with the latent field drawn exactly from the prior at
  ``theta_true = 0`` (see ``_sample_field``), ``beta ~ N(0, I)``, ``eps ~ N(0, 1)``.
* Evaluation point: ``theta ~ N(0, 0.5^2 I_d)``.

Draw order from ``numpy.random.default_rng(seed)``: for each time step (and field) the
locations then the covariates; then the latent noise vector; then ``beta``; then ``eps``;
then ``theta``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Tuple

import numpy as np
import scipy.sparse as sp


def neumann_second_difference(m: int) -> Tuple[np.ndarray, np.ndarray]:
    """1-D Neumann second difference as (diagonal, sub-diagonal)."""
    if m == 1:
        return np.zeros(1), np.zeros(0)
    diag = np.full(m, 2.0)
    diag[0] = diag[-1] = 1.0
    return diag, np.full(m - 1, -1.0)


def _tridiag_csr(diag: np.ndarray, off: np.ndarray) -> sp.csr_matrix:
    m = diag.shape[0]
    return sp.diags([off, diag, off], [-1, 0, 1], shape=(m, m), format="csr")


def _base_matrices(nx: int, ny: int):
    lx = _tridiag_csr(*neumann_second_difference(nx))
    ly = _tridiag_csr(*neumann_second_difference(ny))
    lap = sp.kron(sp.identity(ny), lx) + sp.kron(ly, sp.identity(nx))
    ns = nx * ny
    c0 = sp.identity(ns, format="csr")
    g1 = (lap + 0.1 * sp.identity(ns)).tocsr()
    g2 = (g1 @ g1).tocsr()
    for m in (c0, g1, g2):
        m.sum_duplicates()
        m.sort_indices()
    return c0.tocsr(), g1, g2


def _neumann_eigen(m: int):
    """Orthonormal eigenvectors (columns) and eigenvalues of the Neumann second difference."""
    j = np.arange(m)
    i = np.arange(m)
    v = np.cos(np.pi * np.outer(i + 0.5, j) / m)
    v[:, 0] *= 1.0 / np.sqrt(m)
    if m > 1:
        v[:, 1:] *= np.sqrt(2.0 / m)
    lam = 2.0 - 2.0 * np.cos(np.pi * j / m)
    return v, lam


def _sample_field(nx, ny, nt, xi):
    """Exact draw from N(0, Q^-1) for the unit-scale prior at theta = 0.

    At theta = 0 the prior is ``I (x) (I+g1)^2 + M1 (x) (I+g1) + M2 (x) I``.  In the cosine
    eigenbasis of the grid Laplacian each spatial mode ``mu`` decouples into an ``nt x nt``
    tridiagonal precision; we factor it, solve with the noise and map back to nodes.  Used only
    to make the synthetic data; the objective never takes this route.
    """
    ux, lx = _neumann_eigen(nx)
    uy, ly = _neumann_eigen(ny)
    mu = (ly[:, None] + lx[None, :]).reshape(-1) + 0.1  # mode id = l*nx + j
    ns = nx * ny
    k1 = 1.0 + mu
    m1d, m1o = neumann_second_difference(nt)
    m2d = np.full(nt, 2.0)
    m2o = np.full(max(nt - 1, 0), -1.0)
    # per-mode tridiagonal: diag d[t], sub-diagonal e[t]
    d = (k1 ** 2)[:, None] + k1[:, None] * m1d[None, :] + m2d[None, :]
    e = k1[:, None] * m1o[None, :] + m2o[None, :]
    ldiag = np.empty((ns, nt))
    lsub = np.empty((ns, max(nt - 1, 0)))
    ldiag[:, 0] = np.sqrt(d[:, 0])
    for t in range(1, nt):
        lsub[:, t - 1] = e[:, t - 1] / ldiag[:, t - 1]
        ldiag[:, t] = np.sqrt(d[:, t] - lsub[:, t - 1] ** 2)
    xi = xi.reshape(ns, nt)
    v = np.empty_like(xi)
    v[:, nt - 1] = xi[:, nt - 1] / ldiag[:, nt - 1]
    for t in range(nt - 2, -1, -1):
        v[:, t] = (xi[:, t] - lsub[:, t] * v[:, t + 1]) / ldiag[:, t]
    out = np.empty((nt, ns))
    for t in range(nt):
        vt = v[:, t].reshape(ny, nx)
        out[t] = (uy @ vt @ ux.T).reshape(-1)
    return out


@dataclass
class SpdeModel:
    """All inputs of one synthetic model.  Latent order: time-major, then field, then node;
    the ``a`` fixed effects come last (the arrowhead tip)."""

    kind: str            # "univariate" (d = 4) or "coreg" (d = 4k + k(k-1)/2)
    k: int
    nx: int
    ny: int
    nt: int
    a: int
    c0: sp.csr_matrix
    g1: sp.csr_matrix
    g2: sp.csr_matrix
    m0: Tuple[np.ndarray, np.ndarray]
    m1: Tuple[np.ndarray, np.ndarray]
    m2: Tuple[np.ndarray, np.ndarray]
    obs_t: np.ndarray      # (ny_obs,) int32, time step of each observation
    obs_field: np.ndarray  # (ny_obs,) int32, field of each observation
    obs_node: np.ndarray   # (ny_obs, 4) int32, local node ids (within the field)
    obs_w: np.ndarray      # (ny_obs, 4) float64, bilinear weights
    X: np.ndarray          # (ny_obs, a) covariates
    y: np.ndarray          # (ny_obs,)
    theta: np.ndarray      # (d,) evaluation point
    sigma_prior: float = 0.5
    tip_prec: float = 1e-3
    extra: Dict[str, object] = field(default_factory=dict)

    @property
    def ns(self) -> int:
        return self.nx * self.ny

    @property
    def b(self) -> int:
        return self.k * self.ns

    @property
    def N(self) -> int:
        return self.nt * self.b + self.a

    @property
    def d(self) -> int:
        if self.kind == "univariate":
            return 4
        return 4 * self.k + self.k * (self.k - 1) // 2

    @property
    def n_obs(self) -> int:
        return int(self.y.shape[0])


def _draw_location(rng, nx, ny, m):
    u = rng.uniform(0.0, nx - 1.0, size=m) if nx > 1 else np.zeros(m)
    v = rng.uniform(0.0, ny - 1.0, size=m) if ny > 1 else np.zeros(m)
    return u, v


def _bilinear(nx, ny, u, v):
    m = u.shape[0]
    nodes = np.zeros((m, 4), dtype=np.int32)
    w = np.zeros((m, 4))
    for r in range(m):
        if nx > 1:
            ix = min(int(np.floor(u[r])), nx - 2)
            fx = u[r] - ix
        else:
            ix, fx = 0, 0.0
        if ny > 1:
            iy = min(int(np.floor(v[r])), ny - 2)
            fy = v[r] - iy
        else:
            iy, fy = 0, 0.0
        ix1 = ix + 1 if nx > 1 else ix
        iy1 = iy + 1 if ny > 1 else iy
        cand = [
            (iy * nx + ix, (1 - fx) * (1 - fy)),
            (iy * nx + ix1, fx * (1 - fy)),
            (iy1 * nx + ix, (1 - fx) * fy),
            (iy1 * nx + ix1, fx * fy),
        ]
        for e, (node, wt) in enumerate(cand):
            nodes[r, e] = node
            w[r, e] = wt
        # degenerate grids (nx or ny == 1) repeat a node; keep one copy of its weight
        if nx == 1:
            w[r, 1] = w[r, 3] = 0.0
            w[r, 0] = (1 - fy)
            w[r, 2] = fy
        if ny == 1:
            w[r, 2] = w[r, 3] = 0.0
            w[r, 0] = (1 - fx) if nx > 1 else 1.0
            w[r, 1] = fx if nx > 1 else 0.0
    return nodes, w


def make_model(k: int, nx: int, ny: int, nt: int, a: int, obs_per_step: int, seed: int,
               kind: str = None, with_obs: bool = True) -> SpdeModel:
    """Draw one model.  ``kind`` defaults to "univariate" for ``k == 1`` else "coreg"."""
    if kind is None:
        kind = "univariate" if k == 1 else "coreg"
    if kind == "univariate" and k != 1:
        raise ValueError("univariate model needs k == 1")
    rng = np.random.default_rng(seed)
    c0, g1, g2 = _base_matrices(nx, ny)
    m0 = (np.ones(nt), np.zeros(max(nt - 1, 0)))
    m1 = neumann_second_difference(nt)
    m2 = (np.full(nt, 2.0), np.full(max(nt - 1, 0), -1.0))
    ns = nx * ny
    obs_t, obs_f, obs_node, obs_w, xs, locs = [], [], [], [], [], []
    if with_obs and obs_per_step > 0:
        for t in range(nt):
            for m in range(k):
                u, v = _draw_location(rng, nx, ny, obs_per_step)
                if k == 1:
                    cov = rng.standard_normal((obs_per_step, a))
                else:
                    cov = np.zeros((obs_per_step, a))
                    vals = rng.standard_normal((obs_per_step, 2))
                    if a > 0:
                        cov[:, (2 * m) % a] += vals[:, 0]
                        cov[:, (2 * m + 1) % a] += vals[:, 1]
                nodes, w = _bilinear(nx, ny, u, v)
                locs.append(np.stack([u, v], axis=1))
                obs_t.append(np.full(obs_per_step, t, dtype=np.int32))
                obs_f.append(np.full(obs_per_step, m, dtype=np.int32))
                obs_node.append(nodes)
                obs_w.append(w)
                xs.append(cov)
    if obs_t:
        obs_t = np.concatenate(obs_t)
        obs_f = np.concatenate(obs_f)
        obs_node = np.concatenate(obs_node)
        obs_w = np.concatenate(obs_w)
        X = np.concatenate(xs)
        obs_uv = np.concatenate(locs)
    else:
        obs_t = np.zeros(0, np.int32)
        obs_f = np.zeros(0, np.int32)
        obs_node = np.zeros((0, 4), np.int32)
        obs_w = np.zeros((0, 4))
        X = np.zeros((0, a))
        obs_uv = np.zeros((0, 2))
    xi = rng.standard_normal(k * ns * nt)
    fields = [_sample_field(nx, ny, nt, xi[m * ns * nt:(m + 1) * ns * nt]) for m in range(k)]
    # latent x ordered (t, field, node); at theta_true = 0 the coregional mixing is identity
    x_lat = np.stack(fields, axis=1).reshape(-1)
    beta = rng.standard_normal(a)
    n_obs = obs_t.shape[0]
    eps = rng.standard_normal(n_obs)
    b = k * ns
    y = np.zeros(n_obs)
    for r in range(n_obs):
        base = obs_t[r] * b + obs_f[r] * ns
        y[r] = np.dot(obs_w[r], x_lat[base + obs_node[r]]) + np.dot(X[r], beta)
    y += eps
    d = 4 if kind == "univariate" else 4 * k + k * (k - 1) // 2
    theta = 0.5 * rng.standard_normal(d)
    return SpdeModel(kind=kind, k=k, nx=nx, ny=ny, nt=nt, a=a, c0=c0, g1=g1, g2=g2,
                     m0=m0, m1=m1, m2=m2, obs_t=obs_t, obs_field=obs_f,
                     obs_node=obs_node.astype(np.int32), obs_w=obs_w, X=X, y=y, theta=theta,
                     extra={"seed": seed, "obs_per_step": obs_per_step,
                            # grid coordinates (u, v) of each observation's location
                            "obs_uv": obs_uv})


# name -> (k, nx, ny, nt, a, obs_per_step)
NAMED_CONFIGS = {
    # plain univariate model, 8x8 grid, 8 steps, 2 fixed effects, 4 obs per step
    "uni_8x8_nt8": (1, 8, 8, 8, 2, 4),
    # univariate 32x32 grid (b = 1024), 50 steps, 6 covariates, 200 obs per step
    "uni_32x32_nt50": (1, 32, 32, 50, 6, 200),
    # three coregionalised fields on 30x30 (b = 2700), 48 steps, d = 15
    "coreg3_30x30_nt48": (3, 30, 30, 48, 6, 300),
    # three fields on 20x20 (b = 1200), 32 steps, 4 fixed effects (31-point stencil batch)
    "coreg3_20x20_nt32": (3, 20, 20, 32, 4, 100),
    # production-scale univariate 64x64 grid (b = 4096), 96 steps, 8 covariates
    "uni_64x64_nt96": (1, 64, 64, 96, 8, 1000),
    # reduced replicas of the above (same construction, small grid) for dense-oracle parity
    "uni_6x5_nt5": (1, 6, 5, 5, 6, 20),
    "uni_12x12_nt6": (1, 12, 12, 6, 6, 40),
    "coreg3_4x4_nt4": (3, 4, 4, 4, 6, 5),
    "coreg3_5x4_nt3": (3, 5, 4, 3, 6, 6),
    "uni_9x7_nt4": (1, 9, 7, 4, 3, 9),
    # coregionalised replicas with several 64-wide panels and a ragged last panel
    "coreg3_9x7_nt4": (3, 9, 7, 4, 6, 12),
    "coreg3_12x10_nt3": (3, 12, 10, 3, 6, 15),
}


def named_config(name: str, seed: int = 0) -> SpdeModel:
    k, nx, ny, nt, a, obs = NAMED_CONFIGS[name]
    return make_model(k, nx, ny, nt, a, obs, seed)
