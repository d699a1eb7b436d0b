"""Host checks of the seeded input generators (the workloads package) and of the benchmark's
one-GPU contract.  No GPU and no HIP library are needed.

The generators draw the synthetic models both the oracle and the HIP path evaluate; these
tests pin the properties their docstrings state against what mathematics fixes:
- the cosine eigenbasis of the Neumann second difference is orthonormal and diagonalises it;
- the latent field is an exact draw from N(0, Q^-1) of the prior at theta = 0 (the linear map
  from the noise to the field, applied to every unit vector, gives S with S S^T = Q^-1);
- bilinear observation weights are non-negative, sum to one and reproduce the location;
- the named workloads have the sizes their names state (b = k nx ny, N = n b + a, d);
- the random BTA matrices are symmetric positive definite with the stated block layout.
"""
import os
import subprocess
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from workloads import NAMED_CONFIGS, make_model, named_config, neumann_second_difference
from workloads import spde
from workloads.bta import random_bta

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _l1(m):
    d, o = neumann_second_difference(m)
    return np.diag(d) + np.diag(o, 1) + np.diag(o, -1)


@pytest.mark.parametrize("m", [1, 2, 5, 8])
def test_neumann_eigenbasis_is_orthonormal_and_diagonalises(m):
    v, lam = spde._neumann_eigen(m)
    assert np.allclose(v.T @ v, np.eye(m), atol=1e-13)
    assert np.allclose(_l1(m) @ v, v * lam[None, :], atol=1e-12)
    # the Neumann operator annihilates constants: one zero eigenvalue, row sums zero
    assert abs(lam[0]) < 1e-15 and np.allclose(_l1(m).sum(axis=1), 0.0)


@pytest.mark.parametrize("nx,ny,nt", [(3, 2, 3), (2, 2, 1), (4, 1, 2)])
def test_latent_field_is_an_exact_prior_draw(nx, ny, nt):
    ns = nx * ny
    dim = ns * nt
    cols = []
    for j in range(dim):
        xi = np.zeros(dim)
        xi[j] = 1.0
        cols.append(spde._sample_field(nx, ny, nt, xi).reshape(-1))  # (t, node) order
    S = np.stack(cols, axis=1)
    # the prior precision at theta = 0 in time-major order: the kernel (I + g1), squared, on
    # every step, (I + g1) coupled through M1 and the identity through M2
    _, g1, _ = spde._base_matrices(nx, ny)
    K = np.eye(ns) + g1.toarray()
    m2 = 2.0 * np.eye(nt) - np.eye(nt, k=1) - np.eye(nt, k=-1)
    Q = np.kron(np.eye(nt), K @ K) + np.kron(_l1(nt), K) + np.kron(m2, np.eye(ns))
    assert np.allclose(S @ S.T, np.linalg.inv(Q), rtol=1e-11, atol=1e-13)


def test_base_matrices_are_the_stated_grid_operators():
    nx, ny = 4, 3
    c0, g1, g2 = spde._base_matrices(nx, ny)
    lap = np.kron(np.eye(ny), _l1(nx)) + np.kron(_l1(ny), np.eye(nx))
    assert np.array_equal(c0.toarray(), np.eye(nx * ny))
    assert np.allclose(g1.toarray(), lap + 0.1 * np.eye(nx * ny), atol=0)
    assert np.allclose(g2.toarray(), g1.toarray() @ g1.toarray(), atol=1e-14)
    # Neumann Laplacian: rows of g1 sum to the 0.1 shift; every matrix symmetric, sorted CSR
    assert np.allclose(np.asarray(g1.sum(axis=1)).ravel(), 0.1)
    for m in (c0, g1, g2):
        assert (abs(m - m.T)).max() == 0 and m.has_sorted_indices


@pytest.mark.parametrize("nx,ny", [(6, 5), (1, 4), (5, 1)])
def test_bilinear_weights_reproduce_the_location(nx, ny):
    spec = make_model(1, nx, ny, 3, 2, 17, seed=11)
    w, nodes, uv = spec.obs_w, spec.obs_node, spec.extra["obs_uv"]
    assert (w >= 0).all() and np.allclose(w.sum(axis=1), 1.0)
    assert (nodes >= 0).all() and (nodes < nx * ny).all()
    ix, iy = nodes % nx, nodes // nx
    assert np.allclose((w * ix).sum(axis=1), uv[:, 0])
    assert np.allclose((w * iy).sum(axis=1), uv[:, 1])


def test_models_are_seeded():
    a, b = named_config("uni_6x5_nt5", 3), named_config("uni_6x5_nt5", 3)
    c = named_config("uni_6x5_nt5", 4)
    for f in ("y", "X", "obs_w", "obs_node", "theta"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert not np.array_equal(a.y, c.y) and not np.array_equal(a.theta, c.theta)


@pytest.mark.parametrize("name,b,n,a,d,nobs", [
    ("uni_32x32_nt50", 1024, 50, 6, 4, 50 * 200),
    ("coreg3_30x30_nt48", 2700, 48, 6, 15, 48 * 3 * 300),
    ("coreg3_20x20_nt32", 1200, 32, 4, 15, 32 * 3 * 100),
    ("uni_64x64_nt96", 4096, 96, 8, 4, 96 * 1000),
])
def test_named_workload_sizes(name, b, n, a, d, nobs):
    k, nx, ny, nt, aa, per = NAMED_CONFIGS[name]
    assert (k * nx * ny, nt, aa) == (b, n, a)
    assert nt * k * per == nobs
    if name == "uni_32x32_nt50":  # the benchmark's default workload, drawn in full
        spec = named_config(name, 0)
        assert (spec.b, spec.nt, spec.a, spec.d, spec.N, spec.n_obs) == (b, n, a, d, 51206, nobs)
        assert spec.X.shape == (nobs, a) and np.isfinite(spec.y).all()
    else:
        assert (4 if k == 1 else 4 * k + k * (k - 1) // 2) == d


@pytest.mark.parametrize("n,b,a", [(3, 5, 2), (1, 4, 0), (4, 3, 1)])
def test_random_bta_is_spd_with_the_block_layout(n, b, a):
    m = random_bta(n, b, a, seed=5)
    assert m["D"].shape == (n, b, b) and m["B"].shape == (max(n - 1, 0), b, b)
    assert m["C"].shape == (n, a, b) and m["T"].shape == (a, a) and m["rhs"].shape == (n * b + a,)
    N = n * b + a
    Q = np.zeros((N, N))
    for i in range(n):
        Q[i * b:(i + 1) * b, i * b:(i + 1) * b] = m["D"][i]
        if i < n - 1:
            Q[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = m["B"][i]
            Q[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = m["B"][i].T
        Q[n * b:, i * b:(i + 1) * b] = m["C"][i]
        Q[i * b:(i + 1) * b, n * b:] = m["C"][i].T
    Q[n * b:, n * b:] = m["T"]
    assert np.array_equal(Q, Q.T)
    off = np.abs(Q).sum(axis=1) - np.abs(np.diag(Q))
    assert (np.diag(Q) - off >= 1.0 - 1e-12).all()  # strictly dominant by the shift
    assert np.linalg.eigvalsh(Q).min() > 0


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr and r.stdout == ""
