"""Seeded random SPD block-tridiagonal-arrowhead matrices (Sec. II-B layout).

Off-pattern entries are uniform in [-s, s]; each diagonal entry is set to the absolute row sum
of the off-diagonal entries of the full symmetric matrix plus ``shift``, which makes the matrix
strictly diagonally dominant and hence SPD.  Blocks: D (n,b,b) symmetric, B (n-1,b,b) the
sub-diagonal blocks [Q]_{i+1,i}, C (n,a,b) arrow rows [Q]_{T,i}, T (a,a).
"""
from __future__ import annotations

import numpy as np


def random_bta(n: int, b: int, a: int, seed: int, scale: float = 1.0, shift: float = 1.0):
    rng = np.random.default_rng(seed)
    D = rng.uniform(-scale, scale, size=(n, b, b))
    D = 0.5 * (D + np.transpose(D, (0, 2, 1)))
    B = rng.uniform(-scale, scale, size=(max(n - 1, 0), b, b))
    C = rng.uniform(-scale, scale, size=(n, a, b))
    T = rng.uniform(-scale, scale, size=(a, a))
    T = 0.5 * (T + T.T)
    rhs = rng.standard_normal(n * b + a)
    for i in range(n):
        np.fill_diagonal(D[i], 0.0)
    np.fill_diagonal(T, 0.0)
    for i in range(n):
        rows = np.abs(D[i]).sum(axis=1)
        if i > 0:
            rows += np.abs(B[i - 1]).sum(axis=1)
        if i < n - 1:
            rows += np.abs(B[i]).sum(axis=0)
        if a:
            rows += np.abs(C[i]).sum(axis=0)
        D[i][np.diag_indices(b)] = rows + shift
    if a:
        rows = np.abs(T).sum(axis=1) + sum(np.abs(C[i]).sum(axis=1) for i in range(n))
        T[np.diag_indices(a)] = rows + shift
    return {"D": D, "B": B, "C": C, "T": T, "rhs": rhs}


def random_bta_device(n: int, b: int, a: int, seed: int, device, scale: float = 1.0,
                      shift: float = 1.0):
    """random_bta's recipe drawn with torch's generator on ``device`` (other numbers, the same
    distribution and the same diagonal dominance), for batches too large to draw on the host.
    Blocks are returned row-major, as random_bta returns them."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    f64 = torch.float64

    def u(*shape):
        return (torch.rand(*shape, generator=g, device=device, dtype=f64) * 2 - 1) * scale

    D = u(n, b, b)
    D = 0.5 * (D + D.transpose(1, 2))
    B = u(max(n - 1, 0), b, b)
    C = u(n, a, b)
    T = u(a, a)
    T = 0.5 * (T + T.T)
    rhs = torch.randn(n * b + a, generator=g, device=device, dtype=f64)
    idx = torch.arange(b, device=device)
    D[:, idx, idx] = 0.0
    rows = D.abs().sum(2)
    if n > 1:
        rows[1:] += B.abs().sum(2)
        rows[:-1] += B.abs().sum(1)
    if a:
        rows += C.abs().sum(1)
    D[:, idx, idx] = rows + shift
    if a:
        ia = torch.arange(a, device=device)
        T[ia, ia] = 0.0
        T[ia, ia] = T.abs().sum(1) + C.abs().sum(2).sum(0) + shift
    return {"D": D, "B": B, "C": C, "T": T, "rhs": rhs}
