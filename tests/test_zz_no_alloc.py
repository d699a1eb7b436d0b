"""GPU parity of bta_factor_noalloc (the factorisation without a workspace argument, working in
the library's static device scratch) against bta_factor with a caller workspace, through the C
ABI: two calls in a row, the second on a smaller matrix, each compared with bta_factor's outputs
on the same input (same kernels in the same order, so the results agree bit for bit), and the
first also with dense Cholesky."""
import ctypes as C

import numpy as np
import pytest
import scipy.linalg as sla
import torch

from workloads.bta import random_bta

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _inputs(n, b, a, seed, dev):
    from paper_2605_06392_amd.bta import to_cm
    blk = random_bta(n, b, a, seed)
    t = lambda x: to_cm(torch.from_numpy(np.ascontiguousarray(x)).to(dev))  # noqa: E731
    return blk, dict(D=t(blk["D"]), B=t(blk["B"] if n > 1 else np.zeros((1, b, b))),
                     C=t(blk["C"] if a else np.zeros((n, 1, b))),
                     T=t(blk["T"][None])[0] if a else None,
                     rhs=torch.from_numpy(blk["rhs"].copy()).to(dev))


def _run(n, b, a, seed, dev, noalloc):
    from paper_2605_06392_amd import bta
    from paper_2605_06392_amd._lib import BtaShape, check, lib
    blk, m = _inputs(n, b, a, seed, dev)
    Dinv = torch.empty_like(m["D"])
    logdet = torch.empty(1, dtype=torch.float64, device=dev)
    info = torch.full((1,), -7, dtype=torch.int32, device=dev)
    p = bta._p
    sh = BtaShape(n, b, a)
    args = [bta.context(), sh, p(m["D"]), p(m["B"] if n > 1 else None), p(m["C"] if a else None),
            p(m["T"] if a else None), p(Dinv), p(m["rhs"]), p(logdet), p(info)]
    if noalloc:
        r = lib().bta_factor_noalloc(*args, bta._stream())
        ws = None
    else:
        nbytes = lib().adelia_bta_workspace_bytes(sh, 1)
        ws = bta.workspace(nbytes, dev)
        r = lib().bta_factor(*args, C.c_void_p(bta._ws_ptr(ws)), nbytes, bta._stream())
    check(r, "factor")
    torch.cuda.synchronize()
    out = {k: (v.cpu().numpy().copy() if v is not None else None) for k, v in m.items()}
    out.update(Dinv=Dinv.cpu().numpy(), logdet=float(logdet.item()), info=int(info.item()))
    return blk, out


# two calls in a row: the first fills much of the scratch, the second (smaller, other ragged
# tail and arrow) runs on the leftovers of the first
CASES = [(5, 200, 6, 11), (3, 70, 2, 12)]


def test_noalloc_factor_matches_workspace_factor_twice_in_a_row():
    dev = _dev()
    for (n, b, a, seed) in CASES:
        print(f"bta_factor_noalloc n={n} b={b} a={a} seed={seed}", flush=True)
        _, ref = _run(n, b, a, seed, dev, noalloc=False)
        blk, got = _run(n, b, a, seed, dev, noalloc=True)
        assert got["info"] == 0 and ref["info"] == 0
        for key in ("D", "B", "C", "T", "rhs", "Dinv"):
            if ref[key] is None:
                continue
            assert np.array_equal(got[key], ref[key]), key
        assert got["logdet"] == ref["logdet"]
        # and against the definition: dense Cholesky of the assembled matrix
        import oracle
        Q = oracle.bta_dense(blk["D"], blk["B"], blk["C"], blk["T"])
        L = np.linalg.cholesky(Q)
        ld_ref = 2.0 * np.log(np.diag(L)).sum()
        assert abs(got["logdet"] - ld_ref) <= 1e-12 * abs(ld_ref)
        z_ref = sla.solve_triangular(L, blk["rhs"], lower=True)
        assert np.abs(got["rhs"] - z_ref).max() <= 1e-11 * np.abs(z_ref).max()


def test_noalloc_factor_reports_failure_and_recovers():
    """A matrix that is not positive definite gives info > 0 in the static scratch path too, and
    the next call on a good matrix is unaffected by what the failed one left behind."""
    dev = _dev()
    from paper_2605_06392_amd import bta
    from paper_2605_06392_amd._lib import BtaShape, check, lib
    n, b, a = 2, 64, 2
    blk, m = _inputs(n, b, a, 5, dev)
    m["D"][1].diagonal().mul_(-1.0)  # block 1 indefinite
    Dinv = torch.empty_like(m["D"])
    logdet = torch.empty(1, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    p = bta._p
    r = lib().bta_factor_noalloc(bta.context(), BtaShape(n, b, a), p(m["D"]), p(m["B"]), p(m["C"]),
                                 p(m["T"]), p(Dinv), p(m["rhs"]), p(logdet), p(info),
                                 bta._stream())
    check(r, "factor")
    torch.cuda.synchronize()
    assert int(info.item()) > b  # the first failing column lies in block 1
    _, ref = _run(3, 70, 2, 12, dev, noalloc=False)
    _, got = _run(3, 70, 2, 12, dev, noalloc=True)
    assert got["info"] == 0
    assert np.array_equal(got["D"], ref["D"]) and got["logdet"] == ref["logdet"]
