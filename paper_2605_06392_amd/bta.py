"""Python surface of the BTA entry points (Sec. II-B layout, Sec. III-A algorithms).

Tensors are float64 on a HIP device, column-major per block: a tensor of shape (n, b, b) is
passed with each block transposed in memory, i.e. block i's element (r, c) lives at offset
i*b*b + r + c*b.  The helpers ``to_cm``/``from_cm`` convert from and to row-major numpy-style
blocks.  Only marshalling happens here; every computation runs in libadelia.so.
"""
import ctypes as C

import torch

from ._lib import BtaShape, check, lib

_ctx_cache = {}


def context(device=None):
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _ctx_cache:
        h = C.c_void_p()
        check(lib().adelia_create(C.byref(h), dev), "adelia_create")
        _ctx_cache[dev] = h
    return _ctx_cache[dev]


def _p(t):
    return C.c_void_p(0) if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def to_cm(x: torch.Tensor) -> torch.Tensor:
    """Row-major (..., r, c) blocks -> the same blocks stored column-major (contiguous)."""
    return x.transpose(-1, -2).contiguous()


def from_cm(x: torch.Tensor) -> torch.Tensor:
    return x.transpose(-1, -2)


def workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 256) // 8 + 32, dtype=torch.float64, device=device)


def _ws_ptr(ws):
    p = ws.data_ptr()
    return p + ((-p) % 256)


def dgemm(A, B, C_out, transA=False, transB=False, alpha=1.0, beta=0.0, lower=False):
    """Batched C = alpha op(A) op(B) + beta C on column-major blocks (leading dim = rows)."""
    batch = A.shape[0]
    M = C_out.shape[-1]   # column-major: stored as (cols, rows) in row-major terms
    N = C_out.shape[-2]
    K = A.shape[-2] if not transA else A.shape[-1]
    lda = A.shape[-1]
    ldb = B.shape[-1]
    ldc = C_out.shape[-1]
    sA = A.shape[-1] * A.shape[-2]
    sB = B.shape[-1] * B.shape[-2]
    sC = C_out.shape[-1] * C_out.shape[-2]
    r = lib().adelia_dgemm(context(), int(transA), int(transB), M, N, K, alpha, _p(A), lda, sA,
                           _p(B), ldb, sB, beta, _p(C_out), ldc, sC, batch, int(lower), _stream())
    check(r, "adelia_dgemm")
    return C_out


def bta_factor(D, B, C_arrow, T, rhs=None):
    """In-place factorisation.  D (n,b,b), B (n-1,b,b), C (n, b, a) [column-major a x b],
    T (a, a) column-major, rhs (N,) or None.  Returns (Dinv, logdet, info)."""
    n, b = D.shape[0], D.shape[1]
    a = T.shape[0] if T is not None else 0
    dev = D.device
    sh = BtaShape(n, b, a)
    nbytes = lib().adelia_bta_workspace_bytes(sh, 1)
    ws = workspace(nbytes, dev)
    Dinv = torch.empty_like(D)
    logdet = torch.empty(1, dtype=torch.float64, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    r = lib().bta_factor(context(), sh, _p(D), _p(B if n > 1 else None),
                         _p(C_arrow if a else None), _p(T if a else None), _p(Dinv), _p(rhs),
                         _p(logdet), _p(info), C.c_void_p(_ws_ptr(ws)), nbytes, _stream())
    check(r, "bta_factor")
    return Dinv, logdet, info


def bta_factor_batched(mats, with_rhs=False):
    """Uneven batch: mats is a list of dicts with D (n,b,b), B (n-1,b,b) or None, C (n,b,a) or
    None, T (a,a) or None and, with with_rhs, rhs (N,).  Factorised in place as bta_factor does
    for each; returns (list of Dinv, logdet (count,), info (count,))."""
    count = len(mats)
    dev = mats[0]["D"].device
    shapes = (BtaShape * count)()
    ptr = lambda t: (t.data_ptr() if t is not None else None)  # noqa: E731
    arr = lambda vals: (C.c_void_p * count)(*vals)  # noqa: E731
    dinv = []
    for i, m in enumerate(mats):
        n, b = m["D"].shape[0], m["D"].shape[1]
        a = m["T"].shape[0] if m.get("T") is not None else 0
        shapes[i] = BtaShape(n, b, a)
        dinv.append(torch.empty_like(m["D"]))
    nbytes = lib().adelia_bta_batched_workspace_bytes(count, shapes, int(with_rhs))
    if nbytes == 0:
        raise ValueError("invalid shapes for bta_factor_batched")
    ws = workspace(nbytes, dev)
    logdet = torch.empty(count, dtype=torch.float64, device=dev)
    info = torch.empty(count, dtype=torch.int32, device=dev)
    r = lib().bta_factor_batched(
        context(), count, shapes, arr([ptr(m["D"]) for m in mats]),
        arr([ptr(m.get("B")) for m in mats]), arr([ptr(m.get("C")) for m in mats]),
        arr([ptr(m.get("T")) for m in mats]), arr([ptr(t) for t in dinv]),
        arr([ptr(m["rhs"]) for m in mats]) if with_rhs else None,
        _p(logdet), _p(info), C.c_void_p(_ws_ptr(ws)), nbytes, _stream())
    check(r, "bta_factor_batched")
    return dinv, logdet, info


def bta_logdet(LD, LT):
    n, b = LD.shape[0], LD.shape[1]
    a = LT.shape[0] if LT is not None else 0
    sh = BtaShape(n, b, a)
    ws = workspace((n + 1) * 8 + 256, LD.device)
    out = torch.empty(1, dtype=torch.float64, device=LD.device)
    r = lib().bta_logdet(context(), sh, _p(LD), _p(LT if a else None), _p(out),
                         C.c_void_p(_ws_ptr(ws)), (n + 1) * 8 + 256, _stream())
    check(r, "bta_logdet")
    return out


def bta_solve(Dinv, LB, LC, LT, x, z_input=False):
    n, b = Dinv.shape[0], Dinv.shape[1]
    a = LT.shape[0] if LT is not None else 0
    sh = BtaShape(n, b, a)
    nbytes = lib().adelia_bta_workspace_bytes(sh, 2)
    ws = workspace(nbytes, Dinv.device)
    r = lib().bta_solve(context(), sh, _p(Dinv), _p(LB if n > 1 else None), _p(LC if a else None),
                        _p(LT if a else None), _p(x), int(bool(z_input)), C.c_void_p(_ws_ptr(ws)),
                        nbytes, _stream())
    check(r, "bta_solve")
    return x


def bta_selinv(Dinv, LB, LC, LT):
    n, b = Dinv.shape[0], Dinv.shape[1]
    a = LT.shape[0] if LT is not None else 0
    dev = Dinv.device
    sh = BtaShape(n, b, a)
    nbytes = lib().adelia_bta_workspace_bytes(sh, 4)
    ws = workspace(nbytes, dev)
    ZD = torch.empty((n, b, b), dtype=torch.float64, device=dev)
    ZB = torch.empty((max(n - 1, 1), b, b), dtype=torch.float64, device=dev)
    ZC = torch.empty((n, b, max(a, 1)), dtype=torch.float64, device=dev)
    ZT = torch.empty((max(a, 1), max(a, 1)), dtype=torch.float64, device=dev)
    r = lib().bta_selinv(context(), sh, _p(Dinv), _p(LB if n > 1 else None), _p(LC if a else None),
                         _p(LT if a else None), _p(ZD), _p(ZB if n > 1 else None),
                         _p(ZC if a else None), _p(ZT if a else None), C.c_void_p(_ws_ptr(ws)),
                         nbytes, _stream())
    check(r, "bta_selinv")
    return ZD, ZB, ZC, ZT


class profile:
    """Context manager around adelia_profile_start/stop.  ``stats`` maps kernel name to
    dict(launches, ms, flops, bytes) after exit (the exit synchronises the device)."""

    def __init__(self, max_launches=200000, device=None):
        self.max_launches = max_launches
        self.device = device
        self.stats = {}

    def __enter__(self):
        check(lib().adelia_profile_start(context(self.device), self.max_launches), "profile_start")
        return self

    def __exit__(self, *exc):
        from ._lib import KernelStats
        arr = (KernelStats * 32)()
        n = C.c_int(0)
        check(lib().adelia_profile_stop(context(self.device), arr, 32, C.byref(n)), "profile_stop")
        for i in range(n.value):
            s = arr[i]
            self.stats[s.name.decode()] = dict(launches=int(s.launches), ms=float(s.ms),
                                               flops=float(s.flops), bytes=float(s.bytes))
        return False
