"""CPU-side checks of the C ABI: the library loads and exports every declared entry point
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "adelia.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*\*?\s+\**([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_hot_path_calls():
    names = declared_functions()
    for n in ["bta_factor", "bta_factor_batched", "bta_logdet", "bta_solve", "bta_selinv",
              "inla_objective", "inla_grad", "inla_grad_batched", "inla_fd_grad", "inla_hessian",
              "inla_fd_hessian"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2605_06392_amd._lib import LIB_PATH, SIGNATURES
    if not os.path.exists(LIB_PATH):
        pytest.fail("libadelia.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    for name in SIGNATURES:
        assert name in declared_functions(), name


# ---- argument validation through the C ABI, without a GPU --------------------------------------
# Every entry point validates its arguments on the host before it touches the context or enqueues
# anything, so a dummy non-null context and fake (never dereferenced) device addresses exercise
# the documented return codes on the CPU.  Each call below has at least one invalid argument.

E_SHAPE, E_WORKSPACE, E_UNSUPPORTED = -100, -101, -103
CTX = 0x1000          # non-null, never dereferenced before the checks fail
P = 0x100000          # an aligned fake device address
MIS = 0x100004        # 8-byte aligned but not 256-byte aligned
ODD = 0x100003        # not 8-byte aligned


def _L():
    from paper_2605_06392_amd._lib import lib
    return lib()


def _shape(n, b, a):
    from paper_2605_06392_amd._lib import BtaShape
    return BtaShape(n, b, a)


def test_block_size_limit_keeps_operands_inside_32bit_buffer_range():
    L = _L()
    assert L.adelia_bta_workspace_bytes(_shape(2, 16320, 8), 1) > 0
    for which in (1, 2, 4, 7):
        assert L.adelia_bta_workspace_bytes(_shape(2, 16384, 2), which) == 0
    assert L.adelia_bta_workspace_bytes(_shape(0, 64, 2), 1) == 0
    assert L.adelia_bta_workspace_bytes(_shape(2, 64, 65), 1) == 0
    from paper_2605_06392_amd._lib import BtaShape
    shapes = (BtaShape * 2)(BtaShape(3, 64, 2), BtaShape(2, 16384, 2))
    assert L.adelia_bta_batched_workspace_bytes(2, shapes, 1) == 0
    shapes[1] = BtaShape(2, 128, 2)
    assert L.adelia_bta_batched_workspace_bytes(2, shapes, 1) > 0


def test_bta_factor_argument_codes():
    L = _L()
    ok = _shape(3, 64, 2)

    def call(ctx=CTX, sh=ok, D=P, B=P, C=P, T=P, Dinv=P, rhs=None, ld=P, info=P, ws=P, nb=1 << 40):
        return L.bta_factor(ctx, sh, D, B, C, T, Dinv, rhs, ld, info, ws, nb, None)

    assert call(ctx=None) == -1
    assert call(sh=_shape(2, 16384, 2)) == -2
    assert call(sh=_shape(0, 64, 2)) == -2
    assert call(D=None) == -3
    assert call(D=ODD) == -3
    assert call(B=None) == -4
    assert call(C=None) == -5
    assert call(T=None) == -6
    assert call(Dinv=None) == -7
    assert call(rhs=ODD) == -8
    assert call(ld=None) == -9
    assert call(info=P + 2) == -10
    assert call(ws=None) == -11
    assert call(ws=MIS) == -11
    assert call(nb=256) == E_WORKSPACE


def test_bta_factor_noalloc_argument_codes():
    """The entry point without a workspace numbers its argument errors as bta_factor does and
    rejects shapes whose factor workspace exceeds its static scratch before touching anything."""
    L = _L()
    ok = _shape(3, 64, 2)

    def call(ctx=CTX, sh=ok, D=P, B=P, C=P, T=P, Dinv=P, rhs=None, ld=P, info=P):
        return L.bta_factor_noalloc(ctx, sh, D, B, C, T, Dinv, rhs, ld, info, None)

    assert call(ctx=None) == -1
    assert call(sh=_shape(2, 16384, 2)) == -2
    assert call(D=ODD) == -3
    assert call(B=None) == -4
    assert call(C=None) == -5
    assert call(T=None) == -6
    assert call(Dinv=None) == -7
    assert call(rhs=ODD) == -8
    assert call(ld=None) == -9
    assert call(info=P + 2) == -10
    cap = 64 << 20
    big = _shape(2, 2048, 8)  # (2b + 9) b doubles of block scratch: 68 MB
    assert L.adelia_bta_workspace_bytes(big, 1) > cap
    assert call(sh=big) == E_WORKSPACE
    assert b"static scratch" in L.adelia_last_error()
    # the largest block that fits: the query stays inside the cap
    assert L.adelia_bta_workspace_bytes(_shape(50, 1024, 6), 1) <= cap


def test_bta_solve_selinv_logdet_argument_codes():
    L = _L()
    ok = _shape(3, 64, 2)
    solve = lambda ctx=CTX, sh=ok, G=P, LB=P, LC=P, LT=P, x=P, fl=0, ws=P, nb=1 << 40: (  # noqa: E731
        L.bta_solve(ctx, sh, G, LB, LC, LT, x, fl, ws, nb, None))
    assert solve(ctx=None) == -1
    assert solve(sh=_shape(1, 16384, 0)) == -2
    assert solve(G=None) == -3
    assert solve(LB=None) == -4
    assert solve(LC=ODD) == -5
    assert solve(LT=None) == -6
    assert solve(x=None) == -7
    assert solve(fl=4) == -8
    assert solve(ws=None) == -9
    assert solve(nb=8) == E_WORKSPACE
    sel = lambda ctx=CTX, sh=ok, G=P, LB=P, LC=P, LT=P, ZD=P, ZB=P, ZC=P, ZT=P, ws=P, nb=1 << 40: (  # noqa: E731
        L.bta_selinv(ctx, sh, G, LB, LC, LT, ZD, ZB, ZC, ZT, ws, nb, None))
    assert sel(ctx=None) == -1
    assert sel(sh=_shape(2, 64, 70)) == -2
    for k, kw in enumerate(["G", "LB", "LC", "LT", "ZD", "ZB", "ZC", "ZT", "ws"], start=3):
        assert sel(**{kw: None}) == -k, kw
    assert sel(nb=64) == E_WORKSPACE
    ldet = lambda ctx=CTX, sh=ok, LD=P, LT=P, out=P, ws=P, nb=1 << 20: (  # noqa: E731
        L.bta_logdet(ctx, sh, LD, LT, out, ws, nb, None))
    assert ldet(ctx=None) == -1
    assert ldet(sh=_shape(-1, 64, 2)) == -2
    assert ldet(LD=None) == -3
    assert ldet(LT=None) == -4
    assert ldet(out=ODD) == -5
    assert ldet(ws=None) == -6
    assert ldet(nb=8) == E_WORKSPACE


def test_dgemm_argument_codes():
    L = _L()

    def call(ctx=CTX, tA=0, tB=0, M=64, N=64, K=64, A=P, lda=64, B=P, ldb=64, C=P, ldc=64,
             batch=1, uplo=0):
        return L.adelia_dgemm(ctx, tA, tB, M, N, K, 1.0, A, lda, 0, B, ldb, 0, 0.0, C, ldc, 0,
                              batch, uplo, None)

    assert call(ctx=None) == -1
    assert call(tA=2) == -2
    assert call(tB=-1) == -3
    assert call(M=-1) == -4
    assert call(N=-1) == -5
    assert call(K=-1) == -6
    assert call(A=None) == -8
    assert call(lda=32) == -9
    assert call(B=ODD) == -11
    assert call(ldb=8) == -12
    assert call(C=None) == -15
    assert call(ldc=1) == -16
    assert call(batch=70000) == -18
    assert call(uplo=2) == -19
    assert call(M=64, N=32, uplo=1) == E_SHAPE
    # an operand of 2 GiB or more cannot be read through one buffer descriptor
    assert call(M=20000, N=64, K=20000, lda=20000, ldb=20000, ldc=20000) == E_SHAPE
    assert call(M=64, N=20000, K=20000, lda=64, ldb=20000, ldc=64) == E_SHAPE
    assert call(M=0) == 0  # nothing to do: returns before any launch


def test_batched_and_inla_argument_codes():
    from paper_2605_06392_amd._lib import BtaShape
    L = _L()
    shapes = (BtaShape * 2)(BtaShape(3, 64, 2), BtaShape(2, 16384, 2))
    ptrs = (ctypes.c_void_p * 2)(P, P)
    args = lambda ctx=CTX, cnt=2, sh=shapes: (ctx, cnt, sh, ptrs, ptrs, ptrs, ptrs, ptrs, None,  # noqa: E731
                                              P, P, P, 1 << 40, None)
    assert L.bta_factor_batched(*args(ctx=None)) == -1
    assert L.bta_factor_batched(*args(cnt=0)) == -2
    assert L.bta_factor_batched(*args()) == E_SHAPE
    assert L.inla_workspace_bytes(None, 1, 1) == 0
    assert L.inla_objective(None, P, 1, P, P, P, 1 << 30, 0, None) == -1
    assert L.inla_grad(None, P, P, P, P, P, 1 << 30, 0, None) == -1
    assert L.inla_grad_batched(None, P, 1, P, P, P, P, 1 << 30, None) == -1
    assert L.inla_fd_grad(None, P, 1e-3, 1, P, P, P, P, 1 << 30, None) == -1
    assert L.inla_hessian(None, P, 1e-3, 1, P, P, P, P, P, 1 << 30, None) == -1
    assert L.inla_fd_hessian(None, P, 1e-3, 1, P, P, P, P, 1 << 30, None) == -1
    assert L.inla_model_create(None, None, None) == -1
    h = ctypes.c_void_p()
    assert L.inla_model_create(CTX, None, ctypes.byref(h)) == -2


def test_inla_model_rejects_oversized_blocks():
    from paper_2605_06392_amd._lib import ModelDesc
    L = _L()
    d = ModelDesc()
    d.param, d.k, d.ns, d.nt, d.a, d.n_obs = 1, 1, 16384, 2, 0, 0
    d.sigma_prior, d.tip_prec = 0.5, 1e-3
    h = ctypes.c_void_p()
    assert L.inla_model_create(CTX, ctypes.byref(d), ctypes.byref(h)) == E_SHAPE
    assert b"16320" in L.adelia_last_error()
    d.param, d.k, d.ns = 2, 3, 5500  # b = k * ns = 16500
    assert L.inla_model_create(CTX, ctypes.byref(d), ctypes.byref(h)) == E_SHAPE
    d.param = 7
    assert L.inla_model_create(CTX, ctypes.byref(d), ctypes.byref(h)) == E_SHAPE


def test_tile_table_set_get_save_load(tmp_path):
    """The GEMM tile table: argument codes, and a JSON cache that round-trips and whose
    malformed forms are rejected without loading anything."""
    L = _L()
    L.adelia_tune_clear()
    try:
        assert L.adelia_tune_set(0, 4, 32) == -1
        assert L.adelia_tune_set(16384, 4, 32) == -1
        assert L.adelia_tune_set(128, 0, 32) == -2
        assert L.adelia_tune_set(128, 8, 32) == -2
        assert L.adelia_tune_set(128, 3, 32) == -2  # in-place panel rows keep 64
        assert L.adelia_tune_set(128, 4, 48) == -3
        assert L.adelia_tune_get(128, 4) == 64  # no entry: 64
        assert L.adelia_tune_set(128, 4, 32) == 0
        assert L.adelia_tune_set(1024, 7, 32) == 0
        assert L.adelia_tune_get(128, 4) == 32 and L.adelia_tune_get(1024, 7) == 32
        path = str(tmp_path / "tiles.json")
        assert L.adelia_tune_save(path.encode()) == 0
        import json
        doc = json.load(open(path))
        assert sorted((e["b"], e["role"], e["tile"]) for e in doc["tiles"]) == [
            (128, "schur_update", 32), (1024, "si_ZD", 32)]
        L.adelia_tune_clear()
        assert L.adelia_tune_get(128, 4) == 64
        assert L.adelia_tune_load(path.encode()) == 2
        assert L.adelia_tune_get(128, 4) == 32 and L.adelia_tune_get(1024, 7) == 32
        L.adelia_tune_clear()
        bad = tmp_path / "bad.json"
        bad.write_text('{"tiles": [{"b": 128, "role": "schur_update", "tile": 16}]}')
        assert L.adelia_tune_load(str(bad).encode()) == E_SHAPE
        bad.write_text('{"tiles": [{"b": 128, "role": "no_such_role", "tile": 32}]}')
        assert L.adelia_tune_load(str(bad).encode()) == E_SHAPE
        assert L.adelia_tune_get(128, 4) == 64
        assert L.adelia_tune_load(str(tmp_path / "missing.json").encode()) == E_UNSUPPORTED
    finally:
        L.adelia_tune_clear()


def test_autotune_and_batch_argument_codes():
    L = _L()
    ch = ctypes.c_int32(0)
    assert L.inla_autotune(None, P, 1, 1, 3, P, 1 << 30, None, ctypes.byref(ch)) == -1
    assert L.inla_batch_autotune(None, P, 1, 2, P, 1 << 30, None, ctypes.byref(ch)) == -1
    assert L.inla_batch_create(None, 1, None, None) == -1
    assert L.inla_batch_objective(None, P, P, P, P, 1 << 30, None) == -1
    assert L.inla_batch_grad(None, P, P, P, P, P, 1 << 30, None) == -1
    assert L.inla_batch_workspace_bytes(None, 1) == 0


def test_product_path_has_no_host_fallback():
    """The bindings only marshal arguments: without the built library, or without a GPU, every
    entry of the product path raises instead of computing anything on the host."""
    import subprocess
    import sys
    code = (
        "from paper_2605_06392_amd import _lib\n"
        "_lib.LIB_PATH = '/nonexistent/libadelia.so'\n"
        "_lib._lib = None\n"
        "try:\n"
        "    _lib.lib()\n"
        "except RuntimeError as e:\n"
        "    assert 'no CPU fallback' in str(e), e\n"
        "    print('raised')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                       cwd=ROOT)
    assert r.returncode == 0 and r.stdout.strip() == "raised", r.stderr
    from paper_2605_06392_amd._lib import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("library not built")
    import torch
    from workloads import named_config
    from paper_2605_06392_amd.inla import InlaModel
    spec = named_config("uni_6x5_nt5", 0)
    with pytest.raises(ValueError):
        InlaModel(spec, device="cpu")
    if not torch.cuda.is_available():
        with pytest.raises(RuntimeError):
            InlaModel(spec, device="cuda:0")
