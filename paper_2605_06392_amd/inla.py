"""Python surface of the INLA entry points (argument marshalling only).

``InlaModel`` uploads a model once (``inla_model_create``); ``objective`` evaluates f for a
batch of theta points, ``grad`` returns f and the exact gradient (Sec. III-A-3, Eq. 5),
``fd_grad`` the (2d+1)-point central-difference gradient on the GPU (Sec. II-D, Eq. 2),
``hessian`` the posterior Hessian from 2d+1 exact gradients (Sec. III-D, Eq. 12) and
``fd_hessian`` its (2d^2+1)-point finite-difference counterpart, and
``InlaObjective`` is the torch.autograd.Function whose forward keeps the Cholesky factors of
Qc and Qp in the model's workspace and whose backward runs the hand-written reverse pass
(selected inversion + traces) from them.
"""
import ctypes as C
import itertools

import numpy as np
import torch
from torch.autograd.function import once_differentiable

from ._lib import ModelDesc, check, lib
from .bta import context

PARAM_UNIVARIATE = 1
PARAM_COREG = 2
MODE_OBJECTIVE = 0
MODE_GRAD = 1
MODE_GRAD_CARRY = 2
MODE_OBJECTIVE_SPLIT = 3
MODE_GRAD_SPLIT = 4
SAVE_FACTORS = 1
REUSE_FACTORS = 1
CARRY_ONLY = 2
SPLIT = 4

_token = itertools.count(1)

# GEMM roles whose tile edge (64 or 32) the autotuner chooses, by the library's role number
# (role 3, the split schedule's panel rows, is formed in place and keeps 64 x 64 tiles)
TILE_ROLES = {1: "trailing", 2: "trtri", 4: "schur_update", 5: "si_W", 6: "si_ZB", 7: "si_ZD"}


def tile_table(block_sizes):
    """The tile edge of every tuned role at each block size: {b: {role name: 64 | 32}}."""
    return {int(b): {name: int(lib().adelia_tune_get(int(b), r)) for r, name in TILE_ROLES.items()}
            for b in block_sizes}


def set_tiles(b, tile, roles=None):
    """Set the tile edge of `roles` (names or numbers; default all) at block size b."""
    for r, name in TILE_ROLES.items():
        if roles is None or r in roles or name in roles:
            check(lib().adelia_tune_set(int(b), r, int(tile)), "adelia_tune_set")


def clear_tiles():
    lib().adelia_tune_clear()


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None and a.size else C.c_void_p(0)


class InlaModel:
    """A model on one HIP device.  ``spec`` provides: kind ("univariate" | "coreg"), k, nx, ny,
    nt, a, base matrices c0, g1, g2 (scipy CSR), temporal (diag, off) pairs m0, m1, m2, the
    observations (obs_t, obs_field, obs_node, obs_w, X, y), sigma_prior and tip_prec."""

    def __init__(self, spec, device="cuda:0"):
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.k = int(spec.k)
        self.ns = int(spec.nx * spec.ny)
        self.nt = int(spec.nt)
        self.a = int(spec.a)
        self.b = self.k * self.ns
        host = {}

        def i32(x):
            return np.ascontiguousarray(np.asarray(x, dtype=np.int32))

        def f64(x):
            return np.ascontiguousarray(np.asarray(x, dtype=np.float64))

        for name in ("c0", "g1", "g2"):
            mtx = getattr(spec, name).tocsr()
            mtx.sort_indices()
            host[name] = (i32(mtx.indptr), i32(mtx.indices), f64(mtx.data))
        for name in ("m0", "m1", "m2"):
            dg, off = getattr(spec, name)
            host[name] = (f64(dg), f64(off) if len(off) else np.zeros(1))
        host["obs_t"] = i32(spec.obs_t)
        host["obs_field"] = i32(spec.obs_field)
        host["obs_node"] = i32(spec.obs_node).reshape(-1)
        host["obs_w"] = f64(spec.obs_w).reshape(-1)
        host["X"] = f64(spec.X).reshape(-1)
        host["y"] = f64(spec.y)
        desc = ModelDesc()
        desc.param = PARAM_UNIVARIATE if spec.kind == "univariate" else PARAM_COREG
        desc.k, desc.ns, desc.nt, desc.a = self.k, self.ns, self.nt, self.a
        desc.n_obs = int(len(spec.y))
        desc.c0_ptr, desc.c0_idx, desc.c0_val = (_ptr(v) for v in host["c0"])
        desc.g1_ptr, desc.g1_idx, desc.g1_val = (_ptr(v) for v in host["g1"])
        desc.g2_ptr, desc.g2_idx, desc.g2_val = (_ptr(v) for v in host["g2"])
        desc.m0_diag, desc.m0_off = (_ptr(v) for v in host["m0"])
        desc.m1_diag, desc.m1_off = (_ptr(v) for v in host["m1"])
        desc.m2_diag, desc.m2_off = (_ptr(v) for v in host["m2"])
        desc.obs_t = _ptr(host["obs_t"])
        desc.obs_field = _ptr(host["obs_field"])
        desc.obs_node = _ptr(host["obs_node"])
        desc.obs_w = _ptr(host["obs_w"])
        desc.X = _ptr(host["X"])
        desc.y = _ptr(host["y"])
        desc.sigma_prior = float(spec.sigma_prior)
        desc.tip_prec = float(spec.tip_prec)
        h = C.c_void_p()
        dev_index = self.device.index if self.device.index is not None else torch.cuda.current_device()
        check(lib().inla_model_create(context(dev_index), C.byref(desc), C.byref(h)),
              "inla_model_create")
        self._h = h
        self.d = lib().inla_model_dim(h)
        self._ws = {}
        self.saved_token = 0

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().inla_model_destroy(self._h)
                self._h = None
        except Exception:
            pass

    # -- workspaces (torch-owned device memory, kept per (batch, mode)) -----------------------
    def new_workspace(self, batch, mode):
        """A fresh torch-owned workspace buffer for `batch` points in `mode`: (buffer, bytes)."""
        nbytes = lib().inla_workspace_bytes(self._h, batch, mode)
        if nbytes == 0:
            raise ValueError("invalid workspace request")
        return torch.empty(nbytes // 8 + 64, dtype=torch.float64, device=self.device), nbytes

    @staticmethod
    def _aligned(buf, nbytes):
        p = buf.data_ptr()
        return C.c_void_p(p + ((-p) % 256)), nbytes

    def workspace(self, batch, mode, private=None):
        """The model's shared workspace for (batch, mode), or `private` = (buffer, bytes)."""
        if private is not None:
            return self._aligned(*private)
        key = (batch, mode)
        if key not in self._ws:
            self._ws[key] = self.new_workspace(batch, mode)
        return self._aligned(*self._ws[key])

    def workspace_bytes(self, batch, mode):
        return int(lib().inla_workspace_bytes(self._h, batch, mode))

    @staticmethod
    def _stream():
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def _theta(self, theta):
        t = torch.as_tensor(theta, dtype=torch.float64, device=self.device)
        return t.contiguous()

    # -- evaluations ---------------------------------------------------------------------------
    def objective(self, theta, out=None, info=None, ws=None, split=False):
        """f at a batch of points; split=True (one point): the two-sided split of the sweep."""
        th = self._theta(theta)
        th2 = th.reshape(-1, self.d)
        batch = th2.shape[0]
        f = out if out is not None else torch.empty(batch, dtype=torch.float64, device=self.device)
        inf = info if info is not None else torch.empty(batch, dtype=torch.int32, device=self.device)
        ws, nb = self.workspace(batch, MODE_OBJECTIVE_SPLIT if split else MODE_OBJECTIVE, ws)
        check(lib().inla_objective(self._h, C.c_void_p(th2.data_ptr()), batch,
                                   C.c_void_p(f.data_ptr()), C.c_void_p(inf.data_ptr()), ws, nb,
                                   SPLIT if split else 0, self._stream()), "inla_objective")
        return f, inf

    def forward_saved(self, theta):
        th = self._theta(theta).reshape(self.d)
        f = torch.empty(1, dtype=torch.float64, device=self.device)
        inf = torch.empty(1, dtype=torch.int32, device=self.device)
        ws, nb = self.workspace(1, MODE_GRAD)
        check(lib().inla_objective(self._h, C.c_void_p(th.data_ptr()), 1, C.c_void_p(f.data_ptr()),
                                   C.c_void_p(inf.data_ptr()), ws, nb, SAVE_FACTORS,
                                   self._stream()), "inla_objective(save)")
        self.saved_token = next(_token)
        return f, inf, self.saved_token

    def grad(self, theta, reuse=False, f=None, g=None, info=None, carry=False, split=False):
        """f and the exact gradient; carry=True keeps only the per-block carries and rebuilds
        the factors in the backward pass (less memory, one more block Cholesky per block);
        split=True runs the two-sided split (both halves of the block chain at once, then the
        separator block and the tip as the reduced system)."""
        th = self._theta(theta).reshape(self.d)
        f = f if f is not None else torch.empty(1, dtype=torch.float64, device=self.device)
        g = g if g is not None else torch.empty(self.d, dtype=torch.float64, device=self.device)
        inf = info if info is not None else torch.empty(1, dtype=torch.int32, device=self.device)
        mode = MODE_GRAD_SPLIT if split else (MODE_GRAD_CARRY if carry else MODE_GRAD)
        ws, nb = self.workspace(1, mode)
        flags = ((REUSE_FACTORS if reuse else 0) | (CARRY_ONLY if carry else 0)
                 | (SPLIT if split else 0))
        check(lib().inla_grad(self._h, C.c_void_p(th.data_ptr()), C.c_void_p(f.data_ptr()),
                              C.c_void_p(g.data_ptr()), C.c_void_p(inf.data_ptr()), ws, nb,
                              flags, self._stream()), "inla_grad")
        self.saved_token = 0  # a reuse consumes the saved factors, a new pass overwrites them
        return f, g, inf

    def grad_terms(self, theta, reuse=False, carry=False):
        """f, gradient and its decomposition as a dict of host numpy values."""
        th = self._theta(theta).reshape(self.d)
        d = self.d
        terms = torch.empty(5 + 6 * d, dtype=torch.float64, device=self.device)
        inf = torch.empty(1, dtype=torch.int32, device=self.device)
        ws, nb = self.workspace(1, MODE_GRAD_CARRY if carry else MODE_GRAD)
        flags = (REUSE_FACTORS if reuse else 0) | (CARRY_ONLY if carry else 0)
        check(lib().inla_grad_terms(self._h, C.c_void_p(th.data_ptr()), C.c_void_p(terms.data_ptr()),
                                    C.c_void_p(inf.data_ptr()), ws, nb, flags, self._stream()),
              "inla_grad_terms")
        self.saved_token = 0
        t = terms.cpu().numpy()
        return {"f": t[0], "logdet_p": t[1], "logdet_c": t[2], "zsq": t[3], "trZT": t[4],
                "phaseA": t[5:5 + d], "phaseB": t[5 + d:5 + 2 * d], "phaseC": t[5 + 2 * d:5 + 3 * d],
                "dloglik": t[5 + 3 * d:5 + 4 * d], "dlogprior": t[5 + 4 * d:5 + 5 * d],
                "grad": t[5 + 5 * d:5 + 6 * d], "info": int(inf.item())}

    def fd_grad(self, theta, h=1e-3, max_batch=None, f=None, g=None, info=None):
        th = self._theta(theta).reshape(self.d)
        npts = 2 * self.d + 1
        mb = npts if max_batch is None else int(max_batch)
        mb = min(mb, npts)
        f = f if f is not None else torch.empty(1, dtype=torch.float64, device=self.device)
        g = g if g is not None else torch.empty(self.d, dtype=torch.float64, device=self.device)
        inf = info if info is not None else torch.empty(npts, dtype=torch.int32, device=self.device)
        ws, nb = self.workspace(mb, MODE_OBJECTIVE)
        check(lib().inla_fd_grad(self._h, C.c_void_p(th.data_ptr()), float(h), mb,
                                 C.c_void_p(f.data_ptr()), C.c_void_p(g.data_ptr()),
                                 C.c_void_p(inf.data_ptr()), ws, nb, self._stream()),
              "inla_fd_grad")
        return f, g, inf

    def grad_batched(self, theta, f=None, g=None, info=None, ws=None):
        """f and the exact gradient at a batch of theta points (batch x d) in one pass.  With
        `ws` (a private workspace from new_workspace) the model's shared workspaces, and any
        factors saved in them, are left alone."""
        th = self._theta(theta).reshape(-1, self.d).contiguous()
        B = th.shape[0]
        f = f if f is not None else torch.empty(B, dtype=torch.float64, device=self.device)
        g = g if g is not None else torch.empty((B, self.d), dtype=torch.float64, device=self.device)
        inf = info if info is not None else torch.empty(B, dtype=torch.int32, device=self.device)
        wsp, nb = self.workspace(B, MODE_GRAD, ws)
        check(lib().inla_grad_batched(self._h, C.c_void_p(th.data_ptr()), B,
                                      C.c_void_p(f.data_ptr()), C.c_void_p(g.data_ptr()),
                                      C.c_void_p(inf.data_ptr()), wsp, nb, self._stream()),
              "inla_grad_batched")
        if ws is None:
            self.saved_token = 0
        return f, g, inf

    def autotune(self, theta, kind="grad", batch=1, reps=3):
        """Choose the GEMM tile of each role at this model's block size by timing `batch`
        (<= 2d + 1) evaluations of `kind` at theta (rows of a batch x d array); returns the
        number of roles whose choice changed.  Synchronises."""
        th = self._theta(theta).reshape(-1, self.d)[:batch].contiguous()
        mode = MODE_GRAD if kind == "grad" else MODE_OBJECTIVE
        ws, nb = self.workspace(int(th.shape[0]), mode)
        changed = C.c_int32(0)
        check(lib().inla_autotune(self._h, C.c_void_p(th.data_ptr()), int(th.shape[0]), mode,
                                  int(reps), ws, nb, self._stream(), C.byref(changed)),
              "inla_autotune")
        self.saved_token = 0
        return int(changed.value)

    def fitting_batch(self, npts, mode, fraction=0.5):
        """The largest batch (<= npts) whose workspace fits in `fraction` of the free memory."""
        free, _ = torch.cuda.mem_get_info(self.device)
        for mb in range(npts, 0, -1):
            if self.workspace_bytes(mb, mode) <= fraction * free:
                return mb
        return 1

    def hessian(self, theta, h=5e-3, max_batch=None, f=None, g=None, H=None, info=None):
        """Posterior Hessian from 2d+1 exact gradients (Sec. III-D, Eq. 12), max_batch points per
        pass (default: as many as fit); H[:, j] is the central difference of the gradient along
        e_j (not symmetrised)."""
        th = self._theta(theta).reshape(self.d)
        d = self.d
        if max_batch is None:
            key = ("hessian_batch", d)
            if key not in self._ws:
                self._ws[key] = self.fitting_batch(2 * d + 1, MODE_GRAD)
            max_batch = self._ws[key]
        mb = min(int(max_batch), 2 * d + 1)
        f = f if f is not None else torch.empty(1, dtype=torch.float64, device=self.device)
        g = g if g is not None else torch.empty(d, dtype=torch.float64, device=self.device)
        H = H if H is not None else torch.empty((d, d), dtype=torch.float64, device=self.device)
        inf = info if info is not None else torch.empty(2 * d + 1, dtype=torch.int32,
                                                        device=self.device)
        ws, nb = self.workspace(mb, MODE_GRAD)
        # the library writes H column-major: the storage of H.T
        check(lib().inla_hessian(self._h, C.c_void_p(th.data_ptr()), float(h), mb,
                                 C.c_void_p(f.data_ptr()), C.c_void_p(g.data_ptr()),
                                 C.c_void_p(H.data_ptr()), C.c_void_p(inf.data_ptr()), ws, nb,
                                 self._stream()), "inla_hessian")
        self.saved_token = 0
        return f, g, H.T, inf

    def fd_hessian(self, theta, h=5e-3, max_batch=None, f=None, H=None, info=None):
        """Second-order central-difference Hessian over 2d^2+1 batched objective evaluations."""
        th = self._theta(theta).reshape(self.d)
        d = self.d
        npts = 2 * d * d + 1
        mb = npts if max_batch is None else min(int(max_batch), npts)
        f = f if f is not None else torch.empty(1, dtype=torch.float64, device=self.device)
        H = H if H is not None else torch.empty((d, d), dtype=torch.float64, device=self.device)
        inf = info if info is not None else torch.empty(npts, dtype=torch.int32, device=self.device)
        ws, nb = self.workspace(mb, MODE_OBJECTIVE)
        check(lib().inla_fd_hessian(self._h, C.c_void_p(th.data_ptr()), float(h), mb,
                                    C.c_void_p(f.data_ptr()), C.c_void_p(H.data_ptr()),
                                    C.c_void_p(inf.data_ptr()), ws, nb, self._stream()),
              "inla_fd_hessian")
        return f, H.T, inf


class BatchRunner:
    """f (kind="objective") or f and the exact gradient (kind="grad") at a fixed number of theta
    points per call: the first call captures one batched evaluation (every launch covers all
    points' chains) into a hipGraph, later calls copy the points in and replay it.  The runner
    owns its workspace: a replay runs no host code, so it must not write into a workspace that
    holds factors saved by InlaObjective.forward for a later backward."""

    def __init__(self, model, batch, kind="objective"):
        if kind not in ("objective", "grad"):
            raise ValueError("kind must be 'objective' or 'grad'")
        self.model, self.batch, self.kind = model, int(batch), kind
        dev, d = model.device, model.d
        self.theta = torch.zeros((self.batch, d), dtype=torch.float64, device=dev)
        self.f = torch.empty(self.batch, dtype=torch.float64, device=dev)
        self.info = torch.empty(self.batch, dtype=torch.int32, device=dev)
        self.g = (torch.empty((self.batch, d), dtype=torch.float64, device=dev)
                  if kind == "grad" else None)
        self._ws = model.new_workspace(self.batch, MODE_GRAD if kind == "grad" else MODE_OBJECTIVE)
        self._graph = None

    def _evaluate(self):
        if self.kind == "objective":
            self.model.objective(self.theta, out=self.f, info=self.info, ws=self._ws)
        else:
            self.model.grad_batched(self.theta, f=self.f, g=self.g, info=self.info, ws=self._ws)

    def __call__(self, theta):
        th = torch.as_tensor(theta, dtype=torch.float64, device=self.model.device)
        self.theta.copy_(th.reshape(self.batch, self.model.d))
        if self._graph is None:
            self._evaluate()  # workspaces are allocated outside the capture
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                self._evaluate()
            self._graph = graph
        self._graph.replay()
        if self.kind == "objective":
            return self.f, self.info
        return self.f, self.g, self.info


class InlaBatch:
    """An uneven batch of models (``inla_batch_create``): ``objective(theta)`` and
    ``grad(theta)`` evaluate every model at its own theta (row i of a count x d array) in one
    call; models with the same block size share every launch of the sweeps.  ``capture(kind)``
    records one call into a hipGraph whose ``replay`` re-evaluates at the points then held in
    ``self.theta``.  The models must outlive the batch."""

    def __init__(self, models):
        self.models = list(models)
        self.device = self.models[0].device
        self.count = len(self.models)
        self.d = self.models[0].d
        arr = (C.c_void_p * self.count)(*[m._h.value for m in self.models])
        h = C.c_void_p()
        dev_index = self.device.index if self.device.index is not None else torch.cuda.current_device()
        check(lib().inla_batch_create(context(dev_index), self.count, arr, C.byref(h)),
              "inla_batch_create")
        self._h = h
        self.groups = int(lib().inla_batch_groups(h))
        self._ws = {}
        dev = self.device
        self.theta = torch.zeros((self.count, self.d), dtype=torch.float64, device=dev)
        self.f = torch.empty(self.count, dtype=torch.float64, device=dev)
        self.g = torch.empty((self.count, self.d), dtype=torch.float64, device=dev)
        self.info = torch.empty(self.count, dtype=torch.int32, device=dev)
        self._graphs = {}

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().inla_batch_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def workspace_bytes(self, mode):
        return int(lib().inla_batch_workspace_bytes(self._h, mode))

    def _workspace(self, mode):
        if mode not in self._ws:
            nbytes = self.workspace_bytes(mode)
            if nbytes == 0:
                raise ValueError("invalid workspace request")
            buf = torch.empty(nbytes // 8 + 64, dtype=torch.float64, device=self.device)
            self._ws[mode] = (buf, nbytes)
        buf, nbytes = self._ws[mode]
        p = buf.data_ptr()
        return C.c_void_p(p + ((-p) % 256)), nbytes

    def _run(self, kind):
        ws, nb = self._workspace(MODE_GRAD if kind == "grad" else MODE_OBJECTIVE)
        stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        if kind == "grad":
            check(lib().inla_batch_grad(self._h, C.c_void_p(self.theta.data_ptr()),
                                        C.c_void_p(self.f.data_ptr()), C.c_void_p(self.g.data_ptr()),
                                        C.c_void_p(self.info.data_ptr()), ws, nb, stream),
                  "inla_batch_grad")
        else:
            check(lib().inla_batch_objective(self._h, C.c_void_p(self.theta.data_ptr()),
                                             C.c_void_p(self.f.data_ptr()),
                                             C.c_void_p(self.info.data_ptr()), ws, nb, stream),
                  "inla_batch_objective")

    def _set(self, theta):
        if theta is not None:
            th = torch.as_tensor(theta, dtype=torch.float64, device=self.device)
            self.theta.copy_(th.reshape(self.count, self.d))

    def objective(self, theta=None):
        """f of every model at its theta: (f, info), views of the batch's own buffers."""
        self._set(theta)
        self._run("objective")
        return self.f, self.info

    def grad(self, theta=None):
        """f and the exact gradient of every model: (f, grad, info), the batch's own buffers."""
        self._set(theta)
        self._run("grad")
        return self.f, self.g, self.info

    def autotune(self, kind="grad", reps=2, theta=None):
        """Choose the GEMM tile of each role for every block size of the batch by timing that
        group's part of a call of `kind` at the points in self.theta (or `theta`); returns the
        number of (block size, role) choices that changed.  Synchronises; graphs captured
        before keep their old choices, so they are dropped."""
        self._set(theta)
        mode = MODE_GRAD if kind == "grad" else MODE_OBJECTIVE
        ws, nb = self._workspace(mode)
        changed = C.c_int32(0)
        check(lib().inla_batch_autotune(self._h, C.c_void_p(self.theta.data_ptr()), mode,
                                        int(reps), ws, nb,
                                        C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                        C.byref(changed)), "inla_batch_autotune")
        self._graphs = {}
        return int(changed.value)

    def capture(self, kind):
        """Record one call of `kind` ("objective" or "grad") into a hipGraph (once)."""
        if kind not in self._graphs:
            self._run(kind)  # workspaces are allocated outside the capture
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                self._run(kind)
            self._graphs[kind] = graph
        return self._graphs[kind]

    def replay(self, kind, theta=None):
        self._set(theta)
        self.capture(kind).replay()
        if kind == "grad":
            return self.f, self.g, self.info
        return self.f, self.info


def fd_grad(model, theta, h=1e-3, max_batch=None):
    """The GPU's (2d+1)-point central-difference gradient (Sec. II-D, Eq. 2): (f, grad, info)."""
    return model.fd_grad(theta, h=h, max_batch=max_batch)


def hessian(model, theta, h=5e-3, max_batch=None):
    """The posterior Hessian from exact gradients (Sec. III-D, Eq. 12): (f, grad, H, info)."""
    return model.hessian(theta, h=h, max_batch=max_batch)


class InlaObjective(torch.autograd.Function):
    """f = InlaObjective.apply(theta, model); f.backward() fills theta.grad.

    The forward pass stores the factors of Qc and Qp in the model's gradient workspace; the
    backward pass reuses them when no other forward pass on the model came in between, and
    recomputes them otherwise.  The backward itself is not differentiable."""

    @staticmethod
    def forward(ctx, theta, model):
        f, info, token = model.forward_saved(theta.detach())
        ctx.model = model
        ctx.token = token
        ctx.save_for_backward(theta.detach())
        return f.reshape(())

    @staticmethod
    @once_differentiable
    def backward(ctx, grad_out):
        (theta,) = ctx.saved_tensors
        model = ctx.model
        reuse = model.saved_token == ctx.token
        _, g, _ = model.grad(theta, reuse=reuse)
        return grad_out * g, None
