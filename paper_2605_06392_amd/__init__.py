"""MI355X (gfx950) implementation of the hot path of AD-enabled INLA over
block-tridiagonal-arrowhead precision matrices (arXiv 2605.06392).

The computation lives in ``libadelia.so`` (HIP kernels behind a C ABI, see include/adelia.h);
this package only marshals arguments.  Submodules:

* ``bta``  -- bta_factor / bta_logdet / bta_solve / bta_selinv and a batched FP64 GEMM;
* ``inla`` -- InlaModel, objective, gradient, GPU finite differences, the posterior Hessian,
  the autograd Function, BatchRunner (graph-captured batched evaluation) and InlaBatch (an
  uneven batch of models); the package re-exports InlaModel, InlaObjective, BatchRunner,
  InlaBatch, fd_grad and hessian.
"""
__all__ = ["bta", "inla", "InlaModel", "InlaObjective", "BatchRunner", "InlaBatch", "fd_grad",
           "hessian"]

_FROM_INLA = ("InlaModel", "InlaObjective", "BatchRunner", "InlaBatch", "fd_grad", "hessian")


def __getattr__(name):
    import importlib
    if name in ("bta", "inla"):
        return importlib.import_module(f".{name}", __name__)
    if name in _FROM_INLA:
        return getattr(importlib.import_module(".inla", __name__), name)
    raise AttributeError(name)
