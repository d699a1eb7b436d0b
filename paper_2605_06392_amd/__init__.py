"""MI355X (gfx950) implementation of the hot path of AD-enabled INLA over
block-tridiagonal-arrowhead precision matrices (arXiv 2605.06392).

The computation lives in ``libadelia.so`` (HIP kernels behind a C ABI, see include/adelia.h);
this package only marshals arguments.  Submodules:

* ``bta``  -- bta_factor / bta_logdet / bta_solve / bta_selinv and a batched FP64 GEMM;
* ``inla`` -- InlaModel, objective, gradient, GPU finite differences, the autograd Function.
"""
__all__ = ["bta", "inla"]


def __getattr__(name):
    if name in ("bta", "inla"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
