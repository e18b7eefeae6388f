"""Perturbation-induced static pivoting on MI355X (gfx950), FP64.

Submodules:
  workloads -- seeded synthetic power-flow Jacobians and right-hand sides
  psp       -- binding over the C-ABI library libpsp.so (HIP kernels)
  autograd  -- torch.autograd.Function over the adjoint entry points
The binding is imported on first use so that input generation does not load
the GPU library.
"""
__all__ = ["workloads", "psp"]


def __getattr__(name):
    if name in ("psp", "autograd", "workloads"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
