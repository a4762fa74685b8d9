"""Hierarchical multicontinuum homogenization cell solves on MI355X (gfx950).

The compute path is the C-ABI library ``libmch.so`` (HIP kernels + host
runtime) built from ``csrc/``; ``mch`` is its thin ctypes binding and
``autograd`` wraps forward/backward in a ``torch.autograd.Function``.
Submodules are imported on demand so that ``workloads`` (seeded inputs only)
stays importable without the library.
"""
__all__ = ["workloads", "mch", "autograd", "build"]
