"""CSPH-TVD (arXiv:1912.04855) on MI355X: Python binding of the HIP library.

``Sim`` wraps one simulation behind the C ABI of ``include/csph.h``;
``problems`` describes the synthetic workloads.  Importing the package does not
load the library; creating a ``Sim`` does, and fails if it has not been built.
"""
from . import problems  # noqa: F401

__all__ = ["Sim", "Batch", "from_problem", "problems", "required_bytes"]


def __getattr__(name):
    if name in ("Sim", "Batch", "from_problem", "required_bytes", "make_desc"):
        from . import sim
        return getattr(sim, name)
    raise AttributeError(name)
