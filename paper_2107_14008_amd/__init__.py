"""Short-range PM-FMM gravity on MI355X (gfx950).

The compute path lives in libpmfmm.so (HIP kernels + host planner behind the
C ABI of include/pmfmm.h).  ``binding`` marshals arguments to it, ``api``
offers torch-facing helpers, ``inputs`` draws seeded synthetic particle sets.
Submodules are imported lazily so that ``inputs`` can be used without the
built library.
"""

__all__ = ["binding", "api", "inputs", "build"]
