"""Space-time multigrid for the heat equation on AMD MI355X (gfx950).

The solver lives in a HIP shared library with a C ABI (include/st_mg.h); the
module `stmg` is its thin ctypes binding and `autograd` wraps the forward
solve and the adjoint solve as a torch.autograd.Function.  Submodules are
imported lazily so that `workloads` (seeded inputs) can be used without the
library or a GPU.
"""
__all__ = ["stmg", "autograd", "workloads"]
