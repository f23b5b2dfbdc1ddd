"""MI355X (gfx950) solver for the Crank-Nicolson finite-volume scheme of the
conservative space-fractional diffusion equation with the sine-transform
preconditioner (arXiv 2511.21198).

The solver lives in ``libfsd.so`` (HIP, C ABI in ``include/fsd.h``);
``paper_2511_21198_amd.solver.Problem`` is a thin PyTorch front end.
Importing the front end loads the library and fails if it is not built.
"""

__all__ = ["Problem"]


def __getattr__(name):
    if name == "Problem":
        from .solver import Problem
        return Problem
    raise AttributeError(name)
