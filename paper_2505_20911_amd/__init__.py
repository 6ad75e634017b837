"""MI355X-native explicit finite-difference time step of the compressible
Navier-Stokes equations (Taylor-Green vortex), after "Reduced and mixed
precision turbulent flow simulations using explicit finite difference
schemes" (arXiv 2505.20911).

The computation lives in libtgv.so (HIP kernels for gfx950 behind the C-ABI of
include/tgv.h); this package holds its ctypes binding (``tgv``), a time-stepping
driver (``solver``), binomial checkpointing (``revolve``) and the
torch.autograd wrapper of the discrete adjoint (``adjoint``).
"""
from . import tgv  # noqa: F401
from .tgv import PRESETS, Params, Prec, TgvError  # noqa: F401
