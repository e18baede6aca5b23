"""Iterative Vecchia-Laplace inference for latent Gaussian processes on one
AMD MI355X (gfx950): hand-written HIP kernels behind the C ABI in
include/vl.h, with a thin ctypes binding (vl.py)."""
from .vl import *  # noqa: F401,F403
from .vl import VecchiaLaplace, lib  # noqa: F401
