"""MI355X marching-on-in-time solver for the qHP TD-PMCHWT formulation.

Thin Python binding over libmot.so (C ABI in include/mot.h): argument
marshalling only; every step of the solver runs in HIP kernels.  PyTorch is
used only for device buffers and the current stream when outputs are
requested on the device.
"""
from .solver import Solver, MotError, default_options, footprint, run_batch  # noqa: F401
from . import _lib  # noqa: F401
