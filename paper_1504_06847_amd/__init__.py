"""MI355X (gfx950) implementation of the wide-band ADMM image reconstruction of
Ferrari et al., arXiv 1504.06847: hand-written HIP kernels behind the C ABI of
include/muffin.h, with this thin Python binding on top.

Importing the package does not touch the GPU; ``lib.load()`` (called by
``Solver``) loads libmuffin.so and fails loudly when it is not built.
"""
from . import lib
from .autograd import MuffinUnroll
from .batch import Batch
from .solver import PAPER_DICTIONARY, Solver
from .vis import VisSolver

__all__ = ["lib", "Batch", "MuffinUnroll", "PAPER_DICTIONARY", "Solver", "VisSolver"]
