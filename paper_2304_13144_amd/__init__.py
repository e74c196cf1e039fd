"""MI355X (gfx950) Moment Tensor Potential hot path (MLIP-3, arXiv 2304.13144).

The HIP library ``libmtp.so`` (C ABI in include/mtp.h) does all the work;
``api`` marshals PyTorch device tensors into it.  ``synth`` holds the seeded
synthetic workloads.
"""
from ._lib import MtpError, lib  # noqa: F401
