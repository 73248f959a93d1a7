"""MI355X-native THC second-order-exchange (SOX) self-energy.

The compute path is the C-ABI library ``libsox.so`` (hand-written HIP
kernels for gfx950); :mod:`.binding` marshals arguments to it and
:mod:`.autograd` wraps the forward and adjoint entry points for PyTorch.
:mod:`.synth` draws seeded synthetic inputs.  Importing the package does not
load the library; the first call into :mod:`.binding` does, and raises if it
is missing.
"""
__all__ = ["binding", "synth"]
