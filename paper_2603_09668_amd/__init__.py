"""MI355X-native DiffWind simulation step: MLS-MPM substep coupled to a D3Q19 LBM.

The compute path is ``libdiffwind.so`` (hand-written HIP kernels for gfx950
behind a C ABI, declared in ``include/diffwind.h``).  ``api`` binds those
entry points with the same names; ``autograd`` wraps them in
``torch.autograd.Function``s and builds checkpointed rollouts; ``surrogate``
holds the BF16 convolutional wind surrogate.  Importing this package does not
load the library; the first call does, and raises if it is missing.
"""
__all__ = ["api", "autograd", "scenes", "surrogate"]
