"""MI355X-native Tucker-compressed VSIE coupling-matrix products.

``lib``  ctypes binding of libtuckvsie (include/tuckvsie.h), same names.
``ops``  torch-facing wrappers: ``TuckerPlan`` (device plan with matvec /
         rmatvec on torch complex64 tensors) and ``TuckerMatvec``, a
         ``torch.autograd.Function`` whose backward is the adjoint kernel.

Neither is imported here so that building the library needs no GPU.
"""
