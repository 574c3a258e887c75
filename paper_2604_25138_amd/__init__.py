"""MI355X (gfx950) LAKER solve path: fused attention-kernel products, shrinkage-CCCP
preconditioner fit and PCG in hand-written HIP, behind the C ABI of include/laker.h.

The binding lives in ``paper_2604_25138_amd.laker`` and loads ``liblaker.so``
lazily; importing the package does not touch the GPU.
"""
