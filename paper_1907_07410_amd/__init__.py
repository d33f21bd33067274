"""bmf: block-parallel biased-SVD matrix factorisation on MI355X (gfx950).

The compute lives in ``libbmf.so`` (HIP kernels behind a C ABI declared in
``include/bmf.h``); ``paper_1907_07410_amd.binding`` marshals arguments to it.
"""
