"""MI355X (gfx950) hot path of QML power-spectrum estimation and the pixel-space likelihood.

The computation lives in ``libcf.so`` (hand-written HIP kernels behind the C ABI of
``include/cf.h``); ``paper_2605_21149_amd.cf`` is a thin ctypes binding with the same entry
points.  ``paper_2605_21149_amd.inputs`` synthesises the seeded workloads.
"""
