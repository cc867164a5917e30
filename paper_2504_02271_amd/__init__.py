"""htri: hyper-triangle counting on AMD MI355X (gfx950).

The computation lives in the HIP library ``libhtri.so`` (sources in
``csrc/``, C ABI in ``include/htri.h``); :mod:`paper_2504_02271_amd.htri` is
its ctypes binding and :mod:`paper_2504_02271_amd.synth` draws seeded
synthetic inputs.  Submodules are imported on demand so that input
generation works without the library.
"""
__all__ = ["htri", "synth", "build"]
