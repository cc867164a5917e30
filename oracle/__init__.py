"""CPU oracle for hyper-triangle counting -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
library in ``paper_2504_02271_amd/csrc``.
"""
