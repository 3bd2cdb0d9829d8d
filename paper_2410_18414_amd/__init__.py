"""MI355X-native gauge-conserving PIC step (arXiv 2410.18414).

The compute path is the C-ABI library ``libpic.so`` (hand-written HIP for
gfx950) declared in ``include/pic.h``; :mod:`paper_2410_18414_amd.pic` is its
thin ctypes binding.  Importing this package loads nothing.
"""
