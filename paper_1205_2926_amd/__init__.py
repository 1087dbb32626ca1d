"""Lazy-butterfly number-theoretic transforms on AMD MI355X (gfx950).

The compute path is the C-ABI library built from ``csrc/`` (hand-written HIP
kernels); ``hntt`` is its thin ctypes binding.  Importing this package does
not load the library: ``from paper_1205_2926_amd import hntt`` does.
"""
