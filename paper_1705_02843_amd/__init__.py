"""MI355X (gfx950) Block-Parallel IDA* for the sliding-tile puzzle.

The search runs in hand-written HIP kernels behind the C ABI declared in
``include/bpida.h``; ``paper_1705_02843_amd.bpida`` is the ctypes binding.
Importing this package loads nothing; importing ``bpida`` loads the library.
"""
