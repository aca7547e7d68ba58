"""B-char transfer build and apply on AMD MI355X (gfx950).

The compute path is the C-ABI shared library built from ``csrc/`` (HIP
kernels for gfx950); ``bchar`` is its thin ctypes binding.  ``inputs``
generates seeded synthetic problems.  Nothing is imported eagerly so that
``inputs`` works on machines without a GPU.
"""

__all__ = ["bchar", "inputs"]
