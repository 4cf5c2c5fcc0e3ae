"""Exact higher-order U-statistics on MI355X (gfx950).

The engine lives in ``libustat.so`` (HIP kernels and a C ABI declared in
``include/ustat.h``); ``ustat`` is its thin Python binding.  Importing this
package loads nothing; ``from paper_2508_12627_amd import ustat`` loads the
library and fails loudly if it has not been built.
"""
