"""MI355X-native U(1)xU(1) multitension-string lattice update (arXiv:2208.01525).

The implementation is the HIP library libmts.so (C ABI in include/mts.h);
`paper_2208_01525_amd.mts` is its thin Python binding.
"""
from .mts import Batch, Lattice, MtsError, load, make_params, state_bytes  # noqa: F401
