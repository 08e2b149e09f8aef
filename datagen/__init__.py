"""Seeded synthetic sparse tensors.

The one module that both the CPU oracle (tests) and the HIP path (tests, bench)
consume.  It holds none of the transposition's arithmetic: it draws random
coordinates and values, removes duplicated coordinates where asked, and lists
the nonzeros in the requested input order.
"""
from .tensors import (CONFIGS, SynthTensor, make_tensor, config_tensor, zipf_alias)  # noqa: F401
