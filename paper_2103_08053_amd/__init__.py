"""Exact triangle counting on MI355X by vertex-centric hashing (TRUST method).

The computation lives in the HIP library ``libtrust_tc.so`` (C ABI in
``include/trust_tc.h``); :mod:`.tc` is its ctypes binding.
"""
from .tc import (Batch, Context, Graph, GraphInfo, Params, RangeError, TCError, count, default_context,  # noqa: F401
                 load_library)
