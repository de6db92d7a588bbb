"""MI355X-native MBE-FCI hot path (Eriksen & Gauss, MBE-FCI II).

The computation lives in libmbefci.so (HIP for gfx950 + host C++), exposed by
the C ABI in include/mbefci.h; this package only marshals arguments.
"""
from .api import (Context, MBEFCIError, Order, Result, ResultHandle, default_options,  # noqa: F401
                  string_tables, workspace, TUPLE_OK, TUPLE_MAXITER, TUPLE_NONFINITE, TUPLE_STALLED,
                  TUPLE_PENDING)

__all__ = ["Context", "MBEFCIError", "Order", "Result", "default_options", "string_tables", "workspace"]
