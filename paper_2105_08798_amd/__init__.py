"""MI355X-native line-periodic FBC pad update (HIP library + ctypes binding).

The compute path is libfbc.so (include/fbc.h); this package only marshals arguments.
"""
from .fbc import (FBC, MLP, FORMS, RELAX_OUT_DOUBLES, FbcError, HMatrix, PeriodicGreen,  # noqa: F401
                  Surrogate, load_library, parse_relax_out, probe_read)
