"""MI355X-native line-periodic FBC pad update (HIP library + ctypes binding).

The compute path is libfbc.so (include/fbc.h); this package only marshals arguments.
"""
from .fbc import FBC, FbcError, FORMS, RELAX_OUT_DOUBLES, load_library, parse_relax_out  # noqa: F401
