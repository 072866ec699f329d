"""MI355X (gfx950) multilevel ELM-FBPINN least-squares library: Python binding of libelmfb.so.

The compute path is the C-ABI shared library built from csrc/ (see include/elmfb.h); this
package only marshals arguments.  It fails loudly when the library is missing.
"""
from .elmfb import (  # noqa: F401
    BF16,
    FP16,
    Batch,
    CGLS,
    FP32,
    FP64,
    LSQR,
    MLP,
    ElmfbError,
    Problem,
    define_problem,
    desc_from_spec,
    load_library,
    make_desc,
)
