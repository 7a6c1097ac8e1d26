"""tn3d: coset probabilities of detector error models by boundary-sweep
contraction of layered 3D tensor networks on AMD Instinct MI355X (gfx950).

The compute path is the HIP library libtn3d.so (C-ABI, include/tn3d.h);
`tn3d` holds a thin ctypes binding with the same entry points.
"""

from .tn3d import (  # noqa: F401
    PREC_FP32,
    PREC_FP64,
    FLAG_NEAR_TIE,
    FLAG_NO_CONVERGE,
    FLAG_NUMERIC,
    FLAG_TRUNC_CLUSTER,
    Context,
    Net,
    Params,
    contract_cosets,
    decode,
    exported_symbols,
    load_library,
)
