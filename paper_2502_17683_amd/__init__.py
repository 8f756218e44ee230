"""Matrix-free THC-based CP-ALS on MI355X (gfx950).

The CP-ALS of an order-4 tensor given in THC form,
G[p,q,r,s] = sum_PQ X0[p,P] X1[q,P] Z[P,Q] X2[r,Q] X3[s,Q], runs entirely in
the HIP library libthccp.so (include/thccp.h); this package only marshals
arguments and owns the torch tensors that back the library's workspace.
"""
from ._lib import CpdError, load, LIB_PATH  # noqa: F401
from .cpd import CPD, CPDBatch, lt_scale_rows, test_gemm, test_solve, test_gemm_split, df_to_thc  # noqa: F401
from .cpd import test_flow_spin_limit  # noqa: F401
from .cpd import test_bwd_form  # noqa: F401
from .cpd import test_split_force  # noqa: F401
from .lt import (lt_batch_problems, lt_exchange, lt_exchange_workspace_bytes, lt_mp2,  # noqa: F401
                 lt_mp2_workspace_bytes)
from .warmstart import (WarmStartMLP, ws_features, ws_features_noalloc, ws_select_init, ws_labels, ws_init,  # noqa: F401
                        training_set)
