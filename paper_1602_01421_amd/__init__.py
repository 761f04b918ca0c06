"""MI355X block Krylov-Schur hot path: pattern SpMM, FP64 Gram/update, driver.

The compute lives in libfe.so (HIP for gfx950, C ABI in include/fe.h); this
package is its ctypes binding.  There is no CPU fallback: if the library is
missing or no GPU is present, the entry points raise.
"""
from .fe import (  # noqa: F401
    EXPORTED, FE_BF16, FE_DEDUPE, FE_DROP_SELF, FE_EBREAKDOWN, FE_EDEVICE, FE_EINVAL, FE_ENOCONV,
    FE_ENOMEM, FE_EUNSUPPORTED, FE_F32, FE_F64, FE_GRAPH_DEFAULT, FE_OK, FE_RELABEL_BY_DEGREE,
    FE_SYMMETRIZE, GNN_SHAPES, LIB_PATH, Csr, FeError, Gnn, KsResult, gnn_flatten, gnn_unflatten, fe_block_update, fe_block_update_gram,
    fe_csr_build,
    fe_csr_from_csr, fe_dense_symeig, fe_gram, fe_gram_noalloc, fe_krylov_schur, fe_ks_workspace_bytes, fe_gather_rows, fe_spmm, fe_spmm_gather_bound, fe_svds, lib,
    torch_dtype,
    version)
