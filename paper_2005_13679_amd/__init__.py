"""MI355X-native bosonic multiconfigurational operators (arXiv:2005.13679).

Fock-space hashing, single/double jump maps, the many-body Hamiltonian apply
H.C and the reduced density matrices, as hand-written HIP kernels for gfx950
behind the C ABI of ``include/mc.h``.  This package is the thin Python
binding: torch provides device memory and streams, the library does all the
arithmetic.  There is no CPU fallback.
"""

from ._lib import MCError, LIB_PATH
from .api import (
    DirectSpace,
    Tables,
    apply_H,
    apply_H_adjoint,
    apply_H_direct,
    apply_H_sparse,
    apply_stream_columns,
    build_tables,
    choose_double_jumps,
    dim,
    hash_batch,
    hash_occ,
    is_hermitian,
    rho1,
    rho2,
    t2_lookup,
    tables_bytes,
    tables_size,
    unhash,
    unhash_batch,
    workspace_size,
    zaxpby,
    zdotc,
)
from .autograd import Energy, energy
from .batch import Batch, BatchedLanczos, batched_lanczos
from .propagate import SILStepper, sil_step

__all__ = [
    "MCError", "LIB_PATH", "SILStepper", "sil_step", "Batch", "BatchedLanczos", "batched_lanczos", "Energy", "DirectSpace", "Tables", "apply_H", "apply_H_adjoint", "apply_H_direct", "apply_H_sparse",
    "apply_stream_columns", "energy", "build_tables", "dim", "hash_batch",
    "hash_occ", "rho1", "rho2", "t2_lookup", "tables_size", "unhash", "unhash_batch",
    "workspace_size", "zaxpby", "zdotc", "choose_double_jumps", "is_hermitian", "tables_bytes",
]
