"""Device block stores and batches built through the C ABI only.

The global matrix of the macro-unit array (Sec. III-A) is filled once as
unique displacement blocks (Sec. III-C, finest patterns), its far blocks are
compressed, and the resulting store serves every codebook of a batch.
"""
from __future__ import annotations

import torch

from . import r3m

DT = {"c128": r3m.C128, "c64": r3m.C64}
TORCH_DT = {r3m.C128: torch.complex128, r3m.C64: torch.complex64}


def empty_bytes(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 16), dtype=torch.uint8, device=device)


def fill_blocks(ctx, geom, D: int, dtype: int, device) -> torch.Tensor:
    """All (2D+1)^2 blocks as a complex tensor [slot][n][n]."""
    n = geom.n
    out = torch.empty(((2 * D + 1) ** 2, n, n), dtype=TORCH_DT[dtype], device=device)
    r3m.r3m_fill_unique_blocks(ctx, geom, D, D, dtype, out)
    return out


def dense_store(ctx, geom, L: int, dtype: int, device) -> r3m.Store:
    """Every displacement block dense (plain path)."""
    D = L - 1
    blocks = fill_blocks(ctx, geom, D, dtype, device)
    return r3m.Store(geom.n, geom.n_states, D, D, D, dtype, blocks)


def compressed_store(ctx, geom, L: int, near_radius: int, near_dtype: int, far_dtype: int, tol: float,
                     max_rank: int, device, dense_c128: torch.Tensor | None = None,
                     work_blocks: int = 2048) -> r3m.Store:
    """Dense near blocks (Chebyshev <= near_radius) plus ACA far factors."""
    D = L - 1
    n = geom.n
    nr = min(near_radius, D)
    near = fill_blocks(ctx, geom, nr, near_dtype, device)
    if nr >= D:
        return r3m.Store(n, geom.n_states, D, D, nr, near_dtype, near)
    own_dense = dense_c128 is None
    if own_dense:
        dense_c128 = fill_blocks(ctx, geom, D, r3m.C128, device)
    n_far = r3m.far_count(D, D, nr)
    far = empty_bytes(r3m.far_bytes(n, n_far, max_rank, far_dtype), device)
    work = empty_bytes(r3m.compress_work_bytes(n, max_rank, min(work_blocks, n_far)), device)
    ranks, err = r3m.r3m_compress_far(ctx, dense_c128, n, D, D, nr, tol, max_rank, far_dtype, far, work)
    del work
    if own_dense:
        del dense_c128
    return r3m.Store(n, geom.n_states, D, D, nr, near_dtype, near, far_dtype, far, max_rank, ranks, err)


def spectral_store(ctx, geom, L: int, near_radius: int, dtype: int, device,
                   dense_c128: torch.Tensor | None = None) -> r3m.Store:
    """Block spectra of every displacement (the whole product by FFT) plus the
    dense near blocks (Chebyshev <= near_radius) the preconditioner reads.
    dtype: r3m.C64 or r3m.C128 (spectra and near blocks alike)."""
    D = L - 1
    n = geom.n
    nr = min(near_radius, D)
    near = fill_blocks(ctx, geom, nr, dtype, device)
    own_dense = dense_c128 is None
    if own_dense:
        dense_c128 = fill_blocks(ctx, geom, D, r3m.C128, device)
    sd = r3m.SPEC_C64 if dtype == r3m.C64 else r3m.SPEC_C128
    spec = empty_bytes(r3m.spectral_bytes(n, D, D, sd), device)
    r3m.r3m_build_spectral(ctx, dense_c128, n, D, D, sd, spec)
    if own_dense:
        del dense_c128
    ext = None
    if getattr(geom, "common_ext", None) is not None:  # shared bases of a connected geometry
        ext = torch.from_numpy(geom.common_ext).to(device)
    return r3m.Store(n, geom.n_states, D, D, nr, dtype, near, sd, spec, common_ext=ext)
