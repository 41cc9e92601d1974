"""The matrix-core far kernel (two real-form GEMMs per displacement run) against
the vector-unit far kernel and the oracle's retrieval product, through the C
ABI.  The kernel is chosen per (store, batch) by the autotuner;
R3M_FAR_KERNEL restricts the choice so that each kernel can be checked.

Tolerances: both kernels run the same FP32 arithmetic on the same factors in a
different order, so they agree to the FP32 rounding of an n_a-term sum
(1e-6 relative); against the oracle's complex128 product on the decoded
factors, as for any complex64 store (1e-6)."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_common import FREQ, rel_l2, rel_max, unit  # noqa: E402
from workloads import codebooks as cb  # noqa: E402

DEV = "cuda:0"


def _matvec(r3m, kernel, store, batch, x, vt):
    os.environ["R3M_FAR_KERNEL"] = kernel
    try:
        ctx = r3m.Context(0)
        y = torch.zeros_like(x)
        work = torch.empty(r3m.matvec_work_bytes(ctx, store, batch, vt), dtype=torch.uint8, device=DEV)
        r3m.r3m_retrieved_matvec(ctx, store, batch, vt, x, y, work)
        y2 = torch.zeros_like(x)
        r3m.r3m_retrieved_matvec(ctx, store, batch, vt, x, y2, work, index_ready=True)
        torch.cuda.synchronize()
        ctx.close()
    finally:
        del os.environ["R3M_FAR_KERNEL"]
    assert torch.equal(y, y2), "matvec not bitwise repeatable"
    return y.cpu().numpy()


@pytest.mark.parametrize("bits,far,rhs_per_book", [(2, "c64", 1), (1, "bf16x2", 4), (1, "f16x2", 3), (1, "c64", 2)])
def test_mfma_far_kernel_matches_valu(bits, far, rhs_per_book):
    from paper_2112_05082_amd import pipeline, r3m
    ctx = r3m.Context(0)
    geom = r3m.UnitGeom.from_macro(unit(bits), FREQ, 1)
    L = 12
    fd = {"c64": r3m.C64, "bf16x2": r3m.BF16X2, "f16x2": r3m.F16X2}[far]
    store = pipeline.compressed_store(ctx, geom, L, 2, r3m.C64, fd, 1e-4, 40, DEV)
    # ragged codebooks: 12x12, 9x9, 5x5, 1x1 (several right-hand sides each)
    books = [cb.uniform(s, 2 ** bits, 10 + s) for s in (12, 9, 5, 1)]
    batch = r3m.Batch.from_codebooks(books, [12, 9, 5, 1], DEV, repeat=rhs_per_book)
    N = batch.total_units * unit(bits).n_a
    g = torch.Generator(device=DEV).manual_seed(7)
    x = torch.complex(torch.randn(N, generator=g, device=DEV, dtype=torch.float64),
                      torch.randn(N, generator=g, device=DEV, dtype=torch.float64))
    ya = _matvec(r3m, "valu", store, batch, x, r3m.C128)
    yb = _matvec(r3m, "mfma", store, batch, x, r3m.C128)
    err = rel_max(yb, ya)
    print(f"far mfma vs valu bits={bits} far={far} rhs/book={rhs_per_book}: {err:.2e}", flush=True)
    assert err <= 1e-6, err
    ctx.close()


def test_mfma_far_kernel_vs_oracle_product():
    """1-bit 6x6 and 4x3 arrays, complex64 factors: the matrix-core far kernel
    against the oracle's block retrieval product with the same (decoded) near
    blocks and far factors."""
    from oracle import retrieval
    from paper_2112_05082_amd import pipeline, r3m
    ctx = r3m.Context(0)
    u = unit(1)
    geom = r3m.UnitGeom.from_macro(u, FREQ, 1)
    L, D = 6, 5
    store = pipeline.compressed_store(ctx, geom, L, 1, r3m.C64, r3m.C64, 1e-4, 40, DEV)
    # the store's blocks as complex128 matrices Z(d) = near, or U V^H
    near = store.near.cpu().numpy().astype(np.complex128)
    n_far = r3m.far_count(D, D, 1)
    head = ((n_far * 4 + 255) // 256) * 256
    raw = store.far.cpu().numpy()
    R = store.max_rank
    fac = raw[head: head + n_far * 2 * R * u.n * 8].view(np.complex64).astype(np.complex128)
    fac = fac.reshape(n_far, 2, R, u.n)
    blocks = np.zeros(((2 * D + 1) ** 2, u.n, u.n), np.complex128)
    fi = 0
    for dy in range(-D, D + 1):
        for dx in range(-D, D + 1):
            slot = (dy + D) * (2 * D + 1) + dx + D
            if max(abs(dx), abs(dy)) <= 1:
                blocks[slot] = near[(dy + 1) * 3 + dx + 1]
            else:
                U, V = fac[fi, 0], fac[fi, 1]
                blocks[slot] = U.T @ V.conj()
                fi += 1
    off = np.arange(0, u.n + 1, u.n_a)
    codes = [cb.bernoulli(6, 3), cb.bernoulli(4, 4)]
    sizes = [6, 4]
    uoff = [0, 36]
    states = torch.from_numpy(np.concatenate(codes).astype(np.uint8)).to(DEV)
    batch = r3m.Batch([(s, s) for s in sizes], uoff, uoff, states)
    N = 52 * u.n_a
    xs = cb.random_complex(N, 5)
    x = torch.from_numpy(xs).to(DEV)
    y = _matvec(r3m, "mfma", store, batch, x, r3m.C128)
    for b, (Ls, code) in enumerate(zip(sizes, codes)):
        sl = slice(uoff[b] * u.n_a, (uoff[b] + Ls * Ls) * u.n_a)
        ref = retrieval.retrieved_matvec(blocks, D, D, off, code, Ls, xs[sl])
        err = rel_l2(y[sl], ref)
        print(f"far mfma vs oracle product array {Ls}x{Ls}: {err:.2e}", flush=True)
        assert err <= 1e-6, err
    ctx.close()
