"""Split far-factor formats (BF16X2, F16X2) against the complex128 factors of
the same ACA, the retrieval product on the decoded factors, and a mixed solve
with FP64 refinement.

Format: each complex entry is {re_hi | im_hi << 16, re_lo | im_lo << 16} with
hi = RNE(v), lo = RNE(v - hi) in the 16-bit type; F16X2 columns are scaled by
2^-e (2^e >= the column's largest real or imaginary magnitude) and the scales
2^e follow the factors.  The decoding below is that definition written out on
the host; the retrieval product is the oracle's.

Tolerances:
  * decoded BF16X2 entry vs complex128: 2^-16 of the column's largest
    magnitude (8 + 8 significant bits, then the FP32 rounding of v);
  * decoded F16X2 entry: 2^-20 of the column's largest magnitude;
  * matvec on split factors vs the retrieval product on the decoded factors:
    1e-6 (FP32 arithmetic, as for complex64);
  * refined mixed solve (split far factors, FP64 refinement residual on the
    complex128 store) vs the FP64 solve: residual 1e-6, RCS 1e-6.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_common import FREQ, rel_l2, rel_max, unit  # noqa: E402
from oracle import retrieval  # noqa: E402
from workloads import codebooks as cb  # noqa: E402

DEV = "cuda:0"
L = 8
D = L - 1
NR = 2


@pytest.fixture(scope="module")
def stores():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_05082_amd import pipeline, r3m
    r3m.load()
    ctx = r3m.Context(0)
    geom = r3m.UnitGeom.from_macro(unit(2), FREQ, 1)
    dense = pipeline.fill_blocks(ctx, geom, D, r3m.C128, DEV)
    out = {"ctx": ctx, "geom": geom, "r3m": r3m}
    for name, fd, nd in (("c128", r3m.C128, r3m.C128), ("c64", r3m.C64, r3m.C64), ("bf16x2", r3m.BF16X2, r3m.C64),
                         ("f16x2", r3m.F16X2, r3m.C64)):
        out[name] = pipeline.compressed_store(ctx, geom, L, NR, nd, fd, 1e-4, 40, DEV, dense_c128=dense)
    yield out
    ctx.close()


def decode(r3m, store):
    """Far factors U, V [f][n][max_rank] (complex128) of a store."""
    n_far = r3m.far_count(store.Dx, store.Dy, store.near_radius)
    head = ((n_far * 4 + 255) // 256) * 256
    raw = store.far.cpu().numpy()
    n, R = store.n, store.max_rank
    if store.far_dtype in (r3m.C128, r3m.C64):
        es = 16 if store.far_dtype == r3m.C128 else 8
        body = raw[head: head + n_far * 2 * R * n * es]
        arr = body.view(np.complex128 if es == 16 else np.complex64).astype(np.complex128)
    else:
        nb = n_far * 2 * R * n * 8
        w = raw[head: head + nb].view(np.uint32).reshape(-1, 2)

        def half(bits):
            return bits.astype(np.uint16).view(np.float16).astype(np.float64)

        def bf(bits):
            return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)

        f = bf if store.far_dtype == r3m.BF16X2 else half
        re = f(w[:, 0] & 0xFFFF) + f(w[:, 1] & 0xFFFF)
        im = f(w[:, 0] >> 16) + f(w[:, 1] >> 16)
        arr = re + 1j * im
        if store.far_dtype == r3m.F16X2:
            so = head + ((nb + 255) // 256) * 256
            sc = raw[so: so + n_far * 2 * R * 4].view(np.float32).astype(np.float64)
            arr = (arr.reshape(n_far * 2 * R, n) * sc[:, None]).reshape(-1)
    arr = arr.reshape(n_far, 2, R, n)
    return arr[:, 0].transpose(0, 2, 1), arr[:, 1].transpose(0, 2, 1)


@pytest.mark.parametrize("fmt,bound", [("bf16x2", 2.0 ** -16), ("f16x2", 2.0 ** -20)])
def test_split_factors_decode(stores, fmt, bound):
    r3m = stores["r3m"]
    s = stores[fmt]
    U, V = decode(r3m, s)
    U0, V0 = decode(r3m, stores["c128"])
    assert np.array_equal(s.ranks, stores["c128"].ranks)
    worst = 0.0
    for A, A0 in ((U, U0), (V, V0)):
        colmax = np.maximum(np.abs(A0.real), np.abs(A0.imag)).max(axis=1, keepdims=True)  # [f][1][R]
        err = np.maximum(np.abs(A.real - A0.real), np.abs(A.imag - A0.imag))
        ratio = np.where(colmax > 0, err / np.where(colmax > 0, colmax, 1.0), err)
        worst = max(worst, float(ratio.max()))
    print(f"{fmt}: worst entry error / column max = {worst:.3e}")
    assert worst <= bound


def retrieved_on(blocks_near, U, V, states, x):
    blocks = np.zeros(((2 * D + 1) ** 2, blocks_near.shape[1], blocks_near.shape[2]), np.complex128)
    fi = 0
    for dy in range(-D, D + 1):
        for dx in range(-D, D + 1):
            if max(abs(dx), abs(dy)) <= NR:
                blocks[retrieval.slot(dx, dy, D, D)] = blocks_near[retrieval.slot(dx, dy, NR, NR)]
            else:
                blocks[retrieval.slot(dx, dy, D, D)] = U[fi] @ V[fi].conj().T
                fi += 1
    return retrieval.retrieved_matvec(blocks, D, D, unit(2).state_off, states, L, x)


@pytest.mark.parametrize("fmt", ["bf16x2", "f16x2"])
def test_split_matvec_vs_retrieval_of_decoded(stores, fmt):
    r3m, ctx = stores["r3m"], stores["ctx"]
    s = stores[fmt]
    books = [cb.uniform(L, 4, 51), cb.uniform(L, 4, 52)]
    batch = r3m.Batch.from_codebooks(books, [L, L], DEV)
    x = cb.random_complex(2 * L * L * 40, 14)
    xd = torch.from_numpy(x).to(DEV)
    y = torch.zeros_like(xd)
    work = torch.empty(r3m.matvec_work_bytes(ctx, s, batch, r3m.C128), dtype=torch.uint8, device=DEV)
    r3m.r3m_retrieved_matvec(ctx, s, batch, r3m.C128, xd, y, work)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    U, V = decode(r3m, s)
    near = s.near.cpu().numpy().astype(np.complex128)
    N = L * L * 40
    for b in range(2):
        ref = retrieved_on(near, U, V, books[b], x[b * N:(b + 1) * N])
        assert rel_max(y[b * N:(b + 1) * N], ref) <= 1e-6


def test_split_refined_solve(stores):
    """Inner solve on complex64 near blocks and split BF16 far factors, outer
    FP64 refinement residual on the complex128 store of the same ACA."""
    r3m, ctx, geom = stores["r3m"], stores["ctx"], stores["geom"]
    books = [cb.uniform(L, 4, 61), cb.checkerboard(L, 4) * 3]
    batch = r3m.Batch.from_codebooks(books, [L, L], DEV)
    N = 2 * L * L * 40
    b = torch.zeros(N, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, geom, batch, [[0.0, 0.0, 1.0], [0.35, 0.0, 1.0]], b)
    dirs = cb.phi0_cut(5.0)

    def run(st, st64, tol, refine_tol):
        x = torch.zeros_like(b)
        work = torch.empty(r3m.gmres_work_bytes(ctx, st, batch, 30, st64), dtype=torch.uint8, device=DEV)
        _, rep = r3m.r3m_gmres_solve(ctx, st, st64, batch, b, x, tol, 30, 2000, work, refine_tol=refine_tol,
                                     max_refine=20, precond=r3m.PRECOND_BLOCK_JACOBI)
        sig = torch.zeros(2 * len(dirs), dtype=torch.float64, device=DEV)
        r3m.r3m_rcs(ctx, geom, batch, x, dirs, 1.0, sig)
        torch.cuda.synchronize()
        return x, sig.cpu().numpy(), rep

    x_ref, s_ref, rep_ref = run(stores["c128"], None, 1e-10, 0.0)
    x_mix, s_mix, rep = run(stores["bf16x2"], stores["c128"], 1e-3, 1e-6)
    assert all(r[3] for r in rep) and all(r[2] <= 1e-6 for r in rep)
    assert max(r[1] for r in rep) >= 1  # the refinement loop ran
    err = rel_l2(s_mix, s_ref)
    print(f"refined split solve: refine steps {[r[1] for r in rep]}, residuals {[r[2] for r in rep]}, "
          f"RCS error {err:.2e}")
    assert err <= 1e-6
