"""Spectral (FFT) evaluation of the retrieved product against the oracle.

The retrieved product of eq. (6) over a block-Toeplitz macro system is a 2-D
convolution over units; a spectral store holds the transforms of the
circulant-embedded blocks Z(d) and evaluates it per spatial frequency.  Its
result is the dense retrieval product itself (no compression), so the
references are:
  * oracle blocks uploaded (rectangular store Dx = 3, Dy = 2, ragged and
    rectangular arrays): the oracle's retrieval product, element by element;
  * 2-bit 32 x 32 (the benchmark array): the oracle's rows of Z_k for three
    sampled observer units, computed from the codebook's physical mesh, and
    the plain complex128 path on every row;
  * 128 x 128 x 16: the plain complex128 path on two right-hand sides;
  * solves: the plain FP64 solve's RCS.
Tolerances: complex128 spectra 1e-12 (max-abs, relative to the largest
entry; rounding of O(log2(Gx Gy)) butterfly stages and n-term products in
FP64, ~1e-14 expected) and 1e-10 on sampled rows as for the plain path;
complex64 spectra 2e-6 element-wise and 1e-6 in the 2-norm (the same in FP32:
~12 stages x 6e-8 per transform, two transforms, ~1e-6 at worst); solves
1e-4 RCS (the workload's bar) and 1e-7 after FP64 refinement.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_common import FREQ, K, rel_l2, rel_max, unit  # noqa: E402
from oracle import efie, retrieval  # noqa: E402
from workloads import codebooks as cb  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_05082_amd import pipeline, r3m
    r3m.load()
    ctx = r3m.Context(0)
    yield r3m, pipeline, ctx
    ctx.close()


def to_dev(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dtype)


def spectra_of(r3m, ctx, dense_dev, n, Dx, Dy, dtype):
    sd = r3m.SPEC_C64 if dtype == r3m.C64 else r3m.SPEC_C128
    out = torch.empty(r3m.spectral_bytes(n, Dx, Dy, sd), dtype=torch.uint8, device=DEV)
    r3m.r3m_build_spectral(ctx, dense_dev, n, Dx, Dy, sd, out)
    return sd, out


def matvec(r3m, ctx, store, batch, x, vec_dtype):
    y = torch.zeros_like(x)
    work = torch.empty(max(r3m.matvec_work_bytes(ctx, store, batch, vec_dtype), 16), dtype=torch.uint8,
                       device=DEV)
    r3m.r3m_retrieved_matvec(ctx, store, batch, vec_dtype, x, y, work)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def oracle_rect(blocks, Dx, Dy, n_a, state_off, book, lx, ly, x):
    """Oracle product of an lx x ly array: the array embedded in the oracle's
    square layout with zero x on the padding units (which then add nothing)."""
    Ls = max(lx, ly)
    full = np.zeros(Ls * Ls, np.uint8)
    mask = np.zeros(Ls * Ls, bool)
    for iy in range(ly):
        for ix in range(lx):
            full[iy * Ls + ix] = book[iy * lx + ix]
            mask[iy * Ls + ix] = True
    xf = np.zeros((Ls * Ls, n_a), complex)
    xf[mask] = x.reshape(-1, n_a)
    n = blocks.shape[1]
    sub = np.zeros(((2 * Ls - 1) ** 2, n, n), complex)
    for dy in range(-(Ls - 1), Ls):
        for dx in range(-(Ls - 1), Ls):
            if abs(dx) <= Dx and abs(dy) <= Dy:
                sub[retrieval.slot(dx, dy, Ls - 1, Ls - 1)] = blocks[retrieval.slot(dx, dy, Dx, Dy)]
    yf = retrieval.retrieved_matvec(sub, Ls - 1, Ls - 1, state_off, full, Ls, xf.reshape(-1))
    return yf.reshape(-1, n_a)[mask].reshape(-1)


@pytest.mark.parametrize("dtype,vec,tol,rep", [("c128", "c128", 1e-12, 1), ("c64", "c128", 2e-6, 1),
                                               ("c64", "c64", 2e-6, 1), ("c64", "c64", 2e-6, 3),
                                               ("c128", "c128", 1e-12, 3)])
def test_spectral_oracle_blocks(lib, dtype, vec, tol, rep):
    """rep = 3: every array three times (15 right-hand sides, the matrix-core
    product for complex64 spectra, with a partial 16-wide tile)."""
    r3m, _, ctx = lib
    Dx, Dy = 3, 2
    blocks = efie.displacement_blocks(unit(1), Dx, Dy, K, extract=1)
    st = r3m.C128 if dtype == "c128" else r3m.C64
    vt = r3m.C128 if vec == "c128" else r3m.C64
    sd, spec = spectra_of(r3m, ctx, to_dev(blocks), 80, Dx, Dy, st)
    self_blk = to_dev(blocks[retrieval.slot(0, 0, Dx, Dy)][None], torch.complex128 if st == r3m.C128 else
                      torch.complex64)
    store = r3m.Store(80, 2, Dx, Dy, 0, st, self_blk, sd, spec)
    L1 = np.array([[4, 3], [1, 1], [3, 2], [2, 3], [4, 1]], np.int32)
    books, so = [], []
    s_at = 0
    for b, (lx, ly) in enumerate(L1):
        books.append(cb.bernoulli(4, 70 + b)[: lx * ly])
        so.append(s_at)
        s_at += lx * ly
    L = np.concatenate([L1] * rep)
    book_of = list(range(len(L1))) * rep
    uo = np.concatenate([[0], np.cumsum(L[:, 0] * L[:, 1])[:-1]])
    u = int((L[:, 0] * L[:, 1]).sum())
    batch = r3m.Batch(L, uo, [so[i] for i in book_of], torch.from_numpy(np.concatenate(books)).to(DEV))
    x = cb.random_complex(u * 40, 31)
    y = matvec(r3m, ctx, store, batch, to_dev(x, torch.complex128 if vt == r3m.C128 else torch.complex64), vt)
    if vt == r3m.C64:
        x = x.astype(np.complex64).astype(np.complex128)
    worst = 0.0
    for b, (lx, ly) in enumerate(L):
        sl = slice(uo[b] * 40, (uo[b] + lx * ly) * 40)
        ref = oracle_rect(blocks, Dx, Dy, 40, unit(1).state_off, books[book_of[b]], lx, ly, x[sl])
        worst = max(worst, rel_max(y[sl], ref))
    print(f"spectral {dtype} spectra, {vec} vectors, {len(L)} RHS: worst element error {worst:.2e}")
    assert worst <= tol


@pytest.fixture(scope="module")
def fullsize(lib):
    r3m, pipeline, ctx = lib
    geom = r3m.UnitGeom.from_macro(unit(2), FREQ, 1)
    states = cb.uniform(32, 4, 1)
    batch = r3m.Batch.from_codebooks([states], [32], DEV)
    dense = pipeline.fill_blocks(ctx, geom, 31, r3m.C128, DEV)
    s128 = pipeline.spectral_store(ctx, geom, 32, 2, r3m.C128, DEV, dense_c128=dense)
    s64 = pipeline.spectral_store(ctx, geom, 32, 2, r3m.C64, DEV, dense_c128=dense)
    plain = r3m.Store(160, 4, 31, 31, 31, r3m.C128, dense)
    yield geom, states, batch, s128, s64, plain


def test_spectral_fullsize_rows(lib, fullsize):
    from test_gpu_fullsize import oracle_rows, sample
    r3m, _, ctx = lib
    geom, states, batch, s128, s64, plain = fullsize
    st, Zr, _ = oracle_rows()
    assert np.array_equal(st, states)
    x = cb.random_complex(32 * 32 * 40, 11)
    xd = to_dev(x)
    y_plain = matvec(r3m, ctx, plain, batch, xd, r3m.C128)
    y128 = matvec(r3m, ctx, s128, batch, xd, r3m.C128)
    y64 = matvec(r3m, ctx, s64, batch, xd, r3m.C128)
    e_rows128 = rel_l2(sample(y128), Zr @ x)
    e_rows64 = rel_l2(sample(y64), Zr @ x)
    e128 = rel_max(y128, y_plain)
    e64 = rel_max(y64, y_plain)
    e64_l2 = rel_l2(y64, y_plain)
    print(f"32x32 spectral: c128 rows vs oracle {e_rows128:.2e}, vs plain {e128:.2e}; c64 rows vs oracle "
          f"{e_rows64:.2e}, vs plain max {e64:.2e} l2 {e64_l2:.2e}")
    assert e_rows128 <= 1e-10 and e128 <= 1e-12
    assert e64 <= 2e-6 and e64_l2 <= 1e-6


@pytest.mark.parametrize("pc", [1, 2])
def test_spectral_solves(lib, fullsize, pc):
    """Block-Jacobi (1) or near-field block ILU (2) solves of the 2-bit 32x32
    workload on complex64 spectra, and refined on complex128 spectra."""
    r3m, _, ctx = lib
    geom, _, batch, s128, s64, plain = fullsize
    N = 32 * 32 * 40
    dirs = cb.phi0_cut(1.0)
    b = torch.zeros(N, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, geom, batch, [[0.0, 0.0, 1.0]], b)

    def solve(st, st64, tol, refine_tol):
        x = torch.zeros_like(b)
        work = torch.empty(r3m.gmres_work_bytes(ctx, st, batch, 60, st64, precond=pc), dtype=torch.uint8,
                           device=DEV)
        _, rep = r3m.r3m_gmres_solve(ctx, st, st64, batch, b, x, tol, 60, 6000, work, refine_tol=refine_tol,
                                     max_refine=20, precond=pc)
        sig = torch.zeros(len(dirs), dtype=torch.float64, device=DEV)
        r3m.r3m_rcs(ctx, geom, batch, x, dirs, 1.0, sig)
        torch.cuda.synchronize()
        return sig.cpu().numpy(), rep

    s_ref, rep_ref = solve(plain, None, 1e-10, 0.0)
    assert rep_ref[0][3]
    s_mix, rep = solve(s64, None, 1e-5, 0.0)
    s_ref_spec, rep2 = solve(s64, s128, 1e-4, 1e-9)
    e_mix = rel_l2(s_mix, s_ref)
    e_ref = rel_l2(s_ref_spec, s_ref)
    print(f"spectral solves (precond {pc}): c64 iters {rep[0][0]} RCS error {e_mix:.2e}; refined to 1e-9 on c128 spectra "
          f"(steps {rep2[0][1]}) RCS error {e_ref:.2e}")
    assert rep[0][3] and e_mix <= 1e-4
    assert rep2[0][3] and rep2[0][2] <= 1e-9 and e_ref <= 1e-7


def test_refined_solve_short_restarts(lib, fullsize):
    """Complex64 inner GMRES(4) with block-Jacobi under complex128
    refinement on the 2-bit 32x32 workload: every inner restart takes the
    cycle's residual from its basis (Givens rotations, no residual matvec),
    dozens of restarts per inner solve.  The refined solution must converge
    to 1e-9 and give the RCS of the plain complex128 solve, and each inner
    solve must take no more than twice the iterations of GMRES(4) on the
    plain store (which forms each restart's residual with a matvec)."""
    r3m, _, ctx = lib
    geom, _, batch, s128, s64, plain = fullsize
    N = 32 * 32 * 40
    dirs = cb.phi0_cut(1.0)
    b = torch.zeros(N, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, geom, batch, [[0.0, 0.0, 1.0]], b)

    def solve(st, st64, m, tol, refine_tol):
        x = torch.zeros_like(b)
        work = torch.empty(r3m.gmres_work_bytes(ctx, st, batch, m, st64, precond=r3m.PRECOND_BLOCK_JACOBI),
                           dtype=torch.uint8, device=DEV)
        _, rep = r3m.r3m_gmres_solve(ctx, st, st64, batch, b, x, tol, m, 20000, work, refine_tol=refine_tol,
                                     max_refine=40, precond=r3m.PRECOND_BLOCK_JACOBI)
        sig = torch.zeros(len(dirs), dtype=torch.float64, device=DEV)
        r3m.r3m_rcs(ctx, geom, batch, x, dirs, 1.0, sig)
        torch.cuda.synchronize()
        return sig.cpu().numpy(), rep

    s_ref, rep_ref = solve(plain, None, 60, 1e-10, 0.0)
    assert rep_ref[0][3]
    _, rep_plain4 = solve(plain, None, 4, 1e-4, 0.0)
    s_short, rep = solve(s64, s128, 4, 1e-4, 1e-9)
    err = rel_l2(s_short, s_ref)
    print(f"refined GMRES(4): inner iterations {rep[0][0]} (plain GMRES(4) to 1e-4: {rep_plain4[0][0]}), "
          f"refinement steps {rep[0][1]}, residual {rep[0][2]:.2e}, RCS error {err:.2e}")
    assert rep[0][3] and rep[0][2] <= 1e-9 and err <= 1e-7
    assert rep[0][1] >= 1  # the refinement loop ran
    # each inner solve is a GMRES(4) to 1e-4 on an operator within FP32
    # rounding of the plain one: at most twice the plain solve's iterations
    # per inner solve (refinement steps + 1 of them)
    assert rep[0][0] <= 2 * (rep[0][1] + 1) * rep_plain4[0][0]


@pytest.fixture(scope="module")
def large(lib):
    from workloads.configs import large_128x128
    r3m, pipeline, ctx = lib
    geom = r3m.UnitGeom.from_macro(unit(1), FREQ, 1)
    w = large_128x128(16)
    batch = r3m.Batch.from_codebooks(w.codebooks, w.sizes, DEV)
    dense = pipeline.fill_blocks(ctx, geom, 127, r3m.C128, DEV)
    s64 = pipeline.spectral_store(ctx, geom, 128, 2, r3m.C64, DEV, dense_c128=dense)
    s128 = pipeline.spectral_store(ctx, geom, 128, 2, r3m.C128, DEV, dense_c128=dense)
    plain = r3m.Store(80, 2, 127, 127, 127, r3m.C128, dense)
    yield w, geom, batch, s64, s128, plain


def test_spectral_large(lib, large):
    """16 RHS of 128 x 128 units (the matrix-core product for complex64
    spectra); two RHS against the plain complex128 path."""
    r3m, _, ctx = lib
    w, _, batch, s64, s128, plain = large
    N = batch.total_units * 40
    g = torch.Generator(device=DEV).manual_seed(8)
    x = torch.complex(torch.randn(N, generator=g, device=DEV), torch.randn(N, generator=g, device=DEV))
    y64 = matvec(r3m, ctx, s64, batch, x, r3m.C64)
    y128 = matvec(r3m, ctx, s128, batch, x.to(torch.complex128), r3m.C128)
    n1 = 128 * 128 * 40
    e64, e128 = [], []
    for r in (0, 15):
        sub = r3m.Batch.from_codebooks([w.codebooks[r]], [128], DEV)
        ys = matvec(r3m, ctx, plain, sub, x[r * n1:(r + 1) * n1].to(torch.complex128), r3m.C128)
        e64.append(rel_l2(y64[r * n1:(r + 1) * n1], ys))
        e128.append(rel_max(y128[r * n1:(r + 1) * n1], ys))
    print(f"large 128x128 x16 spectral: c64 errors vs plain {['%.2e' % e for e in e64]}, c128 "
          f"{['%.2e' % e for e in e128]}")
    assert max(e64) <= 1e-6 and max(e128) <= 1e-12


def test_spectral_large_refined_solve(lib, large):
    """The large workload solved: inner GMRES on complex64 spectra,
    refinement residual on complex128 spectra (the dense operator in FP64),
    every RHS to 1e-5; one RHS re-solved on its own in FP64 to 1e-9 as the
    reference for its RCS."""
    r3m, _, ctx = lib
    w, geom, batch, s64, s128, _ = large
    N = batch.total_units * 40
    b = torch.zeros(N, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, geom, batch, [[0.0, 0.0, 1.0]] * batch.B, b)
    x = torch.zeros_like(b)
    work = torch.empty(r3m.gmres_work_bytes(ctx, s64, batch, 30, s128), dtype=torch.uint8, device=DEV)
    _, rep = r3m.r3m_gmres_solve(ctx, s64, s128, batch, b, x, 1e-3, 30, 3000, work, refine_tol=w.refine_tol,
                                 max_refine=20, precond=r3m.PRECOND_BLOCK_JACOBI)
    del work
    assert all(r[3] and r[2] <= w.refine_tol for r in rep)
    dirs = cb.phi0_cut(5.0)
    sig = torch.zeros(batch.B * len(dirs), dtype=torch.float64, device=DEV)
    r3m.r3m_rcs(ctx, geom, batch, x, dirs, 1.0, sig)
    sub = r3m.Batch.from_codebooks([w.codebooks[3]], [128], DEV)
    n1 = 128 * 128 * 40
    b1 = b[3 * n1:4 * n1].clone()
    x1 = torch.zeros_like(b1)
    work = torch.empty(r3m.gmres_work_bytes(ctx, s128, sub, 30), dtype=torch.uint8, device=DEV)
    _, rep1 = r3m.r3m_gmres_solve(ctx, s128, None, sub, b1, x1, 1e-9, 30, 6000, work,
                                  precond=r3m.PRECOND_BLOCK_JACOBI)
    sig1 = torch.zeros(len(dirs), dtype=torch.float64, device=DEV)
    r3m.r3m_rcs(ctx, geom, sub, x1, dirs, 1.0, sig1)
    torch.cuda.synchronize()
    err = rel_l2(sig.cpu().numpy().reshape(batch.B, -1)[3], sig1.cpu().numpy())
    print(f"large refined solve: inner iters max {max(r[0] for r in rep)}, refine steps "
          f"{sorted(set(r[1] for r in rep))}, max residual {max(r[2] for r in rep):.2e}; FP64 reference "
          f"{rep1[0][0]} iters, RCS error {err:.2e}")
    assert rep1[0][3] and err <= 1e-4


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-12), ("c64", 2e-6)])
def test_spectral_degenerate_extent(lib, dtype, tol):
    """Dx = 0: single-column arrays, transforms of length 2 along x (one
    radix-2 stage) and 8 along y; an array of one unit."""
    r3m, _, ctx = lib
    Dx, Dy = 0, 3
    blocks = efie.displacement_blocks(unit(1), Dx, Dy, K, extract=1)
    st = r3m.C128 if dtype == "c128" else r3m.C64
    tdt = torch.complex128 if st == r3m.C128 else torch.complex64
    sd, spec = spectra_of(r3m, ctx, to_dev(blocks), 80, Dx, Dy, st)
    store = r3m.Store(80, 2, Dx, Dy, 0, st, to_dev(blocks[retrieval.slot(0, 0, Dx, Dy)][None], tdt), sd, spec)
    L = np.array([[1, 4], [1, 1], [1, 2]], np.int32)
    books = [cb.bernoulli(4, 90 + b)[: lx * ly] for b, (lx, ly) in enumerate(L)]
    uo = np.concatenate([[0], np.cumsum(L[:, 0] * L[:, 1])[:-1]])
    u = int((L[:, 0] * L[:, 1]).sum())
    batch = r3m.Batch(L, uo, uo, torch.from_numpy(np.concatenate(books)).to(DEV))
    x = cb.random_complex(u * 40, 33)
    y = matvec(r3m, ctx, store, batch, to_dev(x, tdt), st)
    if st == r3m.C64:
        x = x.astype(np.complex64).astype(np.complex128)
    worst = 0.0
    for b, (lx, ly) in enumerate(L):
        sl = slice(uo[b] * 40, (uo[b] + lx * ly) * 40)
        ref = oracle_rect(blocks, Dx, Dy, 40, unit(1).state_off, books[b], lx, ly, x[sl])
        worst = max(worst, rel_max(y[sl], ref))
    print(f"spectral Dx=0 {dtype}: worst element error {worst:.2e}")
    assert worst <= tol


def test_spectral_empty_batch_and_errors(lib):
    r3m, _, ctx = lib
    Dx = Dy = 1
    blocks = efie.displacement_blocks(unit(1), Dx, Dy, K, extract=1)
    dense = to_dev(blocks)
    sd, spec = spectra_of(r3m, ctx, dense, 80, Dx, Dy, r3m.C64)
    near64 = to_dev(blocks[retrieval.slot(0, 0, Dx, Dy)][None], torch.complex64)
    near128 = to_dev(blocks[retrieval.slot(0, 0, Dx, Dy)][None])
    good = r3m.Store(80, 2, Dx, Dy, 0, r3m.C64, near64, sd, spec)
    # an empty batch is a no-op
    empty = r3m.Batch(np.zeros((0, 2), np.int32), [], [], torch.zeros(1, dtype=torch.uint8, device=DEV))
    xe = torch.zeros(1, dtype=torch.complex64, device=DEV)
    r3m.r3m_retrieved_matvec(ctx, good, empty, r3m.C64, xe, xe.clone(), None)
    books = [cb.bernoulli(2, 5)]
    batch = r3m.Batch.from_codebooks(books, [2], DEV)
    x = torch.zeros(160, dtype=torch.complex64, device=DEV)
    work = torch.empty(r3m.matvec_work_bytes(ctx, good, batch, r3m.C64), dtype=torch.uint8, device=DEV)

    def code_of(fn):
        with pytest.raises(r3m.R3MError) as e:
            fn()
        return e.value.code

    # complex64 spectra with complex128 near blocks
    bad = r3m.Store(80, 2, Dx, Dy, 0, r3m.C128, near128, sd, spec)
    assert code_of(lambda: r3m.r3m_retrieved_matvec(ctx, bad, batch, r3m.C64, x, x.clone(), work)) == \
        r3m.R3M_ERR_UNSUPPORTED
    # missing spectra
    nospec = r3m.Store(80, 2, Dx, Dy, 0, r3m.C64, near64, sd, None)
    assert code_of(lambda: r3m.r3m_retrieved_matvec(ctx, nospec, batch, r3m.C64, x, x.clone(), work)) == \
        r3m.R3M_ERR_INVALID_ARG
    # complex128 spectra need complex128 vectors
    sd2, spec2 = spectra_of(r3m, ctx, dense, 80, Dx, Dy, r3m.C128)
    s128 = r3m.Store(80, 2, Dx, Dy, 0, r3m.C128, near128, sd2, spec2)
    w2 = torch.empty(r3m.matvec_work_bytes(ctx, s128, batch, r3m.C64), dtype=torch.uint8, device=DEV)
    assert code_of(lambda: r3m.r3m_retrieved_matvec(ctx, s128, batch, r3m.C64, x, x.clone(), w2)) == \
        r3m.R3M_ERR_UNSUPPORTED
    # a workspace one byte short, a spectra buffer one byte short
    short = torch.empty(work.numel() - 1, dtype=torch.uint8, device=DEV)
    assert code_of(lambda: r3m.r3m_retrieved_matvec(ctx, good, batch, r3m.C64, x, x.clone(), short)) == \
        r3m.R3M_ERR_BUFFER_TOO_SMALL
    small = torch.empty(r3m.spectral_bytes(80, Dx, Dy, r3m.SPEC_C64) - 1, dtype=torch.uint8, device=DEV)
    assert code_of(lambda: r3m.r3m_build_spectral(ctx, dense, 80, Dx, Dy, r3m.SPEC_C64, small)) == \
        r3m.R3M_ERR_BUFFER_TOO_SMALL
    torch.cuda.synchronize()


@pytest.mark.parametrize("relaxed_solve", [False, True])
def test_spectral_graph_replays_match_eager(lib, relaxed_solve):
    """Arnoldi blocks replayed from captured HIP graphs on a spectral store
    (transform kernels with dynamic LDS, per-frequency products) give bitwise
    the eager result on the first capture and on later replays, with eager
    work and synchronisations in between; also for a relaxed transposed solve
    with per-unit block-Jacobi."""
    r3m, pipeline, ctx = lib
    geom = r3m.UnitGeom.from_macro(unit(2), FREQ, 1)
    L = 8
    store = pipeline.spectral_store(ctx, geom, L, 0, r3m.C64 if not relaxed_solve else r3m.C128, DEV)
    batch = r3m.Batch.from_codebooks([cb.uniform(L, 4, 21), cb.uniform(L, 4, 22)], [L, L], DEV)
    b = torch.zeros(2 * L * L * 40, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, geom, batch, [[0.2, 0.1, 1.0], [0.0, 0.0, 1.0]], b)
    w = None
    if relaxed_solve:
        lg = np.random.default_rng(23).standard_normal((2 * L * L, 4))
        w = torch.from_numpy(np.exp(lg) / np.exp(lg).sum(axis=1, keepdims=True)).to(DEV)
    work = torch.empty(r3m.gmres_work_bytes(ctx, store, batch, 20, relaxed=relaxed_solve,
                                            precond=r3m.PRECOND_BLOCK_JACOBI), dtype=torch.uint8, device=DEV)

    def run(eager):
        x = torch.zeros_like(b)
        _, rep = r3m.r3m_gmres_solve(ctx, store, None, batch, b, x, 1e-8 if relaxed_solve else 1e-5, 20, 2000,
                                     work, precond=r3m.PRECOND_BLOCK_JACOBI, eager=eager, relaxed_weights=w,
                                     transpose=relaxed_solve)
        torch.cuda.synchronize()
        return x.cpu().numpy(), rep

    x_e, rep_e = run(True)
    assert all(r[3] for r in rep_e)
    for _ in range(3):
        x_g, rep_g = run(False)
        assert np.array_equal(x_g, x_e) and [r[0] for r in rep_g] == [r[0] for r in rep_e]
        matvec(r3m, ctx, store, batch, b.to(torch.complex64 if not relaxed_solve else torch.complex128),
               r3m.C64 if not relaxed_solve else r3m.C128)
    x_e2, _ = run(True)
    assert np.array_equal(x_e2, x_e)
