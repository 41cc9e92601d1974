"""Batched and large workloads: many codebooks, array sizes and incidence
angles sharing one store (Sec. III-A: one global matrix, many retrievals).

  * reduced batch, solved: 1-bit codebooks of sizes 4, 6 and 8 from the three
    families (Bernoulli, 4x4 checkerboard, stripes), each at four incidence
    angles sharing its mask, one store sized for 8 x 8 (complex64 near blocks,
    split BF16 far factors), FP64 refinement to 1e-6 on the complex128 store
    of the same ACA, all right-hand sides in one solver call.  Reference: the
    plain FP64 GPU path (all blocks dense complex128, solved to 1e-10), and for
    the 4 x 4 codebooks dense LU on the oracle's direct system;
  * full-size batch, one matvec: 384 codebooks (128 each at 32 x 32, 48 x 48
    and 64 x 64) x 4 angles = 1,536 right-hand sides over one store sized for
    64 x 64, split BF16 far factors; three right-hand sides checked against
    the plain complex128 path (the same codebooks in a batch of their own);
  * large array, one matvec: 16 Bernoulli codebooks of 128 x 128 units,
    split FP16 far factors of rank <= 12; two right-hand sides checked against
    the plain complex128 path.
Tolerances: RCS 1e-4 (the workload's bar) and refinement residual 1e-6 for the
solve; for the matvecs the ACA level, 3x the largest achieved block error
plus the split-format error (1e-5).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_common import FREQ, K, rel_l2, unit  # noqa: E402
from oracle import efie, excitation, farfield, solve  # noqa: E402
from workloads import codebooks as cb  # noqa: E402
from workloads.configs import batched_1bit, large_128x128  # noqa: E402

DEV = "cuda:0"
ANGLES = (0.0, 20.0, 40.0, 60.0)


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_05082_amd import pipeline, r3m
    r3m.load()
    ctx = r3m.Context(0)
    geom = r3m.UnitGeom.from_macro(unit(1), FREQ, 1)
    yield r3m, pipeline, ctx, geom
    ctx.close()


def incidences(n_books):
    return [[np.deg2rad(a), 0.0, 1.0] for _ in range(n_books) for a in ANGLES]


def test_batched_solve_reduced(lib):
    r3m, pipeline, ctx, geom = lib
    books, sizes = [], []
    for L in (4, 6, 8):
        for c in range(3):
            books.append(cb.family(c, L, 2000 + 10 * L))
            sizes.append(L)
    batch = r3m.Batch.from_codebooks(books, sizes, DEV, repeat=len(ANGLES))
    D = 7
    dense = pipeline.fill_blocks(ctx, geom, D, r3m.C128, DEV)
    s_bf = pipeline.compressed_store(ctx, geom, 8, 2, r3m.C64, r3m.BF16X2, 1e-4, 12, DEV, dense_c128=dense)
    s_64 = pipeline.compressed_store(ctx, geom, 8, 2, r3m.C128, r3m.C128, 1e-4, 12, DEV, dense_c128=dense)
    plain = r3m.Store(80, 2, D, D, D, r3m.C128, dense)
    N = batch.total_units * 40
    b = torch.zeros(N, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, geom, batch, incidences(len(books)), b)
    dirs = cb.phi0_cut(5.0)

    def run(st, st64, tol, refine_tol, restart):
        x = torch.zeros_like(b)
        work = torch.empty(r3m.gmres_work_bytes(ctx, st, batch, restart, st64), dtype=torch.uint8, device=DEV)
        _, rep = r3m.r3m_gmres_solve(ctx, st, st64, batch, b, x, tol, restart, 3000, work, refine_tol=refine_tol,
                                     max_refine=20, precond=r3m.PRECOND_BLOCK_JACOBI)
        sig = torch.zeros(batch.B * len(dirs), dtype=torch.float64, device=DEV)
        r3m.r3m_rcs(ctx, geom, batch, x, dirs, 1.0, sig)
        torch.cuda.synchronize()
        return x.cpu().numpy(), sig.cpu().numpy().reshape(batch.B, -1), rep

    _, s_ref, rep_ref = run(plain, None, 1e-10, 0.0, 60)
    assert all(r[3] for r in rep_ref)
    x_mix, s_mix, rep = run(s_bf, s_64, 1e-3, 1e-6, 30)
    assert all(r[3] and r[2] <= 1e-6 for r in rep)
    errs = [rel_l2(s_mix[i], s_ref[i]) for i in range(batch.B)]
    print(f"batched reduced: {batch.B} RHS, max RCS error {max(errs):.2e}, "
          f"refine steps {sorted(set(r[1] for r in rep))}")
    assert max(errs) <= 1e-4
    # oracle anchor: the 4 x 4 codebooks at every angle, dense LU on the direct system
    u1 = unit(1)
    for c in range(3):
        st = books[c]
        Zk = efie.direct_system(u1, st, 4, K, 1)
        mesh, _ = efie.active_array_mesh(u1, st, 4)
        for a, ang in enumerate(ANGLES):
            r = c * len(ANGLES) + a
            I = solve.lu_solve(Zk, excitation.plane_wave(mesh, K, np.deg2rad(ang), 0.0))
            sref = farfield.rcs(mesh, I, K, dirs)
            assert rel_l2(s_mix[r], sref) <= 1e-4


def aca_bound(store):
    return 3.0 * float(store.rel_err.max()) + 1e-5


def sub_batch(r3m, books, sizes, rhs, repeat):
    """The codebooks of the chosen right-hand sides in a batch of their own."""
    return r3m.Batch.from_codebooks([books[r // repeat] for r in rhs], [sizes[r // repeat] for r in rhs], DEV)


def test_batched_fullsize_matvec(lib):
    r3m, pipeline, ctx, geom = lib
    w = batched_1bit(128)
    rep = len(w.angles_deg)
    batch = r3m.Batch.from_codebooks(w.codebooks, w.sizes, DEV, repeat=rep)
    assert batch.B == 1536
    D = 63
    dense = pipeline.fill_blocks(ctx, geom, D, r3m.C128, DEV)
    store = pipeline.compressed_store(ctx, geom, 64, 2, r3m.C64, r3m.BF16X2, 1e-4, 12, DEV, dense_c128=dense)
    plain = r3m.Store(80, 2, D, D, D, r3m.C128, dense)
    N = batch.total_units * 40
    g = torch.Generator(device=DEV).manual_seed(7)
    x = torch.complex(torch.randn(N, generator=g, device=DEV), torch.randn(N, generator=g, device=DEV))
    y = torch.zeros_like(x)
    work = torch.empty(r3m.matvec_work_bytes(ctx, store, batch, r3m.C64), dtype=torch.uint8, device=DEV)
    r3m.r3m_retrieved_matvec(ctx, store, batch, r3m.C64, x, y, work)
    torch.cuda.synchronize()
    del work
    rhs = [5, 512 + 6, 1024 + 7]  # one right-hand side of each array size
    sub = sub_batch(r3m, w.codebooks, w.sizes, rhs, rep)
    offs = batch.unit_off[rhs] * 40
    lens = np.array([w.sizes[r // rep] ** 2 * 40 for r in rhs])
    xs = torch.cat([x[o:o + n] for o, n in zip(offs, lens)]).to(torch.complex128)
    ys = torch.zeros_like(xs)
    wp = torch.empty(max(r3m.matvec_work_bytes(ctx, plain, sub, r3m.C128), 16), dtype=torch.uint8, device=DEV)
    r3m.r3m_retrieved_matvec(ctx, plain, sub, r3m.C128, xs, ys, wp)
    torch.cuda.synchronize()
    ys = ys.cpu().numpy()
    yb = np.concatenate([y[o:o + n].cpu().numpy() for o, n in zip(offs, lens)])
    so = np.concatenate([[0], np.cumsum(lens)])
    errs = [rel_l2(yb[so[i]:so[i + 1]], ys[so[i]:so[i + 1]]) for i in range(3)]
    print(f"batched full size: 1536 RHS, errors vs plain {['%.2e' % e for e in errs]}, "
          f"max ACA error {store.rel_err.max():.2e}, mean rank {store.ranks.mean():.2f}")
    assert max(errs) <= aca_bound(store)


def test_large_matvec(lib):
    r3m, pipeline, ctx, geom = lib
    w = large_128x128(16)
    batch = r3m.Batch.from_codebooks(w.codebooks, w.sizes, DEV)
    D = 127
    dense = pipeline.fill_blocks(ctx, geom, D, r3m.C128, DEV)
    store = pipeline.compressed_store(ctx, geom, 128, 2, r3m.C64, r3m.F16X2, 1e-4, 12, DEV, dense_c128=dense)
    plain = r3m.Store(80, 2, D, D, D, r3m.C128, dense)
    N = batch.total_units * 40
    g = torch.Generator(device=DEV).manual_seed(8)
    x = torch.complex(torch.randn(N, generator=g, device=DEV), torch.randn(N, generator=g, device=DEV))
    y = torch.zeros_like(x)
    work = torch.empty(r3m.matvec_work_bytes(ctx, store, batch, r3m.C64), dtype=torch.uint8, device=DEV)
    r3m.r3m_retrieved_matvec(ctx, store, batch, r3m.C64, x, y, work)
    torch.cuda.synchronize()
    del work
    n1 = 128 * 128 * 40
    errs = []
    for r in (0, 15):
        sub = sub_batch(r3m, w.codebooks, w.sizes, [r], 1)
        xs = x[r * n1:(r + 1) * n1].to(torch.complex128)
        ys = torch.zeros_like(xs)
        wp = torch.empty(max(r3m.matvec_work_bytes(ctx, plain, sub, r3m.C128), 16), dtype=torch.uint8,
                         device=DEV)
        r3m.r3m_retrieved_matvec(ctx, plain, sub, r3m.C128, xs, ys, wp)
        torch.cuda.synchronize()
        errs.append(rel_l2(y[r * n1:(r + 1) * n1].cpu().numpy(), ys.cpu().numpy()))
    print(f"large 128x128 x16: errors vs plain {['%.2e' % e for e in errs]}, max ACA error "
          f"{store.rel_err.max():.2e}, ranks at cap {(store.ranks == 12).sum()} of {len(store.ranks)}")
    assert max(errs) <= aca_bound(store)


def test_batched_fullsize_solve_spectral(lib):
    """The batched workload solved at full size on block spectra in the
    configuration the benchmark times (workloads.configs.BATCHED_SOLVE): 384
    1-bit codebooks (128 each at 32x32, 48x48, 64x64) x 4 angles = 1,536 RHS
    in one solver call, complex64 spectra for the inner block-Jacobi GMRES(20)
    to 1e-3, FP64 refinement residual on complex128 spectra to 1e-6.  Every
    RHS must converge.  A stratified sample of 36 RHS (every array size x
    codebook family x angle, the first codebook of each family) is re-solved
    on its own in FP64 to 1e-10 on complex128 spectra, and the RCS of each
    must agree to 1e-4."""
    from workloads.configs import BATCHED_SOLVE as P
    r3m, pipeline, ctx, geom = lib
    w = batched_1bit(128)
    rep_ = len(w.angles_deg)
    batch = r3m.Batch.from_codebooks(w.codebooks, w.sizes, DEV, repeat=rep_)
    assert batch.B == 1536
    dense = pipeline.fill_blocks(ctx, geom, 63, r3m.C128, DEV)
    s64 = pipeline.spectral_store(ctx, geom, 64, 2, r3m.C64, DEV, dense_c128=dense)
    s128 = pipeline.spectral_store(ctx, geom, 64, 2, r3m.C128, DEV, dense_c128=dense)
    del dense
    torch.cuda.empty_cache()
    N = batch.total_units * 40
    inc = incidences(len(w.codebooks))
    b = torch.zeros(N, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, geom, batch, inc, b)
    x = torch.zeros_like(b)
    work = torch.empty(r3m.gmres_work_bytes(ctx, s64, batch, P["restart"], s128), dtype=torch.uint8, device=DEV)
    import time
    torch.cuda.synchronize()
    t0 = time.time()
    _, rep = r3m.r3m_gmres_solve(ctx, s64, s128, batch, b, x, P["inner_tol"], P["restart"], P["max_iter"], work,
                                 refine_tol=P["refine_tol"], max_refine=P["max_refine"],
                                 precond=r3m.PRECOND_BLOCK_JACOBI)
    torch.cuda.synchronize()
    t_solve = time.time() - t0
    del work
    torch.cuda.empty_cache()
    assert all(r[3] and r[2] <= P["refine_tol"] for r in rep)
    dirs = cb.phi0_cut(5.0)
    sig = torch.zeros(batch.B * len(dirs), dtype=torch.float64, device=DEV)
    r3m.r3m_rcs(ctx, geom, batch, x, dirs, 1.0, sig)
    sig = sig.cpu().numpy().reshape(batch.B, -1)
    # codebook c of size index z sits at 128 z + c; family = c mod 3
    sample = [(128 * z + fam) * rep_ + a for z in range(3) for fam in range(3) for a in range(rep_)]
    sub = r3m.Batch.from_codebooks([w.codebooks[r // rep_] for r in sample], [w.sizes[r // rep_] for r in sample],
                                   DEV)
    b1 = torch.zeros(sub.total_units * 40, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, geom, sub, [inc[r] for r in sample], b1)
    x1 = torch.zeros_like(b1)
    wk = torch.empty(r3m.gmres_work_bytes(ctx, s128, sub, 60), dtype=torch.uint8, device=DEV)
    _, rep1 = r3m.r3m_gmres_solve(ctx, s128, None, sub, b1, x1, 1e-10, 60, 6000, wk,
                                  precond=r3m.PRECOND_BLOCK_JACOBI)
    assert all(r[3] for r in rep1)
    s1 = torch.zeros(sub.B * len(dirs), dtype=torch.float64, device=DEV)
    r3m.r3m_rcs(ctx, geom, sub, x1, dirs, 1.0, s1)
    s1 = s1.cpu().numpy().reshape(sub.B, -1)
    errs = [rel_l2(sig[r], s1[i]) for i, r in enumerate(sample)]
    print(f"batched full-size spectral solve: {batch.B} RHS in {t_solve:.1f} s "
          f"({batch.B / t_solve:.0f} solves/s), inner iters max {max(r[0] for r in rep)}, refine steps "
          f"{sorted(set(r[1] for r in rep))}, max residual {max(r[2] for r in rep):.1e}; RCS errors vs FP64 over "
          f"{len(sample)} sampled RHS: max {max(errs):.1e}")
    assert max(errs) <= 1e-4


def test_batched_solves_match_single_solves(lib):
    """Right-hand sides of one batch converge at different iterations; once
    one has converged (or starts converged: a zero excitation), the matvec and
    Krylov kernels skip it for the rest of the cycle, and a restart skips it
    too.  On complex128 spectra every kernel treats each right-hand side
    alone, so the batched solve must reproduce the solves of each right-hand
    side on its own exactly (iterations and solution; short restarts put
    several restarts in the run).  On compressed complex64 / split BF16
    factors with the block ILU and FP64 refinement (correction solves of a
    shrinking set), every right-hand side's residual is checked with the
    refinement store through the matvec call."""
    r3m, pipeline, ctx, geom = lib
    L, D = 8, 7
    books = [cb.family(c % 3, L, 3100 + 7 * c) for c in range(5)]
    sizes = [L] * len(books)
    angles = (0.0, 50.0)
    batch = r3m.Batch.from_codebooks(books, sizes, DEV, repeat=len(angles))
    N1 = L * L * 40
    b = torch.zeros(batch.B * N1, dtype=torch.complex128, device=DEV)
    inc = [[np.deg2rad(a), 0.0, 1.0] for _ in books for a in angles]
    r3m.r3m_plane_wave_rhs(ctx, geom, batch, inc, b)
    b[3 * N1:4 * N1] = 0  # converged before the first step
    dense = pipeline.fill_blocks(ctx, geom, D, r3m.C128, DEV)

    def solve(st, st64, bat, rhs, tol, refine_tol, pc):
        x = torch.zeros_like(rhs)
        work = torch.empty(r3m.gmres_work_bytes(ctx, st, bat, 8, st64, precond=pc), dtype=torch.uint8, device=DEV)
        rc, rep = r3m.r3m_gmres_solve(ctx, st, st64, bat, rhs, x, tol, 8, 4000, work, refine_tol=refine_tol,
                                      max_refine=20, precond=pc)
        torch.cuda.synchronize()
        assert rc == 0
        return x, rep

    spec = pipeline.spectral_store(ctx, geom, L, 2, r3m.C128, DEV, dense_c128=dense)
    xb, repb = solve(spec, None, batch, b, 1e-10, 0.0, r3m.PRECOND_BLOCK_JACOBI)
    its = [r[0] for r in repb]
    assert repb[3][0] == 0 and torch.count_nonzero(xb[3 * N1:4 * N1]) == 0
    assert len(set(its)) >= 3  # staggered convergence: the zero excitation and two distinct counts at least
    worst = 0.0
    for r in range(batch.B):
        one = r3m.Batch.from_codebooks([books[r // len(angles)]], [L], DEV)
        x1, rep1 = solve(spec, None, one, b[r * N1:(r + 1) * N1].clone(), 1e-10, 0.0, r3m.PRECOND_BLOCK_JACOBI)
        assert rep1[0][0] == repb[r][0]
        xr = xb[r * N1:(r + 1) * N1]
        d = float((xr - x1).abs().max()) / max(float(x1.abs().max()), 1e-300)
        worst = max(worst, d)
    print(f"batched vs single solves on complex128 spectra: iterations {its}, max relative difference {worst:.1e}")
    assert worst <= 1e-12

    s_bf = pipeline.compressed_store(ctx, geom, L, 2, r3m.C64, r3m.BF16X2, 1e-4, 12, DEV, dense_c128=dense)
    s_64 = pipeline.compressed_store(ctx, geom, L, 2, r3m.C128, r3m.C128, 1e-4, 12, DEV, dense_c128=dense)
    xc, repc = solve(s_bf, s_64, batch, b, 1e-3, 1e-9, r3m.PRECOND_BLOCK_ILU)
    y = torch.zeros_like(xc)
    work = torch.empty(max(r3m.matvec_work_bytes(ctx, s_64, batch, r3m.C128), 16), dtype=torch.uint8, device=DEV)
    r3m.r3m_retrieved_matvec(ctx, s_64, batch, r3m.C128, xc, y, work)
    torch.cuda.synchronize()
    res = []
    for r in range(batch.B):
        sl = slice(r * N1, (r + 1) * N1)
        bn = float(torch.linalg.vector_norm(b[sl]))
        res.append(float(torch.linalg.vector_norm(b[sl] - y[sl])) / bn if bn > 0 else 0.0)
    print(f"refined compressed batch: iterations {[r[0] for r in repc]}, steps {[r[1] for r in repc]}, "
          f"max residual {max(res):.1e}")
    assert all(r[3] for r in repc) and max(res) <= 1.01e-9
    assert torch.count_nonzero(xc[3 * N1:4 * N1]) == 0


@pytest.mark.parametrize("L,n_books", [(8, 40), (48, 32)])
def test_wide_complex64_batch_matches_aligned_sub_batches(lib, L, n_books):
    """An unrefined complex64-spectra solve of a wide batch (160 or 128 RHS:
    the matrix-core product and its device-built list of live 16-RHS tiles;
    at 48x48, 92,160 unknowns per RHS, the Gram-Schmidt update blocks take
    four 64-element runs) with staggered convergence (three codebook
    families, four angles, and a whole 16-RHS tile of zero excitations idle
    from the start) against the same RHS solved in 16-aligned sub-batches.
    Every kernel computes each right-hand side's column on its own (the
    product's K loop covers all n rows inside one workgroup), so iterations
    and solutions must agree exactly."""
    r3m, pipeline, ctx, geom = lib
    books = [cb.family(c, L, 5100 + 3 * c) for c in range(n_books)]
    batch = r3m.Batch.from_codebooks(books, [L] * n_books, DEV, repeat=len(ANGLES))
    B = batch.B
    N1 = L * L * 40
    spec = pipeline.spectral_store(ctx, geom, L, 2, r3m.C64, DEV)
    b = torch.zeros(B * N1, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, geom, batch, incidences(n_books), b)
    b[32 * N1:48 * N1] = 0  # the third 16-RHS tile starts converged
    restart = 8

    def solve(bat, rhs):
        x = torch.zeros_like(rhs)
        work = torch.empty(r3m.gmres_work_bytes(ctx, spec, bat, restart), dtype=torch.uint8, device=DEV)
        rc, rep = r3m.r3m_gmres_solve(ctx, spec, None, bat, rhs, x, 1e-5, restart, 4000, work,
                                      precond=r3m.PRECOND_BLOCK_JACOBI)
        torch.cuda.synchronize()
        assert rc == 0
        return x, rep

    xb, repb = solve(batch, b)
    its = [r[0] for r in repb]
    assert all(its[r] == 0 for r in range(32, 48))
    assert len(set(its)) >= 8, its  # staggered: tiles go idle at different steps
    worst_it, worst_x = 0, 0.0
    for t0 in range(0, B, 16):
        rhs = list(range(t0, min(B, t0 + 16)))
        sub = r3m.Batch.from_codebooks([books[r // len(ANGLES)] for r in rhs], [L] * len(rhs), DEV)
        xs, reps = solve(sub, b[t0 * N1:(t0 + len(rhs)) * N1].clone())
        for i, r in enumerate(rhs):
            worst_it = max(worst_it, abs(reps[i][0] - repb[r][0]))
        d = float((xs - xb[t0 * N1:(t0 + len(rhs)) * N1]).abs().max())
        worst_x = max(worst_x, d / max(float(xs.abs().max()), 1e-300))
    print(f"wide complex64 batch {L}x{L} x {B} RHS: iterations {min(its)}..{max(its)} "
          f"({len(set(its))} distinct), vs 16-aligned sub-batches: iteration difference {worst_it}, "
          f"max relative solution difference {worst_x:.1e}")
    assert worst_it == 0 and worst_x == 0.0
