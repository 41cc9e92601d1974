"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tolerances (relative, max-abs unless stated):
  * fill, C128: 1e-11 on every block (same formulas, FP64, different
    summation order; extracted blocks carry log/atan edge sums);
  * retrieved matvec, C128 store: 1e-12 against the oracle product with the
    same blocks, and against the direct active-only system Z_k x;
  * GMRES to 1e-12, C128: solution within 1e-8 and RCS within 1e-8 of dense
    LU on the oracle's Z_k (both limited by cond(Z_k) * 1e-12);
  * C64 store vs the C128 store with the same factors: 1e-6 (FP32 products
    of O(40 + r) terms);
  * ACA: achieved error <= tol, product within 2 tol of the oracle's.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_common import (K, FREQ, oracle_blocks, oracle_direct, oracle_rcs, oracle_rhs, rel_l2,  # noqa: E402
                        rel_max, unit)
from oracle import aca, retrieval, solve  # noqa: E402
from workloads import codebooks as cb  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def r3m():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_05082_amd import r3m as mod
    mod.load()
    return mod


@pytest.fixture(scope="module")
def ctx(r3m):
    c = r3m.Context(0)
    yield c
    c.close()


def geom(r3m, bits):
    return r3m.UnitGeom.from_macro(unit(bits), FREQ, 1)


def to_dev(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dtype)


# ---------------------------------------------------------------- fill


@pytest.mark.parametrize("bits,D", [(1, 2), (2, 1)])
def test_fill_matches_oracle_blocks(r3m, ctx, bits, D):
    from paper_2112_05082_amd import pipeline
    g = geom(r3m, bits)
    blocks = pipeline.fill_blocks(ctx, g, D, r3m.C128, DEV).cpu().numpy()
    ref = oracle_blocks(bits, D)
    for s in range(ref.shape[0]):
        assert rel_max(blocks[s], ref[s]) <= 1e-11, s


def test_fill_far_block_2bit(r3m, ctx):
    from oracle import efie
    from paper_2112_05082_amd import pipeline
    g = geom(r3m, 2)
    blocks = pipeline.fill_blocks(ctx, g, 3, r3m.C128, DEV)
    for dx, dy in [(3, -2), (-3, 3), (0, 2)]:
        ref = efie.displacement_block(unit(2), dx, dy, K, 1)
        got = blocks[retrieval.slot(dx, dy, 3, 3)].cpu().numpy()
        assert rel_max(got, ref) <= 1e-11
    c64 = pipeline.fill_blocks(ctx, g, 1, r3m.C64, DEV).cpu().numpy()
    assert rel_max(c64, blocks[[retrieval.slot(dx, dy, 3, 3) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]]
                   .cpu().numpy()) <= 1e-6


# --------------------------------------------------------------- matvec


def batch_for(r3m, books, sizes, repeat=1):
    return r3m.Batch.from_codebooks(books, sizes, DEV, repeat)


def run_matvec(r3m, ctx, store, batch, x, vec_dtype):
    y = torch.zeros_like(x)
    wb = r3m.matvec_work_bytes(ctx, store, batch, vec_dtype)
    work = torch.empty(max(wb, 16), dtype=torch.uint8, device=DEV)
    r3m.r3m_retrieved_matvec(ctx, store, batch, vec_dtype, x, y, work)
    torch.cuda.synchronize()
    return y


def test_matvec_oracle_blocks_c128(r3m, ctx):
    """Matvec kernel alone: oracle blocks uploaded, L = 3, several codebooks."""
    ref_blocks = oracle_blocks(1, 2)
    store = r3m.Store(80, 2, 2, 2, 2, r3m.C128, to_dev(ref_blocks))
    books = [np.zeros(9, np.uint8), np.ones(9, np.uint8), cb.checkerboard(3, 1), cb.bernoulli(3, 5)]
    batch = batch_for(r3m, books, [3] * 4)
    x = cb.random_complex(4 * 9 * 40, 3)
    y = run_matvec(r3m, ctx, store, batch, to_dev(x), r3m.C128).cpu().numpy()
    for b, book in enumerate(books):
        sl = slice(b * 360, (b + 1) * 360)
        ref = retrieval.retrieved_matvec(ref_blocks, 2, 2, unit(1).state_off, book, 3, x[sl])
        assert rel_max(y[sl], ref) <= 1e-12


def test_plain_6x6_matvec_vs_direct(r3m, ctx):
    """Plain path: GPU-filled c128 blocks, GPU matvec vs direct active-only Z_k x."""
    from paper_2112_05082_amd import pipeline
    states, Zk = oracle_direct(1, 6, 0)
    store = pipeline.dense_store(ctx, geom(r3m, 1), 6, r3m.C128, DEV)
    batch = batch_for(r3m, [states], [6])
    x = cb.random_complex(1440, 21)
    y = run_matvec(r3m, ctx, store, batch, to_dev(x), r3m.C128).cpu().numpy()
    assert rel_max(y, Zk @ x) <= 1e-12
    # bitwise reproducible
    y2 = run_matvec(r3m, ctx, store, batch, to_dev(x), r3m.C128).cpu().numpy()
    assert np.array_equal(y, y2)


def test_ragged_batch_sizes(r3m, ctx):
    """RHS of different (non-tile-multiple) sizes sharing one store."""
    ref_blocks = oracle_blocks(1, 2)
    store = r3m.Store(80, 2, 2, 2, 2, r3m.C128, to_dev(ref_blocks))
    L = np.array([[1, 1], [3, 2], [2, 3], [3, 3]], np.int32)
    books, uo, so = [], [], []
    u = 0
    for b, (lx, ly) in enumerate(L):
        books.append(cb.bernoulli(3, 40 + b)[: lx * ly])
        uo.append(u)
        so.append(u)
        u += lx * ly
    states = torch.from_numpy(np.concatenate(books)).to(DEV)
    batch = r3m.Batch(L, uo, so, states)
    x = cb.random_complex(u * 40, 8)
    y = run_matvec(r3m, ctx, store, batch, to_dev(x), r3m.C128).cpu().numpy()
    for b, (lx, ly) in enumerate(L):
        sl = slice(uo[b] * 40, (uo[b] + lx * ly) * 40)
        # embed the lx x ly array in the oracle's square layout
        Lsq = max(lx, ly)
        full_states = np.zeros(Lsq * Lsq, np.uint8)
        mask = np.zeros(Lsq * Lsq, bool)
        for iy in range(ly):
            for ix in range(lx):
                full_states[iy * Lsq + ix] = books[b][iy * lx + ix]
                mask[iy * Lsq + ix] = True
        xf = np.zeros((Lsq * Lsq, 40), complex)
        xf[mask] = x[sl].reshape(-1, 40)
        sub = np.zeros(((2 * Lsq - 1) ** 2, 80, 80), complex)
        for dy in range(-(Lsq - 1), Lsq):
            for dx in range(-(Lsq - 1), Lsq):
                sub[retrieval.slot(dx, dy, Lsq - 1, Lsq - 1)] = ref_blocks[retrieval.slot(dx, dy, 2, 2)]
        yf = retrieval.retrieved_matvec(sub, Lsq - 1, Lsq - 1, unit(1).state_off, full_states, Lsq,
                                        xf.reshape(-1)).reshape(-1, 40)
        assert rel_max(y[sl], yf[mask].reshape(-1)) <= 1e-12


# ----------------------------------------------------------- ACA + mixed


@pytest.fixture(scope="module")
def stores_2bit_8(r3m, ctx):
    from paper_2112_05082_amd import pipeline
    g = geom(r3m, 2)
    dense = pipeline.fill_blocks(ctx, g, 7, r3m.C128, DEV)
    s128 = pipeline.compressed_store(ctx, g, 8, 2, r3m.C128, r3m.C128, 1e-4, 40, DEV, dense_c128=dense)
    s64 = pipeline.compressed_store(ctx, g, 8, 2, r3m.C64, r3m.C64, 1e-4, 40, DEV, dense_c128=dense)
    sden = r3m.Store(160, 4, 7, 7, 7, r3m.C128, dense)
    return s128, s64, sden


def far_factors(r3m, store):
    n_far = r3m.far_count(store.Dx, store.Dy, store.near_radius)
    head = ((n_far * 4 + 255) // 256) * 256
    raw = store.far.cpu().numpy()
    es = 16 if store.far_dtype == r3m.C128 else 8
    body = raw[head: head + n_far * 2 * store.max_rank * store.n * es]
    arr = body.view(np.complex128 if es == 16 else np.complex64).reshape(n_far, 2, store.max_rank, store.n)
    return arr[:, 0].transpose(0, 2, 1), arr[:, 1].transpose(0, 2, 1)  # [f][n][r]


def test_aca_matches_oracle(r3m, ctx, stores_2bit_8):
    s128, _, sden = stores_2bit_8
    U, V = far_factors(r3m, s128)
    dense = sden.near.cpu().numpy()
    D, nr = 7, 2
    fi = 0
    checked = 0
    for dy in range(-D, D + 1):
        for dx in range(-D, D + 1):
            if max(abs(dx), abs(dy)) <= nr:
                continue
            f = fi
            fi += 1
            if f % 37 != 0:
                continue
            Zd = dense[retrieval.slot(dx, dy, D, D)]
            r = int(s128.ranks[f])
            prod = U[f][:, :r] @ V[f][:, :r].conj().T
            err = np.linalg.norm(Zd - prod) / np.linalg.norm(Zd)
            assert err <= 1e-4 * (1 + 1e-9)
            assert abs(err - s128.rel_err[f]) <= 1e-10
            Uo, Vo, erro = aca.aca_full(Zd, 1e-4, 40)
            assert abs(Uo.shape[1] - r) <= 1
            assert np.linalg.norm(prod - Uo @ Vo.conj().T) <= 2e-4 * np.linalg.norm(Zd)
            checked += 1
    assert checked >= 5


def test_compressed_matvec_c128_vs_oracle(r3m, ctx, stores_2bit_8):
    s128, _, sden = stores_2bit_8
    U, V = far_factors(r3m, s128)
    dense = sden.near.cpu().numpy()
    blocks = dense.copy()
    D, nr = 7, 2
    fi = 0
    for dy in range(-D, D + 1):
        for dx in range(-D, D + 1):
            if max(abs(dx), abs(dy)) <= nr:
                continue
            blocks[retrieval.slot(dx, dy, D, D)] = U[fi] @ V[fi].conj().T
            fi += 1
    books = [cb.uniform(8, 4, 7), cb.uniform(8, 4, 8)]
    batch = batch_for(r3m, books, [8, 8])
    x = cb.random_complex(2 * 64 * 40, 4)
    y = run_matvec(r3m, ctx, s128, batch, to_dev(x), r3m.C128).cpu().numpy()
    for b in range(2):
        sl = slice(b * 2560, (b + 1) * 2560)
        ref = retrieval.retrieved_matvec(blocks, D, D, unit(2).state_off, books[b], 8, x[sl])
        assert rel_max(y[sl], ref) <= 1e-12
    # against the uncompressed dense store: ACA error level
    yd = run_matvec(r3m, ctx, sden, batch, to_dev(x), r3m.C128).cpu().numpy()
    assert rel_l2(y, yd) <= 1e-4


def test_c64_matvec_vs_c128_same_factors(r3m, ctx, stores_2bit_8):
    s128, s64, _ = stores_2bit_8
    books = [cb.uniform(8, 4, 9)]
    batch = batch_for(r3m, books, [8])
    x = cb.random_complex(2560, 5)
    y128 = run_matvec(r3m, ctx, s128, batch, to_dev(x), r3m.C128).cpu().numpy()
    y64 = run_matvec(r3m, ctx, s64, batch, to_dev(x, torch.complex64), r3m.C64).cpu().numpy()
    assert rel_max(y64, y128) <= 1e-6
    y64d = run_matvec(r3m, ctx, s64, batch, to_dev(x), r3m.C128).cpu().numpy()
    assert rel_max(y64d, y128) <= 1e-6


# -------------------------------------------------------- solve + RCS


def test_plain_6x6_solve_and_rcs(r3m, ctx):
    from paper_2112_05082_amd import pipeline
    states, Zk = oracle_direct(1, 6, 0)
    g = geom(r3m, 1)
    store = pipeline.dense_store(ctx, g, 6, r3m.C128, DEV)
    batch = batch_for(r3m, [states], [6])
    b = torch.zeros(1440, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, g, batch, [[0.0, 0.0, 1.0]], b)
    U = oracle_rhs(1, states, 6)
    assert rel_max(b.cpu().numpy(), U) <= 1e-13
    x = torch.zeros_like(b)
    work = torch.empty(r3m.gmres_work_bytes(ctx, store, batch, 100), dtype=torch.uint8, device=DEV)
    rc, rep = r3m.r3m_gmres_solve(ctx, store, None, batch, b, x, 1e-12, 100, 1500, work)
    assert rep[0][3] and rep[0][2] <= 1e-12
    # same algorithm family as the oracle's GMRES(100): similar iteration count
    ref_it = solve.gmres(lambda v: Zk @ v, U, tol=1e-12, restart=100, max_iter=3000)
    assert abs(rep[0][0] - ref_it.iters) <= max(10, 0.05 * ref_it.iters)
    I_ref = solve.lu_solve(Zk, U)
    xs = x.cpu().numpy()
    assert rel_l2(xs, I_ref) <= 1e-8
    dirs = cb.phi0_cut(1.0)
    sig = torch.zeros(len(dirs), dtype=torch.float64, device=DEV)
    r3m.r3m_rcs(ctx, g, batch, x, dirs, 1.0, sig)
    sref = oracle_rcs(1, states, 6, I_ref, dirs)
    assert rel_l2(sig.cpu().numpy(), sref) <= 1e-8
    # same currents through both RCS codes: rounding level
    s_same = oracle_rcs(1, states, 6, xs, dirs)
    assert rel_max(sig.cpu().numpy(), s_same) <= 1e-12


@pytest.mark.parametrize("bits", [1, 2])
def test_rcs_random_currents_vs_oracle(r3m, ctx, bits):
    """Bistatic RCS of seeded random currents on three arrays (3 x 3, 5 x 5
    and 9 x 9, the last over two 64-unit tiles) at 150 seeded directions
    (three 64-direction blocks, the last ragged), 1-bit (two states) and
    2-bit (four states) units, against the oracle's far field of the same
    currents: rounding level."""
    rng = np.random.default_rng(40 + bits)
    Ls = [3, 5, 9]
    books = [cb.bernoulli(L, 7 + L) if bits == 1 else cb.uniform(L, 4, 7 + L) for L in Ls]
    g = geom(r3m, bits)
    batch = batch_for(r3m, books, Ls)
    n_a = unit(bits).n_a
    N = sum(L * L for L in Ls) * n_a
    I = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    n_dir = 150
    dirs = np.column_stack([rng.uniform(0.0, 0.5 * np.pi, n_dir), rng.uniform(0.0, 2.0 * np.pi, n_dir)])
    sig = torch.zeros(len(Ls) * n_dir, dtype=torch.float64, device=DEV)
    r3m.r3m_rcs(ctx, g, batch, to_dev(I), dirs, 1.0, sig)
    sig = sig.cpu().numpy()
    off = 0
    for b, L in enumerate(Ls):
        n = L * L * n_a
        ref = oracle_rcs(bits, books[b], L, I[off:off + n], dirs)
        assert rel_max(sig[b * n_dir:(b + 1) * n_dir], ref) <= 1e-11, (bits, L)
        off += n


def test_oblique_excitation(r3m, ctx):
    states = cb.bernoulli(3, 2)
    g = geom(r3m, 1)
    batch = batch_for(r3m, [states], [3], repeat=2)
    b = torch.zeros(2 * 360, dtype=torch.complex128, device=DEV)
    inc = [[np.deg2rad(40.0), 0.0, 1.0], [np.deg2rad(20.0), 0.3, 2.0]]
    r3m.r3m_plane_wave_rhs(ctx, g, batch, inc, b)
    got = b.cpu().numpy()
    assert rel_max(got[:360], oracle_rhs(1, states, 3, np.deg2rad(40.0), 0.0)) <= 1e-13
    assert rel_max(got[360:], 2.0 * oracle_rhs(1, states, 3, np.deg2rad(20.0), 0.3)) <= 1e-13


# ----------------------------------------------------------- error paths


def test_error_paths(r3m, ctx):
    from paper_2112_05082_amd import pipeline
    g = geom(r3m, 1)
    store = pipeline.dense_store(ctx, g, 2, r3m.C128, DEV)
    bad = r3m.Batch([[2, 2]], [0], [0], torch.tensor([0, 1, 7, 0], dtype=torch.uint8, device=DEV))
    good = r3m.Batch([[2, 2]], [0], [0], torch.tensor([0, 1, 1, 0], dtype=torch.uint8, device=DEV))
    b = torch.ones(160, dtype=torch.complex128, device=DEV)
    x = torch.zeros_like(b)
    work = torch.empty(r3m.gmres_work_bytes(ctx, store, good, 10), dtype=torch.uint8, device=DEV)
    with pytest.raises(r3m.R3MError) as e:
        r3m.r3m_gmres_solve(ctx, store, None, bad, b, x, 1e-8, 10, 50, work)
    assert e.value.code == r3m.R3M_ERR_INVALID_ARG
    bn = b.clone()
    bn[5] = complex(float("nan"), 0.0)
    with pytest.raises(r3m.R3MError) as e:
        r3m.r3m_gmres_solve(ctx, store, None, good, bn, x, 1e-8, 10, 50, work)
    assert e.value.code == r3m.R3M_ERR_NONFINITE
    rc, rep = r3m.r3m_gmres_solve(ctx, store, None, good, b, x, 1e-14, 10, 1, work, allow_not_converged=True)
    assert rc == r3m.R3M_ERR_NOT_CONVERGED and rep[0][0] == 1 and not rep[0][3]
    with pytest.raises(r3m.R3MError) as e:
        r3m.r3m_gmres_solve(ctx, store, None, good, b, x, 1e-8, 10, 50, work[:64])
    assert e.value.code == r3m.R3M_ERR_BUFFER_TOO_SMALL
    big = r3m.Batch([[3, 3]], [0], [0], torch.zeros(9, dtype=torch.uint8, device=DEV))
    with pytest.raises(r3m.R3MError) as e:
        run_matvec(r3m, ctx, store, big, torch.zeros(360, dtype=torch.complex128, device=DEV), r3m.C128)
    assert e.value.code == r3m.R3M_ERR_INVALID_ARG


def test_block_jacobi_solve_6x6(r3m, ctx):
    """Right block-Jacobi GMRES: iteration count of the oracle's preconditioned
    GMRES(100) and the LU solution."""
    from paper_2112_05082_amd import pipeline
    states, Zk = oracle_direct(1, 6, 0)
    g = geom(r3m, 1)
    store = pipeline.dense_store(ctx, g, 6, r3m.C128, DEV)
    batch = batch_for(r3m, [states], [6])
    b = torch.zeros(1440, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, g, batch, [[0.0, 0.0, 1.0]], b)
    x = torch.zeros_like(b)
    work = torch.empty(r3m.gmres_work_bytes(ctx, store, batch, 100), dtype=torch.uint8, device=DEV)
    rc, rep = r3m.r3m_gmres_solve(ctx, store, None, batch, b, x, 1e-10, 100, 1000, work,
                                  precond=r3m.PRECOND_BLOCK_JACOBI)
    U = oracle_rhs(1, states, 6)
    ref = solve.gmres(lambda v: Zk @ v, U, tol=1e-10, restart=100, max_iter=1000,
                      precond=solve.block_jacobi(Zk, 40))
    assert rep[0][3] and rep[0][2] <= 1e-10
    assert abs(rep[0][0] - ref.iters) <= max(3, 0.05 * ref.iters)
    assert rel_l2(x.cpu().numpy(), solve.lu_solve(Zk, U)) <= 1e-8


def test_mixed_refinement_to_fp64(r3m, ctx, stores_2bit_8):
    """Inner GMRES on the c64 store, outer FP64 refinement with the c128 store
    of the same factors: converges to the FP64 solution of that store."""
    s128, s64, _ = stores_2bit_8
    g = geom(r3m, 2)
    books = [cb.uniform(8, 4, 11), cb.uniform(8, 4, 12)]
    batch = batch_for(r3m, books, [8, 8])
    b = torch.zeros(2 * 2560, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, g, batch, [[0.0, 0.0, 1.0], [0.3, 0.0, 1.0]], b)
    x = torch.zeros_like(b)
    work = torch.empty(r3m.gmres_work_bytes(ctx, s64, batch, 60, s128), dtype=torch.uint8, device=DEV)
    rc, rep = r3m.r3m_gmres_solve(ctx, s64, s128, batch, b, x, 1e-4, 60, 3000, work, refine_tol=1e-10,
                                  max_refine=20, precond=r3m.PRECOND_BLOCK_JACOBI)
    assert all(r[3] and r[2] <= 1e-10 and r[1] >= 2 for r in rep)
    x64 = torch.zeros_like(b)
    work2 = torch.empty(r3m.gmres_work_bytes(ctx, s128, batch, 60), dtype=torch.uint8, device=DEV)
    r3m.r3m_gmres_solve(ctx, s128, None, batch, b, x64, 1e-11, 60, 3000, work2, precond=r3m.PRECOND_BLOCK_JACOBI)
    assert rel_l2(x.cpu().numpy(), x64.cpu().numpy()) <= 1e-8


def test_graph_replays_match_eager(r3m, ctx, stores_2bit_8):
    """Blocks of Arnoldi steps replayed from captured HIP graphs give bitwise the
    eager result, on the first capture and on later replays with eager work and
    synchronisations in between."""
    _, s64, _ = stores_2bit_8
    g = geom(r3m, 2)
    batch = batch_for(r3m, [cb.uniform(8, 4, 21)], [8])
    b = torch.zeros(2560, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, g, batch, [[0.2, 0.1, 1.0]], b)
    work = torch.empty(r3m.gmres_work_bytes(ctx, s64, batch, 20), dtype=torch.uint8, device=DEV)

    def run(eager):
        x = torch.zeros_like(b)
        _, rep = r3m.r3m_gmres_solve(ctx, s64, None, batch, b, x, 1e-6, 20, 400, work,
                                     precond=r3m.PRECOND_BLOCK_JACOBI, eager=eager)
        torch.cuda.synchronize()
        return x.cpu().numpy(), rep

    x_e, rep_e = run(True)
    for _ in range(3):
        x_g, rep_g = run(False)
        assert np.array_equal(x_g, x_e) and rep_g[0][0] == rep_e[0][0]
        # eager work in between: an unrelated matvec and a synchronisation
        run_matvec(r3m, ctx, s64, batch, b.to(torch.complex64), r3m.C64)
    x_e2, _ = run(True)
    assert np.array_equal(x_e2, x_e)


def test_tuned_group_count(r3m, ctx, stores_2bit_8):
    """The first C128 matvec on a (store, batch) tunes the displacement-group
    count; the chosen count is within the workspace bound, later calls reuse
    it (bitwise equal results), and the result stays at C64 accuracy."""
    s128, s64, _ = stores_2bit_8
    books = [cb.uniform(8, 4, 31), cb.uniform(8, 4, 32), cb.uniform(8, 4, 33)]
    batch = batch_for(r3m, books, [8, 8, 8])
    x = cb.random_complex(3 * 2560, 6)
    y1 = run_matvec(r3m, ctx, s64, batch, to_dev(x), r3m.C128).cpu().numpy()
    g = r3m.matvec_groups(ctx, s64, batch)
    assert 1 <= g <= 128
    y2 = run_matvec(r3m, ctx, s64, batch, to_dev(x), r3m.C128).cpu().numpy()
    assert np.array_equal(y1, y2)
    assert r3m.matvec_groups(ctx, s64, batch) == g
    y128 = run_matvec(r3m, ctx, s128, batch, to_dev(x), r3m.C128).cpu().numpy()
    assert rel_max(y1, y128) <= 1e-6


def test_index_ready_reuses_retrieval_index(r3m, ctx, stores_2bit_8):
    """A matvec that declares the workspace's retrieval index current gives
    bitwise the result of the call that built it; a new codebook through the
    same workspace (index rebuilt) matches the oracle product."""
    s128, s64, sden = stores_2bit_8
    x = cb.random_complex(2 * 2560, 13)
    xd = to_dev(x)
    for store in (s64, s128):
        books = [cb.uniform(8, 4, 41), cb.uniform(8, 4, 42)]
        batch = batch_for(r3m, books, [8, 8])
        wb = r3m.matvec_work_bytes(ctx, store, batch, r3m.C128)
        work = torch.empty(wb, dtype=torch.uint8, device=DEV)
        y1 = torch.zeros_like(xd)
        y2 = torch.zeros_like(xd)
        r3m.r3m_retrieved_matvec(ctx, store, batch, r3m.C128, xd, y1, work)
        r3m.r3m_retrieved_matvec(ctx, store, batch, r3m.C128, xd, y2, work, index_ready=True)
        torch.cuda.synchronize()
        assert torch.equal(y1, y2)
    # new codebook, same workspace and shapes: the index is rebuilt
    books = [cb.uniform(8, 4, 43), cb.uniform(8, 4, 44)]
    batch = batch_for(r3m, books, [8, 8])
    y3 = torch.zeros_like(xd)
    r3m.r3m_retrieved_matvec(ctx, s128, batch, r3m.C128, xd, y3, work)
    yd = run_matvec(r3m, ctx, sden, batch, xd, r3m.C128)
    torch.cuda.synchronize()
    assert rel_l2(y3.cpu().numpy(), yd.cpu().numpy()) <= 1e-4


def test_invalid_codebook_reported(r3m, ctx):
    """A state byte >= n_states is an error at the boundary, not a clamp: the
    asynchronous matvec (dense, compressed and spectral stores) leaves it for
    r3m_ctx_check; excitation, RCS and the ILU factorisation, which
    synchronise, return it themselves; the check clears it."""
    from paper_2112_05082_amd import pipeline
    g = geom(r3m, 1)
    stores = [pipeline.dense_store(ctx, g, 3, r3m.C128, DEV),
              pipeline.compressed_store(ctx, g, 3, 1, r3m.C64, r3m.C64, 1e-4, 40, DEV),
              pipeline.spectral_store(ctx, g, 3, 1, r3m.C128, DEV)]
    bad = r3m.Batch([[3, 3]], [0], [0], torch.tensor([0, 1, 0, 1, 2, 1, 0, 0, 1], dtype=torch.uint8, device=DEV))
    good = r3m.Batch([[3, 3]], [0], [0], torch.tensor([0, 1, 0, 1, 1, 1, 0, 0, 1], dtype=torch.uint8, device=DEV))
    x = torch.ones(360, dtype=torch.complex128, device=DEV)
    for st in stores:
        y = torch.zeros_like(x)
        work = torch.empty(max(r3m.matvec_work_bytes(ctx, st, bad, r3m.C128), 16), dtype=torch.uint8, device=DEV)
        r3m.r3m_retrieved_matvec(ctx, st, good, r3m.C128, x, y, work)
        r3m.r3m_ctx_check(ctx)  # a valid codebook leaves nothing
        r3m.r3m_retrieved_matvec(ctx, st, bad, r3m.C128, x, y, work)  # asynchronous: returns OK
        with pytest.raises(r3m.R3MError) as e:
            r3m.r3m_ctx_check(ctx)
        assert e.value.code == r3m.R3M_ERR_INVALID_ARG
        r3m.r3m_ctx_check(ctx)  # cleared
    with pytest.raises(r3m.R3MError) as e:
        r3m.r3m_plane_wave_rhs(ctx, g, bad, [[0.0, 0.0, 1.0]], x)
    assert e.value.code == r3m.R3M_ERR_INVALID_ARG
    sig = torch.zeros(4, dtype=torch.float64, device=DEV)
    with pytest.raises(r3m.R3MError) as e:
        r3m.r3m_rcs(ctx, g, bad, x, [[0.1, 0.0], [0.2, 0.0], [0.3, 0.0], [0.4, 0.0]], 1.0, sig)
    assert e.value.code == r3m.R3M_ERR_INVALID_ARG
    st = stores[1]
    fac = torch.empty(r3m.ilu_bytes(ctx, st, bad, 1), dtype=torch.uint8, device=DEV)
    with pytest.raises(r3m.R3MError) as e:
        r3m.r3m_ilu_factor(ctx, st, bad, 1, fac)
    assert e.value.code == r3m.R3M_ERR_INVALID_ARG
    r3m.r3m_ilu_factor(ctx, st, good, 1, fac)
    r3m.r3m_ctx_check(ctx)
