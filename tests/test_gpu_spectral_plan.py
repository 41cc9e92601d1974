"""Launch plans of the spectral matvec (r3m_matvec_plan, r3m_matvec_set_plan).

The frequency product Y^(k) = Z^(k) X^(k) has several launch shapes: the
vector-unit kernel and seven matrix-core shapes (frequencies per wave, columns
per staged chunk, 16-RHS tiles per workgroup), and the matrix-core kernel has
two workgroup orders chosen
by a live-tile threshold.  Every matrix-core shape sums each output over the
columns in the same order (16x16x4 tiles of four consecutive columns, in
increasing column order) and the order only decides which workgroup computes
a tile, so matvecs and whole solves must agree bit for bit across shapes and
orders; the vector-unit shape sums in another FP32 order (relative 1e-6 on a
matvec).  Also: the autotuned plan is valid, a pinned plan is what the query
returns, and plans that do not fit the store are refused.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_common import FREQ, rel_max, unit  # noqa: E402
from workloads import codebooks as cb  # noqa: E402

DEV = "cuda:0"
MFMA_SHAPES = (1, 2, 3, 4, 5, 6, 7)


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


def test_matvec_identical_across_shapes(lib):
    """40 right-hand sides (three 16-RHS tiles, the last ragged) at 12 x 12."""
    r3m, pipeline, ctx, geom = lib
    L, B = 12, 40
    spec = pipeline.spectral_store(ctx, geom, L, 2, r3m.C64, DEV)
    books = [cb.family(b % 3, L, 7100 + b) for b in range(B)]
    batch = r3m.Batch.from_codebooks(books, [L] * B, DEV)
    n1 = L * L * 40
    x = torch.from_numpy(cb.random_complex(B * n1, 71)).to(DEV)
    work = torch.empty(r3m.matvec_work_bytes(ctx, spec, batch, r3m.C128), dtype=torch.uint8, device=DEV)

    def mv():
        y = torch.zeros_like(x)
        r3m.r3m_retrieved_matvec(ctx, spec, batch, r3m.C128, x, y, work)
        torch.cuda.synchronize()
        return y

    y_tuned = mv()
    tuned = r3m.matvec_plan(ctx, spec, batch)
    info = r3m.decode_plan(tuned)
    print(f"tuned spectral plan for {B} RHS at {L}x{L}: {info}")
    assert info["kind"] == "spectral" and 0 <= info["shape"] < len(r3m.SPEC_SHAPES) and info["rhs_first"] >= 1
    ref = None
    for shape in MFMA_SHAPES:
        for rf, lkg in ((1, 0), (2, 0), (8, 0), (255, 0), (1, 1), (1, 2), (1, 3)):
            r3m.matvec_set_plan(ctx, spec, batch, r3m.spec_plan(shape, rf, kt_groups=lkg))
            assert r3m.matvec_plan(ctx, spec, batch) == r3m.spec_plan(shape, rf, kt_groups=lkg)
            y = mv()
            if ref is None:
                ref = y
            assert torch.equal(y, ref), (shape, rf)
    if info["mfma"]:
        assert torch.equal(y_tuned, ref)
    r3m.matvec_set_plan(ctx, spec, batch, r3m.spec_plan(0, 8))
    yv = mv()
    err = rel_max(yv.cpu().numpy(), ref.cpu().numpy())
    print(f"vector-unit vs matrix-core frequency product: max relative difference {err:.1e}")
    assert err <= 1e-6


def test_solve_identical_across_shapes(lib):
    """An unrefined complex64-spectra solve of 48 right-hand sides at 8 x 8
    with staggered convergence and a 16-RHS tile idle from the start (so the
    device-built live-tile list shrinks during the solve and both workgroup
    orders are taken): iterations and solutions agree bit for bit across
    matrix-core shapes and thresholds."""
    r3m, pipeline, ctx, geom = lib
    L, n_books = 8, 12
    angles = (0.0, 20.0, 40.0, 60.0)
    books = [cb.family(c % 3, L, 7300 + c) for c in range(n_books)]
    batch = r3m.Batch.from_codebooks(books, [L] * n_books, DEV, repeat=len(angles))
    B = batch.B
    n1 = L * L * 40
    spec = pipeline.spectral_store(ctx, geom, L, 2, r3m.C64, DEV)
    b = torch.zeros(B * n1, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, geom, batch, [[np.deg2rad(a), 0.0, 1.0] for _ in range(n_books) for a in angles], b)
    b[16 * n1:32 * n1] = 0
    restart = 8
    work = torch.empty(r3m.gmres_work_bytes(ctx, spec, batch, restart), dtype=torch.uint8, device=DEV)

    def solve(plan):
        r3m.matvec_set_plan(ctx, spec, batch, plan)
        x = torch.zeros_like(b)
        rc, rep = r3m.r3m_gmres_solve(ctx, spec, None, batch, b, x, 1e-5, restart, 4000, work,
                                      precond=r3m.PRECOND_BLOCK_JACOBI)
        torch.cuda.synchronize()
        assert rc == 0 and all(r[3] for r in rep)
        return x, [r[0] for r in rep]

    x0, it0 = solve(r3m.spec_plan(2, 8))
    assert all(it0[r] == 0 for r in range(16, 32)) and len(set(it0)) >= 4, it0
    for shape in MFMA_SHAPES:
        for rf, lkg in ((1, 0), (2, 0), (255, 0), (1, 2), (2, 3)):
            x, its = solve(r3m.spec_plan(shape, rf, kt_groups=lkg))
            assert its == it0, (shape, rf, lkg)
            assert torch.equal(x, x0), (shape, rf, lkg)
    xv, itv = solve(r3m.spec_plan(0, 8))
    d = float((xv - x0).abs().max()) / float(x0.abs().max())
    print(f"solve, 48 RHS: iterations {min(it0)}..{max(it0)}; vector-unit product: iteration difference "
          f"{max(abs(a - c) for a, c in zip(itv, it0))}, relative solution difference {d:.1e}")
    assert d <= 1e-3


def test_plan_validation(lib):
    r3m, pipeline, ctx, geom = lib
    L = 4
    s128 = pipeline.spectral_store(ctx, geom, L, 2, r3m.C128, DEV)
    s64 = pipeline.spectral_store(ctx, geom, L, 2, r3m.C64, DEV)
    comp = pipeline.compressed_store(ctx, geom, L, 1, r3m.C128, r3m.C128, 1e-4, 40, DEV)
    batch = r3m.Batch.from_codebooks([cb.uniform(L, 2, 1)], [L], DEV)
    bad = [(s128, r3m.spec_plan(2, 8)),        # matrix cores need complex64 spectra
           (s64, r3m.spec_plan(len(r3m.SPEC_SHAPES), 8)),  # no such shape
           (s64, r3m.spec_plan(1, 0)),         # threshold below 1
           (s64, 4),                           # a compressed-store plan
           (comp, r3m.spec_plan(0, 8)),        # a spectral plan on a compressed store
           (comp, 0),                          # zero groups
           (comp, 1 << 20)]                    # unknown bit
    for store, plan in bad:
        with pytest.raises(r3m.R3MError):
            r3m.matvec_set_plan(ctx, store, batch, plan)
    r3m.matvec_set_plan(ctx, s128, batch, r3m.spec_plan(0, 3))
    assert r3m.matvec_plan(ctx, s128, batch) == r3m.spec_plan(0, 3)
    r3m.matvec_set_plan(ctx, comp, batch, 1)
    assert r3m.matvec_plan(ctx, comp, batch) == 1 and r3m.matvec_groups(ctx, comp, batch) == 1
    # the default of an untuned pair: vector units for one right-hand side
    batch2 = r3m.Batch.from_codebooks([cb.uniform(L, 2, 2)], [L], DEV)
    assert r3m.decode_plan(r3m.matvec_plan(ctx, s64, batch2)) == {
        "kind": "spectral", "shape": 0, "mfma": False, "kpw": 0, "pc": 0, "rhs_tiles": 0, "rhs_first": 8,
        "two_pass": False, "kt_groups": 0}


@pytest.mark.parametrize("L", [2, 4, 8, 12, 24, 40])
def test_fused_transforms_match_two_pass(lib, L):
    """The fused 2-D transforms (one grid per workgroup in LDS) against the
    two-pass ones on the same store: transform grids from 4 x 4 to 128 x 128
    (one to three stages per direction, every radix), arrays smaller than the
    store's extent and rectangular ones (rows gy >= Ly and columns gx >= Lx of
    a grid are zero), complex128 and complex64 vectors."""
    r3m, pipeline, ctx, geom = lib
    spec = pipeline.spectral_store(ctx, geom, L, 2, r3m.C64, DEV)
    shapes = [(L, L), (max(1, L // 2), L), (L, max(1, L - 3)), (1, 1), (L, L)]
    rng = np.random.default_rng(900 + L)
    books = [rng.integers(0, 2, lx * ly).astype(np.uint8) for lx, ly in shapes]
    uoff = np.cumsum([0] + [lx * ly for lx, ly in shapes])[:-1].tolist()
    batch = r3m.Batch(shapes, uoff, uoff, torch.from_numpy(np.concatenate(books)).to(DEV))
    n1 = sum(lx * ly for lx, ly in shapes) * 40
    x = torch.from_numpy(cb.random_complex(n1, 77 + L)).to(DEV)
    worst = 0.0
    for vt, xv in ((r3m.C128, x), (r3m.C64, x.to(torch.complex64))):
        work = torch.empty(r3m.matvec_work_bytes(ctx, spec, batch, vt), dtype=torch.uint8, device=DEV)
        ys = []
        for two_pass in (False, True):
            r3m.matvec_set_plan(ctx, spec, batch, r3m.spec_plan(0, 8, two_pass))
            y = torch.zeros_like(xv)
            r3m.r3m_retrieved_matvec(ctx, spec, batch, vt, xv, y, work)
            torch.cuda.synchronize()
            ys.append(y.to(torch.complex128).cpu().numpy())
        assert np.abs(ys[0]).max() > 0
        worst = max(worst, rel_max(ys[0], ys[1]))
    print(f"{L}x{L} store: fused vs two-pass transforms, max relative difference {worst:.1e}")
    assert worst <= 1e-6


def test_fused_transforms_row_major_copies(lib):
    """A batch wide enough (about 1.2 M compact entries) for the fused
    transforms to gather from and scatter to row-major copies of x and y:
    against the two-pass transforms on the same store and product plan, with
    ragged arrays and one 1 x 1 array, complex128 and complex64 vectors."""
    r3m, pipeline, ctx, geom = lib
    L = 24
    spec = pipeline.spectral_store(ctx, geom, L, 2, r3m.C64, DEV)
    shapes = [(L, L), (L // 2, L), (L, L - 3), (1, 1)] * 20
    rng = np.random.default_rng(4242)
    books = [rng.integers(0, 2, lx * ly).astype(np.uint8) for lx, ly in shapes]
    uoff = np.cumsum([0] + [lx * ly for lx, ly in shapes])[:-1].tolist()
    batch = r3m.Batch(shapes, uoff, uoff, torch.from_numpy(np.concatenate(books)).to(DEV))
    n1 = sum(lx * ly for lx, ly in shapes) * 40
    assert n1 >= 1 << 20
    x = torch.from_numpy(cb.random_complex(n1, 4243)).to(DEV)
    worst = 0.0
    for vt, xv in ((r3m.C128, x), (r3m.C64, x.to(torch.complex64))):
        work = torch.empty(r3m.matvec_work_bytes(ctx, spec, batch, vt), dtype=torch.uint8, device=DEV)
        ys = []
        for two_pass in (False, True):
            r3m.matvec_set_plan(ctx, spec, batch, r3m.spec_plan(6, 64, two_pass))
            y = torch.zeros_like(xv)
            r3m.r3m_retrieved_matvec(ctx, spec, batch, vt, xv, y, work)
            torch.cuda.synchronize()
            ys.append(y.to(torch.complex128).cpu().numpy())
        assert np.abs(ys[0]).max() > 0
        worst = max(worst, rel_max(ys[0], ys[1]))
    print(f"wide batch ({n1} entries): fused transforms with row-major copies vs two-pass, "
          f"max relative difference {worst:.1e}")
    assert worst <= 1e-6
