"""Connected geometries on the GPU (Sec. III-B, basis extension of periodic
boundaries): coding patches over a ground plane meshed as a connected patch
array, each unit owning the bridging bases of its -x and -y cell edges.

* fill: the extended macro unit's blocks Z(d) (bridging triangles in the
  neighbouring cells, extraction by the triangles' own cells) against the
  oracle's, 1e-11;
* matvec on spectral stores with the shared ground bases and the D_k masks
  of the extended bases: against the oracle's retrieval from its own blocks
  (itself pinned by the system computed on the physical structure), 1e-12
  on complex128 spectra and 2e-6 on complex64 (FP32 transforms and
  products); masked entries of the output are exactly zero and masked input
  entries are ignored; arrays smaller than the store, rectangular ones, four
  codebooks in one batch; the fused and the two-pass transforms;
* excitation, unpreconditioned GMRES (complex128 spectra; complex64 inner
  solves with complex128 refinement) and RCS on connected arrays against the
  oracle's retrieved pipeline (itself pinned against the physical structure):
  excitation 1e-13 with zeros on the masked bases, RCS 1e-7 and 1e-6;
* the calls that do not take shared bases yet refuse them.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_common import FREQ, K, rel_max  # noqa: E402
from oracle import connected  # noqa: E402
from workloads import codebooks as cb  # noqa: E402
from workloads.mesh import connected_unit  # noqa: E402

DEV = "cuda:0"
L = 3
D = L - 1


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_05082_amd import pipeline, r3m
    r3m.load()
    ctx = r3m.Context(0)
    cu = connected_unit((0.006, 0.009))
    geom = r3m.UnitGeom.from_connected(cu, FREQ, 1)
    ref_blocks = connected.displacement_blocks(cu, D, D, K, extract=1)
    yield r3m, pipeline, ctx, cu, geom, ref_blocks
    ctx.close()


def shapes_and_books(cu):
    rng = np.random.default_rng(77)
    shapes = [(3, 3), (3, 3), (3, 2), (2, 2), (1, 1)]
    books = [np.zeros(9, np.uint8), rng.integers(0, 2, 9).astype(np.uint8),
             np.array([0, 1, 0, 1, 0, 1], np.uint8), np.ones(4, np.uint8), np.ones(1, np.uint8)]
    return shapes, books


def compact_index(cu, u_off, idx):
    """Compact positions (n_a state rows, then the shared rows) of macro indices."""
    n_st = int(cu.state_off[-1])
    n_red = cu.n_a + cu.n_common
    out = []
    for m in idx:
        out.append(u_off * n_red + (m % cu.n_a if m < n_st else cu.n_a + m - n_st))
    return np.asarray(out, dtype=np.int64)


def test_fill_matches_oracle(setup):
    r3m, pipeline, ctx, cu, geom, ref = setup
    blocks = pipeline.fill_blocks(ctx, geom, D, r3m.C128, DEV).cpu().numpy()
    assert blocks.shape == ref.shape and blocks.shape[1] == 128
    worst = max(rel_max(blocks[s], ref[s]) for s in range(ref.shape[0]))
    print(f"connected unit fill (n = 128, 25 blocks): worst relative error {worst:.1e}")
    assert worst <= 1e-11


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-12), ("c64", 2e-6)])
def test_matvec_matches_oracle(setup, dtype, tol):
    r3m, pipeline, ctx, cu, geom, ref = setup
    dt = r3m.C128 if dtype == "c128" else r3m.C64
    store = pipeline.spectral_store(ctx, geom, L, 1, dt, DEV)
    assert store.n_common == 48
    shapes, books = shapes_and_books(cu)
    uoff = np.cumsum([0] + [a * b for a, b in shapes])[:-1]
    batch = r3m.Batch(shapes, uoff, uoff, torch.from_numpy(np.concatenate(books)).to(DEV))
    n_red = cu.n_a + cu.n_common
    N = int(uoff[-1] + shapes[-1][0] * shapes[-1][1]) * n_red
    x = cb.random_complex(N, 123)  # masked entries carry values too: they must be ignored
    xd = torch.from_numpy(x).to(DEV)
    vt = r3m.C128
    plans = [None] if dt == r3m.C128 else [r3m.spec_plan(0, 8), r3m.spec_plan(0, 8, True)]
    for plan in plans:
        if plan is not None:
            r3m.matvec_set_plan(ctx, store, batch, plan)
        y = torch.full_like(xd, complex(7.0, 7.0))  # masked outputs must be overwritten with zero
        work = torch.empty(r3m.matvec_work_bytes(ctx, store, batch, vt), dtype=torch.uint8, device=DEV)
        r3m.r3m_retrieved_matvec(ctx, store, batch, vt, xd, y, work)
        torch.cuda.synchronize()
        y = y.cpu().numpy()
        worst = 0.0
        for b, ((lx, ly), book) in enumerate(zip(shapes, books)):
            active = connected.active_sets(cu, book, lx, ly)
            pos = np.concatenate([compact_index(cu, int(uoff[b]) + u, a) for u, a in enumerate(active)])
            y_ref = connected.retrieved_matvec(ref, D, D, active, lx, ly, x[pos])
            worst = max(worst, rel_max(y[pos], y_ref))
            rows = np.arange(int(uoff[b]) * n_red, int(uoff[b] + lx * ly) * n_red)
            masked = np.setdiff1d(rows, pos)
            # the extended bases of the first column and row, and nothing else
            assert len(masked) == 4 * (lx + ly), (b, len(masked))
            assert np.all(y[masked] == 0)
        print(f"connected {dtype} matvec (plan {plan}): worst relative error vs oracle {worst:.1e}")
        assert worst <= tol


def test_unsupported_calls_refuse_shared_bases(setup):
    r3m, pipeline, ctx, cu, geom, ref = setup
    store = pipeline.spectral_store(ctx, geom, L, 1, r3m.C64, DEV)
    batch = r3m.Batch([(3, 3)], [0], [0], torch.zeros(9, dtype=torch.uint8, device=DEV))
    # preconditioned solves: the size query answers 0 and names the reason
    assert r3m.gmres_work_bytes(ctx, store, batch, 10) > 0
    assert r3m.gmres_work_bytes(ctx, store, batch, 10, precond=r3m.PRECOND_BLOCK_JACOBI) == 0
    assert "shared" in r3m.load().r3m_last_error(ctx.handle).decode()
    # a bridge reaching into the +x neighbour has no extension class
    tc = cu.tri_cell.copy()
    t = int(np.nonzero(tc[:, 0] == -1)[0][0])
    tc[t, 0] = 1
    odd = r3m.UnitGeom(cu.vert, cu.tri, cu.rwg, cu.state_off, FREQ, cu.period, 1, tc, cu.ext)
    b = torch.zeros(9 * 88, dtype=torch.complex128, device=DEV)
    with pytest.raises(r3m.R3MError):
        r3m.r3m_plane_wave_rhs(ctx, odd, batch, [[0.0, 0.0, 1.0]], b)
    assert "-x or the -y" in r3m.load().r3m_last_error(ctx.handle).decode()
    # a compressed store with shared bases
    bad = r3m.Store(store.n, 2, D, D, 1, r3m.C64, store.near, common_ext=store.common_ext)
    x = torch.zeros(9 * 88, dtype=torch.complex64, device=DEV)
    with pytest.raises(r3m.R3MError):
        r3m.r3m_retrieved_matvec(ctx, bad, batch, r3m.C64, x, x.clone(), torch.empty(16, dtype=torch.uint8,
                                                                                       device=DEV))


def test_solve_and_rcs_match_oracle(setup):
    """Five codebooks (3x3, 3x3, 3x2, 2x2, 1x1) at two incidence angles (0 and
    30 degrees, theta polarisation) in one batch on the store for 3x3: the
    plane-wave excitation against the oracle's (every basis over its own
    triangles, zero on the masked bases), then GMRES without preconditioner
    and the RCS of each right-hand side against the oracle's LU solution of
    the retrieved system (RCS over a 10-degree phi = 0 cut, relative L2)."""
    import math

    from oracle import solve
    r3m, pipeline, ctx, cu, geom, ref = setup
    shapes, books = shapes_and_books(cu)
    thetas = (0.0, math.radians(30.0))
    n_red = cu.n_a + cu.n_common
    # RHS r = 2 c + a: codebook c at angle a; the two angles share the codebook's states
    units = [lx * ly for lx, ly in shapes]
    soff = np.cumsum([0] + units)[:-1]
    rshapes = [shapes[c] for c in range(len(shapes)) for _ in thetas]
    rsoff = [int(soff[c]) for c in range(len(shapes)) for _ in thetas]
    ruoff = np.cumsum([0] + [units[c] for c in range(len(shapes)) for _ in thetas])
    batch = r3m.Batch(rshapes, ruoff[:-1], rsoff, torch.from_numpy(np.concatenate(books)).to(DEV))
    B = batch.B
    N = int(ruoff[-1]) * n_red
    inc = [[th, 0.0, 1.0] for _ in shapes for th in thetas]
    b = torch.zeros(N, dtype=torch.complex128, device=DEV)
    r3m.r3m_plane_wave_rhs(ctx, geom, batch, inc, b)
    dirs = cb.phi0_cut(10.0)
    s128 = pipeline.spectral_store(ctx, geom, L, 1, r3m.C128, DEV)
    s64 = pipeline.spectral_store(ctx, geom, L, 1, r3m.C64, DEV)
    torch.cuda.synchronize()
    bh = b.cpu().numpy()
    refs = []
    worst_b = 0.0
    for r in range(B):
        c = r // 2
        lx, ly = shapes[c]
        active = connected.active_sets(cu, books[c], lx, ly)
        pos = np.concatenate([compact_index(cu, int(ruoff[r]) + u, a) for u, a in enumerate(active)])
        Ur = connected.excitation(cu, active, lx, ly, K, thetas[r % 2], 0.0)
        worst_b = max(worst_b, np.abs(bh[pos] - Ur).max() / np.abs(Ur).max())
        rows = np.arange(int(ruoff[r]) * n_red, int(ruoff[r + 1]) * n_red)
        assert np.all(bh[np.setdiff1d(rows, pos)] == 0)
        Ir = solve.lu_solve(connected.retrieved_system(ref, D, D, active, lx, ly), Ur)
        refs.append(connected.rcs(cu, active, lx, ly, Ir, K, dirs))
    print(f"connected excitation vs oracle: {worst_b:.1e}")
    assert worst_b <= 1e-13

    def solve_and_rcs(store, store64, tol, refine_tol):
        x = torch.zeros_like(b)
        work = torch.empty(r3m.gmres_work_bytes(ctx, store, batch, 100, store64), dtype=torch.uint8, device=DEV)
        _, rep = r3m.r3m_gmres_solve(ctx, store, store64, batch, b, x, tol, 100, 4000, work,
                                     refine_tol=refine_tol, max_refine=10 if store64 is not None else 0)
        sig = torch.zeros(B * len(dirs), dtype=torch.float64, device=DEV)
        r3m.r3m_rcs(ctx, geom, batch, x, dirs, 1.0, sig)
        torch.cuda.synchronize()
        sig = sig.cpu().numpy().reshape(B, -1)
        errs = [np.linalg.norm(sig[r] - refs[r]) / np.linalg.norm(refs[r]) for r in range(B)]
        return rep, errs

    rep, errs = solve_and_rcs(s128, None, 1e-10, 0.0)
    print(f"connected complex128 GMRES: iterations {[q[0] for q in rep]}, RCS errors max {max(errs):.1e}")
    assert all(q[3] for q in rep) and max(errs) <= 1e-7
    rep, errs = solve_and_rcs(s64, s128, 1e-3, 1e-10)
    print(f"connected complex64 inner + complex128 refinement: iterations {[q[0] for q in rep]}, "
          f"steps {[q[1] for q in rep]}, RCS errors max {max(errs):.1e}")
    assert all(q[3] for q in rep) and max(errs) <= 1e-6
