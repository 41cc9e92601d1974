"""Relaxed (blended) retrieval on the GPU against the oracle.

The relaxed operator Z_k(w) = P(w)^T Z P(w) (state weights per unit, the
operator of codebook differentiation) and its transpose P(w)^T Z^T P(w) (the
adjoint solve's operator), on spectral stores:
  * oracle blocks uploaded, 3 x 3 arrays, random and one-hot weights, 2 RHS
    and 15 RHS (the latter takes the matrix-core product), both operators:
    element-wise against the oracle's matrix form, 1e-12 (complex128
    spectra) and 2e-6 (complex64), the tolerances of the plain spectral path;
  * 2-bit 32 x 32: one-hot weights give the standard retrieved product
    bitwise (weights 1 and 0 are exact), and the transpose satisfies
    y^T (A x) = (A^T y)^T x for random weights to 1e-12 (complex128 spectra).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_common import FREQ, K, rel_max, unit  # noqa: E402
from oracle import efie, ilu, relaxed, retrieval, solve  # noqa: E402
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


def relaxed_mv(r3m, ctx, store, batch, w, x, vt, transpose):
    y = torch.zeros_like(x)
    work = torch.empty(r3m.relaxed_work_bytes(ctx, store, batch), dtype=torch.uint8, device=DEV)
    r3m.r3m_relaxed_matvec(ctx, store, batch, w, vt, x, y, work, transpose=transpose)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("dtype,tol,nrhs", [("c128", 1e-12, 2), ("c64", 2e-6, 2), ("c64", 2e-6, 15),
                                            ("c128", 1e-12, 15)])
def test_relaxed_vs_oracle(lib, dtype, tol, nrhs):
    r3m, _, ctx = lib
    L, D = 3, 2
    blocks = efie.displacement_blocks(unit(1), D, D, K, extract=1)
    st = r3m.C128 if dtype == "c128" else r3m.C64
    tdt = torch.complex128 if st == r3m.C128 else torch.complex64
    sd = r3m.SPEC_C64 if st == r3m.C64 else r3m.SPEC_C128
    spec = torch.empty(r3m.spectral_bytes(80, D, D, sd), dtype=torch.uint8, device=DEV)
    r3m.r3m_build_spectral(ctx, to_dev(blocks), 80, D, D, sd, spec)
    store = r3m.Store(80, 2, D, D, 0, st, to_dev(blocks[retrieval.slot(0, 0, D, D)][None], tdt), sd, spec)
    rng = np.random.default_rng(40 + nrhs)
    W = rng.random((nrhs, L * L, 2))
    W[0, :4] = np.eye(2)[rng.integers(0, 2, 4)]  # some one-hot units
    batch = r3m.Batch.from_codebooks([np.zeros(L * L, np.uint8)] * nrhs, [L] * nrhs, DEV)
    x = cb.random_complex(nrhs * L * L * 40, 41)
    xd = to_dev(x, tdt)
    if st == r3m.C64:
        x = x.astype(np.complex64).astype(np.complex128)
    wd = torch.from_numpy(W.reshape(-1, 2)).to(DEV)
    worst = 0.0
    for tr in (False, True):
        y = relaxed_mv(r3m, ctx, store, batch, wd, xd, st, tr)
        for b in range(nrhs):
            sl = slice(b * L * L * 40, (b + 1) * L * L * 40)
            ref = relaxed.relaxed_matvec(blocks, D, D, unit(1).state_off, W[b], L, x[sl], transpose=tr)
            worst = max(worst, rel_max(y[sl], ref))
    print(f"relaxed {dtype}, {nrhs} RHS, both operators: worst element error {worst:.2e}")
    assert worst <= tol


@pytest.fixture(scope="module")
def full(lib):
    r3m, pipeline, ctx = lib
    geom = r3m.UnitGeom.from_macro(unit(2), FREQ, 1)
    states = cb.uniform(32, 4, 1)
    batch = r3m.Batch.from_codebooks([states], [32], DEV)
    dense = pipeline.fill_blocks(ctx, geom, 31, r3m.C128, DEV)
    s64 = pipeline.spectral_store(ctx, geom, 32, 2, r3m.C64, DEV, dense_c128=dense)
    s128 = pipeline.spectral_store(ctx, geom, 32, 2, r3m.C128, DEV, dense_c128=dense)
    yield states, batch, s64, s128


def test_relaxed_one_hot_is_retrieval_fullsize(lib, full):
    r3m, _, ctx = lib
    states, batch, s64, _ = full
    w = np.zeros((32 * 32, 4))
    w[np.arange(32 * 32), states] = 1.0
    x = to_dev(cb.random_complex(32 * 32 * 40, 42))
    y_rel = relaxed_mv(r3m, ctx, s64, batch, torch.from_numpy(w).to(DEV), x, r3m.C128, False)
    y = torch.zeros_like(x)
    work = torch.empty(r3m.matvec_work_bytes(ctx, s64, batch, r3m.C128), dtype=torch.uint8, device=DEV)
    r3m.r3m_retrieved_matvec(ctx, s64, batch, r3m.C128, x, y, work)
    torch.cuda.synchronize()
    assert np.array_equal(y_rel, y.cpu().numpy())


def test_relaxed_transpose_identity_fullsize(lib, full):
    r3m, _, ctx = lib
    _, batch, _, s128 = full
    rng = np.random.default_rng(43)
    logits = rng.standard_normal((32 * 32, 4))
    w = np.exp(logits) / np.exp(logits).sum(axis=1, keepdims=True)  # softmax blend
    wd = torch.from_numpy(w).to(DEV)
    x = to_dev(cb.random_complex(32 * 32 * 40, 44))
    y = to_dev(cb.random_complex(32 * 32 * 40, 45))
    ax = relaxed_mv(r3m, ctx, s128, batch, wd, x, r3m.C128, False)
    aty = relaxed_mv(r3m, ctx, s128, batch, wd, y, r3m.C128, True)
    ay = relaxed_mv(r3m, ctx, s128, batch, wd, y, r3m.C128, False)
    xn, yn = x.cpu().numpy(), y.cpu().numpy()
    lhs, rhs, plain = yn @ ax, aty @ xn, ay @ xn
    print(f"32x32 relaxed: |y^T A x - (A^T y)^T x| / |y^T A x| = {abs(lhs - rhs) / abs(lhs):.2e}, "
          f"without the transpose {abs(plain - lhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    assert abs(plain - lhs) > 1e-9 * abs(lhs)


@pytest.mark.parametrize("transpose,precond", [(False, 0), (True, 0), (False, 1), (True, 1), (False, 2), (True, 2)])
def test_relaxed_solve_vs_oracle_lu(lib, transpose, precond):
    """GMRES on the relaxed operator (and on its transpose, the adjoint solve)
    against dense LU on the oracle's relaxed matrix, 3 x 3 x 2 RHS, complex128
    spectra, GMRES to 1e-12, without preconditioner, with the block-Jacobi of
    the blended self blocks and with the block ILU(0) (radius 1) of the
    blended near field: solutions within 1e-8 (cond x 1e-12); with the ILU,
    iterations within 10% of the oracle's ILU GMRES on the same matrix."""
    r3m, _, ctx = lib
    L, D = 3, 2
    blocks = efie.displacement_blocks(unit(1), D, D, K, extract=1)
    spec = torch.empty(r3m.spectral_bytes(80, D, D, r3m.SPEC_C128), dtype=torch.uint8, device=DEV)
    r3m.r3m_build_spectral(ctx, to_dev(blocks), 80, D, D, r3m.SPEC_C128, spec)
    if precond == r3m.PRECOND_BLOCK_ILU:  # near blocks of every |d| <= 2
        store = r3m.Store(80, 2, D, D, D, r3m.C128, to_dev(blocks), r3m.SPEC_C128, spec)
    else:
        store = r3m.Store(80, 2, D, D, 0, r3m.C128, to_dev(blocks[retrieval.slot(0, 0, D, D)][None]),
                          r3m.SPEC_C128, spec)
    rng = np.random.default_rng(50)
    logits = rng.standard_normal((2, L * L, 2))
    W = np.exp(logits) / np.exp(logits).sum(axis=2, keepdims=True)
    batch = r3m.Batch.from_codebooks([np.zeros(L * L, np.uint8)] * 2, [L] * 2, DEV)
    bvec = cb.random_complex(2 * L * L * 40, 51)
    bd = to_dev(bvec)
    x = torch.zeros_like(bd)
    work = torch.empty(r3m.gmres_work_bytes(ctx, store, batch, 60, relaxed=True, precond=precond),
                       dtype=torch.uint8, device=DEV)
    _, rep = r3m.r3m_gmres_solve(ctx, store, None, batch, bd, x, 1e-12, 60, 4000, work,
                                 relaxed_weights=torch.from_numpy(W.reshape(-1, 2)).to(DEV), transpose=transpose,
                                 precond=precond)
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    Zm = retrieval.macro_matrix(blocks, D, D, L)
    errs, oracle_iters = [], []
    for b in range(2):
        P = relaxed.blend_matrix(W[b], unit(1).state_off, L)
        A = P.T @ (Zm.T if transpose else Zm) @ P
        sl = slice(b * L * L * 40, (b + 1) * L * L * 40)
        ref = np.linalg.solve(A, bvec[sl])
        errs.append(np.linalg.norm(x[sl] - ref) / np.linalg.norm(ref))
        if precond == r3m.PRECOND_BLOCK_ILU:
            f = ilu.block_ilu0(A, L, L, 40, 1)
            oracle_iters.append(solve.gmres(lambda v: A @ v, bvec[sl], 1e-12, 60, 4000,
                                            precond=lambda v: ilu.ilu_apply(f, v)).iters)
    print(f"relaxed solve (transpose={transpose}, precond={precond}): iters {[r[0] for r in rep]}, errors vs LU "
          f"{['%.2e' % e for e in errs]}, oracle ILU iters {oracle_iters}")
    assert all(r[3] for r in rep) and max(errs) <= 1e-8
    for r, o in zip(rep, oracle_iters):
        assert abs(r[0] - o) <= max(3, 0.1 * o)


def test_relaxed_objective_and_gradient_vs_oracle(lib):
    """Objective J = mean RCS over a 30-degree cone of the blended current and
    its adjoint gradient dJ/dw, 2-bit 2 x 2 arrays x 2 RHS, complex128
    spectra, GMRES to 1e-12: J and sigma within 1e-9, gradient within 1e-7 of
    its largest entry, against the oracle (dense LU; gradient pinned by
    finite differences of the oracle's J)."""
    from paper_2112_05082_amd.relaxed import RelaxedRcs
    r3m, _, ctx = lib
    L, D = 2, 1
    u2 = unit(2)
    blocks = efie.displacement_blocks(u2, D, D, K, extract=1)
    spec = torch.empty(r3m.spectral_bytes(160, D, D, r3m.SPEC_C128), dtype=torch.uint8, device=DEV)
    r3m.r3m_build_spectral(ctx, to_dev(blocks), 160, D, D, r3m.SPEC_C128, spec)
    store = r3m.Store(160, 4, D, D, 0, r3m.C128, to_dev(blocks[retrieval.slot(0, 0, D, D)][None]), r3m.SPEC_C128,
                      spec)
    geom = r3m.UnitGeom.from_macro(u2, FREQ, 1)
    rng = np.random.default_rng(60)
    logits = rng.standard_normal((2, L * L, 4))
    W = np.exp(logits) / np.exp(logits).sum(axis=2, keepdims=True)
    batch = r3m.Batch.from_codebooks([np.zeros(L * L, np.uint8)] * 2, [L] * 2, DEV)
    dirs = cb.cone16(30.0)
    obj = RelaxedRcs(ctx, geom, store, batch, [[0.0, 0.0, 1.0]] * 2, dirs, tol=1e-12)
    wd = torch.from_numpy(W.reshape(-1, 4)).to(DEV)
    J, sigma, I, G, adj = obj.forward_parts(wd)
    grad = obj.gradient(wd, I, G, adj).cpu().numpy().reshape(2, L * L, 4)
    J, sigma = J.cpu().numpy(), sigma.cpu().numpy()
    for b in range(2):
        Jr, sr, _, gr = relaxed.relaxed_objective(u2, blocks, D, W[b], L, K, dirs, with_grad=True)
        eJ, es = abs(J[b] - Jr) / abs(Jr), rel_max(sigma[b], sr)
        eg = np.abs(grad[b] - gr).max() / np.abs(gr).max()
        print(f"relaxed objective RHS {b}: J {J[b]:.6e} (err {eJ:.1e}), sigma err {es:.1e}, gradient err {eg:.1e}")
        assert eJ <= 1e-9 and es <= 1e-9 and eg <= 1e-7


def test_relaxed_autograd_matches_finite_differences_8x8(lib):
    """The differentiation workload at 8 x 8: 2-bit units, softmax logits
    ~N(0,1) (seed 3), J = mean RCS over 16 directions in a 30-degree cone;
    torch autograd through the relaxed objective against central differences
    (h = 1e-4 on the logits) along three random directions, within 1e-5."""
    from paper_2112_05082_amd import pipeline
    from paper_2112_05082_amd.relaxed import RelaxedRcs
    r3m, _, ctx = lib
    L = 8
    geom = r3m.UnitGeom.from_macro(unit(2), FREQ, 1)
    store = pipeline.spectral_store(ctx, geom, L, 0, r3m.C128, DEV)
    batch = r3m.Batch.from_codebooks([np.zeros(L * L, np.uint8)], [L], DEV)
    obj = RelaxedRcs(ctx, geom, store, batch, [[0.0, 0.0, 1.0]], cb.cone16(30.0), tol=1e-12)
    logits = torch.from_numpy(np.random.default_rng(3).standard_normal((L * L, 4))).to(DEV).requires_grad_(True)
    J = obj(torch.softmax(logits, dim=1))
    J.sum().backward()
    g = logits.grad.detach().cpu().numpy()
    iters = obj.last_reports[0][0]
    rng = np.random.default_rng(4)
    h = 1e-4
    errs = []
    with torch.no_grad():
        for _ in range(3):
            v = rng.standard_normal(g.shape)
            v /= np.linalg.norm(v)
            vd = torch.from_numpy(v).to(DEV)
            Jp = obj(torch.softmax(logits + h * vd, dim=1)).item()
            Jm = obj(torch.softmax(logits - h * vd, dim=1)).item()
            fd = (Jp - Jm) / (2 * h)
            ad = float(np.sum(g * v))
            errs.append(abs(fd - ad) / max(abs(fd), 1e-300))
    print(f"8x8 relaxed autograd: J {J.item():.6e}, adjoint solve iters {iters}, directional FD vs autograd "
          f"errors {['%.1e' % e for e in errs]}")
    assert max(errs) <= 1e-5
