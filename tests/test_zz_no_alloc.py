"""The allocation-free matvec entry point (static device scratch) against the
workspace entry point, through the C ABI: two calls in a row, the second on a
smaller batch, and a batch too large for the scratch rejected on the host."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_static_matvec_matches_workspace_matvec():
    import torch

    from gpu_common import FREQ, rel_max, unit
    from paper_2112_05082_amd import pipeline, r3m
    from workloads import codebooks as cb
    dev = "cuda:0"
    ctx = r3m.Context(0)
    u = unit(2)
    geom = r3m.UnitGeom.from_macro(u, FREQ, 1)
    L = 12
    dense = pipeline.fill_blocks(ctx, geom, L - 1, r3m.C128, dev)
    store = pipeline.compressed_store(ctx, geom, L, 2, r3m.C64, r3m.C64, 1e-4, 40, dev, dense_c128=dense)
    plain = r3m.Store(u.n, 4, L - 1, L - 1, L - 1, r3m.C128, dense)
    # first call: two codebooks of 12x12 and 9x7; second: one 5x5 array
    cases = [([cb.uniform(L, 4, 1), cb.uniform(9, 4, 2)[: 9 * 7]], [(L, L), (9, 7)]),
             ([cb.uniform(5, 4, 3)], [(5, 5)])]
    for codes, sizes in cases:
        uoff = np.cumsum([0] + [a * b for a, b in sizes])[:-1].tolist()
        states = torch.from_numpy(np.concatenate(codes).astype(np.uint8)).to(dev)
        batch = r3m.Batch(sizes, uoff, uoff, states)
        N = batch.total_units * u.n_a
        g = torch.Generator(device=dev).manual_seed(len(codes))
        x = torch.complex(torch.randn(N, generator=g, device=dev, dtype=torch.float64),
                          torch.randn(N, generator=g, device=dev, dtype=torch.float64))
        for st, vt, tol in ((store, r3m.C128, 1e-6), (plain, r3m.C128, 1e-12), (store, r3m.C64, 1e-6)):
            xv = x if vt == r3m.C128 else x.to(torch.complex64)
            y_ref = torch.zeros_like(xv)
            work = torch.empty(r3m.matvec_work_bytes(ctx, st, batch, vt), dtype=torch.uint8, device=dev)
            r3m.r3m_retrieved_matvec(ctx, st, batch, vt, xv, y_ref, work)
            y = torch.full_like(xv, float("nan"))
            r3m.r3m_retrieved_matvec_static(ctx, st, batch, vt, xv, y)
            torch.cuda.synchronize()
            err = rel_max(y.cpu().numpy(), y_ref.cpu().numpy())
            print(f"static matvec sizes={sizes} vec={vt} store={st.far_dtype} err={err:.2e}", flush=True)
            assert np.isfinite(y.cpu().numpy()).all()
            assert err <= tol, err
            del work
    ctx.close()


def test_static_matvec_rejects_batch_beyond_scratch():
    import torch

    from gpu_common import FREQ, unit
    from paper_2112_05082_amd import pipeline, r3m
    from workloads import codebooks as cb
    dev = "cuda:0"
    ctx = r3m.Context(0)
    u = unit(1)
    geom = r3m.UnitGeom.from_macro(u, FREQ, 1)
    L = 32
    dense = pipeline.fill_blocks(ctx, geom, L - 1, r3m.C128, dev)
    store = pipeline.compressed_store(ctx, geom, L, 2, r3m.C64, r3m.C64, 1e-4, 40, dev, dense_c128=dense)
    codes = [cb.bernoulli(L, s) for s in range(24)]
    batch = r3m.Batch.from_codebooks(codes, [L] * len(codes), dev)
    need = r3m.matvec_work_bytes(ctx, store, batch, r3m.C128)
    assert need > r3m.static_scratch_bytes()
    N = batch.total_units * u.n_a
    x = torch.zeros(N, dtype=torch.complex128, device=dev)
    y = torch.zeros_like(x)
    with pytest.raises(r3m.R3MError) as e:
        r3m.r3m_retrieved_matvec_static(ctx, store, batch, r3m.C128, x, y)
    assert e.value.code == r3m.R3M_ERR_BUFFER_TOO_SMALL
    ctx.close()
