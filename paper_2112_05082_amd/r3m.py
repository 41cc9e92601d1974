"""ctypes binding of libr3m (the C ABI declared in include/r3m.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  PyTorch provides device memory (tensors) and streams.  The module
fails loudly when the shared library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libr3m.so")

R3M_OK = 0
R3M_ERR_INVALID_ARG = -1
R3M_ERR_BUFFER_TOO_SMALL = -2
R3M_ERR_HIP = -3
R3M_ERR_NOT_CONVERGED = -4
R3M_ERR_NONFINITE = -5
R3M_ERR_UNSUPPORTED = -6

C128, C64, BF16X2, F16X2, SPEC_C64, SPEC_C128 = 0, 1, 2, 3, 4, 5
BATCH_INDEX_READY = 1
PRECOND_NONE, PRECOND_BLOCK_JACOBI, PRECOND_BLOCK_ILU = 0, 1, 2

EXPORTED = (
    "r3m_ctx_create", "r3m_ctx_destroy", "r3m_last_error", "r3m_version", "r3m_ctx_check",
    "r3m_blocks_bytes", "r3m_fill_unique_blocks",
    "r3m_far_count", "r3m_far_bytes", "r3m_compress_work_bytes", "r3m_compress_far",
    "r3m_spectral_bytes", "r3m_build_spectral", "r3m_relaxed_work_bytes", "r3m_relaxed_matvec",
    "r3m_relaxed_gradient_work_bytes", "r3m_relaxed_gradient", "r3m_relaxed_rhs", "r3m_relaxed_objective",
    "r3m_matvec_work_bytes", "r3m_retrieved_matvec", "r3m_matvec_groups", "r3m_matvec_plan",
    "r3m_matvec_set_plan", "r3m_spectral_product",
    "r3m_static_scratch_bytes", "r3m_retrieved_matvec_static",
    "r3m_gmres_work_bytes", "r3m_gmres_solve", "r3m_ilu_bytes", "r3m_ilu_factor", "r3m_ilu_apply",
    "r3m_plane_wave_rhs", "r3m_rcs",
)


class R3MError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"r3m error {code}: {msg}")
        self.code = code


class UnitGeomC(C.Structure):
    _fields_ = [
        ("freq_hz", C.c_double), ("period_x", C.c_double), ("period_y", C.c_double),
        ("n_states", C.c_int32), ("state_off", C.POINTER(C.c_int32)),
        ("n_vert", C.c_int32), ("vert", C.POINTER(C.c_double)),
        ("n_tri", C.c_int32), ("tri", C.POINTER(C.c_int32)),
        ("n_rwg", C.c_int32), ("rwg", C.POINTER(C.c_int32)),
        ("extract_radius", C.c_int32), ("n_common", C.c_int32), ("tri_cell", C.POINTER(C.c_int32)),
    ]


class StoreC(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("n_states", C.c_int32), ("Dx", C.c_int32), ("Dy", C.c_int32),
        ("near_radius", C.c_int32), ("near_dtype", C.c_int), ("near", C.c_void_p),
        ("far_dtype", C.c_int), ("far", C.c_void_p), ("max_rank", C.c_int32),
        ("n_common", C.c_int32), ("common_ext", C.c_void_p),
    ]


class BatchC(C.Structure):
    _fields_ = [
        ("B", C.c_int32), ("L", C.POINTER(C.c_int32)), ("unit_off", C.POINTER(C.c_int64)),
        ("state_off", C.POINTER(C.c_int64)), ("states", C.c_void_p), ("flags", C.c_uint32),
    ]


class GmresOptsC(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32),
        ("refine_tol", C.c_double), ("max_refine", C.c_int32), ("precond", C.c_int32),
        ("flags", C.c_int32), ("relaxed_weights", C.c_void_p), ("transpose", C.c_int32),
        ("ilu_radius", C.c_int32),
    ]


class GmresReportC(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("refine_steps", C.c_int32), ("rel_residual", C.c_double),
        ("converged", C.c_int32),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load libr3m.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libr3m.so not built at {path}; run __graft_entry__.build()")
    lib = C.CDLL(path)
    vp, sz, i32, dbl = C.c_void_p, C.c_size_t, C.c_int32, C.c_double
    sig = {
        "r3m_ctx_create": (C.c_int, [C.POINTER(vp), C.c_int]),
        "r3m_ctx_destroy": (C.c_int, [vp]),
        "r3m_last_error": (C.c_char_p, [vp]),
        "r3m_version": (C.c_char_p, []),
        "r3m_ctx_check": (C.c_int, [vp, vp]),
        "r3m_blocks_bytes": (sz, [i32, i32, i32, C.c_int]),
        "r3m_fill_unique_blocks": (C.c_int, [vp, C.POINTER(UnitGeomC), i32, i32, C.c_int, vp, sz, vp]),
        "r3m_far_count": (i32, [i32, i32, i32]),
        "r3m_far_bytes": (sz, [i32, i32, i32, C.c_int]),
        "r3m_compress_work_bytes": (sz, [i32, i32, i32]),
        "r3m_compress_far": (C.c_int, [vp, vp, i32, i32, i32, i32, dbl, i32, C.c_int, vp, sz,
                                       C.POINTER(C.c_int32), C.POINTER(C.c_double), vp, sz, vp]),
        "r3m_spectral_bytes": (sz, [i32, i32, i32, C.c_int]),
        "r3m_build_spectral": (C.c_int, [vp, vp, i32, i32, i32, C.c_int, vp, sz, vp]),
        "r3m_relaxed_work_bytes": (sz, [vp, C.POINTER(StoreC), C.POINTER(BatchC)]),
        "r3m_relaxed_gradient_work_bytes": (sz, [vp, C.POINTER(StoreC), C.POINTER(BatchC)]),
        "r3m_relaxed_gradient": (C.c_int, [vp, C.POINTER(StoreC), C.POINTER(BatchC), vp, vp, vp, vp, vp, vp, vp, vp,
                                           sz, vp]),
        "r3m_relaxed_rhs": (C.c_int, [vp, C.POINTER(UnitGeomC), C.POINTER(BatchC), vp, C.POINTER(C.c_double), i32,
                                      vp, vp]),
        "r3m_relaxed_objective": (C.c_int, [vp, C.POINTER(UnitGeomC), C.POINTER(BatchC), vp, vp, i32,
                                            C.POINTER(C.c_double), dbl, vp, vp, vp, vp, vp]),
        "r3m_relaxed_matvec": (C.c_int, [vp, C.POINTER(StoreC), C.POINTER(BatchC), vp, i32, C.c_int, vp, vp, vp,
                                         sz, vp]),
        "r3m_matvec_work_bytes": (sz, [vp, C.POINTER(StoreC), C.POINTER(BatchC), C.c_int]),
        "r3m_retrieved_matvec": (C.c_int, [vp, C.POINTER(StoreC), C.POINTER(BatchC), C.c_int, vp, vp, vp,
                                           sz, vp]),
        "r3m_matvec_groups": (i32, [vp, C.POINTER(StoreC), C.POINTER(BatchC)]),
        "r3m_matvec_plan": (i32, [vp, C.POINTER(StoreC), C.POINTER(BatchC)]),
        "r3m_matvec_set_plan": (C.c_int, [vp, C.POINTER(StoreC), C.POINTER(BatchC), i32]),
        "r3m_spectral_product": (C.c_int, [vp, C.POINTER(StoreC), C.POINTER(BatchC), vp, sz, vp]),
        "r3m_static_scratch_bytes": (sz, []),
        "r3m_retrieved_matvec_static": (C.c_int, [vp, C.POINTER(StoreC), C.POINTER(BatchC), C.c_int, vp, vp, vp]),
        "r3m_gmres_work_bytes": (sz, [vp, C.POINTER(StoreC), C.POINTER(StoreC), C.POINTER(BatchC),
                                      C.POINTER(GmresOptsC)]),
        "r3m_gmres_solve": (C.c_int, [vp, C.POINTER(StoreC), C.POINTER(StoreC), C.POINTER(BatchC), vp, vp,
                                      C.POINTER(GmresOptsC), C.POINTER(GmresReportC), vp, sz, vp]),
        "r3m_ilu_bytes": (sz, [vp, C.POINTER(StoreC), C.POINTER(BatchC), i32]),
        "r3m_ilu_factor": (C.c_int, [vp, C.POINTER(StoreC), C.POINTER(BatchC), i32, vp, sz, vp]),
        "r3m_ilu_apply": (C.c_int, [vp, C.POINTER(StoreC), C.POINTER(BatchC), i32, vp, sz, vp, vp, vp]),
        "r3m_plane_wave_rhs": (C.c_int, [vp, C.POINTER(UnitGeomC), C.POINTER(BatchC), C.POINTER(C.c_double),
                                         vp, vp]),
        "r3m_rcs": (C.c_int, [vp, C.POINTER(UnitGeomC), C.POINTER(BatchC), vp, i32, C.POINTER(C.c_double),
                              dbl, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, ctx=None, allow=()):
    if rc != R3M_OK and rc not in allow:
        msg = load().r3m_last_error(ctx).decode()
        raise R3MError(rc, msg)
    return rc


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


# ------------------------------------------------------------------ objects


class Context:
    def __init__(self, device: int = 0):
        lib = load()
        h = C.c_void_p()
        _check(lib.r3m_ctx_create(C.byref(h), int(device)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            load().r3m_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class UnitGeom:
    """Host geometry of a macro unit (keeps the numpy arrays alive)."""

    def __init__(self, vert, tri, rwg, state_off, freq_hz, period, extract_radius=1, tri_cell=None,
                 common_ext=None):
        self.vert = np.ascontiguousarray(vert, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.rwg = np.ascontiguousarray(rwg, dtype=np.int32)
        self.state_off = np.ascontiguousarray(state_off, dtype=np.int32)
        self.tri_cell = None if tri_cell is None else np.ascontiguousarray(tri_cell, dtype=np.int32)
        # connected geometries: the classes of the shared bases (host copy)
        self.common_ext = None if common_ext is None else np.ascontiguousarray(common_ext, dtype=np.int32)
        self.c = UnitGeomC(
            float(freq_hz), float(period[0]), float(period[1]), len(self.state_off) - 1,
            _ptr(self.state_off, C.c_int32), len(self.vert), _ptr(self.vert, C.c_double),
            len(self.tri), _ptr(self.tri, C.c_int32), len(self.rwg), _ptr(self.rwg, C.c_int32),
            int(extract_radius), self.n_common,
            _ptr(self.tri_cell, C.c_int32) if self.tri_cell is not None else None)

    @property
    def n(self):
        return len(self.rwg)

    @property
    def n_common(self):
        return len(self.rwg) - int(self.state_off[-1])

    @property
    def n_states(self):
        return len(self.state_off) - 1

    @classmethod
    def from_macro(cls, unit, freq_hz, extract_radius=1):
        return cls(unit.vert, unit.tri, unit.rwg, unit.state_off, freq_hz, unit.period, extract_radius)

    @classmethod
    def from_connected(cls, cu, freq_hz, extract_radius=1):
        """An extended macro unit over a connected ground plane (see
        workloads.mesh.connected_unit)."""
        return cls(cu.vert, cu.tri, cu.rwg, cu.state_off, freq_hz, cu.period, extract_radius, cu.tri_cell, cu.ext)


@dataclass
class Store:
    """Device block store (tensors owned by torch)."""
    n: int
    n_states: int
    Dx: int
    Dy: int
    near_radius: int
    near_dtype: int
    near: object  # torch tensor
    far_dtype: int = C128
    far: object = None
    max_rank: int = 0
    ranks: np.ndarray | None = None
    rel_err: np.ndarray | None = None
    common_ext: object = None  # torch int32 device tensor of the shared bases' classes, or None

    @property
    def n_common(self) -> int:
        return 0 if self.common_ext is None else int(self.common_ext.numel())

    def c(self) -> StoreC:
        return StoreC(self.n, self.n_states, self.Dx, self.Dy, self.near_radius, self.near_dtype,
                      C.c_void_p(self.near.data_ptr()), self.far_dtype,
                      C.c_void_p(self.far.data_ptr() if self.far is not None else 0), self.max_rank,
                      self.n_common,
                      C.c_void_p(self.common_ext.data_ptr() if self.common_ext is not None else 0))


class Batch:
    """RHS list sharing one store; states is a torch uint8 device tensor."""

    def __init__(self, L, unit_off, state_off, states):
        self.L = np.ascontiguousarray(np.asarray(L, dtype=np.int32).reshape(-1, 2))
        self.unit_off = np.ascontiguousarray(unit_off, dtype=np.int64)
        self.state_off = np.ascontiguousarray(state_off, dtype=np.int64)
        self.states = states
        if len(self.unit_off):
            need = int((self.state_off + self.L[:, 0].astype(np.int64) * self.L[:, 1]).max())
            if states.numel() < need or states.element_size() != 1:
                raise ValueError(f"states holds {states.numel()} bytes, the batch needs {need}")
        self.cs = BatchC(len(self.unit_off), _ptr(self.L, C.c_int32), _ptr(self.unit_off, C.c_int64),
                         _ptr(self.state_off, C.c_int64), C.c_void_p(states.data_ptr()))

    @property
    def B(self):
        return len(self.unit_off)

    @property
    def total_units(self):
        return int(max((self.unit_off + self.L[:, 0] * self.L[:, 1]).max(), 0)) if self.B else 0

    @classmethod
    def from_codebooks(cls, codebooks, sizes, device, repeat: int = 1):
        """One RHS per (codebook, repeat); repeats share the codebook bytes."""
        import torch
        L, uoff, soff = [], [], []
        s_all = []
        so = 0
        uo = 0
        for book, Lb in zip(codebooks, sizes):
            s_all.append(np.asarray(book, dtype=np.uint8))
            for _ in range(repeat):
                L.append((Lb, Lb))
                uoff.append(uo)
                soff.append(so)
                uo += Lb * Lb
            so += Lb * Lb
        states = torch.from_numpy(np.concatenate(s_all)).to(device)
        return cls(L, uoff, soff, states)


# ------------------------------------------------- the C entry points


def r3m_fill_unique_blocks(ctx: Context, geom: UnitGeom, Dx: int, Dy: int, dtype: int, out, stream=None):
    lib = load()
    need = lib.r3m_blocks_bytes(geom.n, Dx, Dy, dtype)
    _check(lib.r3m_fill_unique_blocks(ctx.handle, C.byref(geom.c), Dx, Dy, dtype, C.c_void_p(out.data_ptr()),
                                      out.numel() * out.element_size(), _stream(stream)), ctx.handle)
    return need


def r3m_compress_far(ctx: Context, dense, n: int, Dx: int, Dy: int, near_radius: int, tol: float,
                     max_rank: int, far_dtype: int, far, work, stream=None):
    lib = load()
    n_far = lib.r3m_far_count(Dx, Dy, near_radius)
    ranks = np.zeros(max(n_far, 1), np.int32)
    err = np.zeros(max(n_far, 1), np.float64)
    _check(lib.r3m_compress_far(ctx.handle, C.c_void_p(dense.data_ptr()), n, Dx, Dy, near_radius, float(tol),
                                max_rank, far_dtype, C.c_void_p(far.data_ptr()), far.numel() * far.element_size(),
                                _ptr(ranks, C.c_int32), _ptr(err, C.c_double), C.c_void_p(work.data_ptr()),
                                work.numel() * work.element_size(), _stream(stream)), ctx.handle)
    return ranks[:n_far], err[:n_far]


def r3m_build_spectral(ctx: Context, dense, n: int, Dx: int, Dy: int, dtype: int, out, stream=None):
    """Block spectra of a C128 dense store into `out` (r3m_spectral_bytes)."""
    lib = load()
    _check(lib.r3m_build_spectral(ctx.handle, C.c_void_p(dense.data_ptr()), n, Dx, Dy, dtype,
                                  C.c_void_p(out.data_ptr()), out.numel() * out.element_size(), _stream(stream)),
           ctx.handle)


def relaxed_work_bytes(ctx: Context, store: Store, batch: Batch) -> int:
    sc = store.c()
    return load().r3m_relaxed_work_bytes(ctx.handle, C.byref(sc), C.byref(batch.cs))


def r3m_relaxed_matvec(ctx: Context, store: Store, batch: Batch, weights, vec_dtype: int, x, y, work,
                       transpose: bool = False, stream=None):
    """y = P(w)^T Z P(w) x (transpose: with Z^T); weights: float64 device
    tensor [total units][n_states]."""
    lib = load()
    _need_vec(x, batch, per_unit(store), "x")
    _need_vec(y, batch, per_unit(store), "y")
    if batch.B and weights.numel() < batch.total_units * store.n_states:
        raise ValueError("weights hold fewer than total_units x n_states entries")
    sc = store.c()
    _check(lib.r3m_relaxed_matvec(ctx.handle, C.byref(sc), C.byref(batch.cs), C.c_void_p(weights.data_ptr()),
                                  1 if transpose else 0, vec_dtype, C.c_void_p(x.data_ptr()),
                                  C.c_void_p(y.data_ptr()), C.c_void_p(work.data_ptr()),
                                  work.numel() * work.element_size(), _stream(stream)), ctx.handle)


def relaxed_gradient_work_bytes(ctx: Context, store: Store, batch: Batch) -> int:
    sc = store.c()
    return load().r3m_relaxed_gradient_work_bytes(ctx.handle, C.byref(sc), C.byref(batch.cs))


def _p(t):
    return C.c_void_p(t.data_ptr() if t is not None else 0)


def r3m_relaxed_rhs(ctx: Context, geom: "UnitGeom", batch: Batch, weights, inc, b, macro: bool = False,
                    stream=None):
    inc = np.ascontiguousarray(np.asarray(inc, dtype=np.float64).reshape(-1, 3))
    if len(inc) != batch.B:
        raise ValueError("one incidence per RHS")
    _check(load().r3m_relaxed_rhs(ctx.handle, C.byref(geom.c), C.byref(batch.cs), _p(weights), _ptr(inc, C.c_double),
                                  1 if macro else 0, _p(b), _stream(stream)), ctx.handle)


def r3m_relaxed_objective(ctx: Context, geom: "UnitGeom", batch: Batch, weights, I, dirs, e0, J, sigma, G, adj,
                          stream=None):
    dirs = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 2))
    _check(load().r3m_relaxed_objective(ctx.handle, C.byref(geom.c), C.byref(batch.cs), _p(weights), _p(I),
                                        len(dirs), _ptr(dirs, C.c_double), float(e0), _p(J), _p(sigma), _p(G),
                                        _p(adj), _stream(stream)), ctx.handle)


def r3m_relaxed_gradient(ctx: Context, store: Store, batch: Batch, weights, I, lam, G, U, dJ, grad, work,
                         stream=None):
    sc = store.c()
    _check(load().r3m_relaxed_gradient(ctx.handle, C.byref(sc), C.byref(batch.cs), _p(weights), _p(I), _p(lam),
                                       _p(G), _p(U), _p(dJ), _p(grad), _p(work), work.numel() * work.element_size(),
                                       _stream(stream)), ctx.handle)


def per_unit(obj) -> int:
    """Vector entries per unit for a Store or UnitGeom: the state's n_a
    bases, then the n_common shared ones (connected geometries)."""
    return (obj.n - obj.n_common) // obj.n_states + obj.n_common


def _need_vec(t, batch: Batch, n_a: int, what: str):
    if batch.B and t.numel() < batch.total_units * n_a:
        raise ValueError(f"{what} holds {t.numel()} complex entries, the batch needs {batch.total_units * n_a}")


def r3m_retrieved_matvec(ctx: Context, store: Store, batch: Batch, vec_dtype: int, x, y, work=None,
                         stream=None, index_ready: bool = False):
    """index_ready: the retrieval index in `work` is current (an earlier call
    with this store, batch and codebook built it there): skip rebuilding it."""
    lib = load()
    _need_vec(x, batch, per_unit(store), "x")
    _need_vec(y, batch, per_unit(store), "y")
    sc = store.c()
    wb = 0 if work is None else work.numel() * work.element_size()
    wp = C.c_void_p(0 if work is None else work.data_ptr())
    batch.cs.flags = BATCH_INDEX_READY if index_ready else 0
    try:
        _check(lib.r3m_retrieved_matvec(ctx.handle, C.byref(sc), C.byref(batch.cs), vec_dtype,
                                        C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), wp, wb,
                                        _stream(stream)), ctx.handle)
    finally:
        batch.cs.flags = 0


def r3m_ctx_check(ctx: Context, stream=None):
    """Synchronise and raise the error an earlier asynchronous call left on the device."""
    _check(load().r3m_ctx_check(ctx.handle, _stream(stream)), ctx.handle)


def r3m_retrieved_matvec_static(ctx: Context, store: Store, batch: Batch, vec_dtype: int, x, y, stream=None,
                                index_ready: bool = False):
    """r3m_retrieved_matvec with the library's static device scratch (no workspace)."""
    lib = load()
    _need_vec(x, batch, per_unit(store), "x")
    _need_vec(y, batch, per_unit(store), "y")
    sc = store.c()
    batch.cs.flags = BATCH_INDEX_READY if index_ready else 0
    try:
        _check(lib.r3m_retrieved_matvec_static(ctx.handle, C.byref(sc), C.byref(batch.cs), vec_dtype,
                                               C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                               _stream(stream)), ctx.handle)
    finally:
        batch.cs.flags = 0


def static_scratch_bytes() -> int:
    return int(load().r3m_static_scratch_bytes())


def r3m_gmres_solve(ctx: Context, store: Store, store64: Store | None, batch: Batch, b, x, tol: float,
                    restart: int, max_iter: int, work, refine_tol: float = 0.0, max_refine: int = 0,
                    stream=None, allow_not_converged: bool = False, precond: int = PRECOND_NONE,
                    eager: bool = False, relaxed_weights=None, transpose: bool = False, ilu_radius: int = 1):
    """relaxed_weights: float64 device tensor [total units][n_states] to solve
    the relaxed system P(w)^T Z P(w) x = b (transpose: with Z^T).
    ilu_radius: pattern radius of PRECOND_BLOCK_ILU."""
    lib = load()
    _need_vec(b, batch, per_unit(store), "b")
    _need_vec(x, batch, per_unit(store), "x")
    sc = store.c()
    s64 = store64.c() if store64 is not None else None
    wp = C.c_void_p(relaxed_weights.data_ptr() if relaxed_weights is not None else 0)
    opts = GmresOptsC(float(tol), int(restart), int(max_iter), float(refine_tol), int(max_refine), int(precond),
                      1 if eager else 0, wp, 1 if transpose else 0, int(ilu_radius))
    rep = (GmresReportC * max(batch.B, 1))()
    rc = lib.r3m_gmres_solve(ctx.handle, C.byref(sc), C.byref(s64) if s64 is not None else None,
                             C.byref(batch.cs), C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                             C.byref(opts), rep, C.c_void_p(work.data_ptr()), work.numel() * work.element_size(),
                             _stream(stream))
    _check(rc, ctx.handle, allow=(R3M_ERR_NOT_CONVERGED,) if allow_not_converged else ())
    return rc, [(r.iters, r.refine_steps, r.rel_residual, bool(r.converged)) for r in rep[: batch.B]]


def ilu_bytes(ctx: Context, store: Store, batch: Batch, radius: int) -> int:
    sc = store.c()
    return load().r3m_ilu_bytes(ctx.handle, C.byref(sc), C.byref(batch.cs), int(radius))


def r3m_ilu_factor(ctx: Context, store: Store, batch: Batch, radius: int, factors, stream=None):
    """Near-field block ILU(0) factors of every RHS's codebook into `factors`
    (a device byte tensor of ilu_bytes(...))."""
    sc = store.c()
    _check(load().r3m_ilu_factor(ctx.handle, C.byref(sc), C.byref(batch.cs), int(radius),
                                 C.c_void_p(factors.data_ptr()), factors.numel() * factors.element_size(),
                                 _stream(stream)), ctx.handle)


def r3m_ilu_apply(ctx: Context, store: Store, batch: Batch, radius: int, factors, x, y, stream=None):
    """y = M^-1 x with the factors of r3m_ilu_factor (complex128 vectors)."""
    for t, name in ((x, "x"), (y, "y")):
        if not (t.is_complex() and t.element_size() == 16):
            raise ValueError(f"{name} must be complex128")
    n_a = store.n // store.n_states
    _need_vec(x, batch, n_a, "x")
    _need_vec(y, batch, n_a, "y")
    sc = store.c()
    _check(load().r3m_ilu_apply(ctx.handle, C.byref(sc), C.byref(batch.cs), int(radius),
                                C.c_void_p(factors.data_ptr()), factors.numel() * factors.element_size(),
                                C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), _stream(stream)), ctx.handle)


def r3m_plane_wave_rhs(ctx: Context, geom: UnitGeom, batch: Batch, inc, b, stream=None):
    inc = np.ascontiguousarray(inc, dtype=np.float64).reshape(-1, 3)
    _need_vec(b, batch, per_unit(geom), "b")
    if len(inc) != batch.B:
        raise ValueError("one incidence row per RHS")
    _check(load().r3m_plane_wave_rhs(ctx.handle, C.byref(geom.c), C.byref(batch.cs), _ptr(inc, C.c_double),
                                     C.c_void_p(b.data_ptr()), _stream(stream)), ctx.handle)


def r3m_rcs(ctx: Context, geom: UnitGeom, batch: Batch, I, dirs, e0, sigma, stream=None):
    dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 2)
    _need_vec(I, batch, per_unit(geom), "I")
    if sigma.numel() < batch.B * len(dirs):
        raise ValueError("sigma too small")
    _check(load().r3m_rcs(ctx.handle, C.byref(geom.c), C.byref(batch.cs), C.c_void_p(I.data_ptr()), len(dirs),
                          _ptr(dirs, C.c_double), float(e0), C.c_void_p(sigma.data_ptr()), _stream(stream)),
           ctx.handle)


# ------------------------------------------------- size queries


def blocks_bytes(n, Dx, Dy, dtype):
    return load().r3m_blocks_bytes(n, Dx, Dy, dtype)


def far_count(Dx, Dy, nr):
    return load().r3m_far_count(Dx, Dy, nr)


def far_bytes(n, n_far, max_rank, dtype):
    return load().r3m_far_bytes(n, n_far, max_rank, dtype)


def spectral_bytes(n, Dx, Dy, dtype):
    return load().r3m_spectral_bytes(n, Dx, Dy, dtype)


def compress_work_bytes(n, max_rank, per_batch):
    return load().r3m_compress_work_bytes(n, max_rank, per_batch)


def matvec_work_bytes(ctx, store: Store, batch: Batch, vec_dtype):
    sc = store.c()
    return load().r3m_matvec_work_bytes(ctx.handle, C.byref(sc), C.byref(batch.cs), vec_dtype)


def matvec_groups(ctx, store: Store, batch: Batch) -> int:
    sc = store.c()
    g = load().r3m_matvec_groups(ctx.handle, C.byref(sc), C.byref(batch.cs))
    if g < 0:
        _check(g, ctx.handle)
    return g


PLAN_SPEC_TWO_PASS, PLAN_MFMA_FAR, PLAN_SPECTRAL = 1 << 12, 1 << 16, 1 << 17
# frequency-product shapes of spectral stores: {frequencies per wave, columns
# per staged chunk} of the matrix-core kernel; (0, 0) is the vector-unit kernel
# (frequencies per wave, columns per staged chunk, 16-RHS tiles per workgroup); 0: vector units
SPEC_SHAPES = ((0, 0, 0), (1, 4, 1), (2, 4, 1), (2, 8, 1), (4, 4, 1), (1, 8, 1), (2, 4, 2), (1, 8, 2))


def spec_plan(shape: int, rhs_first: int = 8, two_pass: bool = False, kt_groups: int = 0) -> int:
    """kt_groups: log2 of the frequency-tile groups the XCDs form in the RHS-first order."""
    return PLAN_SPECTRAL | shape | rhs_first << 4 | (PLAN_SPEC_TWO_PASS if two_pass else 0) | kt_groups << 13


def matvec_plan(ctx, store: Store, batch: Batch) -> int:
    """The launch plan of (store, batch): tuned, pinned or default (see r3m_matvec_plan)."""
    sc = store.c()
    p = load().r3m_matvec_plan(ctx.handle, C.byref(sc), C.byref(batch.cs))
    if p < 0:
        _check(p, ctx.handle)
    return p


def decode_plan(plan: int) -> dict:
    if plan & PLAN_SPECTRAL:
        k = plan & 15
        return {"kind": "spectral", "shape": k, "mfma": k != 0, "kpw": SPEC_SHAPES[k][0] if k < len(SPEC_SHAPES) else None,
                "pc": SPEC_SHAPES[k][1] if k < len(SPEC_SHAPES) else None,
                "rhs_tiles": SPEC_SHAPES[k][2] if k < len(SPEC_SHAPES) else None, "rhs_first": (plan >> 4) & 255,
                "two_pass": bool(plan & PLAN_SPEC_TWO_PASS), "kt_groups": (plan >> 13) & 3}
    return {"kind": "compressed", "groups": plan & 0xFFFF, "mfma_far": bool(plan & PLAN_MFMA_FAR)}


def r3m_spectral_product(ctx, store: Store, batch: Batch, work, stream=None) -> None:
    """The frequency product alone on the grids a preceding matvec left in `work`."""
    sc = store.c()
    _check(load().r3m_spectral_product(ctx.handle, C.byref(sc), C.byref(batch.cs), C.c_void_p(work.data_ptr()),
                                       work.numel() * work.element_size(), _stream(stream)), ctx.handle)


def matvec_set_plan(ctx, store: Store, batch: Batch, plan: int) -> None:
    sc = store.c()
    _check(load().r3m_matvec_set_plan(ctx.handle, C.byref(sc), C.byref(batch.cs), int(plan)), ctx.handle)


def gmres_work_bytes(ctx, store: Store, batch: Batch, restart: int, store64: Store | None = None,
                     relaxed: bool = False, precond: int = PRECOND_NONE, ilu_radius: int = 1):
    """store64: the refinement store the solve will use (None: no refinement);
    relaxed + precond: a relaxed solve with block-Jacobi keeps one inverse per unit;
    PRECOND_BLOCK_ILU adds the factors of radius ilu_radius."""
    sc = store.c()
    s64 = store64.c() if store64 is not None else None
    opts = GmresOptsC(1e-6, int(restart), 1, 0.0, 0, int(precond), 0, C.c_void_p(1 if relaxed else 0), 0,
                      int(ilu_radius))
    return load().r3m_gmres_work_bytes(ctx.handle, C.byref(sc), C.byref(s64) if s64 is not None else None,
                                       C.byref(batch.cs), C.byref(opts))
