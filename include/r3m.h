/*
 * r3m.h -- C ABI of the retrieved-matvec library for MI355X (gfx950).
 *
 * Method: recurrence rebuild and retrieval with hierarchical pattern
 * exploitation (R3M-HPE, arXiv 2112.05082).  Every coding unit of a digital
 * coding metasurface is replaced by the macro unit, the union of all its
 * coding states (Sec. III-A), so the array is rigorously periodic and the
 * Galerkin EFIE matrix of eq. (1) -- the global matrix Z -- depends only on
 * the lattice displacement d = (dx, dy) between observer and source units.
 * The global matrix is therefore stored once as unique displacement blocks,
 * the finest 1x1 pattern (offset, src, obs) of eq. (7) (Sec. III-C): dense
 * near blocks and low-rank far blocks U V^H (Sec. II-B).  A codebook k is
 * applied through implicit retrieval, y_k = P_k^T Z P_k x_k (eq. (3)), i.e.
 * the D_k mask of eq. (6), realised as a per-unit state byte that selects
 * the active rows and columns of each block.  The retrieved system is solved
 * with an MVP-based Krylov method (Sec. III-A, last paragraph).
 *
 * Conventions
 *  - Every function returns an int status (R3M_OK or a negative R3M_ERR_*).
 *    No C++ exception crosses the ABI.  r3m_last_error() gives detail.
 *  - The library never allocates user-visible device memory.  Outputs and
 *    workspaces are caller-owned device pointers sized by the *_bytes
 *    queries; host arrays are caller-owned and only read during the call.
 *  - Every call takes a caller-owned hipStream_t and is asynchronous on it,
 *    except calls that return host data (noted), which synchronise it.
 *  - Shapes, ranges and pointers are validated on the host before any launch.
 *    Data that lives on the device (the codebooks' state bytes) is checked
 *    on the device: a call that synchronises reports its own inputs; an
 *    asynchronous call (r3m_retrieved_matvec) leaves the error in the context
 *    and the next r3m_ctx_check, r3m_gmres_solve, r3m_plane_wave_rhs or
 *    r3m_rcs on that context returns it (and clears it).
 *  - Complex values are interleaved (re, im): R3M_C128 = 2 x double,
 *    R3M_C64 = 2 x float.
 *  - Units: metres, hertz.  Time convention exp(+j w t).
 *  - Unit index u = iy*L + ix; unit u sits at (ix*period_x, iy*period_y, 0).
 *  - Displacement slot of d = (dx, dy) in a store of half-extent (Dx, Dy):
 *        slot(d) = (dy + Dy)*(2*Dx + 1) + (dx + Dx).
 *  - Macro basis order is state-major: state s owns the contiguous RWG range
 *    [state_off[s], state_off[s+1]); all states must own n_a = n/n_states.
 *  - Reduced (retrieved) vectors are [unit][n_a]: the column order of P_k.
 */
#ifndef R3M_H
#define R3M_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  R3M_OK = 0,
  R3M_ERR_INVALID_ARG = -1,
  R3M_ERR_BUFFER_TOO_SMALL = -2,
  R3M_ERR_HIP = -3,
  R3M_ERR_NOT_CONVERGED = -4, /* outputs are still written */
  R3M_ERR_NONFINITE = -5,
  R3M_ERR_UNSUPPORTED = -6
};

typedef enum {
  R3M_C128 = 0,   /* complex double */
  R3M_C64 = 1,    /* complex float, FP32 accumulation */
  R3M_BF16X2 = 2, /* far factors only: hi/lo bfloat16 split, FP32 accumulation */
  R3M_F16X2 = 3,  /* far factors only: hi/lo float16 split with a per-column scale */
  R3M_SPEC_C64 = 4, /* store far part only: block spectra (r3m_build_spectral), complex float */
  R3M_SPEC_C128 = 5 /* store far part only: block spectra, complex double */
} r3m_dtype;

typedef struct r3m_ctx_s* r3m_ctx;

/* Creates a context bound to HIP device `device`.  Returns R3M_ERR_HIP if the
 * device cannot be selected (e.g. no GPU visible). */
int r3m_ctx_create(r3m_ctx* out, int device);
int r3m_ctx_destroy(r3m_ctx ctx);
/* Last error message of ctx (or of the calling thread when ctx is NULL). */
const char* r3m_last_error(r3m_ctx ctx);
/* Library version string. */
const char* r3m_version(void);
/* Synchronises `stream` and returns (then clears) the error an earlier
 * asynchronous call on ctx found on the device: R3M_ERR_INVALID_ARG for a
 * codebook state byte >= n_states (the product of that call is undefined
 * for the units concerned), else R3M_OK. */
int r3m_ctx_check(r3m_ctx ctx, hipStream_t stream);

/* Geometry of the macro unit (host memory, read during the call).
 * The macro unit is the union of its coding states (Sec. III-A): state s owns
 * RWG [state_off[s], state_off[s+1]).  rwg[m] = {T+, T-, edge vertex 0, edge
 * vertex 1} with T+ carrying +(l/2A)(r - free vertex) (RWG basis, Sec. II-A).
 * All vertices lie in the unit's local frame; unit centres are on the lattice.
 * Triangle pairs whose cells are within Chebyshev distance extract_radius
 * use closed-form 1/R singularity extraction.
 * Connected geometries (Sec. III-B, basis extension of periodic boundaries):
 * the last n_common RWG (after state_off[n_states]) belong to every state,
 * e.g. a ground plane; a basis bridging two cells is ascribed to one unit and
 * its triangle in the neighbouring cell carries that cell's lattice offset in
 * tri_cell ([n_tri][2], NULL: every triangle in the unit's own cell), which
 * the extraction rule uses.  n_common = 0 and tri_cell = NULL for isolated
 * units.  The fill, excitation and RCS take connected geometries; the
 * excitation and RCS class each shared basis by the cells of its triangles
 * (both in the unit's cell: 0; one in the -x neighbour: 1; in the -y
 * neighbour: 2) and return R3M_ERR_UNSUPPORTED for any other reach or for a
 * coding-state basis outside its cell. */
typedef struct {
  double freq_hz;
  double period_x, period_y;
  int32_t n_states;
  const int32_t* state_off; /* [n_states + 1] */
  int32_t n_vert;
  const double* vert; /* [n_vert][3] */
  int32_t n_tri;
  const int32_t* tri; /* [n_tri][3] */
  int32_t n_rwg;
  const int32_t* rwg; /* [n_rwg][4] */
  int32_t extract_radius;
  int32_t n_common;        /* RWG shared by every state, after the states' ranges */
  const int32_t* tri_cell; /* [n_tri][2] or NULL */
} r3m_unit_geom;

/* ---------------------------------------------------------------- fill -- */

/* Bytes of (2Dx+1)(2Dy+1) dense n x n blocks of `dtype` (C128 or C64). */
size_t r3m_blocks_bytes(int32_t n, int32_t Dx, int32_t Dy, r3m_dtype dtype);

/* Fills the global-matrix blocks Z(d) for every |dx| <= Dx, |dy| <= Dy:
 * out[slot(d)][m][n] = Z_mn between observer macro RWG m of the unit at d
 * and source macro RWG n of the unit at the origin (eq. (1), Galerkin EFIE:
 * Z_mn = j k eta int int [f_m.f_n - k^-2 div f_m div' f_n] G dS' dS,
 * G = exp(-jkR)/(4 pi R), 7-point rule on both triangles).  Computed in FP64
 * and rounded to `dtype` (C128 or C64).  Sets R3M_ERR_NONFINITE if any entry
 * is not finite (checked before returning; this call synchronises). */
int r3m_fill_unique_blocks(r3m_ctx ctx, const r3m_unit_geom* geom, int32_t Dx, int32_t Dy,
                           r3m_dtype dtype, void* blocks_dev, size_t blocks_bytes,
                           hipStream_t stream);

/* ------------------------------------------------------------ compress -- */

/* Far displacements are those with max(|dx|,|dy|) > near_radius.  They are
 * numbered in slot order, skipping near slots:
 *   far_index(d) = slot(d) - #near slots before slot(d).
 * Far buffer layout: int32 ranks[n_far] (padded to 256 B), then per far
 * block f the factors U_f [max_rank][n] followed by V_f [max_rank][n]
 * (column rho contiguous over rows) so that Z(d) ~ U V^H.  Unused columns
 * (rho >= rank) are zero.  Element type: C128 or C64. */
int32_t r3m_far_count(int32_t Dx, int32_t Dy, int32_t near_radius);
size_t r3m_far_bytes(int32_t n, int32_t n_far, int32_t max_rank, r3m_dtype dtype);
/* Workspace of r3m_compress_far (FP64 residual blocks, processed in batches). */
size_t r3m_compress_work_bytes(int32_t n, int32_t max_rank, int32_t blocks_per_batch);

/* Fully pivoted adaptive cross approximation of every far block of a C128
 * dense store (as written by r3m_fill_unique_blocks with the same Dx, Dy):
 * repeat {pivot = argmax|R|; u = R[:,j*]; v = conj(R[i*,:]/R[i*,j*]);
 * R -= u v^H} until ||R||_F <= tol ||Z(d)||_F or rank == max_rank (Sec. II-B,
 * ACA of admissible blocks).  Work in FP64, output rounded to far_dtype.
 * ranks_host[n_far] and rel_err_host[n_far] (achieved relative Frobenius
 * error, exact) are returned; this call synchronises. */
int r3m_compress_far(r3m_ctx ctx, const void* dense_dev, int32_t n, int32_t Dx, int32_t Dy,
                     int32_t near_radius, double tol, int32_t max_rank, r3m_dtype far_dtype,
                     void* far_dev, size_t far_bytes, int32_t* ranks_host, double* rel_err_host,
                     void* work_dev, size_t work_bytes, hipStream_t stream);

/* ------------------------------------------------------------ spectra -- */

/* The unique blocks Z(d) as spectra of their circulant embedding: the
 * two-level block-Toeplitz structure of the macro system (every block a
 * function of the displacement, Sec. III-C) makes the retrieved product of
 * eq. (6) a 2-D convolution over units, evaluated by FFT.  With
 * Gx = smallest power of two >= 2Dx+1 (>= 2), Gy likewise:
 *   spec[m][n][gy][gx] = sum over |dx| <= Dx, |dy| <= Dy of
 *       Z(d)[m][n] exp(-2 pi i (gx dx / Gx + gy dy / Gy)),
 * complex float (R3M_SPEC_C64) or double (R3M_SPEC_C128), row-major grids.
 * Bytes: n * n * Gx * Gy * (8 or 16); 0 for bad arguments. */
size_t r3m_spectral_bytes(int32_t n, int32_t Dx, int32_t Dy, r3m_dtype dtype);

/* Computes the spectra above from a C128 dense store of the same (n, Dx, Dy)
 * (as written by r3m_fill_unique_blocks), transforms in the output precision.
 * n <= 256; Gx, Gy < 4096 (float) or 2048 (double), else
 * R3M_ERR_UNSUPPORTED.  Asynchronous on `stream`. */
int r3m_build_spectral(r3m_ctx ctx, const void* dense_dev, int32_t n, int32_t Dx, int32_t Dy, r3m_dtype dtype,
                       void* spec_dev, size_t spec_bytes, hipStream_t stream);

/* --------------------------------------------------------------- store -- */

/* A global matrix as unique displacement blocks.
 * near: dense blocks for max(|dx|,|dy|) <= near_radius, laid out as a block
 *       store of half-extent (Nx, Ny) = (min(near_radius, Dx), min(near_radius, Dy)).
 * far : r3m_far layout above (ignored when near covers the whole store).
 * far_dtype R3M_SPEC_C64 / R3M_SPEC_C128: far holds the spectra of every
 *       block (r3m_build_spectral, same Dx, Dy) and the matvec evaluates the
 *       whole product from them; near (precision C64 / C128 to match) then
 *       only feeds the solver's block-Jacobi preconditioner (its d = 0 block),
 *       and max_rank is ignored. */
typedef struct {
  int32_t n;        /* macro RWG per unit */
  int32_t n_states; /* coding states; n_a = (n - n_common) / n_states */
  int32_t Dx, Dy;   /* half-extent of the displacement set */
  int32_t near_radius;
  r3m_dtype near_dtype;
  const void* near;
  r3m_dtype far_dtype;
  const void* far;
  int32_t max_rank;
  /* Connected geometries (Sec. III-B): the last n_common macro RWG are
   * shared by every state and common_ext (device, [n_common]) classes them:
   * 0 active in every unit, 1 extended toward -x (masked by D_k in the units
   * of the array's first column), 2 toward -y (first row).  A unit's reduced
   * vector is then its state's n_a entries followed by the n_common shared
   * ones, masked entries included (products write zero there and ignore
   * the input there).  Spectral stores only (R3M_ERR_UNSUPPORTED
   * otherwise); 0 / NULL for isolated units. */
  int32_t n_common;
  const int32_t* common_ext;
} r3m_store;

/* A batch of right-hand sides sharing one store (Sec. III-A: the global
 * matrix is computed once and shared across codebooks), B <= 65,535
 * (R3M_ERR_UNSUPPORTED above).  RHS b is an
 * L[2b] x L[2b+1] array (Lx, Ly <= Dx+1, Dy+1) whose codebook is
 * states[state_off[b] ...] (uint8, device, one byte per unit, < n_states),
 * and whose reduced vectors start at unit unit_off[b] of x/y.  Several RHS
 * may share one codebook (e.g. several incidence angles).
 * flags: R3M_BATCH_INDEX_READY tells r3m_retrieved_matvec that the retrieval
 * index inside its workspace is current (built by an earlier call with the
 * same store, batch shape, codebook bytes and workspace), so the call skips
 * rebuilding it; with 0 every call rebuilds it. */
#define R3M_BATCH_INDEX_READY 1u
typedef struct {
  int32_t B;
  const int32_t* L;         /* host [B][2] */
  const int64_t* unit_off;  /* host [B] */
  const int64_t* state_off; /* host [B] */
  const uint8_t* states;    /* device */
  uint32_t flags;           /* R3M_BATCH_* */
} r3m_batch;

/* -------------------------------------------------------------- matvec -- */

size_t r3m_matvec_work_bytes(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch,
                             r3m_dtype vec_dtype);

/* y_b = P_k^T Z P_k x_b for every RHS b (eq. (3); eq. (6) in reduced form):
 * y[i] = sum over units j of Z(i - j)[A(s_i), A(s_j)] x[j], with A(s) the
 * basis range of state s.  Far blocks use U (V^H x).  Vectors are C128 or C64
 * (vec_dtype), accumulation is in the store's precision (FP64 for a C128
 * store, FP32 otherwise).  The sum over displacements is reduced in a fixed
 * order (bitwise reproducible run to run).  work: r3m_matvec_work_bytes.
 * Every state byte must be < n_states: the call checks them on the device
 * (unless R3M_BATCH_INDEX_READY) and r3m_ctx_check reports a violation. */
int r3m_retrieved_matvec(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch,
                         r3m_dtype vec_dtype, const void* x_dev, void* y_dev, void* work_dev,
                         size_t work_bytes, hipStream_t stream);

/* Number of displacement groups the matvec splits the unique blocks into for
 * this (store, batch) (a launch-shape choice; results do not depend on it
 * beyond rounding order).  The first C128 r3m_retrieved_matvec or
 * r3m_gmres_solve on a (store, batch) times a few candidates on the caller's
 * stream and keeps the fastest in the context; before that the default is
 * returned.  Returns the count (>= 1), 0 for an empty batch, or a negative
 * r3m_status. */
int32_t r3m_matvec_groups(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch);

/* The whole launch plan of the matvec for this (store, batch), as the
 * autotuner chose it (or r3m_matvec_set_plan pinned it), else the default.
 * Compressed stores: bits 0-15 the displacement-group count,
 * R3M_PLAN_MFMA_FAR when the far blocks run on the matrix cores.  Spectral
 * stores (R3M_SPEC_*): R3M_PLAN_SPECTRAL, in bits 0-3 the frequency-product
 * shape (0: vector units; 1..7: matrix cores with {frequencies per wave,
 * columns per staged chunk, 16-RHS tiles per workgroup} = {1,4,1}, {2,4,1},
 * {2,8,1}, {4,4,1}, {1,8,1}, {2,4,2}, {1,8,2}; complex64 spectra only), in
 * bits 4-11 the count of live 16-RHS tiles from which
 * the matrix-core product orders its workgroups RHS tile first, in bits
 * 13-14 log2 of the groups of frequency tiles the eight XCDs split into in
 * that order (0: each XCD sees every frequency tile), and
 * R3M_PLAN_SPEC_TWO_PASS when the retrieval transforms run as separate row
 * and column passes through HBM although the fused 2-D transform (complex64
 * grids of at most 16,384 points, one grid per workgroup in LDS) applies.
 * The spectral autotuner runs on the first r3m_retrieved_matvec or
 * r3m_gmres_solve of the pair.  Every matrix-core shape and order gives the
 * same bits; the vector-unit shape and the transform form differ by FP32
 * rounding order only.  Returns the plan (> 0), 0 for an empty batch, or a
 * negative r3m_status. */
#define R3M_PLAN_SPEC_TWO_PASS (1 << 12)
#define R3M_PLAN_MFMA_FAR (1 << 16)
#define R3M_PLAN_SPECTRAL (1 << 17)
int32_t r3m_matvec_plan(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch);

/* Pins the plan of (store, batch) (the encoding of r3m_matvec_plan) in the
 * context; later matvecs and solves on the pair use it and the autotuner does
 * not run for it.  R3M_ERR_INVALID_ARG when the plan does not fit the store
 * (a matrix-core shape on complex128 spectra, R3M_PLAN_MFMA_FAR on a store
 * the matrix-core far kernel does not take, a group count outside [1, the
 * workspace's maximum], unknown bits).  An empty batch is a no-op. */
int r3m_matvec_set_plan(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, int32_t plan);

/* The per-frequency product step of the spectral matvec alone (the
 * block-Toeplitz FFT form of eq. (6): Y^(k) = Z^(k) X^(k) for every spatial
 * frequency k of the transform grid), with the (store, batch) plan: it reads
 * the transformed input grids that the last r3m_retrieved_matvec with the
 * same store, batch and workspace left in work_dev and overwrites the
 * workspace's output grids (the result vector is not touched).  Spectral
 * stores only.  For measuring the dominant step of the product on its own. */
int r3m_spectral_product(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, void* work_dev,
                         size_t work_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as r3m_retrieved_matvec, with the workspace taken from a static
 * device scratch of R3M_STATIC_SCRATCH_BYTES that the library holds on each
 * GPU until the process ends (the batch's device tables sit at its head).
 * No device or pinned memory is allocated and no workspace is passed; the
 * caller owns x and y as before.  The displacement-group count is the
 * default one (no autotuning), so results agree with r3m_retrieved_matvec to
 * rounding order, not bitwise.  R3M_ERR_BUFFER_TOO_SMALL when the batch needs
 * more scratch than that (r3m_matvec_work_bytes plus the tables); use
 * r3m_retrieved_matvec then.  Every call on a GPU shares that GPU's scratch
 * and leaves its contents behind, so calls that overlap on one GPU (other
 * streams or threads) race; R3M_BATCH_INDEX_READY refers to the index that
 * the previous static call on this GPU left there.  A new batch layout
 * uploads its tables and synchronises `stream`; otherwise asynchronous. */
#define R3M_STATIC_SCRATCH_BYTES (64u << 20)
size_t r3m_static_scratch_bytes(void);
int r3m_retrieved_matvec_static(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, r3m_dtype vec_dtype,
                                const void* x_dev, void* y_dev, hipStream_t stream);

/* ------------------------------------------------------ relaxed codebook -- */

/* Relaxed (blended) retrieval, the operator of codebook differentiation: unit
 * u of RHS b carries real state weights w[unit_off[b] + u][s] (device, FP64,
 * [total units][n_states], e.g. a softmax of logits) instead of one state.
 * The slicing matrix P_k of eq. (3) becomes the non-square blend
 *   P(w) = blockdiag_u [w[u][0] I; ...; w[u][S-1] I]   (n x n_a per unit),
 * Z_k(w) = P(w)^T Z P(w), which is eq. (3) for one-hot weights.  Computes
 * y = Z_k(w) x, or y = Z_k(w)^T x = P(w)^T Z^T P(w) x with transpose != 0
 * (the adjoint solve's operator; Z^T is block-Toeplitz with blocks Z(-d)^T).
 * The store must be spectral (R3M_SPEC_*; R3M_ERR_UNSUPPORTED otherwise);
 * batch->states must be non-NULL but are not read.  Vectors C128 or C64 as in
 * r3m_retrieved_matvec.  work: r3m_relaxed_work_bytes bytes. */
size_t r3m_relaxed_work_bytes(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch);
int r3m_relaxed_matvec(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, const double* weights_dev,
                       int32_t transpose, r3m_dtype vec_dtype, const void* x_dev, void* y_dev, void* work_dev,
                       size_t work_bytes, hipStream_t stream);

/* Gradient of a relaxed codebook's objective (the backward pass of
 * differentiation), with G = dJ/dI~ the derivative of J with respect to the
 * blended current I~ = P(w) I (Wirtinger, I~* held fixed), lam the adjoint
 * solution of Z_k(w)^T lam = P(w)^T G (r3m_gmres_solve with relaxed weights
 * and transpose), U the macro excitation (r3m_relaxed_rhs, macro = 1):
 *   dJ/dw[u][s] = dJ[b] 2 Re sum_r [ (G - Z^T P(w) lam)[u][s n_a + r] I[u][r]
 *                                   + lam[u][r] (U - Z P(w) I)[u][s n_a + r] ]
 * (dI~ = dP I + P dI and dI = Z_k^-1 (dP^T U - dP^T Z I~ - P^T Z dP I)).
 * I, lam: C128 [unit][n_a]; G, U: C128 macro [unit][n] (n = n_states n_a,
 * state order); dJ_dev: device [B] upstream factors or NULL (1); grad_dev:
 * [total units][n_states] FP64.  Complex128 spectra only. */
size_t r3m_relaxed_gradient_work_bytes(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch);
int r3m_relaxed_gradient(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, const double* weights_dev,
                         const void* I_dev, const void* lam_dev, const void* G_dev, const void* U_dev,
                         const double* dJ_dev, double* grad_dev, void* work_dev, size_t work_bytes,
                         hipStream_t stream);

/* ------------------------------------------------- near-field block ILU -- */

/* Incomplete LU of the retrieved near field (Sec. III-D: the preconditioner
 * is built per codebook after retrieval; a factor of a retrieved matrix is
 * not the retrieval of a factor).  Blocks are whole units (n_a x n_a); the
 * pattern of unit i holds the units j at Chebyshev lattice distance
 * max(|jx - ix|, |jy - iy|) <= radius, with A_ij = Z(p_i - p_j)[A(s_i), A(s_j)]
 * read from the store's near blocks (so radius <= near_radius; 1 <= radius
 * <= 3; n_a <= 64).  No fill is kept outside the pattern (ILU(0)); pivot
 * blocks are inverted by Gauss-Jordan with partial pivoting in FP64.  Units
 * are eliminated in multicolour order: unit (ix, iy) has colour
 * (iy mod (r+1)) (r+1) + (ix mod (r+1)), colours in increasing order (units
 * of one colour never share a pattern, so the order inside a colour does not
 * matter).  Arithmetic in FP64, factors stored in the store's near precision.
 *
 * Factor buffer (r3m_ilu_bytes): one factorisation per distinct codebook
 * (right-hand sides with equal state_off and array shape share it, e.g. the
 * incidence angles of one codebook), the codebooks one after another in the
 * order of their first right-hand side; per unit (u = iy Lx + ix within its
 * codebook) S = (2 radius + 1)^2 blocks; slot (ey + radius)(2 radius + 1) + ex + radius
 * holds the block of the neighbour at offset (ex, ey): the multiplier L_gj
 * (lower colour), the upper factor U_gj (higher colour), or the inverted
 * pivot U_gg^-1 at offset 0; zero for neighbours outside the array.  Blocks
 * are column-major: element (row, col) at col * n_a + row, complex double
 * (C128 near store) or float (C64). */
size_t r3m_ilu_bytes(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, int32_t radius);
/* Factors every distinct codebook of the batch.  R3M_ERR_INVALID_ARG for a
 * state byte >= n_states, R3M_ERR_NONFINITE for a singular pivot block; this
 * call synchronises the stream. */
int r3m_ilu_factor(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, int32_t radius, void* factors_dev,
                   size_t factors_bytes, hipStream_t stream);
/* y = U^-1 L^-1 x for every RHS (C128 [unit][n_a] vectors, x and y distinct;
 * y is also the scratch of the forward solve).  Asynchronous. */
int r3m_ilu_apply(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, int32_t radius, const void* factors_dev,
                  size_t factors_bytes, const void* x_dev, void* y_dev, hipStream_t stream);

/* ---------------------------------------------------------------- GMRES -- */

typedef enum {
  R3M_PRECOND_NONE = 0,
  /* right block-Jacobi preconditioner retrieved from the near field: the
   * inverse of each unit's self block Z(0)[A(s_u), A(s_u)] (one inverse per
   * coding state, FP64).  It is the diagonal-block special case of the
   * near-field block-ILU preconditioner built after retrieval (Sec. III-D). */
  R3M_PRECOND_BLOCK_JACOBI = 1,
  /* right near-field block ILU(0) preconditioner (Sec. III-D), factored once
   * per distinct codebook from its retrieved near blocks (r3m_ilu_factor with
   * opts->ilu_radius) and applied by colour-parallel triangular solves
   * (r3m_ilu_apply).  With relaxed_weights the pattern blocks are those of
   * the blended operator Z_k(w) (of Z_k(w)^T with transpose). */
  R3M_PRECOND_BLOCK_ILU = 2
} r3m_precond;

typedef struct {
  double tol;         /* relative residual target of the (inner) solve */
  int32_t restart;    /* Krylov dimension m */
  int32_t max_iter;   /* total inner iterations per solve */
  double refine_tol;  /* > 0: FP64 refinement with Z64 until ||b - Z64 x||/||b|| <= refine_tol */
  int32_t max_refine; /* outer refinement steps */
  int32_t precond;    /* r3m_precond */
  int32_t flags;      /* bit 0 (R3M_GMRES_EAGER): launch every Arnoldi step eagerly instead of
                         replaying captured HIP graphs of blocks of steps */
  const double* relaxed_weights; /* NULL, or device [total units][n_states]: solve the relaxed
                                    system Z_k(w) x = b of r3m_relaxed_matvec (spectral stores;
                                    Z64 spectral too).  R3M_PRECOND_BLOCK_JACOBI then inverts the
                                    blended self block sum_{s,s'} w_s w_s' Z(0)[A(s), A(s')] of
                                    every unit (its transpose for the adjoint);
                                    R3M_PRECOND_BLOCK_ILU factors the blended near field.  The
                                    work query only tests this pointer for NULL. */
  int32_t transpose;             /* with relaxed_weights: solve Z_k(w)^T x = b (the adjoint) */
  int32_t ilu_radius;            /* R3M_PRECOND_BLOCK_ILU pattern radius (1..3, <= near_radius);
                                    0 selects 1 */
} r3m_gmres_opts;

#define R3M_GMRES_EAGER 1

typedef struct {
  int32_t iters;       /* inner iterations (summed over refinement steps) */
  int32_t refine_steps;
  double rel_residual; /* true relative residual at exit (Z64 if given, else Z) */
  int32_t converged;
} r3m_gmres_report;

/* Workspace of r3m_gmres_solve for (Z, Z64, batch, opts).  Z64 (nullable) is
 * the refinement store the solve will be given; pass NULL when it runs
 * without refinement. */
size_t r3m_gmres_work_bytes(r3m_ctx ctx, const r3m_store* Z, const r3m_store* Z64, const r3m_batch* batch,
                            const r3m_gmres_opts* opts);

/* Solves the retrieved systems Z_k x_b = b_b (C128 vectors) with restarted
 * GMRES(m): zero initial guess, Gram-Schmidt Arnoldi (classical, repeated
 * once; on vectors above 65,536 entries per RHS the repetition runs only
 * where the first pass kept less than a tenth of ||A v_j||, unless the
 * environment sets R3M_CGS2_FULL=1) in FP64, complex Givens rotations in
 * FP64, convergence flags on the
 * device.  Blocks of Arnoldi steps run as HIP graphs captured once per
 * (store, batch, workspace, m) and replayed on a context-owned stream that is
 * ordered after `stream`; the call returns with `stream` ordered after it.  The matvec runs in the precision of Z.  If Z64 (a C128 store of the
 * same matrix) is given and opts->refine_tol > 0, an outer FP64 iterative
 * refinement computes r = b - Z64 x and solves Z d = r with the inner GMRES.
 * rep_host[B] is written; returns R3M_ERR_NOT_CONVERGED if any RHS missed the
 * tolerance (x still holds the last iterate).  Synchronises the stream.
 * Stores with shared (connected-geometry) bases: vectors in the store's
 * reduced layout, R3M_PRECOND_NONE and no relaxed weights
 * (R3M_ERR_UNSUPPORTED otherwise), Z64 with the same shared bases. */
int r3m_gmres_solve(r3m_ctx ctx, const r3m_store* Z, const r3m_store* Z64,
                    const r3m_batch* batch, const void* b_dev, void* x_dev,
                    const r3m_gmres_opts* opts, r3m_gmres_report* rep_host, void* work_dev,
                    size_t work_bytes, hipStream_t stream);

/* --------------------------------------------------- excitation and RCS -- */

/* Plane-wave right-hand sides U_k (eq. (1)), C128 [unit][n_a] per RHS:
 * U_m = int f_m . E_inc dS, E_inc = e0 e_hat exp(-j k k_hat . r),
 * k_hat = -(sin t cos p, sin t sin p, cos t), e_hat = theta_hat(t, p).
 * inc_host: [B][3] = (theta, phi, e0).  Connected geometries: [unit][n_a +
 * n_common], each basis integrated over its own triangles where they lie,
 * zero on the extended bases D_k masks (Sec. III-B). */
int r3m_plane_wave_rhs(r3m_ctx ctx, const r3m_unit_geom* geom, const r3m_batch* batch,
                       const double* inc_host, void* b_dev, hipStream_t stream);

/* Bistatic RCS sigma[b][dir] (m^2, FP64) of currents I (C128 reduced vectors):
 * N(r_hat) = sum_n I_n int f_n exp(j k r_hat . r') dS',
 * sigma = (k^2 eta^2 / 4 pi) |N - (N.r_hat) r_hat|^2 / |e0|^2.
 * dirs_host: [n_dir][2] = (theta, phi) in radians.  Connected geometries as
 * for r3m_plane_wave_rhs (masked entries of I are ignored). */
int r3m_rcs(r3m_ctx ctx, const r3m_unit_geom* geom, const r3m_batch* batch, const void* I_dev,
            int32_t n_dir, const double* dirs_host, double e0, double* sigma_dev,
            hipStream_t stream);

/* Relaxed codebook excitation: macro == 0 writes U_k(w) = P(w)^T U
 * ([unit][n_a] per RHS, C128; weights as in r3m_relaxed_matvec); macro != 0
 * writes the excitation of every macro RWG, U [unit][n] (weights unused).
 * inc_host as in r3m_plane_wave_rhs.  Synchronises the stream. */
int r3m_relaxed_rhs(r3m_ctx ctx, const r3m_unit_geom* geom, const r3m_batch* batch, const double* weights_dev,
                    const double* inc_host, int32_t macro, void* b_dev, hipStream_t stream);

/* Objective of a relaxed codebook: the bistatic RCS sigma[b][dir] of the
 * blended current I~ = P(w) I (as r3m_rcs, currents w[u][s] I[u][r] on the
 * RWGs of every state), J[b] = mean over the directions, the derivative
 * G = dJ/dI~ ([unit][n], C128) and the adjoint right-hand side P(w)^T G
 * ([unit][n_a], C128).  Synchronises the stream. */
int r3m_relaxed_objective(r3m_ctx ctx, const r3m_unit_geom* geom, const r3m_batch* batch, const double* weights_dev,
                          const void* I_dev, int32_t n_dir, const double* dirs_host, double e0, double* J_dev,
                          double* sigma_dev, void* G_dev, void* adj_dev, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* R3M_H */
