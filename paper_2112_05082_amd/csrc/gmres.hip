// Batched restarted GMRES(m) around the retrieved matvec, with optional FP64
// iterative refinement (MVP-based Krylov solution of the retrieved system,
// Sec. III-A; the paper itself used BiCGStab, Sec. IV).
//
// All Krylov vectors, Gram-Schmidt coefficients and Givens rotations are FP64
// (complex double).  Arnoldi uses classical Gram-Schmidt repeated once
// (CGS2: two projections per step, orthogonality at the level of modified
// Gram-Schmidt with two reductions instead of j+1).  Reductions are two-stage
// with fixed order (bitwise reproducible).  Convergence flags live on the
// device and are read by the host once every few iterations.
#include <cstdlib>
#include "matvec_internal.h"
#include "small_dense.h"

#include <algorithm>
#include <type_traits>

namespace r3m {

namespace {

constexpr int kTW = 8, kTH = 8;  // unit block of the matvec workgroups
constexpr int kDotChunk = 1024;
constexpr int kDotThreads = 256;
constexpr int kDotPer = kDotChunk / kDotThreads;  // elements per thread in a chunk
// basis vectors per inner-product work item: 8 for a complex64 basis (w's
// chunk read once per 8), 4 for complex128 (register count)
template <typename VB>
constexpr int dot_vec() { return sizeof(VB) == 8 ? 8 : 4; }
// The folded Gram-Schmidt update keeps up to 4 basis entries per wave in
// registers, so it takes steps with at most 16 basis vectors (with 8 per
// wave its register count leaves three waves per SIMD, and it measured no
// faster than the two separate passes).
constexpr int kFoldMaxVec = 16;
// The element-parallel update (long vectors) keeps one element's entries of
// every basis vector and folds steps of up to 32 vectors.
constexpr int kFoldMaxVecEl = 32;
constexpr int kCheckEvery = 4;

struct RhsVec {
  int64_t off;  // offset (elements) of this RHS in user-layout vectors
  int64_t N;    // unknowns
};

struct RhsState {
  double bnorm;  // norm of the right-hand side of the current (inner) solve
  double beta;   // norm of the residual at the start of the cycle
  double res;    // latest relative residual estimate
  int jdone;     // iteration at which this cycle converged, -1 while running
  int active;    // 1 while the RHS is being solved
  int budget;    // steps this cycle may take (what is left of max_iter)
  int pad;
};

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Krylov basis storage: complex128, or complex64 for inner solves on
// complex64 stores under FP64 refinement (their products carry FP32 error
// already; the basis then takes half the bytes).  Arithmetic stays FP64.
__device__ __forceinline__ double2 ld_b(const double2* p) { return *p; }
__device__ __forceinline__ double2 ld_b(const float2* p) {
  const float2 v = *p;
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st_b(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void st_b(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }

// Lists of right-hand sides with work in an Arnoldi step: rl[0..n) the
// indices in increasing order, rl[B] = n; a NULL list stands for all B (the
// kernels then test idle flags themselves).  The Krylov kernels take a fixed
// grid that strides over (listed RHS x block) items, so that the right-hand
// sides that have converged cost nothing, not even a returning workgroup.
__device__ __forceinline__ int rhs_count(const int* rl, int B) { return rl ? rl[B] : B; }
__device__ __forceinline__ int rhs_at(const int* rl, int li) { return rl ? rl[li] : li; }

// rl from idle (one workgroup of 1024 threads: each thread takes a
// contiguous run of right-hand sides, a scan of the counts places them)
__global__ void __launch_bounds__(1024) live_rhs_kernel(const int* __restrict__ idle, int B, int* __restrict__ rl) {
  __shared__ int cnt[1024];
  const int t = threadIdx.x;
  const int per = (B + 1023) / 1024;
  const int t0 = min(B, t * per), t1 = min(B, t0 + per);
  int c = 0;
  for (int b = t0; b < t1; ++b) c += idle[b] == 0 ? 1 : 0;
  cnt[t] = c;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? cnt[t - o] : 0;
    __syncthreads();
    cnt[t] += v;
    __syncthreads();
  }
  int at = cnt[t] - c;
  for (int b = t0; b < t1; ++b)
    if (idle[b] == 0) rl[at++] = b;
  if (t == 1023) rl[B] = cnt[1023];
}

// batches from which the Arnoldi steps build the list of live right-hand sides
constexpr int kListMinRhs = 64;

// grid of a strided Krylov kernel: every item when there are few, else enough
// workgroups to fill the chip several times over
inline unsigned stride_grid(int64_t items) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(items, 8192)); }

// partial[b][i][p] = sum over chunk p of conj(A_i) B
__global__ void __launch_bounds__(kDotThreads)
dots_kernel(const double2* __restrict__ A, int64_t a_stride, const double2* __restrict__ Bv,
            const RhsVec* __restrict__ rv, int nvec_max, const int* __restrict__ nvec_dev, int maxP,
            double2* __restrict__ partial) {
  __shared__ double2 sh[kDotThreads / 64];
  const int p = blockIdx.x, i = blockIdx.y, b = blockIdx.z;
  const RhsVec r = rv[b];
  const int nvec = nvec_dev ? *nvec_dev : nvec_max;
  if (i >= nvec) return;
  const int64_t P = (r.N + kDotChunk - 1) / kDotChunk;
  if (p >= P) return;
  const double2* a = A + (int64_t)i * a_stride + r.off;
  const double2* bb = Bv + r.off;
  const int64_t lo = (int64_t)p * kDotChunk;
  const int64_t hi = min(r.N, lo + kDotChunk);
  double2 s = make_double2(0.0, 0.0);
  for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
    double2 t = cmulc(a[k], bb[k]);
    s.x += t.x;
    s.y += t.y;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    s.x += __shfl_xor(s.x, o);
    s.y += __shfl_xor(s.y, o);
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 t = sh[0];
    for (int w = 1; w < kDotThreads / 64; ++w) {
      t.x += sh[w].x;
      t.y += sh[w].y;
    }
    partial[((size_t)b * nvec_max + i) * maxP + p] = t;
  }
}

// out[b][i] = sum_p partial[b][i][p] (fixed order); mode 0: store, 1: add to
// H[i][j] (CGS pass 2 accumulation) while also storing the pass value in hbuf
__global__ void dots_finish_kernel(const double2* __restrict__ partial, const RhsVec* __restrict__ rv,
                                   int nvec, int maxP, double2* __restrict__ hbuf) {
  const int b = blockIdx.x, i = threadIdx.x;
  if (i >= nvec) return;
  const int64_t P = (rv[b].N + kDotChunk - 1) / kDotChunk;
  double2 s = make_double2(0.0, 0.0);
  for (int p = 0; p < P; ++p) {
    double2 t = partial[((size_t)b * nvec + i) * maxP + p];
    s.x += t.x;
    s.y += t.y;
  }
  hbuf[(size_t)b * nvec + i] = s;
}

// Givens step on column j of H for RHS b, run by one whole block: the column
// (with H[j+1][j] = hn) and the previous rotations are staged in LDS by all
// threads, thread 0 applies the rotations in order, forms the new one, updates
// g and the convergence state, and the block writes the column back.
// lds: (m + 2) + m double2 and m double.  Every thread must call it.
__device__ void givens_step_block(int b, double2* __restrict__ H, double2* __restrict__ g, double* __restrict__ cs,
                                  double2* __restrict__ sn, RhsState* __restrict__ st, int m, int j, double tol,
                                  int* __restrict__ n_running, double hn, double2* lds, int* __restrict__ idle) {
  RhsState s = st[b];
  if (!s.active || s.jdone >= 0) return;  // uniform over the block
  double2* h = H + (size_t)b * (m + 1) * m;
  double* c = cs + (size_t)b * m;
  double2* sv = sn + (size_t)b * m;
  double2* gg = g + (size_t)b * (m + 1);
  double2* col = lds;
  double2* ssv = lds + (m + 2);
  double* cc = reinterpret_cast<double*>(ssv + m);
  for (int i = threadIdx.x; i <= j; i += blockDim.x) col[i] = h[i * m + j];
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    cc[i] = c[i];
    ssv[i] = sv[i];
  }
  if (threadIdx.x == 0) col[j + 1] = make_double2(hn, 0.0);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < j; ++i) {
      const double2 hi = col[i], hi1 = col[i + 1];
      const double ci = cc[i];
      const double2 si = ssv[i];
      // [c s; -conj(s) c] [hi; hi1]
      col[i] = make_double2(ci * hi.x + (si.x * hi1.x - si.y * hi1.y), ci * hi.y + (si.x * hi1.y + si.y * hi1.x));
      col[i + 1] = make_double2(-(si.x * hi.x + si.y * hi.y) + ci * hi1.x, -(si.x * hi.y - si.y * hi.x) + ci * hi1.y);
    }
    const double2 a = col[j], bb = col[j + 1];
    const double na = hypot(a.x, a.y), nb = hypot(bb.x, bb.y);
    double cj;
    double2 sj, rj;
    if (nb == 0.0) {
      cj = 1.0;
      sj = make_double2(0.0, 0.0);
      rj = a;
    } else if (na == 0.0) {
      cj = 0.0;
      sj = make_double2(1.0, 0.0);
      rj = bb;
    } else {
      const double nu = hypot(na, nb);
      const double2 ph = make_double2(a.x / na, a.y / na);
      cj = na / nu;
      // s = ph * conj(b) / nu
      sj = make_double2((ph.x * bb.x + ph.y * bb.y) / nu, (ph.y * bb.x - ph.x * bb.y) / nu);
      rj = make_double2(ph.x * nu, ph.y * nu);
    }
    c[j] = cj;
    sv[j] = sj;
    col[j] = rj;
    col[j + 1] = make_double2(0.0, 0.0);
    const double2 gj = gg[j];
    // g[j+1] = -conj(s) g[j];  g[j] = c g[j]
    const double2 gj1 = make_double2(-(sj.x * gj.x + sj.y * gj.y), -(sj.x * gj.y - sj.y * gj.x));
    gg[j + 1] = gj1;
    gg[j] = make_double2(cj * gj.x, cj * gj.y);
    const double res = s.bnorm > 0.0 ? hypot(gj1.x, gj1.y) / s.bnorm : 0.0;
    s.res = res;
    if (!(res > tol) || nb == 0.0 || j == m - 1 || j + 1 >= s.budget) {
      s.jdone = j + 1;
      if (idle) idle[b] = 1;  // the rest of the cycle skips this right-hand side
    } else {
      atomicAdd(n_running, 1);
    }
    st[b] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) h[i * m + j] = col[i];
}

// Sum of n partials by the 64 lanes of one wave: lane t adds entries t, t+64,
// ... in order, then a fixed butterfly; every lane returns the total.
__device__ double wave_sum_partials(const volatile double* p, int n) {
  double acc = 0.0;
  for (int q = (int)(threadIdx.x & 63); q < n; q += 64) acc += p[q];
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  return acc;
}
__device__ double2 wave_sum_partials2(const volatile double2* p, int n) {
  double2 acc = make_double2(0.0, 0.0);
  for (int q = (int)(threadIdx.x & 63); q < n; q += 64) {
    acc.x += p[q].x;
    acc.y += p[q].y;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    acc.x += __shfl_xor(acc.x, o);
    acc.y += __shfl_xor(acc.y, o);
  }
  return acc;
}

// Block sum of a double2 over the 256 threads (fixed order).
__device__ double2 block_sum2(double2 v, double2* sh) {
  for (int o = 32; o >= 1; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double2 t = sh[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
    t.x += sh[w].x;
    t.y += sh[w].y;
  }
  __syncthreads();
  return t;
}

__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }

// Sums over the 64 lanes of a wave of NV complex values per lane (NV a power
// of two up to 32), by exchanging half of the remaining values at each of the
// first log2(NV) butterfly steps (lane bit 5 keeps the upper half, bit 4 the
// upper quarter, ...) and plain butterfly steps after that: on return x[0] of
// lane l is the total of value l >> (6 - log2 NV).  Fixed order; NV - 1 +
// 6 - log2(NV) exchanges instead of 6 NV.
// O0 < 32: the exchanges start at that lane distance (the steps above it
// done by the caller).
template <int NV, int O0 = 32>
__device__ __forceinline__ void wave_transpose_sum(double2 (&x)[NV], int lane) {
  constexpr int L = NV == 1 ? 0 : NV == 2 ? 1 : NV == 4 ? 2 : NV == 8 ? 3 : NV == 16 ? 4 : 5;
  static_assert((1 << L) == NV, "NV must be a power of two up to 32");
#pragma unroll
  for (int st = 0; st < L; ++st) {
    const int o = O0 >> st, half = NV >> (st + 1);
    const bool hi = (lane & o) != 0;
#pragma unroll
    for (int t = 0; t < half; ++t) {
      const double2 a = x[t], b = x[t + half];
      const double2 send = hi ? a : b;
      double2 keep = hi ? b : a;
      keep.x += __shfl_xor(send.x, o);
      keep.y += __shfl_xor(send.y, o);
      x[t] = keep;
    }
  }
#pragma unroll
  for (int o = O0 >> L; o >= 1; o >>= 1) {
    x[0].x += __shfl_xor(x[0].x, o);
    x[0].y += __shfl_xor(x[0].y, o);
  }
}

// Chunk partials of <A_i, B> for i < nvec: partial[b][i][p].  Work item
// (b, grp, p) takes chunk p of RHS b against the kDotVec vectors of group
// grp (dot_vec); B's chunk is loaded once and all loads are issued before the products
// (basis entries kept in their stored type).  Each wave sums its lanes'
// products with wave_transpose_sum, then the block adds the waves in a fixed
// order.  The blocks stride over the items of the right-hand sides of rl (a
// live list, see rhs_count), or of all B.  The consumer kernel sums the
// partials itself (no grid-wide fence here).
template <typename VB, typename WB, int DV = dot_vec<VB>()>
__global__ void __launch_bounds__(kDotThreads)
dots_partials_kernel(const VB* __restrict__ A, int64_t a_stride, const WB* __restrict__ Bv,
                     const RhsVec* __restrict__ rv, int nvec, int maxP, double2* __restrict__ partial,
                     int* __restrict__ reset, const int* __restrict__ live, const int* __restrict__ idle,
                     const int* __restrict__ rl, int B) {
  constexpr int kDotVec = DV;  // vectors per item (fewer for small bases)
  constexpr int kShV = kDotVec == 1 ? 6 : kDotVec == 2 ? 5 : kDotVec == 4 ? 4 : kDotVec == 8 ? 3 : 2;
  static_assert(kDotVec == 1 || kDotVec == 2 || kDotVec == 4 || kDotVec == 8 || kDotVec == 16, "kDotVec");
  __shared__ double2 sh[kDotThreads / 64][kDotVec];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // this step's running count starts at zero (done before the exit test, so a
  // skipped step still leaves it zero for the next one)
  if (reset && blockIdx.x == 0 && tid == 0) *reset = 0;
  if (live && *live == 0) return;
  const int ngrp = (nvec + kDotVec - 1) / kDotVec;
  const int64_t per = (int64_t)maxP * ngrp, items = per * rhs_count(rl, B);
  for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {  // uniform over the block
    const int li = (int)(item / per);
    const int64_t rem = item - li * per;
    const int grp = (int)(rem / maxP), p = (int)(rem - (int64_t)grp * maxP);
    const int b = rhs_at(rl, li);
    if (!rl && idle && idle[b]) continue;
    const RhsVec r = rv[b];
    const int64_t P = (r.N + kDotChunk - 1) / kDotChunk;
    if (p >= P) continue;
    const int i0 = grp * kDotVec;
    const int nv = min(kDotVec, nvec - i0);
    const WB* bb = Bv + r.off;
    const int64_t lo = (int64_t)p * kDotChunk + tid;
    double2 wv[kDotPer];
#pragma unroll
    for (int e = 0; e < kDotPer; ++e) {
      const int64_t k = lo + (int64_t)e * kDotThreads;
      wv[e] = k < r.N ? ld_b(bb + k) : make_double2(0.0, 0.0);
    }
    VB av[kDotVec][kDotPer];
#pragma unroll
    for (int q = 0; q < kDotVec; ++q) {
      if (q < nv) {  // uniform
        const VB* a = A + (int64_t)(i0 + q) * a_stride + r.off;
#pragma unroll
        for (int e = 0; e < kDotPer; ++e) {
          const int64_t k = lo + (int64_t)e * kDotThreads;
          av[q][e] = k < r.N ? a[k] : VB{};
        }
      }
    }
    double2 acc[kDotVec];
#pragma unroll
    for (int q = 0; q < kDotVec; ++q) {
      acc[q] = make_double2(0.0, 0.0);
      if (q < nv) {
#pragma unroll
        for (int e = 0; e < kDotPer; ++e) {
          const double2 t = cmulc(to_d2(av[q][e]), wv[e]);
          acc[q].x += t.x;
          acc[q].y += t.y;
        }
      }
    }
    wave_transpose_sum<kDotVec>(acc, lane);
    {
      const int vi = lane >> kShV;
      if ((lane & ((1 << kShV) - 1)) == 0) sh[wave][vi] = acc[0];
    }
    __syncthreads();
    if (tid < nv) {
      double2 t = sh[0][tid];
      for (int w = 1; w < kDotThreads / 64; ++w) {
        t.x += sh[w][tid].x;
        t.y += sh[w][tid].y;
      }
      partial[((size_t)b * nvec + i0 + tid) * maxP + p] = t;
    }
    __syncthreads();  // sh is reused by the next item
  }
}

// Long vectors: the partials of dots_partials_kernel (one per part_chunk
// elements) or of the folded update (one per update block) summed once, in a
// fixed order, into out[b][i] (grid (nvec, B)), so that the update kernel's
// blocks read one value per vector instead of every partial.
__global__ void __launch_bounds__(256)
finish_partials_kernel(const double2* __restrict__ partial, int maxP, int nvec, const RhsVec* __restrict__ rv,
                       double2* __restrict__ out, const int* __restrict__ run_prev, const int* __restrict__ idle,
                       int part_chunk) {
  if (run_prev && *run_prev == 0) return;
  if (idle && idle[blockIdx.y]) return;
  __shared__ double2 sh[4];
  const int i = blockIdx.x, b = blockIdx.y;
  const int64_t P = (rv[b].N + part_chunk - 1) / part_chunk;
  const double2* pp = partial + ((size_t)b * nvec + i) * maxP;
  double2 t = make_double2(0.0, 0.0);
  for (int64_t p = threadIdx.x; p < P; p += blockDim.x) {
    t.x += pp[p].x;
    t.y += pp[p].y;
  }
  t = block_sum2(t, sh);
  if (threadIdx.x == 0) out[(size_t)b * nvec + i] = t;
}

// the per-block parts of ||w||^2 summed once into out[b] (grid B)
__global__ void __launch_bounds__(256)
finish_norm_kernel(const double* __restrict__ npart, int maxB, const RhsVec* __restrict__ rv,
                   double* __restrict__ out, const int* __restrict__ run_prev, const int* __restrict__ idle,
                   int nsub) {
  if (run_prev && *run_prev == 0) return;
  if (idle && idle[blockIdx.x]) return;
  __shared__ double2 sh[4];
  const int b = blockIdx.x;
  const int64_t nb = (rv[b].N + 64 * nsub - 1) / (64 * nsub);  // gs_update_kernel's blocks
  double t = 0.0;
  for (int64_t q = threadIdx.x; q < nb; q += blockDim.x) t += npart[(size_t)b * maxB + q];
  const double2 s2 = block_sum2(make_double2(t, 0.0), sh);
  if (threadIdx.x == 0) out[b] = s2.x;
}

// w -= sum_{i<nvec} h_i V_i with h_i the sum of the partials of the preceding
// dots launch (n_part of them per vector; 0: one per part_chunk elements),
// taken by every block in the same fixed order (block 0 also records them in
// H: mode 0 H[i][j] = h_i, mode 1 H[i][j] += h_i).  A block takes nsub runs of
// 64 elements in turn; its four waves take the vectors i = q mod 4 (q = wave)
// and their sums are added in wave order.  With do_norm, each block also
// writes its part of ||w||^2 to npart[b][block].
// KV > 0 folds the second Gram-Schmidt pass's inner products into the first
// pass's update (nvec <= 4 KV): each wave keeps its KV basis entries of the
// element in registers, and once the updated w is known forms conj(V_i) w for
// them, so that the basis is streamed once for both; partial2[b][i][block]
// receives the block's sums (fixed lane and run order).
// Blocks (of nsub runs, nb_max per RHS) are work items strided over by the
// grid, for the right-hand sides of rl (see rhs_count).
// Dynamic LDS: nvec double2.
template <int KV, typename VB, typename WB>
__global__ void __launch_bounds__(256)
gs_update_kernel(const VB* __restrict__ V, WB* __restrict__ w, const RhsVec* __restrict__ rv,
                 const RhsState* __restrict__ st, const double2* __restrict__ partial, int maxP, int n_part,
                 int nvec, int64_t ut, int do_norm, double* __restrict__ npart, int maxB, double2* __restrict__ H,
                 int m, int j, int mode, const int* __restrict__ run_prev, const int* __restrict__ idle,
                 int nsub, int part_chunk, double2* __restrict__ partial2, int maxP2, const int* __restrict__ rl,
                 int B, int64_t nb_max) {
  if (run_prev && *run_prev == 0) return;
  extern __shared__ double2 hb[];
  __shared__ double2 sh[4];
  __shared__ double2 part[3][64];
  __shared__ double2 wnew[64];
  const int e = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t items = nb_max * rhs_count(rl, B);
  for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {  // uniform over the block
    const int li = (int)(item / nb_max);
    const int64_t blk = item - li * nb_max;
    const int b = rhs_at(rl, li);
    if (!rl && idle && idle[b]) continue;
    const RhsVec r = rv[b];
    const int64_t nb = (r.N + 64 * nsub - 1) / (64 * nsub);
    if (blk >= nb) continue;
    const int P = n_part > 0 ? n_part : (int)((r.N + part_chunk - 1) / part_chunk);
    __syncthreads();  // the previous item's reads of hb are done
    for (int i = threadIdx.x; i < nvec; i += blockDim.x) {
      const double2* pp = partial + ((size_t)b * nvec + i) * maxP;
      double2 t = make_double2(0.0, 0.0);
      for (int p = 0; p < P; ++p) {
        const double2 v = pp[p];
        t.x += v.x;
        t.y += v.y;
      }
      hb[i] = t;
      if (blk == 0) {
        double2* h = H + (size_t)b * (m + 1) * m + (size_t)i * m + j;
        if (mode == 0) {
          *h = t;
        } else {
          h->x += t.x;
          h->y += t.y;
        }
      }
    }
    __syncthreads();
    const bool act = st[b].active;
    double nrm2 = 0.0;
    double2 d2[KV > 0 ? KV : 1];
#pragma unroll
    for (int t = 0; t < (KV > 0 ? KV : 1); ++t) d2[t] = make_double2(0.0, 0.0);
    for (int sb = 0; sb < nsub; ++sb) {  // uniform trip count: the barriers below are reached by all
      const int64_t k = (blk * nsub + sb) * 64 + e;
      const bool live = k < r.N && act;
      double2 acc = make_double2(0.0, 0.0);
      // wave 0 reads w with the basis entries, so that the update after the
      // barrier does not wait for memory
      const double2 wpre = q == 0 && live ? ld_b(w + r.off + k) : make_double2(0.0, 0.0);
      double2 vv[KV > 0 ? KV : 1];
      if (KV > 0) {
        if (live) {
          const VB* vk = V + r.off + k;
#pragma unroll
          for (int t = 0; t < KV; ++t) {
            const int i = q + 4 * t;
            vv[t] = i < nvec ? ld_b(vk + (int64_t)i * ut) : make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int t = 0; t < KV; ++t) {
            const int i = q + 4 * t;
            if (i < nvec) {
              const double2 c = cmul(hb[i], vv[t]);
              acc.x += c.x;
              acc.y += c.y;
            }
          }
        }
      } else if (live) {
        const VB* vk = V + r.off + k;
        int i = q;
        for (; i + 12 < nvec; i += 16) {
          const double2 v0 = ld_b(vk + (int64_t)i * ut), v1 = ld_b(vk + (int64_t)(i + 4) * ut);
          const double2 v2 = ld_b(vk + (int64_t)(i + 8) * ut), v3 = ld_b(vk + (int64_t)(i + 12) * ut);
          const double2 t0 = cmul(hb[i], v0), t1 = cmul(hb[i + 4], v1);
          const double2 t2 = cmul(hb[i + 8], v2), t3 = cmul(hb[i + 12], v3);
          acc.x += t0.x;
          acc.y += t0.y;
          acc.x += t1.x;
          acc.y += t1.y;
          acc.x += t2.x;
          acc.y += t2.y;
          acc.x += t3.x;
          acc.y += t3.y;
        }
        for (; i < nvec; i += 4) {
          const double2 t = cmul(hb[i], ld_b(vk + (int64_t)i * ut));
          acc.x += t.x;
          acc.y += t.y;
        }
      }
      if (q > 0) part[q - 1][e] = acc;
      __syncthreads();
      if (q == 0 && live) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          acc.x += part[t][e].x;
          acc.y += part[t][e].y;
        }
        double2 wk = wpre;
        wk.x -= acc.x;
        wk.y -= acc.y;
        st_b(w + r.off + k, wk);
        nrm2 += wk.x * wk.x + wk.y * wk.y;
        if (KV > 0) wnew[e] = wk;
      }
      __syncthreads();  // part (and wnew) are reused by the next run
      if (KV > 0 && live) {
        // (the next run writes wnew only after its first barrier, which every
        // wave reaches after these reads)
        const double2 wk = wnew[e];
#pragma unroll
        for (int t = 0; t < KV; ++t) {
          const double2 c = cmulc(vv[t], wk);
          d2[t].x += c.x;
          d2[t].y += c.y;
        }
      }
    }
    if (KV > 0) {
#pragma unroll
      for (int t = 0; t < KV; ++t) {
        double2 v = d2[t];
        for (int o = 32; o >= 1; o >>= 1) {
          v.x += __shfl_xor(v.x, o);
          v.y += __shfl_xor(v.y, o);
        }
        const int i = q + 4 * t;
        if (e == 0 && i < nvec) partial2[((size_t)b * nvec + i) * maxP2 + blk] = v;
      }
    }
    if (do_norm) {
      const double2 t = block_sum2(make_double2(nrm2, 0.0), sh);
      if (threadIdx.x == 0) npart[(size_t)b * maxB + blk] = t.x;
    }
  }
}

// The update of gs_update_kernel for long vectors (blocks of four 64-element
// runs): every thread takes its own element of the block and loops over the
// basis vectors (loads issued in groups before the products), so that all
// four waves stream at every basis size.  NV > 0 folds the second pass's
// inner products (nvec <= NV <= kFoldMaxVecEl, NV a power of two up to 16 or
// 20, 24 or 32): the element's basis entries
// stay in registers, each wave sums conj(V_i) w over its lanes
// (wave_transpose_sum) and the block adds the waves in a fixed order into
// partial2[b][i][block].  Same arguments and outputs as gs_update_kernel with
// nsub = 4.  skip_nsum (nullable; a second pass, mode 1): ||w||^2 after the
// first pass per RHS; the pass then leaves w, its norm parts and H alone for
// every RHS whose first pass kept ||w|| >= eta ||A v_j|| (with A v_j =
// sum_i H[i][j] V_i + w: ||w||^2 >= eta^2 / (1 - eta^2) sum_i |H[i][j]|^2),
// the criterion of Kahan and Parlett: after one projection the part of w
// left in the basis's span is of the order of the rounding unit times
// ||A v_j||, at most 1/eta times the rounding unit relative to ||w||.
constexpr double kCgs2Eta = 0.1;
template <int NV, typename VB, typename WB>
__global__ void __launch_bounds__(256, NV == 20 ? 4 : 1)
gs_update_el_kernel(const VB* __restrict__ V, WB* __restrict__ w, const RhsVec* __restrict__ rv,
                    const RhsState* __restrict__ st, const double2* __restrict__ partial, int maxP, int n_part,
                    int nvec, int64_t ut, int do_norm, double* __restrict__ npart, int maxB,
                    double2* __restrict__ H, int m, int j, int mode, const int* __restrict__ run_prev,
                    const int* __restrict__ idle, int part_chunk, double2* __restrict__ partial2, int maxP2,
                    const int* __restrict__ rl, int B, int64_t nb_max, const double* __restrict__ skip_nsum) {
  if (run_prev && *run_prev == 0) return;
  constexpr bool FOLD = NV > 0;
  constexpr int kEl = 256;  // elements per block: four 64-element runs
  extern __shared__ double2 hb[];
  __shared__ double2 sh[4];
  __shared__ double2 red[4][FOLD ? NV : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t items = nb_max * rhs_count(rl, B);
  for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {  // uniform over the block
    const int li = (int)(item / nb_max);
    const int64_t blk = item - li * nb_max;
    const int b = rhs_at(rl, li);
    if (!rl && idle && idle[b]) continue;
    const RhsVec r = rv[b];
    const int64_t nb = (r.N + kEl - 1) / kEl;
    if (blk >= nb) continue;
    if (skip_nsum) {  // the same decision in every block of the RHS
      double hh = 0.0;
      for (int i = 0; i < nvec; ++i) {
        const double2 h = H[(size_t)b * (m + 1) * m + (size_t)i * m + j];
        hh += h.x * h.x + h.y * h.y;
      }
      if (skip_nsum[b] >= kCgs2Eta * kCgs2Eta / (1.0 - kCgs2Eta * kCgs2Eta) * hh) continue;  // uniform
    }
    const int P = n_part > 0 ? n_part : (int)((r.N + part_chunk - 1) / part_chunk);
    // this item's element of w and of the basis (the first 8 vectors without
    // folding) are loaded before the coefficient sums, which do not need them
    const int64_t k = blk * kEl + tid;
    const bool live = k < r.N && st[b].active;
    double2 wk = live ? ld_b(w + r.off + k) : make_double2(0.0, 0.0);
    VB vv[FOLD ? NV : 8];
    const VB* vk = V + r.off + k;
    if (live) {
#pragma unroll
      for (int i = 0; i < (FOLD ? NV : 8); ++i)
        if (i < nvec) vv[i] = vk[(int64_t)i * ut];
    }
    __syncthreads();  // the previous item's reads of hb and red are done
    for (int i = tid; i < nvec; i += blockDim.x) {
      const double2* pp = partial + ((size_t)b * nvec + i) * maxP;
      double2 t = make_double2(0.0, 0.0);
      for (int p = 0; p < P; ++p) {
        const double2 v = pp[p];
        t.x += v.x;
        t.y += v.y;
      }
      hb[i] = t;
      if (blk == 0) {
        double2* h = H + (size_t)b * (m + 1) * m + (size_t)i * m + j;
        if (mode == 0) {
          *h = t;
        } else {
          h->x += t.x;
          h->y += t.y;
        }
      }
    }
    __syncthreads();
    double nrm2 = 0.0;
    if (live) {
      double2 acc = make_double2(0.0, 0.0);
      if (FOLD) {
#pragma unroll
        for (int i = 0; i < (FOLD ? NV : 8); ++i)
          if (i < nvec) {
            const double2 c = cmul(hb[i], to_d2(vv[i]));
            acc.x += c.x;
            acc.y += c.y;
          }
      } else {
        for (int i0 = 0; i0 < nvec; i0 += 8) {
          if (i0 > 0) {  // the first 8 were loaded above
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (i0 + u < nvec) vv[u] = vk[(int64_t)(i0 + u) * ut];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (i0 + u < nvec) {
              const double2 c = cmul(hb[i0 + u], to_d2(vv[u]));
              acc.x += c.x;
              acc.y += c.y;
            }
        }
      }
      wk.x -= acc.x;
      wk.y -= acc.y;
      st_b(w + r.off + k, wk);
      nrm2 = wk.x * wk.x + wk.y * wk.y;
    }
    if (FOLD) {
      constexpr int NF = FOLD ? NV : 1;
      auto dot = [&](int i) {
        return (live && i < nvec && i < NF) ? cmulc(to_d2(vv[i < NF ? i : 0]), wk) : make_double2(0.0, 0.0);
      };
      // the first (up to) 16 products, then the rest padded to a power of
      // two (fewer live registers than one sum over all of them)
      auto fold_sum = [&](auto nh_c, int h0) {
        constexpr int NH = decltype(nh_c)::value;
        constexpr int sh_v = NH == 1 ? 6 : NH == 2 ? 5 : NH == 4 ? 4 : NH == 8 ? 3 : 2;
        double2 d[NH];
#pragma unroll
        for (int i = 0; i < NH; ++i) d[i] = dot(h0 + i);
        wave_transpose_sum<NH>(d, lane);
        const int vi = h0 + (lane >> sh_v);  // the value this lane holds the total of
        if ((lane & ((1 << sh_v) - 1)) == 0 && vi < nvec) red[wave][vi] = d[0];
      };
      constexpr int NA = NF > 16 ? 16 : NF, NR = NF - NA;
      constexpr int NB = NR == 0 ? 1 : NR <= 2 ? 2 : NR <= 4 ? 4 : NR <= 8 ? 8 : 16;
      fold_sum(std::integral_constant<int, NA>(), 0);
      if constexpr (NR > 0) {
        if (nvec > 16) fold_sum(std::integral_constant<int, NB>(), 16);  // uniform
      }
      __syncthreads();
      if (tid < nvec) {
        double2 t = red[0][tid];
#pragma unroll
        for (int q = 1; q < 4; ++q) {
          t.x += red[q][tid].x;
          t.y += red[q][tid].y;
        }
        partial2[((size_t)b * nvec + tid) * maxP2 + blk] = t;
      }
    }
    if (do_norm) {
      const double2 t = block_sum2(make_double2(nrm2, 0.0), sh);
      if (tid == 0) npart[(size_t)b * maxB + blk] = t.x;
    }
  }
}

// The second Gram-Schmidt pass of the folded updates is selective (see
// gs_update_el_kernel's skip_nsum) unless R3M_CGS2_FULL=1 asks for it at
// every step.
bool selective_cgs2() {
  static const bool sel = [] {
    const char* env = std::getenv("R3M_CGS2_FULL");
    return !(env && env[0] == '1');
  }();
  return sel;
}

// ||w|| from the per-block parts of the preceding gs_update_kernel (n_npart
// of them; 0: one per 64 elements), summed by every block in the same fixed
// order; block 0 sets H[j+1][j] = ||w|| and
// applies the Givens step; every block writes V_{j+1} = w / ||w|| (zeros for
// a finished RHS or a breakdown) and, for the next step's matvec, its input
// in the store precision OT: V_{j+1} itself (MODE 1) or M^{-1} V_{j+1}
// (MODE 2, block-Jacobi; a block holds whole units).  MODE 0 writes V only.
// Blocks (nb_max per RHS) are work items strided over by the grid, for the
// right-hand sides of rl (see rhs_count).
// RW = 2 or 4 (MODE 2 with staged inverses, n_a a multiple of RW): a block
// item holds RW times the units, each thread normalises RW elements and then
// forms RW consecutive rows of its unit's product (one read of the unit's
// entry and 8 RW bytes of the inverse per column serve all RW rows).
template <typename OT, int MODE, typename VB, typename WB, int RW = 1>
__global__ void __launch_bounds__(256)
normalize_step_kernel(const WB* __restrict__ w, VB* __restrict__ V, const RhsVec* __restrict__ rv,
                      RhsState* __restrict__ st, const double* __restrict__ npart, int maxB, int n_npart,
                      double2* __restrict__ H, double2* __restrict__ g, double* __restrict__ cs,
                      double2* __restrict__ sn, int m, int j, double tol, int* __restrict__ n_running,
                      double* __restrict__ wn, int64_t ut, const int* __restrict__ live,
                      const double2* __restrict__ Minv, const uint8_t* __restrict__ states,
                      const int64_t* __restrict__ soff, int n_a, int n_states, OT* __restrict__ xs, int per_unit,
                      int* __restrict__ idle, const int* __restrict__ rl, int B, int64_t nb_max, int stage) {
  if (live && *live == 0) return;
  __shared__ double nv_s;
  constexpr bool R2 = RW > 1;
  __shared__ double2 v_s[R2 ? 1 : 256];
  __shared__ float2 v2_s[R2 ? 256 * RW : 1];
  extern __shared__ double2 glds[];
  const int64_t items = nb_max * rhs_count(rl, B);
  // stage: the block-Jacobi inverses of every state, rounded to complex64, in
  // LDS after the Givens scratch (one read per workgroup instead of one per
  // element; a complex64 product needs no more)
  float2* Ms = reinterpret_cast<float2*>(glds + (2 * m + 2) + (m + 1) / 2);
  if (MODE == 2 && stage && (int64_t)blockIdx.x < items) {
    for (int t = threadIdx.x; t < n_states * n_a * n_a; t += blockDim.x)
      Ms[t] = make_float2((float)Minv[t].x, (float)Minv[t].y);
    __syncthreads();
  }
  for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {  // uniform over the block
    const int li = (int)(item / nb_max);
    const int64_t blk = item - li * nb_max;
    const int b = rhs_at(rl, li);
    if (idle) {
      // a right-hand side not being solved, or converged at an earlier step of
      // this cycle, has no step left to finish (its V_{j+1} is never read).
      // Tested on the state, not on idle[b], which the Givens step of this
      // launch may set (the state's jdone changes here only from -1 to j + 1)
      const RhsState si = st[b];
      if (!si.active || (si.jdone >= 0 && si.jdone <= j)) continue;
    }
    const RhsVec r = rv[b];
    const int64_t nb = (r.N + 63) / 64;
    if (blk * RW * blockDim.x >= r.N) continue;  // uniform over the block
    __syncthreads();  // the previous item's reads of nv_s and v_s are done
    if (threadIdx.x < 64) {
      const double sum = wave_sum_partials(npart + (size_t)b * maxB, n_npart > 0 ? n_npart : (int)nb);
      if (threadIdx.x == 0) nv_s = sqrt(fmax(sum, 0.0));
    }
    __syncthreads();
    const double nv = nv_s;
    // the running test reads only fields the Givens step below leaves alone or
    // changes to a value with the same outcome (jdone: -1 -> j + 1)
    const RhsState s0 = st[b];
    const bool ok = s0.active && (s0.jdone < 0 || s0.jdone == j + 1) && nv > 0.0;
    const double inv = ok ? 1.0 / nv : 0.0;  // one division per item, not per element
    if constexpr (R2) {
      const int64_t base = blk * RW * blockDim.x;
#pragma unroll
      for (int e = 0; e < RW; ++e) {
        const int64_t ke = base + e * blockDim.x + threadIdx.x;
        double2 ve = make_double2(0.0, 0.0);
        if (ke < r.N) {
          const double2 wk = ld_b(w + r.off + ke);
          if (ok) ve = make_double2(wk.x * inv, wk.y * inv);
          st_b(V + (int64_t)(j + 1) * ut + r.off + ke, ve);
        }
        v2_s[e * blockDim.x + threadIdx.x] = make_float2((float)ve.x, (float)ve.y);
      }
      __syncthreads();
      const int hp = n_a / RW, ul = threadIdx.x / hp, p2 = RW * (threadIdx.x - ul * hp);
      const int64_t k0 = base + (int64_t)ul * n_a + p2;  // rows p2 .. p2 + RW - 1 of local unit ul
      if (k0 < r.N) {
        const int64_t u = k0 / n_a;
        const int64_t sidx = min((int)states[soff[b] + u], n_states - 1);
        const float2* M = Ms + (size_t)sidx * n_a * n_a + p2;  // column-major
        const float2* vu = v2_s + ul * n_a;
        float ax[RW], ay[RW];
#pragma unroll
        for (int q = 0; q < RW; ++q) ax[q] = ay[q] = 0.f;
        for (int c = 0; c < n_a; ++c) {
          const float2 x = vu[c];
#pragma unroll
          for (int h = 0; h < RW / 2; ++h) {
            const float4 mm = *reinterpret_cast<const float4*>(M + (size_t)c * n_a + 2 * h);
            ax[2 * h] += mm.x * x.x - mm.y * x.y;
            ay[2 * h] += mm.x * x.y + mm.y * x.x;
            ax[2 * h + 1] += mm.z * x.x - mm.w * x.y;
            ay[2 * h + 1] += mm.z * x.y + mm.w * x.x;
          }
        }
#pragma unroll
        for (int q = 0; q < RW; ++q) {
          xs[2 * (r.off + k0 + q)] = (OT)ax[q];
          xs[2 * (r.off + k0 + q) + 1] = (OT)ay[q];
        }
      }
      if (blk == 0) {  // uniform over the block
        if (threadIdx.x == 0) wn[b] = nv;
        givens_step_block(b, H, g, cs, sn, st, m, j, tol, n_running, nv, glds, idle);
      }
      continue;
    }
    const int64_t k = blk * blockDim.x + threadIdx.x;
    const bool in = k < r.N;
    double2 v = make_double2(0.0, 0.0);
    if (in) {
      const double2 wk = ld_b(w + r.off + k);
      if (ok) v = make_double2(wk.x * inv, wk.y * inv);
      st_b(V + (int64_t)(j + 1) * ut + r.off + k, v);
    }
    if (MODE == 1 && in) {
      xs[2 * (r.off + k)] = (OT)v.x;
      xs[2 * (r.off + k) + 1] = (OT)v.y;
    }
    if (MODE == 2) {
      v_s[threadIdx.x] = v;
      __syncthreads();
      if (in) {
        const int64_t u = k / n_a;
        const int mr = (int)(k % n_a);
        const int64_t sidx = per_unit ? r.off / n_a + u : min((int)states[soff[b] + u], n_states - 1);
        const double2* vu = v_s + (threadIdx.x / n_a) * n_a;
        if (stage) {
          const float2* M = Ms + (size_t)sidx * n_a * n_a + mr;  // column-major
          float2 acc = make_float2(0.f, 0.f);
          for (int c = 0; c < n_a; ++c) {
            const float2 mm = M[(size_t)c * n_a];
            const float vx = (float)vu[c].x, vy = (float)vu[c].y;
            acc.x += mm.x * vx - mm.y * vy;
            acc.y += mm.x * vy + mm.y * vx;
          }
          xs[2 * (r.off + k)] = (OT)acc.x;
          xs[2 * (r.off + k) + 1] = (OT)acc.y;
        } else {
          const double2* M = Minv + (size_t)sidx * n_a * n_a + mr;  // column-major
          double2 acc = make_double2(0.0, 0.0);
          for (int c = 0; c < n_a; ++c) {
            const double2 t = cmul(M[(size_t)c * n_a], vu[c]);
            acc.x += t.x;
            acc.y += t.y;
          }
          xs[2 * (r.off + k)] = (OT)acc.x;
          xs[2 * (r.off + k) + 1] = (OT)acc.y;
        }
      }
    }
    if (blk == 0) {  // uniform over the block
      if (threadIdx.x == 0) wn[b] = nv;
      givens_step_block(b, H, g, cs, sn, st, m, j, tol, n_running, nv, glds, idle);
    }
  }
}

// y = R^{-1} g (upper triangular, size jdone), stored in place of g.  One
// block per RHS, column-oriented: y_i = r_i / R_ii, then every lane k < i
// updates its own r_k -= R_ki y_i (fixed order per entry).
__global__ void __launch_bounds__(256)
backsolve_kernel(const double2* __restrict__ H, double2* __restrict__ g, const RhsState* __restrict__ st, int m) {
  __shared__ double2 yi_s;
  const int b = blockIdx.x;
  const RhsState s = st[b];
  if (!s.active) return;
  const int J = s.jdone;
  const double2* h = H + (size_t)b * (m + 1) * m;
  double2* y = g + (size_t)b * (m + 1);
  for (int i = J - 1; i >= 0; --i) {
    if (threadIdx.x == 0) {
      const double2 acc = y[i];
      const double2 d = h[i * m + i];
      const double dd = d.x * d.x + d.y * d.y;
      const double2 v = dd > 0.0 ? make_double2((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd)
                                 : make_double2(0.0, 0.0);
      y[i] = v;
      yi_s = v;
    }
    __syncthreads();
    const double2 v = yi_s;
    for (int k = threadIdx.x; k < i; k += blockDim.x) {
      const double2 t = cmul(h[k * m + i], v);
      y[k].x -= t.x;
      y[k].y -= t.y;
    }
    __syncthreads();
  }
}

// x += V y (first jdone columns)
template <typename VB>
__global__ void update_x_kernel(const VB* __restrict__ V, const double2* __restrict__ g,
                                double2* __restrict__ x, const RhsVec* __restrict__ rv,
                                const RhsState* __restrict__ st, int m, int64_t ut) {
  const int b = blockIdx.y;
  const RhsVec r = rv[b];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const RhsState s = st[b];
  if (k >= r.N || !s.active) return;
  double2 acc = x[r.off + k];
  const double2* y = g + (size_t)b * (m + 1);
  for (int i = 0; i < s.jdone; ++i) {
    double2 t = cmul(y[i], ld_b(V + (int64_t)i * ut + r.off + k));
    acc.x += t.x;
    acc.y += t.y;
  }
  x[r.off + k] = acc;
}

// out = a - b (user layout, per RHS)
__global__ void sub_kernel(const double2* __restrict__ a, const double2* __restrict__ bvec,
                           double2* __restrict__ out, const RhsVec* __restrict__ rv) {
  const int b = blockIdx.y;
  const RhsVec r = rv[b];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= r.N) return;
  double2 u = a[r.off + k], v = bvec[r.off + k];
  out[r.off + k] = make_double2(u.x - v.x, u.y - v.y);
}

// x += d; st (nullable): only right-hand sides being solved
__global__ void add_kernel(double2* __restrict__ x, const double2* __restrict__ d,
                           const RhsVec* __restrict__ rv, const RhsState* __restrict__ st) {
  const int b = blockIdx.y;
  if (st && !st[b].active) return;
  const RhsVec r = rv[b];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= r.N) return;
  double2 u = x[r.off + k], v = d[r.off + k];
  x[r.off + k] = make_double2(u.x + v.x, u.y + v.y);
}

__global__ void zero_kernel(double2* __restrict__ x, const RhsVec* __restrict__ rv) {
  const int b = blockIdx.y;
  const RhsVec r = rv[b];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= r.N) return;
  x[r.off + k] = make_double2(0.0, 0.0);
}

// start of a cycle: beta = ||r||, V_0 = r / beta, g = (beta, 0, ...), jdone = -1
template <typename VB>
__global__ void cycle_start_kernel(const double2* __restrict__ r, VB* __restrict__ V,
                                   const RhsVec* __restrict__ rv, RhsState* __restrict__ st,
                                   const double2* __restrict__ nrm2, double2* __restrict__ g, int m,
                                   int* __restrict__ live0, int* __restrict__ idle) {
  const int b = blockIdx.y;
  if (blockIdx.x == 0 && b == 0 && threadIdx.x == 0) *live0 = 1;  // step 0 runs
  if (blockIdx.x == 0 && threadIdx.x == 0) idle[b] = st[b].active ? 0 : 1;
  const RhsVec rr = rv[b];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double beta = sqrt(fmax(nrm2[b].x, 0.0));
  const bool act = st[b].active && beta > 0.0;
  const double inv = act ? 1.0 / beta : 0.0;
  if (k < rr.N)
    st_b(V + rr.off + k, act ? make_double2(r[rr.off + k].x * inv, r[rr.off + k].y * inv) : make_double2(0.0, 0.0));
  if (k <= m) g[(size_t)b * (m + 1) + k] = (k == 0 && act) ? make_double2(beta, 0.0) : make_double2(0.0, 0.0);
}

__global__ void states_check_kernel(const uint8_t* __restrict__ states, const RhsVec* __restrict__ rv,
                                    const int64_t* __restrict__ soff, int n_a, int n_states,
                                    int* __restrict__ flag) {
  const int b = blockIdx.y;
  const int64_t units = rv[b].N / n_a;
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= units) return;
  if (states[soff[b] + u] >= n_states) atomicOr(flag, 2);
}

__global__ void nonfinite_kernel(const double2* __restrict__ v, const RhsVec* __restrict__ rv,
                                 int* __restrict__ flag) {
  const int b = blockIdx.y;
  const RhsVec r = rv[b];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= r.N) return;
  double2 t = v[r.off + k];
  if (!(isfinite(t.x) && isfinite(t.y))) atomicOr(flag, 4);
}

// Block-Jacobi inverses Z(0)[A(s), A(s)]^-1 (column-major), one workgroup per state.
// Dynamic LDS: (2 n_a^2 + n_a + 1) double2.
template <typename S>
__global__ void __launch_bounds__(256)
selfblock_inverse_kernel(const S* __restrict__ nearb, int slot0, int n, int n_a, double2* __restrict__ Minv,
                         int* __restrict__ flag) {
  extern __shared__ double2 aug[];  // [n_a][2 n_a], then column k [n_a]
  __shared__ int piv_row;
  double2* colk = aug + 2 * n_a * n_a;
  const int st = blockIdx.x;
  const int w = 2 * n_a;
  const S* Z0 = nearb + (size_t)slot0 * n * n * 2;
  for (int e = threadIdx.x; e < n_a * w; e += blockDim.x) {
    const int i = e / w, j = e % w;
    double2 v;
    if (j < n_a) {
      const size_t idx = (size_t)(st * n_a + i) * n + st * n_a + j;
      v = make_double2((double)Z0[2 * idx], (double)Z0[2 * idx + 1]);
    } else {
      v = make_double2(j - n_a == i ? 1.0 : 0.0, 0.0);
    }
    aug[e] = v;
  }
  __syncthreads();
  if (!gj_invert_na(aug, colk, n_a, &piv_row, flag)) return;
  for (int e = threadIdx.x; e < n_a * n_a; e += blockDim.x) {
    const int i = e / n_a, j = e % n_a;
    Minv[(size_t)st * n_a * n_a + (size_t)j * n_a + i] = aug[i * w + n_a + j];  // column-major
  }
}

// Relaxed codebook: per unit u (of RHS b = blockIdx.y) the self block of the
// blended operator, M_u = sum_{s,s'} w[u][s] w[u][s'] Z(0)[A(s), A(s')]
// (transposed for the adjoint operator), inverted into Minv[global unit].
template <typename S>
__global__ void __launch_bounds__(256)
relaxed_selfblock_inverse_kernel(const S* __restrict__ nearb, int slot0, int n, int n_a, int n_states,
                                 const RhsVec* __restrict__ rv, const double* __restrict__ wts, int transpose,
                                 double2* __restrict__ Minv, int* __restrict__ flag) {
  extern __shared__ double2 aug[];
  __shared__ int piv_row;
  double2* colk = aug + 2 * n_a * n_a;
  const int b = blockIdx.y;
  const RhsVec r = rv[b];
  const int64_t u = blockIdx.x;
  if (u * n_a >= r.N) return;  // uniform over the workgroup
  const int64_t gu = r.off / n_a + u;  // global unit
  const double* wu = wts + gu * n_states;
  const int w = 2 * n_a;
  const S* Z0 = nearb + (size_t)slot0 * n * n * 2;
  for (int e = threadIdx.x; e < n_a * w; e += blockDim.x) {
    const int i = e / w, j = e % w;
    double2 v = make_double2(j - n_a == i ? 1.0 : 0.0, 0.0);
    if (j < n_a) {
      const int ri = transpose ? j : i, rj = transpose ? i : j;
      v = make_double2(0.0, 0.0);
      for (int s1 = 0; s1 < n_states; ++s1)
        for (int s2 = 0; s2 < n_states; ++s2) {
          const size_t idx = (size_t)(s1 * n_a + ri) * n + s2 * n_a + rj;
          const double ww = wu[s1] * wu[s2];
          v.x += ww * (double)Z0[2 * idx];
          v.y += ww * (double)Z0[2 * idx + 1];
        }
    }
    aug[e] = v;
  }
  __syncthreads();
  if (!gj_invert_na(aug, colk, n_a, &piv_row, flag)) return;
  for (int e = threadIdx.x; e < n_a * n_a; e += blockDim.x) {
    const int i = e / n_a, j = e % n_a;
    Minv[(size_t)gu * n_a * n_a + (size_t)j * n_a + i] = aug[i * w + n_a + j];  // column-major
  }
}

// out_u = Minv[s_u] in_u for every unit (user layout); OT is the output real
// type.  per_unit: Minv holds one block per global unit (relaxed codebooks)
template <typename OT, typename IT = double2>
__global__ void apply_precond_kernel(const double2* __restrict__ Minv, const uint8_t* __restrict__ states,
                                     const int64_t* __restrict__ soff, const RhsVec* __restrict__ rv, int n_a,
                                     int n_states, const IT* __restrict__ in, OT* __restrict__ out,
                                     const int* __restrict__ live, int per_unit, const RhsState* __restrict__ st) {
  if (live && *live == 0) return;
  const int b = blockIdx.y;
  if (st && !st[b].active) return;  // a right-hand side this cycle does not solve
  const RhsVec r = rv[b];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= r.N) return;
  const int64_t u = k / n_a;
  const int m = (int)(k % n_a);
  const int64_t s = per_unit ? r.off / n_a + u : min((int)states[soff[b] + u], n_states - 1);
  // column-major blocks: the lanes of a unit (consecutive rows m) read
  // consecutive entries for each column c
  const double2* M = Minv + (size_t)s * n_a * n_a + m;
  const IT* v = in + r.off + u * n_a;
  double2 acc = make_double2(0.0, 0.0);
  for (int c = 0; c < n_a; ++c) {
    const double2 t = cmul(M[(size_t)c * n_a], ld_b(v + c));
    acc.x += t.x;
    acc.y += t.y;
  }
  out[2 * (r.off + k)] = (OT)acc.x;
  out[2 * (r.off + k) + 1] = (OT)acc.y;
}

// apply_precond_kernel with the per-state inverses staged in LDS (as TM: float
// for a complex64 output, double otherwise) once per workgroup, over a grid
// strided across (RHS, item): an item holds RW nthr elements of whole units
// (blockDim.x = nthr, a multiple of n_a), each thread loads RW of them and
// then forms RW consecutive rows of its unit's product.  n_a % RW == 0.
// Dynamic LDS: (n_states n_a^2 + RW blockDim.x) complex TM.
template <typename TM, int RW, typename IT, typename OT>
__global__ void __launch_bounds__(256)
apply_precond_staged_kernel(const double2* __restrict__ Minv, const uint8_t* __restrict__ states,
                            const int64_t* __restrict__ soff, const RhsVec* __restrict__ rv, int n_a, int n_states,
                            const IT* __restrict__ in, OT* __restrict__ out, const RhsState* __restrict__ st, int B,
                            int64_t nb_max) {
  struct alignas(2 * sizeof(TM)) CT {
    TM x, y;
  };
  extern __shared__ double2 lds_raw[];
  CT* Ms = reinterpret_cast<CT*>(lds_raw);  // [state][column][row]
  CT* vs = Ms + (size_t)n_states * n_a * n_a;
  for (int t = threadIdx.x; t < n_states * n_a * n_a; t += blockDim.x) Ms[t] = CT{(TM)Minv[t].x, (TM)Minv[t].y};
  const int64_t items = nb_max * B;
  const int hp = n_a / RW, ul = threadIdx.x / hp, p = RW * (threadIdx.x - ul * hp);
  for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {  // uniform over the block
    const int b = (int)(item / nb_max);
    const int64_t blk = item - (int64_t)b * nb_max;
    if (st && !st[b].active) continue;  // a right-hand side this cycle does not solve
    const RhsVec r = rv[b];
    const int64_t base = blk * RW * blockDim.x;
    if (base >= r.N) continue;
    __syncthreads();  // the staged inverses, or the previous item's reads of vs
#pragma unroll
    for (int e = 0; e < RW; ++e) {
      const int64_t ke = base + e * blockDim.x + threadIdx.x;
      const double2 v = ke < r.N ? ld_b(in + r.off + ke) : make_double2(0.0, 0.0);
      vs[e * blockDim.x + threadIdx.x] = CT{(TM)v.x, (TM)v.y};
    }
    __syncthreads();
    const int64_t k0 = base + (int64_t)ul * n_a + p;  // rows p .. p + RW - 1 of local unit ul
    if (k0 < r.N) {
      const int64_t u = k0 / n_a;
      const int sidx = min((int)states[soff[b] + u], n_states - 1);
      const CT* M = Ms + (size_t)sidx * n_a * n_a + p;
      const CT* vu = vs + ul * n_a;
      TM ax[RW], ay[RW];
#pragma unroll
      for (int q = 0; q < RW; ++q) ax[q] = ay[q] = (TM)0;
      for (int c = 0; c < n_a; ++c) {
        const CT x = vu[c];
#pragma unroll
        for (int q = 0; q < RW; ++q) {
          const CT mm = M[(size_t)c * n_a + q];
          ax[q] += mm.x * x.x - mm.y * x.y;
          ay[q] += mm.x * x.y + mm.y * x.x;
        }
      }
#pragma unroll
      for (int q = 0; q < RW; ++q) {
        out[2 * (r.off + k0 + q)] = (OT)ax[q];
        out[2 * (r.off + k0 + q) + 1] = (OT)ay[q];
      }
    }
  }
}

template <typename OT, typename IT = double2>
__global__ void convert_vec_kernel(const RhsVec* __restrict__ rv, const IT* __restrict__ in,
                                   OT* __restrict__ out, const int* __restrict__ live) {
  if (live && *live == 0) return;
  const int b = blockIdx.y;
  const RhsVec r = rv[b];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= r.N) return;
  const double2 v = ld_b(in + r.off + k);
  out[2 * (r.off + k)] = (OT)v.x;
  out[2 * (r.off + k) + 1] = (OT)v.y;
}

// z = V y (first jdone columns)
template <typename VB>
__global__ void combine_basis_kernel(const VB* __restrict__ V, const double2* __restrict__ g,
                                     double2* __restrict__ z, const RhsVec* __restrict__ rv,
                                     const RhsState* __restrict__ st, int m, int64_t ut) {
  const int b = blockIdx.y;
  const RhsVec r = rv[b];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const RhsState s = st[b];
  if (k >= r.N) return;
  double2 acc = make_double2(0.0, 0.0);
  if (s.active) {
    const double2* y = g + (size_t)b * (m + 1);
    for (int i = 0; i < s.jdone; ++i) {
      double2 t = cmul(y[i], ld_b(V + (int64_t)i * ut + r.off + k));
      acc.x += t.x;
      acc.y += t.y;
    }
  }
  z[r.off + k] = acc;
}

// Residual of a finished cycle in its basis: with Givens rotations G_j = [c_j
// s_j; -conj(s_j) c_j] and gamma = g[J] the last rotated entry (J = jdone),
// b - A M^{-1} V y = V_{J+1} u, u = G_0^H ... G_{J-1}^H (gamma e_J):
// u_J = c_{J-1} gamma, u_j = c_{j-1} t_j with t_j = (-s_j) t_{j+1}, t_J =
// gamma, and u_0 = t_0.  One thread per right-hand side, u[b][0..J].
__global__ void residual_coeffs_kernel(const double2* __restrict__ g, const double* __restrict__ cs,
                                       const double2* __restrict__ sn, const RhsState* __restrict__ st, int B,
                                       int m, double2* __restrict__ u) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B || !st[b].active) return;
  const int J = st[b].jdone;
  double2* ub = u + (size_t)b * (m + 1);
  double2 t = g[(size_t)b * (m + 1) + J];
  for (int j = J - 1; j >= 0; --j) {
    const double c = cs[(size_t)b * m + j];
    const double2 sj = sn[(size_t)b * m + j];
    ub[j + 1] = make_double2(c * t.x, c * t.y);
    t = make_double2(-(sj.x * t.x - sj.y * t.y), -(sj.x * t.y + sj.y * t.x));
  }
  ub[0] = t;
}

// combine_basis_kernel and, in the same pass over the basis, the cycle's
// residual r = V_{J+1} u (u from residual_coeffs_kernel) for the restart;
// right-hand sides the cycle did not solve keep their r
template <typename VB>
__global__ void combine_basis_res_kernel(const VB* __restrict__ V, const double2* __restrict__ g,
                                         const double2* __restrict__ u, double2* __restrict__ z,
                                         double2* __restrict__ res, const RhsVec* __restrict__ rv,
                                         const RhsState* __restrict__ st, int m, int64_t ut) {
  const int b = blockIdx.y;
  const RhsVec r = rv[b];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const RhsState s = st[b];
  if (k >= r.N) return;
  double2 acc = make_double2(0.0, 0.0);
  if (s.active) {
    const double2* y = g + (size_t)b * (m + 1);
    const double2* ub = u + (size_t)b * (m + 1);
    double2 ra = make_double2(0.0, 0.0);
    for (int i = 0; i <= s.jdone; ++i) {
      const double2 v = ld_b(V + (int64_t)i * ut + r.off + k);
      if (i < s.jdone) {
        const double2 t = cmul(y[i], v);
        acc.x += t.x;
        acc.y += t.y;
      }
      const double2 q = cmul(ub[i], v);
      ra.x += q.x;
      ra.y += q.y;
    }
    res[r.off + k] = ra;
  }
  z[r.off + k] = acc;
}

// idle[b] = 1 for a right-hand side that the last cycle did not solve: the
// restart's residual skips it
__global__ void idle_from_state_kernel(const RhsState* __restrict__ st, int B, int* __restrict__ idle) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) idle[b] = st[b].active ? 0 : 1;
}

__global__ void finalize_kernel(RhsState* __restrict__ st, int B, int J) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  if (st[b].active && st[b].jdone < 0) st[b].jdone = J;
}

struct Work {
  double2* V;
  double2* w;
  double2* r;
  double2* d;
  double2* ro;
  double2* pz;
  double2* xs;   // matvec input in the store precision
  double2* Minv;
  void* ilu;  // near-field block ILU factors
  double* wn;
  double* npart;
  void* mv_partial;
  void* lists;    // near retrieval lists of the solve's store
  void* lists64;  // and of the refinement store
  double2* H;
  double2* g;
  double* cs;
  double2* sn;
  double2* dpart;
  double2* dpart2;  // second-pass inner products of the folded update, per update block
  double2* hbuf;
  double2* hsum;  // Gram-Schmidt coefficients summed from dpart (long vectors)
  double* nsum;   // ||w||^2 summed from npart (long vectors)
  double2* nrm;
  RhsState* st;
  int* idle;  // per RHS: 1 while it has no work in the current cycle (the matvec and Krylov kernels skip it)
  int* rl;    // the RHS with work in the current Arnoldi step (list, then count; see rhs_count)
  RhsVec* rv;
  int64_t* soff;
  int* counters;
  size_t bytes;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// 64-element runs per update block: four for long vectors (more than 64
// chunks of kDotChunk: a quarter of the workgroups, which matters once most
// right-hand sides of a wide batch are idle and their workgroups only
// return), else one (the single-RHS solve keeps enough workgroups, and
// normalize_step_kernel sums their per-64 parts itself)
int update_runs(int64_t maxN) { return (maxN + kDotChunk - 1) / kDotChunk > 64 ? 4 : 1; }
// basis vectors a folded update takes: the element-parallel kernel (long
// vectors) holds more
int fold_max_vec(int64_t maxN, bool vb32) {
  return update_runs(maxN) == 4 && vb32 ? kFoldMaxVecEl : kFoldMaxVec;
}
int64_t fold_blocks(int64_t maxN) {
  const int nsub = update_runs(maxN);
  return std::max<int64_t>(1, (maxN + 64 * nsub - 1) / (64 * nsub));
}

// n_blocks: block-Jacobi inverses held (one per state, or one per unit for
// relaxed codebooks)
Work layout_work(char* base, const BatchDesc& bd, int n_a, int n_blocks, int m, size_t mv_bytes,
                 size_t lists_bytes, size_t lists64_bytes, size_t ilu_bytes, bool vb32) {
  Work w{};
  const int B = bd.B;
  int64_t maxN = 0;
  for (int b = 0; b < B; ++b) maxN = std::max<int64_t>(maxN, bd.n_units[b] * n_a);
  const size_t ut = (size_t)bd.total_units * n_a;
  const int64_t vtot = (int64_t)(m + 1) * ut;
  const int maxP = (int)((maxN + kDotChunk - 1) / kDotChunk);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return base ? (void*)(base + at) : nullptr;
  };
  w.V = (double2*)take((size_t)vtot * (vb32 ? 8 : 16));  // complex64 entries when vb32
  w.w = (double2*)take(ut * 16);
  w.r = (double2*)take(ut * 16);
  w.d = (double2*)take(ut * 16);
  w.ro = (double2*)take(ut * 16);
  w.pz = (double2*)take(ut * 16);
  w.xs = (double2*)take(ut * 16);
  w.wn = (double*)take((size_t)B * 8);
  w.npart = (double*)take((size_t)B * ((maxN + 63) / 64 + 1) * 8);
  w.Minv = (double2*)take((size_t)n_blocks * n_a * n_a * 16);
  w.ilu = take(ilu_bytes);
  w.mv_partial = take(mv_bytes);
  w.lists = take(lists_bytes);
  w.lists64 = take(lists64_bytes);
  w.H = (double2*)take((size_t)B * (m + 1) * m * 16);
  w.g = (double2*)take((size_t)B * (m + 1) * 16);
  w.cs = (double*)take((size_t)B * m * 8);
  w.sn = (double2*)take((size_t)B * m * 16);
  w.dpart = (double2*)take((size_t)B * (m + 1) * std::max(maxP, 1) * 16);
  w.dpart2 = (double2*)take((size_t)B * std::min(m + 1, fold_max_vec(maxN, vb32)) * fold_blocks(maxN) * 16);
  w.hbuf = (double2*)take((size_t)B * (m + 1) * 16);
  w.hsum = (double2*)take((size_t)B * (m + 1) * 16);
  w.nsum = (double*)take((size_t)B * 8);
  w.nrm = (double2*)take((size_t)B * 16);
  w.st = (RhsState*)take((size_t)B * sizeof(RhsState));
  w.idle = (int*)take((size_t)B * sizeof(int));
  w.rl = (int*)take((size_t)(B + 1) * sizeof(int));
  w.rv = (RhsVec*)take((size_t)B * sizeof(RhsVec));
  w.soff = (int64_t*)take((size_t)B * 8);
  w.counters = (int*)take(256);
  w.bytes = o;
  return w;
}

}  // namespace


struct GmresRun {
  r3m_ctx ctx;
  bool use_graph = true;
  std::vector<int64_t> graph_key;
  const BatchDesc* bd;
  const r3m_batch* batch;
  int n_a, m, maxP, B;
  int n_states = 1;
  bool pre = false;
  const double* wts = nullptr;  // relaxed retrieval weights (spectral stores)
  bool tr = false;              // with wts: the transposed operator
  int pu = 0;                   // block-Jacobi inverses per global unit (relaxed) instead of per state
  int ilu_r = 0;                // > 0: the near-field block ILU(0) of this radius preconditions
  bool vb32 = false;            // the Krylov basis W.V holds complex64 (see basis32)
  int G = 1;  // displacement groups of the matvec (autotuned)
  int64_t maxN, ut;
  Work W;
  hipStream_t s;

  dim3 vgrid() const { return dim3(ceil_div((size_t)maxN, 256), B); }

  // out = M^-1 in per unit with the per-state inverses staged in LDS (OT
  // float: complex64 products, four rows per thread; double: complex128, two);
  // false where that form does not apply (the caller launches
  // apply_precond_kernel)
  template <typename OT, typename IT>
  bool precond_staged(const IT* in, OT* out) {
    constexpr int RW = sizeof(OT) == 4 ? 4 : 2;
    const int nthr = (256 / n_a) * n_a;
    const size_t es = 2 * sizeof(OT);
    const size_t lds = ((size_t)n_states * n_a * n_a + (size_t)RW * nthr) * es;
    if (pu || ilu_r || n_a % RW != 0 || nthr == 0 || lds > 64 * 1024) return false;
    const int64_t nb = ceil_div((size_t)maxN, (size_t)RW * nthr);
    hipLaunchKernelGGL((apply_precond_staged_kernel<OT, RW, IT, OT>), dim3(stride_grid(nb * B)), dim3(nthr), lds, s,
                       W.Minv, batch->states, W.soff, W.rv, n_a, n_states, in, out, (const RhsState*)W.st, B, nb);
    return true;
  }

  void dots(const double2* A, int64_t a_stride, const double2* Bv, int nvec) {
    dim3 grid(maxP, nvec, B);
    hipLaunchKernelGGL(dots_kernel, grid, dim3(kDotThreads), 0, s, A, a_stride, Bv, W.rv, nvec,
                       (const int*)nullptr, maxP, W.dpart);
    hipLaunchKernelGGL(dots_finish_kernel, dim3(B), dim3(((nvec + 63) / 64) * 64), 0, s, W.dpart, W.rv,
                       nvec, maxP, W.hbuf);
  }

  // W.nrm[b].x = ||v_b||^2
  void norms(const double2* v) {
    dots(v, 0, v, 1);
    R3M_CHECK_HIP(hipMemcpyAsync(W.nrm, W.hbuf, (size_t)B * 16, hipMemcpyDeviceToDevice, s));
  }

  std::vector<double> host_norms(const double2* v) {
    norms(v);
    std::vector<double2> h(B);
    R3M_CHECK_HIP(hipMemcpyAsync(h.data(), W.nrm, (size_t)B * 16, hipMemcpyDeviceToHost, s));
    R3M_CHECK_HIP(hipStreamSynchronize(s));
    std::vector<double> out(B);
    for (int b = 0; b < B; ++b) out[b] = std::sqrt(std::max(h[b].x, 0.0));
    return out;
  }

  const r3m_store* Zsolve = nullptr;
  const void* lists_for(const r3m_store* Z) const { return Z == Zsolve ? W.lists : W.lists64; }

  // idle (device, nullable): right-hand sides whose output is not needed
  void matvec(const r3m_store* Z, const double2* x, double2* y, const int* idle = nullptr) {
    if (wts) {
      launch_spectral_ex(Z, *bd, batch->states, R3M_C128, x, R3M_C128, y, W.mv_partial, s, nullptr, wts, tr, idle);
      return;
    }
    launch_matvec(ctx, Z, *bd, batch->states, R3M_C128, x, y, W.mv_partial, lists_for(Z), plan_groups(ctx, Z, *bd),
                  s, idle);
  }

  // out = rhs - Z sol (for a right-hand side with idle[b] set, out[b] is meaningless)
  void residual(const r3m_store* Z, const double2* rhs, const double2* sol, double2* out,
                const int* idle = nullptr) {
    matvec(Z, sol, W.w, idle);
    hipLaunchKernelGGL(sub_kernel, vgrid(), dim3(256), 0, s, rhs, W.w, out, W.rv);
  }

  void precond(const double2* in, double2* out) {
    if (ilu_r) {
      launch_ilu_apply(Zsolve, *bd, ilu_r, W.ilu, in, out, R3M_C128, nullptr, s, nullptr, wts == nullptr);
      return;
    }
    if (precond_staged(in, (double*)out)) return;
    hipLaunchKernelGGL(apply_precond_kernel<double>, vgrid(), dim3(256), 0, s, W.Minv, batch->states, W.soff, W.rv,
                       n_a, n_states, in, (double*)out, (const int*)nullptr, pu, (const RhsState*)W.st);
  }

  // Running-RHS counts of Arnoldi step j live in two slots used in turn: step
  // j's Givens steps count into run_slot(j); every kernel of step j + 1 returns
  // at once if run_slot(j) is zero (all right-hand sides converged), so steps
  // launched past convergence cost only their launches.
  int* run_slot(int j) const { return W.counters + 4 + (j & 1); }

  // The matvec input of an Arnoldi step, M^{-1} V_j (block-Jacobi) or V_j,
  // in the store precision: written into W.xs by the previous step's
  // normalisation, or by prepare_input for V_0.  A complex128 store without
  // preconditioner reads V_j itself.
  bool input_in_xs(const r3m_store* Z) const { return pre || Z->near_dtype == R3M_C64; }
  template <typename VB>
  void prepare_input(const r3m_store* Z, const VB* v) {
    const bool c64 = Z->near_dtype == R3M_C64;
    if (ilu_r) {  // W.w is free here: the forward solve's scratch
      if constexpr (std::is_same<VB, double2>::value)
        launch_ilu_apply(Z, *bd, ilu_r, W.ilu, v, W.w, c64 ? R3M_C64 : R3M_C128, W.xs, s, nullptr, wts == nullptr);
      else
        R3M_REQUIRE(false, R3M_ERR_UNSUPPORTED, "a complex64 basis with the ILU preconditioner");
    } else if (pre) {
      if (c64) {
        if (!precond_staged(v, (float*)W.xs))
          hipLaunchKernelGGL((apply_precond_kernel<float, VB>), vgrid(), dim3(256), 0, s, W.Minv, batch->states,
                             W.soff, W.rv, n_a, n_states, v, (float*)W.xs, (const int*)nullptr, pu,
                             (const RhsState*)W.st);
      } else if (!precond_staged(v, (double*)W.xs)) {
        hipLaunchKernelGGL((apply_precond_kernel<double, VB>), vgrid(), dim3(256), 0, s, W.Minv, batch->states,
                           W.soff, W.rv, n_a, n_states, v, (double*)W.xs, (const int*)nullptr, pu,
                           (const RhsState*)W.st);
      }
    } else if (c64) {
      hipLaunchKernelGGL((convert_vec_kernel<float, VB>), vgrid(), dim3(256), 0, s, W.rv, v, (float*)W.xs,
                         (const int*)nullptr);
    }
  }

  // The Arnoldi vector w (the matvec output, orthogonalised in place) is
  // kept in complex64 with a complex64 basis on spectral stores (the
  // product it holds is an FP32 one; FP64 arithmetic throughout), in the
  // first half of W.w
  void arnoldi_step(const r3m_store* Z, int j, double tol) {
    if (vb32 && store_is_spectral(Z))
      arnoldi_step_t<float2, float2>(Z, j, tol);
    else if (vb32)
      arnoldi_step_t<float2, double2>(Z, j, tol);
    else
      arnoldi_step_t<double2, double2>(Z, j, tol);
  }

  template <typename VB, typename WB>
  void arnoldi_step_t(const r3m_store* Z, int j, double tol) {
    VB* V = reinterpret_cast<VB*>(W.V);
    WB* wv = reinterpret_cast<WB*>(W.w);
    constexpr bool wd = std::is_same<WB, double2>::value;
    const int* live = run_slot(j - 1);  // j = 0: set by the cycle start
    const VB* vj = V + (int64_t)j * ut;
    // the right-hand sides with work in this step (not idle at its start);
    // narrow batches skip the list (their grids are small either way)
    const int* rl = nullptr;
    if (B >= kListMinRhs) {
      hipLaunchKernelGGL(live_rhs_kernel, dim3(1), dim3(1024), 0, s, (const int*)W.idle, B, W.rl);
      rl = W.rl;
    }
    if (wts) {
      R3M_REQUIRE(wd, R3M_ERR_UNSUPPORTED, "relaxed solves keep w in complex128");
      launch_spectral_ex(Z, *bd, batch->states, input_in_xs(Z) ? Z->near_dtype : R3M_C128,
                         input_in_xs(Z) ? (const void*)W.xs : (const void*)vj, R3M_C128, W.w, W.mv_partial, s, live,
                         wts, tr, W.idle);
    } else {
      launch_matvec_pre(Z, *bd, batch->states, input_in_xs(Z) ? (const void*)W.xs : (const void*)vj, wv,
                        W.mv_partial, lists_for(Z), G, s, live, W.idle, rl, wd ? R3M_C128 : R3M_C64);
    }
    const int maxB = (int)((maxN + 63) / 64 + 1);
    // long vectors (more than 64 chunk partials per coefficient): sum the
    // partials once in their own launch rather than in every update block
    const bool long_vec = maxP > 64;
    const int nsub = update_runs(maxN);
    const int nvec = j + 1;
    // inner-product items of dv vectors: the basis count padded to a power of
    // two up to dot_vec (the exchanges of the lane sums scale with dv)
    const int dv = std::min(dot_vec<VB>(), nvec <= 1 ? 1 : nvec <= 2 ? 2 : nvec <= 4 ? 4 : 8);
    const int ngrp = (nvec + dv - 1) / dv;
    const int64_t nb_u = (maxN + 64 * nsub - 1) / (64 * nsub);
    const unsigned dgrid = stride_grid((int64_t)maxP * ngrp * B), ugrid = stride_grid(nb_u * B);
    const size_t ulds = (size_t)nvec * sizeof(double2);
    auto dots = [&](int* reset) {
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(dgrid), dim3(kDotThreads), 0, s, V, ut, wv, W.rv, nvec, maxP, W.dpart, reset,
                           live, W.idle, rl, B);
      };
      if (dv == 1)
        go(dots_partials_kernel<VB, WB, 1>);
      else if (dv == 2)
        go(dots_partials_kernel<VB, WB, 2>);
      else if (dv == 4)
        go(dots_partials_kernel<VB, WB, 4>);
      else
        go(dots_partials_kernel<VB, WB, dot_vec<VB>()>);
    };
    // CGS2, first pass: inner products with the basis, then the update
    dots(run_slot(j));
    if (long_vec)
      hipLaunchKernelGGL(finish_partials_kernel, dim3(nvec, B), dim3(256), 0, s, (const double2*)W.dpart, maxP, nvec,
                         W.rv, W.hsum, live, W.idle, kDotChunk);
    const double2* h0 = long_vec ? (const double2*)W.hsum : (const double2*)W.dpart;
    const int h0P = long_vec ? 1 : maxP, h0n = long_vec ? 1 : 0;
    // one Gram-Schmidt update (kv > 0: folding the second pass's inner
    // products): the element-parallel kernel for long vectors
    auto update = [&](int kv, const double2* hp, int hP, int hn, int do_norm, int mode, int pchunk, double2* p2,
                      int mP2, const double* skip) {
      R3M_REQUIRE(!skip || (nsub == 4 && kv == 0), R3M_ERR_UNSUPPORTED, "selective second pass on the element kernel");
      auto el = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(ugrid), dim3(256), ulds, s, V, wv, W.rv, W.st, hp, hP, hn, nvec, ut, do_norm,
                           W.npart, maxB, W.H, m, j, mode, live, W.idle, pchunk, p2, mP2, rl, B, nb_u, skip);
      };
      if (nsub == 4 && kv > 0) {
        // the basis count padded to a power of two
        if (nvec <= 2)
          el(gs_update_el_kernel<2, VB, WB>);
        else if (nvec <= 4)
          el(gs_update_el_kernel<4, VB, WB>);
        else if (nvec <= 8)
          el(gs_update_el_kernel<8, VB, WB>);
        else if (nvec <= 16 || sizeof(VB) != sizeof(float2))
          el(gs_update_el_kernel<16, VB, WB>);
        else if (nvec <= 20)
          el(gs_update_el_kernel<20, VB, WB>);
        else if (nvec <= 24)
          el(gs_update_el_kernel<24, VB, WB>);
        else
          el(gs_update_el_kernel<32, VB, WB>);
      } else if (nsub == 4)
        el(gs_update_el_kernel<0, VB, WB>);
      else if (kv == 2)
        hipLaunchKernelGGL((gs_update_kernel<2, VB, WB>), dim3(ugrid), dim3(256), ulds, s, V, wv, W.rv, W.st, hp, hP,
                           hn, nvec, ut, do_norm, W.npart, maxB, W.H, m, j, mode, live, W.idle, nsub, pchunk, p2, mP2,
                           rl, B, nb_u);
      else if (kv == 4)
        hipLaunchKernelGGL((gs_update_kernel<4, VB, WB>), dim3(ugrid), dim3(256), ulds, s, V, wv, W.rv, W.st, hp, hP,
                           hn, nvec, ut, do_norm, W.npart, maxB, W.H, m, j, mode, live, W.idle, nsub, pchunk, p2, mP2,
                           rl, B, nb_u);
      else
        hipLaunchKernelGGL((gs_update_kernel<0, VB, WB>), dim3(ugrid), dim3(256), ulds, s, V, wv, W.rv, W.st, hp, hP,
                           hn, nvec, ut, do_norm, W.npart, maxB, W.H, m, j, mode, live, W.idle, nsub, pchunk, p2, mP2,
                           rl, B, nb_u);
    };
    if (nvec <= fold_max_vec(maxN, sizeof(VB) == sizeof(float2)) && W.dpart2) {
      // the first update also forms the second pass's inner products; on
      // long vectors it also takes ||w||^2, and the second pass runs only
      // where the first lost more than half of the squared norm (the first
      // pass's norm parts then stand for the RHS that skip it)
      const int maxP2 = (int)fold_blocks(maxN);
      const bool sel = long_vec && nsub == 4 && selective_cgs2();
      update(nvec <= 8 ? 2 : 4, h0, h0P, h0n, sel ? 1 : 0, 0, kDotChunk, W.dpart2, maxP2, nullptr);
      if (sel)
        hipLaunchKernelGGL(finish_norm_kernel, dim3(B), dim3(256), 0, s, (const double*)W.npart, maxB, W.rv, W.nsum,
                           live, W.idle, nsub);
      if (long_vec)
        hipLaunchKernelGGL(finish_partials_kernel, dim3(nvec, B), dim3(256), 0, s, (const double2*)W.dpart2, maxP2,
                           nvec, W.rv, W.hsum, live, W.idle, 64 * nsub);
      update(0, long_vec ? (const double2*)W.hsum : (const double2*)W.dpart2, long_vec ? 1 : maxP2, long_vec ? 1 : 0,
             1, 1, 64 * nsub, (double2*)nullptr, 0, sel ? (const double*)W.nsum : nullptr);
    } else {
      update(0, h0, h0P, h0n, 0, 0, kDotChunk, (double2*)nullptr, 0, nullptr);
      // CGS2, second pass
      dots((int*)nullptr);
      if (long_vec)
        hipLaunchKernelGGL(finish_partials_kernel, dim3(nvec, B), dim3(256), 0, s, (const double2*)W.dpart, maxP,
                           nvec, W.rv, W.hsum, live, W.idle, kDotChunk);
      update(0, h0, h0P, h0n, 1, 1, kDotChunk, (double2*)nullptr, 0, nullptr);
    }
    if (long_vec)
      hipLaunchKernelGGL(finish_norm_kernel, dim3(B), dim3(256), 0, s, (const double*)W.npart, maxB, W.rv, W.nsum,
                         live, W.idle, nsub);
    const double* np = long_vec ? W.nsum : W.npart;
    const int npB = long_vec ? 1 : maxB, npN = long_vec ? 1 : 0;
    // blocks of whole units (the preconditioner multiplies per unit)
    const int nthr = pre ? (256 / n_a) * n_a : 256;
    const int64_t nb_n = ceil_div((size_t)maxN, nthr);
    const dim3 ngrid(stride_grid(nb_n * B));
    const size_t glds0 = (size_t)(2 * m + 2) * 16 + (size_t)((m + 1) / 2) * 16;
    // complex64 inner solves stage the (per-state) inverses in LDS
    const int stage = pre && !pu && Z->near_dtype == R3M_C64 && glds0 + (size_t)n_states * n_a * n_a * 8 <= 60 * 1024;
    const size_t glds = glds0 + (stage ? (size_t)n_states * n_a * n_a * 8 : 0);
    const bool c64 = Z->near_dtype == R3M_C64;
#define R3M_NORMALIZE(OT, MODE, XS)                                                                                  \
  hipLaunchKernelGGL((normalize_step_kernel<OT, MODE, VB, WB>), ngrid, dim3(nthr), glds, s, wv, V, W.rv, W.st, np, npB, \
                     npN, W.H, W.g, W.cs, W.sn, m, j, tol, run_slot(j), W.wn, ut, live, W.Minv, batch->states, W.soff, \
                     n_a, n_states, XS, pu, W.idle, rl, B, nb_n, stage)
    if (ilu_r) {
      // V_{j+1}, then the next step's input M^-1 V_{j+1} by the colour solves
      // (W.w, the matvec output, is free once normalised)
      R3M_NORMALIZE(double, 0, (double*)nullptr);
      if constexpr (std::is_same<VB, double2>::value && std::is_same<WB, double2>::value)
        launch_ilu_apply(Z, *bd, ilu_r, W.ilu, V + (int64_t)(j + 1) * ut, W.w, c64 ? R3M_C64 : R3M_C128, W.xs, s,
                         run_slot(j), wts == nullptr);
    } else if (pre && c64 && stage && n_a % 2 == 0) {
      // RW rows per thread: blocks of RW times the units
      auto rows = [&](auto kern, int rw) {
        const int64_t nbr = ceil_div((size_t)maxN, (size_t)rw * nthr);
        hipLaunchKernelGGL(kern, dim3(stride_grid(nbr * B)), dim3(nthr), glds, s, wv, V, W.rv, W.st, np, npB, npN,
                           W.H, W.g, W.cs, W.sn, m, j, tol, run_slot(j), W.wn, ut, live, W.Minv, batch->states,
                           W.soff, n_a, n_states, (float*)W.xs, pu, W.idle, rl, B, nbr, stage);
      };
      if (n_a % 4 == 0)
        rows(normalize_step_kernel<float, 2, VB, WB, 4>, 4);
      else
        rows(normalize_step_kernel<float, 2, VB, WB, 2>, 2);
    } else if (pre && c64) {
      R3M_NORMALIZE(float, 2, (float*)W.xs);
    } else if (pre) {
      R3M_NORMALIZE(double, 2, (double*)W.xs);
    } else if (c64) {
      R3M_NORMALIZE(float, 1, (float*)W.xs);
    } else {
      R3M_NORMALIZE(double, 0, (double*)nullptr);
    }
#undef R3M_NORMALIZE
    R3M_CHECK_HIP(hipGetLastError());
  }

  // Arnoldi steps [j0, j1): replayed from a cached HIP graph (captured on the
  // context stream the first time this block is met), or launched eagerly
  void run_steps(const r3m_store* Z, int j0, int j1, double tol) {
    if (!use_graph) {
      for (int j = j0; j < j1; ++j) arnoldi_step(Z, j, tol);
      return;
    }
    std::vector<int64_t> key = graph_key;
    key.push_back((int64_t)(intptr_t)Z->near);
    key.push_back((int64_t)(intptr_t)Z->far);
    key.push_back(Z->near_dtype);
    key.push_back(Z->far_dtype);
    key.push_back(Z->n);
    key.push_back(Z->n_states);
    key.push_back(Z->Dx);
    key.push_back(Z->Dy);
    key.push_back(Z->near_radius);
    key.push_back(Z->max_rank);
    key.push_back(G);
    key.push_back(j0);
    key.push_back(j1);
    int64_t tb;
    std::memcpy(&tb, &tol, sizeof(tb));
    key.push_back(tb);
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
      if (ctx->graphs.size() > 512) {
        R3M_CHECK_HIP(hipStreamSynchronize(s));
        for (auto& kv : ctx->graphs) R3M_CHECK_HIP(hipGraphExecDestroy(kv.second));
        ctx->graphs.clear();
      }
      hipGraph_t g;
      R3M_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      for (int j = j0; j < j1; ++j) arnoldi_step(Z, j, tol);
      R3M_CHECK_HIP(hipStreamEndCapture(s, &g));
      hipGraphExec_t ex;
      R3M_CHECK_HIP(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
      R3M_CHECK_HIP(hipGraphDestroy(g));
      it = ctx->graphs.emplace(key, ex).first;
    }
    R3M_CHECK_HIP(hipGraphLaunch(it->second, s));
  }

  // GMRES(m) on Z for rhs into sol, for RHS with running[b]; sol is zero on
  // entry when x_zero (the first residual is then rhs itself).  The tolerance
  // is relative to rhs_norm[b]; iters[b] accumulates iterations.  Returns the
  // residual norms ||rhs - Z sol|| at exit.
  std::vector<double> solve(const r3m_store* Z, const double2* rhs, double2* sol, std::vector<int> running,
                            const std::vector<double>& rhs_norm, double tol, int max_iter, std::vector<int>& iters,
                            bool x_zero) {
    std::vector<RhsState> hst(B);
    std::vector<double> rnorm(B, 0.0);
    bool first = true;
    bool r_from_basis = false;  // W.r holds the last cycle's residual from its basis
    while (true) {
      if (first && x_zero) {
        R3M_CHECK_HIP(hipMemcpyAsync(W.r, rhs, (size_t)ut * 16, hipMemcpyDeviceToDevice, s));
        norms(W.r);
        rnorm = rhs_norm;
      } else {
        // a restart: right-hand sides the last cycle did not solve keep their
        // residual norm and are skipped by the matvec (or r is already the
        // last cycle's residual from its basis)
        if (!first && !r_from_basis)
          hipLaunchKernelGGL(idle_from_state_kernel, dim3(ceil_div(B, 64)), dim3(64), 0, s, (const RhsState*)W.st, B,
                             W.idle);
        if (first || !r_from_basis) residual(Z, rhs, sol, W.r, first ? nullptr : (const int*)W.idle);
        r_from_basis = false;
        norms(W.r);
        std::vector<double2> nr(B);
        R3M_CHECK_HIP(hipMemcpyAsync(nr.data(), W.nrm, (size_t)B * 16, hipMemcpyDeviceToHost, s));
        R3M_CHECK_HIP(hipStreamSynchronize(s));
        for (int b = 0; b < B; ++b)
          if (first || running[b]) rnorm[b] = std::sqrt(std::max(nr[b].x, 0.0));
      }
      first = false;
      bool any = false;
      int min_used = max_iter;
      for (int b = 0; b < B; ++b) {
        const double rel = rhs_norm[b] > 0 ? rnorm[b] / rhs_norm[b] : 0.0;
        if (running[b] && (!(rel > tol) || iters[b] >= max_iter)) running[b] = 0;
        hst[b] = RhsState{rhs_norm[b], 0.0, rel, -1, running[b], std::max(1, max_iter - iters[b]), 0};
        if (running[b]) {
          any = true;
          min_used = std::min(min_used, iters[b]);
        }
      }
      if (!any) break;
      R3M_CHECK_HIP(hipMemcpyAsync(W.st, hst.data(), (size_t)B * sizeof(RhsState), hipMemcpyHostToDevice, s));
      dim3 g0(std::max(ceil_div((size_t)maxN, 256), ceil_div((size_t)m + 1, 256)), B);
      if (vb32) {
        hipLaunchKernelGGL(cycle_start_kernel<float2>, g0, dim3(256), 0, s, W.r, (float2*)W.V, W.rv, W.st, W.nrm, W.g,
                           m, run_slot(-1), W.idle);
        prepare_input(Z, (const float2*)W.V);
      } else {
        hipLaunchKernelGGL(cycle_start_kernel<double2>, g0, dim3(256), 0, s, W.r, W.V, W.rv, W.st, W.nrm, W.g, m,
                           run_slot(-1), W.idle);
        prepare_input(Z, (const double2*)W.V);
      }
      const int steps = std::max(1, std::min(m, max_iter - min_used));
      // Blocks of kCheckEvery steps.  The running count after a block is read
      // back asynchronously while the next block is already queued: the host
      // stops launching once a read-back shows zero, and the steps launched
      // past that point return at once on the device.
      int j = 0, k = 0;
      for (int j0 = 0; j0 < steps; j0 += kCheckEvery, ++k) {
        const int j1 = std::min(j0 + kCheckEvery, steps);
        run_steps(Z, j0, j1, tol);
        j = j1;
        if (j1 < steps) {
          R3M_CHECK_HIP(hipMemcpyAsync(ctx->run_host + (k & 1), run_slot(j1 - 1), sizeof(int),
                                       hipMemcpyDeviceToHost, s));
          R3M_CHECK_HIP(hipEventRecord(ctx->ev_run[k & 1], s));
        }
        if (k >= 1) {
          R3M_CHECK_HIP(hipEventSynchronize(ctx->ev_run[(k - 1) & 1]));
          if (ctx->run_host[(k - 1) & 1] == 0) break;
        }
      }
      hipLaunchKernelGGL(finalize_kernel, dim3(ceil_div(B, 64)), dim3(64), 0, s, W.st, B, j);
      hipLaunchKernelGGL(backsolve_kernel, dim3(B), dim3(256), 0, s, W.H, W.g, W.st, m);
      if (pre) {
        // x += M^{-1} (V y)
        if (vb32) {
          // with the next restart's residual from the cycle's own basis (the
          // outer FP64 residual checks the solution)
          hipLaunchKernelGGL(residual_coeffs_kernel, dim3(ceil_div(B, 64)), dim3(64), 0, s, (const double2*)W.g,
                             (const double*)W.cs, (const double2*)W.sn, (const RhsState*)W.st, B, m, W.hbuf);
          hipLaunchKernelGGL(combine_basis_res_kernel<float2>, vgrid(), dim3(256), 0, s, (const float2*)W.V, W.g,
                             (const double2*)W.hbuf, W.pz, W.r, W.rv, W.st, m, ut);
          r_from_basis = true;
        } else
          hipLaunchKernelGGL(combine_basis_kernel<double2>, vgrid(), dim3(256), 0, s, (const double2*)W.V, W.g,
                             W.pz, W.rv, W.st, m, ut);
        precond(W.pz, W.w);
        hipLaunchKernelGGL(add_kernel, vgrid(), dim3(256), 0, s, sol, W.w, W.rv, (const RhsState*)W.st);
      } else {
        if (vb32)
          hipLaunchKernelGGL(update_x_kernel<float2>, vgrid(), dim3(256), 0, s, (const float2*)W.V, W.g, sol, W.rv,
                             W.st, m, ut);
        else
          hipLaunchKernelGGL(update_x_kernel<double2>, vgrid(), dim3(256), 0, s, (const double2*)W.V, W.g, sol, W.rv,
                             W.st, m, ut);
      }
      R3M_CHECK_HIP(hipMemcpyAsync(hst.data(), W.st, (size_t)B * sizeof(RhsState), hipMemcpyDeviceToHost, s));
      R3M_CHECK_HIP(hipStreamSynchronize(s));
      for (int b = 0; b < B; ++b)
        if (hst[b].active) iters[b] += hst[b].jdone;
    }
    return rnorm;
  }

  int flag_check(int mask) {
    int f = 0;
    R3M_CHECK_HIP(hipMemcpyAsync(&f, W.counters + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    R3M_CHECK_HIP(hipStreamSynchronize(s));
    return f & mask;
  }
};

// The Krylov basis is stored in complex64 for inner solves on a complex64
// store with a refinement store (the FP64 residual of the outer loop corrects
// what FP32 storage loses), without ILU or relaxed weights
bool basis32(const r3m_store* Z, const r3m_store* Z64, int ilu_r, bool relaxed) {
  return Z64 && Z->near_dtype == R3M_C64 && ilu_r == 0 && !relaxed;
}

size_t gmres_bytes(r3m_ctx ctx, const r3m_store* Z, const r3m_store* Z64, const BatchDesc& bd, int m,
                   bool per_unit, int ilu_r, bool relaxed, bool vb32) {
  const int n_a = vec_per_unit(Z);
  size_t mv = partials_and_x_bytes(bd, Z, max_groups(bd));
  if (Z64) mv = std::max(mv, partials_and_x_bytes(bd, Z64, max_groups(bd)));
  return layout_work(nullptr, bd, n_a, per_unit ? (int)bd.total_units : Z->n_states, m, mv, near_lists_bytes(Z, bd),
                     Z64 ? near_lists_bytes(Z64, bd) : 0, ilu_r ? ilu_factor_bytes(Z, bd, ilu_r, !relaxed) : 0, vb32)
      .bytes;
}

// Shared (connected-geometry) bases: solves without preconditioner on
// spectral stores, the refinement store with the same shared bases
void require_solvable(const r3m_store* Z, const r3m_store* Z64, const r3m_gmres_opts* opts) {
  if (Z->n_common == 0 && (!Z64 || Z64->n_common == 0)) return;
  R3M_REQUIRE(opts->precond == R3M_PRECOND_NONE && !opts->relaxed_weights, R3M_ERR_UNSUPPORTED,
              "solves with shared (connected-geometry) bases take no preconditioner and no relaxed weights yet");
  R3M_REQUIRE(!Z64 || Z64->n_common == Z->n_common, R3M_ERR_INVALID_ARG,
              "the refinement store's shared bases do not match");
}

// the ILU radius a solve uses (0: no ILU), validated against the store
int ilu_radius_of(const r3m_store* Z, const r3m_gmres_opts* opts) {
  if (opts->precond != R3M_PRECOND_BLOCK_ILU) return 0;
  const int r = opts->ilu_radius == 0 ? 1 : opts->ilu_radius;
  validate_ilu(Z, r);
  return r;
}

}  // namespace r3m

using namespace r3m;

extern "C" {

size_t r3m_gmres_work_bytes(r3m_ctx ctx, const r3m_store* Z, const r3m_store* Z64, const r3m_batch* batch,
                            const r3m_gmres_opts* opts) {
  size_t out = 0;
  int rc = guarded(ctx, [&] {
    R3M_REQUIRE(ctx && opts, R3M_ERR_INVALID_ARG, "NULL argument");
    validate_store(Z);
    if (Z64) validate_store(Z64);
    require_solvable(Z, Z64, opts);
    validate_batch(batch, Z->Dx, Z->Dy);
    R3M_REQUIRE(opts->restart >= 1 && opts->restart <= 1024, R3M_ERR_INVALID_ARG, "restart out of range");
    if (batch->B == 0) return;
    const BatchDesc& bd = get_batch(ctx, batch, kTW, kTH, 0);
    const int ilu_r = ilu_radius_of(Z, opts);
    out = gmres_bytes(ctx, Z, Z64, bd, opts->restart,
                      opts->relaxed_weights && opts->precond == R3M_PRECOND_BLOCK_JACOBI, ilu_r,
                      opts->relaxed_weights != nullptr, basis32(Z, Z64, ilu_r, opts->relaxed_weights != nullptr));
  });
  return rc == R3M_OK ? out : 0;
}

int r3m_gmres_solve(r3m_ctx ctx, const r3m_store* Z, const r3m_store* Z64,
                    const r3m_batch* batch, const void* b_dev, void* x_dev,
                    const r3m_gmres_opts* opts, r3m_gmres_report* rep_host, void* work_dev,
                    size_t work_bytes, hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx && opts, R3M_ERR_INVALID_ARG, "NULL argument");
    validate_store(Z);
    validate_batch(batch, Z->Dx, Z->Dy);
    const bool refine = Z64 != nullptr && opts->refine_tol > 0.0;
    require_solvable(Z, refine ? Z64 : nullptr, opts);
    if (refine) {
      validate_store(Z64);
      R3M_REQUIRE(Z64->near_dtype == R3M_C128, R3M_ERR_INVALID_ARG, "refinement store must be C128");
      R3M_REQUIRE(Z64->n == Z->n && Z64->n_states == Z->n_states && Z64->Dx >= Z->Dx && Z64->Dy >= Z->Dy,
                  R3M_ERR_INVALID_ARG, "refinement store does not match");
    }
    R3M_REQUIRE(opts->restart >= 1 && opts->restart <= 1024, R3M_ERR_INVALID_ARG, "restart out of range");
    R3M_REQUIRE(opts->max_iter >= 1, R3M_ERR_INVALID_ARG, "max_iter must be >= 1");
    R3M_REQUIRE(opts->tol > 0.0 && opts->tol < 1.0, R3M_ERR_INVALID_ARG, "tol must be in (0, 1)");
    if (batch->B == 0) return;
    R3M_REQUIRE(b_dev && x_dev && work_dev && rep_host, R3M_ERR_INVALID_ARG, "NULL buffer");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    const BatchDesc& bd = get_batch(ctx, batch, kTW, kTH, stream);
    const int m = opts->restart;
    const int n_a = vec_per_unit(Z);  // vector entries per unit
    const bool per_unit = opts->relaxed_weights && opts->precond == R3M_PRECOND_BLOCK_JACOBI;
    R3M_REQUIRE(opts->precond == R3M_PRECOND_NONE || opts->precond == R3M_PRECOND_BLOCK_JACOBI ||
                    opts->precond == R3M_PRECOND_BLOCK_ILU,
                R3M_ERR_INVALID_ARG, "unknown preconditioner");
    const int ilu_r = ilu_radius_of(Z, opts);
    const bool vb32 = basis32(Z, Z64, ilu_r, opts->relaxed_weights != nullptr);
    const size_t need = gmres_bytes(ctx, Z, refine ? Z64 : nullptr, bd, m, per_unit, ilu_r,
                                    opts->relaxed_weights != nullptr, vb32);
    R3M_REQUIRE(work_bytes >= need, R3M_ERR_BUFFER_TOO_SMALL, "GMRES workspace too small");

    size_t mv = partials_and_x_bytes(bd, Z, max_groups(bd));
    if (refine) mv = std::max(mv, partials_and_x_bytes(bd, Z64, max_groups(bd)));
    // all work runs on the context stream, ordered after the caller's stream
    if (!ctx->work_stream) {
      R3M_CHECK_HIP(hipStreamCreateWithFlags(&ctx->work_stream, hipStreamNonBlocking));
      R3M_CHECK_HIP(hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
      R3M_CHECK_HIP(hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming));
    }
    if (!ctx->run_host) {
      R3M_CHECK_HIP(hipHostMalloc((void**)&ctx->run_host, 2 * sizeof(int), hipHostMallocDefault));
      for (hipEvent_t& e : ctx->ev_run) R3M_CHECK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    R3M_CHECK_HIP(hipEventRecord(ctx->ev_in, stream));
    R3M_CHECK_HIP(hipStreamWaitEvent(ctx->work_stream, ctx->ev_in, 0));
    const hipStream_t user_stream = stream;
    stream = ctx->work_stream;
    struct Rejoin {
      r3m_ctx c;
      hipStream_t us;
      ~Rejoin() {
        (void)hipEventRecord(c->ev_out, c->work_stream);
        (void)hipStreamWaitEvent(us, c->ev_out, 0);
      }
    } rejoin{ctx, user_stream};
    GmresRun run;
    run.ctx = ctx;
    run.use_graph = !(opts->flags & R3M_GMRES_EAGER);
    run.graph_key = {(int64_t)(intptr_t)&bd, (int64_t)(intptr_t)batch->states, (int64_t)(intptr_t)work_dev,
                     (int64_t)m, (int64_t)opts->precond, (int64_t)bd.B, (int64_t)n_a,
                     (int64_t)(intptr_t)opts->relaxed_weights, (int64_t)opts->transpose, (int64_t)ilu_r};
    run.wts = opts->relaxed_weights;
    run.tr = opts->relaxed_weights && opts->transpose;
    run.bd = &bd;
    run.batch = batch;
    run.n_a = n_a;
    run.m = m;
    run.B = bd.B;
    run.s = stream;
    run.W = layout_work((char*)work_dev, bd, n_a, per_unit ? (int)bd.total_units : Z->n_states, m, mv,
                        near_lists_bytes(Z, bd), refine ? near_lists_bytes(Z64, bd) : 0,
                        ilu_r ? ilu_factor_bytes(Z, bd, ilu_r, opts->relaxed_weights == nullptr) : 0, vb32);
    run.vb32 = vb32;
    run.Zsolve = Z;
    run.ut = (int64_t)bd.total_units * n_a;
    run.maxN = 0;
    std::vector<RhsVec> rv(bd.B);
    std::vector<int64_t> soff(bd.B);
    for (int b = 0; b < bd.B; ++b) {
      rv[b] = RhsVec{bd.unit_off[b] * n_a, bd.n_units[b] * n_a};
      run.maxN = std::max(run.maxN, rv[b].N);
      soff[b] = batch->state_off[b];
    }
    run.maxP = (int)((run.maxN + kDotChunk - 1) / kDotChunk);
    R3M_CHECK_HIP(hipMemcpyAsync(run.W.rv, rv.data(), rv.size() * sizeof(RhsVec), hipMemcpyHostToDevice, stream));
    R3M_CHECK_HIP(hipMemcpyAsync(run.W.soff, soff.data(), soff.size() * 8, hipMemcpyHostToDevice, stream));
    R3M_CHECK_HIP(hipMemsetAsync(run.W.counters, 0, 256, stream));

    if (opts->relaxed_weights) {
      R3M_REQUIRE(store_is_spectral(Z) && (!refine || store_is_spectral(Z64)), R3M_ERR_UNSUPPORTED,
                  "relaxed retrieval needs spectral stores");
    }
    // input checks on the device: state bytes and finite right-hand sides
    const int64_t maxU = run.maxN / n_a;
    hipLaunchKernelGGL(states_check_kernel, dim3(ceil_div((size_t)maxU, 256), bd.B), dim3(256), 0, stream,
                       batch->states, run.W.rv, run.W.soff, n_a, Z->n_states, run.W.counters + 1);
    hipLaunchKernelGGL(nonfinite_kernel, run.vgrid(), dim3(256), 0, stream, (const double2*)b_dev, run.W.rv,
                       run.W.counters + 1);
    run.n_states = Z->n_states;
    if (opts->precond == R3M_PRECOND_BLOCK_JACOBI) {
      run.pre = true;
      const int Nx = std::min(Z->near_radius, Z->Dx), Ny = std::min(Z->near_radius, Z->Dy);
      const int slot0 = Ny * (2 * Nx + 1) + Nx;
      const size_t lds = ((size_t)n_a * 2 * n_a + n_a + 1) * sizeof(double2);
      if (per_unit) {  // relaxed codebook: the blended self block of every unit
        run.pu = 1;
        const dim3 ig((unsigned)maxU, bd.B);
        if (Z->near_dtype == R3M_C128)
          hipLaunchKernelGGL(relaxed_selfblock_inverse_kernel<double>, ig, dim3(256), lds, stream,
                             (const double*)Z->near, slot0, Z->n, n_a, Z->n_states, (const RhsVec*)run.W.rv,
                             opts->relaxed_weights, run.tr ? 1 : 0, run.W.Minv, run.W.counters + 1);
        else
          hipLaunchKernelGGL(relaxed_selfblock_inverse_kernel<float>, ig, dim3(256), lds, stream,
                             (const float*)Z->near, slot0, Z->n, n_a, Z->n_states, (const RhsVec*)run.W.rv,
                             opts->relaxed_weights, run.tr ? 1 : 0, run.W.Minv, run.W.counters + 1);
      } else if (Z->near_dtype == R3M_C128)
        hipLaunchKernelGGL(selfblock_inverse_kernel<double>, dim3(Z->n_states), dim3(256), lds, stream,
                           (const double*)Z->near, slot0, Z->n, n_a, run.W.Minv, run.W.counters + 1);
      else
        hipLaunchKernelGGL(selfblock_inverse_kernel<float>, dim3(Z->n_states), dim3(256), lds, stream,
                           (const float*)Z->near, slot0, Z->n, n_a, run.W.Minv, run.W.counters + 1);
      R3M_CHECK_HIP(hipGetLastError());
    } else if (ilu_r) {
      run.pre = true;
      run.ilu_r = ilu_r;
      launch_ilu_factor(Z, bd, batch->states, ilu_r, run.W.ilu, run.W.counters + 1, stream, opts->relaxed_weights,
                        run.tr);
    }
    // one read-back for the input checks and the preconditioner's pivots
    const int f = run.flag_check(14);
    R3M_REQUIRE(!(f & 2), R3M_ERR_INVALID_ARG, "codebook state out of range");
    R3M_REQUIRE(!(f & 4), R3M_ERR_NONFINITE, "non-finite right-hand side");
    R3M_REQUIRE(!(f & 8), R3M_ERR_NONFINITE, "singular self block in the preconditioner");
    const double2* b = (const double2*)b_dev;
    double2* x = (double2*)x_dev;
    // near retrieval lists of this codebook (fixed for the whole solve)
    build_near_lists(Z, bd, batch->states, run.W.lists, stream);
    if (refine) build_near_lists(Z64, bd, batch->states, run.W.lists64, stream);
    // autotune the matvec's displacement groups on the right-hand side (before any capture)
    {
      const void* xin = b;
      if (Z->near_dtype == R3M_C64) {
        hipLaunchKernelGGL(convert_vec_kernel<float>, run.vgrid(), dim3(256), 0, stream, run.W.rv, b,
                           (float*)run.W.xs, (const int*)nullptr);
        xin = run.W.xs;
      }
      run.G = tuned_groups(ctx, Z, bd, batch->states, xin, run.W.w, run.W.mv_partial, run.W.lists, stream);
    }
    std::vector<double> bnorm = run.host_norms(b);
    hipLaunchKernelGGL(zero_kernel, run.vgrid(), dim3(256), 0, stream, x, run.W.rv);
    std::vector<int> iters(bd.B, 0), refine_steps(bd.B, 0);
    std::vector<double> rel(bd.B, 0.0);
    double target = opts->tol;
    if (refine) {
      target = opts->refine_tol;
      const int max_refine = std::max(1, opts->max_refine);
      for (int step = 0; step <= max_refine; ++step) {
        // x is zero at the first step: its residual is b itself
        std::vector<double> rn;
        if (step == 0) {
          R3M_CHECK_HIP(hipMemcpyAsync(run.W.ro, b, (size_t)run.ut * 16, hipMemcpyDeviceToDevice, stream));
          rn = bnorm;
        } else {
          run.residual(Z64, b, x, run.W.ro);
          rn = run.host_norms(run.W.ro);
        }
        std::vector<int> act(bd.B, 0);
        bool any = false;
        for (int i = 0; i < bd.B; ++i) {
          rel[i] = bnorm[i] > 0 ? rn[i] / bnorm[i] : 0.0;
          act[i] = (rel[i] > target && iters[i] < opts->max_iter) ? 1 : 0;
          any = any || act[i];
        }
        if (!any || step == max_refine) break;
        hipLaunchKernelGGL(zero_kernel, run.vgrid(), dim3(256), 0, stream, run.W.d, run.W.rv);
        run.solve(Z, run.W.ro, run.W.d, act, rn, opts->tol, opts->max_iter, iters, true);
        hipLaunchKernelGGL(add_kernel, run.vgrid(), dim3(256), 0, stream, x, run.W.d, run.W.rv,
                           (const RhsState*)nullptr);
        for (int i = 0; i < bd.B; ++i) refine_steps[i] += act[i];
      }
    } else {
      // the true residual at exit comes back from the solve's last check
      const std::vector<double> rn =
          run.solve(Z, b, x, std::vector<int>(bd.B, 1), bnorm, opts->tol, opts->max_iter, iters, true);
      for (int i = 0; i < bd.B; ++i) rel[i] = bnorm[i] > 0 ? rn[i] / bnorm[i] : 0.0;
    }
    hipLaunchKernelGGL(nonfinite_kernel, run.vgrid(), dim3(256), 0, stream, (const double2*)x, run.W.rv,
                       run.W.counters + 1);
    R3M_REQUIRE(!run.flag_check(4), R3M_ERR_NONFINITE, "non-finite solution");
    bool all = true;
    for (int i = 0; i < bd.B; ++i) {
      rep_host[i].iters = iters[i];
      rep_host[i].refine_steps = refine_steps[i];
      rep_host[i].rel_residual = rel[i];
      rep_host[i].converged = rel[i] <= target ? 1 : 0;
      all = all && rep_host[i].converged;
    }
    take_deferred(ctx, stream);  // errors left by earlier asynchronous calls on this context
    R3M_REQUIRE(all, R3M_ERR_NOT_CONVERGED, "some right-hand sides did not converge");
  });
}

}  // extern "C"
