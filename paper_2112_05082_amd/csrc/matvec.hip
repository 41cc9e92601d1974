// Retrieved matrix-vector product y_k = P_k^T Z P_k x_k (eq. (3); the D_k mask
// of eq. (6) in reduced coordinates) over a block store of unique
// displacement blocks (finest 1x1 patterns of eq. (7)).
//
// y[i] = sum_j Z(i - j)[A(s_i), A(s_j)] x[j]
//   near d (Chebyshev <= near_radius): dense block rows/cols of the states,
//   far d: U(d)[A(s_i), :] (V(d)[A(s_j), :]^H x[j]).
//
// Work decomposition: a workgroup owns a TW x TH tile of observer units of one
// right-hand side and a strided chunk of the displacements; its threads are
// (unit, row) pairs.  The partial sums of the chunks are added in a fixed
// order by a second kernel, so the result is bitwise reproducible (no float
// atomics).
#include <cstdlib>
#include "matvec_internal.h"

#include <mutex>

#include <algorithm>
#include <hip/hip_fp16.h>
#include <type_traits>

namespace r3m {
namespace {

constexpr int kTW = 4, kTH = 4, kTU = kTW * kTH;  // tile of one wave
constexpr int kBW = 8, kBH = 8, kBU = kBW * kBH;  // block of one workgroup (2 x 2 tiles)
constexpr int kQ = 4;     // lanes per observer unit (row quarters)


template <typename T>
struct Cx {
  T re, im;
};

// two consecutive complex values (index must be even for the vector load)
template <typename T>
__device__ inline void load2(const T* p, size_t idx, Cx<T>& a, Cx<T>& b);
template <>
__device__ inline void load2<float>(const float* p, size_t idx, Cx<float>& a, Cx<float>& b) {
  const float4 v = *reinterpret_cast<const float4*>(p + 2 * idx);
  a = {v.x, v.y};
  b = {v.z, v.w};
}
template <>
__device__ inline void load2<double>(const double* p, size_t idx, Cx<double>& a, Cx<double>& b) {
  const double2 u = *reinterpret_cast<const double2*>(p + 2 * idx);
  const double2 v = *reinterpret_cast<const double2*>(p + 2 * idx + 2);
  a = {u.x, u.y};
  b = {v.x, v.y};
}

// Workgroups are dispatched round-robin over the 8 XCDs (id % 8).  The 1D grid
// is decoded so that the n_blocks workgroups sharing a displacement group sit
// on one XCD and meet its factor blocks in that XCD's L2.  Returns false for
// padding workgroups.
constexpr int kXcd = 8;
__device__ __forceinline__ bool decode_wg(int id, int n_blocks, int n_groups, int& blk, int& grp) {
  const int total = n_blocks * n_groups;
  const int per = (total + kXcd - 1) / kXcd;
  const int t = (id % kXcd) * per + id / kXcd;
  if (t >= total) return false;
  grp = t / n_blocks;
  blk = t % n_blocks;
  return true;
}

// acc += a * b as two fused multiply-adds per real component
template <typename S>
__device__ __forceinline__ void cmac(S& re, S& im, Cx<S> a, Cx<S> b) {
  re = fma(a.re, b.re, re);
  re = fma(-a.im, b.im, re);
  im = fma(a.re, b.im, im);
  im = fma(a.im, b.re, im);
}
// acc += conj(a) * b
template <typename S>
__device__ __forceinline__ void cmacc(S& re, S& im, Cx<S> a, Cx<S> b) {
  re = fma(a.re, b.re, re);
  re = fma(a.im, b.im, re);
  im = fma(a.re, b.im, im);
  im = fma(-a.im, b.re, im);
}

// lane swaps inside a quad of lanes (DPP quad permutes)
__device__ __forceinline__ float quad_swap1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float quad_swap2(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
}
__device__ __forceinline__ double quad_swap1(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double quad_swap2(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0x4E, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x4E, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Far contribution of one staged rank slice (RC ranks, compile-time) for one
// lane: t = V[A(s_j)]^H x_j over the lane's quarter, summed over the unit's
// four lanes, then y += U[A(s_i)] t on the lane's rows.  The LDS reads of the
// next rank are issued before the products of the current one (scheduling
// barriers keep that order), so one rank of FMAs covers their latency.
#ifndef R3M_FAR_DEPTH
#define R3M_FAR_DEPTH 1
#endif
constexpr int kFarDepth = R3M_FAR_DEPTH;  // factor rows read ahead of their products

template <typename S, int QS>
__device__ __forceinline__ void lds_row(const Cx<S>* __restrict__ lds, size_t at, Cx<S> (&v)[QS]) {
#pragma unroll
  for (int k = 0; k < QS; k += 2) load2<S>(reinterpret_cast<const S*>(lds), at + k, v[k], v[k + 1]);
}

template <typename S, int QS, int RC>
__device__ __forceinline__ void far_slice(const Cx<S>* __restrict__ lds_u, const Cx<S>* __restrict__ lds_v,
                                          int n, int offi, int offj, int m0, bool vj, const Cx<S> (&xr)[QS],
                                          S (&acc_re)[QS], S (&acc_im)[QS]) {
  S t_re[RC], t_im[RC];
#pragma unroll
  for (int rr = 0; rr < RC; ++rr) t_re[rr] = t_im[rr] = 0;
  if constexpr (sizeof(S) == 8) {  // complex128: no room for a second row in registers
    if (vj) {
#pragma unroll
      for (int k = 0; k < QS; k += 2) {
        const Cx<S> x0 = xr[k], x1 = xr[k + 1];
#pragma unroll
        for (int rr = 0; rr < RC; ++rr) {
          Cx<S> v0, v1;
          load2<S>(reinterpret_cast<const S*>(lds_v), (size_t)rr * n + offj + m0 + k, v0, v1);
          cmacc(t_re[rr], t_im[rr], v0, x0);
          cmacc(t_re[rr], t_im[rr], v1, x1);
        }
      }
    }
#pragma unroll
    for (int rr = 0; rr < RC; ++rr) {
      t_re[rr] += quad_swap1(t_re[rr]);
      t_im[rr] += quad_swap1(t_im[rr]);
      t_re[rr] += quad_swap2(t_re[rr]);
      t_im[rr] += quad_swap2(t_im[rr]);
    }
    if (vj) {
#pragma unroll
      for (int rr = 0; rr < RC; ++rr) {
#pragma unroll
        for (int k = 0; k < QS; k += 2) {
          Cx<S> u0, u1;
          load2<S>(reinterpret_cast<const S*>(lds_u), (size_t)rr * n + offi + m0 + k, u0, u1);
          const Cx<S> tv = {t_re[rr], t_im[rr]};
          cmac(acc_re[k], acc_im[k], u0, tv);
          cmac(acc_re[k + 1], acc_im[k + 1], u1, tv);
        }
      }
    }
    return;
  }
  constexpr int NB = kFarDepth + 1;  // rows in flight + the one in use
  Cx<S> vb[NB][QS];
  if (vj) {
#pragma unroll
    for (int rr = 0; rr < kFarDepth && rr < RC; ++rr) lds_row<S, QS>(lds_v, (size_t)rr * n + offj + m0, vb[rr]);
#pragma unroll
    for (int rr = 0; rr < RC; ++rr) {
      if (rr + kFarDepth < RC)
        lds_row<S, QS>(lds_v, (size_t)(rr + kFarDepth) * n + offj + m0, vb[(rr + kFarDepth) % NB]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < QS; ++k) cmacc(t_re[rr], t_im[rr], vb[rr % NB][k], xr[k]);  // conj(v) x
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int rr = 0; rr < RC; ++rr) {
    t_re[rr] += quad_swap1(t_re[rr]);
    t_im[rr] += quad_swap1(t_im[rr]);
    t_re[rr] += quad_swap2(t_re[rr]);
    t_im[rr] += quad_swap2(t_im[rr]);
  }
  if (vj) {
#pragma unroll
    for (int rr = 0; rr < kFarDepth && rr < RC; ++rr) lds_row<S, QS>(lds_u, (size_t)rr * n + offi + m0, vb[rr]);
#pragma unroll
    for (int rr = 0; rr < RC; ++rr) {
      if (rr + kFarDepth < RC)
        lds_row<S, QS>(lds_u, (size_t)(rr + kFarDepth) * n + offi + m0, vb[(rr + kFarDepth) % NB]);
      __builtin_amdgcn_sched_barrier(0);
      const Cx<S> tv = {t_re[rr], t_im[rr]};
#pragma unroll
      for (int k = 0; k < QS; ++k) cmac(acc_re[k], acc_im[k], vb[rr % NB][k], tv);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Near field: one workgroup of four waves per (8x8 block of observer units,
// near displacement d); wave w owns the 4x4 tile (w & 1, w >> 1) of the
// block, lane (unit, quarter q) owns rows [q*QS, q*QS + QS) of y_u and adds
// Z(d)[A(s_i), A(s_j)] x_j.  The result goes to its own partial slot.
// Near field: one workgroup per (8x8 block of observer units, near group h);
// the group's near displacements are taken in turn.  Per displacement the
// block's 64 shifted sources (x_j and state) are staged in LDS; then for each
// observer state a, rows of the slab Z(d)[A(a), :] are staged in LDS with
// coalesced loads (SR rows per pass) and every (unit, row) task of the units
// in state a adds slab[row][A(s_j)] . x_j into an LDS accumulator.  Each
// accumulator entry is written by one task per pass, so the sum is in fixed
// order.  The block's result goes to partial slot slot0 + h.
template <typename S, int SR>
__global__ void __launch_bounds__(256)
near_kernel(const RhsDev* __restrict__ rhs, const TileDev* __restrict__ tiles, const uint8_t* __restrict__ states,
            const S* __restrict__ nearb, int Nx, int Ny, int n, int n_a, int n_states, const S* __restrict__ x,
            S* __restrict__ out, int64_t total_units, int slot0, int hgroups, int n_blocks) {
  extern __shared__ unsigned char smem_raw[];
  // slab rows padded to n + 2 so that lanes reading consecutive rows fall in
  // different LDS banks
  const int ns = n + 2;
  Cx<S>* slab = reinterpret_cast<Cx<S>*>(smem_raw);  // [SR][n + 2]
  Cx<S>* yacc = slab + (size_t)SR * ns;               // [kBU][n_a]
  Cx<S>* xl = yacc + (size_t)kBU * n_a;               // [kBU][n_a]
  __shared__ uint8_t list[kBU];
  __shared__ int cnt[17];
  __shared__ int start[17];
  __shared__ uint8_t ust[kBU];
  __shared__ int sst[kBU];
  int bi, h;
  if (!decode_wg(blockIdx.x, n_blocks, hgroups, bi, h)) return;
  const TileDev blk = tiles[bi];
  const RhsDev R = rhs[blk.b];
  const int tid = threadIdx.x;
  for (int e = tid; e < kBU * n_a; e += blockDim.x) yacc[e] = Cx<S>{0, 0};
  if (tid <= 16) cnt[tid] = 0;
  __syncthreads();
  if (tid < kBU) {
    const int ix = blk.tx + tid % kBW, iy = blk.ty + tid / kBW;
    const int st = (ix < R.Lx && iy < R.Ly) ? min((int)states[R.state_off + (int64_t)iy * R.Lx + ix], n_states - 1)
                                            : 255;
    ust[tid] = (uint8_t)st;
    if (st != 255) atomicAdd(&cnt[st], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int c = 0;
    for (int a = 0; a < n_states; ++a) {
      start[a] = c;
      c += cnt[a];
      cnt[a] = 0;
    }
    start[n_states] = c;
  }
  __syncthreads();
  if (tid < kBU && ust[tid] != 255) {
    const int pos = atomicAdd(&cnt[ust[tid]], 1);
    list[start[ust[tid]] + pos] = (uint8_t)tid;
  }
  const int n_near = (2 * Nx + 1) * (2 * Ny + 1);
  const int bx_hi = min(blk.tx + kBW, R.Lx) - 1, by_hi = min(blk.ty + kBH, R.Ly) - 1;
  for (int nslot = h; nslot < n_near; nslot += hgroups) {
    const int dx = nslot % (2 * Nx + 1) - Nx, dy = nslot / (2 * Nx + 1) - Ny;
    if (bx_hi - dx < 0 || blk.tx - dx > R.Lx - 1 || by_hi - dy < 0 || blk.ty - dy > R.Ly - 1) continue;
    __syncthreads();
    // the block's shifted sources
    if (tid < kBU) {
      const int jx = blk.tx + tid % kBW - dx, jy = blk.ty + tid / kBW - dy;
      const bool v = ust[tid] != 255 && jx >= 0 && jx < R.Lx && jy >= 0 && jy < R.Ly;
      sst[tid] = v ? min((int)states[R.state_off + (int64_t)jy * R.Lx + jx], n_states - 1) : -1;
    }
    for (int e2 = 2 * tid; e2 < kBU * n_a; e2 += 2 * blockDim.x) {
      const int u = e2 / n_a, c = e2 % n_a;
      const int jx = blk.tx + u % kBW - dx, jy = blk.ty + u / kBW - dy;
      Cx<S> x0{0, 0}, x1{0, 0};
      if (jx >= 0 && jx < R.Lx && jy >= 0 && jy < R.Ly)
        load2<S>(x + (size_t)(R.unit_off + (int64_t)jy * R.Lx + jx) * n_a * 2, c, x0, x1);
      xl[e2] = x0;
      xl[e2 + 1] = x1;
    }
    const S* Zb = nearb + (size_t)nslot * n * n * 2;
    for (int a = 0; a < n_states; ++a) {
      const int c0 = start[a], c1 = start[a + 1];
      if (c1 == c0) continue;
      for (int r0 = 0; r0 < n_a; r0 += SR) {
        __syncthreads();
        {
          const S* src = Zb + ((size_t)a * n_a + r0) * n * 2;  // rows A(a)[r0, r0 + SR), contiguous
          for (int e2 = 2 * tid; e2 < SR * n; e2 += 2 * blockDim.x) {
            Cx<S> z0, z1;
            load2<S>(src, e2, z0, z1);
            const int d2 = (e2 / n) * ns + e2 % n;
            slab[d2] = z0;
            slab[d2 + 1] = z1;
          }
        }
        __syncthreads();
        const int ntask = (c1 - c0) * SR;
        for (int t = tid; t < ntask; t += blockDim.x) {
          const int u = list[c0 + t / SR], row = t % SR;
          const int sj = sst[u];
          if (sj < 0) continue;
          const S* xr = reinterpret_cast<const S*>(xl + u * n_a);
          const S* zr = reinterpret_cast<const S*>(slab) + ((size_t)row * ns + sj * n_a) * 2;
          S re = 0, im = 0;
          for (int c = 0; c < n_a; c += 2) {
            Cx<S> x0, x1, z0, z1;
            load2<S>(xr, c, x0, x1);
            load2<S>(zr, c, z0, z1);
            cmac(re, im, z0, x0);
            cmac(re, im, z1, x1);
          }
          Cx<S>& yv = yacc[u * n_a + r0 + row];
          yv.re += re;
          yv.im += im;
        }
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < kBU * n_a; e += blockDim.x) {
    const int u = e / n_a, m = e % n_a;
    const int ix = blk.tx + u % kBW, iy = blk.ty + u / kBW;
    if (ix >= R.Lx || iy >= R.Ly) continue;
    const size_t yb = (size_t)(R.unit_off + (int64_t)iy * R.Lx + ix) * n_a + m;
    S* o = out + ((size_t)(slot0 + h) * total_units * n_a + yb) * 2;
    o[0] = yacc[e].re;
    o[1] = yacc[e].im;
  }
}

// Far field: one workgroup of four waves per (8x8 block of observer units,
// displacement group); wave w owns the 4x4 tile (w & 1, w >> 1).  The far
// displacements of the block (those of the rectangle that keeps a source in
// the array, minus the near square) are dealt out round-robin to the groups.
// Per displacement, the workgroup stages up to kRch rows of U and V (all
// states) in LDS; the next displacement's slice and the lane's quarter of
// x_j are fetched into registers while the current one is computed.  Lane
// (unit u, quarter q) forms its quarter of t = V[A(s_j)]^H x_j, the unit's
// four lanes add their parts with two lane swaps, and the lane expands its own
// rows y += U[A(s_i)] t.  Ranks above kRch take extra synchronous slices.
// complex64: 4-rank slices (most ranks are 4 at tol 1e-4), three waves per
// SIMD at 40 rows per state; complex128 and 64 rows per state: two waves
// per SIMD (register bound)
#ifndef R3M_FAR_RCH_F32
#define R3M_FAR_RCH_F32 4
#endif
#ifndef R3M_FAR_WAVES_PER_EU_F32
#define R3M_FAR_WAVES_PER_EU_F32 3
#endif
#ifndef R3M_FAR_WAVES_PER_EU_F64
#define R3M_FAR_WAVES_PER_EU_F64 2
#endif
// Two consecutive factor entries (complex index idx, even) in storage format
// FT: the store precision itself, or an 8-byte split element
// {re_hi | im_hi << 16, re_lo | im_lo << 16} decoded to hi + lo in FP32
// (BF16X2), times the column scale sc (F16X2).
template <typename S, int FT>
__device__ __forceinline__ void load_factor2(const S* p, size_t idx, float sc, Cx<S>& a, Cx<S>& b) {
  if constexpr (FT == R3M_BF16X2 || FT == R3M_F16X2) {
    static_assert(sizeof(S) == 4, "split factors decode to FP32");
    const uint4 w = *reinterpret_cast<const uint4*>(p + 2 * idx);
    if constexpr (FT == R3M_BF16X2) {
      a = {__uint_as_float(w.x << 16) + __uint_as_float(w.y << 16),
           __uint_as_float(w.x & 0xffff0000u) + __uint_as_float(w.y & 0xffff0000u)};
      b = {__uint_as_float(w.z << 16) + __uint_as_float(w.w << 16),
           __uint_as_float(w.z & 0xffff0000u) + __uint_as_float(w.w & 0xffff0000u)};
    } else {
      auto h = [](uint32_t bits) { return __half2float(__ushort_as_half((unsigned short)(bits & 0xffffu))); };
      a = {(h(w.x) + h(w.y)) * sc, (h(w.x >> 16) + h(w.y >> 16)) * sc};
      b = {(h(w.z) + h(w.w)) * sc, (h(w.z >> 16) + h(w.w >> 16)) * sc};
    }
  } else {
    (void)sc;
    load2<S>(p, idx, a, b);
  }
}

template <typename S>
struct FarArgs {
  const RhsDev* rhs;
  const TileDev* tiles;
  int groups;
  const uint8_t* states;
  const S* farf;        // factors (store precision or split elements)
  const int* ranks;
  const float* fscale;  // F16X2 column scales, else NULL
  int max_rank, Dx, Dy, nr, n, n_a, n_states;
  const S* x;
  S* out;
  int64_t total_units;
  int lds_state_cap, n_blocks;
  const int* idle;  // per right-hand side (nullable): tiles of b with idle[b] != 0 return at once
};

// far field of workgroup wg (see far_kernel)
template <typename S, int QS, int kRch, int FT>
__device__ __forceinline__ void far_body(const FarArgs<S>& A, int wg) {
  const RhsDev* __restrict__ rhs = A.rhs;
  const TileDev* __restrict__ tiles = A.tiles;
  const int groups = A.groups;
  const uint8_t* __restrict__ states = A.states;
  const S* __restrict__ farf = A.farf;
  const int* __restrict__ ranks = A.ranks;
  const float* __restrict__ fscale = A.fscale;
  const int max_rank = A.max_rank, Dx = A.Dx, Dy = A.Dy, nr = A.nr, n = A.n, n_a = A.n_a, n_states = A.n_states;
  const S* __restrict__ x = A.x;
  S* __restrict__ out = A.out;
  const int64_t total_units = A.total_units;
  const int lds_state_cap = A.lds_state_cap, n_blocks = A.n_blocks;
  extern __shared__ unsigned char smem_raw[];
  Cx<S>* lds_u = reinterpret_cast<Cx<S>*>(smem_raw);  // [2][kRch][n]
  Cx<S>* lds_v = lds_u + 2 * kRch * n;                 // [2][kRch][n]
  uint8_t* lds_s = reinterpret_cast<uint8_t*>(lds_v + 2 * kRch * n);
  int bi, g;
  if (!decode_wg(wg, n_blocks, groups, bi, g)) return;
  const TileDev blk = tiles[bi];
  if (A.idle && A.idle[blk.b]) return;  // uniform over the workgroup
  const RhsDev R = rhs[blk.b];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int ul = lane / kQ, q = lane % kQ;
  const int tx = blk.tx + (wave & 1) * kTW, ty = blk.ty + (wave >> 1) * kTH;
  const int ix = tx + ul % kTW, iy = ty + ul / kTW;
  const bool vi = ix < R.Lx && iy < R.Ly;

  const int64_t units = (int64_t)R.Lx * R.Ly;
  const bool st_lds = units <= lds_state_cap;
  if (st_lds)
    for (int64_t u = tid; u < units; u += blockDim.x) lds_s[u] = states[R.state_off + u];
  __syncthreads();
  auto state_at = [&](int64_t u) -> int {
    const int s = st_lds ? lds_s[u] : states[R.state_off + u];
    return min(s, n_states - 1);
  };
  const int si = vi ? state_at((int64_t)iy * R.Lx + ix) : 0;
  const int offi = si * n_a;
  const int m0 = q * QS;

  const int bx_hi = min(blk.tx + 2 * kTW, R.Lx) - 1, by_hi = min(blk.ty + 2 * kTH, R.Ly) - 1;
  const int dx_lo = blk.tx - (R.Lx - 1), dy_lo = blk.ty - (R.Ly - 1);
  const int wdx = bx_hi - dx_lo + 1;
  const int nd = wdx * (by_hi - dy_lo + 1);
  const int ox_hi = min(tx + kTW, R.Lx) - 1, oy_hi = min(ty + kTH, R.Ly) - 1;
  const bool wave_has_obs = tx < R.Lx && ty < R.Ly;
  const int fstride = 2 * max_rank * n * 2;  // reals per far block

  // next far displacement of this group at or after e (uniform); nd if none
  auto next_far = [&](int e) {
    for (; e < nd; e += groups) {
      const int dx = dx_lo + e % wdx, dy = dy_lo + e / wdx;
      if ((dx < 0 ? -dx : dx) > nr || (dy < 0 ? -dy : dy) > nr) return e;
    }
    return nd;
  };

  // per-thread share of one staged slice: rows [rho0, rho0 + rc) of U and V
  constexpr int kPer = (kRch * 256 + 511) / 512;  // pairs per thread for one slice (n <= 256)
  Cx<S> pu[2 * kPer], pv[2 * kPer];
  // column scales of far block f (F16X2 only): U columns, then V columns
  auto col_scale = [&](int f, int col) -> float {
    return FT == R3M_F16X2 ? fscale[(size_t)f * 2 * max_rank + col] : 1.0f;
  };
  auto fetch = [&](int f, int rho0, int rc) {
    const S* Uf = farf + (size_t)f * fstride;
    const int cnt = rc * n;
    const S* us = Uf + (size_t)rho0 * n * 2;
    const S* vs = Uf + (size_t)max_rank * n * 2 + (size_t)rho0 * n * 2;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e2 = 2 * (tid + i * 256);
      if (e2 < cnt) {
        const int col = rho0 + e2 / n;
        load_factor2<S, FT>(us, e2, col_scale(f, col), pu[2 * i], pu[2 * i + 1]);
        load_factor2<S, FT>(vs, e2, col_scale(f, max_rank + col), pv[2 * i], pv[2 * i + 1]);
      }
    }
  };
  auto stash = [&](int rc, int bsel) {
    const int cnt = rc * n;
    Cx<S>* du = lds_u + bsel * kRch * n;
    Cx<S>* dv = lds_v + bsel * kRch * n;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e2 = 2 * (tid + i * 256);
      if (e2 < cnt) {
        du[e2] = pu[2 * i];
        du[e2 + 1] = pu[2 * i + 1];
        dv[e2] = pv[2 * i];
        dv[e2 + 1] = pv[2 * i + 1];
      }
    }
  };
  auto fetch_x = [&](int dx, int dy, Cx<S> (&xr)[QS]) {
    const int jx = ix - dx, jy = iy - dy;
    const bool vj = vi && jx >= 0 && jx < R.Lx && jy >= 0 && jy < R.Ly;
    if (vj) {
      const S* xj = x + (size_t)(R.unit_off + (int64_t)jy * R.Lx + jx) * n_a * 2;
#pragma unroll
      for (int k = 0; k < QS; k += 2) load2<S>(xj, m0 + k, xr[k], xr[k + 1]);
    }
  };

  S acc_re[QS], acc_im[QS];
#pragma unroll
  for (int k = 0; k < QS; ++k) acc_re[k] = acc_im[k] = 0;

  // double-buffered slices: the next displacement's slice is fetched and
  // stashed into the other buffer while this one is computed (one barrier
  // per displacement)
  int buf = 0;
  int e = next_far(g);
  int f = 0, r = 0;
  if (e < nd) {
    const int dx = dx_lo + e % wdx, dy = dy_lo + e / wdx;
    f = far_index(dx, dy, Dx, Dy, nr);
    r = ranks[f];
    fetch(f, 0, min(kRch, r));
    stash(min(kRch, r), 0);
  }
  __syncthreads();
  while (e < nd) {
    const int dx = dx_lo + e % wdx, dy = dy_lo + e / wdx;
    const int rc = min(kRch, r);
    const int en = next_far(e + groups);
    int fnext = 0, rnext = 0;
    if (en < nd) {
      const int dxn = dx_lo + en % wdx, dyn = dy_lo + en / wdx;
      fnext = far_index(dxn, dyn, Dx, Dy, nr);
      rnext = ranks[fnext];
      fetch(fnext, 0, min(kRch, rnext));
    }
    const bool wave_active = wave_has_obs && !(ox_hi - dx < 0 || tx - dx > R.Lx - 1 || oy_hi - dy < 0 ||
                                               ty - dy > R.Ly - 1);
    const int jx = ix - dx, jy = iy - dy;
    const bool vj = vi && jx >= 0 && jx < R.Lx && jy >= 0 && jy < R.Ly;
    const int offj = vj ? state_at((int64_t)jy * R.Lx + jx) * n_a : 0;
    Cx<S> xc[QS];
    fetch_x(dx, dy, xc);
    const Cx<S>* bu = lds_u + buf * kRch * n;
    const Cx<S>* bv = lds_v + buf * kRch * n;
    if (wave_active) {
      switch (rc) {
        case 1: far_slice<S, QS, 1>(bu, bv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
        case 2: far_slice<S, QS, 2>(bu, bv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
        case 3: far_slice<S, QS, 3>(bu, bv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
        case 4: far_slice<S, QS, 4>(bu, bv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
        case 5: far_slice<S, QS, (5 < kRch ? 5 : kRch)>(bu, bv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
        case 6: far_slice<S, QS, (6 < kRch ? 6 : kRch)>(bu, bv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
        case 7: far_slice<S, QS, (7 < kRch ? 7 : kRch)>(bu, bv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
        default: far_slice<S, QS, kRch>(bu, bv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
      }
    }
    // ranks above kRch: further slices through the other buffer, synchronously
    for (int rho0 = kRch; rho0 < r; rho0 += kRch) {
      const int rc2 = min(kRch, r - rho0);
      const int ob = 1 - buf;
      __syncthreads();
      {
        const S* Uf = farf + (size_t)f * fstride;
        const S* us = Uf + (size_t)rho0 * n * 2;
        const S* vs = Uf + (size_t)max_rank * n * 2 + (size_t)rho0 * n * 2;
        Cx<S>* du = lds_u + ob * kRch * n;
        Cx<S>* dv = lds_v + ob * kRch * n;
        for (int e2 = 2 * tid; e2 < rc2 * n; e2 += 2 * blockDim.x) {
          Cx<S> a0, b0, a1, b1;
          const int col = rho0 + e2 / n;
          load_factor2<S, FT>(us, e2, col_scale(f, col), a0, b0);
          load_factor2<S, FT>(vs, e2, col_scale(f, max_rank + col), a1, b1);
          du[e2] = a0;
          du[e2 + 1] = b0;
          dv[e2] = a1;
          dv[e2 + 1] = b1;
        }
      }
      __syncthreads();
      if (wave_active) {
        const Cx<S>* cu = lds_u + ob * kRch * n;
        const Cx<S>* cv = lds_v + ob * kRch * n;
        switch (rc2) {
          case 1: far_slice<S, QS, 1>(cu, cv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
          case 2: far_slice<S, QS, 2>(cu, cv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
          case 3: far_slice<S, QS, 3>(cu, cv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
          case 4: far_slice<S, QS, 4>(cu, cv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
          case 5: far_slice<S, QS, (5 < kRch ? 5 : kRch)>(cu, cv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
          case 6: far_slice<S, QS, (6 < kRch ? 6 : kRch)>(cu, cv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
          case 7: far_slice<S, QS, (7 < kRch ? 7 : kRch)>(cu, cv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
          default: far_slice<S, QS, kRch>(cu, cv, n, offi, offj, m0, vj, xc, acc_re, acc_im); break;
        }
      }
      __syncthreads();
    }
    // the other buffer receives the next slice; one barrier separates it from
    // this displacement's readers
    if (en < nd) stash(min(kRch, rnext), 1 - buf);
    __syncthreads();
    buf = 1 - buf;
    e = en;
    f = fnext;
    r = rnext;
  }
  if (!vi) return;
  const size_t yb = (size_t)(R.unit_off + (int64_t)iy * R.Lx + ix) * n_a;
  S* o = out + ((size_t)g * total_units * n_a + yb) * 2;
#pragma unroll
  for (int k = 0; k < QS; ++k) {
    o[2 * (m0 + k)] = acc_re[k];
    o[2 * (m0 + k) + 1] = acc_im[k];
  }
}

#define R3M_FAR_WAVES(S, QS)                                                                  \
  __attribute__((amdgpu_waves_per_eu((sizeof(S) == 4 && (QS) <= 10) ? R3M_FAR_WAVES_PER_EU_F32 \
                                                                     : R3M_FAR_WAVES_PER_EU_F64)))

template <typename S, int QS, int kRch, int FT>
__global__ void __launch_bounds__(256) R3M_FAR_WAVES(S, QS)
far_kernel(FarArgs<S> A, const int* __restrict__ live) {
  if (live && *live == 0) return;  // every right-hand side has converged
  far_body<S, QS, kRch, FT>(A, blockIdx.x);
}

template <typename S, typename XT>
__global__ void __launch_bounds__(256)
reduce_groups_kernel(const RhsDev* __restrict__ rhs, const S* __restrict__ partial, int slots,
                     int64_t total_units, int n_a, XT* __restrict__ y, const int* __restrict__ live,
                     const int* __restrict__ idle) {
  if (live && *live == 0) return;  // every right-hand side has converged
  if (idle && idle[blockIdx.y]) return;
  const RhsDev R = rhs[blockIdx.y];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)R.Lx * R.Ly * n_a) return;
  const size_t e = (size_t)R.unit_off * n_a + k;
  const size_t stride = (size_t)total_units * n_a;
  // slots are added in order; loads are issued eight at a time
  S re = 0, im = 0;
  int c = 0;
  for (; c + 8 <= slots; c += 8) {
    S pr[8], pi[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const size_t p = ((size_t)(c + q) * stride + e) * 2;
      pr[q] = partial[p];
      pi[q] = partial[p + 1];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      re += pr[q];
      im += pi[q];
    }
  }
  for (; c < slots; ++c) {
    const size_t p = ((size_t)c * stride + e) * 2;
    re += partial[p];
    im += partial[p + 1];
  }
  y[2 * e] = (XT)re;
  y[2 * e + 1] = (XT)im;
}

// ---------------------------------------------------------------- near field
// on the matrix cores.
//
// Retrieval lists (built per batch and codebook, reused by every matvec):
// each (observer unit i, near displacement slot d) falls in one class
// c = (d * S + s_i) * (S + 1) + s_j, where s_j is the state of the source
// unit j = i - d, or S when j is outside the array.  Within a class every pair
// is multiplied by the same sub-block Z(d)[A(s_i), A(s_j)], so a class is a
// dense complex GEMM: Y[:, cols] = Z(d)[A(a), A(b)] X[:, cols] (eq. (3) with
// the columns of one state pair gathered).  Classes are cut into items of
// kNearCols pairs; an item's result goes to the partial slot of d, one write per
// (unit, d), so the order of pairs in a list does not change any result.

constexpr int kNearCols = 64;  // pairs per item: 4 waves x 16 MFMA columns

struct NearItem {
  int32_t cls, start, len, pad;
};
struct NearPair {
  int32_t tgt, src;  // global unit indices (src = -1: no source)
};

__global__ void __launch_bounds__(256) zero_ints_kernel(int* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Block (slot d, chunk of 256 observer units, RHS): the classes of its pairs
// are counted in LDS first, then one global atomic per class present.
// pass 0: class counts; pass 1: pair placement at offsets[c] + cursor[c] + rank.
// Dynamic LDS: 2 S (S + 1) ints.
__global__ void __launch_bounds__(256)
near_classify_kernel(const RhsDev* __restrict__ rhs, const uint8_t* __restrict__ states, int n_states, int Nx,
                     int Ny, int chunks, int* __restrict__ counts, int* __restrict__ cursor,
                     const int* __restrict__ offsets, NearPair* __restrict__ pairs, int pass) {
  extern __shared__ int cl_lds[];
  const int S = n_states, SS = S * (S + 1);
  int* local = cl_lds;       // per-class count in this block
  int* base = cl_lds + SS;   // global base of this block's pairs per class
  const RhsDev R = rhs[blockIdx.y];
  const int slot = blockIdx.x / chunks;
  const int64_t u = (int64_t)(blockIdx.x % chunks) * blockDim.x + threadIdx.x;
  for (int c = threadIdx.x; c < SS; c += blockDim.x) local[c] = 0;
  __syncthreads();
  const bool live = u < (int64_t)R.Lx * R.Ly;
  int lc = 0, rank = 0, tgt = 0, src = -1;
  if (live) {
    const int ix = (int)(u % R.Lx), iy = (int)(u / R.Lx);
    const int dx = slot % (2 * Nx + 1) - Nx, dy = slot / (2 * Nx + 1) - Ny;
    const int jx = ix - dx, jy = iy - dy;
    const bool valid = jx >= 0 && jx < R.Lx && jy >= 0 && jy < R.Ly;
    const int64_t j = (int64_t)jy * R.Lx + jx;
    const int a = min((int)states[R.state_off + u], S - 1);
    const int bs = valid ? min((int)states[R.state_off + j], S - 1) : S;
    lc = a * (S + 1) + bs;
    rank = atomicAdd(&local[lc], 1);
    tgt = (int)(R.unit_off + u);
    src = valid ? (int)(R.unit_off + j) : -1;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < SS; c += blockDim.x) {
    const int k = local[c];
    if (k > 0) base[c] = atomicAdd(pass == 0 ? &counts[slot * SS + c] : &cursor[slot * SS + c], k);
  }
  if (pass == 0) return;
  __syncthreads();
  if (live) pairs[offsets[slot * SS + lc] + base[lc] + rank] = NearPair{tgt, src};
}

// One block: exclusive scans of the class counts (pairs and items), the item
// table, and cleared cursors.
__global__ void __launch_bounds__(1024)
near_scan_kernel(const int* __restrict__ counts, int n_cls, int* __restrict__ offsets, int* __restrict__ cursor,
                 NearItem* __restrict__ items, int* __restrict__ n_items) {
  __shared__ int sp[1024], si[1024];
  const int tid = threadIdx.x;
  const int per = (n_cls + 1023) / 1024;
  const int c0 = min(n_cls, tid * per), c1 = min(n_cls, c0 + per);
  int np = 0, ni = 0;
  for (int c = c0; c < c1; ++c) {
    np += counts[c];
    ni += (counts[c] + kNearCols - 1) / kNearCols;
  }
  sp[tid] = np;
  si[tid] = ni;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int vp = tid >= o ? sp[tid - o] : 0, vi = tid >= o ? si[tid - o] : 0;
    __syncthreads();
    sp[tid] += vp;
    si[tid] += vi;
    __syncthreads();
  }
  int po = sp[tid] - np, io = si[tid] - ni;
  for (int c = c0; c < c1; ++c) {
    const int cnt = counts[c];
    offsets[c] = po;
    cursor[c] = 0;
    for (int k = 0; k * kNearCols < cnt; ++k)
      items[io++] = NearItem{c, po + k * kNearCols, min(kNearCols, cnt - k * kNearCols), 0};
    po += cnt;
  }
  if (tid == 1023) *n_items = si[1023];
}

template <typename S>
struct MfmaAcc;
template <>
struct MfmaAcc<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of the 16 x 16 result held in register r of lane l
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <>
struct MfmaAcc<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * r + (l >> 4); }
};

// One item per workgroup.  Complex GEMM in real form: row 2m + c of Y' is
// the c-th real component of row m, column 2k + c' of Z' multiplies component
// c' of x[k], so Z' holds [[Re, -Im], [Im, Re]] blocks and Y' = Z' X' is a
// real (2 NA) x (2 NA) x 16 product per wave on 16x16x4 MFMA tiles (lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]).  Dynamic LDS: Z' as
// [2 NA][2 NA + 1] reals, then the gathered columns [kNearCols][2 NA + 1].
template <typename S>
struct NearArgs {
  const NearItem* items;
  const int* n_items;
  const NearPair* pairs;
  const S* near;
  int n, n_states;
  const S* x;
  S* out;  // near slot 0
  int64_t total_units;
};

// near-field item wg (see near_mfma_kernel)
template <typename S, int NA>
__device__ __forceinline__ void near_body(const NearArgs<S>& A, int wg) {
  const NearItem* __restrict__ items = A.items;
  const NearPair* __restrict__ pairs = A.pairs;
  const S* __restrict__ near = A.near;
  const int n = A.n, n_states = A.n_states;
  const S* __restrict__ x = A.x;
  S* __restrict__ out = A.out;
  const int64_t total_units = A.total_units;
  constexpr int K2 = 2 * NA, MT = K2 / 16, KT = K2 / 4, XS = K2 + 1;
  constexpr int KC = 4;  // K steps whose operands are read before their MFMAs
  static_assert(KT % KC == 0, "K steps per chunk");
  extern __shared__ unsigned char smem_raw[];
  S* a_lds = reinterpret_cast<S*>(smem_raw);  // Z' [K2][XS]
  S* x_lds = a_lds + (size_t)K2 * XS;         // X' [kNearCols][XS]
  __shared__ int tgt_s[kNearCols], src_s[kNearCols];
  if (wg >= *A.n_items) return;
  const NearItem item = items[wg];
  const int S1 = n_states + 1;
  const int bsrc = item.cls % S1, a = (item.cls / S1) % n_states, slot = item.cls / (S1 * n_states);
  const int tid = threadIdx.x;
  if (tid < kNearCols) {
    const NearPair pr = tid < item.len ? pairs[item.start + tid] : NearPair{-1, -1};
    tgt_s[tid] = pr.tgt;
    src_s[tid] = pr.src;
  }
  __syncthreads();
  S* dst = out + (size_t)slot * total_units * K2;
  if (bsrc == n_states) {  // no source at this displacement: the slot holds zero
    for (int e = tid; e < item.len * K2; e += blockDim.x) dst[(size_t)tgt_s[e / K2] * K2 + e % K2] = S(0);
    return;
  }
  // sub-block and gathered columns: every load is issued before the LDS stores
  const Cx<S>* zb = reinterpret_cast<const Cx<S>*>(near) + (size_t)slot * n * n;
  constexpr int kZ = (NA * NA + 255) / 256, kX = kNearCols * NA / 256;
  Cx<S> zv[kZ], xv[kX];
#pragma unroll
  for (int q = 0; q < kZ; ++q) {
    const int e = tid + q * 256;
    if (e < NA * NA) zv[q] = zb[(size_t)(a * NA + e / NA) * n + bsrc * NA + e % NA];
  }
#pragma unroll
  for (int q = 0; q < kX; ++q) {
    const int e = tid + q * 256;
    const int c = e / NA, src = src_s[c];
    xv[q] = src >= 0 ? reinterpret_cast<const Cx<S>*>(x)[(size_t)src * NA + e % NA] : Cx<S>{0, 0};
  }
#pragma unroll
  for (int q = 0; q < kZ; ++q) {
    const int e = tid + q * 256;
    if (e < NA * NA) {
      const int r = 2 * (e / NA), c = 2 * (e % NA);
      a_lds[r * XS + c] = zv[q].re;
      a_lds[r * XS + c + 1] = -zv[q].im;
      a_lds[(r + 1) * XS + c] = zv[q].im;
      a_lds[(r + 1) * XS + c + 1] = zv[q].re;
    }
  }
#pragma unroll
  for (int q = 0; q < kX; ++q) {
    const int e = tid + q * 256;
    x_lds[(e / NA) * XS + 2 * (e % NA)] = xv[q].re;
    x_lds[(e / NA) * XS + 2 * (e % NA) + 1] = xv[q].im;
  }
  __syncthreads();
  const int wave = tid >> 6, l = tid & 63;
  if (wave * 16 >= item.len) return;
  const int col = wave * 16 + (l & 15), kq = l >> 4, mr = l & 15;
  typename MfmaAcc<S>::v4 acc[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt] = typename MfmaAcc<S>::v4{0, 0, 0, 0};
  for (int k0 = 0; k0 < KT; k0 += KC) {
    S bv[KC], av[KC][MT];
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      const int kp = 4 * (k0 + q) + kq;
      bv[q] = x_lds[col * XS + kp];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) av[q][mt] = a_lds[(16 * mt + mr) * XS + kp];
    }
#pragma unroll
    for (int q = 0; q < KC; ++q)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = MfmaAcc<S>::mma(av[q][mt], bv[q], acc[mt]);
  }
  const int tgt = tgt_s[col];
  if (tgt < 0) return;
  S* o = dst + (size_t)tgt * K2;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) o[16 * mt + MfmaAcc<S>::row(l, r)] = acc[mt][r];
}

template <typename S, int NA>
__global__ void __launch_bounds__(256) near_mfma_kernel(NearArgs<S> A, const int* __restrict__ live) {
  if (live && *live == 0) return;  // every right-hand side has converged
  near_body<S, NA>(A, blockIdx.x);
}

// Far and near field in one launch: the first near_wgs workgroups take the
// near items (matrix cores), the rest the far tiles (vector units), so the
// two kinds of work share the chip.  near_wgs is a multiple of 8, which keeps
// the far workgroups' XCD placement.
template <typename S, int QS, int kRch, int FT, int NA>
__global__ void __launch_bounds__(256) R3M_FAR_WAVES(S, QS)
far_near_kernel(FarArgs<S> F, NearArgs<S> N, int near_wgs, const int* __restrict__ live) {
  if (live && *live == 0) return;  // every right-hand side has converged
  if ((int)blockIdx.x < near_wgs)
    near_body<S, NA>(N, blockIdx.x);
  else
    far_body<S, QS, kRch, FT>(F, blockIdx.x - near_wgs);
}

// ----------------------------------------------------------------- far field
// on the matrix cores.
//
// Work item: a tile of observer units (8 wide, th tall) of one codebook with
// the right-hand sides that share the codebook (a group of up to kGroupRhs;
// th shrinks as the group grows), and the rows dy = g, g + G, ... of the
// tile's displacement rectangle.  Per displacement d the low-rank block
// (Sec. II-B) acts on column (observer slot i, right-hand side) in two steps,
//     t = V(d)[A(s_j), :]^H x_j   (j = i - d),     y_i += U(d)[A(s_i), :] t,
// both evaluated as real-form GEMMs on 16x16x4 FP32 MFMA tiles.  A row of
// displacements is swept in runs of kRun consecutive dx.  The sources of a
// run form a window of kRing columns of units that slides by kRun columns
// from run to run; it is held in an LDS ring, so each source's x is read
// once per displacement row rather than once per displacement.
//  - First product: rows are the run's (displacement, rank, re/im) stacked,
//    K is (basis function, re/im), columns are the window's (source,
//    right-hand side) pairs grouped by source state (one row block A(b) of V
//    per column tile).
//  - Second product: rows are (basis function, re/im) of the observer state,
//    K is the run's (displacement, rank, re/im), columns are the tile's
//    (observer, right-hand side) pairs grouped by observer state (fixed for
//    the tile); the accumulators stay in registers for the whole work item.
// The run's ranks are taken KC / 2 at a time (a sub-chunk); t passes between
// the two products through LDS.  A work item writes its own partial slot, one
// write per (unit, right-hand side), so the sum over the G slots
// (reduce_groups_kernel) has a fixed order.
constexpr int kRun = 4;                    // displacements per run (consecutive dx)
constexpr int kRing = 8 + kRun - 1;        // source columns of a run's window
constexpr int kFNA = 40;                   // active RWG per unit on this path
constexpr int kXS = kFNA + 2;              // complex per window row in LDS (padded: rows 8 banks apart)
constexpr int kWinRows = 8;                // window rows per source column: th rows x (8 / th) rhs slots
constexpr int kWinCols = kRing * kWinRows;
constexpr int kP1Tiles = (kWinCols + 15 * 4 + 15) / 16;  // column tiles of the first product
constexpr int kP2Tiles = (64 + 15 * 4 + 15) / 16;        // ... of the second product
constexpr int kStLds = 4096;               // codebooks up to this many units keep their states in LDS

struct FarMArgs {
  const RhsDev* rhs;
  const GroupDev* groups;
  const TileDev* gtiles;  // TileDev.b: group
  int n_gtiles, n_dgroups;
  const uint8_t* states;
  const float* farf;      // factors (store format)
  const int* ranks;
  const float* fscale;    // F16X2 column scales, else NULL
  int max_rank, Dx, Dy, nr;
  const float* x;         // vectors in FP32
  float* out;             // partial slot 0
  int64_t total_units;
  const int* idle;        // per right-hand side (nullable)
};

// dynamic LDS of far_mfma_body: the x ring, the factor columns of a
// sub-chunk (rows padded by two), the t buffer and the codebook states
template <int KC, int NS>
__host__ __device__ constexpr size_t far_mfma_lds_bytes() {
  return (size_t)kWinCols * kXS * 8 + 2 * (size_t)(KC / 2) * (NS * kFNA + 2) * 8 +
         (size_t)kP1Tiles * 16 * (KC + 4) * 4 + kStLds;
}

template <int FT, int CTW, int KC, int NS>
__device__ __forceinline__ void far_mfma_body(const FarMArgs& A, int wg) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  constexpr int KR = KC / 2, TS = KC + 4, n = NS * kFNA, NP = n + 2, MT1 = KC / 16;
  extern __shared__ unsigned char smem_raw[];
  __shared__ int16_t p2tab[kP2Tiles * 16];   // second product: column -> slot | q << 8, or -1
  __shared__ uint8_t ct2_state[kP2Tiles];
  __shared__ int16_t p1tab[kP1Tiles * 16];   // first product: column -> window row, or -1
  __shared__ int16_t p1col[kWinCols];        // window position (slot th + wy) -> first column, or -1
  __shared__ uint8_t ct1_state[kP1Tiles];
  __shared__ int nct1_s, nct2_s;
  __shared__ int64_t g_uoff[kGroupRhs];

  int ti, g;
  if (!decode_wg(wg, A.n_gtiles, A.n_dgroups, ti, g)) return;
  const TileDev tl = A.gtiles[ti];
  const GroupDev* __restrict__ G = A.groups + tl.b;  // read in place (indexed at run time)
  const int nrhs = G->n, th = G->th;
  const int lth = th == 8 ? 3 : th == 4 ? 2 : 1;      // th = 8 / (rhs slots per row)
  const int lq = 3 - lth;                              // log2 of the rhs slots per window row
  if (A.idle) {
    bool live = false;
    for (int q = 0; q < nrhs; ++q) live |= A.idle[G->rhs[q]] == 0;
    if (!live) return;  // uniform over the workgroup
  }
  const RhsDev R = A.rhs[G->rhs[0]];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nl = lane & 15, kk = lane >> 4;
  Cx<float>* Xr = reinterpret_cast<Cx<float>*>(smem_raw);  // [ring slot][kWinRows][kXS]: the window
  Cx<float>* Uc = Xr + kWinCols * kXS;                      // [KR][NP]
  Cx<float>* Vc = Uc + KR * NP;                             // [KR][NP]
  float* Tb = reinterpret_cast<float*>(Vc + KR * NP);       // [first-product column][TS]
  uint8_t* sts = reinterpret_cast<uint8_t*>(Tb + kP1Tiles * 16 * TS);
  const int64_t units = (int64_t)R.Lx * R.Ly;
  const bool st_lds = units <= kStLds;
  if (st_lds)
    for (int64_t u = tid; u < units; u += blockDim.x) sts[u] = A.states[R.state_off + u];
  __syncthreads();
  // state of unit (jx, jy), or NS outside the array
  auto state_at = [&](int jx, int jy) -> int {
    if (jx < 0 || jx >= R.Lx || jy < 0 || jy >= R.Ly) return NS;
    const int64_t u = (int64_t)jy * R.Lx + jx;
    return min((int)(st_lds ? sts[u] : A.states[R.state_off + u]), NS - 1);
  };
  // ring slot of source column jx (jx > -kRing * 64)
  auto ring = [](int jx) { return (int)((unsigned)(jx + kRing * 64) % (unsigned)kRing); };

  // wave 0: the tile's (observer, rhs) columns grouped by observer state
  if (wave == 0) {
    const int sx = lane & 7, sy = lane >> 3;
    const int st = lane < 8 * th ? state_at(tl.tx + sx, tl.ty + sy) : NS;
    int base = 0, nt = 0;
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      const uint64_t m = __ballot(st == a);
      const int cnt = __popcll(m);
      const int rank =
          __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
      if (st == a)
        for (int q = 0; q < nrhs; ++q) p2tab[base + rank * nrhs + q] = (int16_t)(lane | q << 8);
      const int used = cnt * nrhs, tiles = (used + 15) >> 4;
      for (int c = used + lane; c < tiles * 16; c += 64) p2tab[base + c] = -1;
      if (lane < tiles) ct2_state[nt + lane] = (uint8_t)a;
      base += tiles * 16;
      nt += tiles;
    }
    if (lane == 0) nct2_s = nt;
    if (lane < nrhs) g_uoff[lane] = A.rhs[G->rhs[lane]].unit_off;
  }

  // displacements keeping a source of the tile in the array: a rectangle
  const int bx_hi = min(tl.tx + 8, R.Lx) - 1, by_hi = min(tl.ty + th, R.Ly) - 1;
  const int dx_lo = tl.tx - (R.Lx - 1), dy_lo = tl.ty - (R.Ly - 1);
  const int wdy = by_hi - dy_lo + 1;
  const int fstride = 2 * A.max_rank * n * 2;  // floats per far block
  auto col_scale = [&](int f, int col) -> float {
    return FT == R3M_F16X2 ? A.fscale[(size_t)f * 2 * A.max_rank + col] : 1.0f;
  };

  v4 acc[CTW][5];
#pragma unroll
  for (int q = 0; q < CTW; ++q)
#pragma unroll
    for (int mt = 0; mt < 5; ++mt) acc[q][mt] = v4{0, 0, 0, 0};
  __syncthreads();
  const int nct2 = nct2_s;
  // this lane's second-product columns: observer slot and rhs of each tile it serves
  int o_sx[CTW], o_sy[CTW], o_q[CTW];
  bool o_ok[CTW];
#pragma unroll
  for (int qi = 0; qi < CTW; ++qi) {
    const int ct2 = wave + 4 * qi;
    const int ent = ct2 < nct2 ? p2tab[ct2 * 16 + nl] : -1;
    o_ok[qi] = ent >= 0;
    o_sx[qi] = ent & 7;
    o_sy[qi] = (ent & 0xff) >> 3;
    o_q[qi] = ent >> 8;
  }

  // A step is one sub-chunk (KR ranks) of one run (kRun consecutive dx of a
  // displacement row).  Steps are software-pipelined: while a step computes,
  // the next step's window columns and factor columns are fetched into
  // registers, then stored to LDS where the current step no longer reads
  // them, so each step needs two barriers.
  struct Run {
    int dy, dxa, nrun, jlo, jhi, new_hi, jy0, f0, f1, f2, f3, p1, p2, p3, nrk;
  };
  auto make_run = [&](int row, int dxa) {
    Run r;
    r.dy = dy_lo + row;
    r.dxa = dxa;
    r.nrun = min(kRun, bx_hi - dxa + 1);
    r.jhi = tl.tx - dxa + 7;
    r.jlo = tl.tx - dxa - r.nrun + 1;
    r.new_hi = dxa == dx_lo ? r.jhi : tl.tx - dxa;  // columns the previous run of the row did not hold
    r.jy0 = tl.ty - r.dy;
    r.f0 = r.f1 = r.f2 = r.f3 = 0;
    auto blk = [&](int dl, int& f) {
      const int dx = dxa + dl;
      if (dl < r.nrun && ((dx < 0 ? -dx : dx) > A.nr || (r.dy < 0 ? -r.dy : r.dy) > A.nr)) {
        f = far_index(dx, r.dy, A.Dx, A.Dy, A.nr);
        return min(A.ranks[f], A.max_rank);
      }
      return 0;
    };
    r.p1 = blk(0, r.f0);
    r.p2 = r.p1 + blk(1, r.f1);
    r.p3 = r.p2 + blk(2, r.f2);
    r.nrk = r.p3 + blk(3, r.f3);
    return r;
  };
  static_assert(kRun == 4, "the run's blocks are unrolled for four displacements");
  // run rank rho -> displacement dl of the run
  auto rank_dl = [](const Run& r, int rho) {
    return (rho >= r.p1 ? 1 : 0) + (rho >= r.p2 ? 1 : 0) + (rho >= r.p3 ? 1 : 0);
  };
  // factor columns of run ranks [k0, k0 + KR): fetch (to registers), then store
  constexpr int kPairIt = (KR * n / 2 + 255) / 256;
  Cx<float> fu[2 * kPairIt], fv[2 * kPairIt];
  auto fetch_f = [&](const Run& r, int k0) {
    const int nk = min(KR, r.nrk - k0);
#pragma unroll
    for (int it = 0; it < kPairIt; ++it) {
      const int e2 = 2 * (tid + it * 256);
      if (e2 < nk * n) {
        const int rl = e2 / n, rw = e2 - rl * n;
        const int rho = k0 + rl, dl = rank_dl(r, rho);
        const int f = dl == 0 ? r.f0 : dl == 1 ? r.f1 : dl == 2 ? r.f2 : r.f3;
        const int rr = rho - (dl == 0 ? 0 : dl == 1 ? r.p1 : dl == 2 ? r.p2 : r.p3);
        const float* Uf = A.farf + (size_t)f * fstride;
        load_factor2<float, FT>(Uf + (size_t)rr * n * 2, rw, col_scale(f, rr), fu[2 * it], fu[2 * it + 1]);
        load_factor2<float, FT>(Uf + (size_t)(A.max_rank + rr) * n * 2, rw, col_scale(f, A.max_rank + rr),
                                fv[2 * it], fv[2 * it + 1]);
      }
    }
  };
  auto store_f = [&](const Run& r, int k0, bool u, bool v) {
    const int nk = min(KR, r.nrk - k0);
#pragma unroll
    for (int it = 0; it < kPairIt; ++it) {
      const int e2 = 2 * (tid + it * 256);
      if (e2 < nk * n) {
        const int rl = e2 / n, rw = e2 - rl * n;
        if (u) {
          Uc[rl * NP + rw] = fu[2 * it];
          Uc[rl * NP + rw + 1] = fu[2 * it + 1];
        }
        if (v) {
          Vc[rl * NP + rw] = fv[2 * it];
          Vc[rl * NP + rw + 1] = fv[2 * it + 1];
        }
      }
    }
  };
  // new window columns of a run (x of every right-hand side), window row
  // wr = wy << lq | q: fetch (to registers), then store into the ring
  constexpr int kPer = kWinRows * (kFNA / 2);            // float4 per window column
  constexpr int kColIt = (kRun * kPer + 255) / 256;       // float4 per thread, kRun columns
  v4 fx[kColIt];
  // columns [r.jlo + c0, r.jlo + c0 + kRun) of the new ones (c0 = 0 for a run
  // inside a row, 0, 4, 8 for the first run of a row)
  auto fetch_x = [&](const Run& r, int c0) {
    const int total = min(kRun, r.new_hi - r.jlo + 1 - c0) * kPer;
#pragma unroll
    for (int it = 0; it < kColIt; ++it) {
      const int e4 = tid + it * 256;
      fx[it] = v4{0, 0, 0, 0};
      if (e4 < total) {
        const int c = e4 / kPer, rem = e4 - c * kPer;
        const int wr = rem / (kFNA / 2), part = rem - wr * (kFNA / 2);
        const int wy = wr >> lq, q = wr & ((1 << lq) - 1);
        const int jx = r.jlo + c0 + c, jy = r.jy0 + wy;
        if (q < nrhs && jx >= 0 && jx < R.Lx && jy >= 0 && jy < R.Ly)
          fx[it] = *reinterpret_cast<const v4*>(A.x + ((size_t)(g_uoff[q] + (int64_t)jy * R.Lx + jx) * kFNA) * 2 +
                                                4 * part);
      }
    }
  };
  auto store_x = [&](const Run& r, int c0) {
    const int total = min(kRun, r.new_hi - r.jlo + 1 - c0) * kPer;
#pragma unroll
    for (int it = 0; it < kColIt; ++it) {
      const int e4 = tid + it * 256;
      if (e4 < total) {
        const int c = e4 / kPer, rem = e4 - c * kPer;
        const int wr = rem / (kFNA / 2), part = rem - wr * (kFNA / 2);
        *reinterpret_cast<v4*>(Xr + (ring(r.jlo + c0 + c) * kWinRows + wr) * kXS + 2 * part) = fx[it];
      }
    }
  };
  // a whole window (first run of a row): the columns past the first kRun
  // synchronously, the first kRun through the pipelined path
  auto load_rest = [&](const Run& r) {
    for (int c0 = kRun; c0 < r.new_hi - r.jlo + 1; c0 += kRun) {
      fetch_x(r, c0);
      store_x(r, c0);
    }
  };
  // wave 0: the window's (source, rhs) columns grouped by source state
  auto sort_window = [&](const Run& r) {
    int base = 0, nt = 0;
    int st[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int pos = lane + 64 * h;  // ring slot pos >> lth, row pos & (th - 1)
      st[h] = NS;
      if (pos < kRing * th) {
        const int sl = pos >> lth, wy = pos & (th - 1);
        const int jx = r.jlo + ring(sl - r.jlo);
        if (jx <= r.jhi) st[h] = state_at(jx, r.jy0 + wy);
        p1col[pos] = -1;
      }
    }
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      const uint64_t m0 = __ballot(st[0] == a), m1 = __ballot(st[1] == a);
      const int c0 = __popcll(m0), cnt = c0 + __popcll(m1);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint64_t m = h ? m1 : m0;
        const int rank = (h ? c0 : 0) + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
        if (st[h] == a) {
          const int pos = lane + 64 * h;
          const int wrow = (pos >> lth) * kWinRows + ((pos & (th - 1)) << lq);  // window row of rhs 0
          p1col[pos] = (int16_t)(base + rank * nrhs);
          for (int q = 0; q < nrhs; ++q) p1tab[base + rank * nrhs + q] = (int16_t)(wrow + q);
        }
      }
      const int used = cnt * nrhs, tiles = (used + 15) >> 4;
      for (int c = used + lane; c < tiles * 16; c += 64) p1tab[base + c] = -1;
      if (lane < tiles) ct1_state[nt + lane] = (uint8_t)a;
      base += tiles * 16;
      nt += tiles;
    }
    if (lane == 0) nct1_s = nt;
  };
  // first-product column of this lane's observers' sources for each dl of
  // a run, as four 16-bit fields (dl 0, 1 in pk_lo; 2, 3 in pk_hi)
  uint32_t pk_lo[CTW], pk_hi[CTW];
  auto make_pk = [&](const Run& r) {
#pragma unroll
    for (int qi = 0; qi < CTW; ++qi) {
      uint32_t f4[kRun];
#pragma unroll
      for (int dl = 0; dl < kRun; ++dl) {
        int c1 = -1;
        if (o_ok[qi] && dl < r.nrun) c1 = p1col[(ring(tl.tx + o_sx[qi] - (r.dxa + dl)) << lth) + o_sy[qi]];
        f4[dl] = (uint32_t)(c1 < 0 ? 0xffff : c1 + o_q[qi]) & 0xffffu;
      }
      pk_lo[qi] = f4[0] | f4[1] << 16;
      pk_hi[qi] = f4[2] | f4[3] << 16;
    }
  };

  if (g < wdy) {
    Run ru = make_run(g, dx_lo);
    int row = g, k0 = 0;
    fetch_x(ru, 0);
    if (ru.nrk > 0) fetch_f(ru, 0);
    store_x(ru, 0);
    load_rest(ru);
    if (ru.nrk > 0) store_f(ru, 0, true, true);
    if (wave == 0) sort_window(ru);
    __syncthreads();
    make_pk(ru);
    for (;;) {
      const int Kc = ru.nrk > k0 ? 2 * min(KR, ru.nrk - k0) : 0;
      // the next step
      Run nx = ru;
      int nrow = row, nk0 = k0 + KR;
      bool newrun = false, done = false;
      if (nk0 >= ru.nrk) {
        newrun = true;
        nk0 = 0;
        int ndxa = ru.dxa + kRun;
        if (ndxa > bx_hi) {
          nrow += A.n_dgroups;
          ndxa = dx_lo;
        }
        if (nrow >= wdy)
          done = true;
        else
          nx = make_run(nrow, ndxa);
      }
      const int nct1 = nct1_s;
      // (b) first product: t = V^H x over (row tile, source-state column tile)
      for (int w = wave; w < MT1 * nct1 && Kc > 0; w += 4) {
        const int ct = w / MT1, mt = w - ct * MT1;
        const int b = ct1_state[ct];
        const int m = 16 * mt + nl, rl = m >> 1, c = m & 1;
        float a0[10], a1[10];
        if (m < Kc) {
          const float* vr = reinterpret_cast<const float*>(Vc + rl * NP + b * kFNA + 10 * kk);
#pragma unroll
          for (int k2 = 0; k2 < 10; k2 += 2) {
            Cx<float> p, q2;
            load2<float>(vr, k2, p, q2);
            a0[k2] = c ? -p.im : p.re;
            a1[k2] = c ? p.re : p.im;
            a0[k2 + 1] = c ? -q2.im : q2.re;
            a1[k2 + 1] = c ? q2.re : q2.im;
          }
        } else {
#pragma unroll
          for (int k2 = 0; k2 < 10; ++k2) a0[k2] = a1[k2] = 0.f;
        }
        const int ent = p1tab[ct * 16 + nl];
        float xr[10], xi[10];
        if (ent >= 0) {
          const float* xp = reinterpret_cast<const float*>(Xr + ent * kXS + 10 * kk);
#pragma unroll
          for (int k2 = 0; k2 < 10; k2 += 2) {
            Cx<float> p, q2;
            load2<float>(xp, k2, p, q2);
            xr[k2] = p.re;
            xi[k2] = p.im;
            xr[k2 + 1] = q2.re;
            xi[k2 + 1] = q2.im;
          }
        } else {
#pragma unroll
          for (int k2 = 0; k2 < 10; ++k2) xr[k2] = xi[k2] = 0.f;
        }
        v4 cc = v4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 20; ++s)
          cc = __builtin_amdgcn_mfma_f32_16x16x4f32((s & 1) ? a1[s >> 1] : a0[s >> 1],
                                                    (s & 1) ? xi[s >> 1] : xr[s >> 1], cc, 0, 0, 0);
        if (ent >= 0) {
          float* tc = Tb + (ct * 16 + nl) * TS;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int mr = 16 * mt + 4 * kk + i;
            if (mr < Kc) tc[mr] = cc[i];
          }
        }
      }
      // the next step's data into registers
      if (!done) {
        if (newrun) fetch_x(nx, 0);
        if (nx.nrk > nk0) fetch_f(nx, nk0);
      }
      __syncthreads();
      // (c) second product: y += U t over the step's stacked ranks
      if (Kc > 0) {
        const int S2 = (Kc + 3) >> 2;
        float bt[CTW][8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int k = kk * S2 + s;
          const int dl = rank_dl(ru, k0 + (k >> 1));  // displacement of the run of K entry k
          const int sh = (dl & 1) * 16;
#pragma unroll
          for (int qi = 0; qi < CTW; ++qi) {
            const int c1 = (int)(((dl < 2 ? pk_lo[qi] : pk_hi[qi]) >> sh) & 0xffffu);
            bt[qi][s] = (s < S2 && k < Kc && c1 != 0xffff) ? Tb[c1 * TS + k] : 0.f;
          }
        }
#pragma unroll
        for (int mt = 0; mt < 5; ++mt) {
          const int e = 8 * mt + (nl >> 1), c = nl & 1;
          int cur = -1;
          float au[8];
#pragma unroll
          for (int qi = 0; qi < CTW; ++qi) {
            const int ct2 = wave + 4 * qi;
            if (ct2 >= nct2) break;
            const int a = ct2_state[ct2];
            if (a != cur) {
              cur = a;
#pragma unroll
              for (int s = 0; s < 8; ++s) {
                const int k = kk * S2 + s;
                float v = 0.f;
                if (s < S2 && k < Kc) {
                  const Cx<float> u = Uc[(k >> 1) * NP + a * kFNA + e];
                  v = (k & 1) ? (c ? u.re : -u.im) : (c ? u.im : u.re);
                }
                au[s] = v;
              }
            }
#pragma unroll
            for (int s = 0; s < 8; ++s)
              if (s < S2) acc[qi][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(au[s], bt[qi][s], acc[qi][mt], 0, 0, 0);
          }
        }
      }
      // the next step's window and V columns where this step no longer reads
      if (!done) {
        if (newrun) {
          store_x(nx, 0);
          if (nx.dxa == dx_lo) load_rest(nx);  // a new row: the rest of its first window
          if (wave == 0) sort_window(nx);
        }
        if (nx.nrk > nk0) store_f(nx, nk0, false, true);
      }
      __syncthreads();
      if (done) break;
      if (nx.nrk > nk0) store_f(nx, nk0, true, false);  // read by the next step's second product only
      if (newrun) make_pk(nx);
      ru = nx;
      row = nrow;
      k0 = nk0;
    }
  }
  // the work item's partial slot
#pragma unroll
  for (int qi = 0; qi < CTW; ++qi) {
    if (!o_ok[qi]) continue;
    const int64_t unit = (int64_t)(tl.ty + o_sy[qi]) * R.Lx + tl.tx + o_sx[qi];
    float* o = A.out + ((size_t)g * A.total_units + g_uoff[o_q[qi]] + unit) * kFNA * 2;
#pragma unroll
    for (int mt = 0; mt < 5; ++mt) *reinterpret_cast<v4*>(o + 2 * (8 * mt + 2 * kk)) = acc[qi][mt];
  }
}

template <int FT, int CTW, int KC, int NS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
far_mfma_kernel(FarMArgs A, const int* __restrict__ live) {
  if (live && *live == 0) return;  // every right-hand side has converged
  far_mfma_body<FT, CTW, KC, NS>(A, blockIdx.x);
}

// near items (matrix cores, first near_wgs workgroups) beside the far items
template <int FT, int CTW, int KC, int NS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
far_mfma_near_kernel(FarMArgs F, NearArgs<float> N, int near_wgs, const int* __restrict__ live) {
  if (live && *live == 0) return;  // every right-hand side has converged
  if ((int)blockIdx.x < near_wgs)
    near_body<float, 40>(N, blockIdx.x);
  else
    far_mfma_body<FT, CTW, KC, NS>(F, blockIdx.x - near_wgs);
}

template <typename S, typename XT>
__global__ void __launch_bounds__(256)
convert_flat_kernel(const RhsDev* __restrict__ rhs, int n_a, const XT* __restrict__ x, S* __restrict__ xs) {
  const RhsDev R = rhs[blockIdx.y];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)R.Lx * R.Ly * n_a) return;
  const size_t e = (size_t)R.unit_off * n_a + k;
  xs[2 * e] = (S)x[2 * e];
  xs[2 * e + 1] = (S)x[2 * e + 1];
}

}  // namespace

// default displacement groups per 8x8 block: about 1024 workgroups per launch
int choose_chunks(const BatchDesc& bd, int max_chunks) {
  int want = (int)std::max<int64_t>(1, (1024 + bd.n_tiles - 1) / std::max(1, bd.n_tiles));
  return std::max(1, std::min(want, max_chunks));
}

// largest group count the autotuner may try (the workspace is sized for it)
int max_groups(const BatchDesc& bd) { return std::min(128, 4 * choose_chunks(bd, 64)); }

static bool store_has_far(const r3m_store* Z) { return Z->near_radius < std::max(Z->Dx, Z->Dy); }

static int near_count(const r3m_store* Z) {
  const int Nx = std::min(Z->near_radius, Z->Dx), Ny = std::min(Z->near_radius, Z->Dy);
  return (2 * Nx + 1) * (2 * Ny + 1);
}

// near field on the matrix cores (one partial slot per near displacement)
// unless the near set is large (an all-dense store), where the LDS-slab kernel
// groups displacements
static bool near_on_mfma(const r3m_store* Z) {
  if (store_is_spectral(Z)) return false;
  const int n_a = Z->n / Z->n_states;
  const size_t es = Z->near_dtype == R3M_C128 ? 8 : 4;
  return near_count(Z) <= 128 && ((size_t)2 * n_a + kNearCols) * (2 * n_a + 1) * es <= 96 * 1024;
}

// near partial slots: one per displacement on the matrix-core path; otherwise
// one displacement per workgroup for small batches, fewer groups (longer
// loops) when the batch already fills the chip
static int near_groups(const r3m_store* Z, const BatchDesc& bd) {
  if (near_on_mfma(Z)) return near_count(Z);
  const int want = (int)std::max<int64_t>(1, (2048 + bd.n_tiles - 1) / std::max(1, bd.n_tiles));
  return std::max(1, std::min({near_count(Z), 128, want}));
}

// retrieval lists of the near field (matrix-core path): counts, offsets and
// cursors per class, the item count, the item table and the pair table
struct NearLists {
  int* counts = nullptr;
  int* offsets = nullptr;
  int* cursor = nullptr;
  int* n_items = nullptr;
  NearItem* items = nullptr;
  NearPair* pairs = nullptr;
  int n_cls = 0;
  int64_t max_items = 0;
  size_t bytes = 0;
};

static NearLists near_lists(char* base, int n_near, int S, const BatchDesc& bd) {
  NearLists L;
  const int64_t pairs = (int64_t)n_near * bd.total_units;
  L.n_cls = n_near * S * (S + 1);
  L.max_items = (pairs + kNearCols - 1) / kNearCols + L.n_cls;
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o = (o + b + 255) / 256 * 256;
    return base ? (void*)(base + at) : nullptr;
  };
  L.counts = (int*)take((size_t)L.n_cls * 4);
  L.offsets = (int*)take((size_t)L.n_cls * 4);
  L.cursor = (int*)take((size_t)L.n_cls * 4);
  L.n_items = (int*)take(4);
  L.items = (NearItem*)take((size_t)L.max_items * sizeof(NearItem));
  L.pairs = (NearPair*)take((size_t)pairs * sizeof(NearPair));
  L.bytes = o;
  return L;
}

static NearLists near_lists(char* base, const r3m_store* Z, const BatchDesc& bd) {
  return near_on_mfma(Z) ? near_lists(base, near_count(Z), Z->n_states, bd) : NearLists{};
}

size_t near_lists_bytes(const r3m_store* Z, const BatchDesc& bd) { return near_lists(nullptr, Z, bd).bytes; }
// the most any store with n_states states can need on this batch
size_t near_lists_bytes_bound(int n_states, const BatchDesc& bd) {
  return near_lists(nullptr, 128, n_states, bd).bytes;
}

// builds the near retrieval lists of (batch, codebook states) at lists_dev
void build_near_lists(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, void* lists_dev,
                      hipStream_t stream) {
  if (!near_on_mfma(Z)) return;
  NearLists L = near_lists((char*)lists_dev, Z, bd);
  const int Nx = std::min(Z->near_radius, Z->Dx), Ny = std::min(Z->near_radius, Z->Dy);
  hipLaunchKernelGGL(zero_ints_kernel, dim3(ceil_div((size_t)L.n_cls, 256)), dim3(256), 0, stream, L.counts,
                     L.n_cls);
  const int chunks = (int)ceil_div((size_t)bd.max_units, 256);
  const dim3 grid((unsigned)(chunks * near_count(Z)), bd.B);
  const size_t lds = (size_t)2 * Z->n_states * (Z->n_states + 1) * sizeof(int);
  hipLaunchKernelGGL(near_classify_kernel, grid, dim3(256), lds, stream, bd.rhs, states, Z->n_states, Nx, Ny,
                     chunks, L.counts, L.cursor, (const int*)L.offsets, L.pairs, 0);
  hipLaunchKernelGGL(near_scan_kernel, dim3(1), dim3(1024), 0, stream, (const int*)L.counts, L.n_cls, L.offsets,
                     L.cursor, L.items, L.n_items);
  hipLaunchKernelGGL(near_classify_kernel, grid, dim3(256), lds, stream, bd.rhs, states, Z->n_states, Nx, Ny,
                     chunks, L.counts, L.cursor, (const int*)L.offsets, L.pairs, 1);
  R3M_CHECK_HIP(hipGetLastError());
}

// workspace: partial sums [far groups + near groups][units][n_a] in the store
// precision, a copy of x in the store precision when the vectors are wider,
// then the near retrieval lists
size_t partials_and_x_bytes(const BatchDesc& bd, const r3m_store* Z, int chunks) {
  if (store_is_spectral(Z)) return spectral_work_bytes(bd, Z);
  const size_t es = Z->near_dtype == R3M_C128 ? 16 : 8;
  const int n_a = Z->n / Z->n_states;
  const size_t vec = (size_t)bd.total_units * n_a * es;
  const int slots = (store_has_far(Z) ? std::max(chunks, 1) : 0) + near_groups(Z, bd);
  return ((size_t)slots * vec + (Z->near_dtype == R3M_C128 ? 0 : vec) + 255) / 256 * 256;
}
size_t matvec_partial_bytes(const BatchDesc& bd, const r3m_store* Z, int chunks) {
  return partials_and_x_bytes(bd, Z, chunks) + near_lists_bytes(Z, bd) + 256;
}
// the lists of a workspace sized with max_groups(bd)
void* workspace_lists(void* work, const BatchDesc& bd, const r3m_store* Z) {
  return (char*)work + partials_and_x_bytes(bd, Z, max_groups(bd));
}

void validate_store(const r3m_store* Z) {
  R3M_REQUIRE(Z, R3M_ERR_INVALID_ARG, "store is NULL");
  R3M_REQUIRE(Z->n_common >= 0 && Z->n_common < Z->n, R3M_ERR_INVALID_ARG, "n_common out of range");
  R3M_REQUIRE(Z->n > 0 && Z->n_states >= 1 && (Z->n - Z->n_common) % Z->n_states == 0, R3M_ERR_INVALID_ARG,
              "store n minus n_common must be a multiple of n_states");
  if (Z->n_common > 0) {
    R3M_REQUIRE(store_is_spectral(Z), R3M_ERR_UNSUPPORTED,
                "shared (connected-geometry) bases need a spectral store");
    R3M_REQUIRE(Z->common_ext, R3M_ERR_INVALID_ARG, "common_ext is NULL");
  }
  const int n_a = (Z->n - Z->n_common) / Z->n_states;
  R3M_REQUIRE(n_a == 40 || n_a == 64, R3M_ERR_UNSUPPORTED,
              "the matvec kernels are instantiated for 40 or 64 active RWG per unit");
  R3M_REQUIRE(Z->n <= 256, R3M_ERR_UNSUPPORTED, "at most 256 macro RWG per unit");
  R3M_REQUIRE(Z->Dx >= 0 && Z->Dy >= 0 && Z->near_radius >= 0, R3M_ERR_INVALID_ARG, "bad extents");
  R3M_REQUIRE(Z->near, R3M_ERR_INVALID_ARG, "near blocks are NULL");
  R3M_REQUIRE(Z->near_dtype == R3M_C128 || Z->near_dtype == R3M_C64, R3M_ERR_UNSUPPORTED,
              "near dtype must be C128 or C64");
  if (store_is_spectral(Z)) {
    validate_spectral(Z);
  } else if (store_has_far(Z)) {
    R3M_REQUIRE(Z->far, R3M_ERR_INVALID_ARG, "far factors are NULL");
    R3M_REQUIRE(Z->far_dtype == Z->near_dtype ||
                    (Z->near_dtype == R3M_C64 && (Z->far_dtype == R3M_BF16X2 || Z->far_dtype == R3M_F16X2)),
                R3M_ERR_UNSUPPORTED, "far dtype must match the near dtype (or be split with a C64 near store)");
    R3M_REQUIRE(Z->max_rank >= 1 && Z->max_rank <= Z->n, R3M_ERR_INVALID_ARG, "bad max_rank");
  }
}

// far field on the matrix cores: complex64 near store (FP32 arithmetic), 40
// active RWG per unit, two or four states
static bool far_on_mfma(const r3m_store* Z) {
  return store_has_far(Z) && !store_is_spectral(Z) && Z->near_dtype == R3M_C64 && Z->n / Z->n_states == kFNA &&
         (Z->n_states == 2 || Z->n_states == 4) && Z->max_rank <= 255;
}
static size_t far_mfma_lds(const r3m_store* Z) {
  return Z->n_states == 2 ? far_mfma_lds_bytes<32, 2>() : far_mfma_lds_bytes<16, 4>();
}

// the far field (and, with fuse, the near items) on the matrix cores
static void launch_far_mfma(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, const float* xs,
                        float* part, int groups, const float* fscale, size_t head, int64_t tu, bool fuse,
                        const NearArgs<float>& NA_, int near_wgs, size_t lds_nearm, const int* idle,
                        const int* live, hipStream_t stream) {
  const int ft = (int)Z->far_dtype;
  // matrix-core far field over (codebook tile, displacement group) items
  const FarMArgs FM{bd.rhs, bd.groups, bd.gtiles, bd.n_gtiles, groups, states,
                    (const float*)((const char*)Z->far + head), (const int*)Z->far, fscale, Z->max_rank,
                    Z->Dx, Z->Dy, Z->near_radius, xs, part, tu, idle};
  const size_t lds_m = far_mfma_lds(Z);
  const int nwg_m = (bd.n_gtiles * groups + kXcd - 1) / kXcd * kXcd;
  typedef void (*KF)(FarMArgs, NearArgs<float>, int, const int*);
  typedef void (*KO)(FarMArgs, const int*);
  KF kf = nullptr;
  KO ko = nullptr;
  constexpr int ctw = (kP2Tiles + 3) / 4;
  // two states (n = 80): 16 ranks per sub-chunk; four states (n = 160): 8
#define R3M_FARM_PICK(FTV)                                                                   \
  if (Z->n_states == 2) {                                                                    \
    kf = far_mfma_near_kernel<FTV, ctw, 32, 2>;                                              \
    ko = far_mfma_kernel<FTV, ctw, 32, 2>;                                                   \
  } else {                                                                                   \
    kf = far_mfma_near_kernel<FTV, ctw, 16, 4>;                                              \
    ko = far_mfma_kernel<FTV, ctw, 16, 4>;                                                   \
  }
  if (ft == R3M_BF16X2) {
    R3M_FARM_PICK(R3M_BF16X2)
  } else if (ft == R3M_F16X2) {
    R3M_FARM_PICK(R3M_F16X2)
  } else {
    R3M_FARM_PICK(0)
  }
#undef R3M_FARM_PICK
  if (fuse) {
    hipLaunchKernelGGL(kf, dim3(near_wgs + nwg_m), dim3(256), std::max(lds_m, lds_nearm), stream, FM,
                       NA_, near_wgs, live);
  } else {
    hipLaunchKernelGGL(ko, dim3(nwg_m), dim3(256), lds_m, stream, FM, live);
  }
}

template <typename S, typename XT>
static void launch_core(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, const S* xs, XT* y,
                        char* part, const void* lists, int chunks, hipStream_t stream,
                        const int* live = nullptr, const int* idle = nullptr) {
  const int n_a = Z->n / Z->n_states;
  const int Nx = std::min(Z->near_radius, Z->Dx), Ny = std::min(Z->near_radius, Z->Dy);
  const bool far = store_has_far(Z);
  const int n_far = far ? r3m_far_count(Z->Dx, Z->Dy, Z->near_radius) : 0;
  const size_t head = ((size_t)n_far * 4 + 255) / 256 * 256;
  const int groups = far ? std::max(chunks & kPlanGroups, 1) : 0;
  const bool mfma_far = far && (chunks & kPlanMfmaFar) && far_on_mfma(Z);
  const int hg = near_groups(Z, bd);
  const int64_t tu = (int64_t)bd.total_units;
  const bool mfma_near = near_on_mfma(Z);
  // the vector-unit far kernel shares its launch with the near items; the
  // matrix-core one runs alone (the shared kernel would take the larger
  // register budget of the two bodies)
  const bool fuse = mfma_near && far && sizeof(S) == 4 && !mfma_far;
  NearArgs<S> NA_{};
  size_t lds_nearm = 0;
  int near_wgs = 0;
  if (mfma_near) {
    NearLists L = near_lists((char*)lists, Z, bd);
    NA_ = NearArgs<S>{(const NearItem*)L.items, (const int*)L.n_items, (const NearPair*)L.pairs, (const S*)Z->near,
                      Z->n, Z->n_states, xs, (S*)part + (size_t)groups * tu * n_a * 2, tu};
    lds_nearm = ((size_t)2 * n_a + kNearCols) * (2 * n_a + 1) * sizeof(S);
    near_wgs = (int)((L.max_items + kXcd - 1) / kXcd * kXcd);
  }
  if (far) {
    // the batch's largest state array, when it fits, is staged in LDS
    const int lds_state_cap = bd.max_units <= 16384 ? (int)((bd.max_units + 15) / 16 * 16) : 0;
    constexpr int rch = sizeof(S) == 4 ? R3M_FAR_RCH_F32 : 4;
    const size_t lds = 4 * (size_t)rch * Z->n * 2 * sizeof(S) + lds_state_cap;
    const size_t body = ((size_t)n_far * 2 * Z->max_rank * Z->n * 2 * sizeof(S) + 255) / 256 * 256;
    const float* fscale =
        Z->far_dtype == R3M_F16X2 ? (const float*)((const char*)Z->far + head + body) : nullptr;
    const FarArgs<S> FA{bd.rhs, bd.tiles, groups, states, (const S*)((const char*)Z->far + head),
                        (const int*)Z->far, fscale, Z->max_rank, Z->Dx, Z->Dy, Z->near_radius, Z->n, n_a,
                        Z->n_states, xs, (S*)part, tu, lds_state_cap, bd.n_tiles, idle};
    const int nwg = (bd.n_tiles * groups + kXcd - 1) / kXcd * kXcd;
    const int ft = sizeof(S) == 4 ? (int)Z->far_dtype : 0;
    bool done = false;
    if constexpr (sizeof(S) == 4) {
      if (mfma_far) {
        launch_far_mfma(Z, bd, states, xs, (float*)part, groups, fscale, head, tu, fuse, NA_, near_wgs, lds_nearm, idle,
                        live, stream);
        done = true;
      }
    }
    if (!done && fuse) {
      // one launch for both fields (complex64: the matrix-core near items run
      // beside the vector-unit far tiles; complex128 is faster as two launches)
      decltype(&far_near_kernel<S, 10, rch, 0, 40>) kern;
      if (n_a == 40)
        kern = ft == R3M_BF16X2 ? far_near_kernel<S, 10, rch, sizeof(S) == 4 ? R3M_BF16X2 : 0, 40>
             : ft == R3M_F16X2  ? far_near_kernel<S, 10, rch, sizeof(S) == 4 ? R3M_F16X2 : 0, 40>
                                : far_near_kernel<S, 10, rch, 0, 40>;
      else
        kern = ft == R3M_BF16X2 ? far_near_kernel<S, 16, rch, sizeof(S) == 4 ? R3M_BF16X2 : 0, 64>
             : ft == R3M_F16X2  ? far_near_kernel<S, 16, rch, sizeof(S) == 4 ? R3M_F16X2 : 0, 64>
                                : far_near_kernel<S, 16, rch, 0, 64>;
      hipLaunchKernelGGL(kern, dim3(near_wgs + nwg), dim3(256), std::max(lds, lds_nearm), stream, FA, NA_,
                         near_wgs, live);
    } else if (!done) {
      decltype(&far_kernel<S, 10, rch, 0>) kern;
      if (n_a == 40)
        kern = ft == R3M_BF16X2 ? far_kernel<S, 10, rch, sizeof(S) == 4 ? R3M_BF16X2 : 0>
             : ft == R3M_F16X2  ? far_kernel<S, 10, rch, sizeof(S) == 4 ? R3M_F16X2 : 0>
                                : far_kernel<S, 10, rch, 0>;
      else
        kern = ft == R3M_BF16X2 ? far_kernel<S, 16, rch, sizeof(S) == 4 ? R3M_BF16X2 : 0>
             : ft == R3M_F16X2  ? far_kernel<S, 16, rch, sizeof(S) == 4 ? R3M_F16X2 : 0>
                                : far_kernel<S, 16, rch, 0>;
      hipLaunchKernelGGL(kern, dim3(nwg), dim3(256), lds, stream, FA, live);
    }
    R3M_CHECK_HIP(hipGetLastError());
  }
  if (mfma_near) {
    if (!fuse) {
      auto kern = n_a == 40 ? near_mfma_kernel<S, 40> : near_mfma_kernel<S, 64>;
      hipLaunchKernelGGL(kern, dim3((unsigned)near_wgs), dim3(256), lds_nearm, stream, NA_, live);
    }
  } else {
    const int nwg_near = (bd.n_tiles * hg + kXcd - 1) / kXcd * kXcd;
    // row-slab height: the whole state for complex64, half of it for complex128
    constexpr int sr = sizeof(S) == 4 ? 40 : 20;
    const size_t lds_near = ((size_t)sr * (Z->n + 2) + 2 * (size_t)kBU * n_a) * 2 * sizeof(S);
    R3M_REQUIRE(n_a % sr == 0 && lds_near <= 160 * 1024, R3M_ERR_UNSUPPORTED, "near row slab does not fit in LDS");
    hipLaunchKernelGGL((near_kernel<S, sr>), dim3(nwg_near), dim3(256), lds_near, stream, bd.rhs, bd.tiles, states,
                       (const S*)Z->near, Nx, Ny, Z->n, n_a, Z->n_states, xs, (S*)part, tu, groups, hg, bd.n_tiles);
  }
  R3M_CHECK_HIP(hipGetLastError());
  hipLaunchKernelGGL((reduce_groups_kernel<S, XT>), dim3(ceil_div((size_t)bd.max_units * n_a, 64), bd.B),
                     dim3(64), 0, stream, bd.rhs, (const S*)part, groups + hg, tu, n_a, y, live, idle);
  R3M_CHECK_HIP(hipGetLastError());
}

template <typename S, typename XT>
static void launch_typed(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, const void* x, void* y,
                         void* partial, const void* lists, int chunks, hipStream_t stream, const int* idle) {
  const int n_a = Z->n / Z->n_states;
  const bool far = store_has_far(Z);
  const int hg = near_groups(Z, bd);
  const size_t vec = (size_t)bd.total_units * n_a * 2 * sizeof(S);
  char* part = (char*)partial;
  const S* xs = (const S*)x;
  if (!std::is_same<S, XT>::value) {
    S* xc = (S*)(part + (size_t)((far ? max_groups(bd) : 0) + hg) * vec);
    hipLaunchKernelGGL((convert_flat_kernel<S, XT>), dim3(ceil_div((size_t)bd.max_units * n_a, 256), bd.B),
                       dim3(256), 0, stream, bd.rhs, n_a, (const XT*)x, xc);
    xs = xc;
  }
  launch_core<S, XT>(Z, bd, states, xs, (XT*)y, part, lists, chunks, stream, nullptr, idle);
}

// matvec with x already in the store precision (float for C64, double for
// C128); y is C128
// the near retrieval lists (build_near_lists) must be current at lists
void launch_matvec_pre(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, const void* xs, void* y,
                       void* partial, const void* lists, int chunks, hipStream_t stream, const int* live,
                       const int* idle, const int* rl, r3m_dtype y_type) {
  if (store_is_spectral(Z)) {
    launch_spectral(Z, bd, states, Z->near_dtype, xs, y_type, y, partial, stream, live, idle, chunks, rl);
    return;
  }
  R3M_REQUIRE(y_type == R3M_C128, R3M_ERR_UNSUPPORTED, "compressed stores write complex128 products");
  if (Z->near_dtype == R3M_C128)
    launch_core<double, double>(Z, bd, states, (const double*)xs, (double*)y, (char*)partial, lists, chunks, stream,
                                live, idle);
  else
    launch_core<float, double>(Z, bd, states, (const float*)xs, (double*)y, (char*)partial, lists, chunks, stream,
                               live, idle);
}

static std::vector<int64_t> tune_key(const r3m_store* Z, const BatchDesc& bd) {
  return {(int64_t)(intptr_t)Z->near, (int64_t)(intptr_t)Z->far, Z->near_dtype, Z->far_dtype, Z->n, Z->n_states,
          Z->Dx, Z->Dy, Z->near_radius, Z->max_rank, (int64_t)(intptr_t)&bd};
}

// Autotuner: the first time a (store, batch) pair is seen, time the matvec for
// a few displacement-group counts around the default, with the vector-unit and
// (where it applies) the matrix-core far kernel, and keep the fastest plan.
// xs is the input in the store precision, y a C128 output (overwritten).
int tuned_groups(r3m_ctx ctx, const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, const void* xs,
                 void* y, void* partial, const void* lists, hipStream_t stream) {
  if (store_is_spectral(Z)) return tuned_spectral(ctx, Z, bd, states, Z->near_dtype, xs, R3M_C128, y, partial, stream);
  if (!store_has_far(Z)) return 1;
  const std::vector<int64_t> key = tune_key(Z, bd);
  auto it = ctx->tuned_groups.find(key);
  if (it != ctx->tuned_groups.end()) return it->second;
  const int g0 = choose_chunks(bd, 64), gcap = max_groups(bd);
  // R3M_FAR_KERNEL ("valu" or "mfma") restricts the far kernel and
  // R3M_MATVEC_GROUPS fixes the count (clamped to [1, gcap]); used by tests and
  // to hold the launch shape constant across profiler runs
  std::vector<int> kinds{0};
  if (far_on_mfma(Z)) kinds.push_back(kPlanMfmaFar);
  if (const char* env = std::getenv("R3M_FAR_KERNEL")) {
    if (std::string(env) == "valu") kinds = {0};
    if (std::string(env) == "mfma" && far_on_mfma(Z)) kinds = {kPlanMfmaFar};
  }
  std::vector<int> cand;
  if (const char* env = std::getenv("R3M_MATVEC_GROUPS")) {
    cand.push_back(std::max(1, std::min(gcap, std::atoi(env))));
  } else {
    for (int g = std::max(1, g0 / 4); g <= gcap; g *= 2) cand.push_back(g);
  }
  int best = g0 | kinds[0];
  if (cand.size() * kinds.size() > 1) {
    hipEvent_t e0, e1;
    R3M_CHECK_HIP(hipEventCreate(&e0));
    R3M_CHECK_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    for (int kind : kinds)
      for (int g : cand) {
        const int plan = g | kind;
        launch_matvec_pre(Z, bd, states, xs, y, partial, lists, plan, stream, nullptr);  // warm
        R3M_CHECK_HIP(hipEventRecord(e0, stream));
        for (int rep = 0; rep < 2; ++rep) launch_matvec_pre(Z, bd, states, xs, y, partial, lists, plan, stream, nullptr);
        R3M_CHECK_HIP(hipEventRecord(e1, stream));
        R3M_CHECK_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        R3M_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
        // candidates come in a fixed order; a later one must win by 3% (keeps
        // the choice stable between runs when two plans are within noise)
        if (ms < 0.97f * best_ms) {
          best_ms = ms;
          best = plan;
        }
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  } else {
    best = cand[0] | kinds[0];
  }
  ctx->tuned_groups[key] = best;
  return best;
}

// Spectral autotuner: the first time a (store, batch) pair is seen, time the
// frequency product's shapes (the vector-unit kernel and, for complex64
// spectra from 4 right-hand sides, each matrix-core shape) on the whole
// matvec with the default workgroup order, then the other order of the full
// batch on the two fastest matrix-core shapes, then the two-pass transforms
// against the fused ones; keep the fastest plan.
// R3M_SPEC_SHAPE (an index of kSpecShapes) fixes the shape.
int tuned_spectral(r3m_ctx ctx, const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, r3m_dtype x_type,
                   const void* x, r3m_dtype y_type, void* y, void* work, hipStream_t stream) {
  const std::vector<int64_t> key = tune_key(Z, bd);
  auto it = ctx->tuned_groups.find(key);
  if (it != ctx->tuned_groups.end()) return it->second;
  std::vector<int> shapes{0};
  if (Z->far_dtype == R3M_SPEC_C64 && bd.B >= 4)
    for (int k = 1; k < kSpecShapeCount; ++k) shapes.push_back(k);
  if (const char* env = std::getenv("R3M_SPEC_SHAPE")) {
    const int k = std::atoi(env);
    if (k >= 0 && k < kSpecShapeCount && spectral_plan_valid(Z, spec_plan(k, spec_default_rf(k)))) shapes = {k};
  }
  int best = spectral_default_plan(Z, bd.B);
  if (shapes.size() == 1) {
    best = spec_plan(shapes[0], spec_default_rf(shapes[0]));
  } else {
    hipEvent_t e0, e1;
    R3M_CHECK_HIP(hipEventCreate(&e0));
    R3M_CHECK_HIP(hipEventCreate(&e1));
    // one warm and one timed call per candidate (a wide batch's matvec runs
    // tens of milliseconds, well above the timer's noise)
    auto time_plan = [&](int plan) {
      launch_spectral(Z, bd, states, x_type, x, y_type, y, work, stream, nullptr, nullptr, plan);  // warm
      R3M_CHECK_HIP(hipEventRecord(e0, stream));
      launch_spectral(Z, bd, states, x_type, x, y_type, y, work, stream, nullptr, nullptr, plan);
      R3M_CHECK_HIP(hipEventRecord(e1, stream));
      R3M_CHECK_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      R3M_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
      return ms;
    };
    // candidates in a fixed order; a later one must win by 3% (stable choices
    // between runs when two plans are within noise)
    float best_ms = 1e30f;
    std::vector<std::pair<float, int>> mfma;
    for (int k : shapes) {
      const int plan = spec_plan(k, spec_default_rf(k));
      const float ms = time_plan(plan);
      if (k != 0) mfma.push_back({ms, k});
      if (ms < 0.97f * best_ms) {
        best_ms = ms;
        best = plan;
      }
    }
    // the other workgroup order of the full batch: the shape's default
    // threshold orders RHS tile first from spec_default_rf tiles on, so from
    // there the alternative is the contiguous order at every count, below it
    // RHS tile first from the batch's own tile count
    const int n_bt = (bd.B + 15) / 16;
    std::sort(mfma.begin(), mfma.end());
    for (size_t i = 0; i < mfma.size() && i < 2 && n_bt > 1; ++i) {
      const int k = mfma[i].second;
      const int other = spec_plan(k, n_bt >= spec_default_rf(k) ? 255 : n_bt);
      const float ms = time_plan(other);
      if (ms < 0.97f * best_ms) {
        best_ms = ms;
        best = other;
      }
    }
    // (the XCD groupings of the frequency tiles, bits 13-14, are left at 0:
    // measured no faster on the 1,536-RHS batch, slower with more groups)
    // the transform form: two passes through HBM against the fused 2-D transform
    if (spectral_fused_transforms(Z) && time_plan(best | kPlanSpecTwoPass) < 0.97f * best_ms)
      best |= kPlanSpecTwoPass;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  ctx->tuned_groups[key] = best;
  return best;
}

// the plan of (store, batch): the autotuned (or pinned) value when known,
// else the default
int plan_groups(r3m_ctx ctx, const r3m_store* Z, const BatchDesc& bd) {
  const std::vector<int64_t> key = tune_key(Z, bd);
  auto it = ctx->tuned_groups.find(key);
  if (it != ctx->tuned_groups.end()) return it->second;
  return store_is_spectral(Z) ? spectral_default_plan(Z, bd.B) : choose_chunks(bd, 64);
}

bool plan_valid(const r3m_store* Z, const BatchDesc& bd, int plan) {
  if (store_is_spectral(Z)) return spectral_plan_valid(Z, plan);
  const int g = plan & kPlanGroups;
  return (plan & ~(kPlanGroups | kPlanMfmaFar)) == 0 && g >= 1 && g <= max_groups(bd) &&
         (!(plan & kPlanMfmaFar) || far_on_mfma(Z));
}

// partial: a workspace of matvec_partial_bytes(bd, Z, max_groups(bd)); lists:
// current near lists (build_near_lists), or NULL for the ones inside partial
void launch_matvec(r3m_ctx ctx, const r3m_store* Z, const BatchDesc& bd, const uint8_t* states,
                   r3m_dtype vec_dtype, const void* x, void* y, void* partial, const void* lists, int chunks,
                   hipStream_t stream, const int* idle) {
  (void)ctx;
  if (store_is_spectral(Z)) {
    launch_spectral(Z, bd, states, vec_dtype, x, vec_dtype, y, partial, stream, nullptr, idle, chunks);
    return;
  }
  if (!lists) lists = workspace_lists(partial, bd, Z);
  if (Z->near_dtype == R3M_C128) {
    R3M_REQUIRE(vec_dtype == R3M_C128, R3M_ERR_UNSUPPORTED, "a C128 store needs C128 vectors");
    launch_typed<double, double>(Z, bd, states, x, y, partial, lists, chunks, stream, idle);
  } else if (vec_dtype == R3M_C64) {
    launch_typed<float, float>(Z, bd, states, x, y, partial, lists, chunks, stream, idle);
  } else {
    launch_typed<float, double>(Z, bd, states, x, y, partial, lists, chunks, stream, idle);
  }
}

}  // namespace r3m

using namespace r3m;

extern "C" {

size_t r3m_matvec_work_bytes(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch,
                             r3m_dtype vec_dtype) {
  size_t out = 0;
  int rc = guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    validate_batch(batch, Z->Dx, Z->Dy);
    if (batch->B == 0) return;
    const BatchDesc& bd = get_batch(ctx, batch, kBW, kBH, 0);
    out = matvec_partial_bytes(bd, Z, max_groups(bd));
  });
  return rc == R3M_OK ? out : 0;
}

int r3m_retrieved_matvec(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch,
                         r3m_dtype vec_dtype, const void* x_dev, void* y_dev, void* work_dev,
                         size_t work_bytes, hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    validate_batch(batch, Z->Dx, Z->Dy);
    R3M_REQUIRE(vec_dtype == R3M_C128 || vec_dtype == R3M_C64, R3M_ERR_UNSUPPORTED,
                "vectors must be C128 or C64");
    if (batch->B == 0) return;
    R3M_REQUIRE(x_dev && y_dev, R3M_ERR_INVALID_ARG, "x or y is NULL");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    const BatchDesc& bd = get_batch(ctx, batch, kBW, kBH, stream);
    const size_t need = matvec_partial_bytes(bd, Z, max_groups(bd));
    R3M_REQUIRE(work_bytes >= need, R3M_ERR_BUFFER_TOO_SMALL, "matvec workspace too small");
    R3M_REQUIRE(work_dev, R3M_ERR_INVALID_ARG, "work is NULL");
    // the retrieval index of this codebook (near lists), unless the caller
    // declares the one in the workspace current
    if (!(batch->flags & R3M_BATCH_INDEX_READY)) {
      check_states(bd, batch->states, Z->n_states, deferred_word(ctx), kDeferredBadState, stream);
      build_near_lists(Z, bd, batch->states, workspace_lists(work_dev, bd, Z), stream);
    }
    // first C128 call on this (store, batch): tune the group count on this x
    // (the tuner writes y as C128, so C64 vectors take the tuned or default value)
    if (store_is_spectral(Z))  // first call on this (store, batch): tune the frequency product on this x
      tuned_spectral(ctx, Z, bd, batch->states, vec_dtype, x_dev, vec_dtype, y_dev, work_dev, stream);
    if (vec_dtype == R3M_C128 && store_has_far(Z) && !store_is_spectral(Z)) {
      const void* xs = x_dev;
      if (Z->near_dtype == R3M_C64) {
        const int n_a = Z->n / Z->n_states;
        const size_t vec = (size_t)bd.total_units * n_a * 2 * sizeof(float);
        float* xc = (float*)((char*)work_dev + (size_t)(max_groups(bd) + near_groups(Z, bd)) * vec);
        hipLaunchKernelGGL((convert_flat_kernel<float, double>),
                           dim3(ceil_div((size_t)bd.max_units * n_a, 256), bd.B), dim3(256), 0, stream, bd.rhs,
                           n_a, (const double*)x_dev, xc);
        R3M_CHECK_HIP(hipGetLastError());
        xs = xc;
      }
      tuned_groups(ctx, Z, bd, batch->states, xs, y_dev, work_dev, workspace_lists(work_dev, bd, Z), stream);
    }
    launch_matvec(ctx, Z, bd, batch->states, vec_dtype, x_dev, y_dev, work_dev, nullptr, plan_groups(ctx, Z, bd),
                  stream);
  });
}

}  // extern "C"

extern "C" int32_t r3m_matvec_groups(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch) {
  int32_t out = 0;
  int rc = guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    validate_batch(batch, Z->Dx, Z->Dy);
    if (batch->B == 0) return;
    out = store_is_spectral(Z) ? 1 : plan_groups(ctx, Z, get_batch(ctx, batch, kBW, kBH, 0)) & kPlanGroups;
  });
  return rc == R3M_OK ? out : rc;
}

extern "C" int r3m_spectral_product(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, void* work_dev,
                                    size_t work_bytes, hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    R3M_REQUIRE(store_is_spectral(Z), R3M_ERR_UNSUPPORTED, "the frequency product needs a spectral store");
    validate_batch(batch, Z->Dx, Z->Dy);
    if (batch->B == 0) return;
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    const BatchDesc& bd = get_batch(ctx, batch, kBW, kBH, stream);
    R3M_REQUIRE(work_dev, R3M_ERR_INVALID_ARG, "work is NULL");
    R3M_REQUIRE(work_bytes >= matvec_partial_bytes(bd, Z, max_groups(bd)), R3M_ERR_BUFFER_TOO_SMALL,
                "matvec workspace too small");
    launch_spectral_product(Z, bd, work_dev, plan_groups(ctx, Z, bd), stream);
  });
}

extern "C" int32_t r3m_matvec_plan(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch) {
  int32_t out = 0;
  int rc = guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    validate_batch(batch, Z->Dx, Z->Dy);
    if (batch->B == 0) return;
    out = plan_groups(ctx, Z, get_batch(ctx, batch, kBW, kBH, 0));
  });
  return rc == R3M_OK ? out : rc;
}

extern "C" int r3m_matvec_set_plan(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, int32_t plan) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    validate_batch(batch, Z->Dx, Z->Dy);
    if (batch->B == 0) return;
    const BatchDesc& bd = get_batch(ctx, batch, kBW, kBH, 0);
    R3M_REQUIRE(plan_valid(Z, bd, plan), R3M_ERR_INVALID_ARG, "plan does not fit this store and batch");
    ctx->tuned_groups[tune_key(Z, bd)] = plan;
  });
}

// ------------------------------------------------- allocation-free variant
//
// The library's own device scratch for r3m_retrieved_matvec_static: one copy
// per GPU, held until the process ends.  In host code `scratch` names a
// host-side stand-in, never the device memory: the device address is looked
// up once per device (init_static_scratch, at context creation) and only that
// address is used.
static __device__ __align__(256) unsigned char scratch[R3M_STATIC_SCRATCH_BYTES];

namespace r3m {
namespace {
struct StaticScratch {
  void* ptr = nullptr;           // device address of `scratch` on this GPU
  std::vector<int64_t> key;      // batch layout whose tables sit at its head
};
std::mutex g_scratch_mu;
std::map<int, StaticScratch> g_scratch;  // device -> state
}  // namespace

void init_static_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  StaticScratch& s = g_scratch[device];
  if (s.ptr) return;
  void* p = nullptr;
  R3M_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  R3M_REQUIRE(p, R3M_ERR_HIP, "static scratch has no device address");
  s.ptr = p;
}
}  // namespace r3m

extern "C" size_t r3m_static_scratch_bytes(void) { return (size_t)R3M_STATIC_SCRATCH_BYTES; }

extern "C" int r3m_retrieved_matvec_static(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch,
                                           r3m_dtype vec_dtype, const void* x_dev, void* y_dev,
                                           hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    validate_batch(batch, Z->Dx, Z->Dy);
    R3M_REQUIRE(vec_dtype == R3M_C128 || vec_dtype == R3M_C64, R3M_ERR_UNSUPPORTED,
                "vectors must be C128 or C64");
    if (batch->B == 0) return;
    R3M_REQUIRE(x_dev && y_dev, R3M_ERR_INVALID_ARG, "x or y is NULL");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(ctx->device);
    R3M_REQUIRE(it != g_scratch.end() && it->second.ptr, R3M_ERR_HIP, "static scratch not set up on this device");
    StaticScratch& sc = it->second;
    // the batch tables at the head of the scratch, then the matvec workspace
    BatchDesc bd;
    std::vector<char> host;
    describe_batch(batch, kBW, kBH, &bd, host);
    const size_t head = (host.size() + 255) / 256 * 256;
    const int groups = choose_chunks(bd, 64);
    const size_t need = head + matvec_partial_bytes(bd, Z, max_groups(bd));
    R3M_REQUIRE(need <= (size_t)R3M_STATIC_SCRATCH_BYTES, R3M_ERR_BUFFER_TOO_SMALL,
                "batch needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                    std::to_string((size_t)R3M_STATIC_SCRATCH_BYTES) + " (use r3m_retrieved_matvec)");
    std::vector<int64_t> key = batch_key(batch, kBW, kBH);
    if (key != sc.key) {
      R3M_CHECK_HIP(hipMemcpyAsync(sc.ptr, host.data(), host.size(), hipMemcpyHostToDevice, stream));
      // the host copy of the tables is released when this call returns
      R3M_CHECK_HIP(hipStreamSynchronize(stream));
      sc.key.swap(key);
    }
    point_batch(&bd, sc.ptr);
    char* work = (char*)sc.ptr + head;
    if (!(batch->flags & R3M_BATCH_INDEX_READY)) {
      check_states(bd, batch->states, Z->n_states, deferred_word(ctx), kDeferredBadState, stream);
      build_near_lists(Z, bd, batch->states, workspace_lists(work, bd, Z), stream);
    }
    launch_matvec(ctx, Z, bd, batch->states, vec_dtype, x_dev, y_dev, work, nullptr, groups, stream);
  });
}
