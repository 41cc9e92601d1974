// Small dense kernels shared by the solver's preconditioners (device inline).
#pragma once
#include <hip/hip_runtime.h>

namespace r3m {

__device__ inline double2 dense_cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Gauss-Jordan inversion with partial pivoting of the NA x NA block held in
// the left half of aug [NA][2 NA] (right half: identity), by one workgroup of
// NT threads; the inverse is left in the right half.  The pivot of column k
// is the row of largest modulus at or below k (the lowest such row on ties),
// found by wave 0 with a butterfly reduction.  colk: NA + 1 double2 of LDS
// (the multipliers of the current column, then the inverse pivot).
// Returns false (and sets bit 8 of flag) for a singular block; uniform over
// the workgroup.
template <int NA, int NT>
__device__ inline bool gj_invert(double2* aug, double2* colk, int* piv_row, int* __restrict__ flag) {
  constexpr int w = 2 * NA;
  constexpr int G = NT / w;                   // row groups (one column per thread)
  constexpr int kRows = (NA + G - 1) / G;     // rows per thread
  constexpr int kChunk = kRows < 7 ? kRows : 7;
  const int tid = threadIdx.x;
  double2* piv_inv = colk + NA;
  for (int k = 0; k < NA; ++k) {
    // pivot row and its inverse pivot (wave 0)
    if (tid < 64) {
      double best = -1.0;
      int p = NA;
      for (int i = k + tid; i < NA; i += 64) {
        const double2 a = aug[i * w + k];
        const double m = a.x * a.x + a.y * a.y;
        if (m > best) {
          best = m;
          p = i;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int op = __shfl_xor(p, off);
        if (ob > best || (ob == best && op < p)) {
          best = ob;
          p = op;
        }
      }
      if (tid == 0) {
        if (best > 0.0) {
          const double2 d = aug[p * w + k];
          const double dd = d.x * d.x + d.y * d.y;
          *piv_inv = make_double2(d.x / dd, -d.y / dd);
          *piv_row = p;
        } else {
          *piv_row = -1;
          atomicOr(flag, 8);
        }
      }
    }
    __syncthreads();
    const int p = *piv_row;
    if (p < 0) return false;
    const double2 inv = *piv_inv;
    // rows k and p exchange and the new row k is scaled by the inverse pivot;
    // the multipliers of column k are taken as they stand after the exchange
    for (int j = tid; j < w; j += NT) {
      const double2 a = aug[k * w + j], b = aug[p * w + j];
      aug[k * w + j] = dense_cmul(b, inv);
      if (p != k) {
        aug[p * w + j] = a;
        if (j == k) colk[p] = a;
      }
    }
    for (int i = tid; i < NA; i += NT)
      if (i != k && i != p) colk[i] = aug[i * w + k];  // rows that did not move
    __syncthreads();
    // elimination: thread (g, j) updates column j of rows g, g + G, ...; all of
    // its operands are read before any of its writes
    if (tid < G * w) {
      const int j = tid % w, g = tid / w;
      const double2 pj = aug[k * w + j];
      for (int q0 = 0; q0 < kRows; q0 += kChunk) {
        double2 v[kChunk], c[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
          const int i = g + (q0 + q) * G;
          if (i < NA) {
            v[q] = aug[i * w + j];
            c[q] = colk[i];
          }
        }
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
          const int i = g + (q0 + q) * G;
          if (i < NA && i != k) {
            const double2 u = dense_cmul(c[q], pj);
            aug[i * w + j] = make_double2(v[q].x - u.x, v[q].y - u.y);
          }
        }
      }
    }
    __syncthreads();
  }
  return true;
}

// gj_invert for the unit sizes the kernels are built for (40 or 64), 256 threads
__device__ inline bool gj_invert_na(double2* aug, double2* colk, int n_a, int* piv_row, int* __restrict__ flag) {
  return n_a == 40 ? gj_invert<40, 256>(aug, colk, piv_row, flag) : gj_invert<64, 256>(aug, colk, piv_row, flag);
}

}  // namespace r3m
