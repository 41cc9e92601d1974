// Small dense kernels shared by the solver's preconditioners (device inline).
#pragma once
#include <hip/hip_runtime.h>

namespace r3m {

__device__ inline double2 dense_cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Gauss-Jordan inversion with partial pivoting of the n_a x n_a block held in
// the left half of aug [n_a][2 n_a] (right half: identity), by one workgroup;
// the inverse is left in the right half.  Returns false (and sets bit 8 of
// flag) for a singular block; uniform over the workgroup.
__device__ inline bool gj_invert(double2* aug, double2* colk, int n_a, int* piv_row, int* __restrict__ flag) {
  const int w = 2 * n_a;
  for (int k = 0; k < n_a; ++k) {
    if (threadIdx.x == 0) {
      int p = k;
      double best = -1.0;
      for (int i = k; i < n_a; ++i) {
        const double2 a = aug[i * w + k];
        const double m = a.x * a.x + a.y * a.y;
        if (m > best) {
          best = m;
          p = i;
        }
      }
      *piv_row = best > 0.0 ? p : -1;
      if (best <= 0.0) atomicOr(flag, 8);
    }
    __syncthreads();
    const int p = *piv_row;
    if (p < 0) return false;
    if (p != k)
      for (int j = threadIdx.x; j < w; j += blockDim.x) {
        const double2 t = aug[k * w + j];
        aug[k * w + j] = aug[p * w + j];
        aug[p * w + j] = t;
      }
    __syncthreads();
    const double2 d = aug[k * w + k];
    const double dd = d.x * d.x + d.y * d.y;
    const double2 inv = make_double2(d.x / dd, -d.y / dd);
    __syncthreads();
    for (int j = threadIdx.x; j < w; j += blockDim.x) aug[k * w + j] = dense_cmul(aug[k * w + j], inv);
    // multipliers of column k, read before any row update touches that column
    for (int i = threadIdx.x; i < n_a; i += blockDim.x) colk[i] = aug[i * w + k];
    __syncthreads();
    for (int e = threadIdx.x; e < n_a * w; e += blockDim.x) {
      const int i = e / w, j = e % w;
      if (i == k) continue;
      const double2 t = dense_cmul(colk[i], aug[k * w + j]);
      aug[e] = make_double2(aug[e].x - t.x, aug[e].y - t.y);
    }
    __syncthreads();
  }
  return true;
}

}  // namespace r3m
