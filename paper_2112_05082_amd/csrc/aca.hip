// Low-rank compression of far displacement blocks: Z(d) ~ U V^H by fully
// pivoted adaptive cross approximation (admissible blocks of Sec. II-B).
//
// One workgroup per block, FP64, explicit residual R in global scratch:
//   R = Z;  repeat { (i*, j*) = argmax |R| (ties: lowest row-major index);
//                    stop if ||R||_F <= tol ||Z||_F or rank == cap;
//                    u = R[:, j*];  conj(v) = R[i*, :] / R[i*, j*];  R -= u v^H }
// The achieved relative error ||R||_F / ||Z||_F is exact.
#include "r3m_common.h"

#include <hip/hip_fp16.h>

#include <algorithm>

namespace r3m {
namespace {

constexpr int kAcaThreads = 256;

struct MaxSum {
  double v;   // |R|^2 of the candidate pivot
  int idx;    // row-major index
  double s;   // partial sum of |R|^2
};

__device__ inline void better(MaxSum& a, double v, int idx) {
  if (v > a.v || (v == a.v && idx < a.idx)) {
    a.v = v;
    a.idx = idx;
  }
}

__device__ MaxSum block_reduce(MaxSum x, MaxSum* sh) {
  // wave-level butterfly
  for (int o = 32; o >= 1; o >>= 1) {
    double ov = __shfl_xor(x.v, o);
    int oi = __shfl_xor(x.idx, o);
    double os = __shfl_xor(x.s, o);
    better(x, ov, oi);
    x.s += os;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    MaxSum r = sh[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      better(r, sh[w].v, sh[w].idx);
      r.s += sh[w].s;
    }
    sh[0] = r;
  }
  __syncthreads();
  MaxSum r = sh[0];
  __syncthreads();
  return r;
}

__device__ inline int far_to_slot(int f, int Dx, int Dy, int nr) {
  // inverse of far_index: walk rows (few hundred at most)
  const int W = 2 * Dx + 1;
  const int Nx = nr < Dx ? nr : Dx, Ny = nr < Dy ? nr : Dy;
  int cnt = 0;
  for (int dy = -Dy; dy <= Dy; ++dy) {
    const bool near_row = dy >= -Ny && dy <= Ny;
    const int row_far = near_row ? W - (2 * Nx + 1) : W;
    if (f < cnt + row_far) {
      int r = f - cnt;
      int dx;
      if (!near_row) {
        dx = -Dx + r;
      } else {
        const int left = Dx - Nx;  // far slots left of the near band
        dx = r < left ? -Dx + r : Nx + 1 + (r - left);
      }
      return (dy + Dy) * W + (dx + Dx);
    }
    cnt += row_far;
  }
  return -1;
}

// Split storage of one real value v (already scaled): hi = RNE(v) in the
// 16-bit format, lo = RNE(v - hi); returned as the two 16-bit patterns.
__device__ inline void split_bf16(float v, uint32_t& hi, uint32_t& lo) {
  auto rne = [](float x) -> uint32_t {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;  // finite inputs only
  };
  hi = rne(v);
  lo = rne(v - __uint_as_float(hi << 16));
}
__device__ inline void split_f16(float v, uint32_t& hi, uint32_t& lo) {
  const __half h = __float2half_rn(v);
  const __half l = __float2half_rn(v - __half2float(h));
  hi = __half_as_ushort(h);
  lo = __half_as_ushort(l);
}

// Writes the FP64 factors [2 cap][n] (U columns then V columns) of far block
// f in the store format: C128, C64, or an 8-byte split element
// {re_hi | im_hi << 16, re_lo | im_lo << 16} (BF16X2, F16X2).  F16X2 columns
// are scaled by 2^-e with 2^e >= the column's largest real or imaginary
// magnitude; scales[f][2 cap] holds 2^e.
__device__ void store_factors(const double2* __restrict__ UV, int n, int cap, int f, int mode, void* far_out,
                              float* scales, MaxSum* sh) {
  const int tot = 2 * cap * n;
  if (mode == R3M_C128) {
    double2* o = reinterpret_cast<double2*>(far_out) + (size_t)f * tot;
    for (int e = threadIdx.x; e < tot; e += blockDim.x) o[e] = UV[e];
    return;
  }
  if (mode == R3M_C64) {
    float2* o = reinterpret_cast<float2*>(far_out) + (size_t)f * tot;
    for (int e = threadIdx.x; e < tot; e += blockDim.x) o[e] = make_float2((float)UV[e].x, (float)UV[e].y);
    return;
  }
  uint2* o = reinterpret_cast<uint2*>(far_out) + (size_t)f * tot;
  for (int c = 0; c < 2 * cap; ++c) {
    float sc = 1.0f, inv = 1.0f;
    if (mode == R3M_F16X2) {
      MaxSum m{0.0, 0, 0.0};
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 v = UV[(size_t)c * n + i];
        m.v = fmax(m.v, fmax(fabs(v.x), fabs(v.y)));
      }
      // block maximum (the index field is unused here)
      for (int o2 = 32; o2 >= 1; o2 >>= 1) m.v = fmax(m.v, __shfl_xor(m.v, o2));
      if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
      __syncthreads();
      double mx = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mx = fmax(mx, sh[w].v);
      __syncthreads();
      const int e = mx > 0.0 ? (int)ceil(log2(mx)) : 0;
      sc = ldexpf(1.0f, e);
      inv = ldexpf(1.0f, -e);
      if (threadIdx.x == 0) scales[(size_t)f * 2 * cap + c] = sc;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double2 v = UV[(size_t)c * n + i];
      uint32_t rh, rl, ih, il;
      if (mode == R3M_BF16X2) {
        split_bf16((float)v.x, rh, rl);
        split_bf16((float)v.y, ih, il);
      } else {
        split_f16((float)v.x * inv, rh, rl);
        split_f16((float)v.y * inv, ih, il);
      }
      o[(size_t)c * n + i] = make_uint2(rh | (ih << 16), rl | (il << 16));
    }
  }
}

__global__ void __launch_bounds__(kAcaThreads) aca_kernel(const double2* __restrict__ dense, int n,
                                                          int Dx, int Dy, int nr, int f_begin,
                                                          int f_count, double tol, int cap,
                                                          double2* work, int mode, void* far_out,
                                                          float* scales, int* ranks_out, double* err_out) {
  __shared__ MaxSum sh[kAcaThreads / 64];
  extern __shared__ double2 lds[];  // [n] column u, [n] pivot row
  double2* ucol = lds;
  double2* prow = lds + n;
  const int fb = blockIdx.x;
  if (fb >= f_count) return;
  const int f = f_begin + fb;
  const int slot = far_to_slot(f, Dx, Dy, nr);
  if (slot < 0) return;
  const size_t nn = (size_t)n * n;
  const double2* Z = dense + (size_t)slot * nn;
  double2* R = work + (size_t)fb * (nn + 2 * (size_t)cap * n);
  double2* U = R + nn;        // [cap][n]
  double2* V = U + (size_t)cap * n;

  MaxSum acc{-1.0, 0x7fffffff, 0.0};
  for (int e = threadIdx.x; e < (int)nn; e += blockDim.x) {
    double2 z = Z[e];
    R[e] = z;
    const double v = z.x * z.x + z.y * z.y;
    acc.s += v;
  }
  for (int e = threadIdx.x; e < 2 * cap * n; e += blockDim.x) U[e] = make_double2(0.0, 0.0);
  MaxSum tot = block_reduce(acc, sh);
  const double znorm2 = tot.s;
  const double lim2 = tol * tol * znorm2;

  int rank = 0;
  double err = 0.0;
  for (;;) {
    __syncthreads();
    MaxSum a{-1.0, 0x7fffffff, 0.0};
    for (int e = threadIdx.x; e < (int)nn; e += blockDim.x) {
      double2 r = R[e];
      const double v = r.x * r.x + r.y * r.y;
      a.s += v;
      better(a, v, e);
    }
    MaxSum red = block_reduce(a, sh);
    err = znorm2 > 0.0 ? sqrt(red.s / znorm2) : 0.0;
    if (red.s <= lim2 || rank >= cap || red.v <= 0.0) break;
    const int is = red.idx / n, js = red.idx % n;
    const double2 piv = R[red.idx];
    const double pm = piv.x * piv.x + piv.y * piv.y;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      ucol[i] = R[(size_t)i * n + js];
      // R[i*, j] / piv
      double2 rr = R[(size_t)is * n + i];
      prow[i] = make_double2((rr.x * piv.x + rr.y * piv.y) / pm, (rr.y * piv.x - rr.x * piv.y) / pm);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      U[(size_t)rank * n + i] = ucol[i];
      V[(size_t)rank * n + i] = make_double2(prow[i].x, -prow[i].y);  // v = conj(row / piv)
    }
    for (int e = threadIdx.x; e < (int)nn; e += blockDim.x) {
      const int i = e / n, j = e % n;
      const double2 u = ucol[i], w = prow[j];  // R_ij -= u_i * (R[i*, j] / piv)
      double2 r = R[e];
      r.x -= u.x * w.x - u.y * w.y;
      r.y -= u.x * w.y + u.y * w.x;
      R[e] = r;
    }
    ++rank;
  }
  __syncthreads();
  // factors: U_f [cap][n] then V_f [cap][n]
  store_factors(U, n, cap, f, mode, far_out, scales, sh);
  if (threadIdx.x == 0) {
    ranks_out[f] = rank;
    err_out[f] = err;
  }
}

}  // namespace
}  // namespace r3m

using namespace r3m;

extern "C" {

int32_t r3m_far_count(int32_t Dx, int32_t Dy, int32_t near_radius) {
  if (Dx < 0 || Dy < 0 || near_radius < 0) return 0;
  const int Nx = std::min(near_radius, Dx), Ny = std::min(near_radius, Dy);
  return (2 * Dx + 1) * (2 * Dy + 1) - (2 * Nx + 1) * (2 * Ny + 1);
}

size_t r3m_far_bytes(int32_t n, int32_t n_far, int32_t max_rank, r3m_dtype dtype) {
  if (n <= 0 || n_far < 0 || max_rank < 0) return 0;
  const size_t head = ((size_t)n_far * 4 + 255) / 256 * 256;
  const size_t es = dtype == R3M_C128 ? 16 : (dtype == R3M_C64 || dtype == R3M_BF16X2 || dtype == R3M_F16X2) ? 8 : 0;
  if (es == 0) return 0;
  const size_t body = (size_t)n_far * 2 * max_rank * n * es;
  const size_t scales = dtype == R3M_F16X2 ? (size_t)n_far * 2 * max_rank * 4 : 0;
  return head + (body + 255) / 256 * 256 + scales;
}

size_t r3m_compress_work_bytes(int32_t n, int32_t max_rank, int32_t blocks_per_batch) {
  if (n <= 0 || max_rank < 0 || blocks_per_batch <= 0) return 0;
  const size_t per = ((size_t)n * n + 2 * (size_t)max_rank * n) * 16;
  // + device copies of ranks and errors of one batch
  return per * blocks_per_batch + (size_t)blocks_per_batch * 16 + 256;
}

int r3m_compress_far(r3m_ctx ctx, const void* dense_dev, int32_t n, int32_t Dx, int32_t Dy,
                     int32_t near_radius, double tol, int32_t max_rank, r3m_dtype far_dtype,
                     void* far_dev, size_t far_bytes, int32_t* ranks_host, double* rel_err_host,
                     void* work_dev, size_t work_bytes, hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    R3M_REQUIRE(dense_dev && far_dev && work_dev, R3M_ERR_INVALID_ARG, "NULL buffer");
    R3M_REQUIRE(n > 0 && n <= 4096 && Dx >= 0 && Dy >= 0 && near_radius >= 0, R3M_ERR_INVALID_ARG,
                "bad block shape");
    R3M_REQUIRE(tol >= 0.0 && std::isfinite(tol), R3M_ERR_INVALID_ARG, "tol must be >= 0");
    R3M_REQUIRE(max_rank >= 1 && max_rank <= n, R3M_ERR_INVALID_ARG, "max_rank must be in [1, n]");
    R3M_REQUIRE(far_dtype == R3M_C128 || far_dtype == R3M_C64 || far_dtype == R3M_BF16X2 ||
                    far_dtype == R3M_F16X2,
                R3M_ERR_UNSUPPORTED, "unknown far dtype");
    const int n_far = r3m_far_count(Dx, Dy, near_radius);
    R3M_REQUIRE(far_bytes >= r3m_far_bytes(n, n_far, max_rank, far_dtype), R3M_ERR_BUFFER_TOO_SMALL,
                "far buffer too small");
    R3M_REQUIRE(n_far == 0 || (ranks_host && rel_err_host), R3M_ERR_INVALID_ARG,
                "ranks_host / rel_err_host are NULL");
    const size_t per = ((size_t)n * n + 2 * (size_t)max_rank * n) * 16;
    R3M_REQUIRE(work_bytes >= r3m_compress_work_bytes(n, max_rank, 1), R3M_ERR_BUFFER_TOO_SMALL,
                "compress workspace too small");
    int bpb = (int)std::min<size_t>((work_bytes - 256) / (per + 16), (size_t)std::max(n_far, 1));
    bpb = std::max(bpb, 1);
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    if (n_far == 0) return;
    const size_t head = ((size_t)n_far * 4 + 255) / 256 * 256;
    int32_t* ranks_dev = (int32_t*)far_dev;
    char* factors = (char*)far_dev + head;
    const size_t es = far_dtype == R3M_C128 ? 16 : 8;
    float* scales = far_dtype == R3M_F16X2
                        ? (float*)(factors + ((size_t)n_far * 2 * max_rank * n * es + 255) / 256 * 256)
                        : nullptr;
    char* wbase = (char*)work_dev;
    double2* rwork = (double2*)wbase;
    double* err_dev = (double*)(wbase + per * bpb);
    // factors of far index f land at factors + f * 2*cap*n*esize; errors of a batch are
    // written at err_dev[f - f0] through the pointer offset below
    for (int f0 = 0; f0 < n_far; f0 += bpb) {
      const int cnt = std::min(bpb, n_far - f0);
      const size_t lds = 2 * (size_t)n * sizeof(double2);
      hipLaunchKernelGGL(aca_kernel, dim3(cnt), dim3(kAcaThreads), lds, stream, (const double2*)dense_dev, n, Dx,
                         Dy, near_radius, f0, cnt, tol, max_rank, rwork, (int)far_dtype, (void*)factors, scales,
                         ranks_dev, err_dev - f0);
      R3M_CHECK_HIP(hipGetLastError());
      R3M_CHECK_HIP(hipMemcpyAsync(rel_err_host + f0, err_dev, cnt * sizeof(double),
                                   hipMemcpyDeviceToHost, stream));
      R3M_CHECK_HIP(hipStreamSynchronize(stream));
    }
    R3M_CHECK_HIP(hipMemcpyAsync(ranks_host, ranks_dev, n_far * sizeof(int32_t), hipMemcpyDeviceToHost,
                                 stream));
    R3M_CHECK_HIP(hipStreamSynchronize(stream));
  });
}

}  // extern "C"
