// Spectral evaluation of the retrieved product (FFT form of the macro
// block-Toeplitz matvec).
//
// With every unit-to-unit block a function of the displacement only (the
// periodicity the unique-block store of Sec. III-C rests on) the macro-unit
// system matrix is two-level block-Toeplitz: block (i, j) is Z(i - j).  The
// retrieved product of eq. (6) is therefore a 2-D convolution of the masked
// macro vector with the block kernel Z(d):
//   x~_j = x_j on the rows A(s_j) of unit j, zero on the other macro rows;
//   y~_i = sum_j Z(i - j) x~_j;  y_i = y~_i[A(s_i)].
// Embedding Z(d) in a circulant of Gx x Gy displacements (powers of two,
// Gx >= 2 Dx + 1) turns the convolution into one n x n product per spatial
// frequency: Y^(k) = Z^(k) X^(k) with X^ = FFT2[x~], y~ = IFFT2[Y^].  The
// result is the dense retrieval product up to rounding (no far-field
// compression); the store carries the spectra Z^ in place of far factors.
//
// Layouts (complex, interleaved; grids row-major, k = gy * Gx + gx):
//   spectra  Z^[m][n][Gy][Gx]     (m, n macro rows and columns)
//   work     X[b][n][Gy][Gx], then Y[b][n][Gy][Gx]
#include "matvec_internal.h"

#include <algorithm>

namespace r3m {
namespace {

template <typename T>
struct C2 {
  T re, im;
};

template <typename T>
__device__ __forceinline__ void sincospi_t(T x, T* s, T* c);
template <>
__device__ __forceinline__ void sincospi_t<float>(float x, float* s, float* c) {
  sincospif(x, s, c);
}
template <>
__device__ __forceinline__ void sincospi_t<double>(double x, double* s, double* c) {
  sincospi(x, s, c);
}

int next_pow2(int v) {
  int p = 2;
  while (p < v) p <<= 1;
  return p;
}

// Radix-2 Stockham transforms of lpw lines of length G staged in LDS
// (forward: exp(-2 pi i j k / G); inverse: exp(+...), unnormalised).  Line l
// starts at (l / lines_per_grid) * grid_stride + (l % lines_per_grid) *
// line_step and its elements lie elem_stride apart.  With elem_stride == 1
// consecutive threads move consecutive elements of a line; otherwise they
// move the same element of consecutive lines (columns of a row-major grid),
// so both passes read and write HBM coalesced.  LDS lines are padded to G + 1
// entries so that the column-order staging does not fall on one bank.
// Dynamic LDS: 2 * lpw * (G + 1) complex.
template <typename T>
__global__ void __launch_bounds__(256)
fft_lines_kernel(C2<T>* __restrict__ data, int G, int64_t n_lines, int lines_per_grid, int64_t grid_stride,
                 int line_step, int elem_stride, int lpw, int inverse, const int* __restrict__ live) {
  if (live && *live == 0) return;
  extern __shared__ unsigned char smem_raw[];
  const int P = G + 1;
  C2<T>* bufa = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* bufb = bufa + (size_t)lpw * P;
  const int64_t l0 = (int64_t)blockIdx.x * lpw;
  const int tot = lpw * G;
  const bool rows = elem_stride == 1;
  auto addr = [&](int li, int e) -> int64_t {
    const int64_t l = l0 + li;
    return (l / lines_per_grid) * grid_stride + (l % lines_per_grid) * (int64_t)line_step + (int64_t)e * elem_stride;
  };
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int li = rows ? t / G : t % lpw;
    const int e = rows ? t % G : t / lpw;
    C2<T> v = {0, 0};
    if (l0 + li < n_lines) v = data[addr(li, e)];
    bufa[li * P + e] = v;
  }
  __syncthreads();
  C2<T>* in = bufa;
  C2<T>* out = bufb;
  const int half = G >> 1;
  const T sgn = inverse ? T(1) : T(-1);
  for (int Ns = 1; Ns < G; Ns <<= 1) {
    for (int t = threadIdx.x; t < lpw * half; t += blockDim.x) {
      const int li = t / half, j = t - li * half;
      const int k = j & (Ns - 1);
      const C2<T> u = in[li * P + j];
      const C2<T> c = in[li * P + j + half];
      T s, co;
      sincospi_t<T>((T)k / (T)Ns, &s, &co);
      s *= sgn;  // w = cos(pi k / Ns) + sgn i sin(pi k / Ns)
      const C2<T> cw = {c.re * co - c.im * s, c.re * s + c.im * co};
      const int o = li * P + (j / Ns) * 2 * Ns + k;
      out[o] = {u.re + cw.re, u.im + cw.im};
      out[o + Ns] = {u.re - cw.re, u.im - cw.im};
    }
    __syncthreads();
    C2<T>* tmp = in;
    in = out;
    out = tmp;
  }
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int li = rows ? t / G : t % lpw;
    const int e = rows ? t % G : t / lpw;
    if (l0 + li < n_lines) data[addr(li, e)] = in[li * P + e];
  }
}

// Circulant embedding of the displacement blocks dense[slot][m][n]
// (complex128, slot = (dy + Dy)(2 Dx + 1) + dx + Dx) into grids
// [m][n][Gy][Gx]: entry (gx, gy) holds Z(d)[m][n] for gx = dx mod Gx,
// gy = dy mod Gy, and zero where no |dx| <= Dx, |dy| <= Dy maps.
template <typename T>
__global__ void __launch_bounds__(256)
spec_embed_kernel(const double2* __restrict__ dense, int n, int Dx, int Dy, int Gx, int Gy, C2<T>* __restrict__ out) {
  const int64_t G2 = (int64_t)Gx * Gy;
  const int64_t total = (int64_t)n * n * G2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t mn = e / G2;
    const int64_t k = e - mn * G2;
    const int gy = (int)(k / Gx), gx = (int)(k - (int64_t)gy * Gx);
    const int dx = gx <= Dx ? gx : gx - Gx;
    const int dy = gy <= Dy ? gy : gy - Gy;
    C2<T> v = {0, 0};
    if (dx >= -Dx && dy >= -Dy) {
      const int64_t slot = (int64_t)(dy + Dy) * (2 * Dx + 1) + (dx + Dx);
      const double2 z = dense[slot * n * n + mn];
      v = {(T)z.x, (T)z.y};
    }
    out[e] = v;
  }
}

// x~ of right-hand side b on its grid (blockIdx.y = b)
template <typename T, typename XT>
__global__ void __launch_bounds__(256)
spec_expand_kernel(const RhsDev* __restrict__ rhs, const uint8_t* __restrict__ states, int n_states, int n, int n_a,
                   const XT* __restrict__ x, int Gx, int Gy, C2<T>* __restrict__ X, const int* __restrict__ live) {
  if (live && *live == 0) return;
  const int b = blockIdx.y;
  const RhsDev R = rhs[b];
  const int64_t G2 = (int64_t)Gx * Gy;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * G2) return;
  const int ch = (int)(e / G2);
  const int64_t k = e - (int64_t)ch * G2;
  const int gy = (int)(k / Gx), gx = (int)(k - (int64_t)gy * Gx);
  C2<T> v = {0, 0};
  if (gx < R.Lx && gy < R.Ly) {
    const int64_t u = (int64_t)gy * R.Lx + gx;
    const int s = min((int)states[R.state_off + u], n_states - 1);
    const int r = ch - s * n_a;
    if (r >= 0 && r < n_a) {
      const size_t xi = ((size_t)(R.unit_off + u) * n_a + r) * 2;
      v = {(T)x[xi], (T)x[xi + 1]};
    }
  }
  X[(size_t)b * n * G2 + e] = v;
}

// Y^[b][m][k] = sum_c Z^[m][c][k] X^[b][c][k].  A thread owns one frequency k
// of one row m for a chunk of kBC right-hand sides (each Z^ entry is loaded
// once per chunk).  The chunk index varies fastest over workgroup ids, so the
// chunks that share a slice of Z^ run together and meet it in cache.
constexpr int kBC = 8;
template <typename T>
__global__ void __launch_bounds__(256)
spec_product_kernel(const C2<T>* __restrict__ Zh, const C2<T>* __restrict__ Xh, C2<T>* __restrict__ Yh, int n,
                    int64_t K, int B, int n_kb, const int* __restrict__ live) {
  if (live && *live == 0) return;
  const int nz = (B + kBC - 1) / kBC;
  const int64_t id = blockIdx.x;
  const int z = (int)(id % nz);
  const int64_t rest = id / nz;
  const int kb = (int)(rest % n_kb);
  const int m = (int)(rest / n_kb);
  const int64_t k = (int64_t)kb * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int b0 = z * kBC;
  const int nb = min(kBC, B - b0);
  T ar[kBC], ai[kBC];
#pragma unroll
  for (int q = 0; q < kBC; ++q) ar[q] = ai[q] = 0;
  const C2<T>* zr = Zh + (size_t)m * n * K + k;
  const C2<T>* xr = Xh + (size_t)b0 * n * K + k;
#pragma unroll 2
  for (int c = 0; c < n; ++c) {
    const C2<T> zv = zr[(size_t)c * K];
#pragma unroll
    for (int q = 0; q < kBC; ++q) {
      if (q < nb) {
        const C2<T> xv = xr[((size_t)q * n + c) * K];
        ar[q] = fma(zv.re, xv.re, ar[q]);
        ar[q] = fma(-zv.im, xv.im, ar[q]);
        ai[q] = fma(zv.re, xv.im, ai[q]);
        ai[q] = fma(zv.im, xv.re, ai[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kBC; ++q)
    if (q < nb) Yh[((size_t)(b0 + q) * n + m) * K + k] = {ar[q], ai[q]};
}

// y_i = y~_i[A(s_i)] / (Gx Gy): the active rows of each unit, with the
// normalisation of the unnormalised inverse transform (blockIdx.y = b)
template <typename T, typename YT>
__global__ void __launch_bounds__(256)
spec_gather_kernel(const RhsDev* __restrict__ rhs, const uint8_t* __restrict__ states, int n_states, int n, int n_a,
                   const C2<T>* __restrict__ Y, int Gx, int Gy, YT* __restrict__ y, const int* __restrict__ live) {
  if (live && *live == 0) return;
  const int b = blockIdx.y;
  const RhsDev R = rhs[b];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)R.Lx * R.Ly * n_a) return;
  const int64_t u = e / n_a;
  const int r = (int)(e - u * n_a);
  const int gy = (int)(u / R.Lx), gx = (int)(u - (int64_t)gy * R.Lx);
  const int s = min((int)states[R.state_off + u], n_states - 1);
  const int64_t G2 = (int64_t)Gx * Gy;
  const C2<T> v = Y[((size_t)b * n + s * n_a + r) * G2 + (int64_t)gy * Gx + gx];
  const T sc = T(1) / (T)G2;
  const size_t yi = ((size_t)R.unit_off * n_a + e) * 2;
  y[yi] = (YT)(v.re * sc);
  y[yi + 1] = (YT)(v.im * sc);
}

// lines per workgroup: as many as fill one LDS buffer of `cap` entries, fewer
// while the launch has under 2048 workgroups, down to min_lpw
int lines_per_wg(int G, int other, int64_t lines, int cap, int min_lpw) {
  int lpw = std::max(1, std::min(cap / (G + 1), other));
  int p = 1;
  while (p * 2 <= lpw) p *= 2;  // a power of two, so a workgroup stays inside one grid
  lpw = p;
  while (lpw > min_lpw && (lines + lpw - 1) / lpw < 2048) lpw /= 2;
  return lpw;
}

template <typename T>
void fft2(C2<T>* data, int64_t n_grids, int Gx, int Gy, int inverse, hipStream_t s, const int* live) {
  const int cap = sizeof(T) == 4 ? 4096 : 2048;  // complex entries per LDS buffer (two buffers)
  {  // along x: lines are rows
    const int64_t lines = n_grids * Gy;
    const int lpw = lines_per_wg(Gx, Gy, lines, cap, 1);
    const size_t lds = 2 * (size_t)lpw * (Gx + 1) * sizeof(C2<T>);
    hipLaunchKernelGGL(fft_lines_kernel<T>, dim3((unsigned)((lines + lpw - 1) / lpw)), dim3(256), lds, s, data, Gx,
                       lines, Gy, (int64_t)Gx * Gy, Gx, 1, lpw, inverse, live);
  }
  {  // along y: lines are columns; a workgroup takes lpw adjacent columns of one grid
    const int64_t lines = n_grids * Gx;
    const int lpw = lines_per_wg(Gy, Gx, lines, cap, std::min(Gx, 16));
    const size_t lds = 2 * (size_t)lpw * (Gy + 1) * sizeof(C2<T>);
    hipLaunchKernelGGL(fft_lines_kernel<T>, dim3((unsigned)((lines + lpw - 1) / lpw)), dim3(256), lds, s, data, Gy,
                       lines, Gx, (int64_t)Gx * Gy, 1, Gx, lpw, inverse, live);
  }
  R3M_CHECK_HIP(hipGetLastError());
}

template <typename T, typename XT, typename YT>
void spectral_typed(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, const void* x, void* y,
                    void* work, hipStream_t s, const int* live) {
  const int n = Z->n, n_a = Z->n / Z->n_states;
  const int Gx = next_pow2(2 * Z->Dx + 1), Gy = next_pow2(2 * Z->Dy + 1);
  const int64_t G2 = (int64_t)Gx * Gy;
  const int B = bd.B;
  C2<T>* X = (C2<T>*)work;
  C2<T>* Y = X + (size_t)B * n * G2;
  const C2<T>* Zh = (const C2<T>*)Z->far;
  hipLaunchKernelGGL((spec_expand_kernel<T, XT>), dim3(ceil_div((size_t)n * G2, 256), B), dim3(256), 0, s, bd.rhs,
                     states, Z->n_states, n, n_a, (const XT*)x, Gx, Gy, X, live);
  fft2<T>(X, (int64_t)B * n, Gx, Gy, 0, s, live);
  const int n_kb = (int)ceil_div((size_t)G2, 256);
  const int64_t nwg = (int64_t)n_kb * n * ((B + kBC - 1) / kBC);
  hipLaunchKernelGGL(spec_product_kernel<T>, dim3((unsigned)nwg), dim3(256), 0, s, Zh, (const C2<T>*)X, Y, n, G2, B,
                     n_kb, live);
  fft2<T>(Y, (int64_t)B * n, Gx, Gy, 1, s, live);
  hipLaunchKernelGGL((spec_gather_kernel<T, YT>), dim3(ceil_div((size_t)bd.max_units * n_a, 256), B), dim3(256), 0,
                     s, bd.rhs, states, Z->n_states, n, n_a, (const C2<T>*)Y, Gx, Gy, (YT*)y, live);
  R3M_CHECK_HIP(hipGetLastError());
}

size_t spectra_bytes(int n, int Dx, int Dy, r3m_dtype dtype) {
  const size_t es = dtype == R3M_SPEC_C128 ? 16 : 8;
  return (size_t)n * n * next_pow2(2 * Dx + 1) * next_pow2(2 * Dy + 1) * es;
}

}  // namespace

bool store_is_spectral(const r3m_store* Z) {
  return Z->far_dtype == R3M_SPEC_C64 || Z->far_dtype == R3M_SPEC_C128;
}

void validate_spectral(const r3m_store* Z) {
  R3M_REQUIRE(Z->far, R3M_ERR_INVALID_ARG, "spectra are NULL");
  R3M_REQUIRE((Z->far_dtype == R3M_SPEC_C64 && Z->near_dtype == R3M_C64) ||
                  (Z->far_dtype == R3M_SPEC_C128 && Z->near_dtype == R3M_C128),
              R3M_ERR_UNSUPPORTED, "spectra precision must match the near blocks (SPEC_C64/C64 or SPEC_C128/C128)");
  const int cap = Z->far_dtype == R3M_SPEC_C128 ? 2048 : 4096;
  R3M_REQUIRE(next_pow2(2 * Z->Dx + 1) < cap && next_pow2(2 * Z->Dy + 1) < cap, R3M_ERR_UNSUPPORTED,
              "displacement extent too large for the transform");
}

size_t spectral_work_bytes(const BatchDesc& bd, const r3m_store* Z) {
  const size_t es = Z->far_dtype == R3M_SPEC_C128 ? 16 : 8;
  const size_t G2 = (size_t)next_pow2(2 * Z->Dx + 1) * next_pow2(2 * Z->Dy + 1);
  return 2 * (size_t)bd.B * Z->n * G2 * es + 256;
}

void launch_spectral(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, r3m_dtype x_type,
                     const void* x, r3m_dtype y_type, void* y, void* work, hipStream_t s, const int* live) {
  const bool xd = x_type == R3M_C128, yd = y_type == R3M_C128;
  if (Z->far_dtype == R3M_SPEC_C128) {
    R3M_REQUIRE(xd && yd, R3M_ERR_UNSUPPORTED, "complex128 spectra need C128 vectors");
    spectral_typed<double, double, double>(Z, bd, states, x, y, work, s, live);
  } else if (xd && yd) {
    spectral_typed<float, double, double>(Z, bd, states, x, y, work, s, live);
  } else if (!xd && yd) {
    spectral_typed<float, float, double>(Z, bd, states, x, y, work, s, live);
  } else if (!xd && !yd) {
    spectral_typed<float, float, float>(Z, bd, states, x, y, work, s, live);
  } else {
    R3M_REQUIRE(false, R3M_ERR_UNSUPPORTED, "C128 input with C64 output");
  }
}

}  // namespace r3m

using namespace r3m;

extern "C" {

size_t r3m_spectral_bytes(int32_t n, int32_t Dx, int32_t Dy, r3m_dtype dtype) {
  if (n <= 0 || Dx < 0 || Dy < 0 || (dtype != R3M_SPEC_C64 && dtype != R3M_SPEC_C128)) return 0;
  return spectra_bytes(n, Dx, Dy, dtype);
}

int r3m_build_spectral(r3m_ctx ctx, const void* dense_dev, int32_t n, int32_t Dx, int32_t Dy, r3m_dtype dtype,
                       void* spec_dev, size_t spec_bytes, hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    R3M_REQUIRE(dense_dev && spec_dev, R3M_ERR_INVALID_ARG, "NULL buffer");
    R3M_REQUIRE(n > 0 && n <= 256 && Dx >= 0 && Dy >= 0, R3M_ERR_INVALID_ARG, "bad block shape");
    R3M_REQUIRE(dtype == R3M_SPEC_C64 || dtype == R3M_SPEC_C128, R3M_ERR_INVALID_ARG,
                "dtype must be R3M_SPEC_C64 or R3M_SPEC_C128");
    const int Gx = next_pow2(2 * Dx + 1), Gy = next_pow2(2 * Dy + 1);
    const int cap = dtype == R3M_SPEC_C128 ? 2048 : 4096;
    R3M_REQUIRE(Gx < cap && Gy < cap, R3M_ERR_UNSUPPORTED, "displacement extent too large for the transform");
    R3M_REQUIRE(spec_bytes >= spectra_bytes(n, Dx, Dy, dtype), R3M_ERR_BUFFER_TOO_SMALL,
                "spectra buffer too small");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    const int64_t total = (int64_t)n * n * Gx * Gy;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20);
    if (dtype == R3M_SPEC_C128) {
      hipLaunchKernelGGL(spec_embed_kernel<double>, dim3(blocks), dim3(256), 0, stream, (const double2*)dense_dev, n,
                         Dx, Dy, Gx, Gy, (C2<double>*)spec_dev);
      fft2<double>((C2<double>*)spec_dev, (int64_t)n * n, Gx, Gy, 0, stream, nullptr);
    } else {
      hipLaunchKernelGGL(spec_embed_kernel<float>, dim3(blocks), dim3(256), 0, stream, (const double2*)dense_dev, n,
                         Dx, Dy, Gx, Gy, (C2<float>*)spec_dev);
      fft2<float>((C2<float>*)spec_dev, (int64_t)n * n, Gx, Gy, 0, stream, nullptr);
    }
    R3M_CHECK_HIP(hipGetLastError());
  });
}

}  // extern "C"
