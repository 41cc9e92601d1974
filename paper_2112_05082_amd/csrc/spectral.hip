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
// (Sec. I cites this block-Toeplitz FFT route for periodic arrays, the array
// decomposition method.)
//
// Layouts (complex, interleaved; grids row-major, k = gy * Gx + gx):
//   spectra  Z^[m][n][Gy][Gx]     (m, n macro rows and columns)
//   work     X[b][n][Gy][Gx], then Y[b][n][Gy][Gx], then the relaxed
//            compaction's macro buffer [units][n]
#include "matvec_internal.h"

#include <algorithm>
#include <atomic>

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

// cos and sin of 2 pi m / 16
constexpr double kC1 = 0.92387953251128674;  // cos(pi / 8)
constexpr double kC2 = 0.70710678118654752;  // cos(pi / 4)
constexpr double kC3 = 0.38268343236508977;  // sin(pi / 8)
constexpr double kCos16[16] = {1, kC1, kC2, kC3, 0, -kC3, -kC2, -kC1, -1, -kC1, -kC2, -kC3, 0, kC3, kC2, kC1};
constexpr double kSin16[16] = {0, kC3, kC2, kC1, 1, kC1, kC2, kC3, 0, -kC3, -kC2, -kC1, -1, -kC1, -kC2, -kC3};

template <int LG>
__host__ __device__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 0; b < LG; ++b) r |= ((i >> b) & 1) << (LG - 1 - b);
  return r;
}

// in-register DFT of R <= 16 points, b_q = sum_r a_r exp(sgn 2 pi i r q / R)
// (iterative radix-2 decimation in time on the bit-reversed input)
template <typename T, int R, int SGN>
__device__ __forceinline__ void dft_regs(C2<T>* a) {
  constexpr int LG = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
  C2<T> b[R];
#pragma unroll
  for (int i = 0; i < R; ++i) b[bitrev<LG>(i)] = a[i];
#pragma unroll
  for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
    for (int i = 0; i < R; i += len) {
#pragma unroll
      for (int j = 0; j < len / 2; ++j) {
        const int m = j * (16 / len);  // twiddle exp(sgn 2 pi i m / 16)
        const C2<T> u = b[i + j], v = b[i + j + len / 2];
        C2<T> t;
        if (m == 0) {
          t = v;
        } else if (m == 4) {
          t = {-SGN * v.im, SGN * v.re};
        } else {
          const T c = (T)kCos16[m], sn = (T)(SGN * kSin16[m]);
          t = {v.re * c - v.im * sn, v.re * sn + v.im * c};
        }
        b[i + j] = {u.re + t.re, u.im + t.im};
        b[i + j + len / 2] = {u.re - t.re, u.im - t.im};
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = b[i];
}

// LDS position of element e of staged line li: lines S = G + G / 16 + 1
// apart (odd, so column staging spreads over the banks), one pad entry
// after every 16 elements (spreads the strided writes of the first stage)
__device__ __forceinline__ int lds_at(int li, int e, int S) { return li * S + e + (e >> 4); }

// One Stockham stage of radix R on the lines staged in LDS: with Ns the
// product of the earlier radices, item j < G / R of a line takes the inputs
// j + r G / R, multiplies input r by exp(sgn 2 pi i r k / (Ns R)) with
// k = j mod Ns, applies the R-point DFT and writes output q to
// (j / Ns) Ns R + k + q Ns.  A thread holds KE / R items in registers; the
// barrier between the reads and the writes lets the stage work in place.
template <typename T, int R, int KE, int SGN>
__device__ __forceinline__ void stockham_stage(C2<T>* buf, const C2<T>* tw, int lgG, int lgNs, int n_items, int S) {
  constexpr int LR = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
  constexpr int IT = KE / R;
  const int lgQ = lgG - LR;  // items per line = G / R
  const int Ns = 1 << lgNs;
  C2<T> a[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int item = threadIdx.x + it * 256;
    if (item < n_items) {
      const int li = item >> lgQ, j = item & ((1 << lgQ) - 1);
      const int k = j & (Ns - 1);
      const int tws = lgG - lgNs - LR;  // exp(sgn 2 pi i r k / (Ns R)) = tw[r k G / (Ns R)]
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C2<T> v = buf[lds_at(li, j + (r << lgQ), S)];
        if (r > 0) {
          const C2<T> w = tw[(r * k) << tws];
          v = {v.re * w.re - v.im * w.im, v.re * w.im + v.im * w.re};
        }
        a[it][r] = v;
      }
      dft_regs<T, R, SGN>(a[it]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int item = threadIdx.x + it * 256;
    if (item < n_items) {
      const int li = item >> lgQ, j = item & ((1 << lgQ) - 1);
      const int k = j & (Ns - 1);
      const int o = ((j >> lgNs) << (lgNs + LR)) + k;
#pragma unroll
      for (int q = 0; q < R; ++q) buf[lds_at(li, o + (q << lgNs), S)] = a[it][q];
    }
  }
  __syncthreads();
}

// Mixed-radix Stockham transforms of grid lines staged in LDS (forward:
// exp(-2 pi i j k / G); inverse: exp(+...), unnormalised), radix KE stages
// (16 in single, 8 in double precision) and one smaller stage for the rest
// of log2 G.  Grids are row-major Gy x Gx (element (gx, gy) at gy Gx + gx);
// a pass transforms every row (elements adjacent) or every column (elements
// Gx apart) of n_grids grids.  A workgroup takes lpw <= 256 KE / G adjacent
// lines of one grid: along rows consecutive threads move consecutive
// elements of a line, along columns the same element of consecutive lines,
// so both passes read and write HBM coalesced.  The twiddles exp(-+ 2 pi i m
// / G), m < G, are tabulated in LDS once per workgroup.  All extents are
// powers of two and the index arithmetic is shifts and masks.
//
// The retrieval passes fuse the masking of the product into the transforms
// (grid g = b n + c holds macro channel c of right-hand side b, whose array is
// Lx x Ly units at the grid's origin):
//   kFwdRows  rows from the compact input: entry (gx, gy) is x of unit
//             u = gy Lx + gx at row c - s_u n_a when that row is active
//             (0 <= c - s_u n_a < n_a), else zero; only rows gy < Ly are
//             written (the others are zero and never read);
//   kFwdCols  columns, rows gy >= Ly taken as zero;
//   kInvCols  columns, only rows gy < Ly written back;
//   kInvRows  rows gy < Ly, written straight to the compact output
//             (active rows only, times 1 / (Gx Gy)).
// With relaxed weights w[u][s] (a blended codebook) every channel c = s n_a + r
// is active: kFwdRows reads w[u][s] x[u][r], and kInvRows writes
// w[u][s] y~[u][c] / (Gx Gy) to a macro buffer whose sum over s is y[u][r].
enum FftMode { kPlainRows, kPlainCols, kFwdRows, kFwdCols, kInvCols, kInvRows };

template <typename T>
struct FftArgs {
  C2<T>* data;
  int lgG;      // log2 of the transform length
  int lg_lpg;   // log2 of the lines per grid (the other extent)
  int lg_lpw;   // log2 of the lines per workgroup (<= lg_lpg)
  const RhsDev* rhs;  // retrieval passes only
  const uint8_t* states;
  int n_states, n, n_a;
  // shared bases (connected geometries): macro rows [n_st, n) are in every
  // unit (ext: 0, or 1 / 2 masked in the array's first column / row); a
  // unit's compact vector has n_red = n_a + n - n_st entries
  int n_st, n_red;
  const int* ext;
  const void* x;  // kFwdRows
  void* y;        // kInvRows
  // relaxed retrieval (nullable): state weights [unit][n_states] replace the
  // one-hot state test; kInvRows then writes the weighted channels to
  // ymacro [unit][n] (summed over states afterwards)
  const double* wts;
  C2<T>* ymacro;
  int macro_plain;  // kInvRows with wts: write y~ itself (the macro product Z P(w) x), no weights
  const int* live;
  const int* idle;  // per right-hand side (nullable): lines of b with idle[b] != 0 are left alone
};

template <typename T>
constexpr int fft_ke() {
  return sizeof(T) == 4 ? 16 : 8;
}

template <typename T, int MODE, typename VT>
__global__ void __launch_bounds__(256) fft_kernel(FftArgs<T> A) {
  if (A.live && *A.live == 0) return;
  constexpr bool rows = MODE == kPlainRows || MODE == kFwdRows || MODE == kInvRows;
  constexpr bool masked = MODE >= kFwdRows;
  // the compacting row passes take one row of lpw consecutive channels (grids)
  // of one right-hand side, so that the compact vector is read (kFwdRows) or
  // written (kInvRows) in runs of adjacent rows A(s) of a unit; the other
  // passes take lpw adjacent lines of one grid
  constexpr bool chan = MODE == kFwdRows || MODE == kInvRows;
  // thread -> (line, element) maps: line-fastest for columns and for the
  // compact side of the compacting passes, element-fastest otherwise
  constexpr bool load_lf = !rows || MODE == kFwdRows;
  constexpr bool store_lf = !rows || MODE == kInvRows;
  constexpr int SGN = MODE == kInvCols || MODE == kInvRows ? 1 : -1;
  constexpr int KE = fft_ke<T>();
  extern __shared__ unsigned char smem_raw[];
  const int lgG = A.lgG, G = 1 << lgG;
  const int S = G + (G >> 4) + 1;
  const int lpw = 1 << A.lg_lpw;
  const int lgG2 = lgG + A.lg_lpg;
  const int lgGx = rows ? lgG : A.lg_lpg;
  int64_t g0;  // grid of line 0; line li lies in grid g0 + li (chan) or g0
  int lig0;    // its line within the grid; line li is lig0 (chan) or lig0 + li
  if (chan) {
    const int ncg = A.n >> A.lg_lpw;
    const int64_t id = blockIdx.x;
    const int cg = (int)(id % ncg);
    const int64_t rest = id / ncg;
    lig0 = (int)(rest & ((1 << A.lg_lpg) - 1));
    g0 = (rest >> A.lg_lpg) * A.n + ((int64_t)cg << A.lg_lpw);
  } else {
    const int64_t l0 = (int64_t)blockIdx.x << A.lg_lpw;
    g0 = l0 >> A.lg_lpg;
    lig0 = (int)(l0 & ((1 << A.lg_lpg) - 1));
  }
  int Lx = 0, Ly = 0, c0 = 0;
  RhsDev R{};
  if (masked) {
    const int b = (int)(g0 / A.n);
    c0 = (int)(g0 - (int64_t)b * A.n);
    R = A.rhs[b];
    Lx = R.Lx;
    Ly = R.Ly;
    if (chan && lig0 >= Ly) return;  // a row past the array
  }
  // a workgroup's lines belong to one right-hand side (grids are [B][n])
  if (A.idle && A.idle[g0 / A.n]) return;
  // the compact row of channel c in unit u = gy Lx + gx: -1 when c is not a
  // row of the unit's state, -2 for an extended basis masked by D_k (its
  // output is zero)
  auto active = [&](int64_t u, int gx, int gy, int c) -> int {
    if (c >= A.n_st) {
      const int e = A.ext[c - A.n_st];
      return e == 0 || (e == 1 && gx > 0) || (e == 2 && gy > 0) ? A.n_a + c - A.n_st : -2;
    }
    const int s = min((int)A.states[R.state_off + u], A.n_states - 1);
    const int r = c - s * A.n_a;
    return r >= 0 && r < A.n_a ? r : -1;
  };
  auto grid_at = [&](int li, int gx, int gy) -> C2<T>* {
    return A.data + ((g0 + (chan ? li : 0)) << lgG2) + ((int64_t)gy << lgGx) + gx;
  };
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* tw = buf + (size_t)lpw * S;
  for (int m = threadIdx.x; m < G; m += blockDim.x) {
    T sn, cs;
    sincospi_t<T>((T)(2 * m) / (T)G, &sn, &cs);
    tw[m] = {cs, (T)SGN * sn};
  }
  const int tot = lpw << lgG;
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int li = load_lf ? t & (lpw - 1) : t >> lgG;
    const int e = load_lf ? t >> A.lg_lpw : t & (G - 1);
    const int line = chan ? lig0 : lig0 + li;
    const int gx = rows ? e : line, gy = rows ? line : e;
    C2<T> v = {0, 0};
    if (MODE == kFwdRows) {
      if (gx < Lx) {
        const int64_t u = (int64_t)gy * Lx + gx;
        if (A.wts) {
          const int c = c0 + li, s = c / A.n_a, r = c - s * A.n_a;
          const double wv = A.wts[(R.unit_off + u) * A.n_states + s];
          const VT* xv = (const VT*)A.x + ((R.unit_off + u) * A.n_a + r) * 2;
          v = {(T)(wv * (double)xv[0]), (T)(wv * (double)xv[1])};
        } else {
          const int r = active(u, gx, gy, c0 + li);
          if (r >= 0) {
            const VT* xv = (const VT*)A.x + ((R.unit_off + u) * A.n_red + r) * 2;
            v = {(T)xv[0], (T)xv[1]};
          }
        }
      }
    } else if (MODE == kFwdCols) {
      if (gy < Ly) v = *grid_at(li, gx, gy);
    } else {
      v = *grid_at(li, gx, gy);
    }
    buf[lds_at(li, e, S)] = v;
  }
  __syncthreads();
  constexpr int LKE = KE == 16 ? 4 : 3;
  int lgNs = 0;
  for (; lgNs + LKE <= lgG; lgNs += LKE) stockham_stage<T, KE, KE, SGN>(buf, tw, lgG, lgNs, tot >> LKE, S);
  switch (lgG - lgNs) {
    case 1: stockham_stage<T, 2, KE, SGN>(buf, tw, lgG, lgNs, tot >> 1, S); break;
    case 2: stockham_stage<T, 4, KE, SGN>(buf, tw, lgG, lgNs, tot >> 2, S); break;
    case 3: stockham_stage<T, 8, KE, SGN>(buf, tw, lgG, lgNs, tot >> 3, S); break;
    default: break;
  }
  const T scale = T(1) / (T)((int64_t)1 << lgG2);
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int li = store_lf ? t & (lpw - 1) : t >> lgG;
    const int e = store_lf ? t >> A.lg_lpw : t & (G - 1);
    const int line = chan ? lig0 : lig0 + li;
    const int gx = rows ? e : line, gy = rows ? line : e;
    const C2<T> v = buf[lds_at(li, e, S)];
    if (MODE == kInvRows) {
      if (gx < Lx) {
        const int64_t u = (int64_t)gy * Lx + gx;
        if (A.wts) {
          const int c = c0 + li, s = c / A.n_a;
          const T ws = (A.macro_plain ? T(1) : (T)A.wts[(R.unit_off + u) * A.n_states + s]) * scale;
          A.ymacro[(R.unit_off + u) * A.n + c] = {v.re * ws, v.im * ws};
        } else {
          const int r = active(u, gx, gy, c0 + li);
          if (r >= 0) {
            VT* yv = (VT*)A.y + ((R.unit_off + u) * A.n_red + r) * 2;
            yv[0] = (VT)(v.re * scale);
            yv[1] = (VT)(v.im * scale);
          } else if (r == -2) {
            VT* yv = (VT*)A.y + ((R.unit_off + u) * A.n_red + A.n_a + c0 + li - A.n_st) * 2;
            yv[0] = yv[1] = (VT)0;
          }
        }
      }
    } else if (MODE == kInvCols) {
      if (gy < Ly) *grid_at(li, gx, gy) = v;
    } else {
      *grid_at(li, gx, gy) = v;
    }
  }
}

int ilog2(int v) {
  int l = 0;
  while ((1 << (l + 1)) <= v) ++l;
  return l;
}

// lines per workgroup (log2): up to 256 KE elements per workgroup, at most
// the lines of one grid
template <typename T>
int fft_lpw_log(int lgG, int lg_lpg) {
  constexpr int LKE = fft_ke<T>() == 16 ? 4 : 3;
  return std::max(0, std::min(8 + LKE - lgG, lg_lpg));
}

// one pass over every row or column (by MODE) of n_grids Gy x Gx grids; the
// compacting row passes group lpw channels of one RHS instead (lpw the
// largest power of two dividing n that fits)
template <typename T, int MODE, typename VT>
void fft_pass(FftArgs<T> A, int lgGx, int lgGy, int64_t n_grids, hipStream_t s) {
  constexpr bool rows = MODE == kPlainRows || MODE == kFwdRows || MODE == kInvRows;
  constexpr bool chan = MODE == kFwdRows || MODE == kInvRows;
  A.lgG = rows ? lgGx : lgGy;
  A.lg_lpg = rows ? lgGy : lgGx;
  int64_t n_wg;
  if (chan) {
    constexpr int LKE = fft_ke<T>() == 16 ? 4 : 3;
    int lg = 0;
    while (lg < 8 + LKE - A.lgG && (A.n & ((2 << lg) - 1)) == 0) ++lg;
    A.lg_lpw = std::max(0, lg);
    n_wg = (n_grids >> A.lg_lpw) << A.lg_lpg;
  } else {
    A.lg_lpw = fft_lpw_log<T>(A.lgG, A.lg_lpg);
    n_wg = (n_grids << A.lg_lpg) >> A.lg_lpw;
  }
  const int G = 1 << A.lgG;
  const size_t lds = ((size_t)((size_t)1 << A.lg_lpw) * (G + (G >> 4) + 1) + G) * sizeof(C2<T>);
  hipLaunchKernelGGL((fft_kernel<T, MODE, VT>), dim3((unsigned)n_wg), dim3(256), lds, s, A);
  R3M_CHECK_HIP(hipGetLastError());
}

// ----------------------------------------------------- fused 2-D transforms
//
// Complex64 grids of up to 16,384 points: one workgroup holds a whole Gy x Gx
// grid in LDS (element (gx, gy) at gy Sx + gx + gx / 16 with Sx = Gx + Gx / 16
// + 1, the padding of lds_at) and runs the row and the column stages there, so
// that a grid crosses HBM once per direction; the two-pass form above writes
// it out between its passes and reads it back.
//   forward: the first row stage gathers the masked compact input straight
//            into registers (rows gy < Ly only: the others are zero), the
//            first column stage reads rows gy >= Ly as zero, and the last
//            column stage writes X^ to HBM;
//   inverse: the first column stage reads Y^ from HBM, the last column stage
//            keeps rows gy < Ly only, the row stages run on those rows and
//            the last one writes the active rows of the compact output
//            (times 1 / (Gx Gy)).
// Workgroups are persistent over the grids g = b n + c: the workgroups with
// id = x mod 8 (one XCD) take the contiguous eighth x of the grids,
// interleaved over it, so the consecutive channels of a right-hand side,
// which gather from (or scatter to) the same lines of its compact vector, are
// in flight together in one L2.
struct Fft2Args {
  C2<float>* grid;  // [B][n][Gy][Gx]
  const RhsDev* rhs;
  const uint8_t* states;
  int n_states, n, n_a;
  int lgGx, lgGy;
  int64_t n_grids;
  int n_st, n_red;  // shared bases, as in FftArgs
  const int* ext;
  const void* x;  // forward: compact input
  void* y;        // inverse: compact output
  const int* live;
  const int* idle;
  // the right-hand sides with work (nullable): rl[0..rl[B]) their indices;
  // the workgroups then visit only their grids (the list replaces idle)
  const int* rl;
  int B;
  // x and y by row (SoA): entry (unit u, row r) of RHS b at
  // unit_off n_red + r units + u, so that a grid's gather and scatter touch
  // consecutive units (written and read back by soa_transpose_kernel)
  int soa;
};

__device__ __forceinline__ int at2(int gx, int gy, int Sx) { return gy * Sx + gx + (gx >> 4); }

// One Stockham stage of radix R (the map of stockham_stage) over n_lines
// lines of length 2^lgG of the LDS grid: rows (line = gy, element = gx; a
// thread's items are adjacent elements of one line) or columns (line = gx,
// element = gy; adjacent threads take adjacent lines, so that a wave touches
// 64 adjacent columns, in LDS and in HBM alike).  GSRC: the inputs come from
// the HBM grid gm (row-major, Gx = 2^lg_lines columns) instead of LDS; GDST:
// the outputs go there.  Elements e >= nz read as zero and outputs at e >=
// keep are dropped (first forward and last inverse column stages).  A stage
// that writes LDS does so in place, after a barrier that follows every read,
// and ends with a barrier.  Up to 16 elements per thread.
template <int R, bool COLS, int SGN, bool GSRC, bool GDST>
__device__ __forceinline__ void stage2d(float2* __restrict__ buf, int Sx, const float2* __restrict__ tw,
                                        float2* __restrict__ gm, int lgG, int lgNs, int n_lines, int lg_lines,
                                        int nz, int keep) {
  constexpr int LR = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
  constexpr int IT = 16 / R;
  const int lgQ = lgG - LR;
  const int Ns = 1 << lgNs;
  const int n_items = n_lines << lgQ;
  const int tws = lgG - lgNs - LR;
  C2<float> a[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int item = threadIdx.x + it * blockDim.x;
    if (item < n_items) {
      const int li = COLS ? item & ((1 << lg_lines) - 1) : item >> lgQ;
      const int j = COLS ? item >> lg_lines : item & ((1 << lgQ) - 1);
      const int k = j & (Ns - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = j + (r << lgQ);
        const int gx = COLS ? li : e, gy = COLS ? e : li;
        float2 v = make_float2(0.f, 0.f);
        if (e < nz) v = GSRC ? gm[((int64_t)gy << lg_lines) + gx] : buf[at2(gx, gy, Sx)];
        if (r > 0 && lgNs > 0) {
          const float2 w = tw[(r * k) << tws];
          v = make_float2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
        }
        a[it][r] = {v.x, v.y};
      }
      dft_regs<float, R, SGN>(a[it]);
    }
  }
  if (!GDST) __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int item = threadIdx.x + it * blockDim.x;
    if (item < n_items) {
      const int li = COLS ? item & ((1 << lg_lines) - 1) : item >> lgQ;
      const int j = COLS ? item >> lg_lines : item & ((1 << lgQ) - 1);
      const int k = j & (Ns - 1);
      const int o = ((j >> lgNs) << (lgNs + LR)) + k;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int e = o + (q << lgNs);
        const int gx = COLS ? li : e, gy = COLS ? e : li;
        const float2 v = make_float2(a[it][q].re, a[it][q].im);
        if (GDST)
          gm[((int64_t)gy << lg_lines) + gx] = v;
        else if (e < keep)
          buf[at2(gx, gy, Sx)] = v;
      }
    }
  }
  if (!GDST) __syncthreads();
}

// Every stage of one direction of a G = 2^LG grid: radix-16 stages, then one
// of radix 2, 4 or 8 for the rest of LG.  GSRC: the first stage reads the HBM
// grid; GDST: the last one writes it; nz applies to the first stage, keep to
// the last.
template <bool COLS, int SGN, int LG, bool GSRC, bool GDST, int LGNS = 0>
__device__ __forceinline__ void line_stages(float2* buf, const float2* tw, float2* gm, int n_lines, int nz,
                                            int keep) {
  if constexpr (LGNS < LG) {
    constexpr int LR = LG - LGNS >= 4 ? 4 : LG - LGNS;
    constexpr bool first = LGNS == 0, last = LGNS + LR == LG;
    constexpr int G = 1 << LG, Sx = G + G / 16 + 1;
    stage2d<1 << LR, COLS, SGN, GSRC && first, GDST && last>(buf, Sx, tw, gm, LG, LGNS, n_lines, LG,
                                                             first ? nz : G, last ? keep : G);
    line_stages<COLS, SGN, LG, GSRC, GDST, LGNS + LR>(buf, tw, gm, n_lines, nz, keep);
  }
}

// Square grids G x G, G = 2^LG (the stores' transform grids for square arrays)
// one complex value of a compact vector (float or double pairs, aligned to
// the pair) as a single load or store
template <typename VT>
__device__ __forceinline__ float2 load_c2(const VT* p) {
  if constexpr (sizeof(VT) == 8) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    return make_float2((float)v.x, (float)v.y);
  } else {
    return *reinterpret_cast<const float2*>(p);
  }
}
template <typename VT>
__device__ __forceinline__ void store_c2(VT* p, float re, float im) {
  if constexpr (sizeof(VT) == 8)
    *reinterpret_cast<double2*>(p) = make_double2((double)re, (double)im);
  else
    *reinterpret_cast<float2*>(p) = make_float2(re, im);
}

template <int LG>
constexpr int fft2_threads() {
  return (1 << (2 * LG)) / 16 > 64 ? (1 << (2 * LG)) / 16 : 64;
}

template <bool INV, typename VT, int LG>
__global__ void __launch_bounds__(fft2_threads<LG>()) fft2_kernel(Fft2Args A) {
  if (A.live && *A.live == 0) return;
  constexpr int SGN = INV ? 1 : -1;
  constexpr int G = 1 << LG, Sx = G + G / 16 + 1;
  // threads; points of the rows gy < Ly <= G / 2 per thread (an array of
  // Ly rows has Ly - 1 <= Dy displacements and G >= 2 Dy + 1)
  constexpr int kNT = fft2_threads<LG>(), kPer = (G * G / 2 + kNT - 1) / kNT;
  extern __shared__ unsigned char smem_raw[];
  float2* buf = reinterpret_cast<float2*>(smem_raw);
  float2* tw = buf + G * Sx;
  for (int m = threadIdx.x; m < G; m += blockDim.x) {
    float sn, cs;
    sincospif((float)(2 * m) / (float)G, &sn, &cs);
    tw[m] = make_float2(cs, (float)SGN * sn);
  }
  const float scale = 1.0f / (float)(G * G);
  const int64_t n_grids = A.rl ? (int64_t)A.rl[A.B] * A.n : A.n_grids;
  const int64_t per_x = gridDim.x >> 3, span = (n_grids + 7) >> 3;
  const int64_t g_end = min(n_grids, ((int64_t)blockIdx.x & 7) * span + span);
  for (int64_t gi = ((int64_t)blockIdx.x & 7) * span + (blockIdx.x >> 3); gi < g_end; gi += per_x) {
    const int li = (int)(gi / A.n), c = (int)(gi - (int64_t)li * A.n);
    const int b = A.rl ? A.rl[li] : li;
    const int64_t g = (int64_t)b * A.n + c;
    if (!A.rl && A.idle && A.idle[b]) continue;  // uniform over the workgroup
    const RhsDev R = A.rhs[b];
    const int Lx = R.Lx, Ly = R.Ly;
    // channel c is row rc of state sc: a unit contributes (or receives) it
    // when its state byte is sc; a shared channel (c >= n_st) is compact row
    // rc of every unit, except where D_k masks an extended basis
    const bool shared = c >= A.n_st;
    const int sc = shared ? -1 : c / A.n_a;
    const int rc = shared ? A.n_a + c - A.n_st : c - sc * A.n_a;
    const int ec = shared ? A.ext[c - A.n_st] : 0;
    float2* grid = reinterpret_cast<float2*>(A.grid) + (g << (2 * LG));
    __syncthreads();  // the previous grid's last LDS reads (and the twiddle table) are done
    if (!INV) {
      // masked compact input -> rows gy < Ly of the LDS grid: every state
      // byte first, then every input, so that the loads overlap
      int sv[kPer];
#pragma unroll
      for (int i = 0; i < kPer; ++i) {
        const int t = threadIdx.x + i * kNT, gx = t & (G - 1), gy = t >> LG;
        const bool in = t < (Ly << LG) && gx < Lx;
        if (shared)
          sv[i] = in && (ec == 0 || (ec == 1 && gx > 0) || (ec == 2 && gy > 0)) ? sc : -2;
        else
          sv[i] = in ? (int)A.states[R.state_off + (int64_t)gy * Lx + gx] : -2;
      }
      float2 vv[kPer];
#pragma unroll
      for (int i = 0; i < kPer; ++i) {
        const int t = threadIdx.x + i * kNT, gx = t & (G - 1), gy = t >> LG;
        vv[i] = make_float2(0.f, 0.f);
        if (sv[i] == sc)
          vv[i] = load_c2<VT>((const VT*)A.x +
                              (A.soa ? R.unit_off * A.n_red + (int64_t)rc * Lx * Ly + (int64_t)gy * Lx + gx
                                     : (R.unit_off + (int64_t)gy * Lx + gx) * A.n_red + rc) * 2);
      }
#pragma unroll
      for (int i = 0; i < kPer; ++i) {
        const int t = threadIdx.x + i * kNT;
        if (t < (Ly << LG)) buf[at2(t & (G - 1), t >> LG, Sx)] = vv[i];
      }
      __syncthreads();
      line_stages<false, SGN, LG, false, false>(buf, tw, grid, Ly, G, G);
      line_stages<true, SGN, LG, false, true>(buf, tw, grid, G, Ly, G);
    } else {
      line_stages<true, SGN, LG, true, false>(buf, tw, grid, G, G, Ly);
      line_stages<false, SGN, LG, false, false>(buf, tw, grid, Ly, G, G);
      // active rows of units gx < Lx, gy < Ly -> compact output (state
      // bytes first, as for the input); masked shared rows receive zero
      int sv[kPer];
#pragma unroll
      for (int i = 0; i < kPer; ++i) {
        const int t = threadIdx.x + i * kNT, gx = t & (G - 1), gy = t >> LG;
        const bool in = t < (Ly << LG) && gx < Lx;
        if (shared)
          sv[i] = !in ? -2 : ec == 0 || (ec == 1 && gx > 0) || (ec == 2 && gy > 0) ? sc : -3;
        else
          sv[i] = in ? (int)A.states[R.state_off + (int64_t)gy * Lx + gx] : -2;
      }
#pragma unroll
      for (int i = 0; i < kPer; ++i) {
        const int t = threadIdx.x + i * kNT, gx = t & (G - 1), gy = t >> LG;
        if (sv[i] == sc || sv[i] == -3) {
          const float2 v = sv[i] == sc ? buf[at2(gx, gy, Sx)] : make_float2(0.f, 0.f);
          store_c2<VT>((VT*)A.y + (A.soa ? R.unit_off * A.n_red + (int64_t)rc * Lx * Ly + (int64_t)gy * Lx + gx
                                          : (R.unit_off + (int64_t)gy * Lx + gx) * A.n_red + rc) * 2,
                       v.x * scale,
                       v.y * scale);
        }
      }
    }
  }
}

// Compact vectors between the unit-major layout of the library ([unit][n_red]
// per RHS) and the row-major one of the fused transforms' gathers (SoA, see
// Fft2Args::soa), one 64-unit x 16-row tile per work item through LDS; the
// items of the right-hand sides of rl (a live list), else of every RHS whose
// idle flag is clear.
constexpr int kSoaU = 64, kSoaR = 16;
// batches from this many compact entries on take the row-major copies (two
// extra launches; on the 1,536-RHS batch the matvec takes 26.7 ms with them,
// copies included, against 28.0 ms gathering from the unit-major vectors)
constexpr int64_t kSoaMinEntries = (int64_t)1 << 20;
__device__ __forceinline__ int rhs_count_list(const int* rl, int B) { return rl ? rl[B] : B; }
template <typename VT, bool TO_SOA>
__global__ void __launch_bounds__(256)
soa_transpose_kernel(const RhsDev* __restrict__ rhs, const VT* __restrict__ in, VT* __restrict__ out, int n_red,
                     int64_t per, int n_rc, const int* __restrict__ rl, const int* __restrict__ idle, int B) {
  __shared__ VT tile[kSoaR][kSoaU + 1][2];
  const int64_t items = per * rhs_count_list(rl, B);
  for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {  // uniform over the block
    const int li = (int)(item / per);
    const int64_t rem = item - (int64_t)li * per;
    const int b = rl ? rl[li] : li;
    if (!rl && idle && idle[b]) continue;
    const RhsDev R = rhs[b];
    const int64_t units = (int64_t)R.Lx * R.Ly;
    const int64_t u0 = (rem / n_rc) * kSoaU;
    const int r0 = (int)(rem % n_rc) * kSoaR;
    if (u0 >= units) continue;
    const int64_t base = R.unit_off * n_red;
    __syncthreads();  // the previous item's tile reads are done
    for (int e = threadIdx.x; e < kSoaU * kSoaR; e += blockDim.x) {
      const int u = TO_SOA ? e / kSoaR : e % kSoaU, r = TO_SOA ? e % kSoaR : e / kSoaU;
      if (u0 + u < units && r0 + r < n_red) {
        const int64_t src = TO_SOA ? base + (u0 + u) * n_red + r0 + r : base + (int64_t)(r0 + r) * units + u0 + u;
        tile[r][u][0] = in[2 * src];
        tile[r][u][1] = in[2 * src + 1];
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kSoaU * kSoaR; e += blockDim.x) {
      const int u = TO_SOA ? e % kSoaU : e / kSoaR, r = TO_SOA ? e / kSoaU : e % kSoaR;
      if (u0 + u < units && r0 + r < n_red) {
        const int64_t dst = TO_SOA ? base + (int64_t)(r0 + r) * units + u0 + u : base + (u0 + u) * n_red + r0 + r;
        out[2 * dst] = tile[r][u][0];
        out[2 * dst + 1] = tile[r][u][1];
      }
    }
  }
}

template <typename VT, bool TO_SOA>
void soa_transpose(const BatchDesc& bd, const void* in, void* out, int n_red, const int* rl, const int* idle,
                   hipStream_t s) {
  const int n_rc = (n_red + kSoaR - 1) / kSoaR;
  const int64_t per = (int64_t)((bd.max_units + kSoaU - 1) / kSoaU) * n_rc;
  const int64_t items = per * bd.B;
  hipLaunchKernelGGL((soa_transpose_kernel<VT, TO_SOA>), dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(items, 8192))),
                     dim3(256), 0, s, bd.rhs, (const VT*)in, (VT*)out, n_red, per, n_rc, rl, idle, bd.B);
  R3M_CHECK_HIP(hipGetLastError());
}

// square grids from 4 x 4 to 128 x 128
bool fft2_fits(int lgGx, int lgGy) { return lgGx == lgGy && lgGx >= 2 && lgGx <= 7; }

size_t fft2_lds_bytes(int lgGx, int lgGy) {
  const size_t Gx = (size_t)1 << lgGx, Gy = (size_t)1 << lgGy;
  return (Gy * (Gx + (Gx >> 4) + 1) + Gx + Gy) * sizeof(C2<float>);
}

template <bool INV, typename VT, int LG>
void fft2_launch(const Fft2Args& A, hipStream_t s) {
  const int threads = fft2_threads<LG>();
  const size_t lds = fft2_lds_bytes(LG, LG);
  const int64_t nwg = std::min<int64_t>((A.n_grids + 7) / 8 * 8, 2048);
  // the LDS limit of the kernel, raised once per device (outside any capture
  // in practice: the first call on a device comes before a solve captures)
  static std::atomic<uint64_t> raised{0};
  int dev = 0;
  R3M_CHECK_HIP(hipGetDevice(&dev));
  const uint64_t bit = (uint64_t)1 << (dev & 63);
  if (!(raised.load() & bit)) {
    R3M_CHECK_HIP(hipFuncSetAttribute((const void*)fft2_kernel<INV, VT, LG>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    raised.fetch_or(bit);
  }
  hipLaunchKernelGGL((fft2_kernel<INV, VT, LG>), dim3((unsigned)nwg), dim3(threads), lds, s, A);
  R3M_CHECK_HIP(hipGetLastError());
}

template <bool INV, typename VT>
void fft2_pass(const Fft2Args& A, hipStream_t s) {
  switch (A.lgGx) {
    case 2: return fft2_launch<INV, VT, 2>(A, s);
    case 3: return fft2_launch<INV, VT, 3>(A, s);
    case 4: return fft2_launch<INV, VT, 4>(A, s);
    case 5: return fft2_launch<INV, VT, 5>(A, s);
    case 6: return fft2_launch<INV, VT, 6>(A, s);
    case 7: return fft2_launch<INV, VT, 7>(A, s);
    default: R3M_REQUIRE(false, R3M_ERR_UNSUPPORTED, "fused transform grid out of range");
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

// Y^[b][m][k] = sum_c Z^[m][c][k] X^[b][c][k]: one n x n product per
// frequency k.  A thread owns one frequency, MT rows and BC right-hand sides
// (2 MT BC accumulators); per column c it loads MT spectra entries and BC
// inputs.  The four waves of a workgroup take adjacent row tiles of the same
// 64 frequencies, so they read the same inputs close together (cache hits),
// and workgroup ids run over RHS chunks first, then row tiles, then
// frequency blocks, so the workgroups that share a slice of X^ or Z^ are in
// flight together.
// Transposed operator (TR): the macro system's transpose is block-Toeplitz
// with kernel Z(-d)^T, whose spectrum at frequency k is Z^(-k)^T, so entry
// (m, c) is read from Z^[c][m] at the mirrored frequency (-kx mod Gx, -ky mod
// Gy).
__device__ __forceinline__ int64_t mirror_freq(int64_t k, int lgGx, int lgGy) {
  const int64_t kx = k & ((1 << lgGx) - 1), ky = k >> lgGx;
  return ((((int64_t)1 << lgGy) - ky) & ((1 << lgGy) - 1)) << lgGx | ((((int64_t)1 << lgGx) - kx) & ((1 << lgGx) - 1));
}

template <typename T, int MT, int BC, bool TR>
__global__ void __launch_bounds__(256)
spec_product_kernel(const C2<T>* __restrict__ Zh, const C2<T>* __restrict__ Xh, C2<T>* __restrict__ Yh, int n,
                    int64_t K, int B, int n_mg, int lgGx, int lgGy, const int* __restrict__ live,
                    const int* __restrict__ idle) {
  if (live && *live == 0) return;
  const int nz = (B + BC - 1) / BC;
  const int64_t id = blockIdx.x;
  const int z = (int)(id % nz);
  const int64_t rest = id / nz;
  const int mg = (int)(rest % n_mg);
  const int64_t kb = rest / n_mg;
  const int64_t k = kb * 64 + (threadIdx.x & 63);
  const int m0 = (mg * 4 + (threadIdx.x >> 6)) * MT;
  if (k >= K || m0 >= n) return;
  const int b0 = z * BC;
  const int nb = min(BC, B - b0);
  if (idle) {  // nothing to do when every right-hand side of the chunk is idle
    bool any = false;
    for (int q = 0; q < nb; ++q) any |= idle[b0 + q] == 0;
    if (!any) return;
  }
  T ar[MT][BC], ai[MT][BC];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int q = 0; q < BC; ++q) ar[i][q] = ai[i][q] = 0;
  const int64_t kz = TR ? mirror_freq(k, lgGx, lgGy) : k;
  const C2<T>* xr = Xh + (size_t)b0 * n * K + k;
  const int mt = min(MT, n - m0);
  constexpr int kUnroll = MT * BC <= 4 ? 4 : 2;
#pragma unroll kUnroll
  for (int c = 0; c < n; ++c) {
    C2<T> zv[MT], xv[BC];
#pragma unroll
    for (int i = 0; i < MT; ++i)
      zv[i] = i < mt ? Zh[(TR ? (size_t)c * n + m0 + i : (size_t)(m0 + i) * n + c) * K + kz] : C2<T>{0, 0};
#pragma unroll
    for (int q = 0; q < BC; ++q) xv[q] = q < nb ? xr[((size_t)q * n + c) * K] : C2<T>{0, 0};
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int q = 0; q < BC; ++q) {
        ar[i][q] = fma(zv[i].re, xv[q].re, ar[i][q]);
        ar[i][q] = fma(-zv[i].im, xv[q].im, ar[i][q]);
        ai[i][q] = fma(zv[i].re, xv[q].im, ai[i][q]);
        ai[i][q] = fma(zv[i].im, xv[q].re, ai[i][q]);
      }
  }
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int q = 0; q < BC; ++q)
      if (i < mt && q < nb) Yh[((size_t)(b0 + q) * n + m0 + i) * K + k] = {ar[i][q], ai[i][q]};
}

// Matrix-core form of the same product for complex64 spectra and wide
// batches: per frequency Y^(k) = Z^(k) X^(k) is an (n x n) x (n x B) complex
// GEMM, taken as four real GEMMs (Re Y = Re Z Re X - Im Z Im X, Im Y = Re Z
// Im X + Im Z Re X) on 16x16x4 FP32 MFMA tiles (lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16]; result rows 4 (l / 16) + r, column l % 16).  A
// workgroup owns 4 KPW frequencies x 80 rows x 16 RB right-hand sides; wave
// w takes KPW adjacent frequencies for all five row tiles and RB tiles of 16
// right-hand sides (RB = 2 halves the spectra staged per product: the loads
// of a chunk, not the matrix cores, bound the kernel).  Columns are consumed
// in chunks of PC: the chunk is staged in LDS as [c][k][m] and [c][k][b] (rows
// contiguous per frequency, padded strides) while the next chunk is already
// in flight from global memory (runs of 4 KPW frequencies).  Results
// leave through LDS one row tile at a time, again as 16-frequency runs.
// Tile order.  The two frequency tiles that share the 128-byte lines of their
// 64-byte runs must meet in one L2 (workgroup i runs on XCD i mod 8):
//  - with fewer than 8 RHS tiles each XCD takes a contiguous range of
//    (frequency-tile pair, RHS tile, row group, tile of the pair), so a pair's
//    lines of the spectra and of X stay in its L2;
//  - with 8 or more, workgroup ids run over RHS tiles first and wrap around
//    the XCDs, so each XCD keeps the same RHS tiles for every frequency tile
//    and meets both halves of their X lines (the larger stream there).
// Inside a solve the tiles are those with a live right-hand side (a list
// built on the device each step), and the order follows their count: when
// few are left, the contiguous order spreads them over all eight XCDs,
// where the RHS-first order would put each tile on one XCD.  The count from
// which the RHS-first order is taken (rhs_first) is part of the plan.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f32x4 mfma_16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma_16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kPM = 80, kPB = 16;
constexpr int kZP = kPM + 1, kXP = kPB + 1;

// KPW frequencies per wave, 4 KPW per workgroup; PC columns per staged
// chunk; RB tiles of 16 right-hand sides per workgroup (each staged chunk of
// the spectra then feeds RB times the products)
// T = double: the FP64 16x16x4 matrix-core product of complex128 spectra
// (operands as FP32; the output rows of a lane interleave differently), one
// complex128 frequency per 16-byte access.
template <typename T, int KPW, int PC, int RB, bool TR>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 1
                                       : KPW == 2 && PC == 4 && RB == 1 ? 3 : KPW == 2 && RB == 2 ? 2
                                       : KPW == 1 && PC == 8 && RB == 2 ? 3 : 1)))
spec_product_mfma_kernel(const C2<T>* __restrict__ Zh, const C2<T>* __restrict__ Xh, C2<T>* __restrict__ Yh,
                         int n, int64_t K, int B, int n_mg, int n_bt, int64_t n_tiles, int lgGx, int lgGy,
                         const int* __restrict__ live, const int* __restrict__ idle,
                         const int* __restrict__ tile_list, const int* __restrict__ n_live, int rhs_first,
                         int lkg) {
  if (live && *live == 0) return;
  typedef T v4 __attribute__((ext_vector_type(4)));
  constexpr int PK = 4 * KPW;                   // frequencies per workgroup
  constexpr int LPK = PK == 8 ? 3 : PK == 16 ? 4 : 2;
  constexpr int YP = PK + 1;
  // output tile rows of one right-hand side, padded by one entry so that the
  // 16 lanes of a quarter-wave (16 right-hand sides, one row) write 16
  // different bank pairs (an unpadded stride of 16 YP entries is a multiple
  // of 128 bytes: every lane in one bank)
  constexpr int YB = 16 * YP + 1;
  constexpr int LPC = PC == 8 ? 3 : 2;
  constexpr int NB = kPB * RB, LNB = RB == 2 ? 5 : 4, XP = NB + 1;  // right-hand sides per workgroup
  // (a second staging buffer, which saves one barrier per chunk, measured
  // slower: 13.95 against 13.46 ms on the 1,536-RHS product)
  __shared__ C2<T> Zs[PC * PK * kZP];  // [c][k][m]; reused as the output tile [b][m][k]
  __shared__ C2<T> Xs[PC * PK * XP];   // [c][k][b]
  static_assert(16 * YB <= PC * PK * kZP, "output tile fits the staging buffer");
  // RHS tiles to cover: all n_bt, or the nl live ones of tile_list (the
  // launch is sized for both orders below), taken RB at a time
  const int nl = tile_list ? *n_live : n_bt;
  const int ng = (nl + RB - 1) / RB;  // groups of RB tiles
  int bi, mg;
  int64_t kt;
  if (nl < rhs_first) {
    const int64_t items = (n_tiles + 1) / 2 * 2 * n_mg * ng;
    const int64_t per = (items + 7) / 8, loc = blockIdx.x >> 3;  // grid: a multiple of 8
    if (loc >= per) return;
    const int64_t id = (int64_t)(blockIdx.x & 7) * per + loc;
    if (id >= items) return;
    const int kh = (int)(id & 1);
    const int64_t r0 = id >> 1;
    bi = (int)(r0 % ng);
    const int64_t r1 = r0 / ng;
    mg = (int)(r1 % n_mg);
    kt = (r1 / n_mg) * 2 + kh;
  } else {
    // RHS tile first: the eight XCDs (workgroup id mod 8) form KG = 2^lkg
    // groups of frequency-tile pairs times 8 / KG groups of RHS tiles; an
    // XCD runs its pairs in turn and, within a pair, its RHS tiles with the
    // pair's two halves adjacent, so that the spectra of a few frequency
    // tiles stay in its L2 while the RHS tiles pass (KG = 1: every XCD sees
    // every frequency tile, one RHS tile group in eight)
    const int KG = 1 << lkg, BG = 8 >> lkg;
    const int x = (int)(blockIdx.x & 7), kg = x & (KG - 1), bg = x >> lkg;
    const int nb_x = (ng - bg + BG - 1) / BG;  // RHS tile groups of this XCD
    const int64_t n_pairs = (n_tiles + 1) / 2, np_x = (n_pairs - kg + KG - 1) / KG;
    if (nb_x <= 0 || np_x <= 0) return;
    const int64_t l = blockIdx.x >> 3;
    const int kh = (int)(l & 1);
    const int64_t r0 = l >> 1;
    const int bj = (int)(r0 % nb_x);
    const int64_t r1 = r0 / nb_x;
    mg = (int)(r1 % n_mg);
    const int64_t pj = r1 / n_mg;
    if (pj >= np_x) return;
    kt = (pj * KG + kg) * 2 + kh;
    bi = bg + bj * BG;
  }
  if (kt >= n_tiles) return;  // n_tiles: frequency tiles
  const int64_t k0 = kt * PK;
  const int m0 = mg * kPM;
  // first right-hand side of each of the group's tiles (-1: past the last tile)
  int b0[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int ti = bi * RB + r;
    b0[r] = ti < nl ? (tile_list ? tile_list[ti] : ti) * kPB : -1;
  }
  if (idle && !tile_list) {  // uniform over the workgroup: skip a group of idle right-hand sides
    bool any = false;
#pragma unroll
    for (int r = 0; r < RB; ++r)
      if (b0[r] >= 0)
        for (int q = b0[r]; q < min(b0[r] + kPB, B); ++q) any |= idle[q] == 0;
    if (!any) return;
  }
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  v4 are[KPW][5][RB], aim[KPW][5][RB];
#pragma unroll
  for (int q = 0; q < KPW; ++q)
#pragma unroll
    for (int t = 0; t < 5; ++t)
#pragma unroll
      for (int r = 0; r < RB; ++r) are[q][t][r] = aim[q][t][r] = v4{0, 0, 0, 0};
  // loads of a chunk: VW adjacent frequencies each (one 16-byte load of two
  // complex64 values; the transposed operator reads mirrored frequencies one
  // at a time)
  constexpr int VW = TR || sizeof(T) == 8 ? 1 : 2, LPKV = VW == 2 ? LPK - 1 : LPK;
  constexpr int ZE = PC * PK * kPM / VW, XE = PC * PK * NB / VW;
  constexpr int NZ = (ZE + 255) / 256, NX = (XE + 255) / 256;
  struct alignas(sizeof(C2<T>) * VW) CV {
    C2<T> v[VW];
  };
  CV zp[NZ], xp[NX];
  auto load_chunk = [&](int c0) {
#pragma unroll
    for (int i = 0; i < NZ; ++i) {
      const int e = tid + 256 * i, k = (e & (PK / VW - 1)) * VW, c = (e >> LPKV) & (PC - 1),
                m = e >> (LPKV + LPC);
      const bool ok = e < ZE && m0 + m < n && c0 + c < n && k0 + k < K;
      if (TR) {
        zp[i].v[0] = ok ? Zh[((int64_t)(c0 + c) * n + m0 + m) * K + mirror_freq(k0 + k, lgGx, lgGy)]
                        : C2<T>{0, 0};
      } else {
        const CV* src = reinterpret_cast<const CV*>(Zh + ((int64_t)(m0 + m) * n + c0 + c) * K + k0 + k);
        if (ok) zp[i] = *src;
        else
#pragma unroll
          for (int v = 0; v < VW; ++v) zp[i].v[v] = C2<T>{0, 0};
      }
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int e = tid + 256 * i, k = (e & (PK / VW - 1)) * VW, c = (e >> LPKV) & (PC - 1),
                b = e >> (LPKV + LPC);
      const int bb = (RB == 1 ? b0[0] : b0[(b >> 4) & (RB - 1)]) + (b & 15);
      const bool ok = e < XE && (RB == 1 ? b0[0] : b0[(b >> 4) & (RB - 1)]) >= 0 && bb < B && c0 + c < n &&
                      k0 + k < K;
      const CV* src = reinterpret_cast<const CV*>(Xh + ((int64_t)bb * n + c0 + c) * K + k0 + k);
      if (ok) xp[i] = *src;
      else
#pragma unroll
        for (int v = 0; v < VW; ++v) xp[i].v[v] = C2<T>{0, 0};
    }
  };
  load_chunk(0);
  for (int c0 = 0; c0 < n; c0 += PC) {
    __syncthreads();  // the previous chunk's fragments have been read
#pragma unroll
    for (int i = 0; i < NZ; ++i) {
      const int e = tid + 256 * i, k = (e & (PK / VW - 1)) * VW, c = (e >> LPKV) & (PC - 1),
                m = e >> (LPKV + LPC);
      if (e < ZE)
#pragma unroll
        for (int v = 0; v < VW; ++v) Zs[(c * PK + k + v) * kZP + m] = zp[i].v[v];
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int e = tid + 256 * i, k = (e & (PK / VW - 1)) * VW, c = (e >> LPKV) & (PC - 1),
                b = e >> (LPKV + LPC);
      if (e < XE)
#pragma unroll
        for (int v = 0; v < VW; ++v) Xs[(c * PK + k + v) * XP + b] = xp[i].v[v];
    }
    __syncthreads();
    if (c0 + PC < n) load_chunk(c0 + PC);
#pragma unroll
    for (int cs = 0; cs < PC / 4; ++cs) {
      const int c = cs * 4 + (lane >> 4);  // the fragment's column of the chunk
#pragma unroll
      for (int q = 0; q < KPW; ++q) {
        const int kk = w * KPW + q;
        C2<T> bv[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) bv[r] = Xs[(c * PK + kk) * XP + r * 16 + (lane & 15)];
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          const C2<T> av = Zs[(c * PK + kk) * kZP + t * 16 + (lane & 15)];
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            are[q][t][r] = mfma_16x16x4(av.re, bv[r].re, are[q][t][r]);
            are[q][t][r] = mfma_16x16x4(-av.im, bv[r].im, are[q][t][r]);
            aim[q][t][r] = mfma_16x16x4(av.re, bv[r].im, aim[q][t][r]);
            aim[q][t][r] = mfma_16x16x4(av.im, bv[r].re, aim[q][t][r]);
          }
        }
      }
    }
  }
  C2<T>* Ys = Zs;  // [b 16 (stride YB)][m 16][k YP]
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if (b0[r] < 0) break;  // uniform over the workgroup
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < KPW; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          // accumulator entry i of a lane: row 4 (lane / 16) + i (FP32) or
          // 4 i + lane / 16 (FP64), column lane % 16
          const int m = sizeof(T) == 4 ? 4 * (lane >> 4) + i : 4 * i + (lane >> 4), b = lane & 15;
          Ys[b * YB + m * YP + w * KPW + q] = {are[q][t][r][i], aim[q][t][r][i]};
        }
      __syncthreads();
      // YW adjacent frequencies per 16-byte store
      constexpr int YW = 16 / sizeof(C2<T>), LYW = YW == 2 ? 1 : 0;
#pragma unroll
      for (int i = 0; i < (16 * 16 * PK / YW + 255) / 256; ++i) {
        const int e = tid + 256 * i, k = (e & (PK / YW - 1)) * YW, m = (e >> (LPK - LYW)) & 15,
                  b = e >> (LPK - LYW + 4);
        const int row = m0 + t * 16 + m;
        if (e < 16 * 16 * PK / YW && b0[r] + b < B && row < n && k0 + k < K) {
          struct alignas(16) Y2 {
            C2<T> v[YW];
          } y2;
#pragma unroll
          for (int v = 0; v < YW; ++v) y2.v[v] = Ys[b * YB + m * YP + k + v];
          *reinterpret_cast<Y2*>(Yh + ((int64_t)(b0[r] + b) * n + row) * K + k0 + k) = y2;
        }
      }
    }
  }
  (void)LNB;
}

// The live tiles of the matrix-core product (tiles of kPB right-hand sides
// with any idle[b] == 0) in increasing order, and their count: one workgroup,
// thread t takes a contiguous run of tiles, a scan of the counts places them.
__global__ void __launch_bounds__(1024)
live_tiles_kernel(const int* __restrict__ idle, int B, int n_bt, int* __restrict__ list, int* __restrict__ n_live) {
  __shared__ int cnt[1024];
  const int t = threadIdx.x;
  const int per = (n_bt + 1023) / 1024;
  const int t0 = min(n_bt, t * per), t1 = min(n_bt, t0 + per);
  auto is_live = [&](int bt) {
    for (int q = bt * kPB; q < min(bt * kPB + kPB, B); ++q)
      if (idle[q] == 0) return true;
    return false;
  };
  int c = 0;
  for (int bt = t0; bt < t1; ++bt) c += is_live(bt) ? 1 : 0;
  cnt[t] = c;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? cnt[t - o] : 0;
    __syncthreads();
    cnt[t] += v;
    __syncthreads();
  }
  int at = cnt[t] - c;
  for (int bt = t0; bt < t1; ++bt)
    if (is_live(bt)) list[at++] = bt;
  if (t == 1023) *n_live = cnt[1023];
}

template <typename T, int MT, int BC>
void launch_product(const C2<T>* Zh, const C2<T>* X, C2<T>* Y, int n, int64_t G2, int B, bool tr, int lgGx,
                    int lgGy, hipStream_t s, const int* live, const int* idle) {
  const int n_mg = (n + 4 * MT - 1) / (4 * MT);
  const int64_t nwg = (G2 + 63) / 64 * n_mg * ((B + BC - 1) / BC);
  if (tr)
    hipLaunchKernelGGL((spec_product_kernel<T, MT, BC, true>), dim3((unsigned)nwg), dim3(256), 0, s, Zh, X, Y, n, G2,
                       B, n_mg, lgGx, lgGy, live, idle);
  else
    hipLaunchKernelGGL((spec_product_kernel<T, MT, BC, false>), dim3((unsigned)nwg), dim3(256), 0, s, Zh, X, Y, n,
                       G2, B, n_mg, lgGx, lgGy, live, idle);
}

// The matrix-core product with KPW frequencies per wave and PC columns per
// staged chunk.  tl: room for the live-tile list (ceil(B / 16) + 1 ints),
// used with idle flags on batches of at least rhs_first RHS tiles; with the
// list the kernel picks the order from the live count, so the grid covers
// both orders.
template <typename T, int KPW, int PC, int RB>
void launch_product_mfma(const C2<T>* Zh, const C2<T>* X, C2<T>* Y, int n, int64_t G2, int B, bool tr,
                         int lgGx, int lgGy, hipStream_t s, const int* live, const int* idle, int* tl, int rf,
                         int lkg) {
  constexpr int PK = 4 * KPW;
  const int n_mg = (n + kPM - 1) / kPM, n_bt = (B + kPB - 1) / kPB;
  const int64_t n_kt = (G2 + PK - 1) / PK;
  const bool use_list = idle && tl && n_bt >= rf;
  // groups of RB tiles in each order (the contiguous order runs below rf live tiles)
  const int ng_c = ((use_list ? std::min(rf - 1, n_bt) : n_bt) + RB - 1) / RB, ng = (n_bt + RB - 1) / RB;
  const int64_t nwg_c = ((n_kt + 1) / 2 * 2 * n_mg * ng_c + 7) / 8 * 8;
  const int KG = 1 << lkg, BG = 8 >> lkg;
  const int64_t nwg_r = 8 * (((n_kt + 1) / 2 + KG - 1) / KG) * n_mg * ((ng + BG - 1) / BG) * 2;
  const int64_t nwg = use_list ? std::max(nwg_c, nwg_r) : n_bt < rf ? nwg_c : nwg_r;
  const int* list = use_list ? tl : nullptr;
  const int* cnt = use_list ? tl + n_bt : nullptr;
  if (use_list) {
    hipLaunchKernelGGL(live_tiles_kernel, dim3(1), dim3(1024), 0, s, idle, B, n_bt, tl, tl + n_bt);
    R3M_CHECK_HIP(hipGetLastError());
  }
  if (tr)
    hipLaunchKernelGGL((spec_product_mfma_kernel<T, KPW, PC, RB, true>), dim3((unsigned)nwg), dim3(256), 0, s, Zh, X,
                       Y, n, G2, B, n_mg, n_bt, n_kt, lgGx, lgGy, live, idle, list, cnt, rf, lkg);
  else
    hipLaunchKernelGGL((spec_product_mfma_kernel<T, KPW, PC, RB, false>), dim3((unsigned)nwg), dim3(256), 0, s, Zh, X,
                       Y, n, G2, B, n_mg, n_bt, n_kt, lgGx, lgGy, live, idle, list, cnt, rf, lkg);
  R3M_CHECK_HIP(hipGetLastError());
}

// Per-frequency product by plan (a valid spectral plan).  The vector-unit
// kernel takes its register tile by batch width: 2 rows for one or two
// right-hand sides (a stream of the spectra wants many waves in flight), 4
// rows x 4 or 8 right-hand sides otherwise (arithmetic per load).  Every
// matrix-core shape sums each output over the columns in the same order (16x16x4
// tiles of four consecutive columns, in increasing column order), so all of
// them give the same bits.
template <typename T>
void product(const C2<T>* Zh, const C2<T>* X, C2<T>* Y, int n, int64_t G2, int B, bool tr, int lgGx, int lgGy,
             hipStream_t s, const int* live, const int* idle, int* tl, int plan) {
  if constexpr (sizeof(T) == 4) {
    const C2<float>*zf = Zh, *xf = X;
    C2<float>* yf = Y;
    const int rf = spec_rhs_first(plan), lkg = spec_kt_groups(plan);
    switch (spec_shape(plan)) {
      case 1: return launch_product_mfma<float, 1, 4, 1>(zf, xf, yf, n, G2, B, tr, lgGx, lgGy, s, live, idle, tl, rf, lkg);
      case 2: return launch_product_mfma<float, 2, 4, 1>(zf, xf, yf, n, G2, B, tr, lgGx, lgGy, s, live, idle, tl, rf, lkg);
      case 3: return launch_product_mfma<float, 2, 8, 1>(zf, xf, yf, n, G2, B, tr, lgGx, lgGy, s, live, idle, tl, rf, lkg);
      case 4: return launch_product_mfma<float, 4, 4, 1>(zf, xf, yf, n, G2, B, tr, lgGx, lgGy, s, live, idle, tl, rf, lkg);
      case 5: return launch_product_mfma<float, 1, 8, 1>(zf, xf, yf, n, G2, B, tr, lgGx, lgGy, s, live, idle, tl, rf, lkg);
      case 6: return launch_product_mfma<float, 2, 4, 2>(zf, xf, yf, n, G2, B, tr, lgGx, lgGy, s, live, idle, tl, rf, lkg);
      case 7: return launch_product_mfma<float, 1, 8, 2>(zf, xf, yf, n, G2, B, tr, lgGx, lgGy, s, live, idle, tl, rf, lkg);
      default: break;
    }
  } else {
    // complex128 spectra: the FP64 matrix cores at every batch width (one
    // summation order per output, so a batched product matches its single
    // right-hand sides bit for bit)
    return launch_product_mfma<double, 1, 4, 1>(Zh, X, Y, n, G2, B, tr, lgGx, lgGy, s, live, idle, tl,
                                                 spec_rhs_first(plan), spec_kt_groups(plan));
  }
  if (B == 1)
    launch_product<T, 2, 1>(Zh, X, Y, n, G2, B, tr, lgGx, lgGy, s, live, idle);
  else if (B == 2)
    launch_product<T, 2, 2>(Zh, X, Y, n, G2, B, tr, lgGx, lgGy, s, live, idle);
  else if (B <= 4)
    launch_product<T, 4, 4>(Zh, X, Y, n, G2, B, tr, lgGx, lgGy, s, live, idle);
  else
    launch_product<T, 4, 8>(Zh, X, Y, n, G2, B, tr, lgGx, lgGy, s, live, idle);
}

// relaxed compaction: y[u][r] = sum over states s of ymacro[u][s n_a + r]
// (fixed order), per RHS b = blockIdx.y
template <typename T, typename YT>
__global__ void __launch_bounds__(256)
relaxed_sum_kernel(const RhsDev* __restrict__ rhs, const C2<T>* __restrict__ ym, int n, int n_a, int n_states,
                   YT* __restrict__ y, const int* __restrict__ idle) {
  if (idle && idle[blockIdx.y]) return;
  const RhsDev R = rhs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)R.Lx * R.Ly * n_a) return;
  const int64_t u = e / n_a;
  const int r = (int)(e - u * n_a);
  const C2<T>* p = ym + (R.unit_off + u) * n + r;
  T re = 0, im = 0;
  for (int s = 0; s < n_states; ++s) {
    re += p[s * n_a].re;
    im += p[s * n_a].im;
  }
  YT* yv = y + (R.unit_off * n_a + e) * 2;
  yv[0] = (YT)re;
  yv[1] = (YT)im;
}

size_t spectral_list_offset(const BatchDesc& bd, const r3m_store* Z) {
  const size_t es = Z->far_dtype == R3M_SPEC_C128 ? 16 : 8;
  const size_t G2 = (size_t)next_pow2(2 * Z->Dx + 1) * next_pow2(2 * Z->Dy + 1);
  return (2 * (size_t)bd.B * Z->n * G2 * es + (size_t)bd.total_units * Z->n * es + 255) / 256 * 256;
}

template <typename T, typename XT, typename YT>
void spectral_typed(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, const void* x, void* y,
                    void* work, hipStream_t s, const int* live, const double* wts = nullptr, bool tr = false,
                    C2<T>* macro_out = nullptr, const int* idle = nullptr, int plan = 0,
                    const int* rl = nullptr) {
  const int n = Z->n;
  const int lgGx = ilog2(next_pow2(2 * Z->Dx + 1)), lgGy = ilog2(next_pow2(2 * Z->Dy + 1));
  const int64_t G2 = (int64_t)1 << (lgGx + lgGy);
  const int B = bd.B;
  C2<T>* X = (C2<T>*)work;
  C2<T>* Y = X + (size_t)B * n * G2;
  FftArgs<T> A{};
  A.rhs = bd.rhs;
  A.states = states;
  A.n_states = Z->n_states;
  A.n = n;
  A.n_st = n - Z->n_common;
  A.n_a = A.n_st / Z->n_states;
  A.n_red = A.n_a + Z->n_common;
  A.ext = Z->common_ext;
  A.x = x;
  A.y = y;
  A.wts = wts;
  A.ymacro = macro_out ? macro_out : wts ? Y + (size_t)B * n * G2 : nullptr;  // relaxed: [units][n] after Y
  A.macro_plain = macro_out ? 1 : 0;
  A.live = live;
  A.idle = idle;
  const int64_t ng = (int64_t)B * n;
  if (!(plan & kPlanSpectral)) plan = spectral_default_plan(Z, B);
  // the fused 2-D transforms where the grid fits LDS (complex64, retrieval)
  const bool fused = sizeof(T) == 4 && !wts && !macro_out && !(plan & kPlanSpecTwoPass) && fft2_fits(lgGx, lgGy);
  if (fused)
    for (int b = 0; b < B; ++b)
      R3M_REQUIRE(2 * bd.Ly[b] <= (1 << lgGy) && bd.Lx[b] <= (1 << lgGx), R3M_ERR_INVALID_ARG,
                  "array larger than the store's displacement range");
  Fft2Args F{};
  if (fused) {
    F.rhs = bd.rhs;
    F.states = states;
    F.n_states = Z->n_states;
    F.n = n;
    F.n_a = A.n_a;
    F.n_st = A.n_st;
    F.n_red = A.n_red;
    F.ext = A.ext;
    F.lgGx = lgGx;
    F.lgGy = lgGy;
    F.n_grids = ng;
    F.x = x;
    F.y = y;
    F.live = live;
    F.idle = idle;
    F.rl = rl;
    F.B = B;
    F.grid = (C2<float>*)X;
    // wide batches gather from (and scatter to) row-major copies of the
    // compact vectors: x's in the output grids' space (free until the
    // product), y's in the input grids' space (free after it)
    F.soa = (int64_t)bd.total_units * A.n_red >= kSoaMinEntries;
    if (F.soa) {
      soa_transpose<XT, true>(bd, x, Y, A.n_red, rl, idle, s);
      F.x = Y;
    }
    fft2_pass<false, XT>(F, s);
  } else {
    A.data = X;
    fft_pass<T, kFwdRows, XT>(A, lgGx, lgGy, ng, s);
    fft_pass<T, kFwdCols, XT>(A, lgGx, lgGy, ng, s);
  }
  int* tl = (int*)((char*)work + spectral_list_offset(bd, Z));
  product<T>((const C2<T>*)Z->far, X, Y, n, G2, B, tr, lgGx, lgGy, s, live, idle, tl, plan);
  if (fused) {
    F.grid = (C2<float>*)Y;
    if (F.soa) F.y = X;
    fft2_pass<true, YT>(F, s);
    if (F.soa) soa_transpose<YT, false>(bd, X, y, A.n_red, rl, idle, s);
  } else {
    A.data = Y;
    fft_pass<T, kInvCols, YT>(A, lgGx, lgGy, ng, s);
    fft_pass<T, kInvRows, YT>(A, lgGx, lgGy, ng, s);
  }
  if (wts && !macro_out) {
    hipLaunchKernelGGL((relaxed_sum_kernel<T, YT>), dim3(ceil_div((size_t)bd.max_units * A.n_a, 256), B), dim3(256),
                       0, s, bd.rhs, (const C2<T>*)A.ymacro, n, A.n_a, A.n_states, (YT*)y, idle);
    R3M_CHECK_HIP(hipGetLastError());
  }
}

// dJ/dw[u][s] = dJ[b] 2 Re sum_r [ (G - Q)[u][s n_a + r] I[u][r]
//                                 + lam[u][r] (U - ZI)[u][s n_a + r] ]
// with Q = Z^T P(w) lam and ZI = Z P(w) I (macro layout [unit][n]), per RHS
// b = blockIdx.y, one thread per (unit, state)
__global__ void __launch_bounds__(256)
relaxed_grad_kernel(const RhsDev* __restrict__ rhs, const double2* __restrict__ I, const double2* __restrict__ lam,
                    const double2* __restrict__ G, const double2* __restrict__ U, const double2* __restrict__ ZI,
                    const double2* __restrict__ Q, const double* __restrict__ dJ, int n_a, int n_states,
                    double* __restrict__ grad) {
  const int b = blockIdx.y;
  const RhsDev R = rhs[b];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)R.Lx * R.Ly * n_states) return;
  const int64_t u = e / n_states;
  const int st = (int)(e - u * n_states);
  const int n = n_a * n_states;
  const double2* Iu = I + (R.unit_off + u) * n_a;
  const double2* lu = lam + (R.unit_off + u) * n_a;
  const size_t mb = (size_t)(R.unit_off + u) * n + (size_t)st * n_a;
  double acc = 0.0;
  for (int r = 0; r < n_a; ++r) {
    const double2 gq = make_double2(G[mb + r].x - Q[mb + r].x, G[mb + r].y - Q[mb + r].y);
    const double2 rr = make_double2(U[mb + r].x - ZI[mb + r].x, U[mb + r].y - ZI[mb + r].y);
    acc += gq.x * Iu[r].x - gq.y * Iu[r].y;
    acc += lu[r].x * rr.x - lu[r].y * rr.y;
  }
  grad[(R.unit_off + u) * n_states + st] = (dJ ? dJ[b] : 1.0) * 2.0 * acc;
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

// X and Y grids, then the relaxed compaction's macro buffer [units][n], then
// the live-tile list of the matrix-core product
size_t spectral_work_bytes(const BatchDesc& bd, const r3m_store* Z) {
  return spectral_list_offset(bd, Z) + ((size_t)(bd.B + kPB - 1) / kPB + 1) * sizeof(int) + 256;
}

void launch_spectral_ex(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, r3m_dtype x_type,
                        const void* x, r3m_dtype y_type, void* y, void* work, hipStream_t s, const int* live,
                        const double* wts, bool tr, const int* idle, int plan) {
  const bool xd = x_type == R3M_C128, yd = y_type == R3M_C128;
  if (Z->far_dtype == R3M_SPEC_C128) {
    R3M_REQUIRE(xd && yd, R3M_ERR_UNSUPPORTED, "complex128 spectra need C128 vectors");
    spectral_typed<double, double, double>(Z, bd, states, x, y, work, s, live, wts, tr, nullptr, idle, plan);
  } else if (xd && yd) {
    spectral_typed<float, double, double>(Z, bd, states, x, y, work, s, live, wts, tr, nullptr, idle, plan);
  } else if (!xd && yd) {
    spectral_typed<float, float, double>(Z, bd, states, x, y, work, s, live, wts, tr, nullptr, idle, plan);
  } else if (!xd && !yd) {
    spectral_typed<float, float, float>(Z, bd, states, x, y, work, s, live, wts, tr, nullptr, idle, plan);
  } else {
    R3M_REQUIRE(false, R3M_ERR_UNSUPPORTED, "C128 input with C64 output");
  }
}

void launch_spectral(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, r3m_dtype x_type,
                     const void* x, r3m_dtype y_type, void* y, void* work, hipStream_t s, const int* live,
                     const int* idle, int plan, const int* rl) {
  const bool xd = x_type == R3M_C128, yd = y_type == R3M_C128;
  if (Z->far_dtype == R3M_SPEC_C64 && !xd) {  // the solver's forms: the list reaches the transforms
    if (yd)
      spectral_typed<float, float, double>(Z, bd, states, x, y, work, s, live, nullptr, false, nullptr, idle, plan, rl);
    else
      spectral_typed<float, float, float>(Z, bd, states, x, y, work, s, live, nullptr, false, nullptr, idle, plan, rl);
    return;
  }
  launch_spectral_ex(Z, bd, states, x_type, x, y_type, y, work, s, live, nullptr, false, idle, plan);
}

int spectral_default_plan(const r3m_store* Z, int B) {
  return spec_plan(Z->far_dtype == R3M_SPEC_C64 && B >= 12 ? 2 : 0, kSpecRhsFirst);
}

bool spectral_plan_valid(const r3m_store* Z, int plan) {
  const int shape = spec_shape(plan), rf = spec_rhs_first(plan);
  return (plan & ~(kPlanSpectral | kPlanSpecTwoPass | (3 << 13) | 0xfff)) == 0 && (plan & kPlanSpectral) &&
         shape < kSpecShapeCount && rf >= 1 && (shape == 0 || Z->far_dtype == R3M_SPEC_C64);
}

bool spectral_fused_transforms(const r3m_store* Z) {
  return Z->far_dtype == R3M_SPEC_C64 &&
         fft2_fits(ilog2(next_pow2(2 * Z->Dx + 1)), ilog2(next_pow2(2 * Z->Dy + 1)));
}

size_t relaxed_work_bytes(const BatchDesc& bd, const r3m_store* Z) { return spectral_work_bytes(bd, Z); }

void launch_spectral_product(const r3m_store* Z, const BatchDesc& bd, void* work, int plan, hipStream_t s) {
  const int lgGx = ilog2(next_pow2(2 * Z->Dx + 1)), lgGy = ilog2(next_pow2(2 * Z->Dy + 1));
  const int64_t G2 = (int64_t)1 << (lgGx + lgGy);
  if (!(plan & kPlanSpectral)) plan = spectral_default_plan(Z, bd.B);
  int* tl = (int*)((char*)work + spectral_list_offset(bd, Z));
  const size_t grid = (size_t)bd.B * Z->n * G2;
  if (Z->far_dtype == R3M_SPEC_C128) {
    C2<double>* X = (C2<double>*)work;
    product<double>((const C2<double>*)Z->far, X, X + grid, Z->n, G2, bd.B, false, lgGx, lgGy, s, nullptr, nullptr,
                    tl, plan);
  } else {
    C2<float>* X = (C2<float>*)work;
    product<float>((const C2<float>*)Z->far, X, X + grid, Z->n, G2, bd.B, false, lgGx, lgGy, s, nullptr, nullptr, tl,
                   plan);
  }
}

}  // namespace r3m

using namespace r3m;

extern "C" {

size_t r3m_relaxed_gradient_work_bytes(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch) {
  size_t out = 0;
  int rc = guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    require_isolated(Z);
    R3M_REQUIRE(Z->far_dtype == R3M_SPEC_C128, R3M_ERR_UNSUPPORTED, "the gradient needs complex128 spectra");
    validate_batch(batch, Z->Dx, Z->Dy);
    if (batch->B == 0) return;
    const BatchDesc& bd = get_batch(ctx, batch, 8, 8, 0);
    out = (spectral_work_bytes(bd, Z) + 255) / 256 * 256 + 2 * (size_t)bd.total_units * Z->n * 16;
  });
  return rc == R3M_OK ? out : 0;
}

int r3m_relaxed_gradient(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, const double* weights_dev,
                         const void* I_dev, const void* lam_dev, const void* G_dev, const void* U_dev,
                         const double* dJ_dev, double* grad_dev, void* work_dev, size_t work_bytes,
                         hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    require_isolated(Z);
    R3M_REQUIRE(Z->far_dtype == R3M_SPEC_C128, R3M_ERR_UNSUPPORTED, "the gradient needs complex128 spectra");
    validate_batch(batch, Z->Dx, Z->Dy);
    if (batch->B == 0) return;
    R3M_REQUIRE(weights_dev && I_dev && lam_dev && G_dev && U_dev && grad_dev && work_dev, R3M_ERR_INVALID_ARG,
                "NULL buffer");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    const BatchDesc& bd = get_batch(ctx, batch, 8, 8, stream);
    const size_t sw = (spectral_work_bytes(bd, Z) + 255) / 256 * 256;
    const size_t mac = (size_t)bd.total_units * Z->n;
    R3M_REQUIRE(work_bytes >= sw + 2 * mac * 16, R3M_ERR_BUFFER_TOO_SMALL, "gradient workspace too small");
    C2<double>* ZI = (C2<double>*)((char*)work_dev + sw);
    C2<double>* Q = ZI + mac;
    spectral_typed<double, double, double>(Z, bd, batch->states, I_dev, nullptr, work_dev, stream, nullptr,
                                           weights_dev, false, ZI);
    spectral_typed<double, double, double>(Z, bd, batch->states, lam_dev, nullptr, work_dev, stream, nullptr,
                                           weights_dev, true, Q);
    const int n_a = Z->n / Z->n_states;
    hipLaunchKernelGGL(relaxed_grad_kernel, dim3(ceil_div((size_t)bd.max_units * Z->n_states, 256), bd.B), dim3(256),
                       0, stream, bd.rhs, (const double2*)I_dev, (const double2*)lam_dev, (const double2*)G_dev,
                       (const double2*)U_dev, (const double2*)ZI, (const double2*)Q, dJ_dev, n_a, Z->n_states,
                       grad_dev);
    R3M_CHECK_HIP(hipGetLastError());
  });
}

size_t r3m_relaxed_work_bytes(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch) {
  size_t out = 0;
  int rc = guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    require_isolated(Z);
    R3M_REQUIRE(store_is_spectral(Z), R3M_ERR_UNSUPPORTED, "relaxed retrieval needs a spectral store");
    validate_batch(batch, Z->Dx, Z->Dy);
    if (batch->B == 0) return;
    out = relaxed_work_bytes(get_batch(ctx, batch, 8, 8, 0), Z);
  });
  return rc == R3M_OK ? out : 0;
}

int r3m_relaxed_matvec(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, const double* weights_dev,
                       int32_t transpose, r3m_dtype vec_dtype, const void* x_dev, void* y_dev, void* work_dev,
                       size_t work_bytes, hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    require_isolated(Z);
    R3M_REQUIRE(store_is_spectral(Z), R3M_ERR_UNSUPPORTED, "relaxed retrieval needs a spectral store");
    validate_batch(batch, Z->Dx, Z->Dy);
    R3M_REQUIRE(vec_dtype == R3M_C128 || vec_dtype == R3M_C64, R3M_ERR_UNSUPPORTED, "vectors must be C128 or C64");
    if (batch->B == 0) return;
    R3M_REQUIRE(x_dev && y_dev && weights_dev && work_dev, R3M_ERR_INVALID_ARG, "NULL buffer");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    const BatchDesc& bd = get_batch(ctx, batch, 8, 8, stream);
    R3M_REQUIRE(work_bytes >= relaxed_work_bytes(bd, Z), R3M_ERR_BUFFER_TOO_SMALL, "relaxed workspace too small");
    launch_spectral_ex(Z, bd, batch->states, vec_dtype, x_dev, vec_dtype, y_dev, work_dev, stream, nullptr,
                       weights_dev, transpose != 0);
  });
}

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
      FftArgs<double> A{};
      A.data = (C2<double>*)spec_dev;
      fft_pass<double, kPlainRows, double>(A, ilog2(Gx), ilog2(Gy), (int64_t)n * n, stream);
      fft_pass<double, kPlainCols, double>(A, ilog2(Gx), ilog2(Gy), (int64_t)n * n, stream);
    } else {
      hipLaunchKernelGGL(spec_embed_kernel<float>, dim3(blocks), dim3(256), 0, stream, (const double2*)dense_dev, n,
                         Dx, Dy, Gx, Gy, (C2<float>*)spec_dev);
      FftArgs<float> A{};
      A.data = (C2<float>*)spec_dev;
      fft_pass<float, kPlainRows, float>(A, ilog2(Gx), ilog2(Gy), (int64_t)n * n, stream);
      fft_pass<float, kPlainCols, float>(A, ilog2(Gx), ilog2(Gy), (int64_t)n * n, stream);
    }
    R3M_CHECK_HIP(hipGetLastError());
  });
}

}  // extern "C"
