// Near-field block ILU(0) preconditioner of the retrieved system (Sec. III-D).
//
// The paper preconditions the retrieved system with an incomplete LU of its
// near field, factored per codebook after retrieval (a factor of a retrieved
// matrix is not the retrieval of a factor, so nothing is shared across
// codebooks).  Here the blocks are whole units (n_a x n_a), the pattern holds
// the unit pairs at Chebyshev lattice distance <= r, nothing outside it is
// kept (ILU(0)), and units are taken in multicolour order: unit (ix, iy) has
// colour (iy mod (r+1)) (r+1) + (ix mod (r+1)).  No two units of one colour
// are in each other's pattern, so every colour is one parallel launch of the
// factorisation and of each triangular solve; the order inside a colour does
// not change the factors.
//
// Factor layout (per global unit g, S = (2r+1)^2 blocks): the block of the
// neighbour at offset e = (ex, ey) sits in slot (ey + r)(2r+1) + (ex + r) and
// holds the multiplier L_gj (j of a lower colour), the upper block U_gj (j of
// a higher colour) or, at e = 0, the inverted pivot U_gg^-1.  Blocks are
// column-major (element (row, col) at col * n_a + row, the layout the
// triangular solves read with consecutive lanes on consecutive rows), complex
// in the store precision; blocks of neighbours outside the array are zero.
//
// Work per unit: the factorisation costs about (lower neighbours) x (shared
// pattern blocks) block products of n_a^3 complex MACs; each application
// reads every factor block once (S n_a^2 complex values per unit).
#include "matvec_internal.h"
#include "small_dense.h"

#include <algorithm>

namespace r3m {

namespace {

constexpr int kIluMaxRadius = 3;

template <typename T>
struct Cx;
template <>
struct Cx<float> {
  using t2 = float2;
};
template <>
struct Cx<double> {
  using t2 = double2;
};

__device__ inline double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
__device__ inline double2 to_d2(double2 v) { return v; }
template <typename T2>
__device__ inline T2 from_d2(double2 v);
template <>
__device__ inline float2 from_d2<float2>(double2 v) {
  return make_float2((float)v.x, (float)v.y);
}
template <>
__device__ inline double2 from_d2<double2>(double2 v) {
  return v;
}

__device__ inline void cmac(double2& acc, double2 a, double2 b) {
  acc.x += a.x * b.x - a.y * b.y;
  acc.y += a.x * b.y + a.y * b.x;
}

__device__ inline int colour_of(int ix, int iy, int r) { return (iy % (r + 1)) * (r + 1) + (ix % (r + 1)); }

// The unit of colour `colour` taken by workgroup blockIdx.x of RHS
// blockIdx.y (ncx colour columns per row of the largest array); false when it
// lies outside this RHS's array (uniform over the workgroup).
__device__ inline bool colour_unit(const RhsDev& R, int r, int colour, int ncx, int& ix, int& iy) {
  const int cx = colour % (r + 1), cy = colour / (r + 1);
  ix = cx + (int)(blockIdx.x % ncx) * (r + 1);
  iy = cy + (int)(blockIdx.x / ncx) * (r + 1);
  return ix < R.Lx && iy < R.Ly;
}

// Retrieval of the near-field pattern blocks: F[g][e] = Z(p_g - p_j)[A(s_g),
// A(s_j)] for the neighbour j = g + e, transposed to column-major through
// LDS (rows read along the store's rows, columns written along F's).  With
// relaxed weights wts ([global unit][n_states]) the block is the blend
// sum_{s,s'} w[g][s] w[j][s'] Z(p_g - p_j)[A(s), A(s')], or with transpose
// that of the transposed operator, sum w[g][s] w[j][s'] Z(p_j - p_g)[A(s'), A(s)]^T.
// Grid (max units * S, B); dynamic LDS n_a (n_a + 1) T2.
template <typename T>
__global__ void __launch_bounds__(256)
ilu_fill_kernel(const T* __restrict__ near, int n, int Nx, int Ny, int n_a, int n_states,
                const RhsDev* __restrict__ rhs, const uint8_t* __restrict__ states, int r,
                typename Cx<T>::t2* __restrict__ F, const double* __restrict__ wts, int transpose, int shared) {
  using T2 = typename Cx<T>::t2;
  extern __shared__ double2 ilu_lds[];  // typed: 16-byte aligned after any static LDS
  T2* tile = reinterpret_cast<T2*>(ilu_lds);  // [n_a][n_a + 1]
  const RhsDev R = rhs[blockIdx.y];
  const int S = (2 * r + 1) * (2 * r + 1);
  const int64_t u = blockIdx.x / S;
  const int e = blockIdx.x % S;
  if (u >= (int64_t)R.Lx * R.Ly || (shared && !R.fac_lead)) return;
  const int ix = (int)(u % R.Lx), iy = (int)(u / R.Lx);
  const int ex = e % (2 * r + 1) - r, ey = e / (2 * r + 1) - r;
  const int jx = ix + ex, jy = iy + ey;
  T2* dst = F + ((size_t)((shared ? R.fac_off : R.unit_off) + u) * S + e) * n_a * n_a;
  const int nn = n_a * n_a;
  if (jx < 0 || jx >= R.Lx || jy < 0 || jy >= R.Ly) {
    for (int q = threadIdx.x; q < nn; q += blockDim.x) dst[q] = from_d2<T2>(make_double2(0.0, 0.0));
    return;
  }
  if (wts) {
    const double* wg = wts + (R.unit_off + u) * n_states;
    const double* wj = wts + (R.unit_off + (int64_t)jy * R.Lx + jx) * n_states;
    // observer g, source j: displacement p_g - p_j = -e; the transpose reads +e
    const int sx = transpose ? ex : -ex, sy = transpose ? ey : -ey;
    const T* blk = near + ((size_t)(sy + Ny) * (2 * Nx + 1) + (sx + Nx)) * n * n * 2;
    for (int q = threadIdx.x; q < nn; q += blockDim.x) {
      const int col = q / n_a, row = q % n_a;
      double re = 0.0, im = 0.0;
      for (int s1 = 0; s1 < n_states; ++s1)
        for (int s2 = 0; s2 < n_states; ++s2) {
          const size_t idx = transpose ? (size_t)(s2 * n_a + col) * n + s1 * n_a + row
                                       : (size_t)(s1 * n_a + row) * n + s2 * n_a + col;
          const double ww = wg[s1] * wj[s2];
          re += ww * (double)blk[2 * idx];
          im += ww * (double)blk[2 * idx + 1];
        }
      dst[q] = from_d2<T2>(make_double2(re, im));
    }
    return;
  }
  const int si = min((int)states[R.state_off + u], n_states - 1);
  const int sj = min((int)states[R.state_off + (int64_t)jy * R.Lx + jx], n_states - 1);
  // observer g, source j: displacement p_g - p_j = -e (|e| <= r <= near radius)
  const size_t slot = (size_t)(-ey + Ny) * (2 * Nx + 1) + (-ex + Nx);
  const T* blk = near + slot * n * n * 2;
  for (int q = threadIdx.x; q < nn; q += blockDim.x) {
    const int row = q / n_a, col = q % n_a;
    const size_t idx = (size_t)(si * n_a + row) * n + sj * n_a + col;
    T2 v;
    v.x = blk[2 * idx];
    v.y = blk[2 * idx + 1];
    tile[row * (n_a + 1) + col] = v;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nn; q += blockDim.x) {
    const int col = q / n_a, row = q % n_a;
    dst[q] = tile[row * (n_a + 1) + col];
  }
}

// One colour step of the factorisation: every unit i of colour `colour`
// (one workgroup of kFactorThreads threads each) eliminates its lower-colour neighbours
// k in colour order: L_ik = A_ik U_kk^-1, then A_ij -= L_ik U_kj for every
// neighbour j of i of a colour above k's whose offset from k is in the
// pattern; finally the pivot A_ii is inverted (Gauss-Jordan, FP64).  Rows of
// lower colours are final when this launch runs.  Each thread owns the same
// kPer entries of every n_a x n_a product (column-major index q = tid + NT t),
// so all of its global loads of a block are issued together.  Dynamic LDS
// (2 n_a^2 + n_a + 1) double2.
constexpr int kFactorThreads = 512;

template <typename T, int NA>
__global__ void __launch_bounds__(kFactorThreads)
ilu_factor_kernel(const RhsDev* __restrict__ rhs, int r, int colour, int ncx, typename Cx<T>::t2* __restrict__ F,
                  int* __restrict__ flag, int shared) {
  using T2 = typename Cx<T>::t2;
  constexpr int NT = kFactorThreads;
  constexpr int n_a = NA, nn = NA * NA, kPer = (NA * NA + NT - 1) / NT;
  // products in 2 x 2 register blocks: rows {rb, rb + H}, columns {cb, cb + H}
  constexpr int H = NA / 2, kBlk = (H * H + NT - 1) / NT;
  extern __shared__ double2 ilu_lds[];  // typed: 16-byte aligned after any static LDS
  __shared__ int piv_row;
  const RhsDev R = rhs[blockIdx.y];
  int ix, iy;
  if (!colour_unit(R, r, colour, ncx, ix, iy) || (shared && !R.fac_lead)) return;
  const int W = 2 * r + 1, S = W * W;
  const int tid = threadIdx.x;
  const int64_t fb = shared ? R.fac_off : R.unit_off;  // first factor unit of this codebook
  const int64_t g = fb + (int64_t)iy * R.Lx + ix;
  T2* Fi = F + (size_t)g * S * nn;
  double2* Ls = ilu_lds;   // current multiplier, column-major, FP64
  double2* Bs = Ls + nn;   // pivot inverse or U_kj, column-major, FP64

  // c[b][e] = sum_m Ls[row][m] Bs[m][col] for entry e of this thread's block b
  // (e: bit 0 selects row rb + H, bit 1 column cb + H)
  auto product = [&](double2 (&c)[kBlk][4]) {
#pragma unroll
    for (int b = 0; b < kBlk; ++b) {
      const int blk = tid + b * NT;
      double2 a00 = make_double2(0.0, 0.0), a10 = a00, a01 = a00, a11 = a00;
      if (blk < H * H) {
        const int rb = blk % H, cb = blk / H;
#pragma unroll 4
        for (int m = 0; m < n_a; ++m) {
          const double2 l0 = Ls[m * n_a + rb], l1 = Ls[m * n_a + rb + H];
          const double2 b0 = Bs[cb * n_a + m], b1 = Bs[(cb + H) * n_a + m];
          cmac(a00, l0, b0);
          cmac(a10, l1, b0);
          cmac(a01, l0, b1);
          cmac(a11, l1, b1);
        }
      }
      c[b][0] = a00;
      c[b][1] = a10;
      c[b][2] = a01;
      c[b][3] = a11;
    }
  };
  auto entry = [&](int b, int e) {  // column-major index of entry e of block b
    const int blk = tid + b * NT;
    const int rb = blk % H, cb = blk / H;
    return (cb + (e >> 1) * H) * n_a + rb + (e & 1) * H;
  };

  double2 acc[kBlk][4];
  for (int ck = 0; ck < colour; ++ck) {
    for (int ek = 0; ek < S; ++ek) {
      const int kx = ix + ek % W - r, ky = iy + ek / W - r;
      if (kx < 0 || kx >= R.Lx || ky < 0 || ky >= R.Ly || colour_of(kx, ky, r) != ck) continue;
      const T2* Fk = F + (size_t)(fb + (int64_t)ky * R.Lx + kx) * S * nn;
      // multiplier L_ik = A_ik D_k (D_k: k's inverted pivot, centre slot)
#pragma unroll
      for (int t = 0; t < kPer; ++t) {
        const int q = tid + t * NT;
        if (q < nn) {
          Ls[q] = to_d2(Fi[(size_t)ek * nn + q]);
          Bs[q] = to_d2(Fk[(size_t)(S / 2) * nn + q]);
        }
      }
      __syncthreads();
      product(acc);
      __syncthreads();
#pragma unroll
      for (int b = 0; b < kBlk; ++b) {
        if (tid + b * NT < H * H) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int q = entry(b, e);
            Ls[q] = acc[b][e];
            Fi[(size_t)ek * nn + q] = from_d2<T2>(acc[b][e]);
          }
        }
      }
      // A_ij -= L_ik U_kj for the later part of row k inside i's pattern
      const int dkx = ek % W - r, dky = ek / W - r;
      for (int ej = 0; ej < S; ++ej) {
        const int ejx = ej % W - r, ejy = ej / W - r;
        const int jx = ix + ejx, jy = iy + ejy;
        if (jx < 0 || jx >= R.Lx || jy < 0 || jy >= R.Ly || colour_of(jx, jy, r) <= ck) continue;
        const int ox = ejx - dkx, oy = ejy - dky;  // offset of j from k
        if (ox < -r || ox > r || oy < -r || oy > r) continue;
        __syncthreads();  // Bs free (and Ls complete)
        const int okj = (oy + r) * W + (ox + r);
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
          const int q = tid + t * NT;
          if (q < nn) Bs[q] = to_d2(Fk[(size_t)okj * nn + q]);
        }
        T2 old[kBlk][4];
#pragma unroll
        for (int b = 0; b < kBlk; ++b)
          if (tid + b * NT < H * H)
#pragma unroll
            for (int e = 0; e < 4; ++e) old[b][e] = Fi[(size_t)ej * nn + entry(b, e)];
        __syncthreads();
        product(acc);
#pragma unroll
        for (int b = 0; b < kBlk; ++b) {
          if (tid + b * NT < H * H) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const double2 o = to_d2(old[b][e]);
              Fi[(size_t)ej * nn + entry(b, e)] = from_d2<T2>(make_double2(o.x - acc[b][e].x, o.y - acc[b][e].y));
            }
          }
        }
      }
      __syncthreads();
    }
  }
  // invert the pivot A_ii in FP64 (its last update is this workgroup's own)
  __syncthreads();
  double2* aug = reinterpret_cast<double2*>(ilu_lds);  // [n_a][2 n_a], then a column
  double2* colk = aug + 2 * nn;
  constexpr int w2 = 2 * NA;
  const T2* Aii = Fi + (size_t)(S / 2) * nn;
  for (int q = tid; q < n_a * w2; q += NT) {
    const int row = q / w2, c = q % w2;
    aug[q] = c < n_a ? to_d2(Aii[(size_t)c * n_a + row]) : make_double2(c - n_a == row ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  if (!gj_invert<NA, NT>(aug, colk, &piv_row, flag)) return;
  T2* Dst = Fi + (size_t)(S / 2) * nn;
  for (int q = tid; q < nn; q += NT) {
    const int col = q / n_a, row = q % n_a;
    Dst[q] = from_d2<T2>(aug[row * w2 + n_a + col]);
  }
}

// launch shape of the triangular solves: waves per unit, and the parts each
// neighbour block's columns are split into (work items dealt to the waves)
#ifndef R3M_ILU_APPLY_WAVES
#define R3M_ILU_APPLY_WAVES 8
#endif
#ifndef R3M_ILU_APPLY_PARTS
#define R3M_ILU_APPLY_PARTS 2
#endif
constexpr int kApplyWaves = R3M_ILU_APPLY_WAVES;

// Sum over the neighbour blocks of unit (ix, iy) whose colour is below
// (lower) or above `colour` of  B_ij v_j  (v: [unit][n_a] complex double;
// units of colour 0 are read from v0 instead).
// Work items are (block, part of its columns), dealt to the workgroup's
// waves in turn, lane = row.  Leaves the row sums in red[0..n_a) (LDS
// [kApplyWaves][64] double2).
template <int NA, typename T2>
__device__ inline void neighbour_sum(const RhsDev& R, int r, int colour, bool lower, int ix, int iy,
                                     const T2* __restrict__ Fi, const double2* __restrict__ v0,
                                     const double2* __restrict__ v, double2* red) {
  constexpr int n_a = NA, kParts = R3M_ILU_APPLY_PARTS, kCols = NA / kParts;
  const int W = 2 * r + 1, S = W * W, nn = n_a * n_a;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  double2 acc = make_double2(0.0, 0.0);
  int item = 0;
  for (int e = 0; e < S; ++e) {
    const int jx = ix + e % W - r, jy = iy + e / W - r;
    if (jx < 0 || jx >= R.Lx || jy < 0 || jy >= R.Ly) continue;
    const int cj = colour_of(jx, jy, r);
    if (lower ? cj >= colour : cj <= colour) continue;
    for (int part = 0; part < kParts; ++part) {
      if (item++ % kApplyWaves != wave) continue;
      if (lane < n_a) {
        const T2* Bk = Fi + (size_t)e * nn + (size_t)part * kCols * n_a;
        const double2* vj = (cj == 0 ? v0 : v) + (size_t)(R.unit_off + (int64_t)jy * R.Lx + jx) * n_a + part * kCols;
#pragma unroll
        for (int c = 0; c < kCols; ++c) cmac(acc, to_d2(Bk[(size_t)c * n_a + lane]), vj[c]);
      }
    }
  }
  red[wave * 64 + lane] = acc;
  __syncthreads();
  if (wave == 0) {
    double2 s = red[lane];
#pragma unroll
    for (int q = 1; q < kApplyWaves; ++q) {
      s.x += red[q * 64 + lane].x;
      s.y += red[q * 64 + lane].y;
    }
    red[lane] = s;
  }
  __syncthreads();
}

// x_i = D_i t (t: LDS [64]) into z_i and, when given, out_i (OT: float or
// double); the columns of D_i are dealt to the waves.
template <int NA, typename T2, typename OT>
__device__ inline void pivot_solve(const T2* __restrict__ D, const double2* t, double2* red, int64_t g,
                                   double2* __restrict__ z, OT* __restrict__ out) {
  constexpr int n_a = NA;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  double2 acc = make_double2(0.0, 0.0);
  if (lane < n_a)
#pragma unroll
    for (int c = wave; c < n_a; c += kApplyWaves) cmac(acc, to_d2(D[(size_t)c * n_a + lane]), t[c]);
  red[wave * 64 + lane] = acc;
  __syncthreads();
  if (wave == 0 && lane < n_a) {
    double2 s = red[lane];
#pragma unroll
    for (int q = 1; q < kApplyWaves; ++q) {
      s.x += red[q * 64 + lane].x;
      s.y += red[q * 64 + lane].y;
    }
    z[g * n_a + lane] = s;
    if (out) {
      out[2 * (g * n_a + lane)] = (OT)s.x;
      out[2 * (g * n_a + lane) + 1] = (OT)s.y;
    }
  }
}

// Forward step of colour `colour` (>= 1; colour 0 has z = in and is never
// stored): z_i = in_i - sum over lower neighbours k of L_ik z_k.  For the last
// colour (no upper neighbours) the backward step follows in the same launch:
// x_i = U_ii^-1 z_i.  One workgroup per unit of the colour.
template <typename T, int NA, typename OT>
__global__ void __launch_bounds__(64 * kApplyWaves)
ilu_forward_kernel(const RhsDev* __restrict__ rhs, int r, int colour, int ncx, int last, int shared,
                   const typename Cx<T>::t2* __restrict__ F, const double2* __restrict__ in, double2* __restrict__ z,
                   OT* __restrict__ out, const int* __restrict__ live) {
  constexpr int n_a = NA;
  __shared__ double2 red[kApplyWaves * 64];
  __shared__ double2 t[64];
  if (live && *live == 0) return;
  const RhsDev R = rhs[blockIdx.y];
  int ix, iy;
  if (!colour_unit(R, r, colour, ncx, ix, iy)) return;
  const int S = (2 * r + 1) * (2 * r + 1), nn = n_a * n_a;
  const int64_t g = R.unit_off + (int64_t)iy * R.Lx + ix;  // vectors
  const typename Cx<T>::t2* Fi =
      F + (size_t)((shared ? R.fac_off : R.unit_off) + (int64_t)iy * R.Lx + ix) * S * nn;
  neighbour_sum<NA>(R, r, colour, true, ix, iy, Fi, in, z, red);
  if (threadIdx.x < n_a) {
    const double2 a = in[g * n_a + threadIdx.x], s = red[threadIdx.x];
    const double2 zi = make_double2(a.x - s.x, a.y - s.y);
    if (last)
      t[threadIdx.x] = zi;
    else
      z[g * n_a + threadIdx.x] = zi;
  }
  if (last) {
    __syncthreads();
    pivot_solve<NA>(Fi + (size_t)(S / 2) * nn, t, red, g, z, out);
  }
}

// Backward step of colour `colour`: x_i = U_ii^-1 (z_i - sum over upper
// neighbours j of U_ij x_j), written over z_i (x_j of higher colours are
// already there; z_i of colour 0 is in_i) and, when out is given, into out.
template <typename T, int NA, typename OT>
__global__ void __launch_bounds__(64 * kApplyWaves)
ilu_backward_kernel(const RhsDev* __restrict__ rhs, int r, int colour, int ncx, int shared,
                    const typename Cx<T>::t2* __restrict__ F, const double2* __restrict__ in, double2* __restrict__ z,
                    OT* __restrict__ out, const int* __restrict__ live) {
  using T2 = typename Cx<T>::t2;
  constexpr int n_a = NA;
  __shared__ double2 red[kApplyWaves * 64];
  __shared__ double2 t[64];
  if (live && *live == 0) return;
  const RhsDev R = rhs[blockIdx.y];
  int ix, iy;
  if (!colour_unit(R, r, colour, ncx, ix, iy)) return;
  const int S = (2 * r + 1) * (2 * r + 1), nn = n_a * n_a;
  const int64_t g = R.unit_off + (int64_t)iy * R.Lx + ix;  // vectors
  const T2* Fi = F + (size_t)((shared ? R.fac_off : R.unit_off) + (int64_t)iy * R.Lx + ix) * S * nn;
  neighbour_sum<NA>(R, r, colour, false, ix, iy, Fi, z, z, red);
  if (threadIdx.x < n_a) {
    const double2 a = (colour == 0 ? in : z)[g * n_a + threadIdx.x], s = red[threadIdx.x];
    t[threadIdx.x] = make_double2(a.x - s.x, a.y - s.y);
  }
  __syncthreads();
  pivot_solve<NA>(Fi + (size_t)(S / 2) * nn, t, red, g, z, out);
}

int colour_cols(const BatchDesc& bd, int r) {
  int mx = 0;
  for (int b = 0; b < bd.B; ++b) mx = std::max(mx, bd.Lx[b]);
  return (mx + r) / (r + 1);
}
int colour_rows(const BatchDesc& bd, int r) {
  int my = 0;
  for (int b = 0; b < bd.B; ++b) my = std::max(my, bd.Ly[b]);
  return (my + r) / (r + 1);
}

template <typename T, int NA, typename OT>
void apply_typed(const BatchDesc& bd, int r, int shared, const void* F, const double2* in, double2* z, OT* out,
                 hipStream_t s, const int* live) {
  using T2 = typename Cx<T>::t2;
  const int ncx = colour_cols(bd, r), ncy = colour_rows(bd, r);
  const dim3 grid((unsigned)(ncx * ncy), (unsigned)bd.B);
  const int nc = (r + 1) * (r + 1);
  // colours 1 .. nc-1 forward (the last one also solves its pivots), then
  // nc-2 .. 0 backward
  for (int c = 1; c < nc; ++c)
    hipLaunchKernelGGL((ilu_forward_kernel<T, NA, OT>), grid, dim3(64 * kApplyWaves), 0, s, bd.rhs, r, c, ncx,
                       c == nc - 1 ? 1 : 0, shared, (const T2*)F, in, z, out, live);
  for (int c = nc - 2; c >= 0; --c)
    hipLaunchKernelGGL((ilu_backward_kernel<T, NA, OT>), grid, dim3(64 * kApplyWaves), 0, s, bd.rhs, r, c, ncx,
                       shared, (const T2*)F, in, z, out, live);
  R3M_CHECK_HIP(hipGetLastError());
}

template <typename T, typename OT>
void apply_na(const r3m_store* Z, const BatchDesc& bd, int r, int shared, const void* F, const double2* in,
              double2* z, OT* out, hipStream_t s, const int* live) {
  if (Z->n / Z->n_states == 40)
    apply_typed<T, 40, OT>(bd, r, shared, F, in, z, out, s, live);
  else
    apply_typed<T, 64, OT>(bd, r, shared, F, in, z, out, s, live);
}

template <typename T>
void factor_typed(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, int r, void* F, int* flag,
                  hipStream_t s, const double* wts, bool tr) {
  const int shared = wts ? 0 : 1;  // relaxed weights are per right-hand side
  using T2 = typename Cx<T>::t2;
  const int n_a = Z->n / Z->n_states;
  const int Nx = std::min(Z->near_radius, Z->Dx), Ny = std::min(Z->near_radius, Z->Dy);
  const int S = (2 * r + 1) * (2 * r + 1);
  const dim3 fg((unsigned)(bd.max_units * S), (unsigned)bd.B);
  hipLaunchKernelGGL(ilu_fill_kernel<T>, fg, dim3(256), (size_t)n_a * (n_a + 1) * sizeof(T2), s, (const T*)Z->near,
                     Z->n, Nx, Ny, n_a, Z->n_states, bd.rhs, states, r, (T2*)F, wts, tr ? 1 : 0, shared);
  const int ncx = colour_cols(bd, r), ncy = colour_rows(bd, r);
  const dim3 grid((unsigned)(ncx * ncy), (unsigned)bd.B);
  const size_t lds = ((size_t)2 * n_a * n_a + n_a + 1) * sizeof(double2);
  for (int c = 0; c < (r + 1) * (r + 1); ++c) {
    if (n_a == 40)
      hipLaunchKernelGGL((ilu_factor_kernel<T, 40>), grid, dim3(kFactorThreads), lds, s, bd.rhs, r, c, ncx, (T2*)F, flag,
                         shared);
    else
      hipLaunchKernelGGL((ilu_factor_kernel<T, 64>), grid, dim3(kFactorThreads), lds, s, bd.rhs, r, c, ncx, (T2*)F, flag,
                         shared);
  }
  R3M_CHECK_HIP(hipGetLastError());
}

}  // namespace

void validate_ilu(const r3m_store* Z, int radius) {
  const int n_a = Z->n / Z->n_states;
  R3M_REQUIRE(radius >= 1 && radius <= kIluMaxRadius, R3M_ERR_INVALID_ARG, "ILU radius must be in 1..3");
  R3M_REQUIRE(radius <= Z->near_radius, R3M_ERR_INVALID_ARG, "ILU radius exceeds the store's near radius");
  R3M_REQUIRE(n_a == 40 || n_a == 64, R3M_ERR_UNSUPPORTED, "ILU kernels are built for 40 or 64 active RWG per unit");
}

size_t ilu_factor_bytes(const r3m_store* Z, const BatchDesc& bd, int radius, bool shared) {
  const int n_a = Z->n / Z->n_states;
  const size_t S = (size_t)(2 * radius + 1) * (2 * radius + 1);
  const int64_t units = shared ? bd.codebook_units : bd.total_units;
  return (size_t)units * S * n_a * n_a * (Z->near_dtype == R3M_C128 ? 16 : 8);
}

void launch_ilu_factor(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, int radius, void* F,
                       int* flag, hipStream_t s, const double* wts, bool tr) {
  if (Z->near_dtype == R3M_C128)
    factor_typed<double>(Z, bd, states, radius, F, flag, s, wts, tr);
  else
    factor_typed<float>(Z, bd, states, radius, F, flag, s, wts, tr);
}

void launch_ilu_apply(const r3m_store* Z, const BatchDesc& bd, int radius, const void* F, const double2* in,
                      double2* z, r3m_dtype out_type, void* out, hipStream_t s, const int* live, bool shared) {
  const bool d = Z->near_dtype == R3M_C128;
  const int sh = shared ? 1 : 0;
  if (out_type == R3M_C64) {
    if (d)
      apply_na<double, float>(Z, bd, radius, sh, F, in, z, (float*)out, s, live);
    else
      apply_na<float, float>(Z, bd, radius, sh, F, in, z, (float*)out, s, live);
  } else {
    if (d)
      apply_na<double, double>(Z, bd, radius, sh, F, in, z, (double*)out, s, live);
    else
      apply_na<float, double>(Z, bd, radius, sh, F, in, z, (double*)out, s, live);
  }
}

}  // namespace r3m

using namespace r3m;

extern "C" {

size_t r3m_ilu_bytes(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, int32_t radius) {
  size_t out = 0;
  int rc = guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    require_isolated(Z);
    validate_ilu(Z, radius);
    validate_batch(batch, Z->Dx, Z->Dy);
    if (batch->B == 0) return;
    out = ilu_factor_bytes(Z, get_batch(ctx, batch, 8, 8, 0), radius);
  });
  return rc == R3M_OK ? out : 0;
}

int r3m_ilu_factor(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, int32_t radius, void* factors_dev,
                   size_t factors_bytes, hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    require_isolated(Z);
    validate_ilu(Z, radius);
    validate_batch(batch, Z->Dx, Z->Dy);
    if (batch->B == 0) return;
    R3M_REQUIRE(factors_dev && batch->states, R3M_ERR_INVALID_ARG, "NULL buffer");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    const BatchDesc& bd = get_batch(ctx, batch, 8, 8, stream);
    R3M_REQUIRE(factors_bytes >= ilu_factor_bytes(Z, bd, radius), R3M_ERR_BUFFER_TOO_SMALL,
                "ILU factor buffer too small");
    R3M_CHECK_HIP(hipMemsetAsync(ctx->flag.ptr, 0, sizeof(int), stream));
    check_states(bd, batch->states, Z->n_states, (int*)ctx->flag.ptr, 2, stream);
    launch_ilu_factor(Z, bd, batch->states, radius, factors_dev, (int*)ctx->flag.ptr, stream);
    int flag = 0;
    R3M_CHECK_HIP(hipMemcpyAsync(&flag, ctx->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, stream));
    R3M_CHECK_HIP(hipStreamSynchronize(stream));
    R3M_REQUIRE(!(flag & 2), R3M_ERR_INVALID_ARG, "codebook state out of range");
    R3M_REQUIRE(!(flag & 8), R3M_ERR_NONFINITE, "singular pivot block in the ILU factorisation");
  });
}

int r3m_ilu_apply(r3m_ctx ctx, const r3m_store* Z, const r3m_batch* batch, int32_t radius, const void* factors_dev,
                  size_t factors_bytes, const void* x_dev, void* y_dev, hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_store(Z);
    require_isolated(Z);
    validate_ilu(Z, radius);
    validate_batch(batch, Z->Dx, Z->Dy);
    if (batch->B == 0) return;
    R3M_REQUIRE(factors_dev && x_dev && y_dev, R3M_ERR_INVALID_ARG, "NULL buffer");
    R3M_REQUIRE(x_dev != y_dev, R3M_ERR_INVALID_ARG, "x and y must not alias");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    const BatchDesc& bd = get_batch(ctx, batch, 8, 8, stream);
    R3M_REQUIRE(factors_bytes >= ilu_factor_bytes(Z, bd, radius), R3M_ERR_BUFFER_TOO_SMALL,
                "ILU factor buffer too small");
    launch_ilu_apply(Z, bd, radius, factors_dev, (const double2*)x_dev, (double2*)y_dev, R3M_C128, nullptr, stream,
                     nullptr);
  });
}

}  // extern "C"
