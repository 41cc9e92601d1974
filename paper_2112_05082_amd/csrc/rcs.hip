// Plane-wave excitation U_k of eq. (1) and bistatic RCS of the retrieved
// currents (post-processing of Sec. IV-A), FP64.
//
// Excitation: U_m = int f_m . E_inc dS, E_inc = e0 e_hat exp(-j k k_hat . r),
// 7-point rule, one thread per (RHS, unit, active RWG).  Connected geometries
// (Sec. III-B): a unit's entries are its state's bases, then the shared ones;
// a bridging basis integrates over both of its triangles at their own
// positions, and D_k's masked extended bases get zero.
// RCS: radiation vectors of the macro RWGs of the unit at the origin,
// F_m(r_hat) = int f_m exp(j k r_hat . r) dS, are formed once per direction;
// then N(r_hat) = sum_u exp(j k r_hat . c_u) sum_{m in A(s_u)} I_{u,m} F_m and
// sigma = (k^2 eta^2 / 4 pi) |N - (N . r_hat) r_hat|^2 / |e0|^2.
#include "r3m_common.h"

#include <algorithm>

namespace r3m {
namespace {

struct IncDev {
  double kx, ky, kz;  // propagation direction k_hat
  double ex, ey, ez;  // polarisation e_hat (theta_hat)
  double e0;
  double pad;
};

// U of macro RWG mm of the unit whose origin is (cx, cy, 0), without e0
__device__ double2 plane_wave_value(const GeomDev& g, int mm, double cx, double cy, const IncDev& I, double k) {
  double re = 0.0, im = 0.0;
  for (int a = 0; a < 2; ++a) {
    const int t = g.rwg_tri[2 * mm + a];
    const int fv = g.rwg_free[2 * mm + a];
    const double* v = g.tri_v + 9 * t;
    const double A = g.tri_area[t];
    const double c = (a == 0 ? 1.0 : -1.0) * g.rwg_len[mm] / (2.0 * A);
    const double vx = v[3 * fv] + cx, vy = v[3 * fv + 1] + cy, vz = v[3 * fv + 2];
    for (int i = 0; i < 7; ++i) {
      double b0, b1, b2, w;
      quad7_point(i, b0, b1, b2, w);
      const double rx = b0 * v[0] + b1 * v[3] + b2 * v[6] + cx;
      const double ry = b0 * v[1] + b1 * v[4] + b2 * v[7] + cy;
      const double rz = b0 * v[2] + b1 * v[5] + b2 * v[8];
      const double proj = (rx - vx) * I.ex + (ry - vy) * I.ey + (rz - vz) * I.ez;
      double sn, cs;
      sincos(-k * (I.kx * rx + I.ky * ry + I.kz * rz), &sn, &cs);
      re += c * w * A * proj * cs;
      im += c * w * A * proj * sn;
    }
  }
  return make_double2(re, im);
}

__global__ void plane_wave_kernel(GeomDev g, const RhsDev* __restrict__ rhs, const IncDev* __restrict__ inc,
                                  const uint8_t* __restrict__ states, int n_a, int n_v, int n_states, double k,
                                  double px, double py, double2* __restrict__ out) {
  const int b = blockIdx.y;
  const RhsDev R = rhs[b];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t units = (int64_t)R.Lx * R.Ly;
  if (e >= units * n_v) return;
  const int64_t u = e / n_v;
  const int r = (int)(e % n_v);
  int s = states[R.state_off + u];
  s = s < n_states ? s : n_states - 1;
  const int64_t ix = u % R.Lx, iy = u / R.Lx;
  const double cx = (double)ix * px, cy = (double)iy * py;
  const IncDev I = inc[b];
  const int mm = compact_to_macro(g, n_a, s, r, ix, iy);
  const double2 v = mm >= 0 ? plane_wave_value(g, mm, cx, cy, I, k) : make_double2(0.0, 0.0);
  out[R.unit_off * n_v + e] = make_double2(I.e0 * v.x, I.e0 * v.y);
}

// Relaxed codebook (weights w [unit][n_states]): macro == 0 writes the blended
// excitation U_k(w)[u][m] = sum_s w[u][s] U[u][s n_a + m] ([unit][n_a]);
// macro != 0 writes every macro row U[u][mm] ([unit][n]), weights unused.
__global__ void plane_wave_relaxed_kernel(GeomDev g, const RhsDev* __restrict__ rhs, const IncDev* __restrict__ inc,
                                          const double* __restrict__ wts, int n_a, int n_states, int macro, double k,
                                          double px, double py, double2* __restrict__ out) {
  const int b = blockIdx.y;
  const RhsDev R = rhs[b];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int per = macro ? n_a * n_states : n_a;
  if (e >= (int64_t)R.Lx * R.Ly * per) return;
  const int64_t u = e / per;
  const int m = (int)(e - u * per);
  const double cx = (double)(u % R.Lx) * px, cy = (double)(u / R.Lx) * py;
  const IncDev I = inc[b];
  double2 acc = make_double2(0.0, 0.0);
  if (macro) {
    acc = plane_wave_value(g, m, cx, cy, I, k);
  } else {
    for (int st = 0; st < n_states; ++st) {
      const double w = wts[(R.unit_off + u) * n_states + st];
      const double2 v = plane_wave_value(g, st * n_a + m, cx, cy, I, k);
      acc.x += w * v.x;
      acc.y += w * v.y;
    }
  }
  out[R.unit_off * per + e] = make_double2(I.e0 * acc.x, I.e0 * acc.y);
}

// F[dir][m][3] for the macro unit at the origin
__global__ void macro_radiation_kernel(GeomDev g, const double* __restrict__ dirs, int n_dir, double k,
                                       double2* __restrict__ F) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_dir * g.n_rwg) return;
  const int d = e / g.n_rwg, m = e % g.n_rwg;
  const double th = dirs[2 * d], ph = dirs[2 * d + 1];
  const double rx = sin(th) * cos(ph), ry = sin(th) * sin(ph), rz = cos(th);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int a = 0; a < 2; ++a) {
    const int t = g.rwg_tri[2 * m + a];
    const int fv = g.rwg_free[2 * m + a];
    const double* v = g.tri_v + 9 * t;
    const double A = g.tri_area[t];
    const double c = (a == 0 ? 1.0 : -1.0) * g.rwg_len[m] / (2.0 * A);
    for (int i = 0; i < 7; ++i) {
      double b0, b1, b2, w;
      quad7_point(i, b0, b1, b2, w);
      double p[3];
      for (int q = 0; q < 3; ++q) p[q] = b0 * v[q] + b1 * v[3 + q] + b2 * v[6 + q];
      double sn, cs;
      sincos(k * (rx * p[0] + ry * p[1] + rz * p[2]), &sn, &cs);
      for (int q = 0; q < 3; ++q) {
        const double f = c * w * A * (p[q] - v[3 * fv + q]);
        acc[2 * q] += f * cs;
        acc[2 * q + 1] += f * sn;
      }
    }
  }
  for (int q = 0; q < 3; ++q) F[(size_t)e * 3 + q] = make_double2(acc[2 * q], acc[2 * q + 1]);
}

constexpr int kRcsThreads = 256;
constexpr int kRcsDirs = 64;      // directions per block, one per lane
constexpr int kRcsWaves = kRcsThreads / 64;
constexpr int kRcsExact = 32;     // units between exact phase evaluations

// Array sums of one item over all units of a RHS: for SH false, the compact
// entries rc..rc+MC-1 of units in coding states s0..s0+NSG-1 (A[j][c] for
// state s0 + j); for SH true, shared entries rc..rc+MC-1, zero where D_k
// masks them.  The chunk of each unit is uniform across the wave (scalar
// loads); the lane's phase
// exp(j k r_hat . c_u) advances by one complex product per unit along x from
// an exact value every kRcsExact units and at each row start.
template <bool SH, int NSG, int MC>
__device__ __forceinline__ void rcs_array_sums(const GeomDev& g, const RhsDev& R, const uint8_t* __restrict__ states,
                                               const double2* __restrict__ I, int n_a, int n_v, int n_states,
                                               int s0, int rc, int lane, double k, double rx, double ry, double px,
                                               double py, double stx_r, double stx_i, double (&ar)[NSG][MC],
                                               double (&ai)[NSG][MC]) {
#pragma unroll
  for (int j = 0; j < NSG; ++j)
#pragma unroll
    for (int c = 0; c < MC; ++c) ar[j][c] = ai[j][c] = 0.0;
  int cls[MC];  // a shared entry's class decides where D_k masks it
#pragma unroll
  for (int c = 0; c < MC; ++c) cls[c] = (SH && rc + c >= n_a) ? g.common_ext[rc + c - n_a] : 0;
  const int64_t units = (int64_t)R.Lx * R.Ly;
  const double2* Ip = I + R.unit_off * n_v + rc;
  int ix = 0, iy = 0;
  double pr = 0.0, pi = 0.0;
  for (int64_t u0 = 0; u0 < units; u0 += 64) {
    const int n_in = (int)min<int64_t>(64, units - u0);
    const int st_l = (!SH && lane < n_in) ? (int)states[R.state_off + u0 + lane] : 0;
    for (int i = 0; i < n_in; ++i, Ip += n_v) {
      double2 cur[MC];
#pragma unroll
      for (int c = 0; c < MC; ++c) cur[c] = Ip[c];
      if (ix % kRcsExact == 0) sincos(k * (rx * (double)ix * px + ry * (double)iy * py), &pi, &pr);
      if (SH) {
#pragma unroll
        for (int c = 0; c < MC; ++c) {
          const bool keep = !((cls[c] == 1 && ix == 0) || (cls[c] == 2 && iy == 0));
          const double cx = keep ? cur[c].x : 0.0, cy = keep ? cur[c].y : 0.0;
          ar[0][c] = fma(-pi, cy, fma(pr, cx, ar[0][c]));
          ai[0][c] = fma(pi, cx, fma(pr, cy, ai[0][c]));
        }
      } else {
        int s = __builtin_amdgcn_readlane(st_l, i);
        s = s < n_states ? s : n_states - 1;
#pragma unroll
        for (int j = 0; j < NSG; ++j) {
          if (s == s0 + j) {  // uniform
#pragma unroll
            for (int c = 0; c < MC; ++c) {
              ar[j][c] = fma(-pi, cur[c].y, fma(pr, cur[c].x, ar[j][c]));
              ai[j][c] = fma(pi, cur[c].x, fma(pr, cur[c].y, ai[j][c]));
            }
          }
        }
      }
      const double t = pr * stx_r - pi * stx_i;
      pi = pr * stx_i + pi * stx_r;
      pr = t;
      if (++ix == R.Lx) {
        ix = 0;
        ++iy;
      }
    }
  }
}

// N(d) += sum over an item's entries of A F_{macro RWG}(d), entries r0..r_end-1 only
template <bool SH, int NSG, int MC>
__device__ __forceinline__ void rcs_combine(const GeomDev& g, const double2* __restrict__ Fd, int n_a,
                                            int n_states, int s0, int rc, int r0, int r_end,
                                            const double (&ar)[NSG][MC], const double (&ai)[NSG][MC],
                                            double (&N)[6]) {
#pragma unroll
  for (int j = 0; j < NSG; ++j) {
    if (s0 + j < n_states) {
#pragma unroll
      for (int c = 0; c < MC; ++c) {
        const int r = rc + c;
        if (r >= r0 && r < r_end) {
          const int mm = SH ? g.n_st + (r - n_a) : (s0 + j) * n_a + r;
          const double2* f = Fd + (size_t)mm * 3;
          for (int q = 0; q < 3; ++q) {
            N[2 * q] += ar[j][c] * f[q].x - ai[j][c] * f[q].y;
            N[2 * q + 1] += ar[j][c] * f[q].y + ai[j][c] * f[q].x;
          }
        }
      }
    }
  }
}

// Bistatic RCS of a batch, one block per (RHS, 64 directions), lane =
// direction.  The sum over units is taken first, per compact entry r and
// coding state s (array factor):
//   A_{s,r}(d) = sum_{u in state s} exp(j k r_hat_d . c_u) I_{u,r},
// then N(d) = sum_{s,r} A_{s,r}(d) F_{macro(s,r)}(d) (a shared basis of a
// connected geometry has one A, over the units where D_k keeps it).  Items
// of NSG states x MC contiguous entries are split over the block's waves; N
// is summed over them in a fixed order.  The direction blocks of RHS b share
// one XCD (and its L2 copy of I_b).
template <int NSG, int MC>
__global__ void __launch_bounds__(kRcsThreads, NSG == 4 ? 3 : 4)
rcs_kernel(GeomDev g, const RhsDev* __restrict__ rhs, const uint8_t* __restrict__ states,
           const double2* __restrict__ I, const double2* __restrict__ F, const double* __restrict__ dirs, int n_dir,
           int n, int n_a, int n_v, int n_states, int B, int n_dblk, double k, double px, double py, double scale,
           double* __restrict__ sigma) {
  __shared__ double sh[kRcsWaves][6][kRcsDirs];
  const int id = blockIdx.x, xcd = id % 8, slot = id / 8;
  const int b = (slot / n_dblk) * 8 + xcd, dblk = slot % n_dblk;
  if (b >= B) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int d_raw = dblk * kRcsDirs + lane;
  const bool live = d_raw < n_dir;
  const int d = live ? d_raw : n_dir - 1;
  const double th = dirs[2 * d], ph = dirs[2 * d + 1];
  const double rx = sin(th) * cos(ph), ry = sin(th) * sin(ph), rz = cos(th);
  double stx_i, stx_r;
  sincos(k * rx * px, &stx_i, &stx_r);  // phase step of one unit along x
  const RhsDev R = rhs[b];
  const int n_groups = (n_states + NSG - 1) / NSG;
  const int n_chunks = (n_a + MC - 1) / MC;
  const int n_state_items = n_groups * n_chunks;
  const int n_items = n_state_items + (n_v - n_a + MC - 1) / MC;
  const double2* Fd = F + (size_t)d * n * 3;
  double N[6] = {0, 0, 0, 0, 0, 0};
  for (int it = wave; it < n_items; it += kRcsWaves) {
    // an item reads MC contiguous entries inside the unit's row: a ragged
    // last chunk slides back, and its entries before r0 (another item's)
    // stay out of N
    if (it < n_state_items) {
      const int s0 = (it / n_chunks) * NSG, r0 = (it % n_chunks) * MC;
      const int rc = min(r0, n_v - MC);
      double ar[NSG][MC], ai[NSG][MC];
      rcs_array_sums<false, NSG, MC>(g, R, states, I, n_a, n_v, n_states, s0, rc, lane, k, rx, ry, px, py, stx_r,
                                     stx_i, ar, ai);
      rcs_combine<false, NSG, MC>(g, Fd, n_a, n_states, s0, rc, r0, n_a, ar, ai, N);
    } else {
      const int r0 = n_a + (it - n_state_items) * MC;
      const int rc = min(r0, n_v - MC);
      double ar[1][MC], ai[1][MC];
      rcs_array_sums<true, 1, MC>(g, R, states, I, n_a, n_v, n_states, 0, rc, lane, k, rx, ry, px, py, stx_r,
                                  stx_i, ar, ai);
      rcs_combine<true, 1, MC>(g, Fd, n_a, n_states, 0, rc, r0, n_v, ar, ai, N);
    }
  }
  for (int q = 0; q < 6; ++q) sh[wave][q][lane] = N[q];
  __syncthreads();
  if (wave == 0 && live) {
    for (int q = 0; q < 6; ++q)
      for (int w = 1; w < kRcsWaves; ++w) N[q] += sh[w][q][lane];
    const double rr[3] = {rx, ry, rz};
    const double dre = N[0] * rx + N[2] * ry + N[4] * rz;
    const double dim = N[1] * rx + N[3] * ry + N[5] * rz;
    double p2 = 0.0;
    for (int q = 0; q < 3; ++q) {
      const double qr = N[2 * q] - dre * rr[q], qi = N[2 * q + 1] - dim * rr[q];
      p2 += qr * qr + qi * qi;
    }
    sigma[(size_t)b * n_dir + d] = scale * p2;
  }
}

// Radiation vector of the blended current I~[u][s n_a + r] = w[u][s] I[u][r]
// (relaxed codebook) for direction d and RHS b: sigma as rcs_kernel, and the
// transverse part N_perp (3 complex) kept for the objective's gradient.
__global__ void __launch_bounds__(kRcsThreads)
rcs_relaxed_kernel(const RhsDev* __restrict__ rhs, const double* __restrict__ wts, const double2* __restrict__ I,
                   const double2* __restrict__ F, const double* __restrict__ dirs, int n_dir, int n, int n_a,
                   int n_states, double k, double px, double py, double scale, double* __restrict__ sigma,
                   double2* __restrict__ nperp) {
  __shared__ double sh[kRcsThreads / 64][6];
  const int d = blockIdx.x, b = blockIdx.y;
  const RhsDev R = rhs[b];
  const double th = dirs[2 * d], ph = dirs[2 * d + 1];
  const double rx = sin(th) * cos(ph), ry = sin(th) * sin(ph), rz = cos(th);
  const int64_t units = (int64_t)R.Lx * R.Ly;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const double2* Fd = F + (size_t)d * n * 3;
  for (int64_t u = threadIdx.x; u < units; u += blockDim.x) {
    const double cx = (double)(u % R.Lx) * px, cy = (double)(u / R.Lx) * py;
    double sn, cs;
    sincos(k * (rx * cx + ry * cy), &sn, &cs);
    double loc[6] = {0, 0, 0, 0, 0, 0};
    const double2* Iu = I + (R.unit_off + u) * n_a;
    for (int st = 0; st < n_states; ++st) {
      const double w = wts[(R.unit_off + u) * n_states + st];
      for (int m = 0; m < n_a; ++m) {
        const double2 cur = make_double2(w * Iu[m].x, w * Iu[m].y);
        const double2* f = Fd + (size_t)(st * n_a + m) * 3;
        for (int q = 0; q < 3; ++q) {
          loc[2 * q] += cur.x * f[q].x - cur.y * f[q].y;
          loc[2 * q + 1] += cur.x * f[q].y + cur.y * f[q].x;
        }
      }
    }
    for (int q = 0; q < 3; ++q) {
      acc[2 * q] += loc[2 * q] * cs - loc[2 * q + 1] * sn;
      acc[2 * q + 1] += loc[2 * q] * sn + loc[2 * q + 1] * cs;
    }
  }
  for (int q = 0; q < 6; ++q)
    for (int o = 32; o >= 1; o >>= 1) acc[q] += __shfl_xor(acc[q], o);
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < 6; ++q) sh[threadIdx.x >> 6][q] = acc[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    double N[6];
    for (int q = 0; q < 6; ++q) {
      N[q] = sh[0][q];
      for (int w = 1; w < kRcsThreads / 64; ++w) N[q] += sh[w][q];
    }
    const double rr[3] = {rx, ry, rz};
    const double dre = N[0] * rx + N[2] * ry + N[4] * rz;
    const double dim = N[1] * rx + N[3] * ry + N[5] * rz;
    double p2 = 0.0;
    for (int q = 0; q < 3; ++q) {
      const double pr = N[2 * q] - dre * rr[q], pi = N[2 * q + 1] - dim * rr[q];
      p2 += pr * pr + pi * pi;
      nperp[((size_t)b * n_dir + d) * 3 + q] = make_double2(pr, pi);
    }
    sigma[(size_t)b * n_dir + d] = scale * p2;
  }
}

// J[b] = mean over directions of sigma[b][:] (fixed order)
__global__ void mean_dirs_kernel(const double* __restrict__ sigma, int n_dir, int B, double* __restrict__ J) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double t = 0.0;
  for (int d = 0; d < n_dir; ++d) t += sigma[(size_t)b * n_dir + d];
  J[b] = t / n_dir;
}

// G[u][mm] = dJ/dI~[u][mm] = (scale / n_dir) sum_d conj(N_perp(d)) . F_mm(d)
// exp(j k r_hat_d . c_u) (Wirtinger derivative of the mean RCS), macro layout
__global__ void relaxed_dj_kernel(const RhsDev* __restrict__ rhs, const double2* __restrict__ F,
                                  const double* __restrict__ dirs, const double2* __restrict__ nperp, int n_dir, int n,
                                  double k, double px, double py, double scale, double2* __restrict__ G) {
  const int b = blockIdx.y;
  const RhsDev R = rhs[b];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)R.Lx * R.Ly * n) return;
  const int64_t u = e / n;
  const int mm = (int)(e - u * n);
  const double cx = (double)(u % R.Lx) * px, cy = (double)(u / R.Lx) * py;
  double gr = 0.0, gi = 0.0;
  for (int d = 0; d < n_dir; ++d) {
    const double th = dirs[2 * d], ph = dirs[2 * d + 1];
    double sn, cs;
    sincos(k * (sin(th) * cos(ph) * cx + sin(th) * sin(ph) * cy), &sn, &cs);
    const double2* f = F + ((size_t)d * n + mm) * 3;
    const double2* np_ = nperp + ((size_t)b * n_dir + d) * 3;
    double tr = 0.0, ti = 0.0;  // conj(N_perp) . F_mm
    for (int q = 0; q < 3; ++q) {
      tr += np_[q].x * f[q].x + np_[q].y * f[q].y;
      ti += np_[q].x * f[q].y - np_[q].y * f[q].x;
    }
    gr += tr * cs - ti * sn;
    gi += tr * sn + ti * cs;
  }
  G[R.unit_off * n + e] = make_double2(scale / n_dir * gr, scale / n_dir * gi);
}

// a[u][r] = sum_s w[u][s] G[u][s n_a + r]: P(w)^T G, the adjoint right-hand side
__global__ void blend_transpose_kernel(const RhsDev* __restrict__ rhs, const double* __restrict__ wts,
                                       const double2* __restrict__ G, int n_a, int n_states, double2* __restrict__ a) {
  const int b = blockIdx.y;
  const RhsDev R = rhs[b];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)R.Lx * R.Ly * n_a) return;
  const int64_t u = e / n_a;
  const int r = (int)(e - u * n_a);
  double xr = 0.0, xi = 0.0;
  for (int st = 0; st < n_states; ++st) {
    const double w = wts[(R.unit_off + u) * n_states + st];
    const double2 g = G[(R.unit_off + u) * n_a * n_states + st * n_a + r];
    xr += w * g.x;
    xi += w * g.y;
  }
  a[R.unit_off * n_a + e] = make_double2(xr, xi);
}

}  // namespace
}  // namespace r3m

using namespace r3m;

extern "C" {

int r3m_plane_wave_rhs(r3m_ctx ctx, const r3m_unit_geom* geom, const r3m_batch* batch,
                       const double* inc_host, void* b_dev, hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_geom(geom);
    require_extension_classes(geom);
    validate_batch(batch, 1 << 20, 1 << 20);
    if (batch->B == 0) return;
    R3M_REQUIRE(inc_host && b_dev, R3M_ERR_INVALID_ARG, "NULL argument");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    const int n_a = geom->state_off[1] - geom->state_off[0];
    GeomDev g = upload_geom(ctx, geom, stream);
    const BatchDesc& bd = get_batch(ctx, batch, 4, 4, stream);
    std::vector<IncDev> inc(bd.B);
    for (int b = 0; b < bd.B; ++b) {
      const double th = inc_host[3 * b], ph = inc_host[3 * b + 1];
      R3M_REQUIRE(std::isfinite(th) && std::isfinite(ph) && std::isfinite(inc_host[3 * b + 2]),
                  R3M_ERR_INVALID_ARG, "non-finite incidence");
      inc[b] = IncDev{-std::sin(th) * std::cos(ph), -std::sin(th) * std::sin(ph), -std::cos(th),
                      std::cos(th) * std::cos(ph), std::cos(th) * std::sin(ph), -std::sin(th),
                      inc_host[3 * b + 2], 0.0};
    }
    DevBuf tmp;
    tmp.ensure(inc.size() * sizeof(IncDev));
    R3M_CHECK_HIP(hipMemcpyAsync(tmp.ptr, inc.data(), inc.size() * sizeof(IncDev), hipMemcpyHostToDevice, stream));
    int64_t maxU = 0;
    for (int b = 0; b < bd.B; ++b) maxU = std::max<int64_t>(maxU, bd.n_units[b]);
    const double k = 2.0 * kPi * geom->freq_hz / kC0;
    const int n_v = vec_per_unit(geom);
    dim3 grid(ceil_div((size_t)maxU * n_v, 256), bd.B);
    check_states(bd, batch->states, geom->n_states, deferred_word(ctx), kDeferredBadState, stream);
    hipLaunchKernelGGL(plane_wave_kernel, grid, dim3(256), 0, stream, g, bd.rhs, (const IncDev*)tmp.ptr,
                       batch->states, n_a, n_v, geom->n_states, k, geom->period_x, geom->period_y, (double2*)b_dev);
    R3M_CHECK_HIP(hipGetLastError());
    R3M_CHECK_HIP(hipStreamSynchronize(stream));
    tmp.release();
    take_deferred(ctx, stream);
  });
}

int r3m_rcs(r3m_ctx ctx, const r3m_unit_geom* geom, const r3m_batch* batch, const void* I_dev,
            int32_t n_dir, const double* dirs_host, double e0, double* sigma_dev, hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_geom(geom);
    require_extension_classes(geom);
    validate_batch(batch, 1 << 20, 1 << 20);
    R3M_REQUIRE(n_dir >= 0, R3M_ERR_INVALID_ARG, "n_dir < 0");
    R3M_REQUIRE(e0 != 0.0 && std::isfinite(e0), R3M_ERR_INVALID_ARG, "e0 must be finite and non-zero");
    if (batch->B == 0 || n_dir == 0) return;
    R3M_REQUIRE(I_dev && dirs_host && sigma_dev, R3M_ERR_INVALID_ARG, "NULL argument");
    for (int d = 0; d < 2 * n_dir; ++d)
      R3M_REQUIRE(std::isfinite(dirs_host[d]), R3M_ERR_INVALID_ARG, "non-finite direction");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    const int n_a = geom->state_off[1] - geom->state_off[0];
    GeomDev g = upload_geom(ctx, geom, stream);
    const BatchDesc& bd = get_batch(ctx, batch, 4, 4, stream);
    const double k = 2.0 * kPi * geom->freq_hz / kC0;
    DevBuf tmp;
    const size_t fbytes = (size_t)n_dir * geom->n_rwg * 3 * sizeof(double2);
    tmp.ensure(fbytes + (size_t)n_dir * 16 + 256);
    double* ddev = (double*)((char*)tmp.ptr + fbytes);
    R3M_CHECK_HIP(hipMemcpyAsync(ddev, dirs_host, (size_t)n_dir * 16, hipMemcpyHostToDevice, stream));
    double2* F = (double2*)tmp.ptr;
    hipLaunchKernelGGL(macro_radiation_kernel, dim3(ceil_div((size_t)n_dir * geom->n_rwg, 128)), dim3(128), 0,
                       stream, g, ddev, n_dir, k, F);
    const double scale = k * k * kEta0 * kEta0 / (4.0 * kPi) / (e0 * e0);
    check_states(bd, batch->states, geom->n_states, deferred_word(ctx), kDeferredBadState, stream);
    // items of NSG coding states x MC contiguous compact entries (two per
    // wave for the 1- and 2-bit units of 40 active bases)
    const int n_dblk = ceil_div((size_t)n_dir, kRcsDirs);
    R3M_REQUIRE((size_t)ceil_div((size_t)bd.B, 8) * 8 * n_dblk < (1ull << 31), R3M_ERR_INVALID_ARG,
                "too many right-hand sides x directions for one RCS launch");
    const dim3 grid(ceil_div((size_t)bd.B, 8) * 8 * n_dblk);
    auto launch = [&](auto kern) {
      hipLaunchKernelGGL(kern, grid, dim3(kRcsThreads), 0, stream, g, bd.rhs, batch->states, (const double2*)I_dev,
                         (const double2*)F, (const double*)ddev, n_dir, geom->n_rwg, n_a, vec_per_unit(geom),
                         geom->n_states, bd.B, n_dblk, k, geom->period_x, geom->period_y, scale, sigma_dev);
    };
    const int n_v = vec_per_unit(geom);
    if (n_v < 5)
      launch(rcs_kernel<1, 1>);
    else if (geom->n_states == 1)
      launch(rcs_kernel<1, 5>);
    else if (geom->n_states == 2)
      launch(rcs_kernel<2, 5>);
    else
      launch(rcs_kernel<4, 5>);
    R3M_CHECK_HIP(hipGetLastError());
    R3M_CHECK_HIP(hipStreamSynchronize(stream));
    tmp.release();
    take_deferred(ctx, stream);
  });
}

int r3m_relaxed_rhs(r3m_ctx ctx, const r3m_unit_geom* geom, const r3m_batch* batch, const double* weights_dev,
                    const double* inc_host, int32_t macro, void* b_dev, hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_geom(geom);
    require_isolated(geom);
    validate_batch(batch, 1 << 20, 1 << 20);
    if (batch->B == 0) return;
    R3M_REQUIRE(inc_host && b_dev && (macro || weights_dev), R3M_ERR_INVALID_ARG, "NULL argument");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    const int n_a = geom->state_off[1] - geom->state_off[0];
    GeomDev g = upload_geom(ctx, geom, stream);
    const BatchDesc& bd = get_batch(ctx, batch, 4, 4, stream);
    std::vector<IncDev> inc(bd.B);
    for (int b = 0; b < bd.B; ++b) {
      const double th = inc_host[3 * b], ph = inc_host[3 * b + 1];
      R3M_REQUIRE(std::isfinite(th) && std::isfinite(ph) && std::isfinite(inc_host[3 * b + 2]),
                  R3M_ERR_INVALID_ARG, "non-finite incidence");
      inc[b] = IncDev{-std::sin(th) * std::cos(ph), -std::sin(th) * std::sin(ph), -std::cos(th),
                      std::cos(th) * std::cos(ph), std::cos(th) * std::sin(ph), -std::sin(th),
                      inc_host[3 * b + 2], 0.0};
    }
    DevBuf tmp;
    tmp.ensure(inc.size() * sizeof(IncDev));
    R3M_CHECK_HIP(hipMemcpyAsync(tmp.ptr, inc.data(), inc.size() * sizeof(IncDev), hipMemcpyHostToDevice, stream));
    int64_t maxU = 0;
    for (int b = 0; b < bd.B; ++b) maxU = std::max<int64_t>(maxU, bd.n_units[b]);
    const double k = 2.0 * kPi * geom->freq_hz / kC0;
    const int per = macro ? n_a * geom->n_states : n_a;
    hipLaunchKernelGGL(plane_wave_relaxed_kernel, dim3(ceil_div((size_t)maxU * per, 256), bd.B), dim3(256), 0,
                       stream, g, bd.rhs, (const IncDev*)tmp.ptr, weights_dev, n_a, geom->n_states, macro ? 1 : 0, k,
                       geom->period_x, geom->period_y, (double2*)b_dev);
    R3M_CHECK_HIP(hipGetLastError());
    R3M_CHECK_HIP(hipStreamSynchronize(stream));
    tmp.release();
  });
}

int r3m_relaxed_objective(r3m_ctx ctx, const r3m_unit_geom* geom, const r3m_batch* batch, const double* weights_dev,
                          const void* I_dev, int32_t n_dir, const double* dirs_host, double e0, double* J_dev,
                          double* sigma_dev, void* G_dev, void* adj_dev, hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    validate_geom(geom);
    require_isolated(geom);
    validate_batch(batch, 1 << 20, 1 << 20);
    R3M_REQUIRE(n_dir >= 1, R3M_ERR_INVALID_ARG, "n_dir < 1");
    R3M_REQUIRE(e0 != 0.0 && std::isfinite(e0), R3M_ERR_INVALID_ARG, "e0 must be finite and non-zero");
    if (batch->B == 0) return;
    R3M_REQUIRE(weights_dev && I_dev && dirs_host && J_dev && sigma_dev && G_dev && adj_dev, R3M_ERR_INVALID_ARG,
                "NULL argument");
    for (int d = 0; d < 2 * n_dir; ++d)
      R3M_REQUIRE(std::isfinite(dirs_host[d]), R3M_ERR_INVALID_ARG, "non-finite direction");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    const int n_a = geom->state_off[1] - geom->state_off[0];
    GeomDev g = upload_geom(ctx, geom, stream);
    const BatchDesc& bd = get_batch(ctx, batch, 4, 4, stream);
    const double k = 2.0 * kPi * geom->freq_hz / kC0;
    DevBuf tmp;
    const size_t fbytes = (size_t)n_dir * geom->n_rwg * 3 * sizeof(double2);
    const size_t npbytes = (size_t)bd.B * n_dir * 3 * sizeof(double2);
    tmp.ensure(fbytes + npbytes + (size_t)n_dir * 16 + 512);
    double2* F = (double2*)tmp.ptr;
    double2* np_ = (double2*)((char*)tmp.ptr + fbytes);
    double* ddev = (double*)((char*)tmp.ptr + fbytes + npbytes);
    R3M_CHECK_HIP(hipMemcpyAsync(ddev, dirs_host, (size_t)n_dir * 16, hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(macro_radiation_kernel, dim3(ceil_div((size_t)n_dir * geom->n_rwg, 128)), dim3(128), 0,
                       stream, g, ddev, n_dir, k, F);
    const double scale = k * k * kEta0 * kEta0 / (4.0 * kPi) / (e0 * e0);
    hipLaunchKernelGGL(rcs_relaxed_kernel, dim3(n_dir, bd.B), dim3(kRcsThreads), 0, stream, bd.rhs, weights_dev,
                       (const double2*)I_dev, (const double2*)F, (const double*)ddev, n_dir, geom->n_rwg, n_a,
                       geom->n_states, k, geom->period_x, geom->period_y, scale, sigma_dev, np_);
    hipLaunchKernelGGL(mean_dirs_kernel, dim3(ceil_div((size_t)bd.B, 64)), dim3(64), 0, stream,
                       (const double*)sigma_dev, n_dir, bd.B, J_dev);
    int64_t maxU = 0;
    for (int b = 0; b < bd.B; ++b) maxU = std::max<int64_t>(maxU, bd.n_units[b]);
    hipLaunchKernelGGL(relaxed_dj_kernel, dim3(ceil_div((size_t)maxU * geom->n_rwg, 256), bd.B), dim3(256), 0,
                       stream, bd.rhs, (const double2*)F, (const double*)ddev, (const double2*)np_, n_dir,
                       geom->n_rwg, k, geom->period_x, geom->period_y, scale, (double2*)G_dev);
    hipLaunchKernelGGL(blend_transpose_kernel, dim3(ceil_div((size_t)maxU * n_a, 256), bd.B), dim3(256), 0, stream,
                       bd.rhs, weights_dev, (const double2*)G_dev, n_a, geom->n_states, (double2*)adj_dev);
    R3M_CHECK_HIP(hipGetLastError());
    R3M_CHECK_HIP(hipStreamSynchronize(stream));
    tmp.release();
  });
}

}  // extern "C"
