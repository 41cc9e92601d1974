// Unique displacement-block fill of the global matrix (Galerkin EFIE, RWG).
//
// Z(d)[m][n] couples observer macro RWG m of the unit at lattice offset d to
// source macro RWG n of the unit at the origin (eq. (1), Sec. II-A):
//   Z_mn = j k eta sum_{a,b in +-} s_a s_b l_m l_n / (A_p A_q)
//          int_p int_q [ (r - v_a).(r' - v_b)/4 - 1/k^2 ] G(|r - r'|) dS' dS
// with the 7-point degree-5 rule on both triangles.  For triangle pairs whose
// cells are within Chebyshev distance extract_radius (the cells of the two
// units, shifted by the triangles' own cell offsets for bases that bridge two
// cells, Sec. III-B), G = 1/(4 pi R) + (exp(-jkR) - 1)/(4 pi R):
// the first term is integrated in closed form over the source triangle
// (edge-sum formulas of Wilton et al. / Graglia), the second by quadrature.
// Triangles of different coding states in the same cell overlap (coexistent
// meshes of the macro unit, Sec. III-A): the closed-form inner integral then
// has kinks along the source triangle's edges inside the observer triangle,
// so for those pairs the outer integral takes the composite rule, the 7-point
// rule on each of the 64 triangles of three midpoint subdivisions of the
// observer triangle.  One thread per (block, m, n); everything in FP64.
#include <array>

#include "r3m_common.h"

namespace r3m {
namespace {

struct Quad7 {
  double b[7][3];
  double w[7];
};

__constant__ Quad7 c_quad;

// the composite outer rule for overlapping cross-state pairs
constexpr int kSubLevels = 3;
constexpr int kSubTris = 1 << (2 * kSubLevels);  // 64
constexpr int kCompPts = 7 * kSubTris;           // 448
struct QuadComp {
  double b[kCompPts][3];
  double w[kCompPts];
};
__constant__ QuadComp c_comp;

Quad7 make_quad7() {
  Quad7 q;
  const double s15 = std::sqrt(15.0);
  const double a1 = (6.0 - s15) / 21.0, b1 = 1.0 - 2.0 * a1;
  const double a2 = (6.0 + s15) / 21.0, b2 = 1.0 - 2.0 * a2;
  const double w0 = 9.0 / 40.0, w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
  const double pts[7][3] = {{1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0}, {b1, a1, a1}, {a1, b1, a1},
                            {a1, a1, b1}, {b2, a2, a2}, {a2, b2, a2}, {a2, a2, b2}};
  const double ws[7] = {w0, w1, w1, w1, w2, w2, w2};
  for (int i = 0; i < 7; ++i) {
    for (int c = 0; c < 3; ++c) q.b[i][c] = pts[i][c];
    q.w[i] = ws[i];
  }
  return q;
}

// 7-point rule on each triangle of kSubLevels midpoint subdivisions, in
// barycentric coordinates of the parent triangle (weights sum to one)
QuadComp make_composite(const Quad7& q7) {
  // corners of the sub-triangles, in barycentric coordinates
  std::vector<std::array<std::array<double, 3>, 3>> tris(1);
  for (int c = 0; c < 3; ++c)
    for (int d = 0; d < 3; ++d) tris[0][c][d] = c == d ? 1.0 : 0.0;
  for (int lev = 0; lev < kSubLevels; ++lev) {
    std::vector<std::array<std::array<double, 3>, 3>> next;
    for (const auto& t : tris) {
      std::array<double, 3> m[3];  // midpoints of the edges opposite corners 2, 0, 1
      for (int d = 0; d < 3; ++d) {
        m[0][d] = 0.5 * (t[0][d] + t[1][d]);
        m[1][d] = 0.5 * (t[1][d] + t[2][d]);
        m[2][d] = 0.5 * (t[2][d] + t[0][d]);
      }
      next.push_back({t[0], m[0], m[2]});
      next.push_back({m[0], t[1], m[1]});
      next.push_back({m[2], m[1], t[2]});
      next.push_back({m[1], m[2], m[0]});
    }
    tris.swap(next);
  }
  QuadComp q;
  int i = 0;
  for (const auto& t : tris)
    for (int j = 0; j < 7; ++j, ++i) {
      for (int d = 0; d < 3; ++d)
        q.b[i][d] = q7.b[j][0] * t[0][d] + q7.b[j][1] * t[1][d] + q7.b[j][2] * t[2][d];
      q.w[i] = q7.w[j] / kSubTris;
    }
  return q;
}

struct V3 {
  double x, y, z;
};
__device__ inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline double norm(V3 a) { return sqrt(dot(a, a)); }

// int_T 1/R dS' (S) and int_T (r' - r)/R dS' (V) for the flat triangle (t0,t1,t2)
__device__ void static_potentials(V3 r, V3 t0, V3 t1, V3 t2, double& S, V3& V) {
  V3 nn = cross(t1 - t0, t2 - t0);
  V3 n = (1.0 / norm(nn)) * nn;
  const double d = dot(n, r - t0);
  const double ad = fabs(d);
  V3 rho = r - d * n;
  S = 0.0;
  V3 Vp = {0.0, 0.0, 0.0};
  V3 tv[3] = {t0, t1, t2};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    V3 a = tv[e], b = tv[(e + 1) % 3];
    V3 ab = b - a;
    const double len = norm(ab);
    V3 lh = (1.0 / len) * ab;
    V3 uh = cross(lh, n);  // outward in-plane normal of the edge
    const double tt = dot(a - rho, uh);
    const double lm = dot(a - rho, lh);
    const double lp = dot(b - rho, lh);
    const double R0sq = tt * tt + d * d;
    const double Rm = sqrt(lm * lm + R0sq);
    const double Rp = sqrt(lp * lp + R0sq);
    double f = 0.0;
    if (sqrt(R0sq) > 1e-12 * len) {
      if (lm >= 0.0)
        f = log((Rp + lp) / (Rm + lm));
      else if (lp <= 0.0)
        f = log((Rm - lm) / (Rp - lp));
      else
        f = log((Rp + lp) * (Rm - lm) / R0sq);
    }
    double term = tt * f;
    if (ad > 0.0) term -= ad * (atan(tt * lp / (R0sq + ad * Rp)) - atan(tt * lm / (R0sq + ad * Rm)));
    S += term;
    const double c = 0.5 * (R0sq * f + lp * Rp - lm * Rm);
    Vp = Vp + c * uh;
  }
  V = Vp - (d * S) * n;
}

__device__ inline V3 load_vertex(const double* tv, int t, int a) {
  const double* p = tv + 9 * t + 3 * a;
  return {p[0], p[1], p[2]};
}

template <typename OutT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) fill_blocks_kernel(GeomDev g, double k, double px, double py,
                                                          int Dx, int Dy, int slot_begin,
                                                          int extract_radius, OutT* out,
                                                          int* flag) {
  const int n = g.n_rwg;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int slot = slot_begin + blockIdx.y;
  const int m = e / n, nn = e % n;
  const int dx = slot % (2 * Dx + 1) - Dx;
  const int dy = slot / (2 * Dx + 1) - Dy;
  const V3 off = {dx * px, dy * py, 0.0};
  const double inv4pi = 1.0 / (4.0 * kPi);
  const double invk2 = 1.0 / (k * k);

  double acc_re = 0.0, acc_im = 0.0;
#pragma unroll 1
  for (int a = 0; a < 2; ++a) {
    const int p = g.rwg_tri[2 * m + a];
    const int al = g.rwg_free[2 * m + a];
    V3 P0 = load_vertex(g.tri_v, p, 0) + off;
    V3 P1 = load_vertex(g.tri_v, p, 1) + off;
    V3 P2 = load_vertex(g.tri_v, p, 2) + off;
    V3 va = al == 0 ? P0 : (al == 1 ? P1 : P2);
    const double Ap = g.tri_area[p];
    const double cm = (a == 0 ? 1.0 : -1.0) * g.rwg_len[m] / Ap;
#pragma unroll 1
    for (int b = 0; b < 2; ++b) {
      const int q = g.rwg_tri[2 * nn + b];
      const int be = g.rwg_free[2 * nn + b];
      V3 Q0 = load_vertex(g.tri_v, q, 0);
      V3 Q1 = load_vertex(g.tri_v, q, 1);
      V3 Q2 = load_vertex(g.tri_v, q, 2);
      V3 vb = be == 0 ? Q0 : (be == 1 ? Q1 : Q2);
      const double Aq = g.tri_area[q];
      const double cn = (b == 0 ? 1.0 : -1.0) * g.rwg_len[nn] / Aq;
      // cells of the two triangles (a bridging basis has a triangle in the
      // neighbouring cell)
      int cx = dx, cy = dy;
      if (g.tri_cell) {
        cx += g.tri_cell[2 * p] - g.tri_cell[2 * q];
        cy += g.tri_cell[2 * p + 1] - g.tri_cell[2 * q + 1];
      }
      const bool extract = abs(cx) <= extract_radius && abs(cy) <= extract_radius;
      const int sp = g.tri_state[p], sq = g.tri_state[q];
      const bool overlap = extract && cx == 0 && cy == 0 && sp >= 0 && sq >= 0 && sp != sq;
      const int n_outer = overlap ? kCompPts : 7;
      double t_re = 0.0, t_im = 0.0;
#pragma unroll 1
      for (int i = 0; i < n_outer; ++i) {
        const double* bi = overlap ? c_comp.b[i] : c_quad.b[i];
        V3 r = bi[0] * P0 + bi[1] * P1 + bi[2] * P2;
        const double wi = (overlap ? c_comp.w[i] : c_quad.w[i]) * Ap;
        V3 ra = r - va;
        double s_re = 0.0, s_im = 0.0;
        for (int j = 0; j < 7; ++j) {
          V3 rp = c_quad.b[j][0] * Q0 + c_quad.b[j][1] * Q1 + c_quad.b[j][2] * Q2;
          const double wj = c_quad.w[j] * Aq;
          const double R = norm(r - rp);
          const double kR = k * R;
          double g_re, g_im;
          if (extract) {
            // (exp(-jkR) - 1)/(4 pi R) = (-2 sin^2(kR/2) - j sin(kR)) / (4 pi R)
            if (R == 0.0) {
              g_re = 0.0;
              g_im = -k * inv4pi;
            } else {
              const double sh = sin(0.5 * kR);
              g_re = -2.0 * sh * sh / R * inv4pi;
              g_im = -sin(kR) / R * inv4pi;
            }
          } else {
            double s, c;
            sincos(kR, &s, &c);
            g_re = c / R * inv4pi;
            g_im = -s / R * inv4pi;
          }
          const double kern = 0.25 * dot(ra, rp - vb) - invk2;
          s_re += wj * kern * g_re;
          s_im += wj * kern * g_im;
        }
        t_re += wi * s_re;
        t_im += wi * s_im;
        if (extract) {
          double S;
          V3 V;
          static_potentials(r, Q0, Q1, Q2, S, V);
          // int_q (r' - v_b)/R dS' = V + (r - v_b) S
          V3 inner = V + S * (r - vb);
          t_re += wi * inv4pi * (0.25 * dot(ra, inner) - invk2 * S);
        }
      }
      acc_re += cm * cn * t_re;
      acc_im += cm * cn * t_im;
    }
  }
  // multiply by j k eta
  const double keta = k * kEta0;
  const double z_re = -keta * acc_im;
  const double z_im = keta * acc_re;
  if (!(isfinite(z_re) && isfinite(z_im))) atomicOr(flag, 1);
  const size_t idx = ((size_t)blockIdx.y * n + m) * n + nn;
  out[2 * idx] = (OutT)z_re;
  out[2 * idx + 1] = (OutT)z_im;
}

}  // namespace
}  // namespace r3m

using namespace r3m;

extern "C" {

size_t r3m_blocks_bytes(int32_t n, int32_t Dx, int32_t Dy, r3m_dtype dtype) {
  if (n <= 0 || Dx < 0 || Dy < 0) return 0;
  return (size_t)(2 * Dx + 1) * (2 * Dy + 1) * n * n * dtype_size(dtype);
}

int r3m_fill_unique_blocks(r3m_ctx ctx, const r3m_unit_geom* geom, int32_t Dx, int32_t Dy,
                           r3m_dtype dtype, void* blocks_dev, size_t blocks_bytes,
                           hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    R3M_REQUIRE(Dx >= 0 && Dy >= 0, R3M_ERR_INVALID_ARG, "Dx, Dy must be >= 0");
    R3M_REQUIRE(dtype == R3M_C128 || dtype == R3M_C64, R3M_ERR_UNSUPPORTED, "fill dtype must be C128 or C64");
    R3M_REQUIRE(blocks_dev, R3M_ERR_INVALID_ARG, "blocks_dev is NULL");
    validate_geom(geom);
    const size_t need = r3m_blocks_bytes(geom->n_rwg, Dx, Dy, dtype);
    R3M_REQUIRE(blocks_bytes >= need, R3M_ERR_BUFFER_TOO_SMALL, "blocks buffer too small");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    static bool quad_ready = false;
    static std::mutex quad_mu;
    {
      std::lock_guard<std::mutex> lk(quad_mu);
      if (!quad_ready) {
        Quad7 q = make_quad7();
        R3M_CHECK_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_quad), &q, sizeof(q)));
        QuadComp qc = make_composite(q);
        R3M_CHECK_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_comp), &qc, sizeof(qc)));
        quad_ready = true;
      }
    }
    GeomDev g = upload_geom(ctx, geom, stream);
    const double k = 2.0 * kPi * geom->freq_hz / kC0;
    R3M_CHECK_HIP(hipMemsetAsync(ctx->flag.ptr, 0, sizeof(int), stream));
    const int n = geom->n_rwg;
    const int nslots = (2 * Dx + 1) * (2 * Dy + 1);
    const int per_launch = 65535;
    for (int s0 = 0; s0 < nslots; s0 += per_launch) {
      int cnt = std::min(per_launch, nslots - s0);
      dim3 grid(ceil_div((size_t)n * n, 256), cnt);
      if (dtype == R3M_C128) {
        double* out = (double*)blocks_dev + (size_t)s0 * n * n * 2;
        hipLaunchKernelGGL(fill_blocks_kernel<double>, grid, dim3(256), 0, stream, g, k, geom->period_x,
                           geom->period_y, Dx, Dy, s0, geom->extract_radius, out, (int*)ctx->flag.ptr);
      } else {
        float* out = (float*)blocks_dev + (size_t)s0 * n * n * 2;
        hipLaunchKernelGGL(fill_blocks_kernel<float>, grid, dim3(256), 0, stream, g, k, geom->period_x,
                           geom->period_y, Dx, Dy, s0, geom->extract_radius, out, (int*)ctx->flag.ptr);
      }
      R3M_CHECK_HIP(hipGetLastError());
    }
    int flag = 0;
    R3M_CHECK_HIP(hipMemcpyAsync(&flag, ctx->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, stream));
    R3M_CHECK_HIP(hipStreamSynchronize(stream));
    R3M_REQUIRE(flag == 0, R3M_ERR_NONFINITE, "non-finite entry in the filled blocks");
  });
}

}  // extern "C"
