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
#include "r3m_common.h"

#include <algorithm>

namespace r3m {
namespace {

constexpr int kTW = 4, kTH = 4, kTU = kTW * kTH;

template <typename T>
struct Cx {
  T re, im;
};

template <typename S, typename XT>
__device__ inline Cx<S> load_x(const XT* x, size_t idx) {
  return Cx<S>{(S)x[2 * idx], (S)x[2 * idx + 1]};
}

template <typename S, typename XT>
__global__ void __launch_bounds__(1024)
matvec_tile_kernel(const RhsDev* __restrict__ rhs, const TileDev* __restrict__ tiles, int n_chunks,
                   const uint8_t* __restrict__ states, const S* __restrict__ nearb, int Nx, int Ny,
                   const S* __restrict__ farf, const int* __restrict__ ranks, int max_rank, int Dx,
                   int Dy, int nr, int n, int n_a, int n_states, const XT* __restrict__ x,
                   XT* __restrict__ y, S* __restrict__ partial, int64_t total_units) {
  extern __shared__ unsigned char smem_raw[];
  Cx<S>* tbuf = reinterpret_cast<Cx<S>*>(smem_raw);  // [kTU][max_rank]

  const TileDev tile = tiles[blockIdx.x];
  const int chunk = blockIdx.y;
  const RhsDev R = rhs[tile.b];
  const int t = threadIdx.x;
  const int ul = t / n_a, m = t % n_a;
  const bool active_thread = ul < kTU;
  const int ux = ul % kTW, uy = ul / kTW;
  const int ix = tile.tx + ux, iy = tile.ty + uy;
  const bool vi = active_thread && ix < R.Lx && iy < R.Ly;
  // state bytes >= n_states are clamped (they are rejected by the solver's input check)
  const int si = vi ? min((int)states[R.state_off + (int64_t)iy * R.Lx + ix], n_states - 1) : 0;
  const int offi = si * n_a;

  const int ox_hi = min(tile.tx + kTW, R.Lx) - 1;  // last observer column of the tile
  const int oy_hi = min(tile.ty + kTH, R.Ly) - 1;
  const int Wd = 2 * R.Lx - 1;
  const int nd = Wd * (2 * R.Ly - 1);
  const int NW = 2 * Nx + 1;
  const size_t nn2 = (size_t)n * n;

  S acc_re = 0, acc_im = 0;
  for (int e = chunk; e < nd; e += n_chunks) {
    const int dx = e % Wd - (R.Lx - 1);
    const int dy = e / Wd - (R.Ly - 1);
    // does any observer of the tile have its source inside the array? (uniform)
    if (ox_hi - dx < 0 || tile.tx - dx > R.Lx - 1 || oy_hi - dy < 0 || tile.ty - dy > R.Ly - 1) continue;
    const int jx = ix - dx, jy = iy - dy;
    const bool vj = vi && jx >= 0 && jx < R.Lx && jy >= 0 && jy < R.Ly;
    const int adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
    if (adx <= nr && ady <= nr) {
      if (vj) {
        const int sj = min((int)states[R.state_off + (int64_t)jy * R.Lx + jx], n_states - 1);
        const S* Zb = nearb + ((size_t)((dy + Ny) * NW + (dx + Nx)) * nn2 + (size_t)(offi + m) * n + sj * n_a) * 2;
        const size_t xb = (size_t)(R.unit_off + (int64_t)jy * R.Lx + jx) * n_a;
        for (int c = 0; c < n_a; ++c) {
          const S zr = Zb[2 * c], zi = Zb[2 * c + 1];
          const Cx<S> xv = load_x<S>(x, xb + c);
          acc_re += zr * xv.re - zi * xv.im;
          acc_im += zr * xv.im + zi * xv.re;
        }
      }
    } else {
      const int f = far_index(dx, dy, Dx, Dy, nr);
      const int rank = ranks[f];
      const S* Uf = farf + (size_t)f * 2 * max_rank * n * 2;
      const S* Vf = Uf + (size_t)max_rank * n * 2;
      __syncthreads();
      // stage 1: t[u][rho] = sum_c conj(V[rho][off_j + c]) x_j[c]
      for (int w = t; w < kTU * rank; w += blockDim.x) {
        const int uu = w / rank, rho = w % rank;
        const int jjx = tile.tx + uu % kTW - dx, jjy = tile.ty + uu / kTW - dy;
        const int iix = tile.tx + uu % kTW, iiy = tile.ty + uu / kTW;
        S tr = 0, ti = 0;
        if (iix < R.Lx && iiy < R.Ly && jjx >= 0 && jjx < R.Lx && jjy >= 0 && jjy < R.Ly) {
          const int sj = min((int)states[R.state_off + (int64_t)jjy * R.Lx + jjx], n_states - 1);
          const S* v = Vf + ((size_t)rho * n + sj * n_a) * 2;
          const size_t xb = (size_t)(R.unit_off + (int64_t)jjy * R.Lx + jjx) * n_a;
          for (int c = 0; c < n_a; ++c) {
            const S vr = v[2 * c], vim = v[2 * c + 1];
            const Cx<S> xv = load_x<S>(x, xb + c);
            tr += vr * xv.re + vim * xv.im;
            ti += vr * xv.im - vim * xv.re;
          }
        }
        tbuf[uu * max_rank + rho] = Cx<S>{tr, ti};
      }
      __syncthreads();
      // stage 2: y_i[m] += sum_rho U[rho][off_i + m] t[u][rho]
      if (vj) {
        const S* u = Uf + (size_t)(offi + m) * 2;
        for (int rho = 0; rho < rank; ++rho) {
          const S ur = u[(size_t)rho * n * 2], ui = u[(size_t)rho * n * 2 + 1];
          const Cx<S> tv = tbuf[ul * max_rank + rho];
          acc_re += ur * tv.re - ui * tv.im;
          acc_im += ur * tv.im + ui * tv.re;
        }
      }
    }
  }
  if (!vi) return;
  const size_t yi = (size_t)(R.unit_off + (int64_t)iy * R.Lx + ix) * n_a + m;
  if (partial == nullptr) {
    y[2 * yi] = (XT)acc_re;
    y[2 * yi + 1] = (XT)acc_im;
  } else {
    const size_t pi = ((size_t)chunk * total_units * n_a + yi) * 2;
    partial[pi] = acc_re;
    partial[pi + 1] = acc_im;
  }
}

// y[i][m] = sum over chunks (fixed order) of partial[c][i][m], for the units
// of each tile (units outside every RHS are never touched).
template <typename S, typename XT>
__global__ void __launch_bounds__(1024)
reduce_chunks_kernel(const RhsDev* __restrict__ rhs, const TileDev* __restrict__ tiles,
                     const S* __restrict__ partial, int n_chunks, int64_t total_units, int n_a,
                     XT* __restrict__ y) {
  const TileDev tile = tiles[blockIdx.x];
  const RhsDev R = rhs[tile.b];
  const int ul = threadIdx.x / n_a, m = threadIdx.x % n_a;
  if (ul >= kTU) return;
  const int ix = tile.tx + ul % kTW, iy = tile.ty + ul / kTW;
  if (ix >= R.Lx || iy >= R.Ly) return;
  const size_t e = (size_t)(R.unit_off + (int64_t)iy * R.Lx + ix) * n_a + m;
  const size_t stride = (size_t)total_units * n_a;
  S re = 0, im = 0;
  for (int c = 0; c < n_chunks; ++c) {
    re += partial[((size_t)c * stride + e) * 2];
    im += partial[((size_t)c * stride + e) * 2 + 1];
  }
  y[2 * e] = (XT)re;
  y[2 * e + 1] = (XT)im;
}

}  // namespace

// chunks per tile: enough workgroups to fill the chip several times
int choose_chunks(const BatchDesc& bd, int max_chunks) {
  int want = (int)std::max<int64_t>(1, (2048 + bd.n_tiles - 1) / std::max(1, bd.n_tiles));
  return std::max(1, std::min(want, max_chunks));
}

size_t matvec_partial_bytes(const BatchDesc& bd, int n_a, int chunks, r3m_dtype store_dtype) {
  if (chunks <= 1) return 0;
  const size_t es = store_dtype == R3M_C128 ? 16 : 8;
  return (size_t)chunks * bd.total_units * n_a * es;
}

void validate_store(const r3m_store* Z) {
  R3M_REQUIRE(Z, R3M_ERR_INVALID_ARG, "store is NULL");
  R3M_REQUIRE(Z->n > 0 && Z->n_states >= 1 && Z->n % Z->n_states == 0, R3M_ERR_INVALID_ARG,
              "store n must be a multiple of n_states");
  R3M_REQUIRE(Z->n / Z->n_states <= 64, R3M_ERR_UNSUPPORTED, "at most 64 active RWG per unit");
  R3M_REQUIRE(Z->Dx >= 0 && Z->Dy >= 0 && Z->near_radius >= 0, R3M_ERR_INVALID_ARG, "bad extents");
  R3M_REQUIRE(Z->near, R3M_ERR_INVALID_ARG, "near blocks are NULL");
  R3M_REQUIRE(Z->near_dtype == R3M_C128 || Z->near_dtype == R3M_C64, R3M_ERR_UNSUPPORTED,
              "near dtype must be C128 or C64");
  const bool has_far = Z->near_radius < std::max(Z->Dx, Z->Dy);
  if (has_far) {
    R3M_REQUIRE(Z->far, R3M_ERR_INVALID_ARG, "far factors are NULL");
    R3M_REQUIRE(Z->far_dtype == Z->near_dtype, R3M_ERR_UNSUPPORTED,
                "far and near dtypes must match for this matvec");
    R3M_REQUIRE(Z->max_rank >= 1 && Z->max_rank <= Z->n, R3M_ERR_INVALID_ARG, "bad max_rank");
  }
}

void launch_matvec(r3m_ctx ctx, const r3m_store* Z, const BatchDesc& bd, const uint8_t* states,
                   r3m_dtype vec_dtype, const void* x, void* y, void* partial, int chunks,
                   hipStream_t stream) {
  const int n_a = Z->n / Z->n_states;
  const int Nx = std::min(Z->near_radius, Z->Dx), Ny = std::min(Z->near_radius, Z->Dy);
  const int n_far = r3m_far_count(Z->Dx, Z->Dy, Z->near_radius);
  const size_t head = ((size_t)n_far * 4 + 255) / 256 * 256;
  const int* ranks = n_far > 0 && Z->far ? (const int*)Z->far : nullptr;
  const void* farf = n_far > 0 && Z->far ? (const char*)Z->far + head : nullptr;
  const int threads = ((kTU * n_a + 63) / 64) * 64;
  dim3 grid(bd.n_tiles, chunks);
  const int mr = std::max(1, Z->max_rank);
  const size_t es = Z->near_dtype == R3M_C128 ? 16 : 8;
  const size_t lds = (size_t)kTU * mr * es;
  void* part = chunks > 1 ? partial : nullptr;
#define R3M_LAUNCH_MV(S, XT)                                                                      \
  hipLaunchKernelGGL((matvec_tile_kernel<S, XT>), grid, dim3(threads), lds, stream, bd.rhs, bd.tiles, \
                     chunks, states, (const S*)Z->near, Nx, Ny, (const S*)farf, ranks, mr, Z->Dx,  \
                     Z->Dy, Z->near_radius, Z->n, n_a, Z->n_states, (const XT*)x, (XT*)y, (S*)part, \
                     (int64_t)bd.total_units)
  if (Z->near_dtype == R3M_C128) {
    R3M_REQUIRE(vec_dtype == R3M_C128, R3M_ERR_UNSUPPORTED, "a C128 store needs C128 vectors");
    R3M_LAUNCH_MV(double, double);
  } else if (vec_dtype == R3M_C64) {
    R3M_LAUNCH_MV(float, float);
  } else {
    R3M_LAUNCH_MV(float, double);
  }
#undef R3M_LAUNCH_MV
  R3M_CHECK_HIP(hipGetLastError());
  if (chunks > 1) {
    const int64_t tu = (int64_t)bd.total_units;
    if (Z->near_dtype == R3M_C128)
      hipLaunchKernelGGL((reduce_chunks_kernel<double, double>), dim3(bd.n_tiles), dim3(threads), 0,
                         stream, bd.rhs, bd.tiles, (const double*)partial, chunks, tu, n_a, (double*)y);
    else if (vec_dtype == R3M_C64)
      hipLaunchKernelGGL((reduce_chunks_kernel<float, float>), dim3(bd.n_tiles), dim3(threads), 0,
                         stream, bd.rhs, bd.tiles, (const float*)partial, chunks, tu, n_a, (float*)y);
    else
      hipLaunchKernelGGL((reduce_chunks_kernel<float, double>), dim3(bd.n_tiles), dim3(threads), 0,
                         stream, bd.rhs, bd.tiles, (const float*)partial, chunks, tu, n_a, (double*)y);
    R3M_CHECK_HIP(hipGetLastError());
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
    const BatchDesc& bd = get_batch(ctx, batch, kTW, kTH, 0);
    const int chunks = choose_chunks(bd, 64);
    out = matvec_partial_bytes(bd, Z->n / Z->n_states, chunks, Z->near_dtype);
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
    const BatchDesc& bd = get_batch(ctx, batch, kTW, kTH, stream);
    const int chunks = choose_chunks(bd, 64);
    const size_t need = matvec_partial_bytes(bd, Z->n / Z->n_states, chunks, Z->near_dtype);
    R3M_REQUIRE(work_bytes >= need, R3M_ERR_BUFFER_TOO_SMALL, "matvec workspace too small");
    R3M_REQUIRE(need == 0 || work_dev, R3M_ERR_INVALID_ARG, "work is NULL");
    launch_matvec(ctx, Z, bd, batch->states, vec_dtype, x_dev, y_dev, work_dev, chunks, stream);
  });
}

}  // extern "C"
