// Internal declarations shared by the translation units of libr3m.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "r3m.h"

namespace r3m {

// ----------------------------------------------------------------- errors

struct Error {
  int code;
  std::string msg;
};

void set_thread_error(const std::string& msg);

#define R3M_CHECK_HIP(expr)                                                          \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      throw ::r3m::Error{R3M_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define R3M_REQUIRE(cond, code, text)                                     \
  do {                                                                    \
    if (!(cond)) throw ::r3m::Error{(code), std::string(text)};           \
  } while (0)

// ------------------------------------------------------------- constants

constexpr double kPi = 3.14159265358979323846;
constexpr double kC0 = 299792458.0;
constexpr double kMu0 = 4.0e-7 * kPi;
constexpr double kEta0 = kMu0 * kC0;

// ----------------------------------------------------------- device pool

// Small device tables owned by the context (geometry, batch descriptors).
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  void ensure(size_t want);
  void release();
};

struct BatchKey {
  std::vector<int64_t> v;
  const void* states;
  bool operator<(const BatchKey& o) const {
    if (states != o.states) return states < o.states;
    return v < o.v;
  }
};

// Device descriptor of a batch for a given unit-tile shape and chunk count.
struct BatchDesc {
  int32_t B = 0;
  int64_t total_units = 0;
  int32_t n_tiles = 0;
  int32_t max_L = 0;
  int64_t max_units = 0;  // largest Lx * Ly of the batch
  DevBuf dev;  // rhs table [B], tile table [n_tiles], group table [n_groups], group tiles [n_gtiles]
  const struct RhsDev* rhs = nullptr;
  const struct TileDev* tiles = nullptr;
  // right-hand sides sharing a codebook (same state bytes and array shape),
  // up to kGroupRhs per group, and the unit tiles of each group (TileDev.b =
  // group index)
  int32_t n_groups = 0, n_gtiles = 0, max_group_rhs = 0;
  const struct GroupDev* groups = nullptr;
  const struct TileDev* gtiles = nullptr;
  std::vector<int64_t> unit_off, n_units;
  std::vector<int32_t> Lx, Ly;
  int64_t codebook_units = 0;  // units of the distinct codebooks (RhsDev::fac_off)
  uint64_t epoch = 0;          // entry call that last used it (cache eviction)
};

struct RhsDev {
  int64_t unit_off;
  int64_t state_off;
  int32_t Lx, Ly;
  // per-codebook data (the near-field factors): right-hand sides with equal
  // state_off and array shape share one codebook; fac_off is its unit offset
  // among the distinct codebooks, fac_lead is 1 for its first right-hand side
  int64_t fac_off;
  int32_t fac_lead, pad;
};

struct TileDev {
  int32_t b;   // RHS
  int32_t tx;  // first unit column
  int32_t ty;  // first unit row
  int32_t pad;
};

constexpr int kGroupRhs = 4;
struct GroupDev {
  int32_t n;               // right-hand sides in the group (1..kGroupRhs)
  int32_t rhs[kGroupRhs];  // their indices; rhs[0] carries the codebook
  int32_t th;              // height of the group's unit tiles (width: the call's tile width)
  int32_t pad[2];
};
// tile height of a group of n right-hand sides: tile_h / (n rounded up to a power of two), at least 1
inline int group_tile_h(int tile_h, int n) {
  const int p = n <= 1 ? 1 : n <= 2 ? 2 : 4;
  return tile_h / p > 0 ? tile_h / p : 1;
}

}  // namespace r3m

struct r3m_ctx_s {
  int device = 0;
  std::string last_error;
  std::mutex mu;
  r3m::DevBuf flag;  // int32 flags for device-side checks
  r3m::DevBuf geom;  // geometry tables
  std::map<r3m::BatchKey, r3m::BatchDesc*> batches;
  hipStream_t work_stream = nullptr;  // default-priority stream for graph replays
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int* run_host = nullptr;                   // pinned [2]: running counts read back without a stall
  hipEvent_t ev_run[2] = {nullptr, nullptr};  // completion of those read-backs
  std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
  std::map<std::vector<int64_t>, int> tuned_groups;  // autotuned (or pinned) matvec plans per (store, batch)
  uint64_t epoch = 0;  // counts entry calls (see get_batch)
};

namespace r3m {

// Host-side geometry preprocessing (connectivity only) and upload.
struct GeomDev {
  const double* tri_v;    // [n_tri][9]
  const double* tri_area; // [n_tri]
  const int32_t* rwg_tri; // [n_rwg][2]
  const int32_t* rwg_free;// [n_rwg][2] local index of the free vertex
  const double* rwg_len;  // [n_rwg]
  const int32_t* tri_cell;// [n_tri][2] lattice offset of each triangle's cell, or NULL
  const int32_t* tri_state;// [n_tri] coding state of the bases a triangle carries, -1 for shared bases
  // shared bases (connected geometries): the first is macro RWG n_st; class of
  // each from its triangles' cells: 0 inside the cell, 1 reaching into the
  // -x neighbour, 2 into the -y neighbour, -1 any other reach
  const int32_t* common_ext;
  int32_t n_st, n_common;
  int32_t n_tri, n_rwg;
};

// entries per unit of a solution vector: the state's n_a bases, then the
// shared ones
inline int vec_per_unit(const r3m_store* Z) {
  return (Z->n - Z->n_common) / Z->n_states + Z->n_common;
}
inline int vec_per_unit(const r3m_unit_geom* g) {
  return (g->n_rwg - g->n_common) / g->n_states + g->n_common;
}

// Macro RWG of compact entry r of a unit in state s at lattice position (ix,
// iy), or -1 where D_k masks an extended basis (one that reaches into a
// neighbour the array does not have, Sec. III-B).
__device__ inline int compact_to_macro(const GeomDev& g, int n_a, int s, int r, int64_t ix, int64_t iy) {
  if (r < n_a) return s * n_a + r;
  const int c = r - n_a;
  const int e = g.common_ext[c];
  if ((e == 1 && ix == 0) || (e == 2 && iy == 0)) return -1;
  return g.n_st + c;
}

void validate_geom(const r3m_unit_geom* g);
// calls that do not take connected geometries yet (shared bases)
void require_isolated(const r3m_store* Z);
void require_isolated(const r3m_unit_geom* g);
// class of each shared basis of a geometry (see GeomDev::common_ext)
std::vector<int32_t> shared_classes(const r3m_unit_geom* g);
// calls that need every shared basis to have a class (0, 1 or 2)
void require_extension_classes(const r3m_unit_geom* g);
GeomDev upload_geom(r3m_ctx ctx, const r3m_unit_geom* g, hipStream_t stream);

// At most kMaxBatches descriptors are cached per context; a new one beyond
// that releases those the current entry call has not used (and every captured
// graph and autotuned launch shape, whose keys hold descriptor addresses).
constexpr size_t kMaxBatches = 64;
const BatchDesc& get_batch(r3m_ctx ctx, const r3m_batch* batch, int tile_w, int tile_h,
                           hipStream_t stream);
// host tables of a batch (rhs table, then tiles) and the device pointers into them
void describe_batch(const r3m_batch* batch, int tile_w, int tile_h, BatchDesc* d, std::vector<char>& host);
void point_batch(BatchDesc* d, void* dev);
std::vector<int64_t> batch_key(const r3m_batch* batch, int tile_w, int tile_h);
// Errors found on the device by asynchronous calls are kept in a word of the
// context's flag buffer and reported by the next call that synchronises and
// reads it (r3m_ctx_check, r3m_gmres_solve).
constexpr int kDeferredWord = 16;      // int index in ctx->flag
constexpr int kDeferredBadState = 1;   // a state byte >= n_states
int* deferred_word(r3m_ctx ctx);
// reads (and clears) the deferred word; throws the error it records
void take_deferred(r3m_ctx ctx, hipStream_t s);
// sets `bit` in *word if any codebook of the batch has a state byte >= n_states
void check_states(const BatchDesc& bd, const uint8_t* states, int n_states, int* word, int bit, hipStream_t s);
// looks up the device address of the library's static scratch on `device`
// (current), once per device; called by r3m_ctx_create
void init_static_scratch(int device);
void validate_batch(const r3m_batch* batch, int Dx, int Dy);

inline int32_t slot_of(int dx, int dy, int Dx, int Dy) { return (dy + Dy) * (2 * Dx + 1) + (dx + Dx); }

// far index of displacement d among far slots (near = Chebyshev <= nr)
__host__ __device__ inline int32_t far_index(int dx, int dy, int Dx, int Dy, int nr) {
  int Nx = nr < Dx ? nr : Dx;
  int Ny = nr < Dy ? nr : Dy;
  int slot = (dy + Dy) * (2 * Dx + 1) + (dx + Dx);
  int before;
  if (dy > Ny) {
    before = (2 * Ny + 1) * (2 * Nx + 1);
  } else if (dy < -Ny) {
    before = 0;
  } else {
    before = (dy + Ny) * (2 * Nx + 1) + (dx < -Nx ? 0 : (2 * Nx + 1));
  }
  return slot - before;
}

size_t dtype_size(r3m_dtype t);

// Seven-point degree-5 triangle rule (Radon; Dunavant degree 5): barycentric
// point i and its weight (weights sum to one).
__host__ __device__ inline void quad7_point(int i, double& b0, double& b1, double& b2, double& w) {
  const double s15 = sqrt(15.0);
  const double a1 = (6.0 - s15) / 21.0, c1 = 1.0 - 2.0 * a1;
  const double a2 = (6.0 + s15) / 21.0, c2 = 1.0 - 2.0 * a2;
  if (i == 0) {
    b0 = b1 = b2 = 1.0 / 3.0;
    w = 9.0 / 40.0;
    return;
  }
  const bool first = i <= 3;
  const double a = first ? a1 : a2, c = first ? c1 : c2;
  const int k = (i - 1) % 3;
  b0 = k == 0 ? c : a;
  b1 = k == 1 ? c : a;
  b2 = k == 2 ? c : a;
  w = first ? (155.0 - s15) / 1200.0 : (155.0 + s15) / 1200.0;
}

// guarded entry: converts exceptions into status codes
template <class F>
int guarded(r3m_ctx ctx, F&& f) {
  if (ctx) ++ctx->epoch;
  try {
    f();
    return R3M_OK;
  } catch (const Error& e) {
    if (ctx) ctx->last_error = e.msg;
    set_thread_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    if (ctx) ctx->last_error = e.what();
    set_thread_error(e.what());
    return R3M_ERR_INVALID_ARG;
  }
}

inline unsigned ceil_div(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace r3m
