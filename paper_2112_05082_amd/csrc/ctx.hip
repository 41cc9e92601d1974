// Context, error reporting, geometry upload and batch descriptors.
#include "r3m_common.h"

#include <algorithm>
#include <array>

namespace r3m {

static thread_local std::string g_thread_error;

void set_thread_error(const std::string& msg) { g_thread_error = msg; }

void DevBuf::ensure(size_t want) {
  if (want <= bytes) return;
  if (ptr) {
    // the previous contents may still be read by queued work
    R3M_CHECK_HIP(hipDeviceSynchronize());
    R3M_CHECK_HIP(hipFree(ptr));
  }
  ptr = nullptr;
  bytes = 0;
  size_t b = std::max<size_t>(want, 4096);
  R3M_CHECK_HIP(hipMalloc(&ptr, b));
  bytes = b;
}

void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

size_t dtype_size(r3m_dtype t) {
  switch (t) {
    case R3M_C128: return 16;
    case R3M_C64: return 8;
    default: return 0;
  }
}

void validate_geom(const r3m_unit_geom* g) {
  R3M_REQUIRE(g, R3M_ERR_INVALID_ARG, "geometry is NULL");
  R3M_REQUIRE(g->freq_hz > 0 && std::isfinite(g->freq_hz), R3M_ERR_INVALID_ARG, "freq_hz must be > 0");
  R3M_REQUIRE(g->period_x > 0 && g->period_y > 0, R3M_ERR_INVALID_ARG, "periods must be > 0");
  R3M_REQUIRE(g->n_states >= 1 && g->n_states <= 256, R3M_ERR_INVALID_ARG, "n_states out of range");
  R3M_REQUIRE(g->state_off && g->vert && g->tri && g->rwg, R3M_ERR_INVALID_ARG, "NULL geometry array");
  R3M_REQUIRE(g->n_vert > 0 && g->n_tri > 0 && g->n_rwg > 0, R3M_ERR_INVALID_ARG, "empty mesh");
  R3M_REQUIRE(g->n_common >= 0 && g->n_common < g->n_rwg, R3M_ERR_INVALID_ARG, "n_common out of range");
  R3M_REQUIRE(g->state_off[0] == 0 && g->state_off[g->n_states] == g->n_rwg - g->n_common, R3M_ERR_INVALID_ARG,
              "state_off must run from 0 to n_rwg - n_common");
  int na = g->state_off[1] - g->state_off[0];
  for (int s = 0; s < g->n_states; ++s)
    R3M_REQUIRE(g->state_off[s + 1] - g->state_off[s] == na && na > 0, R3M_ERR_UNSUPPORTED,
                "every state must own the same number of RWG");
  R3M_REQUIRE(g->extract_radius >= 0, R3M_ERR_INVALID_ARG, "extract_radius must be >= 0");
  for (int t = 0; t < 3 * g->n_tri; ++t)
    R3M_REQUIRE(g->tri[t] >= 0 && g->tri[t] < g->n_vert, R3M_ERR_INVALID_ARG, "triangle vertex out of range");
  for (int m = 0; m < g->n_rwg; ++m) {
    const int32_t* r = g->rwg + 4 * m;
    R3M_REQUIRE(r[0] >= 0 && r[0] < g->n_tri && r[1] >= 0 && r[1] < g->n_tri && r[0] != r[1],
                R3M_ERR_INVALID_ARG, "RWG triangle out of range");
    R3M_REQUIRE(r[2] >= 0 && r[2] < g->n_vert && r[3] >= 0 && r[3] < g->n_vert && r[2] != r[3],
                R3M_ERR_INVALID_ARG, "RWG edge vertex out of range");
  }
  for (int v = 0; v < 3 * g->n_vert; ++v)
    R3M_REQUIRE(std::isfinite(g->vert[v]), R3M_ERR_INVALID_ARG, "non-finite vertex");
  if (g->tri_cell)
    for (int t = 0; t < 2 * g->n_tri; ++t)
      R3M_REQUIRE(std::abs(g->tri_cell[t]) <= 1, R3M_ERR_INVALID_ARG, "tri_cell offsets must be -1, 0 or 1");
}

void require_isolated(const r3m_store* Z) {
  R3M_REQUIRE(Z->n_common == 0, R3M_ERR_UNSUPPORTED,
              "this call does not take shared (connected-geometry) bases yet");
}
void require_isolated(const r3m_unit_geom* g) {
  R3M_REQUIRE(g->n_common == 0 && !g->tri_cell, R3M_ERR_UNSUPPORTED,
              "this call does not take connected geometries yet");
}

std::vector<int32_t> shared_classes(const r3m_unit_geom* g) {
  // from the cells of each shared basis's two triangles: one of them may lie
  // in the -x or the -y neighbour (the bridges a unit owns)
  const int n_st = g->n_rwg - g->n_common;
  std::vector<int32_t> cls(g->n_common, 0);
  for (int c = 0; c < g->n_common; ++c)
    for (int a = 0; a < 2 && g->tri_cell; ++a) {
      const int t = g->rwg[4 * (n_st + c) + a];
      const int ox = g->tri_cell[2 * t], oy = g->tri_cell[2 * t + 1];
      const int here = ox == 0 && oy == 0 ? 0 : ox == -1 && oy == 0 ? 1 : ox == 0 && oy == -1 ? 2 : -1;
      if (here != 0) cls[c] = cls[c] == 0 ? here : -1;
    }
  return cls;
}

void require_extension_classes(const r3m_unit_geom* g) {
  for (int32_t c : shared_classes(g))
    R3M_REQUIRE(c >= 0, R3M_ERR_UNSUPPORTED,
                "a shared basis reaches outside its cell other than into the -x or the -y neighbour");
  const int n_st = g->n_rwg - g->n_common;
  for (int m = 0; m < n_st && g->tri_cell; ++m)
    for (int a = 0; a < 2; ++a) {
      const int t = g->rwg[4 * m + a];
      R3M_REQUIRE(g->tri_cell[2 * t] == 0 && g->tri_cell[2 * t + 1] == 0, R3M_ERR_UNSUPPORTED,
                  "a coding-state basis reaches outside its cell");
    }
}

GeomDev upload_geom(r3m_ctx ctx, const r3m_unit_geom* g, hipStream_t stream) {
  validate_geom(g);
  const int nt = g->n_tri, nr = g->n_rwg;
  std::vector<double> tri_v(9 * (size_t)nt), area(nt), len(nr);
  std::vector<int32_t> rtri(2 * (size_t)nr), rfree(2 * (size_t)nr);
  for (int t = 0; t < nt; ++t) {
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) tri_v[9 * t + 3 * a + c] = g->vert[3 * g->tri[3 * t + a] + c];
    const double* v = &tri_v[9 * t];
    double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    double cx = e1[1] * e2[2] - e1[2] * e2[1];
    double cy = e1[2] * e2[0] - e1[0] * e2[2];
    double cz = e1[0] * e2[1] - e1[1] * e2[0];
    area[t] = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
    R3M_REQUIRE(area[t] > 0, R3M_ERR_INVALID_ARG, "degenerate triangle");
  }
  for (int m = 0; m < nr; ++m) {
    const int32_t* r = g->rwg + 4 * m;
    for (int s = 0; s < 2; ++s) {
      int t = r[s];
      int loc = -1, cnt = 0;
      for (int a = 0; a < 3; ++a) {
        int vid = g->tri[3 * t + a];
        if (vid != r[2] && vid != r[3]) {
          loc = a;
          ++cnt;
        }
      }
      R3M_REQUIRE(cnt == 1, R3M_ERR_INVALID_ARG, "RWG edge is not an edge of its triangle");
      rtri[2 * m + s] = t;
      rfree[2 * m + s] = loc;
    }
    double dx = g->vert[3 * r[2]] - g->vert[3 * r[3]];
    double dy = g->vert[3 * r[2] + 1] - g->vert[3 * r[3] + 1];
    double dz = g->vert[3 * r[2] + 2] - g->vert[3 * r[3] + 2];
    len[m] = std::sqrt(dx * dx + dy * dy + dz * dz);
  }
  // the coding state whose patch holds each triangle (coexistent meshes of
  // the macro unit); triangles of shared bases keep -1
  std::vector<int32_t> tstate(nt, -1);
  for (int s = 0; s < g->n_states; ++s)
    for (int m = g->state_off[s]; m < g->state_off[s + 1]; ++m)
      for (int a = 0; a < 2; ++a) {
        int32_t& ts = tstate[rtri[2 * m + a]];
        R3M_REQUIRE(ts == -1 || ts == s, R3M_ERR_INVALID_ARG, "a triangle carries bases of two coding states");
        ts = s;
      }
  const int n_st = g->n_rwg - g->n_common;
  std::vector<int32_t> cext = shared_classes(g);
  if (cext.empty()) cext.push_back(0);
  size_t off_tv = 0;
  size_t off_ar = off_tv + tri_v.size() * 8;
  size_t off_len = off_ar + area.size() * 8;
  size_t off_rt = off_len + len.size() * 8;
  size_t off_rf = off_rt + rtri.size() * 4;
  size_t off_tc = off_rf + rfree.size() * 4;
  size_t off_ts = off_tc + (g->tri_cell ? 8 * (size_t)nt : 0);
  size_t off_ce = off_ts + 4 * (size_t)nt;
  size_t total = off_ce + 4 * cext.size();
  std::vector<char> host(total);
  std::memcpy(host.data() + off_tv, tri_v.data(), tri_v.size() * 8);
  std::memcpy(host.data() + off_ar, area.data(), area.size() * 8);
  std::memcpy(host.data() + off_len, len.data(), len.size() * 8);
  std::memcpy(host.data() + off_rt, rtri.data(), rtri.size() * 4);
  std::memcpy(host.data() + off_rf, rfree.data(), rfree.size() * 4);
  if (g->tri_cell) std::memcpy(host.data() + off_tc, g->tri_cell, 8 * (size_t)nt);
  std::memcpy(host.data() + off_ts, tstate.data(), 4 * (size_t)nt);
  std::memcpy(host.data() + off_ce, cext.data(), 4 * cext.size());
  // previous users of the table may still be queued on this stream
  R3M_CHECK_HIP(hipStreamSynchronize(stream));
  ctx->geom.ensure(total);
  R3M_CHECK_HIP(hipMemcpyAsync(ctx->geom.ptr, host.data(), total, hipMemcpyHostToDevice, stream));
  R3M_CHECK_HIP(hipStreamSynchronize(stream));
  char* base = (char*)ctx->geom.ptr;
  GeomDev d;
  d.tri_v = (const double*)(base + off_tv);
  d.tri_area = (const double*)(base + off_ar);
  d.rwg_len = (const double*)(base + off_len);
  d.rwg_tri = (const int32_t*)(base + off_rt);
  d.rwg_free = (const int32_t*)(base + off_rf);
  d.tri_cell = g->tri_cell ? (const int32_t*)(base + off_tc) : nullptr;
  d.tri_state = (const int32_t*)(base + off_ts);
  d.common_ext = (const int32_t*)(base + off_ce);
  d.n_st = n_st;
  d.n_common = g->n_common;
  d.n_tri = nt;
  d.n_rwg = nr;
  return d;
}

void validate_batch(const r3m_batch* batch, int Dx, int Dy) {
  R3M_REQUIRE(batch, R3M_ERR_INVALID_ARG, "batch is NULL");
  R3M_REQUIRE(batch->B >= 0, R3M_ERR_INVALID_ARG, "batch size < 0");
  // the right-hand side is a grid dimension of the per-RHS launches
  R3M_REQUIRE(batch->B <= 65535, R3M_ERR_UNSUPPORTED, "at most 65,535 right-hand sides per batch");
  if (batch->B == 0) return;
  R3M_REQUIRE(batch->L && batch->unit_off && batch->state_off && batch->states, R3M_ERR_INVALID_ARG,
              "NULL batch array");
  for (int b = 0; b < batch->B; ++b) {
    int Lx = batch->L[2 * b], Ly = batch->L[2 * b + 1];
    R3M_REQUIRE(Lx >= 1 && Ly >= 1, R3M_ERR_INVALID_ARG, "array size must be >= 1");
    R3M_REQUIRE(Lx <= Dx + 1 && Ly <= Dy + 1, R3M_ERR_INVALID_ARG,
                "array larger than the displacement set of the store");
    R3M_REQUIRE(batch->unit_off[b] >= 0 && batch->state_off[b] >= 0, R3M_ERR_INVALID_ARG,
                "negative offset");
  }
}

// Host side of a batch descriptor: the per-RHS table and the unit tiles,
// packed as they are laid out on the device (rhs table, then tile table).
void describe_batch(const r3m_batch* batch, int tile_w, int tile_h, BatchDesc* d, std::vector<char>& host) {
  d->B = batch->B;
  std::vector<RhsDev> rhs(batch->B);
  std::vector<TileDev> tiles, gtiles;
  std::vector<GroupDev> groups;
  int64_t total = 0;
  std::map<std::vector<int64_t>, int64_t> codebook_at;  // (state_off, Lx, Ly) -> fac_off
  std::map<std::vector<int64_t>, int32_t> open_group;   // (state_off, Lx, Ly) -> group being filled
  std::vector<std::array<int32_t, 3>> gshape;           // group -> (Lx, Ly, first tile) for its tiles
  for (int b = 0; b < batch->B; ++b) {
    int Lx = batch->L[2 * b], Ly = batch->L[2 * b + 1];
    const std::vector<int64_t> ck{batch->state_off[b], Lx, Ly};
    auto f = codebook_at.find(ck);
    const bool lead = f == codebook_at.end();
    if (lead) {
      f = codebook_at.emplace(ck, d->codebook_units).first;
      d->codebook_units += (int64_t)Lx * Ly;
    }
    rhs[b] = RhsDev{batch->unit_off[b], batch->state_off[b], Lx, Ly, f->second, lead ? 1 : 0, 0};
    d->Lx.push_back(Lx);
    d->Ly.push_back(Ly);
    d->unit_off.push_back(batch->unit_off[b]);
    d->n_units.push_back((int64_t)Lx * Ly);
    total = std::max<int64_t>(total, batch->unit_off[b] + (int64_t)Lx * Ly);
    d->max_L = std::max(d->max_L, std::max(Lx, Ly));
    d->max_units = std::max<int64_t>(d->max_units, (int64_t)Lx * Ly);
    for (int ty = 0; ty < Ly; ty += tile_h)
      for (int tx = 0; tx < Lx; tx += tile_w) tiles.push_back(TileDev{b, tx, ty, 0});
    auto g = open_group.find(ck);
    if (g == open_group.end() || groups[g->second].n == kGroupRhs) {
      GroupDev nw{};
      nw.n = 0;
      groups.push_back(nw);
      gshape.push_back({Lx, Ly, 0});
      open_group[ck] = (int32_t)groups.size() - 1;
      g = open_group.find(ck);
    }
    GroupDev& gd = groups[g->second];
    gd.rhs[gd.n++] = b;
    d->max_group_rhs = std::max(d->max_group_rhs, gd.n);
  }
  // group tiles: tile_w wide, and tile_h divided by the group's right-hand
  // sides (rounded up to a power of two) tall
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    GroupDev& gd = groups[gi];
    gd.th = group_tile_h(tile_h, gd.n);
    for (int ty = 0; ty < gshape[gi][1]; ty += gd.th)
      for (int tx = 0; tx < gshape[gi][0]; tx += tile_w) gtiles.push_back(TileDev{(int32_t)gi, tx, ty, 0});
  }
  d->total_units = total;
  d->n_tiles = (int32_t)tiles.size();
  d->n_groups = (int32_t)groups.size();
  d->n_gtiles = (int32_t)gtiles.size();
  const size_t b_rhs = rhs.size() * sizeof(RhsDev), b_t = tiles.size() * sizeof(TileDev);
  const size_t b_g = groups.size() * sizeof(GroupDev), b_gt = gtiles.size() * sizeof(TileDev);
  host.assign(std::max<size_t>(b_rhs + b_t + b_g + b_gt, 16), 0);
  char* h = host.data();
  std::memcpy(h, rhs.data(), b_rhs);
  std::memcpy(h + b_rhs, tiles.data(), b_t);
  std::memcpy(h + b_rhs + b_t, groups.data(), b_g);
  std::memcpy(h + b_rhs + b_t + b_g, gtiles.data(), b_gt);
}

void point_batch(BatchDesc* d, void* dev) {
  char* p = (char*)dev;
  d->rhs = (const RhsDev*)p;
  p += (size_t)d->B * sizeof(RhsDev);
  d->tiles = (const TileDev*)p;
  p += (size_t)d->n_tiles * sizeof(TileDev);
  d->groups = (const GroupDev*)p;
  p += (size_t)d->n_groups * sizeof(GroupDev);
  d->gtiles = (const TileDev*)p;
}

std::vector<int64_t> batch_key(const r3m_batch* batch, int tile_w, int tile_h) {
  std::vector<int64_t> v{tile_w, tile_h};
  v.reserve(2 + 4 * (size_t)batch->B);
  for (int b = 0; b < batch->B; ++b) {
    v.push_back(batch->L[2 * b]);
    v.push_back(batch->L[2 * b + 1]);
    v.push_back(batch->unit_off[b]);
    v.push_back(batch->state_off[b]);
  }
  return v;
}

// Bounded cache: when full, the descriptors no call of the current entry has
// used are released, together with every captured graph and autotuned launch
// shape (their keys hold descriptor addresses).
static void evict_batches(r3m_ctx ctx) {
  R3M_CHECK_HIP(hipDeviceSynchronize());  // queued work may still read the tables
  for (auto it = ctx->batches.begin(); it != ctx->batches.end();) {
    if (it->second->epoch != ctx->epoch) {
      it->second->dev.release();
      delete it->second;
      it = ctx->batches.erase(it);
    } else {
      ++it;
    }
  }
  for (auto& kv : ctx->graphs) R3M_CHECK_HIP(hipGraphExecDestroy(kv.second));
  ctx->graphs.clear();
  ctx->tuned_groups.clear();
}

const BatchDesc& get_batch(r3m_ctx ctx, const r3m_batch* batch, int tile_w, int tile_h,
                           hipStream_t stream) {
  BatchKey key;
  key.states = nullptr;  // the descriptor holds offsets only
  key.v = batch_key(batch, tile_w, tile_h);
  auto it = ctx->batches.find(key);
  if (it != ctx->batches.end()) {
    it->second->epoch = ctx->epoch;
    return *it->second;
  }
  if (ctx->batches.size() >= kMaxBatches) evict_batches(ctx);

  auto* d = new BatchDesc();
  std::vector<char> host;
  describe_batch(batch, tile_w, tile_h, d, host);
  d->dev.ensure(host.size());
  R3M_CHECK_HIP(hipMemcpyAsync(d->dev.ptr, host.data(), host.size(), hipMemcpyHostToDevice, stream));
  R3M_CHECK_HIP(hipStreamSynchronize(stream));
  point_batch(d, d->dev.ptr);
  d->epoch = ctx->epoch;
  ctx->batches[key] = d;
  return *d;
}

// One thread per unit of every codebook (the first right-hand side of each):
// a state byte >= n_states sets `bit` in *word.
__global__ void __launch_bounds__(256)
bad_states_kernel(const RhsDev* __restrict__ rhs, const uint8_t* __restrict__ states, int n_states, int* word,
                  int bit) {
  const RhsDev R = rhs[blockIdx.y];
  if (!R.fac_lead) return;
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= (int64_t)R.Lx * R.Ly) return;
  if (states[R.state_off + u] >= n_states) atomicOr(word, bit);
}

void check_states(const BatchDesc& bd, const uint8_t* states, int n_states, int* word, int bit, hipStream_t s) {
  if (bd.B == 0) return;
  hipLaunchKernelGGL(bad_states_kernel, dim3(ceil_div((size_t)bd.max_units, 256), bd.B), dim3(256), 0, s, bd.rhs,
                     states, n_states, word, bit);
  R3M_CHECK_HIP(hipGetLastError());
}

int* deferred_word(r3m_ctx ctx) { return (int*)ctx->flag.ptr + kDeferredWord; }

void take_deferred(r3m_ctx ctx, hipStream_t s) {
  int w = 0;
  R3M_CHECK_HIP(hipMemcpyAsync(&w, deferred_word(ctx), sizeof(int), hipMemcpyDeviceToHost, s));
  R3M_CHECK_HIP(hipStreamSynchronize(s));
  if (w == 0) return;
  R3M_CHECK_HIP(hipMemsetAsync(deferred_word(ctx), 0, sizeof(int), s));
  R3M_CHECK_HIP(hipStreamSynchronize(s));
  R3M_REQUIRE(!(w & kDeferredBadState), R3M_ERR_INVALID_ARG,
              "a codebook given to an earlier asynchronous call has a state byte >= n_states");
}

}  // namespace r3m

using namespace r3m;

extern "C" {

int r3m_ctx_create(r3m_ctx* out, int device) {
  if (!out) {
    set_thread_error("out is NULL");
    return R3M_ERR_INVALID_ARG;
  }
  *out = nullptr;
  r3m_ctx ctx = new r3m_ctx_s();
  int rc = guarded(nullptr, [&] {
    int count = 0;
    R3M_CHECK_HIP(hipGetDeviceCount(&count));
    R3M_REQUIRE(device >= 0 && device < count, R3M_ERR_HIP, "no such HIP device");
    R3M_CHECK_HIP(hipSetDevice(device));
    ctx->device = device;
    ctx->flag.ensure(256);
    R3M_CHECK_HIP(hipMemset(ctx->flag.ptr, 0, 256));
    init_static_scratch(device);
  });
  if (rc != R3M_OK) {
    delete ctx;
    return rc;
  }
  *out = ctx;
  return R3M_OK;
}

int r3m_ctx_destroy(r3m_ctx ctx) {
  if (!ctx) return R3M_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
  if (ctx->work_stream) (void)hipStreamDestroy(ctx->work_stream);
  if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
  if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
  for (hipEvent_t e : ctx->ev_run)
    if (e) (void)hipEventDestroy(e);
  if (ctx->run_host) (void)hipHostFree(ctx->run_host);
  ctx->flag.release();
  ctx->geom.release();
  for (auto& kv : ctx->batches) {
    kv.second->dev.release();
    delete kv.second;
  }
  delete ctx;
  return R3M_OK;
}

const char* r3m_last_error(r3m_ctx ctx) {
  if (ctx) return ctx->last_error.c_str();
  return g_thread_error.c_str();
}

const char* r3m_version(void) { return "r3m 0.2 gfx950"; }

int r3m_ctx_check(r3m_ctx ctx, hipStream_t stream) {
  return guarded(ctx, [&] {
    R3M_REQUIRE(ctx, R3M_ERR_INVALID_ARG, "ctx is NULL");
    R3M_CHECK_HIP(hipSetDevice(ctx->device));
    take_deferred(ctx, stream);
  });
}

}  // extern "C"
