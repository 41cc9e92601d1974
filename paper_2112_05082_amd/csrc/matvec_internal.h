// Library-internal interface of the retrieved matvec (used by the solver).
#pragma once
#include "r3m_common.h"

namespace r3m {

void validate_store(const r3m_store* Z);
// A matvec plan (the value the autotuner keeps per store and batch).
// Compressed stores: the displacement-group count in the low bits,
// kPlanMfmaFar for the matrix-core far kernel.  Spectral stores: kPlanSpectral,
// the frequency-product shape in bits 0-3 (kSpecShapes) and in bits 4-11 the
// count of live 16-RHS tiles from which the matrix-core product orders its
// workgroups RHS tile first, in bits 13-14 how the XCDs share the frequency
// tiles in that order, and kPlanSpecTwoPass for the row and column
// transform passes through HBM where the fused 2-D transform would apply
constexpr int kPlanGroups = 0xffff;
constexpr int kPlanMfmaFar = 1 << 16;
constexpr int kPlanSpectral = 1 << 17;
constexpr int kPlanSpecTwoPass = 1 << 12;
static_assert(kPlanMfmaFar == R3M_PLAN_MFMA_FAR && kPlanSpectral == R3M_PLAN_SPECTRAL &&
                  kPlanSpecTwoPass == R3M_PLAN_SPEC_TWO_PASS,
              "plan bits as published");
// frequency-product shapes: {frequencies per wave, columns per staged chunk}
// of the matrix-core kernel; {0, 0} is the vector-unit kernel (register tile
// by batch width)
struct SpecShape {
  int kpw, pc, rb;  // frequencies per wave, columns per staged chunk, 16-RHS tiles per workgroup
};
constexpr SpecShape kSpecShapes[] = {{0, 0, 0}, {1, 4, 1}, {2, 4, 1}, {2, 8, 1}, {4, 4, 1},
                                     {1, 8, 1}, {2, 4, 2}, {1, 8, 2}};
constexpr int kSpecShapeCount = (int)(sizeof(kSpecShapes) / sizeof(kSpecShapes[0]));
constexpr int kSpecRhsFirst = 8;  // default ordering threshold
// the default threshold of a shape: workgroups of two 16-RHS tiles keep the
// contiguous order up to 64 live tiles (measured on the 1,536-RHS solve:
// 7.29, 7.17, 7.13, 7.10 s at 8, 24, 40, 64; 7.81 s never RHS tile first)
inline int spec_default_rf(int shape) { return kSpecShapes[shape].rb == 2 ? 64 : kSpecRhsFirst; }
inline int spec_plan(int shape, int rhs_first) { return kPlanSpectral | shape | rhs_first << 4; }
inline int spec_shape(int plan) { return plan & 15; }
inline int spec_rhs_first(int plan) { return (plan >> 4) & 255; }
// bits 13-14: log2 of the frequency-tile-pair groups the XCDs form in the
// RHS-first order (0: every XCD sees every frequency tile)
inline int spec_kt_groups(int plan) { return (plan >> 13) & 3; }
// the untuned plan: matrix cores for complex64 spectra once a 16-wide RHS
// tile is mostly full, the vector units otherwise
int spectral_default_plan(const r3m_store* Z, int B);
// the plan is valid for this store (shape and threshold in range)
bool spectral_plan_valid(const r3m_store* Z, int plan);
// the store's retrieval transforms can run fused (complex64 grids that fit LDS)
bool spectral_fused_transforms(const r3m_store* Z);
int choose_chunks(const BatchDesc& bd, int max_chunks);
// largest displacement-group count the autotuner may pick (workspaces are sized for it)
int max_groups(const BatchDesc& bd);
// the autotuned plan of (store, batch) if known, else the default
int plan_groups(r3m_ctx ctx, const r3m_store* Z, const BatchDesc& bd);
// times candidate plans once per (store, batch); xs in the store precision, y C128
int tuned_groups(r3m_ctx ctx, const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, const void* xs,
                 void* y, void* partial, const void* lists, hipStream_t stream);
// matvec workspace: partial slots, converted x, near retrieval lists
size_t matvec_partial_bytes(const BatchDesc& bd, const r3m_store* Z, int chunks);
// the same without the lists (for callers that keep the lists elsewhere)
size_t partials_and_x_bytes(const BatchDesc& bd, const r3m_store* Z, int chunks);
size_t near_lists_bytes(const r3m_store* Z, const BatchDesc& bd);
size_t near_lists_bytes_bound(int n_states, const BatchDesc& bd);
void build_near_lists(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, void* lists_dev,
                      hipStream_t stream);
// y (C128 or C64 vectors); lists NULL: the ones inside partial.  idle
// (device, nullable, one int per right-hand side): the output of a right-hand
// side b with idle[b] != 0 is not computed and keeps whatever it held (the
// vector-unit far tiles, the reduction and every spectral pass skip it; the
// matrix-core near items, which mix right-hand sides, still run)
void launch_matvec(r3m_ctx ctx, const r3m_store* Z, const BatchDesc& bd, const uint8_t* states,
                   r3m_dtype vec_dtype, const void* x, void* y, void* partial, const void* lists, int chunks,
                   hipStream_t stream, const int* idle = nullptr);
// xs already in the store precision; y C128.  live (device, nullable): the
// kernels return at once when *live == 0 (used to skip Arnoldi steps after
// every right-hand side has converged); idle as above
// rl (device, nullable): the right-hand sides with work, as a list (rl[0..n)
// indices, rl[B] = n, every other one idle); the spectral transforms then
// visit only their grids; y_type: R3M_C128, or R3M_C64 on spectral stores
void launch_matvec_pre(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, const void* xs, void* y,
                       void* partial, const void* lists, int chunks, hipStream_t stream, const int* live,
                       const int* idle = nullptr, const int* rl = nullptr, r3m_dtype y_type = R3M_C128);

// spectral stores (far_dtype R3M_SPEC_*): the whole product by FFT
bool store_is_spectral(const r3m_store* Z);
void validate_spectral(const r3m_store* Z);
size_t spectral_work_bytes(const BatchDesc& bd, const r3m_store* Z);
// x (x_type) to y (y_type); work: spectral_work_bytes; live and idle as above
// plan: a spectral plan (kPlanSpectral set), anything else takes the default
void launch_spectral(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, r3m_dtype x_type,
                     const void* x, r3m_dtype y_type, void* y, void* work, hipStream_t s, const int* live,
                     const int* idle = nullptr, int plan = 0, const int* rl = nullptr);
// relaxed retrieval (wts [units][n_states], nullable) and the transposed operator
void launch_spectral_ex(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, r3m_dtype x_type,
                        const void* x, r3m_dtype y_type, void* y, void* work, hipStream_t s, const int* live,
                        const double* wts, bool tr, const int* idle = nullptr, int plan = 0);
// the per-frequency product alone, on the transformed input grids in work
// (spectral_work_bytes layout) into the output grids there
void launch_spectral_product(const r3m_store* Z, const BatchDesc& bd, void* work, int plan, hipStream_t s);
// times the frequency-product shapes once per (store, batch) on x (x_type) into
// y (y_type) and keeps the fastest plan (the same map as tuned_groups)
int tuned_spectral(r3m_ctx ctx, const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, r3m_dtype x_type,
                   const void* x, r3m_dtype y_type, void* y, void* work, hipStream_t stream);

// near-field block ILU(0) (r3m_ilu_*): factors of every distinct codebook
// (shared: right-hand sides with the same codebook share them; relaxed
// weights are per right-hand side, so those factors are not shared)
void validate_ilu(const r3m_store* Z, int radius);
size_t ilu_factor_bytes(const r3m_store* Z, const BatchDesc& bd, int radius, bool shared = true);
// retrieval of the pattern blocks, then one launch per colour; singular
// pivots set bit 8 of *flag.  wts (nullable): relaxed weights [unit][n_states]
// (blended blocks; tr: of the transposed operator)
void launch_ilu_factor(const r3m_store* Z, const BatchDesc& bd, const uint8_t* states, int radius, void* F,
                       int* flag, hipStream_t s, const double* wts = nullptr, bool tr = false);
// z = M^-1 in (C128; z must not alias in); out (nullable, C128 or C64 per
// out_type) receives a copy.  live as for the matvec
void launch_ilu_apply(const r3m_store* Z, const BatchDesc& bd, int radius, const void* F, const double2* in,
                      double2* z, r3m_dtype out_type, void* out, hipStream_t s, const int* live,
                      bool shared = true);

}  // namespace r3m
