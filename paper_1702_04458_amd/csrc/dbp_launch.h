// Kernel argument blocks and launcher declarations (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dbp {

struct c32;

// per-subcarrier status bits (the values of DBP_STATUS_NONFINITE / DBP_STATUS_RESLICED)
constexpr int kStatusNonfinite = 1;
constexpr int kStatusReslice = 2;
constexpr int kStatusIllcond = 4;
// workgroups (FP64 slots) of the re-slice pass at most
constexpr int kFixMaxSlots = 256;

struct UlArgs {
  const c32* H;       // [n_sc][B][U]
  const c32* y;       // [n_sc][n_sym][B]
  c32* shat;          // [n_sc][n_sym][U]
  uint8_t* hard;      // [n_sc][n_sym][U] or null
  int n_sc, n_sym, B, C, Cp, S, T;
  int sc_per_block;
  int reg;            // 0 MMSE, 1 ZF, 2 BOX
  int L;              // QAM levels per dimension
  float rho;          // ADMM penalty (Alg. 1) or N0/Es regulariser (Alg. 2)
  float gamma;
  float inv_den;      // 1 / (N0/(rho Es) + C)  (MMSE), 1 / C (ZF)
  float invC;
  float box_r;
  float kappa;
  c32* fac;           // [n_sc][C][U(U+1)/2] resident factors B_c^{-1}: upper triangle, entry (i, v), i <= v, at v(v+1)/2 + i; or null
  const uint32_t* H16;  // [n_sc][B][U] packed FP16 channel (real part in the low half), or null
  const float* hscale;  // [n_sc][C] power-of-two scale of each (subcarrier, cluster) tile of H16
  int32_t* flags;     // [n_sc] per-subcarrier status bits written by the detection kernels, or null
  float guard;        // re-slice guard in slicer units t = (kappa x + L) / 2; 0: no re-slice
  int nw;             // waves per workgroup of the call's launch plan
  int blk;            // block index within this frame's launch (set by the kernel)
  // FP64 factor rule of the mixed modes: a subcarrier with a cluster whose
  // estimate tr(B_c) ||B_c^{-1}||_F exceeds cond_max is flagged for the FP64
  // pass (kStatusReslice | kStatusIllcond); 0: off; < 0: every subcarrier.
  // Below it the re-slice guard is scaled by max(1, estimate / cond_ref).
  float cond_max;
  float cond_ref;
  // *any is set to epoch by the kernels when they flag a subcarrier for the
  // FP64 pass; the pass does nothing unless it reads this call's epoch there
  // (epoch before the pointer: no padding, the batch block stays in 4 KiB).
  uint32_t epoch;
  uint32_t* any;
};

// Exact re-slicing: the subcarriers the FP32 kernel flagged (a soft value
// within the guard of a decision threshold) are recomputed in FP64 and their
// outputs overwritten.
struct FixArgs {
  const c32* H;       // [n_sc][B][U]
  const c32* y;       // [n_sc][n_sym][B]
  c32* shat;          // [n_sc][n_sym][U]
  uint8_t* hard;      // [n_sc][n_sym][U] or null (the FP64 factor rule without hard decisions)
  int32_t* flags;     // [n_sc] status bits of the FP32 pass (read; the re-slice bit is kept)
  void* ws;           // n_slots blocks of C U^2 complex FP64 (ADMM), or null (CG)
  int* list0;         // [n_slots] subcarriers recomputed with one workgroup per cluster (split)
  int split;          // 1: each workgroup's first subcarrier goes to the per-cluster kernels
  int n_sc, n_sym, B, U, C, S, T, reg, L, n_slots;
  const uint32_t* any;   // equals epoch when the FP32 pass flagged any subcarrier of this call
  uint32_t epoch;
  double rho;         // ADMM penalty (Alg. 1) or N0/Es (Alg. 2)
  double gamma, inv_den, invC, box_r, kappa;
};

struct DlArgs {
  const c32* H;       // [n_sc][B][U] uplink layout
  const c32* s;       // [n_sc][n_sym][U]
  c32* x;             // [n_sc][n_sym][B]
  float* beta;        // [n_sc][n_sym] or null
  const float* P;     // [C] device per-cluster budgets or null
  int n_sc, n_sym, B, C, Cp, S, T;
  int sc_per_block;
  float rho, gamma, invC, f0;
  float eps;          // radius of ||s - sum_c z_c|| <= eps (Lemma 2); 0 = equality (Alg. 3)
  int budget;         // with P: 0 common gain after Algorithm 3, 1 budgeted step (P1) in every x-update
  int h_layout;       // 0: H in the uplink layout [n_sc][B][U]; 1: downlink layout [n_sc][U][B]
};

// Several frames of one U in one launch: the argument blocks travel by value
// in the kernel arguments (at most 4 KiB), so a batch needs no device copy.
constexpr int kMaxBatch = 24;
struct UlBatch {
  UlArgs f[kMaxBatch];
  int first[kMaxBatch + 1];   // first virtual block of each frame, first[n] = total
  int n;
};
struct FixBatch {
  FixArgs f[kMaxBatch];
  int n;
};
static_assert(sizeof(UlBatch) <= 4096 && sizeof(FixBatch) <= 4096, "kernel argument blocks exceed 4 KiB");

size_t smem_bytes(int nw);
// persistent launch of grid workgroups (nw waves each) over all frames of b
hipError_t launch_admm_ul_f32_batch(const UlBatch& b, int U, int nw, int grid, hipStream_t st);
// FP64 re-slice of the flagged subcarriers of every frame of b
hipError_t launch_admm_ul_fix64_batch(const FixBatch& b, int U, int n_slots, hipStream_t st);
// stage: 0 detect, 1 only factor (write B_c^{-1} to a.fac)
hipError_t launch_admm_ul_f32(const UlArgs& a, int U, int nw, hipStream_t st, int stage = 0);
// U = 32, FP32: the factors and, in the same launch, H as the packed FP16
// channel (a.H16 / a.hscale, written)
hipError_t launch_factor_pack_u32(const UlArgs& a, int nw, hipStream_t st);
// inv: 0 FP32 matrix-core inverse, 1 FP64 VALU inverse (U = 32), 2 split-FP16 matrix-core inverse
hipError_t launch_admm_ul_mixed(const UlArgs& a, int U, int half, int inv, int nw, hipStream_t st, int stage = 0);
// detection against resident factors a.fac (no Gram, no inverse)
hipError_t launch_admm_ul_factored(const UlArgs& a, int U, int nw, hipStream_t st);
// the same with H read from the packed FP16 channel a.H16 / a.hscale
hipError_t launch_admm_ul_factored_h16(const UlArgs& a, int U, int nw, hipStream_t st);
// H [n_sc][B][U] complex64 -> H16 (same layout, complex FP16) and hscale [n_sc][C]
hipError_t launch_pack_h16(const c32* H, uint32_t* H16, float* hscale, int n_sc, int B, int U, int C,
                           hipStream_t st);
hipError_t launch_dcg_ul_f32(const UlArgs& a, int U, int nw, hipStream_t st);
// status[k] = 1 if any of the floats_per_sc floats of subcarrier k is NaN or infinite, else 0
hipError_t launch_scan_nonfinite(const float* x, size_t floats_per_sc, int n_sc, int32_t* status,
                                 hipStream_t st);
hipError_t launch_admm_dl_f32(const DlArgs& a, int U, int nw, hipStream_t st);

// Library-internal pieces of the C entry points (dbp_capi.cpp).
int set_error(int code, const char* msg);   // records msg for dbp_last_error, returns code
// smallest re-slice workspace of a call with hard decisions: the flag region
// (none when the caller passes a status array) and one FP64 slot
size_t reslice_bytes_min(int n_sc, int U, int C, bool with_status);
int detect_admm_impl(const char* who, const void* H, const void* y, void* s_hat, uint8_t* hard, int32_t* status,
                     void* workspace, size_t workspace_bytes, int max_slots, int n_sc, int n_sym, int B, int U, int C,
                     int T, float rho, float gamma, float N0, float Es, int reg, int qam, int prec, void* stream);

// FP64 recomputation of the flagged subcarriers (Algorithm 1 or 2), n_slots workgroups
hipError_t launch_admm_ul_fix64(const FixArgs& f, hipStream_t st);
hipError_t launch_dcg_ul_fix64(const FixArgs& f, hipStream_t st);
// bytes of one FP64 slot of the ADMM re-slice (C blocks of U x U complex FP64)
size_t fix64_slot_bytes(int U, int C);

}  // namespace dbp
