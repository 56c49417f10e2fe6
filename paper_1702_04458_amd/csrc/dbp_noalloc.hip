// dbp_detect_admm_noalloc: the ADMM detection entry point for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).  The only device memory the
// detection path needs beyond the caller's inputs and outputs is the
// workspace of the exact FP64 re-slice (a flag per subcarrier and the FP64
// regularised inverses of the subcarriers being recomputed).  This variant
// takes it from a file-scope device array instead of a workspace argument.
//
// The array's name is only a host-side stand-in in host code; its device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and used for every kernel argument.  Every call on a device
// shares that device's array: calls that overlap in time on one GPU race, and
// nothing in the array needs clearing between calls (the FP32 kernel writes
// every subcarrier's flag before the FP64 pass reads it, and the FP64 pass
// writes every entry of a slot before reading it).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/dbp.h"
#include "dbp_launch.h"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;   // 16 MiB per device, held until the process ends
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of scratch (looked up on first use).
int scratch_ptr(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return dbp::set_error(DBP_ERR_DEVICE, "dbp_detect_admm_noalloc: no usable current device");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      char msg[256];
      snprintf(msg, sizeof msg, "dbp_detect_admm_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
      return dbp::set_error(DBP_ERR_DEVICE, msg);
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return DBP_OK;
}

}  // namespace

extern "C" {

size_t dbp_noalloc_scratch_bytes(void) { return kScratchBytes; }

int dbp_detect_admm_noalloc(const void* H, const void* y, void* s_hat, uint8_t* hard, int32_t* status, int n_sc,
                            int n_sym, int B, int U, int C, int T, float rho, float gamma, float N0, float Es, int reg,
                            int qam, int prec, void* stream) {
  const char* who = "dbp_detect_admm_noalloc";
  // every argument check first (n_sc = 0 validates and queues nothing)
  const int vrc = dbp::detect_admm_impl(who, H, y, s_hat, hard, status, nullptr, 0, dbp::kFixMaxSlots, 0, n_sym, B, U,
                                        C, T, rho, gamma, N0, Es, reg, qam, prec, stream);
  if (vrc != DBP_OK || n_sc == 0) return vrc;
  void* ws = nullptr;
  if (hard || (prec & 0xF) != DBP_PREC_FP32) {   // the FP64 pass: hard decisions or the mixed modes' factor rule
    // the flags (without a status array) and at least one FP64 slot must fit
    const size_t need = dbp::reslice_bytes_min(n_sc, U, C, status != nullptr);
    if (need > kScratchBytes) {
      char msg[256];
      snprintf(msg, sizeof msg,
               "%s: n_sc=%d, U=%d, C=%d needs %zu bytes of re-slice scratch, more than the %zu-byte static array "
               "(pass a status array, split the call, or use dbp_detect_admm with a workspace)",
               who, n_sc, U, C, need, kScratchBytes);
      return dbp::set_error(DBP_ERR_UNSUPPORTED, msg);
    }
    const int rc = scratch_ptr(&ws);
    if (rc != DBP_OK) return rc;
  }
  return dbp::detect_admm_impl(who, H, y, s_hat, hard, status, ws, ws ? kScratchBytes : 0, dbp::kFixMaxSlots, n_sc,
                               n_sym, B, U, C, T, rho, gamma, N0, Es, reg, qam, prec, stream);
}

}  // extern "C"
