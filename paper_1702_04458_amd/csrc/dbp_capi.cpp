// C ABI entry points: host-side validation, launch planning and dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <atomic>
#include <cstdint>
#include <mutex>

#include "../../include/dbp.h"
#include "dbp_launch.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int ok() {
  g_last_error.clear();
  return DBP_OK;
}

bool supported_u(int U) { return U == 8 || U == 16 || U == 32 || U == 64; }

int qam_side(int qam) {
  switch (qam) {
    case 4: return 2;
    case 16: return 4;
    case 64: return 8;
  }
  return 0;
}

// Waves per workgroup when the clusters of one subcarrier need fewer (1, 2,
// 4 or 8): the workgroup then holds several subcarriers.  The default is a
// build-time knob; dbp_autotune replaces it per (kernel family, U, Cp) by
// the fastest measured value.  Results do not depend on the choice (the
// consensus sums run in fixed cluster order inside one workgroup).
#ifndef DBP_MIN_WAVES
#define DBP_MIN_WAVES 4
#endif

enum PlanKind { kPlanAdmm = 0, kPlanCg = 1, kPlanDl = 2, kPlanKinds = 3 };

int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

std::atomic<int> g_min_waves[kPlanKinds][4][5];   // [kind][log2 U - 3][log2 Cp]

void init_min_waves() {
  static std::once_flag once;
  std::call_once(once, [] {
    for (auto& k : g_min_waves)
      for (auto& u : k)
        for (auto& c : u) c.store(DBP_MIN_WAVES, std::memory_order_relaxed);
  });
}

int min_waves(int kind, int U, int Cp) {
  init_min_waves();
  return g_min_waves[kind][log2i(U) - 3][log2i(Cp)].load(std::memory_order_relaxed);
}

// Launch plan: a lane group of U lanes per (subcarrier, cluster) problem,
// P = 64 / U problems per wave, the Cp >= C (power of two) cluster slots of a
// subcarrier in one workgroup of nw waves holding scpb subcarriers.  The
// plan is made once per call (the kernels' index mapping depends on it).
struct Plan {
  int Cp, nw, scpb;
};

Plan make_plan(int U, int C, int kind, int mw = 0) {
  Plan p;
  const int P = 64 / U;
  p.Cp = 1;
  while (p.Cp < C) p.Cp <<= 1;
  if (mw <= 0) mw = min_waves(kind, U, p.Cp);
  if (p.Cp >= P) {
    const int wps = p.Cp / P;
    p.nw = wps > mw ? wps : mw;
    p.scpb = p.nw / wps;
  } else {
    p.nw = mw;
    p.scpb = mw * (P / p.Cp);
  }
  return p;
}

int common_shape(const char* who, int n_sc, int n_sym, int B, int U, int C, int T) {
  if (n_sc < 0) return fail(DBP_ERR_INVALID, "%s: n_sc must be >= 0", who);
  if (n_sym < 1) return fail(DBP_ERR_INVALID, "%s: n_sym must be >= 1", who);
  if (B < 1 || U < 1 || C < 1) return fail(DBP_ERR_INVALID, "%s: B, U, C must be >= 1", who);
  if (B % C) return fail(DBP_ERR_INVALID, "%s: B=%d is not a multiple of C=%d", who, B, C);
  if (U > B) return fail(DBP_ERR_INVALID, "%s: U=%d exceeds B=%d", who, U, B);
  if (T < 1) return fail(DBP_ERR_INVALID, "%s: T must be >= 1", who);
  if (!supported_u(U)) return fail(DBP_ERR_UNSUPPORTED, "%s: U=%d not built (8, 16, 32, 64)", who, U);
  if (C > 16) return fail(DBP_ERR_UNSUPPORTED, "%s: C=%d > 16 clusters per subcarrier not built", who, C);
  // all cluster groups of one subcarrier share a workgroup of at most 8 waves
  int Cp = 1;
  while (Cp < C) Cp <<= 1;
  if (Cp > 8 * (64 / U))
    return fail(DBP_ERR_UNSUPPORTED, "%s: C=%d clusters of U=%d users exceed one 512-lane workgroup", who, C, U);
  return DBP_OK;
}

int device_status(const char* who, hipError_t e) {
  if (e != hipSuccess) return fail(DBP_ERR_DEVICE, "%s: %s", who, hipGetErrorString(e));
  return ok();
}

}  // namespace

extern "C" {

const char* dbp_version(void) { return "dbp-mi355x 0.1 (gfx950)"; }

const char* dbp_strerror(int status) {
  switch (status) {
    case DBP_OK: return "ok";
    case DBP_ERR_INVALID: return "invalid argument";
    case DBP_ERR_UNSUPPORTED: return "unsupported configuration";
    case DBP_ERR_NOMEM: return "out of memory / budget";
    case DBP_ERR_DEVICE: return "device error";
    case DBP_ERR_BUSY: return "busy";
    case DBP_ERR_NOTFOUND: return "not found";
  }
  return "unknown status";
}

const char* dbp_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {

// Validation and argument block shared by the ADMM uplink entry points
// (everything except the pointers and the precision flags).
int admm_args(const char* who, int n_sc, int n_sym, int B, int U, int C, int T, float rho, float gamma, float N0,
              float Es, int reg, int qam, dbp::UlArgs* a, int* Sout) {
  int st = common_shape(who, n_sc, n_sym, B, U, C, T);
  if (st) return st;
  if (!(rho > 0.f) || !std::isfinite(rho)) return fail(DBP_ERR_INVALID, "%s: rho must be > 0", who);
  if (!(gamma > 0.f) || !std::isfinite(gamma)) return fail(DBP_ERR_INVALID, "%s: gamma must be > 0", who);
  if (!(N0 >= 0.f) || !std::isfinite(N0)) return fail(DBP_ERR_INVALID, "%s: N0 must be >= 0", who);
  if (!(Es > 0.f) || !std::isfinite(Es)) return fail(DBP_ERR_INVALID, "%s: Es must be > 0", who);
  if (reg < DBP_REG_MMSE || reg > DBP_REG_BOX) return fail(DBP_ERR_INVALID, "%s: reg=%d", who, reg);
  const int L = qam_side(qam);
  if (!L) return fail(DBP_ERR_INVALID, "%s: qam=%d not in {4,16,64}", who, qam);
  const int S = B / C;
  *Sout = S;
  const Plan pl = make_plan(U, C, kPlanAdmm);
  *a = dbp::UlArgs{};
  a->nw = pl.nw;
  a->n_sc = n_sc;
  a->n_sym = n_sym;
  a->B = B;
  a->C = C;
  a->Cp = pl.Cp;
  a->S = S;
  a->T = T;
  a->sc_per_block = pl.scpb;
  a->reg = reg;
  a->L = L;
  a->rho = rho;
  a->gamma = gamma;
  const double nu = (reg == DBP_REG_MMSE) ? (double)N0 / ((double)rho * (double)Es) : 0.0;
  a->inv_den = (float)(1.0 / (nu + C));
  a->invC = (float)(1.0 / C);
  a->box_r = (float)((L - 1) / std::sqrt(2.0 * (qam - 1) / 3.0));
  a->kappa = (float)std::sqrt(2.0 * (qam - 1) / 3.0);
  return DBP_OK;
}

// Threshold of the FP64 factor rule on kappa_hat = tr(B_c) ||B_c^{-1}||_F, an
// upper bound of kappa_2(B_c) (at most U^1.5 times it): above 2^14 the FP32
// inverse may lose more than about 1e-3 (relative error of order kappa u,
// u = 2^-24), the low-precision bar.  i.i.d. Rayleigh clusters at S = U = 32
// and rho = 1 give kappa_hat of 1.1e3 .. 2.1e3, so the rule costs nothing
// there; rho = 0.01 flags most clusters.
constexpr float kCondMax = 16384.f;
// kappa_hat of the channels the re-slice guards were measured on (i.i.d.
// Rayleigh, S = U, rho = 1: largest values about 2.0e3 at U = 32 and 9.1e3 at
// U = 64); the guard of a subcarrier grows by its largest kappa_hat over this.
inline float cond_ref(int U) { return U >= 64 ? 8192.f : 2048.f; }

// Precision flags of the ADMM preprocessing -> (gram_prec, inverse kind,
// FP64 factor rule).  one_shot: a detection call, which can recompute flagged
// subcarriers in FP64; otherwise the factorisation alone (dbp_factor_admm),
// which keeps the FP64 inverse at U = 32 for the rule.
int admm_prec(const char* who, int prec, int U, int S, int* gram_prec, int* inv, float* cond = nullptr,
              bool one_shot = false) {
  *gram_prec = prec & 0xF;
  const int factor = prec & ~0xF;
  if (*gram_prec < DBP_PREC_FP32 || *gram_prec > DBP_PREC_MIXED_BF16 ||
      (factor != 0 && factor != DBP_FACTOR_FP32 && factor != DBP_FACTOR_FP64 && factor != DBP_FACTOR_F16X2))
    return fail(DBP_ERR_INVALID, "%s: prec=%d", who, prec);
  if (S < U) return fail(DBP_ERR_UNSUPPORTED, "%s: S=%d < U=%d (S x S branch) not built", who, S, U);
  if (*gram_prec != DBP_PREC_FP32 && U != 32 && U != 64)
    return fail(DBP_ERR_UNSUPPORTED, "%s: mixed precision is built for U=32 and U=64 only", who);
  if (*gram_prec != DBP_PREC_FP32 && U == 64 && factor == DBP_FACTOR_FP64 && !one_shot)
    return fail(DBP_ERR_UNSUPPORTED, "%s: the stored FP64 inverse is built for U=32 only (a 64x64 FP64 row set exceeds a "
                "wave's registers)", who);
  if (*gram_prec == DBP_PREC_FP32 && (factor == DBP_FACTOR_FP64 || factor == DBP_FACTOR_F16X2))
    return fail(DBP_ERR_UNSUPPORTED, "%s: the FP64 and split-FP16 inverses are built for the mixed modes only", who);
  // Default rule: FP64 for poorly conditioned regularised Grams (aspect
  // ratio U/S > 0.8), the FP32 matrix-core inverse otherwise.  A detection
  // call takes the FP32 inverse, estimates each cluster's condition number
  // and recomputes the subcarriers of clusters above kCondMax entirely in
  // FP64 (an explicit FP64 request at U = 64 sends every subcarrier there);
  // the factorisation alone uses the FP64 inverse on the vector units (U = 32).
  *inv = 0;
  if (cond) *cond = 0.f;
  const bool rule = factor == 0 && 5 * U > 4 * S && *gram_prec != DBP_PREC_FP32;
  if (factor == DBP_FACTOR_F16X2) {
    *inv = 2;
  } else if (one_shot && rule) {
    *cond = kCondMax;
  } else if (one_shot && factor == DBP_FACTOR_FP64 && U == 64) {
    *cond = -1.f;
  } else if (factor == DBP_FACTOR_FP64 || (rule && U == 32)) {
    *inv = 1;
  }
  return DBP_OK;
}

hipError_t launch_preprocessing(const dbp::UlArgs& a, int U, int gram_prec, int inv, hipStream_t st, int stage) {
  if (gram_prec == DBP_PREC_FP32) return dbp::launch_admm_ul_f32(a, U, a.nw, st, stage);
  return dbp::launch_admm_ul_mixed(a, U, gram_prec, inv, a.nw, st, stage);
}

// Re-slice guard (slicer units t = (kappa x + L) / 2, thresholds at the
// integers) of a preprocessing mode and user count.  The FP32 soft-value
// error against the FP64 oracle grows with U (the conditioning of the U x U
// regularised Grams): largest measured errors 2.4e-6 (U <= 16), 8.1e-6
// (U = 32) and 1.6e-5 (U = 64), so the guard is 2^-14, 2^-13 and 2^-12
// (at least 7.5x the measured error) for the FP32 Gram and inverse and the
// FP16 split Gram; the BF16 split Gram and the split-FP16 inverse (errors up
// to 4e-3) take 2^-8 and 2^-4.
float reslice_guard(int gram_prec, int inv, int U) {
  if (inv == 2) return 0x1p-4f;
  if (gram_prec == DBP_PREC_MIXED_BF16) return 0x1p-8f;
  return U <= 16 ? 0x1p-14f : (U == 32 ? 0x1p-13f : 0x1p-12f);
}

size_t flags_region(int n_sc) { return ((size_t)n_sc * 4 + 255) & ~size_t(255); }

// The list of subcarriers the split FP64 pass recomputes with one workgroup
// per cluster (one int per workgroup), at the end of the workspace, and 256
// bytes before it the word where the kernels mark that they flagged
// anything.
constexpr size_t kList0Room = dbp::kFixMaxSlots * sizeof(int) + 512;

// A fresh value per call for that mark (never 0).
std::atomic<uint32_t> g_epoch{0};
uint32_t next_epoch() {
  uint32_t e;
  do e = ++g_epoch; while (e == 0);
  return e;
}

// (list0, any) in the last kList0Room bytes of a workspace ending at end.
void bookkeeping(char* ws, size_t ws_bytes, int** list0, uint32_t** any) {
  const uintptr_t end = reinterpret_cast<uintptr_t>(ws) + ws_bytes;
  const uintptr_t l0 = (end - dbp::kFixMaxSlots * sizeof(int)) & ~uintptr_t(255);
  *list0 = reinterpret_cast<int*>(l0);
  *any = reinterpret_cast<uint32_t*>(l0 - 256);
}

// Status and exact re-slicing of a detection call.  Without hard decisions
// only the optional status is written (non-finite bit).  With them the FP32
// kernel flags near-threshold subcarriers into `status` (or, without it, the
// workspace's flag region) and the FP64 pass recomputes them; `slots` is the
// number of FP64 slots of slot_bytes the workspace holds after the flags.
int setup_reslice(const char* who, dbp::UlArgs& a, dbp::FixArgs& f, int32_t* status, void* ws, size_t ws_bytes,
                  float guard, size_t slot_bytes, int max_slots) {
  a.flags = status;
  a.guard = 0.f;
  f = dbp::FixArgs{};
  if (!a.hard && a.cond_max == 0.f) return DBP_OK;
  const size_t fb = status ? 0 : flags_region(a.n_sc);
  if (!ws && !a.hard)
    return fail(DBP_ERR_INVALID, "%s: the FP64 factor rule of the mixed modes (U/S > 0.8) needs a workspace "
                "(dbp_detect_workspace_bytes)", who);
  if (!ws) return fail(DBP_ERR_INVALID, "%s: hard decisions need a workspace (dbp_detect_workspace_bytes)", who);
  if (reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(DBP_ERR_INVALID, "%s: workspace must be 256-byte aligned", who);
  int slots = max_slots;
  const size_t room = ws_bytes > fb + kList0Room ? ws_bytes - fb - kList0Room : 0;
  if (slot_bytes) {
    if ((size_t)slots * slot_bytes > room) slots = (int)(room / slot_bytes);
  } else if (ws_bytes < fb + kList0Room) {
    slots = 0;
  }
  if (slots < 1) return fail(DBP_ERR_INVALID, "%s: workspace of %zu bytes is too small", who, ws_bytes);
  a.flags = status ? status : static_cast<int32_t*>(ws);
  a.guard = a.hard ? guard : 0.f;
  f.flags = a.flags;
  f.ws = static_cast<char*>(ws) + fb;
  // 256-byte aligned, inside the last kList0Room bytes
  bookkeeping(static_cast<char*>(ws), ws_bytes, &f.list0, &a.any);
  a.epoch = next_epoch();
  f.any = a.any;
  f.epoch = a.epoch;
  f.split = 0;
  f.n_slots = slots;
  f.H = a.H;
  f.y = a.y;
  f.shat = a.shat;
  f.hard = a.hard;
  f.n_sc = a.n_sc;
  f.n_sym = a.n_sym;
  f.B = a.B;
  f.C = a.C;
  f.S = a.S;
  f.T = a.T;
  f.reg = a.reg;
  f.L = a.L;
  return DBP_OK;
}

// FP64 parameters of the re-slice pass, from the caller's FP32 arguments.
void fix_params(dbp::FixArgs& f, int U, float rho, float gamma, float N0, float Es, int reg, int qam, bool admm) {
  f.U = U;
  f.gamma = gamma;
  if (admm) {
    f.rho = rho;
    const double nu = (reg == DBP_REG_MMSE) ? (double)N0 / ((double)rho * (double)Es) : 0.0;
    f.inv_den = nu + f.C;   // the denominator itself (the FP64 pass divides)
  } else {
    f.rho = (reg == DBP_REG_MMSE) ? (double)N0 / (double)Es : 0.0;
  }
  f.invC = 1.0 / f.C;
  const double kappa = std::sqrt(2.0 * (qam - 1) / 3.0);
  f.kappa = kappa;
  f.box_r = (f.L - 1) / kappa;
}

// Slots of the ADMM re-slice a workspace of the documented size holds.
int full_slots(int n_sc) { return n_sc < dbp::kFixMaxSlots ? (n_sc > 0 ? n_sc : 1) : dbp::kFixMaxSlots; }

}  // namespace

extern "C" {

size_t dbp_detect_workspace_bytes(int n_sc, int U, int C) {
  if (n_sc < 0 || U < 1 || C < 1) return 0;
  return flags_region(n_sc) + (size_t)full_slots(n_sc) * dbp::fix64_slot_bytes(U, C) + kList0Room;
}

}  // extern "C"

namespace dbp {

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

size_t reslice_bytes_min(int n_sc, int U, int C, bool with_status) {
  return (with_status ? 0 : flags_region(n_sc)) + fix64_slot_bytes(U, C) + kList0Room;
}

// dbp_detect_admm with the re-slice workspace bounded by max_slots FP64 slots
// (the entry point without workspace argument passes its static scratch).
int detect_admm_impl(const char* who, const void* H, const void* y, void* s_hat, uint8_t* hard, int32_t* status,
                     void* workspace, size_t workspace_bytes, int max_slots, int n_sc, int n_sym, int B, int U, int C,
                     int T, float rho, float gamma, float N0, float Es, int reg, int qam, int prec, void* stream) {
  dbp::UlArgs a;
  int S = 0;
  int st = admm_args(who, n_sc, n_sym, B, U, C, T, rho, gamma, N0, Es, reg, qam, &a, &S);
  if (st) return st;
  int gram_prec = 0, inv = 0;
  float cond = 0.f;
  st = admm_prec(who, prec, U, S, &gram_prec, &inv, &cond, true);
  if (st) return st;
  if (n_sc > 0 && (!H || !y || !s_hat)) return fail(DBP_ERR_INVALID, "%s: null H, y or s_hat", who);
  if (n_sc == 0) return ok();
  a.H = static_cast<const dbp::c32*>(H);
  a.y = static_cast<const dbp::c32*>(y);
  a.shat = static_cast<dbp::c32*>(s_hat);
  a.hard = hard;
  a.cond_max = cond;
  a.cond_ref = cond_ref(U);
  dbp::FixArgs f;
  st = setup_reslice(who, a, f, status, workspace, workspace_bytes, reslice_guard(gram_prec, inv, U),
                     dbp::fix64_slot_bytes(U, C), max_slots < full_slots(n_sc) ? max_slots : full_slots(n_sc));
  if (st) return st;
  const hipStream_t hs = static_cast<hipStream_t>(stream);
  st = device_status(who, launch_preprocessing(a, U, gram_prec, inv, hs, 0));
  if (st || (!hard && cond == 0.f)) return st;
  fix_params(f, U, rho, gamma, N0, Es, reg, qam, true);
  f.split = U >= 32;   // large inverses: one workgroup per cluster for each workgroup's first subcarrier
  return device_status(who, dbp::launch_admm_ul_fix64(f, hs));
}

}  // namespace dbp

extern "C" {

int dbp_detect_admm(const void* H, const void* y, void* s_hat, uint8_t* hard, int32_t* status, void* workspace,
                    size_t workspace_bytes, int n_sc, int n_sym, int B, int U, int C, int T, float rho, float gamma,
                    float N0, float Es, int reg, int qam, int prec, void* stream) {
  // the workspace serves the FP64 pass: hard decisions, or the FP64 factor rule of the mixed modes
  if ((hard || (prec & 0xF) != DBP_PREC_FP32) && workspace &&
      workspace_bytes < dbp_detect_workspace_bytes(n_sc, U, C))
    return fail(DBP_ERR_INVALID, "dbp_detect_admm: workspace of %zu bytes, %zu needed", workspace_bytes,
                dbp_detect_workspace_bytes(n_sc, U, C));
  return dbp::detect_admm_impl("dbp_detect_admm", H, y, s_hat, hard, status, workspace, workspace_bytes,
                               dbp::kFixMaxSlots, n_sc, n_sym, B, U, C, T, rho, gamma, N0, Es, reg, qam, prec, stream);
}

size_t dbp_factor_bytes(int n_sc, int U, int C) {
  if (n_sc < 0 || U < 1 || C < 1) return 0;
  return (size_t)n_sc * C * (U * (U + 1) / 2) * 8;   // the Hermitian blocks' upper triangles
}

int dbp_factor_admm(const void* H, void* factors, int n_sc, int B, int U, int C, float rho, int prec, void* stream) {
  const char* who = "dbp_factor_admm";
  dbp::UlArgs a;
  int S = 0;
  int st = admm_args(who, n_sc, 1, B, U, C, 1, rho, 1.0f, 0.0f, 1.0f, DBP_REG_ZF, 4, &a, &S);
  if (st) return st;
  int gram_prec = 0, inv = 0;
  st = admm_prec(who, prec, U, S, &gram_prec, &inv);
  if (st) return st;
  if (n_sc > 0 && (!H || !factors)) return fail(DBP_ERR_INVALID, "%s: null H or factors", who);
  if (n_sc == 0) return ok();
  a.H = static_cast<const dbp::c32*>(H);
  // the preprocessing also forms H_c^H y_c, which is discarded here: H itself
  // serves as a readable stand-in for y (n_sym = 1 keeps every read inside it)
  a.y = a.H;
  a.fac = static_cast<dbp::c32*>(factors);
  return device_status(who, launch_preprocessing(a, U, gram_prec, inv, static_cast<hipStream_t>(stream), 1));
}

int dbp_detect_admm_factored(const void* H, const void* factors, const void* y, void* s_hat, uint8_t* hard,
                             int32_t* status, void* workspace, size_t workspace_bytes, int n_sc, int n_sym, int B,
                             int U, int C, int T, float rho, float gamma, float N0, float Es, int reg, int qam,
                             void* stream) {
  const char* who = "dbp_detect_admm_factored";
  dbp::UlArgs a;
  int S = 0;
  int st = admm_args(who, n_sc, n_sym, B, U, C, T, rho, gamma, N0, Es, reg, qam, &a, &S);
  if (st) return st;
  if (S < U) return fail(DBP_ERR_UNSUPPORTED, "%s: S=%d < U=%d (S x S branch) not built", who, S, U);
  if (n_sc > 0 && (!H || !factors || !y || !s_hat)) return fail(DBP_ERR_INVALID, "%s: null pointer", who);
  if (n_sc == 0) return ok();
  if (hard && workspace && workspace_bytes < dbp_detect_workspace_bytes(n_sc, U, C))
    return fail(DBP_ERR_INVALID, "%s: workspace of %zu bytes, %zu needed", who, workspace_bytes,
                dbp_detect_workspace_bytes(n_sc, U, C));
  a.H = static_cast<const dbp::c32*>(H);
  a.y = static_cast<const dbp::c32*>(y);
  a.shat = static_cast<dbp::c32*>(s_hat);
  a.hard = hard;
  a.fac = const_cast<dbp::c32*>(static_cast<const dbp::c32*>(factors));
  dbp::FixArgs f;
  st = setup_reslice(who, a, f, status, workspace, workspace_bytes, reslice_guard(DBP_PREC_FP32, 0, U),
                     dbp::fix64_slot_bytes(U, C), full_slots(n_sc));
  if (st) return st;
  const hipStream_t hs = static_cast<hipStream_t>(stream);
  st = device_status(who, dbp::launch_admm_ul_factored(a, U, a.nw, hs));
  if (st || !hard) return st;
  fix_params(f, U, rho, gamma, N0, Es, reg, qam, true);
  f.split = U >= 32;
  return device_status(who, dbp::launch_admm_ul_fix64(f, hs));
}

int dbp_flag_nonfinite(const void* x, int n_sc, int per_sc, int32_t* status, void* stream) {
  const char* who = "dbp_flag_nonfinite";
  if (n_sc < 0 || per_sc < 1) return fail(DBP_ERR_INVALID, "%s: n_sc must be >= 0 and per_sc >= 1", who);
  if (n_sc > 0 && (!x || !status)) return fail(DBP_ERR_INVALID, "%s: null x or status", who);
  if (n_sc == 0) return ok();
  return device_status(who, dbp::launch_scan_nonfinite(static_cast<const float*>(x), 2 * (size_t)per_sc, n_sc,
                                                       status, static_cast<hipStream_t>(stream)));
}

size_t dbp_channel_h16_bytes(int n_sc, int B, int U, int C) {
  if (n_sc < 0 || B < 1 || U < 1 || C < 1 || B % C) return 0;
  return (size_t)n_sc * B * U * 4 + (size_t)n_sc * C * 4;
}

int dbp_pack_channel_h16(const void* H, void* packed, int n_sc, int B, int U, int C, void* stream) {
  const char* who = "dbp_pack_channel_h16";
  int st = common_shape(who, n_sc, 1, B, U, C, 1);
  if (st) return st;
  if (n_sc > 0 && (!H || !packed)) return fail(DBP_ERR_INVALID, "%s: null H or packed", who);
  if (n_sc == 0) return ok();
  uint32_t* h16 = static_cast<uint32_t*>(packed);
  float* scale = reinterpret_cast<float*>(h16 + (size_t)n_sc * B * U);
  return device_status(who, dbp::launch_pack_h16(static_cast<const dbp::c32*>(H), h16, scale, n_sc, B, U, C,
                                                 static_cast<hipStream_t>(stream)));
}

int dbp_factor_admm_h16(const void* H, void* factors, void* packed, int n_sc, int B, int U, int C, float rho,
                        int prec, void* stream) {
  const char* who = "dbp_factor_admm_h16";
  dbp::UlArgs a;
  int S = 0;
  int st = admm_args(who, n_sc, 1, B, U, C, 1, rho, 1.0f, 0.0f, 1.0f, DBP_REG_ZF, 4, &a, &S);
  if (st) return st;
  int gram_prec = 0, inv = 0;
  st = admm_prec(who, prec, U, S, &gram_prec, &inv);
  if (st) return st;
  if (n_sc > 0 && (!H || !factors || !packed)) return fail(DBP_ERR_INVALID, "%s: null H, factors or packed", who);
  if (n_sc == 0) return ok();
  if (U != 32 || gram_prec != DBP_PREC_FP32) {
    st = dbp_factor_admm(H, factors, n_sc, B, U, C, rho, prec, stream);
    if (st) return st;
    return dbp_pack_channel_h16(H, packed, n_sc, B, U, C, stream);
  }
  a.H = static_cast<const dbp::c32*>(H);
  a.y = a.H;   // as in dbp_factor_admm: H stands in for the unused y
  a.fac = static_cast<dbp::c32*>(factors);
  a.H16 = static_cast<const uint32_t*>(packed);
  a.hscale = reinterpret_cast<const float*>(a.H16 + (size_t)n_sc * B * U);
  return device_status(who, dbp::launch_factor_pack_u32(a, a.nw, static_cast<hipStream_t>(stream)));
}

int dbp_detect_admm_factored_h16(const void* packed, const void* factors, const void* y, void* s_hat,
                                 uint8_t* hard, int32_t* status, int n_sc, int n_sym, int B, int U, int C, int T,
                                 float rho, float gamma, float N0, float Es, int reg, int qam, void* stream) {
  const char* who = "dbp_detect_admm_factored_h16";
  dbp::UlArgs a;
  int S = 0;
  int st = admm_args(who, n_sc, n_sym, B, U, C, T, rho, gamma, N0, Es, reg, qam, &a, &S);
  if (st) return st;
  if (S < U) return fail(DBP_ERR_UNSUPPORTED, "%s: S=%d < U=%d (S x S branch) not built", who, S, U);
  if (n_sc > 0 && (!packed || !factors || !y || !s_hat)) return fail(DBP_ERR_INVALID, "%s: null pointer", who);
  if (n_sc == 0) return ok();
  a.H16 = static_cast<const uint32_t*>(packed);
  a.hscale = reinterpret_cast<const float*>(a.H16 + (size_t)n_sc * B * U);
  a.y = static_cast<const dbp::c32*>(y);
  a.shat = static_cast<dbp::c32*>(s_hat);
  a.hard = hard;
  a.fac = const_cast<dbp::c32*>(static_cast<const dbp::c32*>(factors));
  a.flags = status;   // non-finite bit only: the low-precision path is not re-sliced
  a.guard = 0.f;
  return device_status(who, dbp::launch_admm_ul_factored_h16(a, U, a.nw, static_cast<hipStream_t>(stream)));
}

int dbp_detect_cg(const void* H, const void* y, void* x_hat, uint8_t* hard, int32_t* status, void* workspace,
                  size_t workspace_bytes, int n_sc, int n_sym, int B, int U, int C, int T, float N0, float Es,
                  int reg, int qam, void* stream) {
  const char* who = "dbp_detect_cg";
  int st = common_shape(who, n_sc, n_sym, B, U, C, T);
  if (st) return st;
  if (!(N0 >= 0.f) || !std::isfinite(N0)) return fail(DBP_ERR_INVALID, "%s: N0 must be >= 0", who);
  if (!(Es > 0.f) || !std::isfinite(Es)) return fail(DBP_ERR_INVALID, "%s: Es must be > 0", who);
  if (reg != DBP_REG_MMSE && reg != DBP_REG_ZF)
    return fail(DBP_ERR_INVALID, "%s: CG needs a quadratic regularizer (MMSE or ZF)", who);
  const int L = qam_side(qam);
  if (!L) return fail(DBP_ERR_INVALID, "%s: qam=%d not in {4,16,64}", who, qam);
  if (n_sc > 0 && (!H || !y || !x_hat)) return fail(DBP_ERR_INVALID, "%s: null H, y or x_hat", who);
  if (n_sc == 0) return ok();
  const Plan pl = make_plan(U, C, kPlanCg);
  dbp::UlArgs a{};
  a.H = static_cast<const dbp::c32*>(H);
  a.y = static_cast<const dbp::c32*>(y);
  a.shat = static_cast<dbp::c32*>(x_hat);
  a.hard = hard;
  a.n_sc = n_sc;
  a.n_sym = n_sym;
  a.B = B;
  a.C = C;
  a.Cp = pl.Cp;
  a.S = B / C;
  a.T = T;
  a.sc_per_block = pl.scpb;
  a.reg = reg;
  a.L = L;
  a.rho = (reg == DBP_REG_MMSE) ? (float)((double)N0 / (double)Es) : 0.f;
  a.gamma = 1.f;
  a.kappa = (float)std::sqrt(2.0 * (qam - 1) / 3.0);
  if (hard && workspace && workspace_bytes < dbp_detect_workspace_bytes(n_sc, U, C))
    return fail(DBP_ERR_INVALID, "%s: workspace of %zu bytes, %zu needed", who, workspace_bytes,
                dbp_detect_workspace_bytes(n_sc, U, C));
  dbp::FixArgs f;
  st = setup_reslice(who, a, f, status, workspace, workspace_bytes, reslice_guard(DBP_PREC_FP32, 0, U), 0,
                     full_slots(n_sc));
  if (st) return st;
  const hipStream_t hs = static_cast<hipStream_t>(stream);
  st = device_status(who, dbp::launch_dcg_ul_f32(a, U, pl.nw, hs));
  if (st || !hard) return st;
  fix_params(f, U, 1.0f, 1.0f, N0, Es, reg, qam, false);
  return device_status(who, dbp::launch_dcg_ul_fix64(f, hs));
}

int dbp_precode_admm(const void* H, int h_layout, const void* s, void* x, float* beta, const float* P_cluster,
                     int power_mode, int n_sc, int n_sym, int B, int U, int C, int T, float rho, float gamma,
                     float eps, void* stream) {
  const char* who = "dbp_precode_admm";
  int st = common_shape(who, n_sc, n_sym, B, U, C, T);
  if (st) return st;
  if (h_layout != DBP_LAYOUT_UPLINK && h_layout != DBP_LAYOUT_DOWNLINK)
    return fail(DBP_ERR_INVALID, "%s: h_layout=%d", who, h_layout);
  if (power_mode != DBP_POWER_COMMON_GAIN && power_mode != DBP_POWER_PER_CLUSTER)
    return fail(DBP_ERR_INVALID, "%s: power_mode=%d", who, power_mode);
  if (!(rho > 0.f) || !std::isfinite(rho)) return fail(DBP_ERR_INVALID, "%s: rho must be > 0", who);
  if (!(gamma > 0.f) || !std::isfinite(gamma)) return fail(DBP_ERR_INVALID, "%s: gamma must be > 0", who);
  if (!(eps >= 0.f) || !std::isfinite(eps)) return fail(DBP_ERR_INVALID, "%s: eps must be >= 0", who);
  if (n_sc > 0 && (!H || !s || !x)) return fail(DBP_ERR_INVALID, "%s: null H, s or x", who);
  const int S = B / C;
  if (S > U) return fail(DBP_ERR_UNSUPPORTED, "%s: S=%d > U=%d (U x U branch) not built", who, S, U);
  if (n_sc == 0) return ok();
  const Plan pl = make_plan(U, C, kPlanDl);
  dbp::DlArgs a{};
  a.H = static_cast<const dbp::c32*>(H);
  a.s = static_cast<const dbp::c32*>(s);
  a.x = static_cast<dbp::c32*>(x);
  a.beta = beta;
  a.P = P_cluster;
  a.n_sc = n_sc;
  a.n_sym = n_sym;
  a.B = B;
  a.C = C;
  a.Cp = pl.Cp;
  a.S = S;
  a.T = T;
  a.sc_per_block = pl.scpb;
  a.rho = rho;
  a.gamma = gamma;
  a.invC = (float)(1.0 / C);
  a.f0 = (float)std::fmax((double)U / B, 1.0 / C);
  a.eps = eps;
  a.budget = (power_mode == DBP_POWER_PER_CLUSTER) ? 1 : 0;
  a.h_layout = h_layout;
  return device_status(who, dbp::launch_admm_dl_f32(a, U, pl.nw, static_cast<hipStream_t>(stream)));
}

int dbp_autotune(int kind, const void* H, const void* in, void* out, int n_sc, int B, int U, int C, int T,
                 int reps, void* stream, int* best_waves) {
  const char* who = "dbp_autotune";
  if (kind < DBP_TUNE_ADMM || kind > DBP_TUNE_PRECODE) return fail(DBP_ERR_INVALID, "%s: kind=%d", who, kind);
  if (reps < 1 || n_sc < 1) return fail(DBP_ERR_INVALID, "%s: reps and n_sc must be >= 1", who);
  if (!H || !in || !out) return fail(DBP_ERR_INVALID, "%s: null H, input or output", who);
  int st = common_shape(who, n_sc, 1, B, U, C, T);
  if (st) return st;
  const hipStream_t hs = static_cast<hipStream_t>(stream);
  auto run = [&]() -> int {
    switch (kind) {
      case DBP_TUNE_ADMM:
        return dbp_detect_admm(H, in, out, nullptr, nullptr, nullptr, 0, n_sc, 1, B, U, C, T, 1.0f, 1.0f, 0.1f, 1.0f,
                               DBP_REG_MMSE, 16, DBP_PREC_FP32, stream);
      case DBP_TUNE_CG:
        return dbp_detect_cg(H, in, out, nullptr, nullptr, nullptr, 0, n_sc, 1, B, U, C, T, 0.1f, 1.0f,
                             DBP_REG_MMSE, 16, stream);
      default:
        return dbp_precode_admm(H, DBP_LAYOUT_UPLINK, in, out, nullptr, nullptr, DBP_POWER_COMMON_GAIN, n_sc, 1, B,
                                U, C, T, 1.0f, 1.0f, 0.0f, stream);
    }
  };
  const int pk = kind == DBP_TUNE_ADMM ? kPlanAdmm : (kind == DBP_TUNE_CG ? kPlanCg : kPlanDl);
  int Cp = 1;
  while (Cp < C) Cp <<= 1;
  init_min_waves();
  std::atomic<int>& slot = g_min_waves[pk][log2i(U) - 3][log2i(Cp)];
  const int before = slot.load();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(DBP_ERR_DEVICE, "%s: hipEventCreate failed", who);
  }
  float best_ms = 0.f;
  int best = before, last_nw = -1;
  for (int mw : {1, 2, 4, 8}) {
    // candidates that give the same workgroup as one already timed are skipped
    const int nw = make_plan(U, C, pk, mw).nw;
    if (nw == last_nw) continue;
    last_nw = nw;
    slot.store(mw);
    st = run();                                        // warm-up
    if (st) break;
    if (hipEventRecord(e0, hs) != hipSuccess) { st = fail(DBP_ERR_DEVICE, "%s: hipEventRecord", who); break; }
    for (int r = 0; r < reps && !st; ++r) st = run();
    if (st) break;
    float ms = 0.f;
    if (hipEventRecord(e1, hs) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(DBP_ERR_DEVICE, "%s: event timing failed", who);
      break;
    }
    if (best_ms == 0.f || ms < best_ms) {
      best_ms = ms;
      best = mw;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  slot.store(st ? before : best);
  if (st) return st;
  if (best_waves) *best_waves = best;
  return ok();
}

int dbp_autotune_get(int kind, int U, int C) {
  if (kind < DBP_TUNE_ADMM || kind > DBP_TUNE_PRECODE || !supported_u(U) || C < 1 || C > 16) return -1;
  int Cp = 1;
  while (Cp < C) Cp <<= 1;
  const int pk = kind == DBP_TUNE_ADMM ? kPlanAdmm : (kind == DBP_TUNE_CG ? kPlanCg : kPlanDl);
  return min_waves(pk, U, Cp);
}

int dbp_detect_admm_batch(const dbp_frame* frames, int n_frames, int U, void* stream) {
  const char* who = "dbp_detect_admm_batch";
  if (n_frames < 0 || n_frames > DBP_MAX_BATCH)
    return fail(DBP_ERR_INVALID, "%s: n_frames=%d outside 0..%d", who, n_frames, DBP_MAX_BATCH);
  if (n_frames > 0 && !frames) return fail(DBP_ERR_INVALID, "%s: null frames", who);
  if (!supported_u(U)) return fail(DBP_ERR_UNSUPPORTED, "%s: U=%d not built (8, 16, 32, 64)", who, U);
  // validation of every frame, and the common waves per workgroup
  int nw = 1, C_max = 1;
  for (int i = 0; i < n_frames; ++i) {
    const dbp_frame& fr = frames[i];
    dbp::UlArgs a;
    int S = 0;
    int st = admm_args(who, fr.n_sc, fr.n_sym, fr.B, U, fr.C, fr.T, fr.rho, fr.gamma, fr.N0, fr.Es, fr.reg, fr.qam,
                       &a, &S);
    if (st) return st;
    if (S < U) return fail(DBP_ERR_UNSUPPORTED, "%s: frame %d: S=%d < U=%d (S x S branch) not built", who, i, S, U);
    if (fr.n_sc > 0 && (!fr.H || !fr.y || !fr.s_hat)) return fail(DBP_ERR_INVALID, "%s: frame %d: null pointer", who, i);
    if (fr.hard && fr.n_sc > 0) {
      if (!fr.workspace || fr.workspace_bytes < dbp_detect_workspace_bytes(fr.n_sc, U, fr.C) ||
          reinterpret_cast<uintptr_t>(fr.workspace) % 256)
        return fail(DBP_ERR_INVALID, "%s: frame %d: hard decisions need a 256-byte aligned workspace of "
                    "dbp_detect_workspace_bytes bytes", who, i);
    }
    nw = a.nw > nw ? a.nw : nw;
    C_max = fr.C > C_max ? fr.C : C_max;
  }
  dbp::UlBatch b{};
  dbp::FixBatch fb{};
  // FP64 slots: in the workspace (after its flags) with the most room
  const size_t slot = dbp::fix64_slot_bytes(U, C_max);
  char* slots = nullptr;
  size_t slot_room = 0;
  for (int i = 0; i < n_frames; ++i) {
    const dbp_frame& fr = frames[i];
    if (!fr.hard || fr.n_sc == 0) continue;
    const size_t fl = (fr.status ? 0 : flags_region(fr.n_sc)) + kList0Room;
    if (fr.workspace_bytes - fl > slot_room) {
      slot_room = fr.workspace_bytes - fl;
      slots = static_cast<char*>(fr.workspace) + fl - kList0Room;
    }
  }
  int n_slots = (int)(slot_room / slot);
  if (n_slots > dbp::kFixMaxSlots) n_slots = dbp::kFixMaxSlots;
  int total = 0;
  for (int i = 0; i < n_frames; ++i) {
    const dbp_frame& fr = frames[i];
    dbp::UlArgs& a = b.f[b.n];
    int S = 0;
    (void)admm_args(who, fr.n_sc, fr.n_sym, fr.B, U, fr.C, fr.T, fr.rho, fr.gamma, fr.N0, fr.Es, fr.reg, fr.qam, &a,
                    &S);
    if (fr.n_sc == 0) continue;
    // the frame's plan at the batch's waves per workgroup
    const Plan pl = make_plan(U, fr.C, kPlanAdmm, nw);
    a.nw = pl.nw;
    a.Cp = pl.Cp;
    a.sc_per_block = pl.scpb;
    a.H = static_cast<const dbp::c32*>(fr.H);
    a.y = static_cast<const dbp::c32*>(fr.y);
    a.shat = static_cast<dbp::c32*>(fr.s_hat);
    a.hard = fr.hard;
    a.flags = fr.status;
    a.guard = 0.f;
    if (fr.hard) {
      dbp::FixArgs& f = fb.f[fb.n++];
      int32_t* flags = fr.status ? fr.status : static_cast<int32_t*>(fr.workspace);
      a.flags = flags;
      a.guard = reslice_guard(DBP_PREC_FP32, 0, U);
      f = dbp::FixArgs{};
      int* unused_list0 = nullptr;
      bookkeeping(static_cast<char*>(fr.workspace), fr.workspace_bytes, &unused_list0, &a.any);
      a.epoch = next_epoch();
      f.any = a.any;
      f.epoch = a.epoch;
      f.flags = flags;
      f.ws = slots;
      f.n_slots = n_slots;
      f.H = a.H;
      f.y = a.y;
      f.shat = a.shat;
      f.hard = a.hard;
      f.n_sc = a.n_sc;
      f.n_sym = a.n_sym;
      f.B = a.B;
      f.C = a.C;
      f.S = a.S;
      f.T = a.T;
      f.reg = a.reg;
      f.L = a.L;
      fix_params(f, U, fr.rho, fr.gamma, fr.N0, fr.Es, fr.reg, fr.qam, true);
    }
    b.first[b.n] = total;
    total += (fr.n_sc + pl.scpb - 1) / pl.scpb;
    ++b.n;
  }
  b.first[b.n] = total;
  if (total == 0) return ok();
  const hipStream_t hs = static_cast<hipStream_t>(stream);
  // persistent grid: enough workgroups to fill the chip at four waves per SIMD
  const int cap = 256 * (16 / nw > 0 ? 16 / nw : 1);
  int st = device_status(who, dbp::launch_admm_ul_f32_batch(b, U, nw, total < cap ? total : cap, hs));
  if (st || fb.n == 0) return st;
  return device_status(who, dbp::launch_admm_ul_fix64_batch(fb, U, n_slots, hs));
}

}  // extern "C"
