/* dbp.h -- C ABI of the MI355X decentralized baseband processing library.
 *
 * Method: K. Li, R. Sharan, Y. Chen, T. Goldstein, J. R. Cavallaro, C. Studer,
 * "Decentralized Baseband Processing for Massive MU-MIMO Systems",
 * arXiv:1702.04458.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Complex data is interleaved single precision (re, im) -- "complex64".
 * - H is the UPLINK channel in layout [n_sc][B][U] (row b = antenna b,
 *   column u = user u), row-major.  Cluster c owns rows c*S .. c*S+S-1 with
 *   S = B / C (the row partition of Section II-A2).  The downlink channel is
 *   taken in place as H^d = H^T (channel reciprocity, Section II-B1).
 * - All array arguments are DEVICE pointers owned by the caller; the library
 *   never frees, retains or reallocates them, and never writes outside the
 *   documented output arrays.
 * - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *   stream-ordered and asynchronous: they return after enqueueing the work,
 *   without a host synchronisation.
 * - Argument errors are detected on the host BEFORE any device work is queued
 *   and return DBP_ERR_INVALID or DBP_ERR_UNSUPPORTED; nothing is written then.
 *   A launch failure returns DBP_ERR_DEVICE.  dbp_last_error() gives a
 *   human-readable reason for the last failure on the calling thread.
 * - Results are deterministic: for fixed inputs and parameters every output
 *   bit is independent of the launch shape and of other work on the device.
 */
#ifndef DBP_H_
#define DBP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DBP_OK 0
#define DBP_ERR_INVALID 1      /* malformed arguments                            */
#define DBP_ERR_UNSUPPORTED 2  /* valid for the method, not built for the GPU     */
#define DBP_ERR_NOMEM 3        /* device memory or serving budget exhausted       */
#define DBP_ERR_DEVICE 4       /* HIP runtime or launch failure                   */
#define DBP_ERR_BUSY 5         /* resource still in use (resident channel)        */
#define DBP_ERR_NOTFOUND 6     /* unknown serving ticket or channel handle        */

/* Regularizer g(s) of the equalization problem (E0), Section III-A. */
#define DBP_REG_MMSE 0   /* g = N0/(2 Es) ||s||^2, proximal step (E2-MMSE)     */
#define DBP_REG_ZF 1     /* g = 0, proximal step (E2-ZF)                      */
#define DBP_REG_BOX 2    /* indicator of the QAM bounding box, (E2-BOX)        */

/* Arithmetic of the preprocessing (Gram matrix and its regularised inverse). */
#define DBP_PREC_FP32 0        /* everything in FP32                                     */
#define DBP_PREC_MIXED_FP16 1  /* Gram on FP16 MFMA (FP32 accumulate) + FP32 refinement */
#define DBP_PREC_MIXED_BF16 2  /* Gram on BF16 MFMA (FP32 accumulate) + FP32 refinement */
/* Precision of the regularised inverse in the mixed modes, OR-ed into prec:
 *   DBP_FACTOR_FP32   Gauss-Jordan on the FP32 matrix cores;
 *   DBP_FACTOR_FP64   Gauss-Jordan in FP64 on the vector units at U = 32; at
 *                     U = 64 the detection calls recompute every subcarrier
 *                     in FP64 (the FP64 pass below: Gram, inverse and
 *                     iterations) and dbp_factor_admm returns
 *                     DBP_ERR_UNSUPPORTED;
 *   DBP_FACTOR_F16X2  Gauss-Jordan on the FP16 matrix cores with every
 *                     operand split into an FP16 hi + lo pair (about 22
 *                     significant bits) and FP32 accumulation; the FP16
 *                     matrix cores run beside the vector units, but their
 *                     accumulation is not correctly rounded under
 *                     cancellation, so the inverse is about 30x less
 *                     accurate than DBP_FACTOR_FP32 (frame error ~5e-5).
 * By default (no flag) the inverse is FP32, and FP64 serves the poorly
 * conditioned regularised Grams, which occur at aspect ratios U/S > 0.8:
 * there dbp_detect_admm inverts on the FP32 matrix cores, bounds each
 * cluster's condition number by kappa_hat = tr(B_c) ||B_c^{-1}||_F (at
 * least kappa_2(B_c), at most U^1.5 times it) and recomputes the subcarriers
 * with a cluster above 2^14 entirely in FP64 (status DBP_STATUS_ILLCOND; this
 * needs the workspace even without hard decisions), U = 32 and 64;
 * dbp_factor_admm takes the FP64 inverse at U = 32 instead.  The FP32 mode
 * (DBP_PREC_FP32) always inverts on the FP32 matrix cores and accepts no
 * other factor flag. */
#define DBP_FACTOR_FP32 0x10
#define DBP_FACTOR_FP64 0x20
#define DBP_FACTOR_F16X2 0x30

/* Per-subcarrier status bits (status arrays of the detection calls and of
 * dbp_flag_nonfinite). */
#define DBP_STATUS_NONFINITE 1   /* a real or imaginary part of an output is NaN or infinite      */
#define DBP_STATUS_RESLICED 2    /* recomputed in FP64 (exact hard decisions, see below, or bit 4) */
#define DBP_STATUS_ILLCOND 4     /* a cluster's regularised Gram exceeded the FP64 factor rule's
                                    bound (mixed modes, U/S > 0.8): recomputed in FP64            */

/* Exact hard decisions.  Slicing (Section III-A) takes the nearest point of
 * the constellation; an FP32 soft value that lies within rounding distance of
 * a decision threshold could be sliced differently from an exact evaluation.
 * Every detection call that returns hard decisions (hard != NULL) therefore
 * flags each subcarrier that has a soft value within a guard of a threshold
 * -- in the slicer's units t = (kappa x + L) / 2 (thresholds at the
 * integers 1 .. L-1), 2^-14 for U <= 16, 2^-13 for U = 32 and 2^-12 for
 * U = 64, at least 7.5x the largest FP32 error measured against an FP64
 * evaluation at each U; 2^-8 with the BF16 split Gram and 2^-4 with the split-FP16
 * inverse -- and recomputes the flagged subcarriers entirely in FP64 on the
 * GPU (Gram, regularised inverse or CG, every iteration), overwriting their
 * soft outputs (FP64 result rounded to FP32) and their hard decisions (taken
 * in FP64).  Such subcarriers carry DBP_STATUS_RESLICED.  The FP64 pass keeps
 * its state in a caller-provided device workspace:
 *
 * dbp_detect_workspace_bytes(n_sc, U, C): bytes of workspace a call with hard
 *   decisions needs (0 for malformed sizes): a flag per subcarrier, up to
 *   256 blocks of C U^2 complex FP64 and 1536 bytes of bookkeeping.  The workspace must be 256-byte aligned;
 *   its contents need no initialisation and are garbage afterwards.  Calls
 *   that share one workspace must not overlap in time.
 */
size_t dbp_detect_workspace_bytes(int n_sc, int U, int C);

const char* dbp_version(void);
const char* dbp_strerror(int status);
/* Reason for the most recent failed call on this thread ("" if none). */
const char* dbp_last_error(void);

/* Decentralized ADMM-based data detection: Algorithm 1 (Section III-C) with
 * the U x U closed form of step (E1) (eq. StepE1variant1), the consensus of
 * Lemma 1 and the proximal steps (E2-MMSE / E2-ZF / E2-BOX).
 *
 *   H      [n_sc][B][U] complex64   uplink channel (shared by all n_sym symbols)
 *   y      [n_sc][n_sym][B] complex64  receive vectors
 *   s_hat  [n_sc][n_sym][U] complex64  output: s^(T) of Algorithm 1
 *   hard   [n_sc][n_sym][U] uint8 or NULL  output: nearest unit-energy square
 *          QAM point per entry, as index iI + L*iQ (L = sqrt(qam); level i of a
 *          dimension is (2i - (L-1)) / sqrt(2 (qam-1) / 3); ties go up), exact
 *          by the FP64 re-slice above
 *   status [n_sc] int32 or NULL  output: DBP_STATUS_* bits of every subcarrier
 *   workspace, workspace_bytes  device workspace of at least
 *          dbp_detect_workspace_bytes(n_sc, U, C) bytes when hard != NULL
 *          or when the FP64 factor rule applies (mixed modes without a
 *          factor flag at U/S > 0.8, or DBP_FACTOR_FP64 at U = 64); may be
 *          NULL otherwise; DBP_ERR_INVALID if missing, smaller or not
 *          256-byte aligned
 *   T      number of estimates s^(1..T) (T - 1 ADMM iterations after the
 *          initial consensus), T >= 1
 *   rho    ADMM penalty > 0;  gamma  dual step > 0 (the paper uses 1)
 *   N0     noise variance >= 0 (MMSE);  Es  symbol energy > 0
 *   reg    DBP_REG_*;  qam  4, 16 or 64 (slicer and BOX radius)
 *   prec   DBP_PREC_*, optionally OR DBP_FACTOR_*.  In the mixed modes each
 *          cluster's H_c is scaled by a power of two, split as H_hi + H_lo in
 *          the half format, and the Gram accumulates H_hi^H H_hi + H_hi^H H_lo
 *          + H_lo^H H_hi in FP32 on the matrix cores (mixed modes: U = 32 and
 *          U = 64; other U return DBP_ERR_UNSUPPORTED).
 * Requires B % C == 0, S = B / C >= U (the U x U branch, S > U in the paper;
 * at S = U the S x S and U x U branches coincide), U in {8, 16, 32, 64},
 * C <= 16, n_sc >= 0 (0 validates every other argument and queues no work),
 * n_sym >= 1.
 */
int dbp_detect_admm(const void* H, const void* y, void* s_hat, uint8_t* hard,
                    int32_t* status, void* workspace, size_t workspace_bytes,
                    int n_sc, int n_sym, int B, int U, int C, int T,
                    float rho, float gamma, float N0, float Es,
                    int reg, int qam, int prec, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * dbp_detect_admm without the workspace arguments.  The FP64 re-slice takes
 * its workspace from a static device array of dbp_noalloc_scratch_bytes()
 * bytes (16 MiB) that each GPU the library runs on holds until the process
 * ends; the call allocates nothing.  Every call on one GPU shares that GPU's
 * array, so calls that overlap in time on one GPU race; nothing in it needs
 * clearing between calls.  Returns DBP_ERR_UNSUPPORTED when hard decisions
 * are requested and the flags of n_sc subcarriers (4 n_sc bytes, none when
 * `status` is given) plus one FP64 block of C U^2 complex values (16 C U^2
 * bytes) and 1536 bytes of bookkeeping exceed the array.  Arguments, outputs and errors otherwise as
 * dbp_detect_admm; the results are bit-identical to it. */
size_t dbp_noalloc_scratch_bytes(void);
int dbp_detect_admm_noalloc(const void* H, const void* y, void* s_hat, uint8_t* hard,
                            int32_t* status, int n_sc, int n_sym, int B, int U, int C, int T,
                            float rho, float gamma, float N0, float Es,
                            int reg, int qam, int prec, void* stream);

/* Resident factorisation for a static channel.  Algorithm 1's preprocessing
 * (Section III-B, the U x U form of step E1: B_c = H_c^H H_c + rho I_U and its
 * inverse) depends on H and rho only; the paper precomputes B_c^{-1} once per
 * channel.  dbp_factor_admm runs that preprocessing for every (subcarrier,
 * cluster) and writes B_c^{-1} to `factors` (device, caller-owned,
 * dbp_factor_bytes(n_sc, U, C) bytes, an internal layout of n_sc * C blocks
 * of U (U + 1) / 2 complex64: each block's upper triangle, B_c^{-1} being
 * Hermitian).  dbp_detect_admm_factored then runs Algorithm 1's
 * iterations for any received frame y against that channel: it reads H (for
 * H_c^H y_c) and the factors, and forms no Gram and no inverse.
 *   prec (factor only)  as for dbp_detect_admm: the Gram and inverse
 *          precision of the stored B_c^{-1};
 *   rho    must be the value the factors were made with (not checked).
 * Other arguments (hard decisions, status and workspace included),
 * requirements and errors are those of dbp_detect_admm; the FP64 re-slice
 * recomputes flagged subcarriers from H (the FP32 guards, for FP32 factors).
 * The result equals dbp_detect_admm up to the rounding of H_c^H y_c, which
 * the factored path forms on the vector units. */
size_t dbp_factor_bytes(int n_sc, int U, int C);
int dbp_factor_admm(const void* H, void* factors, int n_sc, int B, int U, int C,
                    float rho, int prec, void* stream);
int dbp_detect_admm_factored(const void* H, const void* factors, const void* y,
                             void* s_hat, uint8_t* hard, int32_t* status,
                             void* workspace, size_t workspace_bytes,
                             int n_sc, int n_sym, int B, int U, int C, int T,
                             float rho, float gamma, float N0, float Es,
                             int reg, int qam, void* stream);

/* Per-subcarrier status of any result.  Non-finite outputs (NaN or infinite
 * parts, e.g. from inputs whose Gram overflows FP32, or a ZF system that is
 * singular) are not errors of the calls above; the detection calls report
 * them in their status output, and this call reports them for any output
 * array (e.g. the precoder's x).
 *   x       [n_sc][per_sc] complex64, device: any output of the library
 *           (s_hat or x_hat with per_sc = n_sym * U, precoder x with
 *           per_sc = n_sym * B)
 *   status  [n_sc] int32, device, caller-allocated: every entry is written,
 *           DBP_STATUS_NONFINITE if a real or imaginary part of subcarrier k
 *           is NaN or infinite, else 0.
 * Stream-ordered like the other calls; DBP_ERR_INVALID for n_sc < 0,
 * per_sc < 1 or null pointers with n_sc > 0. */
int dbp_flag_nonfinite(const void* x, int n_sc, int per_sc, int32_t* status, void* stream);

/* Mixed-precision resident channel (served form of Algorithm 1 for a static
 * channel): H is kept in HBM as complex FP16 with one power-of-two scale per
 * (subcarrier, cluster) tile, the factors B_c^{-1} stay FP32, and the
 * iterations run in FP32.  Per subcarrier the iterations then read
 * 4 B U + 4 C U (U + 1) bytes instead of 8 B U + 4 C U (U + 1).
 *
 * dbp_channel_h16_bytes(n_sc, B, U, C) = 4 n_sc B U + 4 n_sc C: the size of a
 *   packed channel (0 for malformed sizes).
 * dbp_pack_channel_h16(H, packed, ...): H [n_sc][B][U] complex64 (device) ->
 *   packed (device, caller-allocated, dbp_channel_h16_bytes): first
 *   [n_sc][B][U] pairs of IEEE binary16 (real part in the low 16 bits of each
 *   32-bit word) holding H * 2^-e rounded to nearest even, then [n_sc][C]
 *   floats 2^e.  e = floor(log2 m) - 14 for the largest |real or imaginary
 *   part| m of the S x U tile of cluster c on subcarrier k (e >= -126; e = 0
 *   for an all-zero tile), so entries keep 11 significant bits.
 * dbp_factor_admm_h16(H, factors, packed, ...): dbp_factor_admm and
 *   dbp_pack_channel_h16 of the same H in one call, with the same outputs bit
 *   for bit.  At U = 32 with the FP32 preprocessing (prec DBP_PREC_FP32 or
 *   0) both come from one launch that reads H for the Gram and once more to
 *   convert it (the tile maxima are taken during the Gram's pass); otherwise
 *   the two calls run in turn on `stream`.  Arguments and errors as the two
 *   calls.
 * dbp_detect_admm_factored_h16(packed, factors, y, ...): as
 *   dbp_detect_admm_factored, with H_c^H y_c formed from the packed channel
 *   (entries widened to FP32, FP32 accumulation).  The rounding of H to 11
 *   significant bits makes this a low-precision path: frame-level relative
 *   error within 1e-3 of the exact result (about 2e-4 at B = 256, U = 32, C = 8,
 *   25 dB, T = 5).  Being a low-precision path it is not re-sliced: its hard
 *   decisions are those of its own soft output, and `status` (may be NULL)
 *   carries the non-finite bit only.
 * Arguments, requirements and errors otherwise as dbp_detect_admm_factored. */
size_t dbp_channel_h16_bytes(int n_sc, int B, int U, int C);
int dbp_pack_channel_h16(const void* H, void* packed, int n_sc, int B, int U, int C, void* stream);
int dbp_factor_admm_h16(const void* H, void* factors, void* packed, int n_sc, int B, int U, int C,
                        float rho, int prec, void* stream);
int dbp_detect_admm_factored_h16(const void* packed, const void* factors, const void* y,
                                 void* s_hat, uint8_t* hard, int32_t* status,
                                 int n_sc, int n_sym, int B, int U, int C, int T,
                                 float rho, float gamma, float N0, float Es,
                                 int reg, int qam, void* stream);

/* Decentralized conjugate-gradient data detection: Algorithm 2 (Section
 * III-D) with the broadcast-w variant (every cluster keeps its own x, r, p).
 * The CG regulariser is N0/Es for DBP_REG_MMSE and 0 for DBP_REG_ZF; T >= 1
 * CG iterations.  x_hat [n_sc][n_sym][U] complex64; hard, status and
 * workspace as for dbp_detect_admm (the FP64 re-slice runs Algorithm 2 again).
 * Requires B % C == 0, U in {8, 16, 32, 64}, C <= 16.
 */
int dbp_detect_cg(const void* H, const void* y, void* x_hat, uint8_t* hard,
                  int32_t* status, void* workspace, size_t workspace_bytes,
                  int n_sc, int n_sym, int B, int U, int C, int T,
                  float N0, float Es, int reg, int qam, void* stream);

/* Decentralized ADMM-based beamforming: Algorithm 3 (Section IV-C), S x S
 * branch (A_c = H_c^H H_c + rho^-1 I_S with the downlink cluster channel
 * H_c, U x S: columns cS .. cS+S-1 of the downlink channel H^d).
 *
 *   H, h_layout  the channel, device: DBP_LAYOUT_UPLINK: the uplink channel
 *          [n_sc][B][U] (complex64), taken in place as H^d = H^T (channel
 *          reciprocity, Section II-B1); DBP_LAYOUT_DOWNLINK: the downlink
 *          channel H^d itself, [n_sc][U][B] row-major.  DBP_ERR_INVALID for
 *          any other value.
 *   s      [n_sc][n_sym][U] complex64  precoding targets
 *   x      [n_sc][n_sym][B] complex64  output [x_1; ...; x_C]
 *   beta   [n_sc][n_sym] float or NULL  output common gain (1 without budgets)
 *   P_cluster  [C] float DEVICE array of per-cluster transmit-energy budgets
 *          P_c > 0, or NULL (no budgets).  The paper's problem P0 has no such
 *          budgets; power_mode selects how they are met:
 *   power_mode DBP_POWER_COMMON_GAIN: after Algorithm 3, x is scaled by
 *          beta = min(1, min_c sqrt(P_c / ||x_c||^2)) so that every cluster
 *          meets its budget while H^d x = beta * H^d x_unscaled stays
 *          interference-free;
 *          DBP_POWER_PER_CLUSTER: every x-update is step (P1) of Section
 *          IV-B solved exactly under ||x_c||^2 <= P_c (problem P0 with the
 *          budgets added as constraints; the unconstrained step when it fits
 *          the budget, else the minimiser on the budget sphere through the
 *          Lagrange multiplier, found by Newton's method on the shifted
 *          regularised Gram), and beta = 1.  Ignored without P_cluster.
 *   T      number of x-updates (T - 1 consensus steps), T >= 1
 *   eps    radius of the precoding constraint ||s - H^d x|| <= eps of
 *          problem P0 (Section IV-A), eps >= 0.  eps = 0 is Algorithm 3 as
 *          printed (z_c = w_c + (s - w)/C); eps > 0 uses the z-update of
 *          Lemma 2, z_c = w_c + max{0, 1 - eps/||s - w||} (s - w)/C with
 *          w = sum_c w_c (the norm of the lemma's proof).
 * Requires B % C == 0, S = B / C <= U, U in {8, 16, 32, 64}, C <= 16.
 */
#define DBP_POWER_COMMON_GAIN 0
#define DBP_POWER_PER_CLUSTER 1
#define DBP_LAYOUT_UPLINK 0
#define DBP_LAYOUT_DOWNLINK 1
int dbp_precode_admm(const void* H, int h_layout, const void* s, void* x, float* beta,
                     const float* P_cluster, int power_mode, int n_sc, int n_sym, int B, int U,
                     int C, int T, float rho, float gamma, float eps, void* stream);

/* Uneven batches in one launch: up to DBP_MAX_BATCH frames of ADMM
 * detection (Algorithm 1, FP32) that share U but may differ in every other
 * shape and parameter (n_sc, n_sym, B, C, T, regulariser, QAM, rho, N0) run
 * in one persistent kernel over all their subcarriers, followed by one FP64
 * re-slice pass over the frames with hard decisions.  Each dbp_frame holds
 * what dbp_detect_admm takes for one frame (device pointers, caller-owned;
 * workspace as there, needed with hard decisions).  Results are
 * bit-identical to dbp_detect_admm on each frame alone.  Frames are
 * validated first (DBP_ERR_INVALID / DBP_ERR_UNSUPPORTED name the frame);
 * n_frames = 0 is a no-op; prec is FP32 only. */
#define DBP_MAX_BATCH 24
typedef struct dbp_frame {
  const void* H;          /* [n_sc][B][U] complex64 */
  const void* y;          /* [n_sc][n_sym][B] complex64 */
  void* s_hat;            /* [n_sc][n_sym][U] complex64 */
  uint8_t* hard;          /* [n_sc][n_sym][U] or NULL */
  int32_t* status;        /* [n_sc] or NULL */
  void* workspace;        /* dbp_detect_workspace_bytes(n_sc, U, C) bytes with hard decisions */
  size_t workspace_bytes;
  int n_sc, n_sym, B, C, T, reg, qam;
  float rho, gamma, N0, Es;
} dbp_frame;
int dbp_detect_admm_batch(const dbp_frame* frames, int n_frames, int U, void* stream);

/* Launch-plan autotuner.  All clusters of a subcarrier share one workgroup;
 * when they need fewer waves than the plan's minimum, a workgroup holds
 * several subcarriers.  dbp_autotune times the candidate minimums 1, 2, 4
 * and 8 waves (those giving distinct workgroups) on the caller's data, reps
 * launches each, and keeps the fastest for every later call of that kernel
 * family with the same U and padded cluster count (process-wide, all
 * devices).  It synchronises the stream: a set-up call, not for the hot
 * path.  Results of the detection and precoding calls do not depend on the
 * plan.
 *   kind  DBP_TUNE_ADMM (dbp_detect_admm and its factored forms),
 *         DBP_TUNE_CG (dbp_detect_cg), DBP_TUNE_PRECODE (dbp_precode_admm)
 *   H     [n_sc][B][U] device; in: y [n_sc][1][B] (ADMM, CG) or the targets
 *         s [n_sc][1][U] (precode); out: s_hat [n_sc][1][U] or x [n_sc][1][B]
 *         (overwritten with results of the tuned kernel: MMSE with N0 = 0.1,
 *         rho = 1, no budgets)
 *   best_waves  output (may be NULL): the chosen minimum
 * dbp_autotune_get returns the minimum in use for (kind, U, C), -1 for
 * malformed arguments. */
#define DBP_TUNE_ADMM 0
#define DBP_TUNE_CG 1
#define DBP_TUNE_PRECODE 2
int dbp_autotune(int kind, const void* H, const void* in, void* out, int n_sc, int B, int U, int C, int T,
                 int reps, void* stream, int* best_waves);
int dbp_autotune_get(int kind, int U, int C);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of uplink detection frames (Algorithm 1).
 *
 * A server owns a device arena of hbm_budget_bytes and n_slots streams.
 * dbp_server_submit queues a frame (arrival time = the call); a scheduler
 * thread admits queued frames in arrival order as soon as a slot is free and
 * the frame's device footprint (H, y, outputs) fits in the arena, then runs
 * host-to-device copies, dbp_detect_admm and device-to-host copies on the
 * slot's stream.  Admitted frames overlap on the device; a finished frame
 * returns its slot and arena space, so waiting frames are admitted as
 * resources free up.  Results are bit-identical to a lone dbp_detect_admm
 * call on the same inputs.
 *
 * H_host [n_sc][B][U], y_host [n_sc][n_sym][B], s_hat_host [n_sc][n_sym][U]
 * (complex64) and hard_host [n_sc][n_sym][U] (uint8, or NULL) are caller-owned
 * PINNED host buffers that must stay valid until dbp_server_wait returns for
 * the ticket.  With flags = DBP_SERVE_DEVICE_IO they are instead caller-owned
 * DEVICE buffers (frames already resident in HBM): no copies are made and the
 * arena space the frame reserves only bounds the in-flight working set.  Submit returns DBP_ERR_INVALID for malformed shapes and
 * DBP_ERR_NOMEM for a frame larger than the whole budget; other errors (e.g.
 * an unsupported shape) are reported by dbp_server_wait.
 * ------------------------------------------------------------------------ */
typedef struct dbp_server dbp_server;
#define DBP_SERVE_DEVICE_IO 1
#define DBP_CHANNEL_H16 2      /* dbp_channel_load: keep H as the packed FP16 channel */

int dbp_server_create(int device, size_t hbm_budget_bytes, int n_slots, dbp_server** out);
/* Waits for in-flight work, then frees the arena and streams. */
int dbp_server_destroy(dbp_server* srv);
int dbp_server_submit(dbp_server* srv, const void* H_host, const void* y_host, void* s_hat_host,
                      uint8_t* hard_host, int n_sc, int n_sym, int B, int U, int C, int T,
                      float rho, float N0, int reg, int qam, int prec, int flags, uint64_t* ticket);
/* Non-blocking: *done = 1 once the frame's results are in the host buffers;
 * latency_us (may be NULL) = completion - submit in microseconds, -1 if not done. */
int dbp_server_poll(dbp_server* srv, uint64_t ticket, int* done, double* latency_us);
/* Blocks until the frame is done, reports latency and queueing time (submit to
 * admission), and forgets the ticket.  Returns the frame's status. */
int dbp_server_wait(dbp_server* srv, uint64_t ticket, double* latency_us, double* queue_us);
int dbp_server_stats(dbp_server* srv, size_t* peak_bytes, int* peak_inflight, uint64_t* completed);
/* Admission batching: a frame admitted to a free slot takes up to
 * max_frames - 1 more queued frames of the same U and I/O mode (FP32, not
 * against a resident channel; the next 64 queued frames are looked at) into
 * one dbp_detect_admm_batch launch.  max_frames = 1 turns batching off;
 * the default is 8.  DBP_ERR_INVALID outside 1 .. DBP_MAX_BATCH. */
int dbp_server_set_batching(dbp_server* srv, int max_frames);

/* Static channels (resident state of the serving loop).  The channel of a
 * coherence interval is loaded once: dbp_channel_load copies H (pinned host
 * buffer, or device buffer with DBP_SERVE_DEVICE_IO) into the arena and runs
 * dbp_factor_admm on it (Algorithm 1's preprocessing, B_c^{-1} kept
 * resident); it returns once H is copied (H may then be released) while the
 * factorisation runs on asynchronously.  Frames of received vectors are then
 * submitted
 * with dbp_server_submit_factored, which carries only y and runs Algorithm
 * 1's iterations (dbp_detect_admm_factored) against the resident factors,
 * ordered after the factorisation.  The channel holds
 * n_sc*B*U*8 + dbp_factor_bytes(n_sc, U, C) bytes of the budget until
 * dbp_channel_free, which returns DBP_ERR_BUSY while frames against it are
 * queued or running and DBP_ERR_NOTFOUND for an unknown handle.  Load returns
 * DBP_ERR_NOMEM if the channel does not fit in what is free of the budget now;
 * a frame that cannot fit beside the resident channels is refused with
 * DBP_ERR_NOMEM at submission.  y / s_hat / hard follow the rules of
 * dbp_server_submit.
 * With flags | DBP_CHANNEL_H16 the channel keeps H in the packed FP16 form of
 * dbp_pack_channel_h16 (dbp_channel_h16_bytes(n_sc, B, U, C) +
 * dbp_factor_bytes(n_sc, U, C) bytes of the budget) and its frames run
 * dbp_detect_admm_factored_h16 (low-precision path).  During such a load a
 * temporary complex64 copy of H also takes n_sc*B*U*8 bytes of the budget,
 * and the load returns only after packing and factorisation have finished. */
int dbp_channel_load(dbp_server* srv, const void* H, int n_sc, int B, int U, int C,
                     float rho, int prec, int flags, uint64_t* channel);
int dbp_channel_free(dbp_server* srv, uint64_t channel);
int dbp_server_submit_factored(dbp_server* srv, uint64_t channel, const void* y,
                               void* s_hat, uint8_t* hard, int n_sym, int T, float N0,
                               int reg, int qam, int flags, uint64_t* ticket);

#ifdef __cplusplus
}
#endif

#endif /* DBP_H_ */
