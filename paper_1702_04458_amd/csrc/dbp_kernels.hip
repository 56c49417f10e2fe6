// HIP kernels for decentralized uplink detection and downlink precoding on gfx950.
//
// Method: Li et al., "Decentralized Baseband Processing for Massive MU-MIMO
// Systems" (arXiv:1702.04458).  Algorithm 1 (decentralized ADMM detection,
// U x U branch, eq. StepE1variant1), Algorithm 2 (decentralized CG detection,
// eqs. CGiteration / CGdecentralization) and Algorithm 3 (decentralized ADMM
// beamforming, S x S branch).  On one GPU the antenna clusters are a batch
// axis: each (subcarrier, cluster) problem is a lane group of a wave64, the
// clusters of one subcarrier sit in one workgroup, and the consensus sum of the
// paper's fusion node is an LDS reduction in fixed cluster order (so every
// result is independent of how the work is tiled).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dbp_device.h"
#include "dbp_launch.h"

namespace dbp {

constexpr int kStageRows = 8;   // rows of H_c staged per pass through LDS
// c32 slots of one wave's stage buffer: the staged rows, plus room for the
// padded transposes (a 32 x 32 float tile with a row pitch of 33, or two
// 16 x 16 problems as planes of 32 x 17 floats), whose offsets are then
// compile-time constants
constexpr int kStageWave = kStageRows * 64 + 32;

// Loads in the Gram prologues never branch: a request outside the problem
// (padding cluster, subcarrier past the end, ragged row past S) reads a valid
// address of the same array instead (row min(s, S-1) of a base clamped to the
// array start) and is zeroed by a select.
__device__ __forceinline__ c32 ld_or_zero(const c32* p, bool ok) {
  const c32 v = *p;
  return ok ? v : c32{0.f, 0.f};
}

// Fourth word of a raw buffer descriptor on gfx9-family GPUs (32-bit data
// format, no swizzle, stride 0: the range check is on bytes).
constexpr int kBufferWord3 = 0x00020000;

// Prefetch depth of the matrix-core Gram prologues (row pairs for U = 32, row
// quadruples for U = 16): the loads of the next chunk are in flight while the
// current chunk's MFMAs run.  Build-time tuning knobs.
#ifndef DBP_PREFETCH_U32
#define DBP_PREFETCH_U32 2
#endif
#ifndef DBP_PREFETCH_U16
#define DBP_PREFETCH_U16 1
#endif

// LDS carve-up shared by the kernels (all offsets in c32 units):
//   stage[nw][kStageWave]       staged H rows (kStageRows x 64, one slot per lane)
//   ystage[nw][kStageRows][8]   staged y entries (one per problem of the wave)
//   line[nw][64]                per-wave broadcast line
//   cons[2][nw][64]             double-buffered consensus slots (one per lane)
//   aux[nw][64]                 per-problem scalars (precoder power scaling)
struct Smem {
  c32* stage;
  c32* ystage;
  c32* line;
  c32* cons;
  c32* aux;
};

__device__ __forceinline__ Smem carve(c32* base, int nw) {
  Smem s;
  s.stage = base;
  s.ystage = s.stage + nw * kStageWave;
  s.line = s.ystage + nw * kStageRows * 8;
  s.cons = s.line + nw * 64;
  s.aux = s.cons + 2 * nw * 64;
  return s;
}

size_t smem_bytes(int nw) { return sizeof(c32) * (size_t)nw * (kStageWave + kStageRows * 8 + 64 + 128 + 64); }

// One pass over the S rows of H_c (and of y_c for symbol n): accumulates the
// Gram row A[v] += conj(H[s][u]) H[s][v] when WITH_GRAM, and always
// hy = sum_s conj(H[s][u]) y[s] (row u of H_c^H y_c).
template <int G, bool WITH_GRAM>
__device__ __forceinline__ c32 cluster_pass(const c32* __restrict__ H, const c32* __restrict__ y, c32 (&A)[G],
                                            int k, int c, int n, int u, int g, int lane, int wave, bool active,
                                            int B, int S, int U, int n_sym, const Smem& sm) {
  constexpr int R = kStageRows;
  c32 hy = cz();
  c32* stage = sm.stage + wave * kStageWave;
  c32* yst = sm.ystage + wave * R * 8;
  const c32* Hk = H + (size_t)k * B * U + (size_t)c * S * U;
  const c32* yk = y + ((size_t)k * n_sym + n) * B + (size_t)c * S;
  for (int s0 = 0; s0 < S; s0 += R) {
    c32 h[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int s = s0 + r;
      h[r] = (active && s < S) ? Hk[(size_t)s * U + u] : cz();
      if (WITH_GRAM) stage[r * 64 + lane] = h[r];
    }
    if (u < R) {
      const int s = s0 + u;
      yst[u * 8 + g] = (active && s < S) ? yk[s] : cz();
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (WITH_GRAM) {
#pragma unroll
        for (int v0 = 0; v0 < G; v0 += 8) {
          c32 row[8];
          lds_read_vec<8>(stage + r * 64 + g * G + v0, row);
#pragma unroll
          for (int v = 0; v < 8; ++v) cmacc(A[v0 + v], h[r], row[v]);
        }
      }
      cmacc(hy, h[r], yst[r * 8 + g]);
    }
    wave_lds_sync();
  }
  return hy;
}

// Entries of the packed FP16 channel: a pair of binary16 values (real part in
// the low half), widened to FP32 exactly.
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));

// One complex entry scaled by 2^-e and rounded to complex FP16 (real part in
// the low half), the packed channel's format.
__device__ __forceinline__ uint32_t pack_pair(c32 v, int e) {
  const h16x2 p = {(_Float16)ldexpf(v.re, -e), (_Float16)ldexpf(v.im, -e)};
  return __builtin_bit_cast(uint32_t, p);
}

// The packed channel's exponent of a tile whose largest component is m: its
// largest component lands in [2^14, 2^15).
__device__ __forceinline__ int pack_exponent(float m) {
  return (m > 0.f && m <= 3.4028235e38f) ? min(max(ilogbf(m) - 14, -126), 113) : 0;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ c32 widen_h16(uint32_t w) {
  const h16x2 v = __builtin_bit_cast(h16x2, w);
  return c32{(float)v.x, (float)v.y};
}

// Row u of H_c^H y_c for symbol n for the resident forms (no Gram to share
// the pass with): every lane reads its column entry of each row of H_c
// (complex64, or the packed FP16 channel widened to FP32, the products
// accumulated in FP32 and the tile's power-of-two scale applied once at the
// end, which is exact) and the row's y entry directly (one address per lane
// group), with no LDS staging, so the loads of several rows are in flight
// together.  The FP16 channel uses it; for complex64 H the LDS-staged pass
// measured the same.
template <int G, bool H16>
__device__ __forceinline__ c32 cluster_hy_direct(const UlArgs& a, int k, int c, int n, int u, bool active) {
  c32 hy = cz();
  if (!active) return hy;
  const c32* yk = a.y + ((size_t)k * a.n_sym + n) * a.B + (size_t)c * a.S;
  const size_t hb = (size_t)k * a.B * G + (size_t)c * a.S * G + u;
  constexpr int CH = G >= 64 ? 4 : 8;   // rows in flight per lane (register budget at U = 64)
  int s = 0;
  for (; s + CH <= a.S; s += CH) {
    c32 hv[CH], yv[CH];
#pragma unroll
    for (int r = 0; r < CH; ++r) {
      if constexpr (H16)
        hv[r] = widen_h16(a.H16[hb + (size_t)(s + r) * G]);
      else
        hv[r] = a.H[hb + (size_t)(s + r) * G];
      yv[r] = yk[s + r];
    }
#pragma unroll
    for (int r = 0; r < CH; ++r) cmacc(hy, hv[r], yv[r]);
  }
  for (; s < a.S; ++s) {
    const c32 h = H16 ? widen_h16(a.H16[hb + (size_t)s * G]) : a.H[hb + (size_t)s * G];
    cmacc(hy, h, yk[s]);
  }
  if constexpr (H16) hy = cscale(hy, a.hscale[(size_t)k * a.C + c]);
  return hy;
}

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Gauss-Jordan inversion of the HPD matrix B = G + rho I in the 32x32
// accumulator layout (lane l: column l%32, rows 8(r/4) + 4(l/32) + r%4), for
// the two Gram matrices of a wave, with lazy row and column scales: the stored
// matrix S relates to the partially swept one by true_ij = S_ij tau_i sigma_j,
// where a row / column not yet swept has scale 1 and sweeping pivot k (value
// d = B[k][k] of the current Schur complement) sets tau_k = 1/d and
// sigma_k = -1/d.  With these scales the sweep leaves row k and column k of S
// unchanged except for the diagonal, which becomes -d, and every other entry
// takes the plain Hermitian rank-1 update
//   S_ij -= conj(S_ki) S_kj / d,
// so S stays Hermitian throughout (the signed symmetry of the swept matrix is
// absorbed by the opposite signs of tau and sigma) and the multipliers of the
// update come from row k alone.  At the end every index is swept and
// B^{-1}_ij = -S_ij / (d_i d_j).
//
// Row k lives in register 4(k/8) + k%4 of lane half (k/4)&1.  On the FP32
// matrix cores the complex rank-1 update is two v_mfma_f32_32x32x2f32 whose
// K = 2 slots are the two lane halves, so row k is first copied into the
// other half (lanes < 32 get (Re, Im), lanes >= 32 (Im, Re)).
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Undo the lazy scales of one swept 32x32 accumulator: entry (i, j) becomes
// -S_ij * pv_i * pv_j * extra, pv the reciprocal pivots.  pvv holds pv of this
// lane's column; the row factors come through 32 floats of wave-private LDS.
__device__ __forceinline__ void gj_unscale_u32(f32x16& re, f32x16& im, float pvv, float extra, int lane, float* line) {
  const int h = lane >> 5, col = lane & 31;
  if (h == 0) line[col] = pvv;
  wave_lds_sync();
  float4 q[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) q[g] = *reinterpret_cast<const float4*>(line + 8 * g + 4 * h);
  wave_lds_sync();
  const float cs = -pvv * extra;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const float4 v = q[r / 4];
    const float pr = (r % 4 == 0) ? v.x : (r % 4 == 1) ? v.y : (r % 4 == 2) ? v.z : v.w;
    const float sc = cs * pr;
    re[r] *= sc;
    im[r] *= sc;
  }
}

// ADD_RHO: add rho to the diagonal first (false: the caller's accumulators
// already hold G + rho I).  LAZY: leave the swept matrix S with its scales
// (B^{-1}_ij = -S_ij pv_i pv_j) and return in pvs[0] the reciprocal pivot of
// this lane's own row (problem l / 32, row l % 32); the diagonal is also not
// negated at its pivot, so that S_ii ends 2 d_i above the negated form's
// (no later update reads it) and B^{-1}_ii = -S_ii pv_i^2 + 2 pv_i.
template <bool ADD_RHO = true, bool LAZY = false>
__device__ __forceinline__ void gj_invert_mfma_u32(f32x16 (&re)[2], f32x16 (&im)[2], int lane, float rho, float* line,
                                                   float* pvs = nullptr) {
  const int h = lane >> 5, col = lane & 31;
  if constexpr (ADD_RHO) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const bool dg = (8 * (r / 4) + 4 * h + (r % 4) == col);
      re[0][r] += dg ? rho : 0.f;
      re[1][r] += dg ? rho : 0.f;
    }
  } else {
    (void)rho;
  }
  float pvv[2] = {0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const int rr = 4 * (k / 8) + (k % 4);   // register holding row k
    const int hk = (k / 4) & 1;             // lane half holding row k
    const bool isk = (col == k);
    const bool dg = isk && h == hk;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const float sr = re[p][rr], si = im[p][rr];
      // Row k at column col with entry k zeroed (row and column k are left
      // alone by the update): lanes < 32 get (first, second) = (Re, Im),
      // lanes >= 32 (Im, Re).  A lane reads the lane of its own column in
      // either half, so zeroing at the source zeroes column k everywhere.
      // The imaginary update takes the same A operand and (Im, -Re) as B, so
      // the real part enters that swap negated.
      const float srm = isk ? 0.f : sr, sim = isk ? 0.f : si, srn = isk ? 0.f : -sr;
      const auto fs = __builtin_amdgcn_permlane32_swap(__float_as_uint(srm), __float_as_uint(sim), false, false);
      const auto sf = __builtin_amdgcn_permlane32_swap(__float_as_uint(sim), __float_as_uint(srn), false, false);
      const float first = __uint_as_float(fs[hk]);
      const float second = __uint_as_float(sf[hk]);
      const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sr), k + 32 * hk));
      const float pv = __builtin_amdgcn_rcpf(d);
      // Re: -pv (Re_i Re_j + Im_i Im_j), Im: -pv (Re_i Im_j - Im_i Re_j)
      const float Are = -pv * first;
      const float Aim = Are;
      if constexpr (!LAZY) re[p][rr] = dg ? -sr : sr;
      re[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(Are, first, re[p], 0, 0, 0);
      im[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(Aim, second, im[p], 0, 0, 0);
      if constexpr (LAZY) {
        // the pivot reciprocals go to LDS (no vector instruction per pivot)
        if (lane == 0) line[32 * p + k] = pv;
      } else {
        pvv[p] = isk ? pv : pvv[p];
        // select in place (otherwise the compiler keeps every pivot's pv live
        // until the end)
        asm volatile("" : "+v"(pvv[p]));
      }
    }
  }
  if constexpr (LAZY) {
    wave_lds_sync();
    pvs[0] = line[32 * h + col];   // pv of this lane's own row (problem h, row col)
    wave_lds_sync();
    __builtin_amdgcn_sched_barrier(0);
  } else {
#pragma unroll
    for (int p = 0; p < 2; ++p) gj_unscale_u32(re[p], im[p], pvv[p], 1.f, lane, line);
  }
}

// Exchange between the wave's two 32-lane halves: v_permlane32_swap(X, Y)
// leaves [X of lanes 0-31 | Y of lanes 0-31] in its first result and
// [X of lanes 32-63 | Y of lanes 32-63] in its second.  With X and Y the two
// halves' accumulators of tile columns 0 and 1 (or problems 0 and 1), the
// first result is every lane's half-0 entry and the second its half-1 entry.
struct f32pair {
  float lo, hi;
};
__device__ __forceinline__ f32pair swap_halves(float x, float y) {
  const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return f32pair{__uint_as_float(s[0]), __uint_as_float(s[1])};
}

// v(lane) + v(lane ^ D) for D = 16 (odd and even rows of 16 lanes swapped by
// v_permlane16_swap) or D = 32 (wave halves, v_permlane32_swap); any other D
// goes through a lane shuffle.
template <int D>
__device__ __forceinline__ float pair_sum(float v) {
  if constexpr (D == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  } else if constexpr (D == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  } else {
    return v + __shfl_xor(v, D, 64);
  }
}

// Gram matrices of the two problems of a wave (U = 32, P = 2) on the matrix
// cores with v_mfma_f32_32x32x2f32, K running over pairs of antenna rows:
//   Re G = sum_s Hr[s]^T Hr[s] + Hi[s]^T Hi[s],
//   Im G = sum_s Hr[s]^T Hi[s] - Hi[s]^T Hr[s].
// For the Gram of one problem lane l supplies H[s0 + l/32][l%32] (or its
// P = Hr + Hi) as both the A and the B operand.  Only P^T P and M = Hr^T Hi
// are accumulated (two MFMAs per row pair instead of four), and
// Re G = P^T P - M - M^T, Im G = M - M^T are formed at the end.  The 32x32 result leaves lane l holding column l%32 for
// rows 8(r/4) + 4(l/32) + r%4 (r = 0..15); by Hermitian symmetry that is row
// l%32 conjugated, for half h = l/32 of the columns.  With INVERT the
// accumulators are replaced by (G + rho I)^{-1} on the matrix cores first.
// One exchange between lanes l and l^32 then gives every lane the full row of
// its own problem (lane-row layout, problem = l/32).  Returns row u of
// H_c^H y_c for symbol 0.  LAZY (with INVERT): A receives row u of the swept
// matrix S with its scales left in place, and *pvl the reciprocal pivot pv_u
// of this lane's row, so that B^{-1} q = -pv_u sum_v S_uv (pv_v q_v).
// PACK (factor-only kernel): when a.H16 is set, H is also written as the
// packed FP16 channel (a.H16, a.hscale; the format of pack_h16, bit for bit):
// the tile maxima are taken during the Gram's pass and one more pass converts.
template <bool INVERT, bool LAZY = false, bool FLAT = false, bool PACK = false>
__device__ __forceinline__ c32 gram_mfma_u32(const UlArgs& a, c32 (&A)[32], int lane, int wave, float* line,
                                             float* stage, float* pvl = nullptr) {
  const int h = lane >> 5, col = lane & 31;
  f32x16 re[2], im[2];
  c32 hyp[2];
  const c32* Hp[2];
  const c32* yp[2];
  bool act[2];
  // With INVERT the real part starts from rho I: the diagonal entry (col, col)
  // sits in register 4 (col / 8) + col % 4 of lane half (col / 4) % 2.
  const int dr = (INVERT && h == ((col >> 2) & 1)) ? 4 * (col >> 3) + (col & 3) : -1;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int lp = wave * 2 + p;
    const int ls = lp / a.Cp, c = lp % a.Cp;
    const int k = a.blk * a.sc_per_block + ls;
    act[p] = (k < a.n_sc) && (c < a.C);
    Hp[p] = act[p] ? a.H + (size_t)k * a.B * 32 + (size_t)c * a.S * 32 : a.H;
    yp[p] = act[p] ? a.y + (size_t)k * a.n_sym * a.B + (size_t)c * a.S : a.y;
#pragma unroll
    for (int r = 0; r < 16; ++r) re[p][r] = (r == dr) ? a.rho : 0.f;
    im[p] = f32x16{};
    hyp[p] = cz();
  }
  // Software pipeline: the loads of the next CH row pairs are in flight while
  // the MFMAs of the current ones run.
  constexpr int CH = DBP_PREFETCH_U32;
  c32 hv[2][CH], yv[2][CH], hn[2][CH], yn[2][CH];
  // Buffer loads over each problem's S rows of H_c and S entries of y_c (no
  // bytes for an inactive problem): the hardware range check returns zero
  // past the end, which pads the last row pair and the inactive problems
  // without a select, and the per-problem bases stay in scalar registers.
  // The whole offset is in the vector operand (the scalar offset is outside
  // the range check).
  __amdgpu_buffer_rsrc_t hrs[2], yrs[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    hrs[p] = __builtin_amdgcn_make_buffer_rsrc(const_cast<c32*>(Hp[p]), 0, act[p] ? a.S * 256 : 0, kBufferWord3);
    yrs[p] = __builtin_amdgcn_make_buffer_rsrc(const_cast<c32*>(yp[p]), 0, act[p] ? a.S * 8 : 0, kBufferWord3);
  }
  auto fetch = [&](int s0, c32 (&hd)[2][CH], c32 (&yd)[2][CH]) {
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int s = s0 + 2 * q + h;   // row s, column col: byte 256 s + 8 col
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        hd[p][q] = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(hrs[p], s * 256 + col * 8, 0, 0));
        yd[p][q] = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(yrs[p], s * 8, 0, 0));
      }
    }
  };
  const bool pk = PACK && a.H16 != nullptr;   // uniform
  float mx[2] = {0.f, 0.f};
  auto accumulate = [&](const c32 (&hd)[2][CH], const c32 (&yd)[2][CH]) {
#pragma unroll
    for (int q = 0; q < CH; ++q) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const c32 x = hd[p][q];
        if constexpr (PACK)
          if (pk) mx[p] = fmaxf(mx[p], fmaxf(fabsf(x.re), fabsf(x.im)));
        const float pr = x.re + x.im;
        re[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(pr, pr, re[p], 0, 0, 0);       // P^T P, P = Hr + Hi
        im[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(x.re, x.im, im[p], 0, 0, 0);   // M = Hr^T Hi
        cmacc(hyp[p], x, yd[p][q]);
      }
    }
  };
  // the two buffers in turn (no copies).  FLAT: the loop body always runs
  // both halves and the rows past the last full double step follow it (with
  // an exit between the halves the compiler copies the accumulators of the
  // factor-only kernel on every step; the other kernels are compiled best
  // with the exit)
  fetch(0, hv, yv);
  if constexpr (FLAT) {
    int s0 = 0;
    for (; s0 + 4 * CH <= a.S; s0 += 4 * CH) {
      fetch(s0 + 2 * CH, hn, yn);
      accumulate(hv, yv);
      fetch(s0 + 4 * CH, hv, yv);   // zeros past S
      accumulate(hn, yn);
    }
    if (s0 < a.S) {
      if (s0 + 2 * CH < a.S) fetch(s0 + 2 * CH, hn, yn);
      accumulate(hv, yv);
      if (s0 + 2 * CH < a.S) accumulate(hn, yn);
    }
  } else {
    for (int s0 = 0; s0 < a.S; s0 += 4 * CH) {
      if (s0 + 2 * CH < a.S) fetch(s0 + 2 * CH, hn, yn);
      accumulate(hv, yv);
      if (s0 + 2 * CH >= a.S) break;
      if (s0 + 4 * CH < a.S) fetch(s0 + 4 * CH, hv, yv);
      accumulate(hn, yn);
    }
  }
  if constexpr (PACK) {
    if (pk) {
      // rows of this lane's parity, both problems, four rows in flight
      uint32_t* h16 = const_cast<uint32_t*>(a.H16);
      int e[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) e[p] = pack_exponent(wave_max(mx[p]));
      for (int s0 = h; s0 < a.S; s0 += 8) {
        c32 v[2][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int s = s0 + 2 * t;
#pragma unroll
          for (int p = 0; p < 2; ++p) v[p][t] = ld_or_zero(Hp[p] + (size_t)min(s, a.S - 1) * 32 + col, true);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int s = s0 + 2 * t;
#pragma unroll
          for (int p = 0; p < 2; ++p)
            if (act[p] && s < a.S) h16[(Hp[p] - a.H) + (size_t)s * 32 + col] = pack_pair(v[p][t], e[p]);
        }
      }
      if (lane == 0) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int lp = wave * 2 + p;
          const int k = a.blk * a.sc_per_block + lp / a.Cp, c = lp % a.Cp;
          if (act[p]) const_cast<float*>(a.hscale)[(size_t)k * a.C + c] = ldexpf(1.f, e[p]);
        }
      }
    }
  }
  // re holds rho I + P^T P and im holds M = Hr^T Hi; since P^T P = Hr^T Hr
  // + Hi^T Hi + M + M^T, Re G = P^T P - M - M^T and Im G = M - M^T (two MFMAs
  // per row pair instead of three).  M goes through the wave's stage buffer
  // with a row pitch of 33 floats (entry (i, j) at 33 i + j), conflict-free
  // both for the row-wise write and the transposed read, and with a per-lane
  // base plus a compile-time offset for every register.
#pragma unroll
  for (int p = 0; p < 2; ++p) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r / 4) + 4 * h + (r % 4);
      stage[33 * i + col] = im[p][r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r / 4) + 4 * h + (r % 4);
      const float mt = stage[33 * col + i];
      re[p][r] -= im[p][r] + mt;
      im[p][r] -= mt;
    }
    wave_lds_sync();
  }
  if constexpr (INVERT && LAZY) {
    gj_invert_mfma_u32<false, true>(re, im, lane, a.rho, line, pvl);
  } else if constexpr (INVERT) {
    gj_invert_mfma_u32<false>(re, im, lane, a.rho, line);
  }
  // exchange halves: lanes < 32 keep problem 0, lanes >= 32 keep problem 1
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m0 = 8 * (r / 4) + (r % 4);      // column of this slot in half 0
    const f32pair xr = swap_halves(re[0][r], re[1][r]);
    const f32pair xi = swap_halves(im[0][r], im[1][r]);
    A[m0] = c32{xr.lo, -xi.lo};
    A[m0 + 4] = c32{xr.hi, -xi.hi};
  }
  // rows of parity 0 (first result) plus rows of parity 1 (second result)
  const f32pair yr = swap_halves(hyp[0].re, hyp[1].re);
  const f32pair yi = swap_halves(hyp[0].im, hyp[1].im);
  return c32{yr.lo + yr.hi, yi.lo + yi.hi};
}

// ---------------------------------------------------------------------------
// Mixed precision preprocessing for U = 32: the Gram on FP16 / BF16 matrix
// cores with FP32 accumulation.  Each problem's H_c is scaled by a power of two
// 2^e chosen from its largest entry (so its half-precision image uses the top
// of the format; exact, undone on the FP32 Gram), then split as
// H = H_hi + H_lo with H_hi = half(H) and H_lo = half(H - H_hi).  The Gram is
// refined to near FP32 accuracy by accumulating the correction products:
//   G ~ H_hi^H H_hi + H_hi^H H_lo + H_lo^H H_hi
// (the dropped H_lo^H H_lo term is below FP32 rounding for FP16).  Every
// v_mfma_f32_32x32x16 covers 16 real rows: lane l supplies column l%32 of the
// 8 rows 8(l/32) .. 8(l/32)+7 of its 16-row chunk as both the A and the B
// operand; the result uses the same 32x32 accumulator layout as the FP32 path.
// ---------------------------------------------------------------------------
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename HT>
struct HalfMma;
template <>
struct HalfMma<_Float16> {
  typedef f16x8 V;
  static __device__ __forceinline__ f32x16 mma(V x, V y, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(x, y, c, 0, 0, 0);
  }
};
template <>
struct HalfMma<__bf16> {
  typedef bf16x8 V;
  static __device__ __forceinline__ f32x16 mma(V x, V y, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, c, 0, 0, 0);
  }
};


// Normalisation of the mixed-mode Gram before the FP16 inverse.  H_c is scaled
// by 2^ex so that its largest entry lies in [2^13, 2^14); the Gram of i.i.d.
// entries then has diagonal about S * 2^24, and a shift of 9 + ceil(log2 S)
// brings it to about 2^15.  The FP16 inverse works on the operands r 2^-7 and
// 2^7 r / d of a pivot row r (both about 2^8 for entries of the diagonal's
// size, far below the FP16 limit of 2^16), so that values the matrix cores
// would flush (below 2^-14) only occur for contributions 2^-21 or more below
// the entries they update.  The shift
// depends on S only, so scaling H by 2^k changes ex alone and the result stays
// bit-exact.
__device__ __forceinline__ int norm_shift(int S) { return 9 + (32 - __builtin_clz((unsigned)(S > 1 ? S - 1 : 1))); }

// With NORM the Gram leaves scaled by 2^-norm_shift(S) instead of being
// returned to the units of H (see gj_invert_split16_u32); ex receives each
// problem's scaling exponent either way.
template <typename HT, bool NORM>
__device__ __forceinline__ void gram_split_u32(const UlArgs& a, f32x16 (&re)[2], f32x16 (&im)[2], c32 (&hyp)[2],
                                               int lane, int wave, int (&ex)[2], float* stage, float (&trg)[2]) {
  typedef typename HalfMma<HT>::V V;
  const int h = lane >> 5, col = lane & 31;
  const c32* Hp[2];
  const c32* yp[2];
  bool act[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int lp = wave * 2 + p;
    const int ls = lp / a.Cp, c = lp % a.Cp;
    const int k = a.blk * a.sc_per_block + ls;
    act[p] = (k < a.n_sc) && (c < a.C);
    Hp[p] = act[p] ? a.H + (size_t)k * a.B * 32 + (size_t)c * a.S * 32 : a.H;
    yp[p] = act[p] ? a.y + (size_t)k * a.n_sym * a.B + (size_t)c * a.S : a.y;
    re[p] = f32x16{};
    im[p] = f32x16{};
    hyp[p] = cz();
  }
  // buffer loads over each problem's S rows (as in gram_mfma_u32)
  __amdgpu_buffer_rsrc_t hrs[2], yrs[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    hrs[p] = __builtin_amdgcn_make_buffer_rsrc(const_cast<c32*>(Hp[p]), 0, act[p] ? a.S * 256 : 0, kBufferWord3);
    yrs[p] = __builtin_amdgcn_make_buffer_rsrc(const_cast<c32*>(yp[p]), 0, act[p] ? a.S * 8 : 0, kBufferWord3);
  }
  // pass 1: largest |Re|, |Im| of each problem -> scale exponent (and
  // ||H_c||_F^2 = tr(G_c))
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    float m = 0.f, ss = 0.f;
    for (int s0 = 0; s0 < a.S; s0 += 16) {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int s = s0 + 8 * h + t;
        const c32 v = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(hrs[p], s * 256 + col * 8, 0, 0));
        m = fmaxf(m, fmaxf(fabsf(v.re), fabsf(v.im)));
        ss = fmaf(v.re, v.re, fmaf(v.im, v.im, ss));
      }
    }
    trg[p] = wave_sum(ss);
    m = wave_max(m);
    int x = 0;
    if (m > 0.f) frexpf(m, &x);      // m < 2^x
    ex[p] = 14 - x;                  // scaled entries stay below 2^14
  }
  // pass 2: split and accumulate
  for (int s0 = 0; s0 < a.S; s0 += 16) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      c32 v[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int s = s0 + 8 * h + t;
        v[t] = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(hrs[p], s * 256 + col * 8, 0, 0));
        const c32 yv = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(yrs[p], s * 8, 0, 0));
        cmacc(hyp[p], v[t], yv);
      }
      V rh, rl, ih, il;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float xr = ldexpf(v[t].re, ex[p]), xi = ldexpf(v[t].im, ex[p]);
        const HT hr = (HT)xr, hi = (HT)xi;
        rh[t] = hr;
        rl[t] = (HT)(xr - (float)hr);
        ih[t] = hi;
        il[t] = (HT)(xi - (float)hi);
      }
      // Re G = Hr^T Hr + Hi^T Hi
      re[p] = HalfMma<HT>::mma(rh, rh, re[p]);
      re[p] = HalfMma<HT>::mma(rh, rl, re[p]);
      re[p] = HalfMma<HT>::mma(rl, rh, re[p]);
      re[p] = HalfMma<HT>::mma(ih, ih, re[p]);
      re[p] = HalfMma<HT>::mma(ih, il, re[p]);
      re[p] = HalfMma<HT>::mma(il, ih, re[p]);
      // M = Hr^T Hi (Im G = M - M^T, below)
      im[p] = HalfMma<HT>::mma(rh, ih, im[p]);
      im[p] = HalfMma<HT>::mma(rh, il, im[p]);
      im[p] = HalfMma<HT>::mma(rl, ih, im[p]);
    }
  }
  // antisymmetrise through the stage buffer, as in gram_mfma_u32
#pragma unroll
  for (int p = 0; p < 2; ++p) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r / 4) + 4 * h + (r % 4);
      stage[33 * i + col] = im[p][r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r / 4) + 4 * h + (r % 4);
      im[p][r] -= stage[33 * col + i];
    }
    wave_lds_sync();
  }
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int sh = NORM ? norm_shift(a.S) : 2 * ex[p];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      re[p][r] = ldexpf(re[p][r], -sh);
      im[p][r] = ldexpf(im[p][r], -sh);
    }
  }
}

// Accumulator layout -> lane-row layout (lanes < 32: problem 0, >= 32: problem 1)
__device__ __forceinline__ void acc_to_rows_u32(const f32x16 (&re)[2], const f32x16 (&im)[2], c32 (&A)[32], int h) {
  (void)h;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m0 = 8 * (r / 4) + (r % 4);
    const f32pair xr = swap_halves(re[0][r], re[1][r]);
    const f32pair xi = swap_halves(im[0][r], im[1][r]);
    A[m0] = c32{xr.lo, -xi.lo};
    A[m0 + 4] = c32{xr.hi, -xi.hi};
  }
}

// rows of parity 0 plus rows of parity 1 of H_c^H y_c, for this lane's problem
__device__ __forceinline__ c32 combine_hy(const c32 (&hyp)[2], int h) {
  (void)h;
  const f32pair yr = swap_halves(hyp[0].re, hyp[1].re);
  const f32pair yi = swap_halves(hyp[0].im, hyp[1].im);
  return c32{yr.lo + yr.hi, yi.lo + yi.hi};
}

// Regularised inverse in FP64 on the VALU (lane-row layout, rotated
// Gauss-Jordan as in gj_invert), for the poorly conditioned case U/S > 0.8.
struct c64 {
  double re, im;
};

template <int G>
__device__ __forceinline__ void gj_invert64(c64 (&A)[G], int u, c64* line) {
  for (int k = 0; k < G; ++k) {
    const double sg = (u < k) ? -1.0 : 1.0;
    line[(u - k) & (G - 1)] = c64{sg * A[0].re, -sg * A[0].im};
    wave_lds_sync();
    const double p = 1.0 / line[0].re;
    const bool me = (u == k);
    const c64 m = me ? c64{-p, 0.0} : c64{A[0].re * p, A[0].im * p};
    const c64 pivot_new = me ? c64{p, 0.0} : c64{-m.re, -m.im};
#pragma unroll
    for (int j0 = 0; j0 < G; j0 += 4) {
      c64 rk[4];
      const double2* q = reinterpret_cast<const double2*>(line + j0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double2 t = q[i];
        rk[i] = c64{t.x, t.y};
      }
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int j = j0 + jj;
        if (j == 0) continue;
        c64 base = me ? c64{0.0, 0.0} : A[j];
        base.re = fma(-m.re, rk[jj].re, base.re);
        base.re = fma(m.im, rk[jj].im, base.re);
        base.im = fma(-m.re, rk[jj].im, base.im);
        base.im = fma(-m.im, rk[jj].re, base.im);
        A[j - 1] = base;
      }
    }
    A[G - 1] = pivot_new;
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// Regularised inverse on the FP16 matrix cores (mixed modes): the sweep of
// gj_invert_mfma_u32 (lazy row / column scales, Hermitian update
// S_ij -= conj(S_ki) S_kj / d), with the rank-1 update issued as one
// v_mfma_f32_32x32x16_f16 per real / imaginary part.  The update is a_i b_j
// with a = -conj(r) 2^7 / d and b = r 2^-7 (r = row k): the same FP32
// coefficient 1/d as the FP32 sweep and its final unscaling, and two operands
// of comparable size (the power of two is exact).  Each operand is split into
// an FP16 hi + lo pair (round to nearest, about 22 significant bits together)
// and the K-terms hi.hi, hi.lo, lo.hi of the two real products take six of
// the eight K-slots of the lane half that holds row k: every operand a lane
// supplies comes from its own registers, and the other half supplies zeros,
// so nothing crosses lane halves.  Accumulation is FP32; the dropped lo.lo
// terms are 2^-22 relative.  FP16 MFMA runs beside the VALU, unlike FP32
// MFMA.  The matrix arrives normalised (norm_shift): rho is the normalised
// regulariser and post the power of two that undoes it.
// ---------------------------------------------------------------------------
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// (x, y) -> packed FP16 pairs hi = (x_hi, y_hi) and lo = (x - x_hi, y - y_hi)
__device__ __forceinline__ void split_f16(float x, float y, unsigned& hi, unsigned& lo) {
  const f16x2 hv = f16x2{(_Float16)x, (_Float16)y};
  const f16x2 lv = f16x2{(_Float16)(x - (float)hv[0]), (_Float16)(y - (float)hv[1])};
  hi = __builtin_bit_cast(unsigned, hv);
  lo = __builtin_bit_cast(unsigned, lv);
}

__device__ __forceinline__ f16x8 as_f16x8(u32x4 v) { return __builtin_bit_cast(f16x8, v); }

// S += a (x) b from the split pairs ah / al = (Re a, Im a), bh / bl = (Re b, Im b).
// K-slot pairs (dwords): real part (Re a, -Im a).(Re b, Im b), imaginary part
// (Re a, Im a).(Im b, Re b).
__device__ __forceinline__ void rank1_split16(f32x16& re, f32x16& im, unsigned ah, unsigned al, unsigned bh,
                                              unsigned bl) {
  const unsigned ahc = ah ^ 0x80000000u, alc = al ^ 0x80000000u;
  const unsigned bhs = __builtin_amdgcn_alignbit(bh, bh, 16), bls = __builtin_amdgcn_alignbit(bl, bl, 16);
  re = __builtin_amdgcn_mfma_f32_32x32x16_f16(as_f16x8(u32x4{ahc, ahc, alc, 0u}), as_f16x8(u32x4{bh, bl, bh, 0u}), re,
                                              0, 0, 0);
  im = __builtin_amdgcn_mfma_f32_32x32x16_f16(as_f16x8(u32x4{ah, ah, al, 0u}), as_f16x8(u32x4{bhs, bls, bhs, 0u}), im,
                                              0, 0, 0);
}

__device__ __forceinline__ void gj_invert_split16_u32(f32x16 (&re)[2], f32x16 (&im)[2], int lane, const float (&rho)[2],
                                                      const float (&post)[2], float* line) {
  const int h = lane >> 5, col = lane & 31;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const bool dg = (8 * (r / 4) + 4 * h + (r % 4) == col);
    re[0][r] += dg ? rho[0] : 0.f;
    re[1][r] += dg ? rho[1] : 0.f;
  }
  float pvv[2] = {0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const int rr = 4 * (k / 8) + (k % 4);   // register holding row k
    const int hk = (k / 4) & 1;             // lane half holding row k
    const bool isk = (col == k);
    const bool here = (h == hk);
    // operand masks (row k's half, column k excluded) with the 2^7 / 2^-7 balance
    const float ma = (here && !isk) ? 128.f : 0.f;
    const float mb = (here && !isk) ? 0.0078125f : 0.f;
    const float dn = (here && isk) ? -1.f : 1.f;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const float sr = re[p][rr], si = im[p][rr];
      const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sr), k + 32 * hk));
      const float pv = __builtin_amdgcn_rcpf(d);
      const float t = pv * ma;
      unsigned ah, al, bh, bl;
      split_f16(-sr * t, si * t, ah, al);
      split_f16(sr * mb, si * mb, bh, bl);
      re[p][rr] = sr * dn;
      rank1_split16(re[p], im[p], ah, al, bh, bl);
      pvv[p] = isk ? pv : pvv[p];
    }
  }
#pragma unroll
  for (int p = 0; p < 2; ++p) gj_unscale_u32(re[p], im[p], pvv[p], post[p], lane, line);
}

// Mixed-precision Gram + regularised inverse for U = 32; returns row u of
// H_c^H y_c and leaves row u of (G + rho I)^{-1} in A.  INV selects the
// inverse: 0 FP32 matrix cores, 1 FP64 VALU, 2 split FP16 matrix cores.
template <typename HT, int INV>
__device__ __forceinline__ c32 gram_inv_mixed_u32(const UlArgs& a, c32 (&A)[32], int lane, int wave, c64* line64,
                                                  float& trg) {
  const int h = lane >> 5;
  f32x16 re[2], im[2];
  c32 hyp[2];
  int ex[2];
  float tr[2];
  gram_split_u32<HT, INV == 2>(a, re, im, hyp, lane, wave, ex, reinterpret_cast<float*>(line64), tr);
  trg = h ? tr[1] : tr[0];
  if (INV == 0) {
    gj_invert_mfma_u32(re, im, lane, a.rho, reinterpret_cast<float*>(line64));
    acc_to_rows_u32(re, im, A, h);
  } else if (INV == 2) {
    float rho_n[2], post[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int e = 2 * ex[p] - norm_shift(a.S);
      rho_n[p] = ldexpf(a.rho, e);
      post[p] = ldexpf(1.f, e);
    }
    gj_invert_split16_u32(re, im, lane, rho_n, post, reinterpret_cast<float*>(line64));
    acc_to_rows_u32(re, im, A, h);
  } else {
    acc_to_rows_u32(re, im, A, h);
    const int u = lane & 31;
    c64 D[32];
#pragma unroll
    for (int v = 0; v < 32; ++v) D[v] = c64{(double)A[v].re + ((v == u) ? (double)a.rho : 0.0), (double)A[v].im};
    gj_invert64<32>(D, u, line64 + h * 32);
#pragma unroll
    for (int v = 0; v < 32; ++v) A[v] = c32{(float)D[v].re, (float)D[v].im};
  }
  return combine_hy(hyp, h);
}

// Gram matrices of the four problems of a wave for U = 16 (P = 4) on the
// matrix cores with v_mfma_f32_16x16x4f32, K running over quadruples of
// antenna rows: lane l supplies H[s0 + l/16][l%16] (or P = Hr + Hi) as both
// operands.  Only P^T P and M = Hr^T Hi are accumulated (two MFMAs per row
// quadruple instead of four); Re G = P^T P - M - M^T and Im G = M - M^T are
// formed in the transpose.  The
// 16x16 result leaves lane l holding column l%16 for rows 4(l/16) + r
// (r = 0..3) of every problem; by Hermitian symmetry that is row l%16
// conjugated, columns 4(l/16) .. 4(l/16)+3.  An LDS transpose (two problems
// per pass through the wave's stage buffer) gives lane 16p + u the full row u
// of problem p.  Returns row u of H_c^H y_c for symbol 0.
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Regularised inverses of the four problems of a U = 16 wave on the matrix
// cores: v_mfma_f32_16x16x1f32 runs four independent 16 x 16 x 1 products, one
// per problem (block p of the A and B operands is lane group p, block p of the
// result is registers 4p .. 4p+3).  On entry re[p] holds P^T P + rho I and
// im[p] holds M = Hr^T Hi of problem p in the accumulator layout (lane
// 16 q + col, register r: row 4 q + r, column col), so that B = H^H H + rho I
// has Re B = P^T P - M - M^T and Im B = M - M^T (M^T through LDS).
//
// The sweep is the Hermitian Gauss-Jordan elimination with lazy scales: for
// each pivot k, S_ij -= conj(w_i) w_j / S_kk for i, j != k, where w is row k;
// row and column k are left alone and the diagonal is not negated, so that
// B^{-1} = 2 D - D S D with D = diag(pv) the pivot reciprocals.  One pivot is
// four rank-1 matrix-core updates of all four problems (real and imaginary
// parts), against 60 vector FMAs per lane for the same work.  Row k of every
// problem sits in lane group k / 4, register 4 p + k % 4: it reaches problem
// p's lane group through the wave's stage buffer.  Entry k of w is zeroed in
// both operands, which leaves row and column k alone.
//
// On return lane 16 p + u holds row u of problem p's S in A (S is Hermitian:
// read as column u, conjugated) and its pivot reciprocal pv_u in *pvl.
__device__ __forceinline__ void gj_invert_mfma_u16(f32x4 (&re)[4], f32x4 (&im)[4], c32 (&A)[16], int lane,
                                                   c32* stage, float* pvl) {
  const int q = lane >> 4, col = lane & 15;
  float* pm = reinterpret_cast<float*>(stage);   // M of the four problems, row pitch 17
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int r = 0; r < 4; ++r) pm[(16 * p + 4 * q + r) * 17 + col] = im[p][r];
  wave_lds_sync();
  f32x16 sr, si;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float mt = pm[(16 * p + col) * 17 + 4 * q + r];
      sr[4 * p + r] = re[p][r] - im[p][r] - mt;
      si[4 * p + r] = im[p][r] - mt;
    }
  wave_lds_sync();
  // row k through two float planes [lane group][problem][column] (the real
  // and imaginary registers need not be paired for the stores)
  float* wre = reinterpret_cast<float*>(stage);
  float* wim = wre + 256;
  float pvm = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int g = k >> 2, rr = k & 3;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      wre[(4 * q + p) * 16 + col] = sr[4 * p + rr];
      wim[(4 * q + p) * 16 + col] = si[4 * p + rr];
    }
    wave_lds_sync();
    const c32 w = c32{wre[(4 * g + q) * 16 + col], wim[(4 * g + q) * 16 + col]};   // row k of problem q
    const float d = wre[(4 * g + q) * 16 + k];                                     // its pivot
    wave_lds_sync();
    const float pv = __builtin_amdgcn_rcpf(d);
    const bool isk = (col == k);
    const float wr = isk ? 0.f : w.re, wi = isk ? 0.f : w.im, nwr = isk ? 0.f : -w.re;
    // Re: -pv (wr_i wr_j + wi_i wi_j), Im: -pv (wr_i wi_j - wi_i wr_j)
    const float ar = -pv * wr, ai = -pv * wi;
    sr = __builtin_amdgcn_mfma_f32_16x16x1f32(ar, wr, sr, 0, 0, 0);
    sr = __builtin_amdgcn_mfma_f32_16x16x1f32(ai, wi, sr, 0, 0, 0);
    si = __builtin_amdgcn_mfma_f32_16x16x1f32(ar, wi, si, 0, 0, 0);
    si = __builtin_amdgcn_mfma_f32_16x16x1f32(ai, nwr, si, 0, 0, 0);
    // lane 16 p + u keeps pivot u of problem p (selected in place: otherwise
    // the compiler keeps every pivot's pv live until the end)
    pvm = isk ? pv : pvm;
    asm volatile("" : "+v"(pvm));
  }
  *pvl = pvm;
  // to rows, two problems per pass (two float planes of row pitch 17)
  float* pre = reinterpret_cast<float*>(stage);
  float* pim = pre + 32 * 17;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
#pragma unroll
    for (int pp = 0; pp < 2; ++pp)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * q + r;
        pre[(16 * pp + i) * 17 + col] = sr[4 * (2 * half + pp) + r];
        pim[(16 * pp + i) * 17 + col] = si[4 * (2 * half + pp) + r];
      }
    wave_lds_sync();
    if ((q >> 1) == half) {
      const int pp = q & 1;
#pragma unroll
      for (int v = 0; v < 16; ++v) A[v] = c32{pre[(16 * pp + v) * 17 + col], -pim[(16 * pp + v) * 17 + col]};
    }
    wave_lds_sync();
  }
}

// RHO: the real part starts from rho I (the diagonal entry (col, col) sits in
// register col - 4 q of lane group q = col / 4), so A leaves as G + rho I.
// INV (with RHO): A leaves as the lazily scaled inverse S of G + rho I
// (gj_invert_mfma_u16) and *pvl as the pivot reciprocal of this lane's row.
template <bool RHO = false, bool INV = false>
__device__ __forceinline__ c32 gram_mfma_u16(const UlArgs& a, c32 (&A)[16], int lane, int wave, c32* stage,
                                             float* pvl = nullptr) {
  const int q = lane >> 4, col = lane & 15;
  const int dr = RHO ? col - 4 * q : -1;
  f32x4 re[4], im[4];
  c32 hyp[4];
  const c32* Hp[4];
  const c32* yp[4];
  bool act[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int lp = wave * 4 + p;
    const int ls = lp / a.Cp, c = lp % a.Cp;
    const int k = a.blk * a.sc_per_block + ls;
    act[p] = (k < a.n_sc) && (c < a.C);
    Hp[p] = act[p] ? a.H + (size_t)k * a.B * 16 + (size_t)c * a.S * 16 : a.H;
    yp[p] = act[p] ? a.y + (size_t)k * a.n_sym * a.B + (size_t)c * a.S : a.y;
    #pragma unroll
    for (int r = 0; r < 4; ++r) re[p][r] = (r == dr) ? a.rho : 0.f;
    im[p] = f32x4{};
    hyp[p] = cz();
  }
  constexpr int CH = DBP_PREFETCH_U16;   // row quadruples per prefetch chunk
  c32 hv[4][CH], yv[4][CH], hn[4][CH], yn[4][CH];
  // Buffer loads over each problem's S rows (as in gram_mfma_u32).
  __amdgpu_buffer_rsrc_t hrs[4], yrs[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    hrs[p] = __builtin_amdgcn_make_buffer_rsrc(const_cast<c32*>(Hp[p]), 0, act[p] ? a.S * 128 : 0, kBufferWord3);
    yrs[p] = __builtin_amdgcn_make_buffer_rsrc(const_cast<c32*>(yp[p]), 0, act[p] ? a.S * 8 : 0, kBufferWord3);
  }
  auto fetch = [&](int s0, c32 (&hd)[4][CH], c32 (&yd)[4][CH]) {
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int s = s0 + 4 * j + q;   // row s, column col: byte 128 s + 8 col
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        hd[p][j] = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(hrs[p], s * 128 + col * 8, 0, 0));
        yd[p][j] = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(yrs[p], s * 8, 0, 0));
      }
    }
  };
  auto accumulate = [&](const c32 (&hd)[4][CH], const c32 (&yd)[4][CH]) {
#pragma unroll
    for (int j = 0; j < CH; ++j) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const c32 x = hd[p][j];
        const float pr = x.re + x.im;
        re[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(pr, pr, re[p], 0, 0, 0);       // P^T P, P = Hr + Hi
        im[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.re, x.im, im[p], 0, 0, 0);   // M = Hr^T Hi
        cmacc(hyp[p], x, yd[p][j]);
      }
    }
  };
  // two buffers used in turn (no copies): the next chunk's loads are in
  // flight while the current one is accumulated
  fetch(0, hv, yv);
  for (int s0 = 0; s0 < a.S; s0 += 8 * CH) {
    if (s0 + 4 * CH < a.S) fetch(s0 + 4 * CH, hn, yn);
    accumulate(hv, yv);
    if (s0 + 4 * CH >= a.S) break;
    if (s0 + 8 * CH < a.S) fetch(s0 + 8 * CH, hv, yv);
    accumulate(hn, yn);
  }
  // Transpose through LDS, two problems per pass: the real and imaginary
  // accumulators go to two float planes, entry (i, j) of problem pp at
  // (16 pp + i) 17 + j (a row pitch of 17: the column read and the transposed
  // read are conflict-free, and every offset is a compile-time constant).
  // re holds P^T P and im holds M = Hr^T Hi, so
  // Re G[v][col] = (P^T P)[v][col] - M[v][col] - M[col][v] and
  // Im G[v][col] = M[v][col] - M[col][v].
  float* pre = reinterpret_cast<float*>(stage);
  float* pim = pre + 32 * 17;
  if constexpr (INV) {
    gj_invert_mfma_u16(re, im, A, lane, stage, pvl);
  } else {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
#pragma unroll
      for (int pp = 0; pp < 2; ++pp)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 4 * q + r;
          pre[(16 * pp + i) * 17 + col] = re[2 * half + pp][r];
          pim[(16 * pp + i) * 17 + col] = im[2 * half + pp][r];
        }
      wave_lds_sync();
      if ((q >> 1) == half) {
        const int pp = q & 1;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const float gr = pre[(16 * pp + v) * 17 + col], gi = pim[(16 * pp + v) * 17 + col];
          const float mt = pim[(16 * pp + col) * 17 + v];
          A[v] = c32{gr - gi - mt, mt - gi};
        }
      }
      wave_lds_sync();
    }
  }
  // H_c^H y_c: sum the four row classes (lanes col, col+16, col+32, col+48)
  // and hand problem p's sum to row p: v_permlane16_swap of problems (0, 1)
  // and (2, 3) adds rows in pairs (problem 0 or 2 on even rows, 1 or 3 on odd
  // rows), v_permlane32_swap then adds the halves, leaving problem q on row q.
  auto scatter_sum = [](float v0, float v1, float v2, float v3) {
    const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v0), __float_as_uint(v1), false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(__float_as_uint(v2), __float_as_uint(v3), false, false);
    const float s01 = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    const float s23 = __uint_as_float(b[0]) + __uint_as_float(b[1]);
    const auto c = __builtin_amdgcn_permlane32_swap(__float_as_uint(s01), __float_as_uint(s23), false, false);
    return __uint_as_float(c[0]) + __uint_as_float(c[1]);
  };
  return c32{scatter_sum(hyp[0].re, hyp[1].re, hyp[2].re, hyp[3].re),
             scatter_sum(hyp[0].im, hyp[1].im, hyp[2].im, hyp[3].im)};
}

// Downlink S x S Gram A_c[a][b] = sum_u conj(Hu[a][u]) Hu[b][u] (S <= 16,
// U = 32 users as the contraction index, two problems per wave) on the matrix
// cores with v_mfma_f32_16x16x4f32: lane l supplies Hu[l%16][u0 + l/16] (or
// its P = Hr + Hi) as both operands; only P P^T and M = Hr Hi^T are
// accumulated (two MFMAs per four users instead of four).  The operands come
// from the register copy hcol (lane u of group g: Hu[i][u]) through LDS, so H
// is read from memory once.  The 16x16 result (lane l: column l%16, rows 4(l/16)+r) goes
// through the wave's stage buffer so that lane b < 16 of each problem's lane
// group reads row b.
// SPLITOUT: the result in the split-row layout of gj_invert_sym_split16 (lane
// r of DPP row h of the group gets entries 8h .. 8h+7 of row r) instead of
// one row per lane u < 16.
template <bool SPLITOUT = false>
__device__ __forceinline__ void gram_dl_mfma_s16_u32(const c32 (&hcol)[16], c32 (&A)[SPLITOUT ? 8 : 16], int lane,
                                                     int g, int u, c32* stage) {
  const int q = lane >> 4, r16 = lane & 15;
  f32x4 re[2], im[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    // problem p's tile (from the register copy hcol, zero past S) through
    // the stage buffer: entry (i, w) at 33 i + w (a row pitch of 33 complex
    // values: conflict-free, and every offset a compile-time constant)
    if (g == p) {
#pragma unroll
      for (int i = 0; i < 16; ++i) stage[i * 33 + u] = hcol[i];
    }
    wave_lds_sync();
    c32 x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = stage[r16 * 33 + q + 4 * j];
    wave_lds_sync();
    re[p] = f32x4{};
    im[p] = f32x4{};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float pr = x[j].re + x[j].im;
      re[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(pr, pr, re[p], 0, 0, 0);               // P P^T, P = Hr + Hi
      im[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[j].re, x[j].im, im[p], 0, 0, 0);   // M = Hr Hi^T
    }
  }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int r = 0; r < 4; ++r) stage[p * 256 + (4 * q + r) * 16 + r16] = c32{re[p][r], im[p][r]};
  wave_lds_sync();
  // Re A[b][v] = (P P^T)[b][v] - M[b][v] - M[v][b], Im A[b][v] = M[b][v] - M[v][b]
  const int p = lane >> 5, b = lane & 31;
  const float* stf = reinterpret_cast<const float*>(stage + p * 256);
  if constexpr (SPLITOUT) {
    const int r = b & 15, v0 = 8 * (b >> 4);
    c32 row[8];
    lds_read_vec<8>(stage + p * 256 + r * 16 + v0, row);
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const float mt = stf[2 * ((v0 + v) * 16 + r) + 1];
      A[v] = c32{row[v].re - row[v].im - mt, row[v].im - mt};
    }
  } else if (b < 16) {
#pragma unroll
    for (int v0 = 0; v0 < 16; v0 += 8) {
      c32 row[8];
      lds_read_vec<8>(stage + p * 256 + b * 16 + v0, row);
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const float mt = stf[2 * ((v0 + v) * 16 + b) + 1];
        A[v0 + v] = c32{row[v].re - row[v].im - mt, row[v].im - mt};
      }
    }
  }
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// U = 64 (one problem per wave): the 64x64 Gram and its regularised inverse as
// four 32x32 accumulator tiles (I, J) (rows 32I.., columns 32J..; lane l holds
// column 32J + l%32 of tile (I, J) for rows 32I + 8(r/4) + 4(l/32) + r%4).
// Gram: lane l supplies H[s0 + l/32][32I + l%32] as A and H[s0 + l/32][32J + l%32]
// as B.  Gauss-Jordan as in gj_invert_mfma_u32, with the rank-1 update of every
// pivot issued on all four tiles.
// ---------------------------------------------------------------------------
// Undo the lazy scales of the four swept tiles (as gj_unscale_u32): pvv[J]
// holds pv of column 32J + l%32; the 64 row factors go through LDS.
__device__ __forceinline__ void gj_unscale_u64(f32x16 (&re)[2][2], f32x16 (&im)[2][2], const float (&pvv)[2],
                                               float extra, int lane, float* line) {
  const int h = lane >> 5, col = lane & 31;
  line[32 * h + col] = pvv[h];
  wave_lds_sync();
  const float cs[2] = {-pvv[0] * extra, -pvv[1] * extra};
#pragma unroll
  for (int I = 0; I < 2; ++I) {
    float4 q[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) q[g] = *reinterpret_cast<const float4*>(line + 32 * I + 8 * g + 4 * h);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float4 v = q[r / 4];
      const float pr = (r % 4 == 0) ? v.x : (r % 4 == 1) ? v.y : (r % 4 == 2) ? v.z : v.w;
#pragma unroll
      for (int J = 0; J < 2; ++J) {
        const float sc = cs[J] * pr;
        re[I][J][r] *= sc;
        im[I][J][r] *= sc;
      }
    }
  }
  wave_lds_sync();
}

// dst = src^H for one 32x32 tile pair (real, imaginary) through the wave's
// stage buffer, a row pitch of 33 floats (as the Gram's transposes).
__device__ __forceinline__ void tile_conj_transpose(const f32x16& sre, const f32x16& sim, f32x16& dre, f32x16& dim,
                                                    int h, int col, float* stage) {
#pragma unroll
  for (int part = 0; part < 2; ++part) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r / 4) + 4 * h + (r % 4);
      stage[33 * i + col] = part ? sim[r] : sre[r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r / 4) + 4 * h + (r % 4);
      const float t = stage[33 * col + i];
      if (part)
        dim[r] = -t;
      else
        dre[r] = t;
    }
    wave_lds_sync();
  }
}

// The swept matrix S stays Hermitian, so tile (1, 0) is tile (0, 1)^H
// throughout.  While the pivots of the first block column are swept (rows
// from tiles (0, 0), (0, 1)) tile (1, 0) is not updated; it is formed as
// (0, 1)^H before the second block's pivots (rows from tiles (1, 0), (1, 1)),
// which in turn leave tile (0, 1) alone until it is formed as (1, 0)^H at the
// end: six matrix-core updates per pivot instead of eight.
__device__ __forceinline__ void gj_invert_mfma_u64(f32x16 (&re)[2][2], f32x16 (&im)[2][2], int lane, float rho,
                                                   float* line, float* stage) {
  const int h = lane >> 5, col = lane & 31;
  // B = G + rho I
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const bool dg = (8 * (r / 4) + 4 * h + (r % 4) == col);
    re[0][0][r] += dg ? rho : 0.f;
    re[1][1][r] += dg ? rho : 0.f;
  }
  float pvv[2] = {0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < 64; ++kk) {
    const int Ik = kk / 32, kr = kk % 32;
    const int rr = 4 * (kr / 8) + (kr % 4);
    const int hk = (kr / 4) & 1;
    if (kk == 32) tile_conj_transpose(re[0][1], im[0][1], re[1][0], im[1][0], h, col, stage);
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(re[Ik][Ik][rr]), kr + 32 * hk));
    const float pv = __builtin_amdgcn_rcpf(d);
    // row kk with entry kk zeroed at the source lanes, as in gj_invert_mfma_u32
    float first[2], second[2];
#pragma unroll
    for (int J = 0; J < 2; ++J) {
      const float sr = re[Ik][J][rr], si = im[Ik][J][rr];
      const bool isk = (32 * J + col == kk);
      // (Im, -Re) as the imaginary update's B operand, as at U = 32
      const float srm = isk ? 0.f : sr, sim = isk ? 0.f : si, srn = isk ? 0.f : -sr;
      const auto fs = __builtin_amdgcn_permlane32_swap(__float_as_uint(srm), __float_as_uint(sim), false, false);
      const auto sf = __builtin_amdgcn_permlane32_swap(__float_as_uint(sim), __float_as_uint(srn), false, false);
      first[J] = __uint_as_float(fs[hk]);
      second[J] = __uint_as_float(sf[hk]);
      re[Ik][J][rr] = (isk && h == hk) ? -sr : sr;
    }
    float Are[2], Aim[2];
#pragma unroll
    for (int J = 0; J < 2; ++J) {
      Are[J] = -pv * first[J];
      Aim[J] = Are[J];
    }
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int J = 0; J < 2; ++J) {
        if (I != J && I != Ik) continue;   // the off-diagonal tile outside the pivot's block row
        re[I][J] = __builtin_amdgcn_mfma_f32_32x32x2f32(Are[I], first[J], re[I][J], 0, 0, 0);
        im[I][J] = __builtin_amdgcn_mfma_f32_32x32x2f32(Aim[I], second[J], im[I][J], 0, 0, 0);
      }
#pragma unroll
    for (int J = 0; J < 2; ++J) pvv[J] = (32 * J + col == kk) ? pv : pvv[J];
    asm volatile("" : "+v"(pvv[0]), "+v"(pvv[1]));
  }
  tile_conj_transpose(re[1][0], im[1][0], re[0][1], im[0][1], h, col, stage);
  gj_unscale_u64(re, im, pvv, 1.f, lane, line);
}

// accumulator tiles -> lane-row layout: lane u < 32 takes column u of tile
// column 0, lane 32 + u column u of tile column 1 (conjugated into rows)
__device__ __forceinline__ void acc_to_rows_u64(const f32x16 (&re)[2][2], const f32x16 (&im)[2][2], c32 (&A)[64],
                                                int h) {
#pragma unroll
  for (int I = 0; I < 2; ++I)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m0 = 32 * I + 8 * (r / 4) + (r % 4);
      const f32pair xr = swap_halves(re[I][0][r], re[I][1][r]);
      const f32pair xi = swap_halves(im[I][0][r], im[I][1][r]);
      A[m0] = c32{xr.lo, -xi.lo};
      A[m0 + 4] = c32{xr.hi, -xi.hi};
    }
  (void)h;
}

// lane u < 32 owns entry u of H_c^H y_c, lane 32 + u entry 32 + u; e0 / e1 are
// this lane's partial sums of entries col / 32 + col over its half of the rows
__device__ __forceinline__ c32 combine_hy_u64(c32 e0, c32 e1, int h) {
  (void)h;
  const f32pair yr = swap_halves(e0.re, e1.re);
  const f32pair yi = swap_halves(e0.im, e1.im);
  return c32{yr.lo + yr.hi, yi.lo + yi.hi};
}

template <bool INVERT>
__device__ __forceinline__ c32 gram_mfma_u64(const UlArgs& a, c32 (&A)[64], int lane, int wave, float* line,
                                             float* stage) {
  const int h = lane >> 5, col = lane & 31;
  f32x16 re[2][2], im[2][2];
  c32 hy0 = cz(), hy1 = cz();
  const int ls = wave / a.Cp, c = wave % a.Cp;
  const int k = a.blk * a.sc_per_block + ls;
  const bool act = (k < a.n_sc) && (c < a.C);
  const c32* Hk = act ? a.H + (size_t)k * a.B * 64 + (size_t)c * a.S * 64 : a.H;
  const c32* yk = act ? a.y + (size_t)k * a.n_sym * a.B + (size_t)c * a.S : a.y;
#pragma unroll
  for (int I = 0; I < 2; ++I)
#pragma unroll
    for (int J = 0; J < 2; ++J) {
      re[I][J] = f32x16{};
      im[I][J] = f32x16{};
    }
  c32 x0 = cz(), x1 = cz(), yv = cz();
  // buffer loads over the problem's S rows (as in gram_mfma_u32)
  const __amdgpu_buffer_rsrc_t hrs = __builtin_amdgcn_make_buffer_rsrc(const_cast<c32*>(Hk), 0, act ? a.S * 512 : 0, kBufferWord3);
  const __amdgpu_buffer_rsrc_t yrs = __builtin_amdgcn_make_buffer_rsrc(const_cast<c32*>(yk), 0, act ? a.S * 8 : 0, kBufferWord3);
  auto fetch = [&](int s0, c32& o0, c32& o1, c32& oy) {
    const int s = s0 + h;   // row s, columns col and 32 + col: bytes 512 s + 8 col (+ 256)
    o0 = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(hrs, s * 512 + col * 8, 0, 0));
    o1 = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(hrs, s * 512 + 256 + col * 8, 0, 0));
    oy = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(yrs, s * 8, 0, 0));
  };
  fetch(0, x0, x1, yv);
  for (int s0 = 0; s0 < a.S; s0 += 2) {
    c32 n0, n1, ny;
    if (s0 + 2 < a.S) fetch(s0 + 2, n0, n1, ny);
    const c32 xs[2] = {x0, x1};
    const float ps[2] = {x0.re + x0.im, x1.re + x1.im};
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int J = 0; J < 2; ++J) {
        // with INVERT tile (1, 0) of G is never read before the inverse forms
        // it as tile (0, 1)^H, so its P^T P part is not accumulated
        if (!(INVERT && I == 1 && J == 0))
          re[I][J] = __builtin_amdgcn_mfma_f32_32x32x2f32(ps[I], ps[J], re[I][J], 0, 0, 0);        // P^T P
        im[I][J] = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[I].re, xs[J].im, im[I][J], 0, 0, 0);   // M
      }
    // entries col and 32 + col of H_c^H y_c over the rows of this lane's parity
    cmacc(hy0, x0, yv);
    cmacc(hy1, x1, yv);
    x0 = n0;
    x1 = n1;
    yv = ny;
  }
  // Tile (I, J) holds P^T P and M = Hr^T Hi restricted to rows 32 I.. and
  // columns 32 J..; Re G_IJ = (P^T P)_IJ - M_IJ - (M_JI)^T and
  // Im G_IJ = M_IJ - (M_JI)^T.  The transposes go through the wave's stage
  // buffer, one 32 x 32 tile at a time, with a row pitch of 33 as for U = 32;
  // both off-diagonal transposes are read before either off-diagonal tile
  // changes.
  auto transposed = [&](const f32x16& m, float (&out)[16]) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r / 4) + 4 * h + (r % 4);
      stage[33 * i + col] = m[r];
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r / 4) + 4 * h + (r % 4);
      out[r] = stage[33 * col + i];
    }
    wave_lds_sync();
  };
  {
    float t01[16] = {}, t10[16];
    if constexpr (!INVERT) transposed(im[0][1], t01);
    transposed(im[1][0], t10);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      re[0][1][r] -= im[0][1][r] + t10[r];
      im[0][1][r] -= t10[r];
      if (!INVERT) {
        re[1][0][r] -= im[1][0][r] + t01[r];
        im[1][0][r] -= t01[r];
      }
    }
  }
#pragma unroll
  for (int D = 0; D < 2; ++D) {
    float td[16];
    transposed(im[D][D], td);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      re[D][D][r] -= im[D][D][r] + td[r];
      im[D][D][r] -= td[r];
    }
  }
  if (INVERT) gj_invert_mfma_u64(re, im, lane, a.rho, line, stage);
  acc_to_rows_u64(re, im, A, h);
  return combine_hy_u64(hy0, hy1, h);
}

// Split-FP16 Gauss-Jordan inverse for U = 64 (four 32x32 tiles, one problem
// per wave), as gj_invert_split16_u32: the pivot row kk lives in tile row Ik,
// half hk of tiles (Ik, 0) and (Ik, 1); with the Hermitian stored matrix the
// operand a of tile row I comes from tile (Ik, I) and b of tile column J from
// tile (Ik, J), all in half hk, so each of the four tile updates is two FP16
// MFMAs built from lane-local registers.
__device__ __forceinline__ void gj_invert_split16_u64(f32x16 (&re)[2][2], f32x16 (&im)[2][2], int lane, float rho,
                                                      float post, float* line) {
  const int h = lane >> 5, col = lane & 31;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const bool dg = (8 * (r / 4) + 4 * h + (r % 4) == col);
    re[0][0][r] += dg ? rho : 0.f;
    re[1][1][r] += dg ? rho : 0.f;
  }
  float pvv[2] = {0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < 64; ++kk) {
    const int Ik = kk / 32, kr = kk % 32;
    const int rr = 4 * (kr / 8) + (kr % 4);
    const int hk = (kr / 4) & 1;
    const bool here = (h == hk);
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(re[Ik][Ik][rr]), kr + 32 * hk));
    const float pv = __builtin_amdgcn_rcpf(d);
    unsigned ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int J = 0; J < 2; ++J) {
      const bool isk = (32 * J + col == kk);
      const float t = (here && !isk) ? pv * 128.f : 0.f;
      const float mb = (here && !isk) ? 0.0078125f : 0.f;
      const float sr = re[Ik][J][rr], si = im[Ik][J][rr];
      split_f16(-sr * t, si * t, ah[J], al[J]);
      split_f16(sr * mb, si * mb, bh[J], bl[J]);
      re[Ik][J][rr] = (here && isk) ? -sr : sr;
    }
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int J = 0; J < 2; ++J) rank1_split16(re[I][J], im[I][J], ah[I], al[I], bh[J], bl[J]);
#pragma unroll
    for (int J = 0; J < 2; ++J) pvv[J] = (32 * J + col == kk) ? pv : pvv[J];
  }
  gj_unscale_u64(re, im, pvv, post, lane, line);
}

// Mixed-precision Gram for U = 64 (one problem per wave): split half-precision
// H = H_hi + H_lo after a power-of-two scaling, four 32x32 tiles on
// v_mfma_f32_32x32x16_{f16,bf16}; lane l supplies rows 8(l/32) .. 8(l/32)+7 of
// each 16-row chunk at column 32I + l%32 (A) and 32J + l%32 (B).  Then the
// Gauss-Jordan inverse on the matrix cores: FP32 (INV = 0) or split FP16 on
// the normalised Gram (INV = 2).
template <typename HT, int INV>
__device__ __forceinline__ c32 gram_inv_mixed_u64(const UlArgs& a, c32 (&A)[64], int lane, int wave,
                                                  float* line, float* stage, float& trg) {
  typedef typename HalfMma<HT>::V V;
  const int h = lane >> 5, col = lane & 31;
  const int ls = wave / a.Cp, c = wave % a.Cp;
  const int k = a.blk * a.sc_per_block + ls;
  const bool act = (k < a.n_sc) && (c < a.C);
  const c32* Hk = act ? a.H + (size_t)k * a.B * 64 + (size_t)c * a.S * 64 : a.H;
  const c32* yk = act ? a.y + (size_t)k * a.n_sym * a.B + (size_t)c * a.S : a.y;
  f32x16 re[2][2], im[2][2];
#pragma unroll
  for (int I = 0; I < 2; ++I)
#pragma unroll
    for (int J = 0; J < 2; ++J) {
      re[I][J] = f32x16{};
      im[I][J] = f32x16{};
    }
  // buffer loads over the problem's S rows (as in gram_mfma_u32)
  const __amdgpu_buffer_rsrc_t hrs = __builtin_amdgcn_make_buffer_rsrc(const_cast<c32*>(Hk), 0, act ? a.S * 512 : 0, kBufferWord3);
  const __amdgpu_buffer_rsrc_t yrs = __builtin_amdgcn_make_buffer_rsrc(const_cast<c32*>(yk), 0, act ? a.S * 8 : 0, kBufferWord3);
  // pass 1: scale exponent from the largest |Re|, |Im| (and ||H_c||_F^2 = tr(G_c))
  float mx = 0.f, ss = 0.f;
  for (int s0 = 0; s0 < a.S; s0 += 16) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int s = s0 + 8 * h + t;
      const c32 v0 = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(hrs, s * 512 + col * 8, 0, 0));
      const c32 v1 = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(hrs, s * 512 + 256 + col * 8, 0, 0));
      mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v0.re), fabsf(v0.im)), fmaxf(fabsf(v1.re), fabsf(v1.im))));
      ss = fmaf(v0.re, v0.re, fmaf(v0.im, v0.im, fmaf(v1.re, v1.re, fmaf(v1.im, v1.im, ss))));
    }
  }
  trg = wave_sum(ss);
  mx = wave_max(mx);
  int x = 0;
  if (mx > 0.f) frexpf(mx, &x);
  const int ex = 14 - x;
  c32 hy0 = cz(), hy1 = cz();
  // pass 2: split and accumulate
  for (int s0 = 0; s0 < a.S; s0 += 16) {
    V rh[2], rl[2], ih[2], il[2], nih[2], nil[2];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int s = s0 + 8 * h + t;
      const c32 yv = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(yrs, s * 8, 0, 0));
#pragma unroll
      for (int I = 0; I < 2; ++I) {
        const c32 v = __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(hrs, s * 512 + 256 * I + col * 8, 0, 0));
        cmacc(I ? hy1 : hy0, v, yv);
        const float xr = ldexpf(v.re, ex), xi = ldexpf(v.im, ex);
        const HT hr = (HT)xr, hi = (HT)xi;
        rh[I][t] = hr;
        rl[I][t] = (HT)(xr - (float)hr);
        ih[I][t] = hi;
        il[I][t] = (HT)(xi - (float)hi);
        nih[I][t] = -ih[I][t];
        nil[I][t] = -il[I][t];
      }
    }
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int J = 0; J < 2; ++J) {
        re[I][J] = HalfMma<HT>::mma(rh[I], rh[J], re[I][J]);
        re[I][J] = HalfMma<HT>::mma(rh[I], rl[J], re[I][J]);
        re[I][J] = HalfMma<HT>::mma(rl[I], rh[J], re[I][J]);
        re[I][J] = HalfMma<HT>::mma(ih[I], ih[J], re[I][J]);
        re[I][J] = HalfMma<HT>::mma(ih[I], il[J], re[I][J]);
        re[I][J] = HalfMma<HT>::mma(il[I], ih[J], re[I][J]);
        im[I][J] = HalfMma<HT>::mma(rh[I], ih[J], im[I][J]);
        im[I][J] = HalfMma<HT>::mma(rh[I], il[J], im[I][J]);
        im[I][J] = HalfMma<HT>::mma(rl[I], ih[J], im[I][J]);
        im[I][J] = HalfMma<HT>::mma(nih[I], rh[J], im[I][J]);
        im[I][J] = HalfMma<HT>::mma(nih[I], rl[J], im[I][J]);
        im[I][J] = HalfMma<HT>::mma(nil[I], rh[J], im[I][J]);
      }
  }
  const int sh = (INV == 2) ? norm_shift(a.S) : 2 * ex;
#pragma unroll
  for (int I = 0; I < 2; ++I)
#pragma unroll
    for (int J = 0; J < 2; ++J)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        re[I][J][r] = ldexpf(re[I][J][r], -sh);
        im[I][J][r] = ldexpf(im[I][J][r], -sh);
      }
  if (INV == 2)
    gj_invert_split16_u64(re, im, lane, ldexpf(a.rho, 2 * ex - sh), ldexpf(1.f, 2 * ex - sh), line);
  else
    gj_invert_mfma_u64(re, im, lane, a.rho, line, stage);
  acc_to_rows_u64(re, im, A, h);
  return combine_hy_u64(hy0, hy1, h);
}

// Consensus: every lane of cluster c writes its entry of w_c into its slot;
// after the barrier each lane sums the C clusters of its subcarrier in cluster
// order 1..C (identical sum on every cluster, as if broadcast by the fusion
// node).
// The padding clusters C..Cp-1 of a subcarrier write zeros, so with UNROLL the
// sum runs over all Cp slots (a power of two) with a fully unrolled loop;
// adding the trailing zeros leaves the value unchanged.  Without UNROLL (kernels
// whose register budget the unrolled form would cut into) it is a loop over C.
template <int N>
__device__ __forceinline__ c32 sum_slots(const c32* src, int G) {
  c32 w = src[0];
#pragma unroll
  for (int cc = 1; cc < N; ++cc) w = cadd(w, src[cc * G]);
  return w;
}

// Sum of a complex value over the P = 64 / G lane groups of a wave (lanes l,
// l ^ G, l ^ 2G, ...), the same bits on every lane: pairs of groups first,
// then pairs of pairs.  The real and imaginary parts travel together: one
// v_permlane16_swap of (re, im) leaves the pair sums of re on the even and of
// im on the odd rows of 16 lanes, one v_permlane32_swap adds the halves, and a
// last swap hands every lane both components.
template <int P>
__device__ __forceinline__ c32 wave_group_sum(c32 w) {
  if constexpr (P >= 8) w = c32{pair_sum<8>(w.re), pair_sum<8>(w.im)};
  if constexpr (P >= 4) {
    const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(w.re), __float_as_uint(w.im), false, false);
    const float s = __uint_as_float(a[0]) + __uint_as_float(a[1]);   // rows: re01 im01 re23 im23
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(s), __float_as_uint(s), false, false);
    const float t = __uint_as_float(b[0]) + __uint_as_float(b[1]);   // rows: re im re im (totals)
    const auto c = __builtin_amdgcn_permlane16_swap(__float_as_uint(t), __float_as_uint(t), false, false);
    return c32{__uint_as_float(c[0]), __uint_as_float(c[1])};
  } else {
    const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(w.re), __float_as_uint(w.im), false, false);
    const float s = __uint_as_float(a[0]) + __uint_as_float(a[1]);   // halves: re | im
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(s), __float_as_uint(s), false, false);
    return c32{__uint_as_float(b[0]), __uint_as_float(b[1])};
  }
}

template <bool UNROLL = true>
__device__ __forceinline__ c32 consensus(c32 wc, int buf, int ls, int G, int u, int C, int Cp, const Smem& sm,
                                         int slot, int nw) {
  c32* cb = sm.cons + buf * nw * 64;
  cb[slot] = wc;
  __syncthreads();
  const c32* src = cb + (size_t)ls * Cp * G + u;
  if (!UNROLL) {
    c32 w = cz();
    for (int cc = 0; cc < C; ++cc) w = cadd(w, src[cc * G]);
    return w;
  }
  switch (Cp) {
    case 1: return src[0];
    case 2: return sum_slots<2>(src, G);
    case 4: return sum_slots<4>(src, G);
    case 8: return sum_slots<8>(src, G);
    default: return sum_slots<16>(src, G);
  }
}

// The consensus of the lane-group layout with P = 64 / G problems per wave.
// When the padded cluster count Cp is at least P, the wave's P problems are
// clusters P j .. P j + P - 1 of one subcarrier: their vectors are summed in
// registers first (pairs of lanes l, l ^ G, then l, l ^ 2G, ...: the same
// tree on every lane, so every lane holds the same bits), and only the
// first group of each wave writes its slot; the readers then add Cp / P
// slots in cluster order.  Otherwise, as consensus().
template <int G>
__device__ __forceinline__ c32 consensus_w(c32 wc, int buf, int ls, int u, int g, int C, int Cp, const Smem& sm,
                                           int slot, int nw) {
  constexpr int P = 64 / G;
  if constexpr (P == 1) {
    (void)g;
    return consensus<true>(wc, buf, ls, G, u, C, Cp, sm, slot, nw);
  } else {
    if (Cp < P) return consensus<true>(wc, buf, ls, G, u, C, Cp, sm, slot, nw);
    const c32 w = wave_group_sum<P>(wc);
    c32* cb = sm.cons + buf * nw * 64;
    if (g == 0) cb[slot] = w;
    __syncthreads();
    const c32* src = cb + (size_t)ls * Cp * G + u;
    switch (Cp / P) {
      case 1: return src[0];
      case 2: return sum_slots<2>(src, P * G);
      case 4: return sum_slots<4>(src, P * G);
      default: return sum_slots<8>(src, P * G);
    }
  }
}

// ---------------------------------------------------------------------------
// Algorithm 1, U x U branch (S >= U), FP32.  Group size G = U.
// ---------------------------------------------------------------------------
// HALF: 0 FP32 Gram, 1 / 2 split FP16 / BF16 Gram (mixed modes, U = 32, 64).
// INV (mixed modes): 0 FP32 matrix-core inverse, 1 FP64 VALU inverse (U = 32),
// 2 split-FP16 matrix-core inverse.
// STAGE: 0 preprocessing and iterations; 1 preprocessing only, B_c^{-1} is
// written to a.fac (a static channel factored once); 2 iterations only, B_c^{-1}
// read from a.fac (every symbol's H_c^H y_c by the VALU pass); 3 as 2 with H
// read from the packed FP16 channel; 4 (U = 32, FP32) as 1, and H also
// written as the packed FP16 channel in the same launch.
template <int G, int HALF, int INV, int STAGE>
__device__ __forceinline__ void admm_ul_body(const UlArgs& a);

template <int G, int HALF, int INV, int STAGE>
__global__ void __launch_bounds__(512) admm_ul_f32(UlArgs a) {
  a.blk = blockIdx.x;
  admm_ul_body<G, HALF, INV, STAGE>(a);
}

// Several frames of the same U in one persistent launch (FP32, one-shot):
// frame f owns the virtual blocks first[f] .. first[f+1]-1 of its own launch
// plan (all frames share the waves per workgroup); each workgroup takes
// virtual blocks in grid stride and finds its frame by binary search over
// first[].  The frames' argument blocks travel in the kernel arguments.
template <int G>
__global__ void __launch_bounds__(512) admm_ul_f32_batch(UlBatch b) {
  for (int vb = blockIdx.x; vb < b.first[b.n]; vb += gridDim.x) {
    int lo = 0, hi = b.n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (b.first[mid] <= vb) lo = mid;
      else hi = mid - 1;
    }
    UlArgs a = b.f[lo];
    a.blk = vb - b.first[lo];
    admm_ul_body<G, 0, 0, 0>(a);
    __syncthreads();   // the next virtual block reuses the LDS
  }
}

template <int G, int HALF, int INV, int STAGE>
__device__ __forceinline__ void admm_ul_body(const UlArgs& a) {
  constexpr int P = 64 / G;
  constexpr bool RESIDENT = (STAGE == 2 || STAGE == 3);   // iterations against stored factors
  constexpr bool FACTOR = (STAGE == 1 || STAGE == 4);     // preprocessing only
  extern __shared__ float4 smem_raw[];
  const int nw = blockDim.x >> 6;
  Smem sm = carve(reinterpret_cast<c32*>(smem_raw), nw);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: addresses in SALU
  const int g = lane / G, u = lane % G;
  const int lp = wave * P + g;
  const int ls = lp / a.Cp, c = lp % a.Cp;
  const int k = a.blk * a.sc_per_block + ls;
  const bool active = (k < a.n_sc) && (c < a.C);
  const int slot = wave * 64 + lane;
  c32* line = sm.line + wave * 64;
  const int gbase = g * G;

  // Preprocessing (Alg. 1, S > U branch): B_c = H_c^H H_c + rho I, B_c^{-1}.
  c32 A[G];
  // (the U = 16 Gram and the U = 32 factor staging write every entry of every
  // lane's row: no clearing)
  if constexpr (!(G == 16 && !RESIDENT) && !(G == 32 && RESIDENT)) {
#pragma unroll
    for (int v = 0; v < G; ++v) A[v] = cz();
  }
  c32 hy0 = cz();
  float trg = 0.f;   // tr(G_c) (mixed modes)
  // U = 16 and 32, FP32, iterations in the same launch: the inverse keeps its lazy
  // scales (B^{-1} = 2 D - D S D, D = diag(pv): off the diagonal
  // -S_uv pv_u pv_v), which every product applies to its operand and result
  // instead of to the U x U entries.
  constexpr bool LAZY = ((G == 32 || G == 16) && HALF == 0 && STAGE == 0);
  float pvl = 1.f;
  auto bmat = [&](c32 q) -> c32 {
    if constexpr (LAZY) {
      // (the sweeps leave the diagonal un-negated: + 2 pv_u q_u)
      const c32 r = group_matvec<G>(A, cscale(q, pvl), u, line, gbase);
      const float tp = 2.f * pvl;
      return c32{fmaf(tp, q.re, -pvl * r.re), fmaf(tp, q.im, -pvl * r.im)};
    } else {
      return group_matvec<G>(A, q, u, line, gbase);
    }
  };
  // Resident factors of this problem: B_c^{-1} is Hermitian, so only its
  // upper triangle is stored, column by column (entry (i, v), i <= v, at
  // v (v + 1) / 2 + i; G (G + 1) / 2 values per problem).  Lane u's row
  // takes entry v from column v (v >= u) or, conjugated, from column u
  // (v < u): one load per entry, coalesced over the lanes of the first kind.
  constexpr int NT = G * (G + 1) / 2;
  const size_t fo = ((size_t)k * a.C + c) * NT;
  if constexpr (RESIDENT && G == 32) {
    // The lanes of the other kind would read 32 different cache lines per
    // load, so each problem's triangle (NT = 528 values, the size of the
    // wave's stage buffer) first goes through LDS with 16-byte coalesced
    // loads, one problem of the wave at a time.  Both candidate entries are
    // inside the triangle for every (u, v) (indices at most NT - 1), so each
    // lane reads both and keeps one.
    // Both problems' factor loads are issued first, and symbol 0's
    // H_c^H y_c is formed while they are in flight.
    c32* tri = sm.stage + wave * kStageWave;
    const int csu = u * (u + 1) / 2;
    constexpr int NQ = (NT / 2 + 63) / 64;
    float4 tq[P][NQ];
    bool tv[P];
#pragma unroll
    for (int pp = 0; pp < P; ++pp) {
      const int lq = wave * P + pp;
      const int kq = a.blk * a.sc_per_block + lq / a.Cp, cq = lq % a.Cp;
      tv[pp] = kq < a.n_sc && cq < a.C;
      // a buffer load over the problem's NT entries (none when inactive):
      // the range check zeroes the slots past the triangle without selects
      const __amdgpu_buffer_rsrc_t frs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<c32*>(a.fac + (tv[pp] ? ((size_t)kq * a.C + cq) * NT : 0)), 0, tv[pp] ? NT * 8 : 0, kBufferWord3);
#pragma unroll
      for (int i = 0; i < NQ; ++i)
        tq[pp][i] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(frs, (i * 64 + lane) * 16, 0, 0));
    }
    if constexpr (STAGE == 3)
      hy0 = cluster_hy_direct<G, true>(a, k, c, 0, u, active);
    else
      hy0 = cluster_pass<G, false>(a.H, a.y, A, k, c, 0, u, g, lane, wave, active, a.B, a.S, G, a.n_sym, sm);
#pragma unroll
    for (int pp = 0; pp < P; ++pp) {
      if (tv[pp]) {
        float4* dst = reinterpret_cast<float4*>(tri);
#pragma unroll
        for (int i = 0; i < NQ; ++i)
          if (i * 64 + lane < NT / 2) dst[i * 64 + lane] = tq[pp][i];
      }
      wave_lds_sync();
      // (an inactive problem reads whatever the buffer holds; its results
      // are never stored)
      if (g == pp) {
#pragma unroll
        for (int v = 0; v < G; ++v) {
          const c32 e1 = tri[v * (v + 1) / 2 + u];   // entry (u, v), v >= u
          const c32 e2 = tri[csu + v];               // entry (v, u), v < u
          A[v] = (v >= u) ? e1 : c32{e2.re, -e2.im};
        }
      }
      wave_lds_sync();
    }
  } else if constexpr (RESIDENT) {
    if (active) {
      const int csu = u * (u + 1) / 2;
#pragma unroll
      for (int v = 0; v < G; ++v) {
        const bool up = v >= u;
        const c32 e = a.fac[fo + (up ? (size_t)(v * (v + 1) / 2 + u) : (size_t)(csu + v))];
        A[v] = up ? e : c32{e.re, -e.im};
      }
    }
  } else if constexpr (G == 32 && HALF == 0) {
    hy0 = gram_mfma_u32<true, LAZY, FACTOR, STAGE == 4>(a, A, lane, wave, reinterpret_cast<float*>(line),
                                    reinterpret_cast<float*>(sm.stage + wave * kStageWave), &pvl);
  } else if constexpr (G == 32 && HALF == 1) {
    hy0 = gram_inv_mixed_u32<_Float16, INV>(a, A, lane, wave, reinterpret_cast<c64*>(sm.stage + wave * kStageWave),
                                            trg);
  } else if constexpr (G == 32 && HALF == 2) {
    hy0 = gram_inv_mixed_u32<__bf16, INV>(a, A, lane, wave, reinterpret_cast<c64*>(sm.stage + wave * kStageWave),
                                          trg);
  } else if constexpr (G == 16) {
    if constexpr (LAZY) {
      hy0 = gram_mfma_u16<true, true>(a, A, lane, wave, sm.stage + wave * kStageWave, &pvl);
    } else {
      hy0 = gram_mfma_u16<true>(a, A, lane, wave, sm.stage + wave * kStageWave);
      gj_invert<G>(A, u, line, gbase);
    }
  } else if constexpr (G == 64 && HALF == 0) {
    hy0 = gram_mfma_u64<true>(a, A, lane, wave, reinterpret_cast<float*>(line),
                              reinterpret_cast<float*>(sm.stage + wave * kStageWave));
  } else if constexpr (G == 64 && HALF == 1) {
    hy0 = gram_inv_mixed_u64<_Float16, INV>(a, A, lane, wave, reinterpret_cast<float*>(line),
                                            reinterpret_cast<float*>(sm.stage + wave * kStageWave), trg);
  } else if constexpr (G == 64 && HALF == 2) {
    hy0 = gram_inv_mixed_u64<__bf16, INV>(a, A, lane, wave, reinterpret_cast<float*>(line),
                                          reinterpret_cast<float*>(sm.stage + wave * kStageWave), trg);
  } else {
    hy0 = cluster_pass<G, true>(a.H, a.y, A, k, c, 0, u, g, lane, wave, active, a.B, a.S, G, a.n_sym, sm);
#pragma unroll
    for (int v = 0; v < G; ++v)
      if (v == u) A[v].re += a.rho;
    gj_invert<G>(A, u, line, gbase);
  }
  if constexpr (FACTOR && G == 32) {
    // Through the wave's stage buffer, one problem at a time, then 16-byte
    // coalesced stores.  Lane u writes entry v of its row to v (v + 1) / 2 + u
    // for every v in increasing order: for v >= u that is entry (u, v) of the
    // triangle; for v < u the position belongs to a later column w > v, whose
    // own write (step w, lane u') comes after it and replaces it.  Every
    // position is inside the triangle (at most NT - 1).
    c32* tri = sm.stage + wave * kStageWave;
#pragma unroll
    for (int pp = 0; pp < P; ++pp) {
      if (g == pp) {
#pragma unroll
        for (int v = 0; v < G; ++v) tri[v * (v + 1) / 2 + u] = A[v];
      }
      wave_lds_sync();
      const int lq = wave * P + pp;
      const int kq = a.blk * a.sc_per_block + lq / a.Cp, cq = lq % a.Cp;
      if (kq < a.n_sc && cq < a.C) {
        float4* dst = reinterpret_cast<float4*>(a.fac + ((size_t)kq * a.C + cq) * NT);
        const float4* src = reinterpret_cast<const float4*>(tri);
#pragma unroll
        for (int i = 0; i < (NT / 2 + 63) / 64; ++i)
          if (i * 64 + lane < NT / 2) dst[i * 64 + lane] = src[i * 64 + lane];
      }
      wave_lds_sync();
    }
    return;
  } else if constexpr (FACTOR) {
    if (active) {
#pragma unroll
      for (int v = 0; v < G; ++v)
        if (v >= u) a.fac[fo + (size_t)(v * (v + 1) / 2 + u)] = A[v];
    }
    return;
  }

  // FP64 factor rule (mixed modes, FP32 inverse): kappa_hat = tr(B_c)
  // ||B_c^{-1}||_F bounds the condition number kappa_2(B_c) from above (the
  // largest eigenvalue is at most the trace, and ||B_c^{-1}||_2 at most the
  // Frobenius norm).  A subcarrier with a cluster above cond_max goes to the
  // FP64 pass.  Below it the FP32 error grows in proportion to the
  // conditioning, so the re-slice guard is widened by kappa_hat / cond_ref
  // (cond_ref: the largest kappa_hat of the channels the guard was measured
  // on).  Each problem's kappa_hat reaches the output lanes of cluster 0
  // through one LDS slot, read after the first consensus barrier.
  constexpr bool COND = (HALF > 0 && INV == 0 && STAGE == 0);
  float* cond_slot = reinterpret_cast<float*>(sm.aux);
  float guard = a.guard;
  if constexpr (COND) {
    if (a.cond_max != 0.f) {
      float f2 = 0.f;
#pragma unroll
      for (int v = 0; v < G; ++v) f2 = fmaf(A[v].re, A[v].re, fmaf(A[v].im, A[v].im, f2));
      f2 = group_sum<G>(f2);
      const float kh = (trg + (float)G * a.rho) * sqrtf(f2);
      if (u == 0) cond_slot[ls * a.Cp + c] = active ? kh : 0.f;
    }
  }

  int buf = 0;
  int fl = 0;   // status bits of this lane's outputs (bit 0 non-finite, bit 1 re-slice, bit 2 ill-conditioned)
  for (int n = 0; n < a.n_sym; ++n) {
    c32 hy = hy0;
    // (with U = 32 factors, symbol 0's H_c^H y_c was formed with the factor loads)
    constexpr bool HY0 = (RESIDENT && G == 32);
    if constexpr (STAGE == 3) {
      if (!HY0 || n > 0) hy = cluster_hy_direct<G, true>(a, k, c, n, u, active);
    } else if (n > 0 || (STAGE == 2 && !HY0)) {
      hy = cluster_pass<G, false>(a.H, a.y, A, k, c, n, u, g, lane, wave, active, a.B, a.S, G, a.n_sym, sm);
    }
    // y_c^reg = B_c^{-1} H_c^H y_c; z = y^reg; lambda = 0
    const c32 yreg = bmat(hy);
    c32 z = yreg, lam = cz();
    c32 w = (HALF == 0) ? consensus_w<G>(active ? z : cz(), buf, ls, u, g, a.C, a.Cp, sm, slot, nw)
                        : consensus<false>(active ? z : cz(), buf, ls, G, u, a.C, a.Cp, sm, slot, nw);
    buf ^= 1;
    if constexpr (COND) {
      // the barrier inside the consensus above has made every cluster's estimate visible
      if (n == 0 && a.cond_max != 0.f && c == 0) {
        float km = 0.f;
        bool bad = a.cond_max < 0.f;
        for (int cc = 0; cc < a.C; ++cc) {
          const float kc = cond_slot[ls * a.Cp + cc];
          bad = bad || !(kc <= a.cond_max);   // NaN and infinity fail the comparison
          km = fmaxf(km, kc);
        }
        if (bad) fl |= kStatusReslice | kStatusIllcond;
        guard = a.guard * fmaxf(1.f, km / a.cond_ref);
      }
    }
    c32 s;
    if (a.reg == 2) {
      c32 v = cscale(w, a.invC);
      s = c32{fminf(fmaxf(v.re, -a.box_r), a.box_r), fminf(fmaxf(v.im, -a.box_r), a.box_r)};
    } else {
      s = cscale(w, a.inv_den);
    }
    for (int t = 2; t <= a.T; ++t) {
      lam.re = fmaf(a.gamma, z.re - s.re, lam.re);
      lam.im = fmaf(a.gamma, z.im - s.im, lam.im);
      const c32 q = csub(s, lam);
      const c32 bq = bmat(q);
      z = c32{fmaf(a.rho, bq.re, yreg.re), fmaf(a.rho, bq.im, yreg.im)};
      w = (HALF == 0) ? consensus_w<G>(active ? cadd(z, lam) : cz(), buf, ls, u, g, a.C, a.Cp, sm, slot, nw)
                      : consensus<false>(active ? cadd(z, lam) : cz(), buf, ls, G, u, a.C, a.Cp, sm, slot, nw);
      buf ^= 1;
      if (a.reg == 2) {
        c32 v = cscale(w, a.invC);
        s = c32{fminf(fmaxf(v.re, -a.box_r), a.box_r), fminf(fmaxf(v.im, -a.box_r), a.box_r)};
      } else {
        s = cscale(w, a.inv_den);
      }
    }
    if (active && c == 0) {
      const size_t o = ((size_t)k * a.n_sym + n) * G + u;
      a.shat[o] = s;
      if (a.hard) {
        const int iI = slice_dim(s.re, a.kappa, a.L), iQ = slice_dim(s.im, a.kappa, a.L);
        a.hard[o] = (uint8_t)(iI + a.L * iQ);
        if (near_threshold(s.re, a.kappa, a.L, guard) || near_threshold(s.im, a.kappa, a.L, guard)) fl |= 2;
      }
      if (nonfinite(s)) fl |= 1;
    }
  }
  if (a.flags) {
    const int bits = group_flags<G>(fl, g);
    if (c == 0 && u == 0 && k < a.n_sc) {
      a.flags[k] = bits;
      if ((bits & kStatusReslice) && a.any) *a.any = a.epoch;
    }
  }
}

// ---------------------------------------------------------------------------
// Algorithm 2 (decentralized CG), FP32.  Each cluster keeps its own copy of
// x, r, p (the broadcast-w variant) and contributes w_c = H_c^H H_c p through
// its local Gram G_c held in registers (one matvec per iteration).
// ---------------------------------------------------------------------------
template <int G>
__global__ void __launch_bounds__(512) dcg_ul_f32(UlArgs a) {
  a.blk = blockIdx.x;
  constexpr int P = 64 / G;
  extern __shared__ float4 smem_raw[];
  const int nw = blockDim.x >> 6;
  Smem sm = carve(reinterpret_cast<c32*>(smem_raw), nw);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: addresses in SALU
  const int g = lane / G, u = lane % G;
  const int lp = wave * P + g;
  const int ls = lp / a.Cp, c = lp % a.Cp;
  const int k = a.blk * a.sc_per_block + ls;
  const bool active = (k < a.n_sc) && (c < a.C);
  const int slot = wave * 64 + lane;
  c32* line = sm.line + wave * 64;
  const int gbase = g * G;

  c32 A[G];
  // (the U = 16 Gram writes every entry of every lane's row: no clearing)
  if constexpr (G != 16) {
#pragma unroll
    for (int v = 0; v < G; ++v) A[v] = cz();
  }
  c32 hy0;
  if constexpr (G == 32)
    hy0 = gram_mfma_u32<false>(a, A, lane, wave, reinterpret_cast<float*>(line),
                               reinterpret_cast<float*>(sm.stage + wave * kStageWave));
  else if constexpr (G == 16)
    hy0 = gram_mfma_u16(a, A, lane, wave, sm.stage + wave * kStageWave);
  else if constexpr (G == 64)
    hy0 = gram_mfma_u64<false>(a, A, lane, wave, reinterpret_cast<float*>(line),
                               reinterpret_cast<float*>(sm.stage + wave * kStageWave));
  else
    hy0 = cluster_pass<G, true>(a.H, a.y, A, k, c, 0, u, g, lane, wave, active, a.B, a.S, G, a.n_sym, sm);

  int buf = 0;
  int fl = 0;   // status bits of this lane's outputs (bit 0 non-finite, bit 1 re-slice)
  for (int n = 0; n < a.n_sym; ++n) {
    c32 hy = hy0;
    if (n > 0) hy = cluster_pass<G, false>(a.H, a.y, A, k, c, n, u, g, lane, wave, active, a.B, a.S, G, a.n_sym, sm);
    // y^MRC = sum_c H_c^H y_c (consensus); r = p = y^MRC; x = 0
    c32 r = consensus_w<G>(active ? hy : cz(), buf, ls, u, g, a.C, a.Cp, sm, slot, nw);
    buf ^= 1;
    c32 pv = r, x = cz();
    float rr = group_sum<G>(r.re * r.re + r.im * r.im);
    for (int t = 1; t <= a.T; ++t) {
      const c32 wc = group_matvec<G>(A, pv, u, line, gbase);
      const c32 w = consensus_w<G>(active ? wc : cz(), buf, ls, u, g, a.C, a.Cp, sm, slot, nw);
      buf ^= 1;
      const c32 e = c32{fmaf(a.rho, pv.re, w.re), fmaf(a.rho, pv.im, w.im)};
      const float pe = group_sum<G>(pv.re * e.re + pv.im * e.im);
      // quotients by the hardware reciprocal (1 ulp) instead of a full division
      const float alpha = (rr > 0.f) ? rr * __builtin_amdgcn_rcpf(pe) : 0.f;
      x.re = fmaf(alpha, pv.re, x.re);
      x.im = fmaf(alpha, pv.im, x.im);
      r.re = fmaf(-alpha, e.re, r.re);
      r.im = fmaf(-alpha, e.im, r.im);
      const float rr_new = group_sum<G>(r.re * r.re + r.im * r.im);
      const float beta = (rr > 0.f) ? rr_new * __builtin_amdgcn_rcpf(rr) : 0.f;
      pv.re = fmaf(beta, pv.re, r.re);
      pv.im = fmaf(beta, pv.im, r.im);
      rr = rr_new;
    }
    if (active && c == 0) {
      const size_t o = ((size_t)k * a.n_sym + n) * G + u;
      a.shat[o] = x;
      if (a.hard) {
        const int iI = slice_dim(x.re, a.kappa, a.L), iQ = slice_dim(x.im, a.kappa, a.L);
        a.hard[o] = (uint8_t)(iI + a.L * iQ);
        if (near_threshold(x.re, a.kappa, a.L, a.guard) || near_threshold(x.im, a.kappa, a.L, a.guard)) fl |= 2;
      }
      if (nonfinite(x)) fl |= 1;
    }
  }
  if (a.flags) {
    const int bits = group_flags<G>(fl, g);
    if (c == 0 && u == 0 && k < a.n_sc) {
      a.flags[k] = bits;
      if ((bits & kStatusReslice) && a.any) *a.any = a.epoch;
    }
  }
}

// Newton steps of the budgeted (P1) at most (quadratic convergence from
// below: about four to six steps reach FP32 accuracy).
constexpr int kBudgetNewton = 12;

// ---------------------------------------------------------------------------
// Algorithm 3 (decentralized ADMM beamforming, epsilon = 0), S x S branch
// (S <= U), FP32.  Group size G = U.  The downlink cluster channel is
// H_c = (Hu_c)^T with Hu_c the S x U uplink block (reciprocity), read in place
// from the uplink layout.  Lane u holds column u of Hu_c (entries Hu_c[a][u],
// a < S) for m_c = H_c x_c; lane a < S holds row a of Hu_c for H_c^H v and
// row a of A_c^{-1}.
// ---------------------------------------------------------------------------
// BUDGET: every x-update is the budgeted step (P1) with ||x_c||^2 <= P_c.
// When the unconstrained step exceeds the budget, x = (H_c^H H_c + tau I)^{-1}
// H_c^H v with tau > 1/rho the root of ||x(tau)|| = sqrt(P_c) (the Lagrange
// multiplier of the budget is rho tau - 1): Newton's method on
// 1/||x(tau)|| - 1/sqrt(P_c), which is concave and increasing in tau, so the
// iterates from tau = 1/rho rise monotonically to the root (the trust-region
// update tau += ||x||^2 (||x|| - sqrt(P)) / (sqrt(P) x^H (G + tau I)^{-1} x)).
// Each step forms the Gram again and inverts the shifted matrix.
template <int G, int SG, bool BUDGET = false>
__device__ __forceinline__ void admm_dl_body(const DlArgs& a) {
  constexpr int P = 64 / G;
  extern __shared__ float4 smem_raw[];
  const int nw = blockDim.x >> 6;
  Smem sm = carve(reinterpret_cast<c32*>(smem_raw), nw);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: addresses in SALU
  const int g = lane / G, u = lane % G;
  const int lp = wave * P + g;
  const int ls = lp / a.Cp, c = lp % a.Cp;
  const int k = blockIdx.x * a.sc_per_block + ls;
  const bool active = (k < a.n_sc) && (c < a.C);
  const int slot = wave * 64 + lane;
  c32* line = sm.line + wave * 64;
  const int gbase = g * G;
  const int S = a.S;
  // Entry (a, u) of the S x U uplink block Hu_c: row-major in the uplink
  // layout [n_sc][B][U] (strides U and 1), or read from the downlink layout
  // H^d [n_sc][U][B] (strides 1 and B).
  const bool dl_layout = a.h_layout == 1;
  const c32* Hk = a.H + (size_t)k * a.B * G + (dl_layout ? (size_t)c * S : (size_t)c * S * G);
  const size_t sa = dl_layout ? 1 : G, su = dl_layout ? (size_t)a.B : 1;

  // When SG = G / 2 the row of Hu_c that H_c^H v needs is split over two
  // lanes: lane u holds entries RS * (u / SG) .. + RS - 1 of row u % SG, and
  // the two half sums are combined by one exchange.  Otherwise lane u < S
  // holds the whole row u.
  constexpr bool SPLIT = (2 * SG == G);
  constexpr int RS = SPLIT ? SG : G;       // row entries held per lane
  const int ra = SPLIT ? (u % SG) : u;     // row of Hu_c held by this lane
  const int r0 = SPLIT ? RS * (u / SG) : 0;
  // With the matrix-core Gram (U = 32, S <= 16) the row copy hrow is formed
  // only after the inverse, from hcol through LDS, so that it is not live
  // during the Gram and the sweep (register budget of four waves per SIMD).
  constexpr bool LATE_H = (G == 32 && SG == 16);
  // There (without the budget) A_c and its inverse also take the split-row
  // layout: lane u holds entries 8 (u / 16) .. + 7 of row u % 16, so that all
  // 32 lanes of the group share the sweep and the products A_c^{-1} r.
  constexpr bool ASPLIT = LATE_H && !BUDGET;
  c32 hcol[SG], hrow[RS], A[ASPLIT ? 8 : SG];
#pragma unroll
  for (int i = 0; i < SG; ++i) hcol[i] = (active && i < S) ? Hk[(size_t)i * sa + (size_t)u * su] : cz();
#pragma unroll
  for (int i = 0; i < (ASPLIT ? 8 : SG); ++i) A[i] = cz();
  if constexpr (!LATE_H) {
#pragma unroll
    for (int i = 0; i < RS; ++i) hrow[i] = (active && ra < S) ? Hk[(size_t)ra * sa + (size_t)(r0 + i) * su] : cz();
  }
  // The Gram H_c^H H_c, (H_c^H H_c)[a][b] = sum_u conj(Hu[a][u]) Hu[b][u], into
  // M (rows a < S; M must hold zeros).  Every lane of the wave takes part.
  auto gram_into = [&](c32 (&M)[SG]) {
    if constexpr (LATE_H) {
      gram_dl_mfma_s16_u32<false>(hcol, M, lane, g, u, sm.stage + wave * kStageWave);
    } else {
      // Row b of Hu_c is broadcast from the stage buffer of this wave.
      c32* stage = sm.stage + wave * kStageWave;
      for (int b = 0; b < S; ++b) {
        // lane u of the group publishes Hu[b][u] = hcol[b]
        c32 hb = cz();
#pragma unroll
        for (int i = 0; i < SG; ++i)
          if (i == b) hb = hcol[i];
        stage[lane] = hb;
        wave_lds_sync();
        c32 acc = cz();
#pragma unroll
        for (int v0 = 0; v0 < RS; v0 += 8) {
          c32 row[8];
          lds_read_vec<8>(stage + gbase + r0 + v0, row);
#pragma unroll
          for (int v = 0; v < 8; ++v) cmacc(acc, hrow[v0 + v], row[v]);
        }
        wave_lds_sync();
        if (SPLIT) acc = c32{pair_sum<SG>(acc.re), pair_sum<SG>(acc.im)};
#pragma unroll
        for (int i = 0; i < SG; ++i)
          if (i == b) M[i] = (u < S) ? acc : cz();
      }
    }
  };
  // A_c = H_c^H H_c + rho^{-1} I_S
  const float irho = 1.0f / a.rho;
  if constexpr (ASPLIT) {
    gram_dl_mfma_s16_u32<true>(hcol, A, lane, g, u, sm.stage + wave * kStageWave);
    const int h = u >> 4, r = u & 15;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (8 * h + i == r) A[i].re += (r < S) ? irho : 1.0f;
    gj_invert_sym_split16(A, r, h, line + gbase);
  } else {
    gram_into(A);
#pragma unroll
    for (int v = 0; v < SG; ++v)
      if (v == u) A[v].re += (u < S) ? irho : 1.0f;
    gj_invert<SG>(A, u, line, gbase);
  }
  if constexpr (LATE_H) {
    // Transpose the S x G tile of each problem through the wave's stage
    // buffer, one problem at a time: entry (i, w) at i (G + 2) + w.  The
    // pitch of G + 2 complex values keeps column pairs together and 16-byte
    // aligned, puts the rows that a read instruction touches into different
    // LDS banks, and makes every offset a compile-time constant
    // (SG (G + 2) = 544 values, the size of the stage buffer).
    c32* tile = sm.stage + wave * kStageWave;
    static_assert(SG * (G + 2) <= kStageWave, "tile exceeds the stage buffer");
    for (int pp = 0; pp < P; ++pp) {
      if (g == pp) {
#pragma unroll
        for (int i = 0; i < SG; ++i) tile[i * (G + 2) + u] = hcol[i];
      }
      wave_lds_sync();
      if (g == pp) {
#pragma unroll
        for (int m = 0; m < RS / 2; ++m) {
          const float4 v = *reinterpret_cast<const float4*>(tile + ra * (G + 2) + r0 + 2 * m);
          hrow[2 * m] = c32{v.x, v.y};
          hrow[2 * m + 1] = c32{v.z, v.w};
        }
      }
      wave_lds_sync();
    }
  }

  // Broadcast line of the iterations, in the wave's stage buffer (free once
  // the Gram is formed): group g at g (G + 8), and with split rows the second
  // half of a group 4 entries further on, so that the (up to four) distinct
  // 16-byte addresses a read instruction touches fall into different LDS
  // banks.
  c32* bl = sm.stage + wave * kStageWave + g * (G + 8);
  const int bw = u + (SPLIT ? 4 * (u / RS) : 0);      // this lane's slot
  const int br = r0 + (SPLIT ? 4 * (r0 / RS) : 0);    // start of the half this lane reads
  int buf = 0;
  for (int n = 0; n < a.n_sym; ++n) {
    const size_t vo = ((size_t)k * a.n_sym + n);
    const c32 s = (k < a.n_sc) ? a.s[vo * G + u] : cz();
    c32 z = cscale(s, a.f0), lam = cz();
    // H_c^H v: entry a held by lane a < S
    auto hhv = [&](c32 v) -> c32 {
      c32 acc = cz();
      if constexpr (ASPLIT) {
        // entry r0 + i of v sits in lane i of this lane's own 16-lane DPP row:
        // broadcast inside the FMAs, no LDS
        acc = matvec16c(hrow, v);
      } else {
        bl[bw] = v;
        wave_lds_sync();
#pragma unroll
        for (int v0 = 0; v0 < RS; v0 += 4) {
          c32 vv[4];
          lds_read_vec<4>(bl + br + v0, vv);
#pragma unroll
          for (int i = 0; i < 4; ++i) cmacc(acc, hrow[v0 + i], vv[i]);
        }
        wave_lds_sync();
      }
      if (SPLIT) acc = c32{pair_sum<SG>(acc.re), pair_sum<SG>(acc.im)};
      // the split-row product below takes entry a from both lanes of row a
      if constexpr (ASPLIT) return (ra < S) ? acc : cz();
      return (u < S) ? acc : cz();
    };
    // x_c = A_c^{-1} H_c^H (z + lambda), entry a held by lane a < S.  At
    // S = U (SG = G) the regularised Gram is as poorly conditioned as it gets
    // (condition numbers of a few hundred at S = U = 64), and the FP32 Gram
    // and Gauss-Jordan inverse lose about a factor three against an exactly
    // rounded solve there; one step of refinement whose residual is formed
    // from H itself, r - H_c^H (H_c x) - x / rho, wins it back.
    auto apply = [&](c32 v) -> c32 {
      const c32 r = hhv(v);
      // entry a of x_c on lane a < S (with the split rows, on both lanes of row a)
      c32 xa;
      if constexpr (ASPLIT)
        xa = matvec_split16(A, r);
      else
        xa = group_matvec<SG>(A, r, u, line, gbase);
      if constexpr (SG == G) {
        bl[bw] = xa;
        wave_lds_sync();
        c32 m = cz();
#pragma unroll
        for (int v0 = 0; v0 < SG; v0 += 4) {
          c32 xv[4];
          lds_read_vec<4>(bl + v0, xv);
#pragma unroll
          for (int i = 0; i < 4; ++i) cmac(m, hcol[v0 + i], xv[i]);
        }
        wave_lds_sync();
        const c32 q = hhv(m);
        const c32 res = (u < S) ? c32{fmaf(-irho, xa.re, r.re - q.re), fmaf(-irho, xa.im, r.im - q.im)} : cz();
        xa = cadd(xa, group_matvec<SG>(A, res, u, line, gbase));
      }
      if constexpr (BUDGET) {
        // padding cluster slots carry no budget
        const float Pc = active ? a.P[c] : 0.f;
        const float e = group_sum<G>((u < S) ? xa.re * xa.re + xa.im * xa.im : 0.f);
        const bool need = active && e > Pc;
        if (__ballot(need)) {   // wave-uniform: the Gram and sweep below are wave operations
          const float sp = sqrtf(Pc);
          float tau = irho, et = e;
          c32 xn = xa;
          for (int it = 0; it < kBudgetNewton; ++it) {
            c32 Mt[SG];
#pragma unroll
            for (int v = 0; v < SG; ++v) Mt[v] = cz();
            gram_into(Mt);
#pragma unroll
            for (int v = 0; v < SG; ++v)
              if (v == u) Mt[v].re += (u < S) ? tau : 1.0f;
            gj_invert<SG>(Mt, u, line, gbase);
            xn = group_matvec<SG>(Mt, r, u, line, gbase);
            const c32 mx = group_matvec<SG>(Mt, xn, u, line, gbase);
            et = group_sum<G>((u < S) ? xn.re * xn.re + xn.im * xn.im : 0.f);
            const float w2 = group_sum<G>((u < S) ? xn.re * mx.re + xn.im * mx.im : 0.f);
            const float sq = sqrtf(et);
            const bool go = need && sq - sp > 1e-6f * sp && w2 > 0.f;
            if (go) tau += et * (sq - sp) / (sp * w2);
            if (!__ballot(go)) break;
          }
          // the last iterate lies on the budget up to rounding; a final
          // scale keeps it feasible
          if (need) xa = (et > Pc) ? cscale(xn, sqrtf(Pc / et)) : xn;
        }
      }
      return xa;
    };
    c32 x = apply(z);
    for (int t = 2; t <= a.T; ++t) {
      // m_c = H_c x_c: m[u] = sum_a Hu[a][u] x[a]
      c32 m = cz();
      if constexpr (ASPLIT) {
        // x[a] sits in lane a of both 16-lane DPP rows of the group
        m = matvec16(hcol, x);
      } else {
        bl[bw] = x;
        wave_lds_sync();
#pragma unroll
        for (int v0 = 0; v0 < SG; v0 += 4) {
          c32 xv[4];
          lds_read_vec<4>(bl + v0, xv);
#pragma unroll
          for (int i = 0; i < 4; ++i) cmac(m, hcol[v0 + i], xv[i]);
        }
        wave_lds_sync();
      }
      const c32 wc = csub(m, lam);
      const c32 w = consensus_w<G>(active ? wc : cz(), buf, ls, u, g, a.C, a.Cp, sm, slot, nw);
      buf ^= 1;
      // Lemma 2: z_c = w_c + f (s - w) / C, f = max{0, 1 - eps / ||s - w||}
      // (f = 1 at eps = 0); every group holds the same s and w, one user per lane
      float fC = a.invC;
      if (a.eps > 0.f) {
        const float dre = s.re - w.re, dim = s.im - w.im;
        const float nd = sqrtf(group_sum<G>(dre * dre + dim * dim));
        fC = nd > a.eps ? a.invC * (1.0f - a.eps / nd) : 0.f;
      }
      z = c32{fmaf(fC, s.re - w.re, wc.re), fmaf(fC, s.im - w.im, wc.im)};
      lam.re = fmaf(-a.gamma, m.re - z.re, lam.re);
      lam.im = fmaf(-a.gamma, m.im - z.im, lam.im);
      x = apply(cadd(z, lam));
    }
    // optional common power scaling: beta = min(1, min_c sqrt(P_c / ||x_c||^2))
    // (with the budgeted step the budgets are met by every x-update instead)
    float beta = 1.0f;
    if (a.P && !BUDGET) {
      const float e = group_sum<G>((u < S) ? (x.re * x.re + x.im * x.im) : 0.f);
      float ratio = 1.0f;
      if (active && e > 0.f) ratio = fminf(1.0f, sqrtf(a.P[c] / e));
      c32* ab = sm.aux;
      if (u == 0) ab[wave * 64 + g] = c32{ratio, 0.f};
      __syncthreads();
      // problems of subcarrier ls occupy local problem indices ls*Cp .. ls*Cp+C-1
      for (int cc = 0; cc < a.C; ++cc) {
        const int q = ls * a.Cp + cc;
        beta = fminf(beta, ab[(q / P) * 64 + (q % P)].re);
      }
      __syncthreads();
    }
    if (active && u < S) a.x[vo * a.B + (size_t)c * S + u] = cscale(x, beta);
    if (active && c == 0 && u == 0 && a.beta) a.beta[vo] = beta;
  }
}

template <int G, int SG, bool BUDGET = false>
__global__ void __launch_bounds__(512) admm_dl_f32(DlArgs a) {
  admm_dl_body<G, SG, BUDGET>(a);
}

// The same with the register budget of four waves per SIMD: at B = 256,
// U = 32, C = 16 a subcarrier's workgroup has eight waves, and 128 VGPRs let
// two such workgroups share a CU instead of one.
template <int G, int SG>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) admm_dl_f32_w4(DlArgs a) {
  admm_dl_body<G, SG>(a);
}

// ---------------------------------------------------------------------------
// Packed FP16 channel: one 256-lane workgroup per (subcarrier, cluster) tile
// of S x U entries.  The tile's largest |component| m fixes the exponent
// e = floor(log2 m) - 14 (at least -126), so that the scaled entries H * 2^-e
// lie below 2^15 in magnitude (no overflow) and stay normal FP16 numbers (11
// significant bits) down to 2^-28 m; each entry is rounded to nearest even, and
// 2^e is stored as the tile's scale.  Tiles of up to 256 * kPackRegs entries
// stay in registers between the two steps (one read of H); larger tiles read
// the tile a second time.
// ---------------------------------------------------------------------------
constexpr int kPackRegs = 8;


__global__ void __launch_bounds__(256) pack_h16(const c32* __restrict__ H, uint32_t* __restrict__ H16,
                                                float* __restrict__ hscale, int B, int U, int C) {
  __shared__ float wmax[4];
  const int S = B / C;
  const int k = blockIdx.x / C, c = blockIdx.x % C;
  const size_t base = (size_t)k * B * U + (size_t)c * S * U;
  const int n = S * U;
  const bool cached = n <= 256 * kPackRegs;
  c32 r[kPackRegs];
  float m = 0.f;
  if (cached) {
#pragma unroll
    for (int j = 0; j < kPackRegs; ++j) {
      const int i = threadIdx.x + 256 * j;
      r[j] = i < n ? H[base + i] : cz();
      m = fmaxf(m, fmaxf(fabsf(r[j].re), fabsf(r[j].im)));
    }
  } else {
    for (int i = threadIdx.x; i < n; i += 256) {
      const c32 v = H[base + i];
      m = fmaxf(m, fmaxf(fabsf(v.re), fabsf(v.im)));
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  m = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
  const int e = pack_exponent(m);
  if (cached) {
#pragma unroll
    for (int j = 0; j < kPackRegs; ++j) {
      const int i = threadIdx.x + 256 * j;
      if (i < n) H16[base + i] = pack_pair(r[j], e);
    }
  } else {
    for (int i = threadIdx.x; i < n; i += 256) H16[base + i] = pack_pair(H[base + i], e);
  }
  if (threadIdx.x == 0) hscale[blockIdx.x] = ldexpf(1.f, e);
}

// ---------------------------------------------------------------------------
// Per-subcarrier status: one 256-lane workgroup per subcarrier ORs "not
// finite" over the subcarrier's floats and writes the flag (every entry of
// the status array is written, so it needs no clearing).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) scan_nonfinite(const float* __restrict__ x, size_t per_sc,
                                                      int32_t* __restrict__ status) {
  const float* p = x + (size_t)blockIdx.x * per_sc;
  int bad = 0;
  for (size_t i = threadIdx.x; i < per_sc; i += 256) bad |= !__builtin_isfinite(p[i]);
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) status[blockIdx.x] = bad ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename K, typename Args>
static hipError_t launch(K kernel, const Args& a, int nw, hipStream_t st) {
  const int nblocks = (a.n_sc + a.sc_per_block - 1) / a.sc_per_block;
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(kernel, dim3(nblocks), dim3(64 * nw), smem_bytes(nw), st, a);
  return hipGetLastError();
}

template <int G, int HALF, int INV>
static hipError_t launch_stage(const UlArgs& a, int nw, hipStream_t st, int stage) {
  return stage == 1 ? launch(admm_ul_f32<G, HALF, INV, 1>, a, nw, st) : launch(admm_ul_f32<G, HALF, INV, 0>, a, nw, st);
}

hipError_t launch_factor_pack_u32(const UlArgs& a, int nw, hipStream_t st) {
  return launch(admm_ul_f32<32, 0, 0, 4>, a, nw, st);
}

hipError_t launch_admm_ul_f32(const UlArgs& a, int U, int nw, hipStream_t st, int stage) {
  switch (U) {
    case 8: return launch_stage<8, 0, 0>(a, nw, st, stage);
    case 16: return launch_stage<16, 0, 0>(a, nw, st, stage);
    case 32: return launch_stage<32, 0, 0>(a, nw, st, stage);
    case 64: return launch_stage<64, 0, 0>(a, nw, st, stage);
  }
  return hipErrorInvalidValue;
}

template <int G, int HALF>
static hipError_t launch_mixed_inv(const UlArgs& a, int inv, int nw, hipStream_t st, int stage) {
  switch (inv) {
    case 0: return launch_stage<G, HALF, 0>(a, nw, st, stage);
    case 2: return launch_stage<G, HALF, 2>(a, nw, st, stage);
  }
  if constexpr (G == 32) {
    if (inv == 1) return launch_stage<G, HALF, 1>(a, nw, st, stage);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_admm_ul_mixed(const UlArgs& a, int U, int half, int inv, int nw, hipStream_t st, int stage) {
  if (U == 32)
    return half == 1 ? launch_mixed_inv<32, 1>(a, inv, nw, st, stage) : launch_mixed_inv<32, 2>(a, inv, nw, st, stage);
  if (U == 64)
    return half == 1 ? launch_mixed_inv<64, 1>(a, inv, nw, st, stage) : launch_mixed_inv<64, 2>(a, inv, nw, st, stage);
  return hipErrorInvalidValue;
}

hipError_t launch_admm_ul_f32_batch(const UlBatch& b, int U, int nw, int grid, hipStream_t st) {
  if (b.n < 1 || b.first[b.n] == 0) return hipSuccess;
  const dim3 g((unsigned)grid), blk((unsigned)(64 * nw));
  switch (U) {
    case 8: hipLaunchKernelGGL(admm_ul_f32_batch<8>, g, blk, smem_bytes(nw), st, b); break;
    case 16: hipLaunchKernelGGL(admm_ul_f32_batch<16>, g, blk, smem_bytes(nw), st, b); break;
    case 32: hipLaunchKernelGGL(admm_ul_f32_batch<32>, g, blk, smem_bytes(nw), st, b); break;
    case 64: hipLaunchKernelGGL(admm_ul_f32_batch<64>, g, blk, smem_bytes(nw), st, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_admm_ul_factored(const UlArgs& a, int U, int nw, hipStream_t st) {
  switch (U) {
    case 8: return launch(admm_ul_f32<8, 0, 0, 2>, a, nw, st);
    case 16: return launch(admm_ul_f32<16, 0, 0, 2>, a, nw, st);
    case 32: return launch(admm_ul_f32<32, 0, 0, 2>, a, nw, st);
    case 64: return launch(admm_ul_f32<64, 0, 0, 2>, a, nw, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_admm_ul_factored_h16(const UlArgs& a, int U, int nw, hipStream_t st) {
  switch (U) {
    case 8: return launch(admm_ul_f32<8, 0, 0, 3>, a, nw, st);
    case 16: return launch(admm_ul_f32<16, 0, 0, 3>, a, nw, st);
    case 32: return launch(admm_ul_f32<32, 0, 0, 3>, a, nw, st);
    case 64: return launch(admm_ul_f32<64, 0, 0, 3>, a, nw, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pack_h16(const c32* H, uint32_t* H16, float* hscale, int n_sc, int B, int U, int C,
                           hipStream_t st) {
  const size_t tiles = (size_t)n_sc * C;
  if (tiles == 0) return hipSuccess;
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pack_h16, dim3((unsigned)tiles), dim3(256), 0, st, H, H16, hscale, B, U, C);
  return hipGetLastError();
}

hipError_t launch_scan_nonfinite(const float* x, size_t floats_per_sc, int n_sc, int32_t* status,
                                 hipStream_t st) {
  if (n_sc == 0) return hipSuccess;
  hipLaunchKernelGGL(scan_nonfinite, dim3((unsigned)n_sc), dim3(256), 0, st, x, floats_per_sc, status);
  return hipGetLastError();
}

hipError_t launch_dcg_ul_f32(const UlArgs& a, int U, int nw, hipStream_t st) {
  switch (U) {
    case 8: return launch(dcg_ul_f32<8>, a, nw, st);
    case 16: return launch(dcg_ul_f32<16>, a, nw, st);
    case 32: return launch(dcg_ul_f32<32>, a, nw, st);
    case 64: return launch(dcg_ul_f32<64>, a, nw, st);
  }
  return hipErrorInvalidValue;
}

template <bool BUDGET>
static hipError_t launch_dl(const DlArgs& a, int U, int nw, hipStream_t st) {
  const int S = a.S;
  switch (U) {
    case 8: return launch(admm_dl_f32<8, 8, BUDGET>, a, nw, st);
    case 16:
      return S <= 8 ? launch(admm_dl_f32<16, 8, BUDGET>, a, nw, st) : launch(admm_dl_f32<16, 16, BUDGET>, a, nw, st);
    case 32:
      if (S <= 8) return launch(admm_dl_f32<32, 8, BUDGET>, a, nw, st);
      if (S <= 16) {
        // the budgeted form keeps a second S x S matrix live: no 128-register cap
        if constexpr (BUDGET) return launch(admm_dl_f32<32, 16, true>, a, nw, st);
        return launch(admm_dl_f32_w4<32, 16>, a, nw, st);
      }
      return launch(admm_dl_f32<32, 32, BUDGET>, a, nw, st);
    case 64:
      if (S <= 8) return launch(admm_dl_f32<64, 8, BUDGET>, a, nw, st);
      if (S <= 16) return launch(admm_dl_f32<64, 16, BUDGET>, a, nw, st);
      if (S <= 32) return launch(admm_dl_f32<64, 32, BUDGET>, a, nw, st);
      return launch(admm_dl_f32<64, 64, BUDGET>, a, nw, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_admm_dl_f32(const DlArgs& a, int U, int nw, hipStream_t st) {
  return (a.P && a.budget) ? launch_dl<true>(a, U, nw, st) : launch_dl<false>(a, U, nw, st);
}

}  // namespace dbp
