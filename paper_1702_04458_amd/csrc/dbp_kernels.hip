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
//   stage[nw][kStageRows][64]   staged H rows (one slot per lane)
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
  s.ystage = s.stage + nw * kStageRows * 64;
  s.line = s.ystage + nw * kStageRows * 8;
  s.cons = s.line + nw * 64;
  s.aux = s.cons + 2 * nw * 64;
  return s;
}

size_t smem_bytes(int nw) { return sizeof(c32) * (size_t)nw * (kStageRows * 64 + kStageRows * 8 + 64 + 128 + 64); }

// One pass over the S rows of H_c (and of y_c for symbol n): accumulates the
// Gram row A[v] += conj(H[s][u]) H[s][v] when WITH_GRAM, and always
// hy = sum_s conj(H[s][u]) y[s] (row u of H_c^H y_c).
template <int G, bool WITH_GRAM>
__device__ __forceinline__ c32 cluster_pass(const c32* __restrict__ H, const c32* __restrict__ y, c32 (&A)[G],
                                            int k, int c, int n, int u, int g, int lane, int wave, bool active,
                                            int B, int S, int U, int n_sym, const Smem& sm) {
  constexpr int R = kStageRows;
  c32 hy = cz();
  c32* stage = sm.stage + wave * R * 64;
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

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Regularised inverse on the matrix cores, for the two Gram matrices of a wave
// held in the 32x32 accumulator layout (lane l: column l%32, rows
// 8(r/4) + 4(l/32) + r%4).  Gauss-Jordan elimination of the HPD matrix
// B = G + rho I, where every pivot step k is a complex rank-1 update
// S -= m (x) row_k, issued as two v_mfma_f32_32x32x2f32 (real part with
// operands [-Re m, Im m] x [Re row; Im row], imaginary part with
// [-Re m, -Im m] x [Im row; Re row]).  The multipliers m_i = B[i][k] / B[k][k]
// come from row k through the signed Hermitian symmetry of the partially swept
// matrix (entry (i, k) is the conjugate of entry (k, i), negated when exactly
// one of i, k has been swept).  The swept pivot column is not rewritten: each
// column carries a scale factor sigma_j (true = stored * sigma_j), and the new
// column k is the old one times -1/B[k][k], so only sigma_k changes.  Row k is
// rescaled in place.  The result is multiplied out by sigma at the end.
__device__ __forceinline__ void gj_invert_mfma_u32(f32x16 (&re)[2], f32x16 (&im)[2], int lane, float rho) {
  const int h = lane >> 5, col = lane & 31;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 8 * (r / 4) + 4 * h + (r % 4);
    const float add = (i == col) ? rho : 0.f;
    re[0][r] += add;
    re[1][r] += add;
  }
  const float hs = h ? 1.f : -1.f;
  float sig[2] = {1.f, 1.f};
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const int rr = 4 * (k / 8) + (k % 4);   // register holding row k
    const int hk = (k / 4) & 1;             // lane half holding row k
    const bool isk = (col == k);
    const bool rowk_here = (h == hk);
    // multiplier sign: -1 for swept rows (col < k), 0 for the pivot row itself
    const float f = (col < k) ? -1.f : (isk ? 0.f : 1.f);
    const float mk = isk ? 0.f : 1.f;
    const float g = (rowk_here && isk) ? -1.f : 0.f;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const float sr = re[p][rr], si = im[p][rr];
      // row k at column col, arranged for the operands: lanes < 32 get
      // (first, second) = (Re, Im), lanes >= 32 get (Im, Re)
      const auto fs = __builtin_amdgcn_permlane32_swap(__float_as_uint(sr), __float_as_uint(si), false, false);
      const auto sf = __builtin_amdgcn_permlane32_swap(__float_as_uint(si), __float_as_uint(sr), false, false);
      const float first = __uint_as_float(fs[hk]);
      const float second = __uint_as_float(sf[hk]);
      const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sr), k + 32 * hk));
      const float pv = __builtin_amdgcn_rcpf(d);
      const float c = f * pv * sig[p];          // m_col = c * conj(stored row k entry)
      const float Are = -c * first;             // lanes < 32: -Re m, lanes >= 32: Im m
      const float Aim = (hs * c) * first;       // lanes < 32: -Re m, lanes >= 32: -Im m
      const float Bre = mk * first, Bim = mk * second;
      // row k <- row k / B[k][k]; the diagonal becomes 1/B[k][k], stored as -1
      // under sigma_k = -1/B[k][k]
      const float fr = rowk_here ? pv * mk : 1.f;
      re[p][rr] = fmaf(sr, fr, g);
      im[p][rr] = si * fr;
      re[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(Are, Bre, re[p], 0, 0, 0);
      im[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(Aim, Bim, im[p], 0, 0, 0);
      sig[p] = isk ? -pv : sig[p];
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      re[p][r] *= sig[p];
      im[p][r] *= sig[p];
    }
  }
}

// Gram matrices of the two problems of a wave (U = 32, P = 2) on the matrix
// cores with v_mfma_f32_32x32x2f32, K running over pairs of antenna rows:
//   Re G = sum_s Hr[s]^T Hr[s] + Hi[s]^T Hi[s],
//   Im G = sum_s Hr[s]^T Hi[s] - Hi[s]^T Hr[s].
// For the Gram of one problem lane l supplies H[s0 + l/32][l%32] as both the A
// and the B operand.  The 32x32 result leaves lane l holding column l%32 for
// rows 8(r/4) + 4(l/32) + r%4 (r = 0..15); by Hermitian symmetry that is row
// l%32 conjugated, for half h = l/32 of the columns.  With INVERT the
// accumulators are replaced by (G + rho I)^{-1} on the matrix cores first.
// One exchange between lanes l and l^32 then gives every lane the full row of
// its own problem (lane-row layout, problem = l/32).  Returns row u of
// H_c^H y_c for symbol 0.
template <bool INVERT>
__device__ __forceinline__ c32 gram_mfma_u32(const UlArgs& a, c32 (&A)[32], int lane, int wave) {
  const int h = lane >> 5, col = lane & 31;
  f32x16 re[2], im[2];
  c32 hyp[2];
  const c32* Hp[2];
  const c32* yp[2];
  bool act[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int lp = wave * 2 + p;
    const int ls = lp / a.Cp, c = lp % a.Cp;
    const int k = blockIdx.x * a.sc_per_block + ls;
    act[p] = (k < a.n_sc) && (c < a.C);
    Hp[p] = a.H + (size_t)k * a.B * 32 + (size_t)c * a.S * 32;
    yp[p] = a.y + (size_t)k * a.n_sym * a.B + (size_t)c * a.S;
    re[p] = f32x16{};
    im[p] = f32x16{};
    hyp[p] = cz();
  }
  // Software pipeline: the loads of the next CH row pairs are in flight while
  // the MFMAs of the current ones run.
  constexpr int CH = DBP_PREFETCH_U32;
  c32 hv[2][CH], yv[2][CH], hn[2][CH], yn[2][CH];
  auto fetch = [&](int s0, c32 (&hd)[2][CH], c32 (&yd)[2][CH]) {
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int s = s0 + 2 * q + h;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const bool ok = act[p] && s < a.S;
        hd[p][q] = ok ? Hp[p][(size_t)s * 32 + col] : cz();
        yd[p][q] = ok ? yp[p][s] : cz();
      }
    }
  };
  fetch(0, hv, yv);
  for (int s0 = 0; s0 < a.S; s0 += 2 * CH) {
    if (s0 + 2 * CH < a.S) fetch(s0 + 2 * CH, hn, yn);
#pragma unroll
    for (int q = 0; q < CH; ++q) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const c32 x = hv[p][q];
        re[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(x.re, x.re, re[p], 0, 0, 0);
        re[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(x.im, x.im, re[p], 0, 0, 0);
        im[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(x.re, x.im, im[p], 0, 0, 0);
        im[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(-x.im, x.re, im[p], 0, 0, 0);
        cmacc(hyp[p], x, yv[p][q]);
      }
    }
#pragma unroll
    for (int q = 0; q < CH; ++q)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        hv[p][q] = hn[p][q];
        yv[p][q] = yn[p][q];
      }
  }
  if (INVERT) gj_invert_mfma_u32(re, im, lane, a.rho);
  // exchange halves: lanes < 32 keep problem 0, lanes >= 32 keep problem 1
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m0 = 8 * (r / 4) + (r % 4);      // column of this slot in half 0
    const float sr = h ? re[0][r] : re[1][r];
    const float si = h ? im[0][r] : im[1][r];
    const float tr = __shfl_xor(sr, 32, 64);
    const float ti = __shfl_xor(si, 32, 64);
    const float h0r = h ? tr : re[0][r], h0i = h ? ti : im[0][r];
    const float h1r = h ? re[1][r] : tr, h1i = h ? im[1][r] : ti;
    A[m0] = c32{h0r, -h0i};
    A[m0 + 4] = c32{h1r, -h1i};
  }
  const c32 send = h ? hyp[0] : hyp[1];
  const c32 got = c32{__shfl_xor(send.re, 32, 64), __shfl_xor(send.im, 32, 64)};
  const c32 mine = h ? hyp[1] : hyp[0];
  // rows of parity 0 first, then parity 1 (same order on every lane)
  return h ? cadd(got, mine) : cadd(mine, got);
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

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

template <typename HT>
__device__ __forceinline__ void gram_split_u32(const UlArgs& a, f32x16 (&re)[2], f32x16 (&im)[2], c32 (&hyp)[2],
                                               int lane, int wave) {
  typedef typename HalfMma<HT>::V V;
  const int h = lane >> 5, col = lane & 31;
  const c32* Hp[2];
  const c32* yp[2];
  bool act[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int lp = wave * 2 + p;
    const int ls = lp / a.Cp, c = lp % a.Cp;
    const int k = blockIdx.x * a.sc_per_block + ls;
    act[p] = (k < a.n_sc) && (c < a.C);
    Hp[p] = a.H + (size_t)k * a.B * 32 + (size_t)c * a.S * 32;
    yp[p] = a.y + (size_t)k * a.n_sym * a.B + (size_t)c * a.S;
    re[p] = f32x16{};
    im[p] = f32x16{};
    hyp[p] = cz();
  }
  // pass 1: largest |Re|, |Im| of each problem -> scale exponent
  int ex[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    float m = 0.f;
    for (int s0 = 0; s0 < a.S; s0 += 16) {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int s = s0 + 8 * h + t;
        const c32 v = (act[p] && s < a.S) ? Hp[p][(size_t)s * 32 + col] : cz();
        m = fmaxf(m, fmaxf(fabsf(v.re), fabsf(v.im)));
      }
    }
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
        const bool ok = act[p] && s < a.S;
        v[t] = ok ? Hp[p][(size_t)s * 32 + col] : cz();
        const c32 yv = ok ? yp[p][s] : cz();
        cmacc(hyp[p], v[t], yv);
      }
      V rh, rl, ih, il, nih, nil;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float xr = ldexpf(v[t].re, ex[p]), xi = ldexpf(v[t].im, ex[p]);
        const HT hr = (HT)xr, hi = (HT)xi;
        rh[t] = hr;
        rl[t] = (HT)(xr - (float)hr);
        ih[t] = hi;
        il[t] = (HT)(xi - (float)hi);
        nih[t] = -ih[t];
        nil[t] = -il[t];
      }
      // Re G = Hr^T Hr + Hi^T Hi
      re[p] = HalfMma<HT>::mma(rh, rh, re[p]);
      re[p] = HalfMma<HT>::mma(rh, rl, re[p]);
      re[p] = HalfMma<HT>::mma(rl, rh, re[p]);
      re[p] = HalfMma<HT>::mma(ih, ih, re[p]);
      re[p] = HalfMma<HT>::mma(ih, il, re[p]);
      re[p] = HalfMma<HT>::mma(il, ih, re[p]);
      // Im G = Hr^T Hi - Hi^T Hr
      im[p] = HalfMma<HT>::mma(rh, ih, im[p]);
      im[p] = HalfMma<HT>::mma(rh, il, im[p]);
      im[p] = HalfMma<HT>::mma(rl, ih, im[p]);
      im[p] = HalfMma<HT>::mma(nih, rh, im[p]);
      im[p] = HalfMma<HT>::mma(nih, rl, im[p]);
      im[p] = HalfMma<HT>::mma(nil, rh, im[p]);
    }
  }
#pragma unroll
  for (int p = 0; p < 2; ++p) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      re[p][r] = ldexpf(re[p][r], -2 * ex[p]);
      im[p][r] = ldexpf(im[p][r], -2 * ex[p]);
    }
  }
}

// Accumulator layout -> lane-row layout (lanes < 32: problem 0, >= 32: problem 1)
__device__ __forceinline__ void acc_to_rows_u32(const f32x16 (&re)[2], const f32x16 (&im)[2], c32 (&A)[32], int h) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m0 = 8 * (r / 4) + (r % 4);
    const float sr = h ? re[0][r] : re[1][r];
    const float si = h ? im[0][r] : im[1][r];
    const float tr = __shfl_xor(sr, 32, 64);
    const float ti = __shfl_xor(si, 32, 64);
    const float h0r = h ? tr : re[0][r], h0i = h ? ti : im[0][r];
    const float h1r = h ? re[1][r] : tr, h1i = h ? im[1][r] : ti;
    A[m0] = c32{h0r, -h0i};
    A[m0 + 4] = c32{h1r, -h1i};
  }
}

__device__ __forceinline__ c32 combine_hy(const c32 (&hyp)[2], int h) {
  const c32 send = h ? hyp[0] : hyp[1];
  const c32 got = c32{__shfl_xor(send.re, 32, 64), __shfl_xor(send.im, 32, 64)};
  const c32 mine = h ? hyp[1] : hyp[0];
  return h ? cadd(got, mine) : cadd(mine, got);
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

// Mixed-precision Gram + regularised inverse for U = 32; returns row u of
// H_c^H y_c and leaves row u of (G + rho I)^{-1} in A.
template <typename HT, bool F64>
__device__ __forceinline__ c32 gram_inv_mixed_u32(const UlArgs& a, c32 (&A)[32], int lane, int wave, c64* line64) {
  const int h = lane >> 5;
  f32x16 re[2], im[2];
  c32 hyp[2];
  gram_split_u32<HT>(a, re, im, hyp, lane, wave);
  if (!F64) {
    gj_invert_mfma_u32(re, im, lane, a.rho);
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
// antenna rows: lane l supplies H[s0 + l/16][l%16] as both operands.  The
// 16x16 result leaves lane l holding column l%16 for rows 4(l/16) + r
// (r = 0..3) of every problem; by Hermitian symmetry that is row l%16
// conjugated, columns 4(l/16) .. 4(l/16)+3.  An LDS transpose (two problems
// per pass through the wave's stage buffer) gives lane 16p + u the full row u
// of problem p.  Returns row u of H_c^H y_c for symbol 0.
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ c32 gram_mfma_u16(const UlArgs& a, c32 (&A)[16], int lane, int wave, c32* stage) {
  const int q = lane >> 4, col = lane & 15;
  f32x4 re[4], im[4];
  c32 hyp[4];
  const c32* Hp[4];
  const c32* yp[4];
  bool act[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int lp = wave * 4 + p;
    const int ls = lp / a.Cp, c = lp % a.Cp;
    const int k = blockIdx.x * a.sc_per_block + ls;
    act[p] = (k < a.n_sc) && (c < a.C);
    Hp[p] = a.H + (size_t)k * a.B * 16 + (size_t)c * a.S * 16;
    yp[p] = a.y + (size_t)k * a.n_sym * a.B + (size_t)c * a.S;
    re[p] = f32x4{};
    im[p] = f32x4{};
    hyp[p] = cz();
  }
  constexpr int CH = DBP_PREFETCH_U16;   // row quadruples per prefetch chunk
  c32 hv[4][CH], yv[4][CH], hn[4][CH], yn[4][CH];
  auto fetch = [&](int s0, c32 (&hd)[4][CH], c32 (&yd)[4][CH]) {
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int s = s0 + 4 * j + q;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const bool ok = act[p] && s < a.S;
        hd[p][j] = ok ? Hp[p][(size_t)s * 16 + col] : cz();
        yd[p][j] = ok ? yp[p][s] : cz();
      }
    }
  };
  fetch(0, hv, yv);
  for (int s0 = 0; s0 < a.S; s0 += 4 * CH) {
    if (s0 + 4 * CH < a.S) fetch(s0 + 4 * CH, hn, yn);
#pragma unroll
    for (int j = 0; j < CH; ++j) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const c32 x = hv[p][j];
        re[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.re, x.re, re[p], 0, 0, 0);
        re[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.im, x.im, re[p], 0, 0, 0);
        im[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.re, x.im, im[p], 0, 0, 0);
        im[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(-x.im, x.re, im[p], 0, 0, 0);
        cmacc(hyp[p], x, yv[p][j]);
      }
    }
#pragma unroll
    for (int j = 0; j < CH; ++j)
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        hv[p][j] = hn[p][j];
        yv[p][j] = yn[p][j];
      }
  }
  // transpose through LDS: buf[pp][q'][r][col], two problems per pass
#pragma unroll
  for (int half = 0; half < 2; ++half) {
#pragma unroll
    for (int pp = 0; pp < 2; ++pp)
#pragma unroll
      for (int r = 0; r < 4; ++r) stage[((pp * 4 + q) * 4 + r) * 16 + col] = c32{re[2 * half + pp][r], im[2 * half + pp][r]};
    wave_lds_sync();
    if ((q >> 1) == half) {
      const int pp = q & 1;
#pragma unroll
      for (int qq = 0; qq < 4; ++qq)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const c32 v = stage[((pp * 4 + qq) * 4 + r) * 16 + col];
          A[4 * qq + r] = c32{v.re, -v.im};
        }
    }
    wave_lds_sync();
  }
  // H_c^H y_c: sum the four row classes (lanes col, col+16, col+32, col+48)
  c32 out = cz();
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    float hr = hyp[p].re, hi = hyp[p].im;
    hr += __shfl_xor(hr, 16, 64);
    hi += __shfl_xor(hi, 16, 64);
    hr += __shfl_xor(hr, 32, 64);
    hi += __shfl_xor(hi, 32, 64);
    if (p == q) out = c32{hr, hi};
  }
  return out;
}

// Downlink S x S Gram A_c[a][b] = sum_u conj(Hu[a][u]) Hu[b][u] (S <= 16,
// U = 32 users as the contraction index, two problems per wave) on the matrix
// cores with v_mfma_f32_16x16x4f32: lane l supplies Hu[l%16][u0 + l/16] as
// both operands.  The 16x16 result (lane l: column l%16, rows 4(l/16)+r) goes
// through the wave's stage buffer so that lane b < 16 of each problem's lane
// group reads row b.
__device__ __forceinline__ void gram_dl_mfma_s16_u32(const DlArgs& a, c32 (&A)[16], int lane, int wave, c32* stage) {
  const int q = lane >> 4, r16 = lane & 15;
  f32x4 re[2], im[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int lp = wave * 2 + p;
    const int ls = lp / a.Cp, c = lp % a.Cp;
    const int k = blockIdx.x * a.sc_per_block + ls;
    const bool act = (k < a.n_sc) && (c < a.C) && (r16 < a.S);
    const c32* Hk = a.H + (size_t)k * a.B * 32 + (size_t)c * a.S * 32 + (size_t)r16 * 32 + q;
    c32 x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = act ? Hk[4 * j] : cz();
    re[p] = f32x4{};
    im[p] = f32x4{};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      re[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[j].re, x[j].re, re[p], 0, 0, 0);
      re[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[j].im, x[j].im, re[p], 0, 0, 0);
      im[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[j].re, x[j].im, im[p], 0, 0, 0);
      im[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(-x[j].im, x[j].re, im[p], 0, 0, 0);
    }
  }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int r = 0; r < 4; ++r) stage[p * 256 + (4 * q + r) * 16 + r16] = c32{re[p][r], im[p][r]};
  wave_lds_sync();
  const int p = lane >> 5, b = lane & 31;
  if (b < 16) {
#pragma unroll
    for (int v0 = 0; v0 < 16; v0 += 8) {
      c32 row[8];
      lds_read_vec<8>(stage + p * 256 + b * 16 + v0, row);
#pragma unroll
      for (int v = 0; v < 8; ++v) A[v0 + v] = row[v];
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
// pivot issued on all four tiles and one column scale per tile column.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gj_invert_mfma_u64(f32x16 (&re)[2][2], f32x16 (&im)[2][2], int lane, float rho) {
  const int h = lane >> 5, col = lane & 31;
  // B = G + rho I
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 8 * (r / 4) + 4 * h + (r % 4);
    const float add = (i == col) ? rho : 0.f;
    re[0][0][r] += add;
    re[1][1][r] += add;
  }
  const float hs = h ? 1.f : -1.f;
  float sig[2] = {1.f, 1.f};
#pragma unroll
  for (int kk = 0; kk < 64; ++kk) {
    const int Ik = kk / 32, kr = kk % 32;
    const int rr = 4 * (kr / 8) + (kr % 4);
    const int hk = (kr / 4) & 1;
    const bool rowk_here = (h == hk);
    float first[2], second[2], Sr0[2], Si0[2];
#pragma unroll
    for (int J = 0; J < 2; ++J) {
      const float sr = re[Ik][J][rr], si = im[Ik][J][rr];
      Sr0[J] = sr;
      Si0[J] = si;
      const auto fs = __builtin_amdgcn_permlane32_swap(__float_as_uint(sr), __float_as_uint(si), false, false);
      const auto sf = __builtin_amdgcn_permlane32_swap(__float_as_uint(si), __float_as_uint(sr), false, false);
      first[J] = __uint_as_float(fs[hk]);
      second[J] = __uint_as_float(sf[hk]);
    }
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Sr0[Ik]), kr + 32 * hk));
    const float pv = __builtin_amdgcn_rcpf(d);
    float Are[2], Aim[2], Bre[2], Bim[2], mk[2];
#pragma unroll
    for (int J = 0; J < 2; ++J) {
      const int cidx = 32 * J + col;   // global index of this lane in tile column / row J
      const float f = (cidx < kk) ? -1.f : (cidx == kk ? 0.f : 1.f);
      mk[J] = (cidx == kk) ? 0.f : 1.f;
      const float cc = f * pv * sig[J];
      Are[J] = -cc * first[J];
      Aim[J] = (hs * cc) * first[J];
      Bre[J] = mk[J] * first[J];
      Bim[J] = mk[J] * second[J];
    }
#pragma unroll
    for (int J = 0; J < 2; ++J) {
      const bool isk = (32 * J + col == kk);
      const float fr = rowk_here ? pv * mk[J] : 1.f;
      const float g = (rowk_here && isk) ? -1.f : 0.f;
      re[Ik][J][rr] = fmaf(Sr0[J], fr, g);
      im[Ik][J][rr] = Si0[J] * fr;
    }
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int J = 0; J < 2; ++J) {
        re[I][J] = __builtin_amdgcn_mfma_f32_32x32x2f32(Are[I], Bre[J], re[I][J], 0, 0, 0);
        im[I][J] = __builtin_amdgcn_mfma_f32_32x32x2f32(Aim[I], Bim[J], im[I][J], 0, 0, 0);
      }
#pragma unroll
    for (int J = 0; J < 2; ++J) sig[J] = (32 * J + col == kk) ? -pv : sig[J];
  }
#pragma unroll
  for (int r = 0; r < 16; ++r)
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int J = 0; J < 2; ++J) {
        re[I][J][r] *= sig[J];
        im[I][J][r] *= sig[J];
      }
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
      const float sr = h ? re[I][0][r] : re[I][1][r];
      const float si = h ? im[I][0][r] : im[I][1][r];
      const float tr = __shfl_xor(sr, 32, 64);
      const float ti = __shfl_xor(si, 32, 64);
      const float h0r = h ? tr : re[I][0][r], h0i = h ? ti : im[I][0][r];
      const float h1r = h ? re[I][1][r] : tr, h1i = h ? im[I][1][r] : ti;
      A[m0] = c32{h0r, -h0i};
      A[m0 + 4] = c32{h1r, -h1i};
    }
}

// lane u < 32 owns entry u of H_c^H y_c, lane 32 + u entry 32 + u; e0 / e1 are
// this lane's partial sums of entries col / 32 + col over its half of the rows
__device__ __forceinline__ c32 combine_hy_u64(c32 e0, c32 e1, int h) {
  const c32 send = h ? e0 : e1;
  const c32 got = c32{__shfl_xor(send.re, 32, 64), __shfl_xor(send.im, 32, 64)};
  return h ? cadd(got, e1) : cadd(e0, got);
}

template <bool INVERT>
__device__ __forceinline__ c32 gram_mfma_u64(const UlArgs& a, c32 (&A)[64], int lane, int wave) {
  const int h = lane >> 5, col = lane & 31;
  f32x16 re[2][2], im[2][2];
  c32 hy0 = cz(), hy1 = cz();
  const int ls = wave / a.Cp, c = wave % a.Cp;
  const int k = blockIdx.x * a.sc_per_block + ls;
  const bool act = (k < a.n_sc) && (c < a.C);
  const c32* Hk = a.H + (size_t)k * a.B * 64 + (size_t)c * a.S * 64;
  const c32* yk = a.y + (size_t)k * a.n_sym * a.B + (size_t)c * a.S;
#pragma unroll
  for (int I = 0; I < 2; ++I)
#pragma unroll
    for (int J = 0; J < 2; ++J) {
      re[I][J] = f32x16{};
      im[I][J] = f32x16{};
    }
  c32 x0 = cz(), x1 = cz(), yv = cz();
  auto fetch = [&](int s0, c32& o0, c32& o1, c32& oy) {
    const int s = s0 + h;
    const bool ok = act && s < a.S;
    o0 = ok ? Hk[(size_t)s * 64 + col] : cz();
    o1 = ok ? Hk[(size_t)s * 64 + 32 + col] : cz();
    oy = ok ? yk[s] : cz();
  };
  fetch(0, x0, x1, yv);
  for (int s0 = 0; s0 < a.S; s0 += 2) {
    c32 n0, n1, ny;
    if (s0 + 2 < a.S) fetch(s0 + 2, n0, n1, ny);
    const c32 xs[2] = {x0, x1};
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int J = 0; J < 2; ++J) {
        re[I][J] = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[I].re, xs[J].re, re[I][J], 0, 0, 0);
        re[I][J] = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[I].im, xs[J].im, re[I][J], 0, 0, 0);
        im[I][J] = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[I].re, xs[J].im, im[I][J], 0, 0, 0);
        im[I][J] = __builtin_amdgcn_mfma_f32_32x32x2f32(-xs[I].im, xs[J].re, im[I][J], 0, 0, 0);
      }
    // entries col and 32 + col of H_c^H y_c over the rows of this lane's parity
    cmacc(hy0, x0, yv);
    cmacc(hy1, x1, yv);
    x0 = n0;
    x1 = n1;
    yv = ny;
  }
  if (INVERT) gj_invert_mfma_u64(re, im, lane, a.rho);
  acc_to_rows_u64(re, im, A, h);
  return combine_hy_u64(hy0, hy1, h);
}

// Mixed-precision Gram for U = 64 (one problem per wave): split half-precision
// H = H_hi + H_lo after a power-of-two scaling, four 32x32 tiles on
// v_mfma_f32_32x32x16_{f16,bf16}; lane l supplies rows 8(l/32) .. 8(l/32)+7 of
// each 16-row chunk at column 32I + l%32 (A) and 32J + l%32 (B).  Then the FP32
// Gauss-Jordan inverse on the matrix cores.
template <typename HT>
__device__ __forceinline__ c32 gram_inv_mixed_u64(const UlArgs& a, c32 (&A)[64], int lane, int wave) {
  typedef typename HalfMma<HT>::V V;
  const int h = lane >> 5, col = lane & 31;
  const int ls = wave / a.Cp, c = wave % a.Cp;
  const int k = blockIdx.x * a.sc_per_block + ls;
  const bool act = (k < a.n_sc) && (c < a.C);
  const c32* Hk = a.H + (size_t)k * a.B * 64 + (size_t)c * a.S * 64;
  const c32* yk = a.y + (size_t)k * a.n_sym * a.B + (size_t)c * a.S;
  f32x16 re[2][2], im[2][2];
#pragma unroll
  for (int I = 0; I < 2; ++I)
#pragma unroll
    for (int J = 0; J < 2; ++J) {
      re[I][J] = f32x16{};
      im[I][J] = f32x16{};
    }
  // pass 1: scale exponent from the largest |Re|, |Im|
  float mx = 0.f;
  for (int s0 = 0; s0 < a.S; s0 += 16) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int s = s0 + 8 * h + t;
      const bool ok = act && s < a.S;
      const c32 v0 = ok ? Hk[(size_t)s * 64 + col] : cz();
      const c32 v1 = ok ? Hk[(size_t)s * 64 + 32 + col] : cz();
      mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v0.re), fabsf(v0.im)), fmaxf(fabsf(v1.re), fabsf(v1.im))));
    }
  }
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
      const bool ok = act && s < a.S;
      const c32 yv = ok ? yk[s] : cz();
#pragma unroll
      for (int I = 0; I < 2; ++I) {
        const c32 v = ok ? Hk[(size_t)s * 64 + 32 * I + col] : cz();
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
#pragma unroll
  for (int I = 0; I < 2; ++I)
#pragma unroll
    for (int J = 0; J < 2; ++J)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        re[I][J][r] = ldexpf(re[I][J][r], -2 * ex);
        im[I][J][r] = ldexpf(im[I][J][r], -2 * ex);
      }
  gj_invert_mfma_u64(re, im, lane, a.rho);
  acc_to_rows_u64(re, im, A, h);
  return combine_hy_u64(hy0, hy1, h);
}

// Consensus: every lane of cluster c writes its entry of w_c into its slot;
// after the barrier each lane sums the C clusters of its subcarrier in cluster
// order 1..C (identical sum on every cluster, as if broadcast by the fusion
// node).
__device__ __forceinline__ c32 consensus(c32 wc, int buf, int ls, int G, int u, int C, int Cp, const Smem& sm,
                                         int slot, int nw) {
  c32* cb = sm.cons + buf * nw * 64;
  cb[slot] = wc;
  __syncthreads();
  c32 w = cz();
  const c32* src = cb + (size_t)ls * Cp * G + u;
  for (int cc = 0; cc < C; ++cc) w = cadd(w, src[cc * G]);
  return w;
}

// ---------------------------------------------------------------------------
// Algorithm 1, U x U branch (S >= U), FP32.  Group size G = U.
// ---------------------------------------------------------------------------
// MODE: 0 FP32; 1 / 2 mixed FP16 / BF16 Gram with an FP32 (MFMA) inverse;
// 3 / 4 the same with an FP64 inverse.  Mixed modes exist for U = 32 only.
template <int G, int MODE>
__global__ void __launch_bounds__(512) admm_ul_f32(UlArgs a) {
  constexpr int P = 64 / G;
  extern __shared__ float4 smem_raw[];
  const int nw = blockDim.x >> 6;
  Smem sm = carve(reinterpret_cast<c32*>(smem_raw), nw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane / G, u = lane % G;
  const int lp = wave * P + g;
  const int ls = lp / a.Cp, c = lp % a.Cp;
  const int k = blockIdx.x * a.sc_per_block + ls;
  const bool active = (k < a.n_sc) && (c < a.C);
  const int slot = wave * 64 + lane;
  c32* line = sm.line + wave * 64;
  const int gbase = g * G;

  // Preprocessing (Alg. 1, S > U branch): B_c = H_c^H H_c + rho I, B_c^{-1}.
  c32 A[G];
#pragma unroll
  for (int v = 0; v < G; ++v) A[v] = cz();
  c32 hy0;
  if constexpr (G == 32 && MODE == 0) {
    hy0 = gram_mfma_u32<true>(a, A, lane, wave);
  } else if constexpr (G == 32 && (MODE == 1 || MODE == 3)) {
    hy0 = gram_inv_mixed_u32<_Float16, MODE == 3>(a, A, lane, wave, reinterpret_cast<c64*>(sm.stage + wave * kStageRows * 64));
  } else if constexpr (G == 32 && (MODE == 2 || MODE == 4)) {
    hy0 = gram_inv_mixed_u32<__bf16, MODE == 4>(a, A, lane, wave, reinterpret_cast<c64*>(sm.stage + wave * kStageRows * 64));
  } else if constexpr (G == 16) {
    hy0 = gram_mfma_u16(a, A, lane, wave, sm.stage + wave * kStageRows * 64);
#pragma unroll
    for (int v = 0; v < G; ++v)
      if (v == u) A[v].re += a.rho;
    gj_invert<G>(A, u, line, gbase);
  } else if constexpr (G == 64 && MODE == 0) {
    hy0 = gram_mfma_u64<true>(a, A, lane, wave);
  } else if constexpr (G == 64 && MODE == 1) {
    hy0 = gram_inv_mixed_u64<_Float16>(a, A, lane, wave);
  } else if constexpr (G == 64 && MODE == 2) {
    hy0 = gram_inv_mixed_u64<__bf16>(a, A, lane, wave);
  } else {
    hy0 = cluster_pass<G, true>(a.H, a.y, A, k, c, 0, u, g, lane, wave, active, a.B, a.S, G, a.n_sym, sm);
#pragma unroll
    for (int v = 0; v < G; ++v)
      if (v == u) A[v].re += a.rho;
    gj_invert<G>(A, u, line, gbase);
  }

  int buf = 0;
  for (int n = 0; n < a.n_sym; ++n) {
    c32 hy = hy0;
    if (n > 0) hy = cluster_pass<G, false>(a.H, a.y, A, k, c, n, u, g, lane, wave, active, a.B, a.S, G, a.n_sym, sm);
    // y_c^reg = B_c^{-1} H_c^H y_c; z = y^reg; lambda = 0
    const c32 yreg = group_matvec<G>(A, hy, u, line, gbase);
    c32 z = yreg, lam = cz();
    c32 w = consensus(active ? z : cz(), buf, ls, G, u, a.C, a.Cp, sm, slot, nw);
    buf ^= 1;
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
      const c32 bq = group_matvec<G>(A, q, u, line, gbase);
      z = c32{fmaf(a.rho, bq.re, yreg.re), fmaf(a.rho, bq.im, yreg.im)};
      w = consensus(active ? cadd(z, lam) : cz(), buf, ls, G, u, a.C, a.Cp, sm, slot, nw);
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
      }
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
  constexpr int P = 64 / G;
  extern __shared__ float4 smem_raw[];
  const int nw = blockDim.x >> 6;
  Smem sm = carve(reinterpret_cast<c32*>(smem_raw), nw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane / G, u = lane % G;
  const int lp = wave * P + g;
  const int ls = lp / a.Cp, c = lp % a.Cp;
  const int k = blockIdx.x * a.sc_per_block + ls;
  const bool active = (k < a.n_sc) && (c < a.C);
  const int slot = wave * 64 + lane;
  c32* line = sm.line + wave * 64;
  const int gbase = g * G;

  c32 A[G];
#pragma unroll
  for (int v = 0; v < G; ++v) A[v] = cz();
  c32 hy0;
  if constexpr (G == 32)
    hy0 = gram_mfma_u32<false>(a, A, lane, wave);
  else if constexpr (G == 16)
    hy0 = gram_mfma_u16(a, A, lane, wave, sm.stage + wave * kStageRows * 64);
  else if constexpr (G == 64)
    hy0 = gram_mfma_u64<false>(a, A, lane, wave);
  else
    hy0 = cluster_pass<G, true>(a.H, a.y, A, k, c, 0, u, g, lane, wave, active, a.B, a.S, G, a.n_sym, sm);

  int buf = 0;
  for (int n = 0; n < a.n_sym; ++n) {
    c32 hy = hy0;
    if (n > 0) hy = cluster_pass<G, false>(a.H, a.y, A, k, c, n, u, g, lane, wave, active, a.B, a.S, G, a.n_sym, sm);
    // y^MRC = sum_c H_c^H y_c (consensus); r = p = y^MRC; x = 0
    c32 r = consensus(active ? hy : cz(), buf, ls, G, u, a.C, a.Cp, sm, slot, nw);
    buf ^= 1;
    c32 pv = r, x = cz();
    float rr = group_sum<G>(r.re * r.re + r.im * r.im);
    for (int t = 1; t <= a.T; ++t) {
      const c32 wc = group_matvec<G>(A, pv, u, line, gbase);
      const c32 w = consensus(active ? wc : cz(), buf, ls, G, u, a.C, a.Cp, sm, slot, nw);
      buf ^= 1;
      const c32 e = c32{fmaf(a.rho, pv.re, w.re), fmaf(a.rho, pv.im, w.im)};
      const float pe = group_sum<G>(pv.re * e.re + pv.im * e.im);
      const float alpha = (rr > 0.f) ? rr / pe : 0.f;
      x.re = fmaf(alpha, pv.re, x.re);
      x.im = fmaf(alpha, pv.im, x.im);
      r.re = fmaf(-alpha, e.re, r.re);
      r.im = fmaf(-alpha, e.im, r.im);
      const float rr_new = group_sum<G>(r.re * r.re + r.im * r.im);
      const float beta = (rr > 0.f) ? rr_new / rr : 0.f;
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
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Algorithm 3 (decentralized ADMM beamforming, epsilon = 0), S x S branch
// (S <= U), FP32.  Group size G = U.  The downlink cluster channel is
// H_c = (Hu_c)^T with Hu_c the S x U uplink block (reciprocity), read in place
// from the uplink layout.  Lane u holds column u of Hu_c (entries Hu_c[a][u],
// a < S) for m_c = H_c x_c; lane a < S holds row a of Hu_c for H_c^H v and
// row a of A_c^{-1}.
// ---------------------------------------------------------------------------
template <int G, int SG>
__global__ void __launch_bounds__(512) admm_dl_f32(DlArgs a) {
  constexpr int P = 64 / G;
  extern __shared__ float4 smem_raw[];
  const int nw = blockDim.x >> 6;
  Smem sm = carve(reinterpret_cast<c32*>(smem_raw), nw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane / G, u = lane % G;
  const int lp = wave * P + g;
  const int ls = lp / a.Cp, c = lp % a.Cp;
  const int k = blockIdx.x * a.sc_per_block + ls;
  const bool active = (k < a.n_sc) && (c < a.C);
  const int slot = wave * 64 + lane;
  c32* line = sm.line + wave * 64;
  const int gbase = g * G;
  const int S = a.S;
  const c32* Hk = a.H + (size_t)k * a.B * G + (size_t)c * S * G;

  c32 hcol[SG], hrow[G], A[SG];
#pragma unroll
  for (int i = 0; i < SG; ++i) {
    hcol[i] = (active && i < S) ? Hk[(size_t)i * G + u] : cz();
    A[i] = cz();
  }
#pragma unroll
  for (int i = 0; i < G; ++i) hrow[i] = (active && u < S) ? Hk[(size_t)u * G + i] : cz();
  // A_c = H_c^H H_c + rho^{-1} I_S with (H_c^H H_c)[a][b] = sum_u conj(Hu[a][u]) Hu[b][u].
  if constexpr (G == 32 && SG == 16) {
    gram_dl_mfma_s16_u32(a, A, lane, wave, sm.stage + wave * kStageRows * 64);
  } else {
    // Row b of Hu_c is broadcast from the stage buffer of this wave.
    c32* stage = sm.stage + wave * kStageRows * 64;
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
      for (int v0 = 0; v0 < G; v0 += 8) {
        c32 row[8];
        lds_read_vec<8>(stage + gbase + v0, row);
#pragma unroll
        for (int v = 0; v < 8; ++v) cmacc(acc, hrow[v0 + v], row[v]);
      }
      wave_lds_sync();
#pragma unroll
      for (int i = 0; i < SG; ++i)
        if (i == b) A[i] = (u < S) ? acc : cz();
    }
  }
  const float irho = 1.0f / a.rho;
#pragma unroll
  for (int v = 0; v < SG; ++v)
    if (v == u) A[v].re += (u < S) ? irho : 1.0f;
  gj_invert<SG>(A, u, line, gbase);

  int buf = 0;
  for (int n = 0; n < a.n_sym; ++n) {
    const size_t vo = ((size_t)k * a.n_sym + n);
    const c32 s = (k < a.n_sc) ? a.s[vo * G + u] : cz();
    c32 z = cscale(s, a.f0), lam = cz();
    // x_c = A_c^{-1} H_c^H (z + lambda), entry a held by lane a < S
    auto apply = [&](c32 v) -> c32 {
      line[gbase + u] = v;
      wave_lds_sync();
      c32 acc = cz();
#pragma unroll
      for (int v0 = 0; v0 < G; v0 += 8) {
        c32 vv[8];
        lds_read_vec<8>(line + gbase + v0, vv);
#pragma unroll
        for (int i = 0; i < 8; ++i) cmacc(acc, hrow[v0 + i], vv[i]);
      }
      wave_lds_sync();
      return group_matvec<SG>(A, (u < S) ? acc : cz(), u, line, gbase);
    };
    c32 x = apply(z);
    for (int t = 2; t <= a.T; ++t) {
      // m_c = H_c x_c: m[u] = sum_a Hu[a][u] x[a]
      line[gbase + u] = x;
      wave_lds_sync();
      c32 m = cz();
#pragma unroll
      for (int v0 = 0; v0 < SG; v0 += 8) {
        c32 xv[8];
        lds_read_vec<8>(line + gbase + v0, xv);
#pragma unroll
        for (int i = 0; i < 8; ++i) cmac(m, hcol[v0 + i], xv[i]);
      }
      wave_lds_sync();
      const c32 wc = csub(m, lam);
      const c32 w = consensus(active ? wc : cz(), buf, ls, G, u, a.C, a.Cp, sm, slot, nw);
      buf ^= 1;
      z = c32{fmaf(a.invC, s.re - w.re, wc.re), fmaf(a.invC, s.im - w.im, wc.im)};
      lam.re = fmaf(-a.gamma, m.re - z.re, lam.re);
      lam.im = fmaf(-a.gamma, m.im - z.im, lam.im);
      x = apply(cadd(z, lam));
    }
    // optional common power scaling: beta = min(1, min_c sqrt(P_c / ||x_c||^2))
    float beta = 1.0f;
    if (a.P) {
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

hipError_t launch_admm_ul_f32(const UlArgs& a, int U, int nw, hipStream_t st) {
  switch (U) {
    case 8: return launch(admm_ul_f32<8, 0>, a, nw, st);
    case 16: return launch(admm_ul_f32<16, 0>, a, nw, st);
    case 32: return launch(admm_ul_f32<32, 0>, a, nw, st);
    case 64: return launch(admm_ul_f32<64, 0>, a, nw, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_admm_ul_mixed(const UlArgs& a, int U, int half, bool f64, int nw, hipStream_t st) {
  if (U == 64 && !f64) return half == 1 ? launch(admm_ul_f32<64, 1>, a, nw, st) : launch(admm_ul_f32<64, 2>, a, nw, st);
  if (U != 32) return hipErrorInvalidValue;
  if (half == 1) return f64 ? launch(admm_ul_f32<32, 3>, a, nw, st) : launch(admm_ul_f32<32, 1>, a, nw, st);
  return f64 ? launch(admm_ul_f32<32, 4>, a, nw, st) : launch(admm_ul_f32<32, 2>, a, nw, st);
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

hipError_t launch_admm_dl_f32(const DlArgs& a, int U, int nw, hipStream_t st) {
  const int S = a.S;
  switch (U) {
    case 8: return launch(admm_dl_f32<8, 8>, a, nw, st);
    case 16:
      return S <= 8 ? launch(admm_dl_f32<16, 8>, a, nw, st) : launch(admm_dl_f32<16, 16>, a, nw, st);
    case 32:
      if (S <= 8) return launch(admm_dl_f32<32, 8>, a, nw, st);
      if (S <= 16) return launch(admm_dl_f32<32, 16>, a, nw, st);
      return launch(admm_dl_f32<32, 32>, a, nw, st);
    case 64:
      if (S <= 8) return launch(admm_dl_f32<64, 8>, a, nw, st);
      if (S <= 16) return launch(admm_dl_f32<64, 16>, a, nw, st);
      if (S <= 32) return launch(admm_dl_f32<64, 32>, a, nw, st);
      return launch(admm_dl_f32<64, 64>, a, nw, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace dbp
