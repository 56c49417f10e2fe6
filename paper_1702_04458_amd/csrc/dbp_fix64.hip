// Exact hard decisions: FP64 recomputation of the subcarriers whose FP32
// result lies near a decision threshold.
//
// The FP32 detection kernels flag every subcarrier with a soft value within a
// guard of a slicing threshold (Section III-A: nearest-point slicing of the
// equalized estimate; the guard is a stated multiple of the FP32 path's
// measured error).  For those subcarriers these kernels run the whole method
// again in FP64 -- Algorithm 1 (U x U branch: B_c = H_c^H H_c + rho I,
// y_c^reg, Lemma 1's consensus, the proximal steps E2-MMSE / E2-ZF / E2-BOX)
// or Algorithm 2 (decentralized CG, residual update with e^(t)) -- and
// overwrite the soft output (rounded to FP32) and the hard decision (taken in
// FP64).  The decisions then agree with an FP64 evaluation of the method
// everywhere except within about 1e-14 of a threshold.
//
// Work split: the flags are scanned in windows of up to 16,384 subcarriers;
// the flagged subcarriers of a window are ranked in index order and dealt
// out round-robin over the n_slots workgroups, each of which recomputes its
// share one subcarrier after another with all 1024 threads.  The ADMM pass keeps the C regularised inverses of the current
// subcarrier (C U^2 complex FP64) in the workgroup's slot of the workspace;
// every entry of a slot is written before it is read, so the workspace needs
// no clearing.
#include <hip/hip_runtime.h>

#include "dbp_device.h"
#include "dbp_launch.h"

namespace dbp {
namespace {

constexpr int kFixThreads = 1024;

struct d2 {
  double re, im;
};

__device__ __forceinline__ d2 dzero() { return d2{0.0, 0.0}; }
__device__ __forceinline__ d2 dld(const c32* p) {
  const c32 v = *p;
  return d2{(double)v.re, (double)v.im};
}
// acc += conj(x) * y
__device__ __forceinline__ void dmacc(d2& acc, d2 x, d2 y) {
  acc.re += x.re * y.re + x.im * y.im;
  acc.im += x.re * y.im - x.im * y.re;
}
// acc += x * y
__device__ __forceinline__ void dmac(d2& acc, d2 x, d2 y) {
  acc.re += x.re * y.re - x.im * y.im;
  acc.im += x.re * y.im + x.im * y.re;
}

// i = clamp(floor((kappa x + L) / 2), 0, L - 1) in FP64, ties up
__device__ __forceinline__ int slice64(double x, double kappa, int L) {
  double i = floor((kappa * x + (double)L) / 2.0);
  i = fmin(fmax(i, 0.0), (double)(L - 1));
  return (int)i;
}

// True when the FP32 pass of this call flagged nothing (it stores the call's
// epoch at f.any when it flags a subcarrier): the pass then neither scans
// the flags nor recomputes anything.  A stale value from an earlier call
// differs from this call's epoch, so the test errs only towards scanning.
__device__ __forceinline__ bool nothing_flagged(const FixArgs& f) { return f.any && *f.any != f.epoch; }

// Flags per thread in one scan of the flag array, and the LDS list capacity.
constexpr int kPerThread = 16;
constexpr int kListCap = kFixThreads;

// Subcarriers per round: every workgroup scans the whole window, so that the
// flagged subcarriers can be shared out evenly; the window is small enough
// that a workgroup's share fits the LDS list.
__device__ __forceinline__ long fix_window() {
  const long w = (long)kFixThreads * kPerThread, cap = (long)kListCap * gridDim.x;
  return w < cap ? w : cap;
}

// Round r covers subcarriers [r W, (r + 1) W).  Every workgroup ranks the
// flagged subcarriers of the window in index order (a block-wide prefix sum
// of per-thread counts) and takes those of rank q with (q + r) mod G = g
// (G workgroups, this one g), in rank order, into list[0 .. n); returns n.
// The flagged subcarriers of a window are thus spread over the workgroups,
// at most ceil(count / G) per workgroup.  wsum: LDS scratch of
// kFixThreads / 64 + 1 ints.
__device__ int collect_round(const FixArgs& f, long r, long W, int* list, int* wsum) {
  __syncthreads();   // the previous round's list and sums are no longer read
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nwv = kFixThreads / 64;
  const long end = ((r + 1) * W < f.n_sc) ? (r + 1) * W : f.n_sc;
  const long base = r * W + (long)t * kPerThread;
  unsigned bits = 0;
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const long k = base + i;
    if (k < end && (f.flags[k] & kStatusReslice)) bits |= 1u << i;
  }
  const int mine = __popc(bits);
  int incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int w = 0; w < nwv; ++w) {
      const int v = wsum[w];
      wsum[w] = acc;
      acc += v;
    }
    wsum[nwv] = acc;
  }
  __syncthreads();
  const int G = gridDim.x, g = blockIdx.x;
  const int q0 = (int)(((long)g - r % G + G) % G);   // first rank this workgroup takes
  int q = wsum[wv] + incl - mine;                    // rank of this thread's first flagged subcarrier
  const int total = wsum[nwv];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    if ((bits >> i) & 1u) {
      if (q >= q0 && (q - q0) % G == 0) list[(q - q0) / G] = (int)(base + i);
      ++q;
    }
  }
  __syncthreads();
  return total > q0 ? (total - q0 + G - 1) / G : 0;
}

// Proximal step of Lemma 1 on the summed vector w (E2-MMSE / E2-ZF: w / den,
// den = N0 / (rho Es) + C; E2-BOX: clip of w / C to the QAM box).
__device__ __forceinline__ d2 prox64(const FixArgs& f, d2 w) {
  if (f.reg == 2) {
    const double vr = w.re * f.invC, vi = w.im * f.invC;
    return d2{fmin(fmax(vr, -f.box_r), f.box_r), fmin(fmax(vi, -f.box_r), f.box_r)};
  }
  return d2{w.re / f.inv_den, w.im / f.inv_den};
}

__device__ __forceinline__ void write_out(const FixArgs& f, int k, int n, int u, d2 s) {
  const size_t o = ((size_t)k * f.n_sym + n) * f.U + u;
  f.shat[o] = c32{(float)s.re, (float)s.im};
  if (f.hard) f.hard[o] = (uint8_t)(slice64(s.re, f.kappa, f.L) + f.L * slice64(s.im, f.kappa, f.L));
}

}  // namespace

// Algorithm 1 in FP64 for the flagged subcarriers.  The regularised Grams
// are formed and inverted in registers: thread t owns a TI x TI tile of one
// cluster's U x U matrix, NTH / (U / TI)^2 clusters at a time.  Gram: each
// thread accumulates its tile over the S rows of H_c straight from memory
// (the lanes of a wave that share tile rows read the same addresses).
// Inverse: Gauss-Jordan elimination without pivoting (HPD) on all clusters
// of the group at once; per pivot p the owners of row p and column p publish
// them through LDS (colp, rowp: [clusters][U]) and every thread updates its
// tile.  The inverses go to M ([C][U][U], entry (i, j) at i U + j).
// Rows of H_c per staging step of the one-cluster form.
constexpr int kStageH = 16;

// hbuf (one-cluster form, NTH = 256, or null): kStageH x U complex values of
// LDS through which the Gram's rows are staged: every thread loads its share
// of the next block of rows while the current one is used, so the loads of a
// whole block are in flight together instead of one row's at a time.
template <int U, int TI, int NTH>
__device__ __forceinline__ void fix64_factor_group(const FixArgs& f, const c32* Hk, int cb, d2* M, d2* colp,
                                                   d2* rowp, c32* hbuf = nullptr) {
  constexpr int NT = U / TI, T2 = NT * NT, UU = U * U;
  const int tid = threadIdx.x;
  const int cl = tid / T2, tt = tid % T2, i0 = (tt / NT) * TI, j0 = (tt % NT) * TI;
  const int c = cb + cl;
  const bool own = cl < NTH / T2 && c < f.C;   // this thread's cluster exists
  d2 A[TI][TI];
#pragma unroll
  for (int a = 0; a < TI; ++a)
#pragma unroll
    for (int b = 0; b < TI; ++b) A[a][b] = dzero();
  // B_c = H_c^H H_c + rho I, tile rows i0.., columns j0..
  auto gram_row = [&](const c32* row) {
    d2 hj[TI];
#pragma unroll
    for (int b = 0; b < TI; ++b) hj[b] = dld(row + j0 + b);
#pragma unroll
    for (int a = 0; a < TI; ++a) {
      const d2 hi = dld(row + i0 + a);
#pragma unroll
      for (int b = 0; b < TI; ++b) dmacc(A[a][b], hi, hj[b]);
    }
  };
  const c32* Hc = Hk + (size_t)(c < f.C ? c : 0) * f.S * U;
  if constexpr (NTH == 256 && (kStageH * U) % NTH == 0) {
    // one cluster per workgroup, every thread takes part in the staging
    constexpr int PER = kStageH * U / NTH;
    const int nblk = (f.S + kStageH - 1) / kStageH;
    c32 pre[PER];
    auto fetch = [&](int blk) {
#pragma unroll
      for (int t = 0; t < PER; ++t) {
        const int e = tid + t * NTH, s = blk * kStageH + e / U;
        pre[t] = (own && s < f.S) ? Hc[(size_t)s * U + e % U] : c32{0.f, 0.f};   // rows past S add nothing
      }
    };
    fetch(0);
    for (int blk = 0; blk < nblk; ++blk) {
      __syncthreads();   // the previous block's readers are done with hbuf
#pragma unroll
      for (int t = 0; t < PER; ++t) hbuf[tid + t * NTH] = pre[t];
      __syncthreads();
      if (blk + 1 < nblk) fetch(blk + 1);
#pragma unroll 4
      for (int r = 0; r < kStageH; ++r) gram_row(hbuf + r * U);
    }
  } else if (own) {
    for (int s = 0; s < f.S; ++s) gram_row(Hc + (size_t)s * U);
  }
  if (own) {
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
      for (int b = 0; b < TI; ++b)
        if (i0 + a == j0 + b) A[a][b].re += f.rho;
  }
  // Gauss-Jordan: after pivot p, A[p][p] = 1/d, A[p][j] = B[p][j]/d,
  // A[i][p] = -B[i][p]/d and A[i][j] -= B[i][p] B[p][j]/d elsewhere
  for (int p = 0; p < U; ++p) {
    __syncthreads();   // the previous step's readers are done with colp / rowp
    if (own && j0 <= p && p < j0 + TI) {
#pragma unroll
      for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TI; ++b)
          if (j0 + b == p) colp[cl * U + i0 + a] = A[a][b];
    }
    if (own && i0 <= p && p < i0 + TI) {
#pragma unroll
      for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TI; ++b)
          if (i0 + a == p) rowp[cl * U + j0 + b] = A[a][b];
    }
    __syncthreads();
    if (own) {
      const double inv = 1.0 / rowp[cl * U + p].re;
      d2 rj[TI];
#pragma unroll
      for (int b = 0; b < TI; ++b) rj[b] = rowp[cl * U + j0 + b];
      // the rank-1 update on every entry of the tile (straight-line code);
      // the entries of pivot row p and column p are then overwritten, by the
      // few threads whose tile holds them
      d2 m[TI];
#pragma unroll
      for (int a = 0; a < TI; ++a) {
        const d2 ci = colp[cl * U + i0 + a];
        m[a] = d2{ci.re * inv, ci.im * inv};   // the multiplier B[i][p] / d
#pragma unroll
        for (int b = 0; b < TI; ++b) {
          A[a][b].re -= m[a].re * rj[b].re - m[a].im * rj[b].im;
          A[a][b].im -= m[a].re * rj[b].im + m[a].im * rj[b].re;
        }
      }
      if (i0 <= p && p < i0 + TI) {
#pragma unroll
        for (int a = 0; a < TI; ++a)
          if (i0 + a == p) {
#pragma unroll
            for (int b = 0; b < TI; ++b) A[a][b] = d2{rj[b].re * inv, rj[b].im * inv};
          }
      }
      if (j0 <= p && p < j0 + TI) {
#pragma unroll
        for (int b = 0; b < TI; ++b)
          if (j0 + b == p) {
#pragma unroll
            for (int a = 0; a < TI; ++a) A[a][b] = (i0 + a == p) ? d2{inv, 0.0} : d2{-m[a].re, -m[a].im};
          }
      }
    }
  }
  if (own) {
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
      for (int b = 0; b < TI; ++b) M[(size_t)c * UU + (i0 + a) * U + j0 + b] = A[a][b];
  }
}

// Algorithm 1's iterations in FP64 for subcarrier k with the inverses
// B_c^{-1} in M, all symbols; writes the outputs.  LDS: Y, Z, LM ([C][U])
// and Sv ([U]).  Ends with a barrier.
template <int U, int NTH, bool UNROLL = false>
__device__ __forceinline__ void fix64_iterate(const FixArgs& f, int k, const d2* M, d2* Y, d2* Z, d2* LM, d2* Sv) {
  constexpr int UU = U * U;
  const int C = f.C, S = f.S, CU = C * U, tid = threadIdx.x;
  const c32* Hk = f.H + (size_t)k * f.B * U;
  for (int n = 0; n < f.n_sym; ++n) {
    const c32* yk = f.y + ((size_t)k * f.n_sym + n) * f.B;
    // H_c^H y_c
    for (int e = tid; e < CU; e += NTH) {
      const int c = e / U, i = e - c * U;
      const c32* Hc = Hk + (size_t)c * S * U;
      d2 acc = dzero();
      if constexpr (UNROLL) {
        // eight rows per step: their loads in flight together
#pragma unroll 8
        for (int s = 0; s < S; ++s) dmacc(acc, dld(Hc + (size_t)s * U + i), dld(yk + (size_t)c * S + s));
      } else {
        for (int s = 0; s < S; ++s) dmacc(acc, dld(Hc + (size_t)s * U + i), dld(yk + (size_t)c * S + s));
      }
      Z[e] = acc;
    }
    __syncthreads();
    // y_c^reg = B_c^{-1} H_c^H y_c
    for (int e = tid; e < CU; e += NTH) {
      const int c = e / U, i = e - c * U;
      const d2* Mi = M + (size_t)c * UU + i * U;
      d2 acc = dzero();
      for (int j = 0; j < U; ++j) dmac(acc, Mi[j], Z[c * U + j]);
      Y[e] = acc;
    }
    __syncthreads();
    for (int e = tid; e < CU; e += NTH) {
      Z[e] = Y[e];
      LM[e] = dzero();
    }
    __syncthreads();
    for (int i = tid; i < U; i += NTH) {
      d2 w = dzero();
      for (int c = 0; c < C; ++c) {
        w.re += Z[c * U + i].re;
        w.im += Z[c * U + i].im;
      }
      Sv[i] = prox64(f, w);
    }
    __syncthreads();
    for (int t = 2; t <= f.T; ++t) {
      // lambda_c += gamma (z_c - s)
      for (int e = tid; e < CU; e += NTH) {
        const int i = e % U;
        LM[e].re += f.gamma * (Z[e].re - Sv[i].re);
        LM[e].im += f.gamma * (Z[e].im - Sv[i].im);
      }
      __syncthreads();
      // z_c = y_c^reg + rho B_c^{-1} (s - lambda_c)
      for (int e = tid; e < CU; e += NTH) {
        const int c = e / U, i = e - c * U;
        const d2* Mi = M + (size_t)c * UU + i * U;
        d2 acc = dzero();
        for (int j = 0; j < U; ++j)
          dmac(acc, Mi[j], d2{Sv[j].re - LM[c * U + j].re, Sv[j].im - LM[c * U + j].im});
        Z[e] = d2{Y[e].re + f.rho * acc.re, Y[e].im + f.rho * acc.im};
      }
      __syncthreads();
      // s = prox(sum_c (z_c + lambda_c))
      for (int i = tid; i < U; i += NTH) {
        d2 w = dzero();
        for (int c = 0; c < C; ++c) {
          w.re += Z[c * U + i].re + LM[c * U + i].re;
          w.im += Z[c * U + i].im + LM[c * U + i].im;
        }
        Sv[i] = prox64(f, w);
      }
      __syncthreads();
    }
    for (int i = tid; i < U; i += NTH) write_out(f, k, n, i, Sv[i]);
    __syncthreads();
  }
}

// Tile side of the whole-workgroup factorisation (1024 threads) and of the
// per-cluster one (256 threads, one cluster per workgroup).
template <int U>
constexpr int tile_all() { return (U >= 32) ? 4 : U / 8; }
template <int U>
constexpr int tile_one() { return (U >= 16) ? U / 16 : 1; }

// The whole re-slice of the flagged subcarriers of one frame, 1024 threads
// per workgroup.  With f.split, each workgroup's first subcarrier of the
// first window is not done here: its index goes to f.list0 (-1 for none),
// and admm_ul_factor64 / admm_ul_iter64 recompute it with one workgroup per
// cluster for the inverses.  f.inv_den holds the denominator
// N0 / (rho Es) + C itself (FP64 divides by it).
template <int U>
__device__ __forceinline__ void admm_ul_fix64_body(const FixArgs& f) {
  if (nothing_flagged(f)) return;   // uniform
  constexpr int TI = tile_all<U>();
  constexpr int CG = kFixThreads / ((U / TI) * (U / TI));   // clusters per group
  extern __shared__ d2 fsm[];
  const int C = f.C, CU = C * U;
  // LDS: the iteration vectors, overlaid during the inversion by the pivot
  // rows and columns of the group's clusters
  d2* Y = fsm;            // y_c^reg (first H_c^H y_c)
  d2* Z = Y + CU;         // z_c
  d2* LM = Z + CU;        // lambda_c
  d2* Sv = LM + CU;       // s
  d2* colp = fsm;         // [CG][U] pivot columns
  d2* rowp = fsm + CG * U;   // [CG][U] pivot rows
  int* list = reinterpret_cast<int*>(fsm + (3 * CU + U > 2 * CG * U ? 3 * CU + U : 2 * CG * U));
  int* wsum = list + kListCap;
  d2* Mslot = static_cast<d2*>(f.ws) + (size_t)blockIdx.x * C * U * U;   // [C][U][U]

  const long W = fix_window();
  for (long r = 0; r * W < f.n_sc; ++r) {
    const int nl = collect_round(f, r, W, list, wsum);
    int q = 0;
    if (f.split && r == 0) {
      if (threadIdx.x == 0) f.list0[blockIdx.x] = nl > 0 ? list[0] : -1;
      q = 1;
    }
    for (; q < nl; ++q) {
      const int k = list[q];
      const c32* Hk = f.H + (size_t)k * f.B * U;
      for (int cb = 0; cb < C; cb += CG) fix64_factor_group<U, TI, kFixThreads>(f, Hk, cb, Mslot, colp, rowp);
      __syncthreads();   // inverses in the slot; the LDS overlay is free again
      fix64_iterate<U, kFixThreads>(f, k, Mslot, Y, Z, LM, Sv);
    }
  }
}

template <int U>
__global__ void __launch_bounds__(kFixThreads) admm_ul_fix64(FixArgs f) {
  admm_ul_fix64_body<U>(f);
}

// The re-slice of a batch of frames (one U): the frames one after another,
// each over all workgroups (they share the workspace slots).
template <int U>
__global__ void __launch_bounds__(kFixThreads) admm_ul_fix64_batch(FixBatch b) {
  for (int i = 0; i < b.n; ++i) admm_ul_fix64_body<U>(b.f[i]);
}

// Split recomputation, step 1: workgroup (g, c) forms and inverts cluster c's
// regularised Gram of the subcarrier f.list0[g] into slot g.
template <int U>
__global__ void __launch_bounds__(256) admm_ul_factor64(FixArgs f) {
  __shared__ d2 piv[2 * U];
  __shared__ c32 hbuf[kStageH * U];
  if (nothing_flagged(f)) return;   // uniform
  const int k = f.list0[blockIdx.x];
  if (k < 0 || (int)blockIdx.y >= f.C) return;   // uniform
  d2* Mslot = static_cast<d2*>(f.ws) + (size_t)blockIdx.x * f.C * U * U;
  fix64_factor_group<U, tile_one<U>(), 256>(f, f.H + (size_t)k * f.B * U, blockIdx.y, Mslot, piv, piv + U, hbuf);
}

// Split recomputation, step 2: the iterations of subcarrier f.list0[g] with
// the inverses of slot g.
template <int U>
__global__ void __launch_bounds__(kFixThreads) admm_ul_iter64(FixArgs f) {
  extern __shared__ d2 fsm[];
  if (nothing_flagged(f)) return;   // uniform
  const int k = f.list0[blockIdx.x];
  if (k < 0) return;   // uniform
  const int CU = f.C * U;
  const d2* Mslot = static_cast<const d2*>(f.ws) + (size_t)blockIdx.x * f.C * U * U;
  fix64_iterate<U, kFixThreads, true>(f, k, Mslot, fsm, fsm + CU, fsm + 2 * CU, fsm + 3 * CU);
}

// Largest B U (complex entries of H[k]) the CG pass keeps in LDS (16 KiB:
// the pass's LDS stays under 64 KiB).
constexpr int kCgStage = 2048;

// Sum over the first wave of v (lanes past the data pass 0); lane 0 stores
// it at *out.  Every thread of the workgroup must call (it ends with a barrier).
__device__ __forceinline__ void wave0_sum(double v, double* out) {
  if (threadIdx.x < 64) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (threadIdx.x == 0) *out = v;
  }
  __syncthreads();
}

// Algorithm 2 in FP64 for the flagged subcarriers (f.rho = N0 / Es, or 0 for
// ZF).  H[k] is staged in LDS when it fits.  w = sum_c H_c^H (H_c p): H p for
// all B rows by one thread per row (blocks of 1024 rows for larger B), then
// one partial sum per (cluster, user) and the sum over the clusters in
// cluster order; the inner products by the first wave.
__global__ void __launch_bounds__(kFixThreads) dcg_ul_fix64(FixArgs f) {
  if (nothing_flagged(f)) return;   // uniform
  extern __shared__ d2 fsm[];
  constexpr int kChunk = 1024;
  const int U = f.U, C = f.C, S = f.S, B = f.B, CU = C * U;
  d2* R = fsm;
  d2* P = R + U;
  d2* X = P + U;
  d2* W = X + U;
  d2* Hp = W + U;                // kChunk entries: H_c p for a block of rows
  d2* Wp = Hp + kChunk;          // [C][U] per-cluster partial sums
  c32* Hs = reinterpret_cast<c32*>(Wp + CU);   // H[k] when B U <= kCgStage
  double* red = reinterpret_cast<double*>(Hs + kCgStage);   // [0] rr, [1] pe, [2] rr_new
  int* list = reinterpret_cast<int*>(red + 4);
  int* wsum = list + kListCap;
  const int tid = threadIdx.x;
  const bool staged = B * U <= kCgStage;

  // w = sum_c H_c^H v_c, with v the B entries at vb (stride vs) or, when
  // vb is null, Hp: per-cluster partial sums by C U threads, then the sum
  // over the clusters in cluster order.  Ends with a barrier.
  auto hh_sum = [&](const c32* rows, const c32* yv, d2* out) {
    for (int e = tid; e < CU; e += kFixThreads) {
      const int c = e / U, i = e - c * U;
      d2 acc = dzero();
      for (int s = 0; s < S; ++s) {
        const int j = c * S + s;
        dmacc(acc, dld(rows + (size_t)j * U + i), yv ? dld(yv + j) : Hp[j]);
      }
      Wp[e] = acc;
    }
    __syncthreads();
    for (int i = tid; i < U; i += kFixThreads) {
      d2 acc = dzero();
      for (int c = 0; c < C; ++c) {
        acc.re += Wp[c * U + i].re;
        acc.im += Wp[c * U + i].im;
      }
      out[i] = acc;
    }
    __syncthreads();
  };

  const long win = fix_window();
  for (long r = 0; r * win < f.n_sc; ++r) {
    const int nl = collect_round(f, r, win, list, wsum);
    for (int q = 0; q < nl; ++q) {
      const int k = list[q];
      const c32* Hk = f.H + (size_t)k * B * U;
      if (staged) {
        for (int e = tid; e < B * U; e += kFixThreads) Hs[e] = Hk[e];
        __syncthreads();
      }
      const c32* rows = staged ? Hs : Hk;
      for (int n = 0; n < f.n_sym; ++n) {
        const c32* yk = f.y + ((size_t)k * f.n_sym + n) * B;
        // y^MRC = sum_c H_c^H y_c; r = p = y^MRC; x = 0
        hh_sum(rows, yk, R);
        for (int i = tid; i < U; i += kFixThreads) {
          P[i] = R[i];
          X[i] = dzero();
        }
        wave0_sum(tid < U ? R[tid].re * R[tid].re + R[tid].im * R[tid].im : 0.0, red);
        for (int t = 1; t <= f.T; ++t) {
          const double rr = red[0];
          if (rr == 0.0) break;   // uniform: every thread read the same value
          // H p for all B rows (blocks of kChunk rows when B is larger), then w = sum_c H_c^H (H_c p)
          if (B <= kChunk) {
            for (int j = tid; j < B; j += kFixThreads) {
              d2 acc = dzero();
              for (int u = 0; u < U; ++u) dmac(acc, dld(rows + (size_t)j * U + u), P[u]);
              Hp[j] = acc;
            }
            __syncthreads();
            hh_sum(rows, nullptr, W);
          } else {
            for (int i = tid; i < U; i += kFixThreads) W[i] = dzero();
            __syncthreads();
            for (int c = 0; c < C; ++c) {
              for (int s0 = 0; s0 < S; s0 += kChunk) {
                const int ns = (S - s0 < kChunk) ? S - s0 : kChunk;
                for (int s = tid; s < ns; s += kFixThreads) {
                  const c32* row = rows + ((size_t)c * S + s0 + s) * U;
                  d2 acc = dzero();
                  for (int u = 0; u < U; ++u) dmac(acc, dld(row + u), P[u]);
                  Hp[s] = acc;
                }
                __syncthreads();
                for (int i = tid; i < U; i += kFixThreads) {
                  d2 acc = dzero();
                  for (int s = 0; s < ns; ++s) dmacc(acc, dld(rows + ((size_t)c * S + s0 + s) * U + i), Hp[s]);
                  W[i].re += acc.re;
                  W[i].im += acc.im;
                }
                __syncthreads();
              }
            }
          }
          // e = rho p + w (kept in W); alpha = ||r||^2 / Re(p^H e)
          for (int i = tid; i < U; i += kFixThreads) W[i] = d2{f.rho * P[i].re + W[i].re, f.rho * P[i].im + W[i].im};
          __syncthreads();
          wave0_sum(tid < U ? P[tid].re * W[tid].re + P[tid].im * W[tid].im : 0.0, red + 1);
          const double alpha = rr / red[1];
          for (int i = tid; i < U; i += kFixThreads) {
            X[i] = d2{X[i].re + alpha * P[i].re, X[i].im + alpha * P[i].im};
            R[i] = d2{R[i].re - alpha * W[i].re, R[i].im - alpha * W[i].im};
          }
          __syncthreads();
          wave0_sum(tid < U ? R[tid].re * R[tid].re + R[tid].im * R[tid].im : 0.0, red + 2);
          const double rr_new = red[2];
          const double beta = rr_new / rr;
          for (int i = tid; i < U; i += kFixThreads) P[i] = d2{R[i].re + beta * P[i].re, R[i].im + beta * P[i].im};
          __syncthreads();
          if (tid == 0) red[0] = rr_new;
          __syncthreads();
        }
        for (int i = tid; i < U; i += kFixThreads) write_out(f, k, n, i, X[i]);
        __syncthreads();
      }
    }
  }
}

size_t fix64_slot_bytes(int U, int C) { return (size_t)C * U * U * sizeof(d2); }

hipError_t launch_admm_ul_fix64(const FixArgs& f, hipStream_t st) {
  const int U = f.U, CU = f.C * f.U;
  const int TI = (U >= 32) ? 4 : U / 8;
  const int CG = kFixThreads / ((U / TI) * (U / TI));
  const int vec = 3 * CU + U, piv = 2 * CG * U;
  const size_t lds = (size_t)(vec > piv ? vec : piv) * sizeof(d2) + (kListCap + kFixThreads / 64 + 4) * sizeof(int);
  const size_t lds_iter = (size_t)vec * sizeof(d2);
  const dim3 grid((unsigned)f.n_slots), block(kFixThreads), grid2((unsigned)f.n_slots, (unsigned)f.C), block2(256);
  switch (U) {
    case 8: hipLaunchKernelGGL(admm_ul_fix64<8>, grid, block, lds, st, f); break;
    case 16: hipLaunchKernelGGL(admm_ul_fix64<16>, grid, block, lds, st, f); break;
    case 32:
      hipLaunchKernelGGL(admm_ul_fix64<32>, grid, block, lds, st, f);
      if (f.split) {
        hipLaunchKernelGGL(admm_ul_factor64<32>, grid2, block2, 0, st, f);
        hipLaunchKernelGGL(admm_ul_iter64<32>, grid, block, lds_iter, st, f);
      }
      break;
    case 64:
      hipLaunchKernelGGL(admm_ul_fix64<64>, grid, block, lds, st, f);
      if (f.split) {
        hipLaunchKernelGGL(admm_ul_factor64<64>, grid2, block2, 0, st, f);
        hipLaunchKernelGGL(admm_ul_iter64<64>, grid, block, lds_iter, st, f);
      }
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_admm_ul_fix64_batch(const FixBatch& b, int U, int n_slots, hipStream_t st) {
  if (b.n < 1) return hipSuccess;
  int vec = 0, piv = 0;
  for (int i = 0; i < b.n; ++i) {
    const int C = b.f[i].C, TI = (U >= 32) ? 4 : U / 8, CG = kFixThreads / ((U / TI) * (U / TI));
    vec = vec > 3 * C * U + U ? vec : 3 * C * U + U;
    piv = piv > 2 * CG * U ? piv : 2 * CG * U;
  }
  const size_t lds = (size_t)(vec > piv ? vec : piv) * sizeof(d2) + (kListCap + kFixThreads / 64 + 4) * sizeof(int);
  const dim3 grid((unsigned)n_slots), block(kFixThreads);
  switch (U) {
    case 8: hipLaunchKernelGGL(admm_ul_fix64_batch<8>, grid, block, lds, st, b); break;
    case 16: hipLaunchKernelGGL(admm_ul_fix64_batch<16>, grid, block, lds, st, b); break;
    case 32: hipLaunchKernelGGL(admm_ul_fix64_batch<32>, grid, block, lds, st, b); break;
    case 64: hipLaunchKernelGGL(admm_ul_fix64_batch<64>, grid, block, lds, st, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_dcg_ul_fix64(const FixArgs& f, hipStream_t st) {
  const size_t lds = (size_t)(4 * f.U + 1024 + f.C * f.U) * sizeof(d2) + kCgStage * sizeof(c32) + 4 * sizeof(double) +
                    (kListCap + kFixThreads / 64 + 4) * sizeof(int);
  hipLaunchKernelGGL(dcg_ul_fix64, dim3((unsigned)f.n_slots), dim3(kFixThreads), lds, st, f);
  return hipGetLastError();
}

}  // namespace dbp
