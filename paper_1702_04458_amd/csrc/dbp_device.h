// Device-side building blocks shared by the detection and precoding kernels.
//
// Layout convention used throughout: a "problem" is one (subcarrier, antenna
// cluster) pair.  A problem owns a group of G = 64 / P consecutive lanes of a
// wave64 (P problems per wave); lane u of the group owns row u of every
// G x G matrix of that problem and entry u of every length-G vector.  Matrices
// live in registers (one row per lane, fully unrolled loops so that row slots
// are compile-time register indices); vectors that another lane needs are
// broadcast through a per-wave LDS scratch line.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace dbp {

struct alignas(8) c32 {
  float re, im;
};

__device__ __forceinline__ c32 cz() { return c32{0.f, 0.f}; }
__device__ __forceinline__ c32 cadd(c32 a, c32 b) { return c32{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ c32 csub(c32 a, c32 b) { return c32{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ c32 cscale(c32 a, float f) { return c32{a.re * f, a.im * f}; }
__device__ __forceinline__ c32 cmul(c32 a, c32 b) {
  return c32{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// acc += x * y
__device__ __forceinline__ void cmac(c32& acc, c32 x, c32 y) {
  acc.re = fmaf(x.re, y.re, acc.re);
  acc.re = fmaf(-x.im, y.im, acc.re);
  acc.im = fmaf(x.re, y.im, acc.im);
  acc.im = fmaf(x.im, y.re, acc.im);
}
// acc += conj(x) * y
__device__ __forceinline__ void cmacc(c32& acc, c32 x, c32 y) {
  acc.re = fmaf(x.re, y.re, acc.re);
  acc.re = fmaf(x.im, y.im, acc.re);
  acc.im = fmaf(x.re, y.im, acc.im);
  acc.im = fmaf(-x.im, y.re, acc.im);
}
// acc -= x * y
__device__ __forceinline__ void cmsub(c32& acc, c32 x, c32 y) {
  acc.re = fmaf(-x.re, y.re, acc.re);
  acc.re = fmaf(x.im, y.im, acc.re);
  acc.im = fmaf(-x.re, y.im, acc.im);
  acc.im = fmaf(-x.im, y.re, acc.im);
}

// Completes this wave's outstanding LDS operations and stops the compiler from
// moving memory accesses across this point.  LDS instructions of one wave are
// executed in order, so after this a lane sees what other lanes of the same
// wave wrote before it.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Reads N consecutive complex values starting at p (16-byte aligned, N even)
// into r[0..N-1] with 128-bit LDS loads.
template <int N>
__device__ __forceinline__ void lds_read_vec(const c32* p, c32* r) {
  const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    float4 v = q[i];
    r[2 * i] = c32{v.x, v.y};
    r[2 * i + 1] = c32{v.z, v.w};
  }
}

// Sum over the G lanes of a group (G a power of two, groups aligned); every
// lane of the group receives the identical value (the butterfly adds the same
// pair of operands on both partners at every level).
// Within a row of 16 lanes the butterfly uses DPP: quad_perm [1,0,3,2]
// (xor 1), quad_perm [2,3,0,1] (xor 2), row_half_mirror and row_mirror (which
// pair the already uniform quads / half-rows); wider groups add a swap of
// odd and even rows (v_permlane16_swap) and of wave halves
// (v_permlane32_swap), each of which gives a lane its partner's value beside
// its own.
// Every control used here (quad_perm, row mirrors, row_newbcast) reads a valid
// lane of the same row for every lane, so no "old" value is needed and the
// move carries no initialisation of its destination.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <int G>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (G >= 2) v += dpp<0xB1>(v);
  if constexpr (G >= 4) v += dpp<0x4E>(v);
  if constexpr (G >= 8) v += dpp<0x141>(v);
  if constexpr (G >= 16) v += dpp<0x140>(v);
  if constexpr (G >= 32) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  if constexpr (G >= 64) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  return v;
}
template <int G>
__device__ __forceinline__ float group_min(float v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
  return v;
}

// In-place inversion of the Hermitian positive definite matrix whose row u is
// held by lane u of the group, by Gauss-Jordan elimination without pivoting
// (the pivots of an HPD matrix are positive Schur complements).  Block-diagonal
// padding [M 0; 0 I] stays block-diagonal, so groups may pad a smaller system
// with identity rows.
//
// Register layout is rotated so that every register index is a compile-time
// constant while the pivot loop stays rolled: before step k, slot j of a row
// holds column (k + j) mod G; the pivot column is always slot 0, and after the
// step the row shifts left by one slot with the new pivot-column entry
// appended.  After G steps the natural order is restored.
//
// Row k of the partially swept matrix is the conjugate of column k, with the
// sign flipped on columns already swept; each lane publishes its entry of the
// pivot column already conjugated and signed, at the rotated position of the
// column it stands for, so one broadcast line per step gives row k in slot
// order.
template <int G>
__device__ __forceinline__ void gj_invert_rot(c32 (&A)[G], int u, c32* line, int gbase) {
  for (int k = 0; k < G; ++k) {
    const float sg = (u < k) ? -1.f : 1.f;
    // lanes past the matrix (a group wider than G) must not publish
    if (u < G) line[gbase + ((u - k) & (G - 1))] = c32{sg * A[0].re, -sg * A[0].im};
    wave_lds_sync();
    const float p = 1.0f / line[gbase].re;
    const bool me = (u == k);
    const c32 m = me ? c32{-p, 0.f} : c32{A[0].re * p, A[0].im * p};
    const c32 pivot_new = me ? c32{p, 0.f} : c32{-m.re, -m.im};
#pragma unroll
    for (int j0 = 0; j0 < G; j0 += 8) {
      c32 rk[8];
      lds_read_vec<8>(line + gbase + j0, rk);
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const int j = j0 + jj;
        if (j == 0) continue;
        c32 base = me ? cz() : A[j];
        cmsub(base, m, rk[jj]);
        A[j - 1] = base;
      }
    }
    A[G - 1] = pivot_new;
    wave_lds_sync();
  }
}

// The same inversion with lazy row and column scales, fully unrolled (small
// G): the stored matrix S stays Hermitian, so lane u's multiplier for pivot k
// is its own entry conj(S[k][u]) = S[u][k] and only column k is broadcast.
// Sweeping pivot k (value d) leaves row k and column k unchanged except the
// diagonal, which becomes -d, and updates every other entry by
// S[u][j] -= S[u][k] conj(S[j][k]) / d; at the end
// B^{-1}[u][j] = -S[u][j] / (d_u d_j).  Lanes u >= N (a group wider than the
// matrix) take no part.
template <int N>
__device__ __forceinline__ void gj_invert_sym(c32 (&A)[N], int u, c32* line, int gbase) {
  float pvv = 0.f;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (u < N) line[gbase + u] = A[k];
    wave_lds_sync();
    c32 col[N];
#pragma unroll
    for (int j = 0; j < N; j += 2) {
      const float4 v = *reinterpret_cast<const float4*>(line + gbase + j);
      col[j] = c32{v.x, v.y};
      col[j + 1] = c32{v.z, v.w};
    }
    wave_lds_sync();
    const float pv = __builtin_amdgcn_rcpf(col[k].re);
    const bool me = (u == k);
    // t = -S[u][k] / d (zero on the pivot row, which the sweep leaves alone)
    const float tr = me ? 0.f : -A[k].re * pv, ti = me ? 0.f : -A[k].im * pv;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      if (j == k) continue;
      // A[j] += t * conj(col[j])
      A[j].re = fmaf(tr, col[j].re, A[j].re);
      A[j].re = fmaf(ti, col[j].im, A[j].re);
      A[j].im = fmaf(ti, col[j].re, A[j].im);
      A[j].im = fmaf(-tr, col[j].im, A[j].im);
    }
    if (me) {
      A[k].re = -A[k].re;
      pvv = pv;
    }
    // Keep every update of this step in place: without this the compiler
    // defers updates to the entries a later step reads, keeping the broadcast
    // columns of many steps live at once.
#pragma unroll
    for (int j = 0; j < N; ++j) asm volatile("" : "+v"(A[j].re), "+v"(A[j].im));
  }
  if (u < N) line[gbase + u] = c32{pvv, 0.f};
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < N; j += 2) {
    const float4 v = *reinterpret_cast<const float4*>(line + gbase + j);
    const float s0 = -pvv * v.x, s1 = -pvv * v.z;
    A[j].re *= s0;
    A[j].im *= s0;
    A[j + 1].re *= s1;
    A[j + 1].im *= s1;
  }
  wave_lds_sync();
}

// Regularised-matrix inverse of the lane-row layout: the unrolled Hermitian
// sweep for matrices up to 16 x 16 (N a multiple of 8), the rolled rotated
// sweep above for larger ones (code size).
template <int G>
__device__ __forceinline__ void gj_invert(c32 (&A)[G], int u, c32* line, int gbase) {
  if constexpr (G <= 16 && G % 8 == 0)
    gj_invert_sym<G>(A, u, line, gbase);
  else
    gj_invert_rot<G>(A, u, line, gbase);
}

// out = M q for the group matrix M (row u in A), q distributed one entry per
// lane.  A group of 16 lanes is one DPP row: entry v of q is broadcast from
// lane v with row_newbcast; wider groups go through the wave's LDS line.
// Four entries v0 .. v0+3 of the 16-lane matrix-vector product: every FMA
// takes its broadcast operand straight through DPP (row_newbcast), so the
// broadcast costs no separate move.  The surrounding s_nop 1 covers the two
// wait states a DPP read needs after a VALU write of its source (q), and the
// same for any DPP consumer of the results after the block.
#define DBP_MV16_BLOCK(V0, V1, V2, V3)                                                     \
  asm volatile(                                                                          \
      "s_nop 1\n\t"                                                                      \
      "v_fmac_f32_dpp %0, %4, %6 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %0, -%5, %7 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %1, %5, %6 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %1, %4, %7 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %2, %4, %8 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %2, -%5, %9 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %3, %5, %8 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %3, %4, %9 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %0, %4, %10 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %0, -%5, %11 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"  \
      "v_fmac_f32_dpp %1, %5, %10 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %1, %4, %11 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %2, %4, %12 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %2, -%5, %13 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"  \
      "v_fmac_f32_dpp %3, %5, %12 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %3, %4, %13 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"   \
      "s_nop 1"                                                                          \
      : "+v"(a0.re), "+v"(a0.im), "+v"(a1.re), "+v"(a1.im)                               \
      : "v"(q.re), "v"(q.im), "v"(A[V0].re), "v"(A[V0].im), "v"(A[V1].re), "v"(A[V1].im), \
        "v"(A[V2].re), "v"(A[V2].im), "v"(A[V3].re), "v"(A[V3].im))
// The first block of a product: the first product of each accumulator is a
// v_mul (no zeroed accumulators).
#define DBP_MV16_FIRST(V0, V1, V2, V3)                                                     \
  asm volatile(                                                                          \
      "s_nop 1\n\t"                                                                      \
      "v_mul_f32_dpp  %0, %4, %6 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %0, -%5, %7 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_mul_f32_dpp  %1, %5, %6 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %1, %4, %7 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_mul_f32_dpp  %2, %4, %8 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %2, -%5, %9 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_mul_f32_dpp  %3, %5, %8 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %3, %4, %9 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %0, %4, %10 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %0, -%5, %11 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"  \
      "v_fmac_f32_dpp %1, %5, %10 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %1, %4, %11 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %2, %4, %12 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %2, -%5, %13 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"  \
      "v_fmac_f32_dpp %3, %5, %12 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %3, %4, %13 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"   \
      "s_nop 1"                                                                          \
      : "=&v"(a0.re), "=&v"(a0.im), "=&v"(a1.re), "=&v"(a1.im)                               \
      : "v"(q.re), "v"(q.im), "v"(A[V0].re), "v"(A[V0].im), "v"(A[V1].re), "v"(A[V1].im), \
        "v"(A[V2].re), "v"(A[V2].im), "v"(A[V3].re), "v"(A[V3].im))

// acc = sum_v A[v] * q_v with q_v held by lane v of the 16-lane row
__device__ __forceinline__ c32 matvec16(const c32 (&A)[16], c32 q) {
  c32 a0, a1;
  DBP_MV16_FIRST(0, 1, 2, 3);
  DBP_MV16_BLOCK(4, 5, 6, 7);
  DBP_MV16_BLOCK(8, 9, 10, 11);
  DBP_MV16_BLOCK(12, 13, 14, 15);
  return cadd(a0, a1);
}
// The same with conjugated matrix entries: acc = sum_v conj(A[v]) * q_v.
#define DBP_MV16C_BLOCK(V0, V1, V2, V3)                                                    \
  asm volatile(                                                                          \
      "s_nop 1\n\t"                                                                      \
      "v_fmac_f32_dpp %0, %4, %6 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %0, %5, %7 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %1, %5, %6 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %1, -%4, %7 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %2, %4, %8 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %2, %5, %9 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %3, %5, %8 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %3, -%4, %9 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %0, %4, %10 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %0, %5, %11 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %1, %5, %10 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %1, -%4, %11 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"  \
      "v_fmac_f32_dpp %2, %4, %12 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %2, %5, %13 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %3, %5, %12 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %3, -%4, %13 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"  \
      "s_nop 1"                                                                          \
      : "+v"(a0.re), "+v"(a0.im), "+v"(a1.re), "+v"(a1.im)                               \
      : "v"(q.re), "v"(q.im), "v"(A[V0].re), "v"(A[V0].im), "v"(A[V1].re), "v"(A[V1].im), \
        "v"(A[V2].re), "v"(A[V2].im), "v"(A[V3].re), "v"(A[V3].im))
#define DBP_MV16C_FIRST(V0, V1, V2, V3)                                                    \
  asm volatile(                                                                          \
      "s_nop 1\n\t"                                                                      \
      "v_mul_f32_dpp  %0, %4, %6 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %0, %5, %7 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_mul_f32_dpp  %1, %5, %6 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %1, -%4, %7 row_newbcast:" #V0 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_mul_f32_dpp  %2, %4, %8 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %2, %5, %9 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_mul_f32_dpp  %3, %5, %8 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"    \
      "v_fmac_f32_dpp %3, -%4, %9 row_newbcast:" #V1 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %0, %4, %10 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %0, %5, %11 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %1, %5, %10 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %1, -%4, %11 row_newbcast:" #V2 " row_mask:0xf bank_mask:0xf\n\t"  \
      "v_fmac_f32_dpp %2, %4, %12 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %2, %5, %13 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %3, %5, %12 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"   \
      "v_fmac_f32_dpp %3, -%4, %13 row_newbcast:" #V3 " row_mask:0xf bank_mask:0xf\n\t"  \
      "s_nop 1"                                                                          \
      : "=&v"(a0.re), "=&v"(a0.im), "=&v"(a1.re), "=&v"(a1.im)                               \
      : "v"(q.re), "v"(q.im), "v"(A[V0].re), "v"(A[V0].im), "v"(A[V1].re), "v"(A[V1].im), \
        "v"(A[V2].re), "v"(A[V2].im), "v"(A[V3].re), "v"(A[V3].im))

__device__ __forceinline__ c32 matvec16c(const c32 (&A)[16], c32 q) {
  c32 a0, a1;
  DBP_MV16C_FIRST(0, 1, 2, 3);
  DBP_MV16C_BLOCK(4, 5, 6, 7);
  DBP_MV16C_BLOCK(8, 9, 10, 11);
  DBP_MV16C_BLOCK(12, 13, 14, 15);
  return cadd(a0, a1);
}
#undef DBP_MV16C_BLOCK
#undef DBP_MV16C_FIRST

// Rows of a 16 x 16 matrix split over the two 16-lane DPP rows of a 32-lane
// group: lane r of DPP row h holds entries 8h .. 8h+7 of matrix row r (A[i] is
// column 8h + i).  Every lane of the group holds data, where the lane-row
// layout leaves half of a 32-lane group idle in the sweep and the products.
//
// out_r = sum_j M[r][j] q_j with q_j held by lane j of both DPP rows; both
// lanes of row r receive out_r.  The odd DPP rows take q rotated by eight
// lanes (row_ror:8), so that broadcasting lane i gives every lane q_{8h+i}.
__device__ __forceinline__ c32 matvec_split16(const c32 (&A)[8], c32 q) {
  q.re = __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(q.re), __float_as_int(q.re), 0x128, 0xA, 0xF, false));
  q.im = __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(q.im), __float_as_int(q.im), 0x128, 0xA, 0xF, false));
  c32 a0, a1;
  DBP_MV16_FIRST(0, 1, 2, 3);
  DBP_MV16_BLOCK(4, 5, 6, 7);
  c32 acc = cadd(a0, a1);
  // pair sum over the two DPP rows for both parts at once: swapping (re, im)
  // leaves re + re' on the even and im + im' on the odd rows, a second swap
  // hands both to every lane (the same sums, in the same order, as two
  // separate pair sums)
  const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(acc.re), __float_as_uint(acc.im), false, false);
  const float t = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
  const auto tt = __builtin_amdgcn_permlane16_swap(__float_as_uint(t), __float_as_uint(t), false, false);
  return c32{__uint_as_float(tt[0]), __uint_as_float(tt[1])};
}
#undef DBP_MV16_BLOCK
#undef DBP_MV16_FIRST

// gj_invert_sym for a 16 x 16 matrix in the split-row layout above (r = matrix
// row of this lane, h = its DPP row within the group; line = the group's 32
// broadcast slots).  Pivot k publishes column k (slot 16 h_k + r holds S[r][k],
// h_k = k / 8); a lane reads the eight entries S[8h + i][k] of its half and
// its own multiplier S[r][k], and updates its eight entries: 8 complex MACs
// per pivot instead of 16.  Rows past the matrix are identity padding.
__device__ __forceinline__ void gj_invert_sym_split16(c32 (&A)[8], int r, int h, c32* line) {
  float pvv = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int hk = k >> 3, kk = k & 7;
    line[16 * h + r] = A[kk];
    wave_lds_sync();
    c32 col[8];
#pragma unroll
    for (int i = 0; i < 8; i += 2) {
      const float4 v = *reinterpret_cast<const float4*>(line + 16 * hk + 8 * h + i);
      col[i] = c32{v.x, v.y};
      col[i + 1] = c32{v.z, v.w};
    }
    const c32 own = line[16 * hk + r];
    const float d = line[16 * hk + k].re;
    wave_lds_sync();
    const float pv = __builtin_amdgcn_rcpf(d);
    const bool me = (r == k);
    // t = -S[r][k] / d (zero on the pivot row, which the sweep leaves alone)
    const float tr = me ? 0.f : -own.re * pv, ti = me ? 0.f : -own.im * pv;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float ur = tr, ui = ti;
      if (i == kk) {
        // column k itself is left alone (it sits in slot kk of half h_k)
        ur = (h == hk) ? 0.f : tr;
        ui = (h == hk) ? 0.f : ti;
      }
      A[i].re = fmaf(ur, col[i].re, A[i].re);
      A[i].re = fmaf(ui, col[i].im, A[i].re);
      A[i].im = fmaf(ui, col[i].re, A[i].im);
      A[i].im = fmaf(-ur, col[i].im, A[i].im);
    }
    if (me && h == hk) A[kk].re = -A[kk].re;
    if (me) pvv = pv;
#pragma unroll
    for (int i = 0; i < 8; ++i) asm volatile("" : "+v"(A[i].re), "+v"(A[i].im));
  }
  // B^{-1}[r][j] = -S[r][j] / (d_r d_j): the column factors from half 0's slots
  if (h == 0) line[r] = c32{pvv, 0.f};
  wave_lds_sync();
#pragma unroll
  for (int i = 0; i < 8; i += 2) {
    const float4 v = *reinterpret_cast<const float4*>(line + 8 * h + i);
    const float s0 = -pvv * v.x, s1 = -pvv * v.z;
    A[i].re *= s0;
    A[i].im *= s0;
    A[i + 1].re *= s1;
    A[i + 1].im *= s1;
  }
  wave_lds_sync();
}

template <int G>
__device__ __forceinline__ c32 group_matvec(const c32 (&A)[G], c32 q, int u, c32* line, int gbase) {
  if constexpr (G == 16) {
    (void)u;
    (void)line;
    (void)gbase;
    return matvec16(A, q);
  }
  line[gbase + u] = q;
  wave_lds_sync();
  c32 acc0 = cz(), acc1 = cz();
#pragma unroll
  for (int v0 = 0; v0 < G; v0 += 8) {
    c32 qv[8];
    lds_read_vec<8>(line + gbase + v0, qv);
#pragma unroll
    for (int v = 0; v < 8; v += 2) {
      cmac(acc0, A[v0 + v], qv[v]);
      cmac(acc1, A[v0 + v + 1], qv[v + 1]);
    }
  }
  wave_lds_sync();
  (void)u;
  return cadd(acc0, acc1);
}

// Nearest-point slicing of one real dimension of a unit-energy square QAM
// (L levels, kappa = sqrt(2 (M - 1) / 3)): i = clamp(floor((kappa x + L) / 2)),
// ties to the upper level.  The products and sums are rounded individually so
// the decision is reproducible on any IEEE single-precision implementation.
__device__ __forceinline__ int slice_dim(float x, float kappa, int L) {
  float t = __fadd_rn(__fmul_rn(x, kappa), (float)L);
  float f = floorf(t * 0.5f);
  f = fminf(fmaxf(f, 0.f), (float)(L - 1));
  return (int)f;
}

// True when x lies within `guard` (in the slicer's units t = (kappa x + L) / 2,
// where the thresholds are the integers 1 .. L-1) of a decision threshold.
// NaN is never near.
__device__ __forceinline__ bool near_threshold(float x, float kappa, int L, float guard) {
  const float h = __fadd_rn(__fmul_rn(x, kappa), (float)L) * 0.5f;
  const float j = fminf(fmaxf(rintf(h), 1.f), (float)(L - 1));
  return fabsf(h - j) < guard;
}

__device__ __forceinline__ bool nonfinite(c32 v) { return !(isfinite(v.re) && isfinite(v.im)); }

// Status bits of one subcarrier from the per-lane bits of the G lanes of lane
// group g (bit 0 non-finite, bit 1 re-slice, bit 2 poorly conditioned Gram);
// every lane of the wave must call.
template <int G>
__device__ __forceinline__ int group_flags(int fl, int g) {
  const unsigned long long gm = (G == 64) ? ~0ull : (((1ull << G) - 1) << (g * G));
  const unsigned long long m1 = __ballot(fl & 1), m2 = __ballot(fl & 2), m4 = __ballot(fl & 4);
  return ((m1 & gm) ? 1 : 0) | ((m2 & gm) ? 2 : 0) | ((m4 & gm) ? 4 : 0);
}

}  // namespace dbp
