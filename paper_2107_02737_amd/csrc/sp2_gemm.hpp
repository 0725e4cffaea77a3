// Symmetric-output MFMA products for the DNN-SP2 layers (Section II.D,
// Eq. 19-22).  Every product here has a symmetric result, so only the
// upper-triangle tiles are computed and each is mirror-written.  Because the
// operands are symmetric too, column j of B equals row j, so both operand
// panels are row panels with contiguous K -- the layout MFMA wants.
//
//   k_sym_split  16-bit dual representation (Eq. 20-22): per K step three
//                32x32x16 MFMAs  A0 B0 + A0 B1 + A1 B0  (or one for BF16X1),
//                FP32 accumulation.
//   k_sym_f32    FP32 32x32x2 MFMA over up to four K segments
//                sum_s A_s B_s^T (plain FP32 layers, refinement, JVP/VJP).
//
// Both end in the same fused epilogue: out = alpha*acc + beta*C with the
// coefficients given by the layer's branch (S^2 or 2S - S^2) or fixed, the
// mirror write, optional re-split of the result into hi/lo planes for the
// next layer, and FP64 (Tr, ||.||_F^2) partials of the result for the next
// branch/stop decision.
#pragma once

#include "sp2_common.hpp"

namespace sp2 {

enum SplitKind { kBF16X3 = 0, kBF16X1 = 1, kFP16X3 = 2 };

// LDS swizzle of the 16-byte chunk index within a 64-byte row: any 8 or 16
// consecutive rows read at one logical chunk land in distinct banks.
__device__ inline int swz(int row) { return ((row >> 1) & 3) ^ ((row >> 3) & 1); }

struct Epi {
  const float* c;        // addend C (ld = np); read only where needed
  float* out;            // result, leading dimension ld_out
  int64_t ld_out;
  int n_valid;           // rows/cols >= n_valid are not written to out
  int vec_ok;            // out rows are 16-byte aligned (float4 mirror stores)
  uint16_t* hi_out;      // optional hi/lo planes of the result (ld = np)
  uint16_t* lo_out;
  int split_out;         // 0 none, 1 bf16, 2 fp16 scaled
  double* parts_out;     // optional (Tr, ||.||_F^2) pair per work-group
  float alpha, beta;     // used when the launch has no branch
  float oscale;          // scale of the raw accumulator (2^-28 for scaled fp16)
  int np;
};

struct SplitArgs {
  const uint16_t* a_hi;
  const uint16_t* a_lo;
  const uint16_t* b_hi;
  const uint16_t* b_lo;
  Epi epi;
  int nb, ntiles, band;
  Decide dec;
};

struct F32Args {
  const float* a[4];
  const float* b[4];
  int nseg;
  Epi epi;
  int nb, ntiles, band;
  Decide dec;
};

__device__ __forceinline__ void split_value(float v, int kind, uint16_t& h, uint16_t& l) {
  if (kind == 1)
    split_bf16(v, h, l);
  else
    split_fp16s(v, h, l);
}

// Epilogue over the MI x NI 32x32 accumulator blocks of one wave.  MFMA
// 32x32 output layout: accumulator element 4q+e of lane l holds row
// 8q + 4(l/32) + e, column l%32 of the block.
template <int NT, int BM, int TM, int TN, int MI, int NI>
__device__ __forceinline__ void sym_epilogue(const f32x16 (&acc)[MI][NI], const Epi& p, float alpha,
                                    float beta, int ti, int tj, int wm, int wn, int lane,
                                    double* red) {
  const int64_t np = p.np;
  const bool diag = ti == tj;
  double t1 = 0.0, t2 = 0.0;
#pragma clang loop unroll(full)
  for (int mi = 0; mi < MI; ++mi) {
#pragma clang loop unroll(full)
    for (int ni = 0; ni < NI; ++ni) {
      const int cl = wn * TN + ni * 32 + (lane & 31);
      const int64_t gj = int64_t(tj) * BM + cl;
#pragma clang loop unroll(full)
      for (int q = 0; q < 4; ++q) {
        const int rl0 = wm * TM + mi * 32 + 8 * q + 4 * (lane >> 5);
        const int64_t gi0 = int64_t(ti) * BM + rl0;
        float v[4];
        bool keep[4];
#pragma clang loop unroll(full)
        for (int e = 0; e < 4; ++e) {
          keep[e] = !diag || (rl0 + e <= cl);
          float x = acc[mi][ni][4 * q + e] * p.oscale;
          if (keep[e] && beta != 0.0f) x = alpha * x + beta * p.c[(gi0 + e) * np + gj];
          else x = alpha * x;
          v[e] = x;
        }
        // traces of the result: off-diagonal entries count for (i,j) and (j,i)
#pragma clang loop unroll(full)
        for (int e = 0; e < 4; ++e) {
          if (!keep[e]) continue;
          const double d = static_cast<double>(v[e]);
          if (diag && rl0 + e == cl) {
            t1 += d;
            t2 += d * d;
          } else {
            t2 += 2.0 * d * d;
          }
        }
        // FP32 result, direct and mirrored
        const bool full = !diag && gi0 + 3 < p.n_valid && gj < p.n_valid;
        if (full && p.vec_ok) {
#pragma clang loop unroll(full)
          for (int e = 0; e < 4; ++e) p.out[(gi0 + e) * p.ld_out + gj] = v[e];
          *reinterpret_cast<f32x4*>(p.out + gj * p.ld_out + gi0) = f32x4{v[0], v[1], v[2], v[3]};
        } else {
#pragma clang loop unroll(full)
          for (int e = 0; e < 4; ++e) {
            const int64_t gi = gi0 + e;
            if (!keep[e] || gi >= p.n_valid || gj >= p.n_valid) continue;
            p.out[gi * p.ld_out + gj] = v[e];
            if (gi != gj) p.out[gj * p.ld_out + gi] = v[e];
          }
        }
        // dual 16-bit representation of the result for the next layer
        if (p.split_out) {
          uint16_t h[4], l[4];
#pragma clang loop unroll(full)
          for (int e = 0; e < 4; ++e) split_value(v[e], p.split_out, h[e], l[e]);
          if (!diag) {
#pragma clang loop unroll(full)
            for (int e = 0; e < 4; ++e) {
              p.hi_out[(gi0 + e) * np + gj] = h[e];
              p.lo_out[(gi0 + e) * np + gj] = l[e];
            }
            *reinterpret_cast<u32x2*>(p.hi_out + gj * np + gi0) =
                u32x2{uint32_t(h[0]) | (uint32_t(h[1]) << 16), uint32_t(h[2]) | (uint32_t(h[3]) << 16)};
            *reinterpret_cast<u32x2*>(p.lo_out + gj * np + gi0) =
                u32x2{uint32_t(l[0]) | (uint32_t(l[1]) << 16), uint32_t(l[2]) | (uint32_t(l[3]) << 16)};
          } else {
#pragma clang loop unroll(full)
            for (int e = 0; e < 4; ++e) {
              if (!keep[e]) continue;
              const int64_t gi = gi0 + e;
              p.hi_out[gi * np + gj] = h[e];
              p.lo_out[gi * np + gj] = l[e];
              p.hi_out[gj * np + gi] = h[e];
              p.lo_out[gj * np + gi] = l[e];
            }
          }
        }
      }
    }
  }
  if (p.parts_out) {
    block_sum2<NT>(t1, t2, red);
    if (threadIdx.x == 0) {
      p.parts_out[2 * blockIdx.x] = t1;
      p.parts_out[2 * blockIdx.x + 1] = t2;
    }
  }
}

// ---------------------------------------------------------------------------
// 16-bit split product.  Block tile BM x BM, WM x WN waves, wave tile
// (BM/WM) x (BM/WN) of 32x32 MFMA blocks; K staged 32 at a time through a
// double-buffered, swizzled LDS (A hi, A lo, B hi, B lo planes).
// ---------------------------------------------------------------------------

template <int KIND, int BM, int WM, int WN>
__global__ __launch_bounds__(WM* WN* kWave) void k_sym_split(SplitArgs p) {
  constexpr int NT = WM * WN * kWave;
  constexpr int BK = 32;
  constexpr int TM = BM / WM, TN = BM / WN;
  constexpr int MI = TM / 32, NI = TN / 32;
  constexpr bool kLo = KIND != kBF16X1;
  constexpr int NARR = kLo ? 4 : 2;
  constexpr int ARR = BM * BK;          // 16-bit elements per staged plane
  constexpr int CPA = ARR / 8;          // 16-byte chunks per plane
  constexpr int CPT = CPA / NT;         // chunks per thread per plane
  static_assert(CPA % NT == 0, "tile / thread mismatch");
  static_assert(MI >= 1 && NI >= 1, "wave tile too small");

  __shared__ __attribute__((aligned(16))) uint16_t lds[2 * NARR * ARR];
  __shared__ double red[2 * (NT / kWave)];

  const int sign = decide_layer<NT>(p.dec, red);
  if (sign == 0) return;
  float alpha = p.epi.alpha, beta = p.epi.beta;
  if (p.dec.mode != 0) {
    alpha = sign > 0 ? 1.0f : -1.0f;
    beta = sign > 0 ? 0.0f : 2.0f;
  }

  int ti, tj;
  tile_of(xcd_remap(blockIdx.x, p.ntiles), p.nb, p.band, ti, tj);
  const int64_t np = p.epi.np;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int wm = wid / WN, wn = wid % WN;

  // Row panels of A (tile row ti) and B (tile row tj); plane order in LDS:
  // A hi, [A lo], B hi, [B lo].
  const int64_t offa = int64_t(ti) * BM * np, offb = int64_t(tj) * BM * np;
  const uint16_t* g0 = p.a_hi + offa;
  const uint16_t* g1 = kLo ? p.a_lo + offa : p.b_hi + offb;
  const uint16_t* g2 = kLo ? p.b_hi + offb : nullptr;
  const uint16_t* g3 = kLo ? p.b_lo + offb : nullptr;

  // This thread's 16-byte chunks: element offset in the panel and in LDS.
  int64_t goff[CPT];
  int loff[CPT];
#pragma clang loop unroll(full)
  for (int i = 0; i < CPT; ++i) {
    const int q = tid + NT * i;
    const int row = q >> 2, c = q & 3;
    goff[i] = int64_t(row) * np + c * 8;
    loff[i] = row * BK + ((c ^ swz(row)) * 8);
  }

  u32x4 st0[CPT], st1[CPT], st2[CPT], st3[CPT];
  f32x16 acc[MI][NI];
#pragma clang loop unroll(full)
  for (int mi = 0; mi < MI; ++mi)
#pragma clang loop unroll(full)
    for (int ni = 0; ni < NI; ++ni)
#pragma clang loop unroll(full)
      for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;

#define SP2_GLOAD(KT)                                                                   \
  _Pragma("unroll") for (int i = 0; i < CPT; ++i) {                                     \
    const int64_t o = goff[i] + int64_t(KT) * BK;                                       \
    st0[i] = *reinterpret_cast<const u32x4*>(g0 + o);                                   \
    st1[i] = *reinterpret_cast<const u32x4*>(g1 + o);                                   \
    if constexpr (kLo) {                                                                \
      st2[i] = *reinterpret_cast<const u32x4*>(g2 + o);                                 \
      st3[i] = *reinterpret_cast<const u32x4*>(g3 + o);                                 \
    }                                                                                   \
  }
#define SP2_LSTORE(BUF)                                                                 \
  _Pragma("unroll") for (int i = 0; i < CPT; ++i) {                                     \
    uint16_t* d = lds + (BUF) * NARR * ARR + loff[i];                                   \
    *reinterpret_cast<u32x4*>(d) = st0[i];                                              \
    *reinterpret_cast<u32x4*>(d + ARR) = st1[i];                                        \
    if constexpr (kLo) {                                                                \
      *reinterpret_cast<u32x4*>(d + 2 * ARR) = st2[i];                                  \
      *reinterpret_cast<u32x4*>(d + 3 * ARR) = st3[i];                                  \
    }                                                                                   \
  }

  const int KT = static_cast<int>(np / BK);
  SP2_GLOAD(0);
  SP2_LSTORE(0);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < KT) {
      SP2_GLOAD(kt + 1);
    }
    const uint16_t* L = lds + buf * NARR * ARR;
#pragma clang loop unroll(full)
    for (int s = 0; s < 2; ++s) {
      const int c = 2 * s + (lane >> 5);
      u32x4 ah[MI], al[MI], bh[NI], bl[NI];
#pragma clang loop unroll(full)
      for (int mi = 0; mi < MI; ++mi) {
        const int row = wm * TM + mi * 32 + (lane & 31);
        const int off = row * BK + ((c ^ swz(row)) * 8);
        ah[mi] = *reinterpret_cast<const u32x4*>(L + off);
        if constexpr (kLo) al[mi] = *reinterpret_cast<const u32x4*>(L + ARR + off);
      }
#pragma clang loop unroll(full)
      for (int ni = 0; ni < NI; ++ni) {
        const int row = wn * TN + ni * 32 + (lane & 31);
        const int off = row * BK + ((c ^ swz(row)) * 8);
        bh[ni] = *reinterpret_cast<const u32x4*>(L + (kLo ? 2 : 1) * ARR + off);
        if constexpr (kLo) bl[ni] = *reinterpret_cast<const u32x4*>(L + 3 * ARR + off);
      }
#pragma clang loop unroll(full)
      for (int mi = 0; mi < MI; ++mi)
#pragma clang loop unroll(full)
        for (int ni = 0; ni < NI; ++ni) {
          if constexpr (KIND == kFP16X3) {
            const f16x8 a0 = __builtin_bit_cast(f16x8, ah[mi]);
            const f16x8 b0 = __builtin_bit_cast(f16x8, bh[ni]);
            acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0, b0, acc[mi][ni], 0, 0, 0);
            acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                a0, __builtin_bit_cast(f16x8, bl[ni]), acc[mi][ni], 0, 0, 0);
            acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                __builtin_bit_cast(f16x8, al[mi]), b0, acc[mi][ni], 0, 0, 0);
          } else {
            const bf16x8 a0 = __builtin_bit_cast(bf16x8, ah[mi]);
            const bf16x8 b0 = __builtin_bit_cast(bf16x8, bh[ni]);
            acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[mi][ni], 0, 0, 0);
            if constexpr (kLo) {
              acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  a0, __builtin_bit_cast(bf16x8, bl[ni]), acc[mi][ni], 0, 0, 0);
              acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  __builtin_bit_cast(bf16x8, al[mi]), b0, acc[mi][ni], 0, 0, 0);
            }
          }
        }
    }
    if (kt + 1 < KT) {
      SP2_LSTORE(buf ^ 1);
    }
    __syncthreads();
  }
#undef SP2_GLOAD
#undef SP2_LSTORE
  sym_epilogue<NT, BM, TM, TN, MI, NI>(acc, p.epi, alpha, beta, ti, tj, wm, wn, lane, red);
}

// ---------------------------------------------------------------------------
// FP32 product sum_s A_s B_s^T over up to four K segments.  32x32x2 f32
// MFMA; each lane feeds 8 consecutive K values of its row per 16-wide K
// tile (the same K order for A and B, so the sum is unchanged).
// ---------------------------------------------------------------------------

template <int BM, int WM, int WN>
__global__ __launch_bounds__(WM* WN* kWave) void k_sym_f32(F32Args p) {
  constexpr int NT = WM * WN * kWave;
  constexpr int BK = 16;
  constexpr int TM = BM / WM, TN = BM / WN;
  constexpr int MI = TM / 32, NI = TN / 32;
  constexpr int ARR = BM * BK;          // floats per staged operand
  constexpr int CPA = ARR / 4;          // 16-byte chunks per operand
  constexpr int CPT = CPA / NT;
  static_assert(CPA % NT == 0, "tile / thread mismatch");

  __shared__ __attribute__((aligned(16))) float lds[2 * 2 * ARR];
  __shared__ double red[2 * (NT / kWave)];

  const int sign = decide_layer<NT>(p.dec, red);
  if (sign == 0) return;
  float alpha = p.epi.alpha, beta = p.epi.beta;
  if (p.dec.mode != 0) {
    alpha = sign > 0 ? 1.0f : -1.0f;
    beta = sign > 0 ? 0.0f : 2.0f;
  }

  int ti, tj;
  tile_of(xcd_remap(blockIdx.x, p.ntiles), p.nb, p.band, ti, tj);
  const int64_t np = p.epi.np;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int wm = wid / WN, wn = wid % WN;

  int64_t goff[CPT];
  int loff[CPT];
#pragma clang loop unroll(full)
  for (int i = 0; i < CPT; ++i) {
    const int q = tid + NT * i;
    const int row = q >> 2, c = q & 3;
    goff[i] = int64_t(row) * np + c * 4;
    loff[i] = row * BK + ((c ^ swz(row)) * 4);
  }
  u32x4 sa[CPT], sb[CPT];
  f32x16 acc[MI][NI];
#pragma clang loop unroll(full)
  for (int mi = 0; mi < MI; ++mi)
#pragma clang loop unroll(full)
    for (int ni = 0; ni < NI; ++ni)
#pragma clang loop unroll(full)
      for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;

  const int KT = static_cast<int>(np / BK);
  const int IT = KT * p.nseg;
  const int64_t offa = int64_t(ti) * BM * np, offb = int64_t(tj) * BM * np;

#define SP2_GLOAD32(IT_)                                                                \
  {                                                                                     \
    const int s_ = (IT_) / KT, kt_ = (IT_)-s_ * KT;                                     \
    const float* pa_ = (s_ == 0 ? p.a[0] : s_ == 1 ? p.a[1] : s_ == 2 ? p.a[2] : p.a[3]) + offa + kt_ * BK; \
    const float* pb_ = (s_ == 0 ? p.b[0] : s_ == 1 ? p.b[1] : s_ == 2 ? p.b[2] : p.b[3]) + offb + kt_ * BK; \
    _Pragma("unroll") for (int i = 0; i < CPT; ++i) {                                   \
      sa[i] = *reinterpret_cast<const u32x4*>(pa_ + goff[i]);                           \
      sb[i] = *reinterpret_cast<const u32x4*>(pb_ + goff[i]);                           \
    }                                                                                   \
  }
#define SP2_LSTORE32(BUF)                                                               \
  _Pragma("unroll") for (int i = 0; i < CPT; ++i) {                                     \
    float* d = lds + (BUF) * 2 * ARR + loff[i];                                         \
    *reinterpret_cast<u32x4*>(d) = sa[i];                                               \
    *reinterpret_cast<u32x4*>(d + ARR) = sb[i];                                         \
  }

  SP2_GLOAD32(0);
  SP2_LSTORE32(0);
  __syncthreads();
  for (int it = 0; it < IT; ++it) {
    const int buf = it & 1;
    if (it + 1 < IT) {
      SP2_GLOAD32(it + 1);
    }
    const float* LA = lds + (buf * 2) * ARR;
    const float* LB = LA + ARR;
    const int h = lane >> 5;
    f32x4 af[MI][2], bf[NI][2];
#pragma clang loop unroll(full)
    for (int mi = 0; mi < MI; ++mi) {
      const int row = wm * TM + mi * 32 + (lane & 31);
#pragma clang loop unroll(full)
      for (int u = 0; u < 2; ++u)
        af[mi][u] = *reinterpret_cast<const f32x4*>(LA + row * BK + (((2 * h + u) ^ swz(row)) * 4));
    }
#pragma clang loop unroll(full)
    for (int ni = 0; ni < NI; ++ni) {
      const int row = wn * TN + ni * 32 + (lane & 31);
#pragma clang loop unroll(full)
      for (int u = 0; u < 2; ++u)
        bf[ni][u] = *reinterpret_cast<const f32x4*>(LB + row * BK + (((2 * h + u) ^ swz(row)) * 4));
    }
#pragma clang loop unroll(full)
    for (int k = 0; k < 8; ++k)
#pragma clang loop unroll(full)
      for (int mi = 0; mi < MI; ++mi)
#pragma clang loop unroll(full)
        for (int ni = 0; ni < NI; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[mi][k >> 2][k & 3],
                                                             bf[ni][k >> 2][k & 3], acc[mi][ni], 0,
                                                             0, 0);
    if (it + 1 < IT) {
      SP2_LSTORE32(buf ^ 1);
    }
    __syncthreads();
  }
#undef SP2_GLOAD32
#undef SP2_LSTORE32
  sym_epilogue<NT, BM, TM, TN, MI, NI>(acc, p.epi, alpha, beta, ti, tj, wm, wn, lane, red);
}

}  // namespace sp2
