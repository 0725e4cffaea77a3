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
// Both end in the same fused epilogue: out = alpha*acc + beta*C (+ gamma on
// the diagonal) with the coefficients of the layer (S^2, 2S - S^2 or their
// shifted and scaled forms, S_{n+1} = a S_n^2 + b S_n + c I) or fixed, the
// mirror write, optional re-split of the result into hi/lo planes for the
// next layer, and FP64 (Tr, ||.||_F^2) partials of the result for the next
// branch/stop decision.
#pragma once

#include "sp2_common.hpp"

namespace sp2 {

enum SplitKind { kBF16X3 = 0, kBF16X1 = 1, kFP16X3 = 2 };

// Centred operands (c = kPlaneCentre): the split planes of a symmetric X
// hold X - cI, so the raw product of a square is X^2 - 2c X + c^2 I and that
// of a pair (X Y + Y X) is X Y + Y X - 2c Y.  With a branch coefficient
// (a, b, c') a launch flagged kCentredSquare uses beta = b + 2c a and
// gamma = c' - c^2 a, one flagged kCentredPair beta = b + 2c a; without a
// branch the host folds the same terms into alpha, beta and gamma.
// kCentredOut: the planes written for the result hold v - cI (real
// diagonal), as the next layer expects.
constexpr int kCentredSquare = 1, kCentredPair = 2, kCentredOut = 4;

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
  float gamma;           // diagonal term of a launch without branch
  int centring;          // kCentredSquare / kCentredPair / kCentredOut bits
  float oscale;          // scale of the raw accumulator (2^-28 for scaled fp16)
  int np;
  int mirror_out;        // 1: FP32 result in both triangles; 0: upper triangle only
  int n_diag;            // the layer's c I term reaches diagonal entries < n_diag
                         // (the real rows: padding stays exactly 0)
};

// Work decomposition of one product launch.  Work-groups [0, nfull) each
// compute a whole tile (logical tiles 0 .. nfull-1).  The remaining tiles
// ("tail", the last partial round of the machine) are split along K into
// nsplit pieces, one per work-group; every piece stores its FP32 partial
// accumulator, and k_split_tail, launched next on the same stream, sums
// the pieces in a fixed order and runs the epilogue.  No work-group ever
// waits for another.
struct Decomp {
  int nb, ntiles, band;
  int nfull;        // whole-tile work-groups
  int nsplit;       // K pieces per tail tile (1: no tail)
  float* partial;   // (ntiles - nfull) * nsplit accumulators of NT * MI*NI*16 floats
};

struct SplitArgs {
  const uint16_t* a_hi;
  const uint16_t* a_lo;
  const uint16_t* b_hi;
  const uint16_t* b_lo;
  // second K segment (two-segment launches: A = [A1|A2], B = [B1|B2])
  const uint16_t* a2_hi;
  const uint16_t* a2_lo;
  const uint16_t* b2_hi;
  const uint16_t* b2_lo;
  Epi epi;
  Decomp dc;
  Decide dec;
};

struct F32Args {
  const float* a[4];
  const float* b[4];
  int nseg;
  Epi epi;
  Decomp dc;
  Decide dec;
};

// Tile and K range [k0, k1) (in K steps out of ksteps) of this work-group.
__device__ __forceinline__ void work_of(const Decomp& dc, int ksteps, int& tile, int& ti, int& tj,
                                        int& k0, int& k1, int& tail, int& piece) {
  const int b = blockIdx.x;
  if (b < dc.nfull) {
    tile = xcd_remap(b, dc.nfull);
    k0 = 0;
    k1 = ksteps;
    tail = -1;
    piece = 0;
  } else {
    const int j = b - dc.nfull;
    tail = j / dc.nsplit;
    piece = j - tail * dc.nsplit;
    tile = dc.nfull + tail;
    k0 = static_cast<int>((int64_t(ksteps) * piece) / dc.nsplit);
    k1 = static_cast<int>((int64_t(ksteps) * (piece + 1)) / dc.nsplit);
  }
  tile_of(tile, dc.nb, dc.band, ti, tj);
}

__device__ __forceinline__ void split_value(float v, int kind, uint16_t& h, uint16_t& l) {
  if (kind == 1)
    split_bf16(v, h, l);
  else
    split_fp16s(v, h, l);
}

// ---------------------------------------------------------------------------
// LDS-staged epilogue of the 256 x 256 split tile (4 waves of 128 x 128).
// One round per 128-row half: the two waves that own the half dump their
// accumulators into a [128][257] FP32 LDS image (odd row stride: a column
// read by consecutive lanes and a row read by consecutive lanes are both
// bank-conflict free).  Then four passes over the image, each mapping
// lanes so that every global access of a wave is contiguous: (A) upper
// elements, v = alpha acc + beta C, FP32 result and FP64 traces, v written
// back; (B) upper elements as hi/lo planes, lane = row; (C) the mirrored
// FP32 result, lane = image row; (D) the mirrored planes, lane = image
// column.  On diagonal tiles only elements on or above the diagonal are
// taken, each also mirrored, so the result is exactly symmetric.
// ---------------------------------------------------------------------------

constexpr int kEpiLd = 257;   // padded LDS row (floats)

// Elements [first, last) of 8 consecutive plane elements starting at
// offset o (one chunk row) as the hi/lo pair.
__device__ __forceinline__ void store_planes8(const Epi& p, int64_t o, const float (&v)[8], int first,
                                              int last) {
  uint16_t h[8], l[8];
#pragma clang loop unroll(full)
  for (int e = 0; e < 8; ++e) split_value(v[e], p.split_out, h[e], l[e]);
  if (first == 0 && last == 8) {
    u32x4 hv, lv;
#pragma clang loop unroll(full)
    for (int e = 0; e < 4; ++e) {
      hv[e] = uint32_t(h[2 * e]) | (uint32_t(h[2 * e + 1]) << 16);
      lv[e] = uint32_t(l[2 * e]) | (uint32_t(l[2 * e + 1]) << 16);
    }
    *reinterpret_cast<u32x4*>(p.hi_out + o) = hv;
    *reinterpret_cast<u32x4*>(p.lo_out + o) = lv;
  } else {
#pragma clang loop unroll(full)
    for (int e = 0; e < 8; ++e)
      if (e >= first && e < last) {
        p.hi_out[o + e] = h[e];
        p.lo_out[o + e] = l[e];
      }
  }
}

// The four passes over an image of H rows of one 256 x 256 tile (tile rows
// hr .. hr+H-1), 256 threads.  as = alpha * output scale; gamma is added to
// diagonal entries below p.n_diag.  Adds the trace contributions of the
// upper elements to (t1, t2).
template <int H>
__device__ __forceinline__ void epilogue_passes(const Epi& p, float as, float beta, float gamma,
                                                int ti, int tj, int hr, float* img, double& t1,
                                                double& t2) {
  static_assert(H == 16 || H == 32 || H == 128, "image height");
  constexpr int BM = 256, S = kEpiLd, G = BM / H;
  const int64_t np = p.np;
  const bool diag = ti == tj;
  const int t = threadIdx.x, w = t / kWave, lane = t & (kWave - 1);
  const int64_t R0 = int64_t(ti) * BM, C0 = int64_t(tj) * BM;   // tile origin
  const int64_t nv = p.n_valid;
  // Pass A, upper elements: v = alpha acc + beta C (+ gamma on the real
  // diagonal), FP32 result, traces;
  // v goes back into the image for the other passes (C is symmetric, so
  // the mirrored element takes the same v).  Lane = column (4 of them),
  // wave = every 4th row, 4 rows per step: every access is 64 consecutive
  // floats and 16 loads are in flight per lane.
  for (int rb = 0; rb < H / 4; rb += 4) {
    float v[4][4], cv[4][4];
#pragma clang loop unroll(full)
    for (int i = 0; i < 4; ++i)
#pragma clang loop unroll(full)
      for (int j = 0; j < 4; ++j) v[i][j] = img[(w + 4 * (rb + i)) * S + lane + 64 * j];
    if (beta != 0.0f) {
#pragma clang loop unroll(full)
      for (int i = 0; i < 4; ++i)
#pragma clang loop unroll(full)
        for (int j = 0; j < 4; ++j)
          cv[i][j] = p.c[(R0 + hr + w + 4 * (rb + i)) * np + C0 + lane + 64 * j];
#pragma clang loop unroll(full)
      for (int i = 0; i < 4; ++i)
#pragma clang loop unroll(full)
        for (int j = 0; j < 4; ++j) v[i][j] = as * v[i][j] + beta * cv[i][j];
    } else {
#pragma clang loop unroll(full)
      for (int i = 0; i < 4; ++i)
#pragma clang loop unroll(full)
        for (int j = 0; j < 4; ++j) v[i][j] = as * v[i][j];
    }
    const float oc = (p.centring & kCentredOut) ? kPlaneCentre : 0.0f;
#pragma clang loop unroll(full)
    for (int i = 0; i < 4; ++i) {
      const int rh = w + 4 * (rb + i), rl = hr + rh;
      const int64_t row = R0 + rl;
#pragma clang loop unroll(full)
      for (int j = 0; j < 4; ++j) {
        const int c = lane + 64 * j;
        const bool up = !diag || c >= rl;   // below the diagonal: mirrored from above
        const bool on = diag && c == rl;
        const bool real_on = on && row < p.n_diag;
        if (real_on) v[i][j] += gamma;
        // the image feeds the plane passes (centred) and the mirrored FP32
        // pass (off the diagonal only, where the two agree)
        img[rh * S + c] = real_on ? v[i][j] - oc : v[i][j];
        const double d = up ? static_cast<double>(v[i][j]) : 0.0;
        t1 += on ? d : 0.0;
        t2 += (on ? 1.0 : 2.0) * d * d;     // each unordered pair counted once
        const int64_t col = C0 + c;
        if (p.out && up && row < nv && col < nv) p.out[row * p.ld_out + col] = v[i][j];
      }
    }
  }
  __syncthreads();
  // Pass B, upper elements as hi/lo planes: thread = row (consecutive rows:
  // one contiguous store per chunk of 8 columns); the G thread groups take
  // interleaved chunks.
  if (p.split_out) {
    const int rh = t % H, rl = hr + rh;
    const int64_t row = R0 + rl;
    for (int k8 = t / H; k8 < BM / 8; k8 += 2 * G) {
      float v[2][8];
#pragma clang loop unroll(full)
      for (int u = 0; u < 2; ++u)
#pragma clang loop unroll(full)
        for (int e = 0; e < 8; ++e) v[u][e] = img[rh * S + (k8 + G * u) * 8 + e];
#pragma clang loop unroll(full)
      for (int u = 0; u < 2; ++u) {
        const int c0 = (k8 + G * u) * 8;
        const int first = !diag ? 0 : (rl <= c0 ? 0 : (rl >= c0 + 8 ? 8 : rl - c0));
        store_planes8(p, plane_off(row, C0 + c0, np), v[u], first, 8);
      }
    }
  }
  // Pass C, mirrored FP32: output row C0 + cl, columns R0 + hr + r; thread =
  // image row (consecutive output columns per store), 8 columns per step.
  if (p.out && p.mirror_out) {
    const int r = t % H, rl = hr + r;
    const int64_t col = R0 + rl;
    const int cb = (t / H) * H;
    for (int cl0 = cb; cl0 < cb + H; cl0 += 8) {
      float v[8];
#pragma clang loop unroll(full)
      for (int e = 0; e < 8; ++e) v[e] = img[r * S + cl0 + e];
#pragma clang loop unroll(full)
      for (int e = 0; e < 8; ++e) {
        const int cl = cl0 + e;
        const int64_t row = C0 + cl;
        if ((!diag || rl < cl) && row < nv && col < nv) p.out[row * p.ld_out + col] = v[e];
      }
    }
  }
  // Pass D, mirrored planes: thread = output row C0 + cl (consecutive rows
  // per chunk store), chunks of 8 image rows.
  if (p.split_out) {
    const int cl = t;
    const int64_t row = C0 + cl;
    for (int k8 = 0; k8 < H / 8; k8 += 2) {
      float v[2][8];
#pragma clang loop unroll(full)
      for (int u = 0; u < 2; ++u)
#pragma clang loop unroll(full)
        for (int e = 0; e < 8; ++e) v[u][e] = img[((k8 + u) * 8 + e) * S + cl];
#pragma clang loop unroll(full)
      for (int u = 0; u < 2; ++u) {
        const int rl0 = hr + (k8 + u) * 8;
        const int last = !diag ? 8 : (rl0 + 8 <= cl ? 8 : (rl0 >= cl ? 0 : cl - rl0));
        store_planes8(p, plane_off(row, R0 + rl0, np), v[u], 0, last);
      }
    }
  }
}

// Epilogue of a 256x256 tile through LDS.  MFMA 32x32 output layout:
// accumulator element 4q+e of lane l holds row 8q + 4(l/32) + e, column
// l%32 of its block.  The two waves of each 128-row half dump their
// accumulators into the [128][257] image, then epilogue_passes finish it.
template <int NT, int MI, int NI>
__device__ __forceinline__ void sym_epilogue_lds(const f32x16 (&acc)[MI][NI], const Epi& p, float alpha,
                                                 float beta, float gamma, int ti, int tj, int wm,
                                                 int wn, int lane, double* red, int tile, float* img) {
  static_assert(NT == 256, "four waves");
  constexpr int TM = 128, TN = 128, S = kEpiLd;
  const float as = alpha * p.oscale;   // exact: oscale is a power of two
  double t1 = 0.0, t2 = 0.0;
  for (int half = 0; half < 2; ++half) {
    __syncthreads();   // the image (and before it, the operand ring) is free
    if (wm == half) {
#pragma clang loop unroll(full)
      for (int mi = 0; mi < MI; ++mi)
#pragma clang loop unroll(full)
        for (int ni = 0; ni < NI; ++ni) {
          const int cl = wn * TN + ni * 32 + (lane & 31);
#pragma clang loop unroll(full)
          for (int q = 0; q < 4; ++q)
#pragma clang loop unroll(full)
            for (int e = 0; e < 4; ++e)
              img[(mi * 32 + 8 * q + 4 * (lane >> 5) + e) * S + cl] = acc[mi][ni][4 * q + e];
        }
    }
    __syncthreads();
    epilogue_passes<TM>(p, as, beta, gamma, ti, tj, half * TM, img, t1, t2);
  }
  if (p.parts_out) {
    block_sum2<NT>(t1, t2, red);
    if (threadIdx.x == 0) {
      p.parts_out[2 * tile] = t1;
      p.parts_out[2 * tile + 1] = t2;
    }
  }
}

// Split-K tail: a piece stores its raw accumulator (layout: 16 floats per
// block, 4 at a time, thread-minor) for k_split_tail to sum.
template <int NT, int MI, int NI>
__device__ __forceinline__ void store_piece(const f32x16 (&acc)[MI][NI], const Decomp& dc, int tail,
                                            int piece) {
  float* mine = dc.partial + (int64_t(tail) * dc.nsplit + piece) * (NT * MI * NI * 16);
#pragma clang loop unroll(full)
  for (int mi = 0; mi < MI; ++mi)
#pragma clang loop unroll(full)
    for (int ni = 0; ni < NI; ++ni)
#pragma clang loop unroll(full)
      for (int r4 = 0; r4 < 4; ++r4) {
        const int v = (mi * NI + ni) * 4 + r4;
        *reinterpret_cast<f32x4*>(mine + (int64_t(v) * NT + threadIdx.x) * 4) =
            f32x4{acc[mi][ni][4 * r4], acc[mi][ni][4 * r4 + 1], acc[mi][ni][4 * r4 + 2],
                  acc[mi][ni][4 * r4 + 3]};
      }
}

// ---------------------------------------------------------------------------
// 16-bit split product.  256 x 256 output tile per work-group of 4 waves
// (2 x 2, each 128 x 128 = 4 x 4 blocks of 32x32 MFMA), one wave per SIMD
// with the 256 accumulators in AGPRs.  K advances 16 at a time through a
// four-slot LDS ring (32 KB per slot: A hi, A lo, B hi, B lo) filled by
// global_load_lds DMA straight from the K-tiled planes, four K steps ahead:
// while one slot is consumed, up to three (96 KB) are in flight, and each
// wave waits only for the oldest of its outstanding copies.  Fragments are
// double buffered in registers: one barrier per K step.  A wave issues its
// copies for K step k + 4 between the MFMAs of the first product of step k
// (one copy after every second MFMA), and the LDS reads of step k + 1
// between those of the other two products (one read per two MFMAs), so its
// instruction stream keeps the matrix pipe fed (with one wave per SIMD,
// a copy or read issued alone would leave the pipe idle).
// ---------------------------------------------------------------------------

// One 16-byte chunk per lane from global memory into LDS at m0 + 16 * lane.
// Issued as inline assembly so that the compiler does not wait on it before
// every LDS read; the kernel waits for the DMA explicitly (vmcnt) before
// the barrier that publishes a slot.
__device__ __forceinline__ void dma_chunk(uint32_t off, const void* base, uint32_t m0) {
  asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %0, %1" ::"v"(off), "s"(base), "s"(m0)
               : "memory", "m0");
}

__device__ __forceinline__ void wait_vmem_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Wait until at most `later` K steps of this wave's DMA (C copies each) are
// outstanding, and for its own LDS reads.
template <int C>
__device__ __forceinline__ void wait_ring(int later) {
  static_assert(C == 4 || C == 8, "copies per K step");
  if (later >= 3) {
    if constexpr (C == 8) asm volatile("s_waitcnt vmcnt(24) lgkmcnt(0)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(12) lgkmcnt(0)" ::: "memory");
  } else if (later == 2) {
    if constexpr (C == 8) asm volatile("s_waitcnt vmcnt(16) lgkmcnt(0)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(8) lgkmcnt(0)" ::: "memory");
  } else if (later == 1) {
    if constexpr (C == 8) asm volatile("s_waitcnt vmcnt(8) lgkmcnt(0)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(4) lgkmcnt(0)" ::: "memory");
  } else {
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
  }
}

template <int KIND, int NSEG = 1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_sym_split(SplitArgs p) {
  static_assert(NSEG == 1 || NSEG == 2, "one or two K segments");
  constexpr int BM = 256, NT = 256, BK = 16, NS = 4, MI = 4, NI = 4, TM = 128, TN = 128;
  constexpr bool kLo = KIND != kBF16X1;
  constexpr int PLANE_B = BM * BK * 2;   // bytes of one plane per K step (8 KB)
  constexpr int SLOT_B = 4 * PLANE_B;    // A hi, A lo, B hi, B lo
  static_assert(NS * SLOT_B <= 128 * kEpiLd * 4, "ring exceeds the LDS image");
  // four operand slots (128 KB), reused as the [128][257] FP32 epilogue image
  __shared__ __attribute__((aligned(1024))) uint16_t lds[128 * kEpiLd * 2];
  __shared__ double red[2 * (NT / kWave)];

  const LayerCoef cf = decide_layer<NT>(p.dec, red);
  if (cf.sign == 0) return;
  float alpha = p.epi.alpha, beta = p.epi.beta, gamma = p.epi.gamma;
  if (p.dec.mode != 0) {
    const int cn = p.epi.centring;
    alpha = cf.a;
    beta = (cn & (kCentredSquare | kCentredPair)) ? cf.b + 2.0f * kPlaneCentre * cf.a : cf.b;
    gamma = (cn & kCentredSquare) ? cf.c - kPlaneCentre * kPlaneCentre * cf.a : cf.c;
  }
  const int64_t np = p.epi.np;
  const int KT = static_cast<int>(np / BK);
  int tile, ti, tj, kb, ke, tail, piece;
  work_of(p.dc, NSEG * KT / 2, tile, ti, tj, kb, ke, tail, piece);
  kb *= 2;
  ke *= 2;
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int wm = w >> 1, wn = w & 1;

  // DMA: plane block (panel P, K step kt) starts at element (P*KT + kt)*4096;
  // this wave copies the 1 KB pieces (i*4 + w), i = 0..1, of each plane.
  // K steps KT..2KT-1 of a two-segment launch read the second planes.
  const int64_t pa = int64_t(ti) * KT * 4096, pb = int64_t(tj) * KT * 4096;
  const uint16_t* ga_hi = p.a_hi + pa;
  const uint16_t* ga_lo = kLo ? p.a_lo + pa : nullptr;
  const uint16_t* gb_hi = p.b_hi + pb;
  const uint16_t* gb_lo = kLo ? p.b_lo + pb : nullptr;
  const uint16_t* ga2_hi = NSEG == 2 ? p.a2_hi + pa : nullptr;
  const uint16_t* ga2_lo = NSEG == 2 && kLo ? p.a2_lo + pa : nullptr;
  const uint16_t* gb2_hi = NSEG == 2 ? p.b2_hi + pb : nullptr;
  const uint16_t* gb2_lo = NSEG == 2 && kLo ? p.b2_lo + pb : nullptr;
  // Plane sources of K step KTI: gah_, gal_, gbh_, gbl_ at that K step.
#define SP2_SRC(KTI)                                                                      \
  const int sg_ = (NSEG == 2 && (KTI) >= KT) ? 1 : 0;                                     \
  const int64_t kofs_ = int64_t((KTI) - sg_ * KT) * 4096;                                 \
  const uint16_t* gah_ = (sg_ ? ga2_hi : ga_hi) + kofs_;                                  \
  const uint16_t* gal_ = kLo ? (sg_ ? ga2_lo : ga_lo) + kofs_ : nullptr;                  \
  const uint16_t* gbh_ = (sg_ ? gb2_hi : gb_hi) + kofs_;                                  \
  const uint16_t* gbl_ = kLo ? (sg_ ? gb2_lo : gb_lo) + kofs_ : nullptr;
  const uint32_t lds0 = static_cast<uint32_t>(
      reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) uint16_t*)(lds)));
  // Per K step every wave issues kCopies copies (2 per plane).
  constexpr int kCopies = kLo ? 8 : 4;
#define SP2_DMA_STAGE(SLOT, KTI)                                                          \
  {                                                                                       \
    SP2_SRC(KTI)                                                                          \
    const uint32_t m0s_ = lds0 + (SLOT) * SLOT_B + w * 1024;                              \
    _Pragma("clang loop unroll(full)") for (int i = 0; i < 2; ++i) {                      \
      const uint32_t off_ = static_cast<uint32_t>(((i * 4 + w) * 64 + lane) * 16);        \
      dma_chunk(off_, gah_, m0s_ + 0 * PLANE_B + i * 4096);                               \
      dma_chunk(off_, gbh_, m0s_ + 2 * PLANE_B + i * 4096);                               \
      if constexpr (kLo) {                                                                \
        dma_chunk(off_, gal_, m0s_ + 1 * PLANE_B + i * 4096);                             \
        dma_chunk(off_, gbl_, m0s_ + 3 * PLANE_B + i * 4096);                             \
      }                                                                                   \
    }                                                                                     \
  }

  // Fragment addresses (bytes within a slot): row r of a 32-row block,
  // h = lane/32 reads column chunk h (16 bytes per row, chunk h at +4 KB).
  const int r = lane & 31, h = lane >> 5;
  const int fa = h * 4096 + (wm * TM + r) * 16;
  const int fb = h * 4096 + (wn * TN + r) * 16;
  const char* L = reinterpret_cast<const char*>(lds);

  f32x16 acc[MI][NI];
#pragma clang loop unroll(full)
  for (int mi = 0; mi < MI; ++mi)
#pragma clang loop unroll(full)
    for (int ni = 0; ni < NI; ++ni)
#pragma clang loop unroll(full)
      for (int q = 0; q < 16; ++q) acc[mi][ni][q] = 0.0f;

  u32x4 Ah0[MI], Al0[MI], Bh0[NI], Bl0[NI];
  u32x4 Ah1[MI], Al1[MI], Bh1[NI], Bl1[NI];

#define SP2_FRAG(AH, AL, BH, BL, SLOT)                                                    \
  {                                                                                       \
    const char* S_ = L + (SLOT) * SLOT_B;                                                 \
    _Pragma("clang loop unroll(full)") for (int mi = 0; mi < MI; ++mi)                    \
      AH[mi] = *reinterpret_cast<const u32x4*>(S_ + 0 * PLANE_B + fa + mi * 512);         \
    _Pragma("clang loop unroll(full)") for (int ni = 0; ni < NI; ++ni)                    \
      BH[ni] = *reinterpret_cast<const u32x4*>(S_ + 2 * PLANE_B + fb + ni * 512);         \
    if constexpr (kLo) {                                                                  \
      _Pragma("clang loop unroll(full)") for (int ni = 0; ni < NI; ++ni)                  \
        BL[ni] = *reinterpret_cast<const u32x4*>(S_ + 3 * PLANE_B + fb + ni * 512);       \
      _Pragma("clang loop unroll(full)") for (int mi = 0; mi < MI; ++mi)                  \
        AL[mi] = *reinterpret_cast<const u32x4*>(S_ + 1 * PLANE_B + fa + mi * 512);       \
    }                                                                                     \
  }

#define SP2_MFMA1(X, Y)                                                                   \
  _Pragma("clang loop unroll(full)") for (int mi = 0; mi < MI; ++mi)                      \
  _Pragma("clang loop unroll(full)") for (int ni = 0; ni < NI; ++ni) {                    \
    if constexpr (KIND == kFP16X3)                                                        \
      acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_f16(                               \
          __builtin_bit_cast(f16x8, X[mi]), __builtin_bit_cast(f16x8, Y[ni]), acc[mi][ni], 0, 0, 0); \
    else                                                                                  \
      acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(                              \
          __builtin_bit_cast(bf16x8, X[mi]), __builtin_bit_cast(bf16x8, Y[ni]), acc[mi][ni], 0, 0, 0); \
  }
  // Per K step, hi*hi first for every block, then hi*lo, then lo*hi: an
  // accumulator is revisited only every 16 MFMAs.
  // First product of a K step with the refill of slot SLOT (K step KTI)
  // woven in: one copy after every second MFMA (every fourth for one plane
  // pair), so that the address arithmetic and copy issue of one wave run
  // while its matrix pipe is busy.  sched_barrier keeps the order as written.
#define SP2_MFMA1_DMA(X, Y, SLOT, KTI)                                                    \
  {                                                                                       \
    SP2_SRC(KTI)                                                                          \
    const uint32_t m0s_ = lds0 + (SLOT) * SLOT_B + w * 1024;                              \
    _Pragma("clang loop unroll(full)") for (int mi = 0; mi < MI; ++mi)                    \
    _Pragma("clang loop unroll(full)") for (int ni = 0; ni < NI; ++ni) {                  \
      if constexpr (KIND == kFP16X3)                                                      \
        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_f16(                             \
            __builtin_bit_cast(f16x8, X[mi]), __builtin_bit_cast(f16x8, Y[ni]), acc[mi][ni], 0, 0, 0); \
      else                                                                                \
        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(                            \
            __builtin_bit_cast(bf16x8, X[mi]), __builtin_bit_cast(bf16x8, Y[ni]), acc[mi][ni], 0, 0, 0); \
      constexpr int kEvery_ = 16 / kCopies;                                               \
      const int j_ = mi * NI + ni;                                                        \
      if (j_ % kEvery_ == kEvery_ - 1) {                                                  \
        const int c_ = j_ / kEvery_, i_ = c_ & 1, pl_ = c_ >> 1;                          \
        const uint32_t off_ = static_cast<uint32_t>(((i_ * 4 + w) * 64 + lane) * 16);     \
        const uint16_t* g_ = pl_ == 0 ? gah_ : pl_ == 1 ? gbh_ : pl_ == 2 ? gal_ : gbl_;  \
        const int lp_ = pl_ == 0 ? 0 : pl_ == 1 ? 2 : pl_ == 2 ? 1 : 3;                   \
        dma_chunk(off_, g_, m0s_ + lp_ * PLANE_B + i_ * 4096);                            \
      }                                                                                   \
      __builtin_amdgcn_sched_barrier(0);                                                  \
    }                                                                                     \
  }
  // Second and third products of a K step, with the LDS reads of the next
  // K step interleaved 1:2.
#define SP2_MFMA23(CAH, CAL, CBH, CBL)                                                    \
  if constexpr (kLo) {                                                                    \
    SP2_MFMA1(CAH, CBL);                                                                  \
    SP2_MFMA1(CAL, CBH);                                                                  \
    _Pragma("clang loop unroll(full)") for (int g = 0; g < 16; ++g) {                    \
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);                                  \
      __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);                                  \
    }                                                                                     \
  }
  // One K step: K step K is in registers (CUR); publish K + 1, refill the
  // slot K came from with K + 4, compute K while reading K + 1 into NXT.
  // Copies are issued in every step, so the wait is the same in every step:
  // in the last four steps of a range they re-copy step ke - 1 into slots
  // that are never read again (and the NXT reads after the last step fetch
  // such a slot); the ring drains before the epilogue reuses the LDS.
#define SP2_STEP(K, CAH, CAL, CBH, CBL, NAH, NAL, NBH, NBL)                               \
  {                                                                                       \
    const int k_ = (K);                                                                   \
    wait_ring<kCopies>(2);                                                                \
    __syncthreads();                                                                      \
    SP2_MFMA1_DMA(CAH, CBH, (k_ - kb) & (NS - 1), min(k_ + 4, ke - 1));                   \
    SP2_FRAG(NAH, NAL, NBH, NBL, (k_ + 1 - kb) & (NS - 1));                               \
    SP2_MFMA23(CAH, CAL, CBH, CBL);                                                       \
  }

  // K ranges are whole pairs of K steps (work_of splits in units of 32).
#pragma clang loop unroll(full)
  for (int s = 0; s < NS; ++s) SP2_DMA_STAGE(s, min(kb + s, ke - 1));
  wait_ring<kCopies>(3);
  __syncthreads();
  SP2_FRAG(Ah0, Al0, Bh0, Bl0, 0);
  for (int kt = kb; kt < ke; kt += 2) {
    SP2_STEP(kt, Ah0, Al0, Bh0, Bl0, Ah1, Al1, Bh1, Bl1);
    SP2_STEP(kt + 1, Ah1, Al1, Bh1, Bl1, Ah0, Al0, Bh0, Bl0);
  }
  wait_vmem_all();
  __syncthreads();
#undef SP2_SRC
#undef SP2_DMA_STAGE
#undef SP2_FRAG
#undef SP2_MFMA1
#undef SP2_MFMA1_DMA
#undef SP2_MFMA23
#undef SP2_STEP
  if (tail >= 0) {   // summed and finished by k_split_tail
    store_piece<NT, MI, NI>(acc, p.dc, tail, piece);
    return;
  }
  sym_epilogue_lds<NT, MI, NI>(acc, p.epi, alpha, beta, gamma, ti, tj, wm, wn, lane, red, tile,
                               reinterpret_cast<float*>(lds));
}

// ---------------------------------------------------------------------------
// Split-K tail of k_sym_split and k_sym_f32, spread over the machine:
// work-group (tail tile, strip s) sums the nsplit stored pieces of rows
// 16 s .. 16 s + 15 of the tile in piece order (so the result does not depend
// on which piece finished last) and runs the epilogue passes on that strip;
// 16 strips per tile keep the work-groups many and small enough to spread
// evenly over the CUs.  The branch is the one the layer's product launch
// recorded.  Trace partials go to parts_out[nfull + 16 * tail + s].
// ---------------------------------------------------------------------------
constexpr int kTailStrips = 16;
__global__ __launch_bounds__(256) void k_split_tail(SplitArgs p) {
  constexpr int NT = 256, H = 16, S = kEpiLd, NI = 4;
  __shared__ float img[H * S];
  __shared__ double red[2 * (NT / kWave)];
  const LayerCoef cf = recorded_coef(p.dec);
  if (cf.sign == 0) return;
  float alpha = p.epi.alpha, beta = p.epi.beta, gamma = p.epi.gamma;
  if (p.dec.mode != 0) {
    const int cn = p.epi.centring;
    alpha = cf.a;
    beta = (cn & (kCentredSquare | kCentredPair)) ? cf.b + 2.0f * kPlaneCentre * cf.a : cf.b;
    gamma = (cn & kCentredSquare) ? cf.c - kPlaneCentre * kPlaneCentre * cf.a : cf.c;
  }
  const Decomp& dc = p.dc;
  const int tail = blockIdx.x / kTailStrips, s = blockIdx.x % kTailStrips;
  const int tile = dc.nfull + tail;
  int ti, tj;
  tile_of(tile, dc.nb, dc.band, ti, tj);
  // Strip s lies in the 128-row half wm = s / 8, 32-row block mi = (s / 2) % 4,
  // accumulator rows 8 r4 + 4 (lane / 32) + e of that block with
  // r4 in {2 hf, 2 hf + 1}, hf = s % 2.  Item j = t + 256 k (k = 0..3): wave
  // wn = j / 512, block (ni, r4 - 2 hf) = (j % 512) / 64, lane j % 64 --
  // consecutive threads read consecutive 16-byte pieces of an accumulator.
  const int wm = s >> 3, mi = (s >> 1) & 3, hf = s & 1, t = threadIdx.x;
  int off[4];
#pragma clang loop unroll(full)
  for (int k = 0; k < 4; ++k) {
    const int j = t + 256 * k, wn = j >> 9, blk = (j & 511) >> 6, ln = j & 63;
    const int v = (mi * NI + (blk >> 1)) * 4 + 2 * hf + (blk & 1);
    off[k] = (v * NT + (2 * wm + wn) * kWave + ln) * 4;
  }
  f32x4 sum[4];
#pragma clang loop unroll(full)
  for (int k = 0; k < 4; ++k) sum[k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int q = 0; q < dc.nsplit; ++q) {
    const float* src = dc.partial + (int64_t(tail) * dc.nsplit + q) * (NT * 4 * NI * 16);
    f32x4 x[4];
#pragma clang loop unroll(full)
    for (int k = 0; k < 4; ++k) x[k] = *reinterpret_cast<const f32x4*>(src + off[k]);
#pragma clang loop unroll(full)
    for (int k = 0; k < 4; ++k) sum[k] += x[k];
  }
#pragma clang loop unroll(full)
  for (int k = 0; k < 4; ++k) {
    const int j = t + 256 * k, wn = j >> 9, blk = (j & 511) >> 6, ln = j & 63;
    const int col = wn * 128 + (blk >> 1) * 32 + (ln & 31);
    const int row = 8 * (blk & 1) + 4 * (ln >> 5);
#pragma clang loop unroll(full)
    for (int e = 0; e < 4; ++e) img[(row + e) * S + col] = sum[k][e];
  }
  __syncthreads();
  double t1 = 0.0, t2 = 0.0;
  epilogue_passes<H>(p.epi, alpha * p.epi.oscale, beta, gamma, ti, tj, H * s, img, t1, t2);
  if (p.epi.parts_out) {
    block_sum2<NT>(t1, t2, red);
    if (threadIdx.x == 0) {
      const int idx = dc.nfull + kTailStrips * tail + s;
      p.epi.parts_out[2 * idx] = t1;
      p.epi.parts_out[2 * idx + 1] = t2;
    }
  }
}

// ---------------------------------------------------------------------------
// FP32 product sum_s A_s B_s^T over up to four K segments (row-major
// operands, leading dimension np).  The same work-group shape, LDS ring,
// copy weaving, split-K tail and epilogue as k_sym_split, with the
// 32x32x2 f32 MFMA (eight per 32x32 block and 16-wide K step).  The
// copies gather each 16-byte piece (four consecutive K values of one row)
// straight from the row-major operands into a chunk-major slot: piece
// (row, c) at byte c * 4096 + row * 16, so that a fragment read (32
// consecutive rows of one chunk) is one contiguous 512-byte run.  Lane
// (r, h) feeds the eight K values of chunks 2h and 2h + 1 of its row over
// the eight MFMAs, in the same order for A and B, so the sum is unchanged.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_sym_f32(F32Args p) {
  constexpr int NT = 256, BK = 16, NS = 4, MI = 4, NI = 4, TM = 128, TN = 128;
  constexpr int PANEL_B = 256 * BK * 4;   // one operand panel per K step (16 KB)
  constexpr int SLOT_B = 2 * PANEL_B;     // A, B
  constexpr int kCopies = 8;              // per wave and K step: 4 chunks of A and of B
  static_assert(NS * SLOT_B <= 128 * kEpiLd * 4, "ring exceeds the LDS image");
  __shared__ __attribute__((aligned(1024))) float lds[128 * kEpiLd];
  __shared__ double red[2 * (NT / kWave)];

  const LayerCoef cf = decide_layer<NT>(p.dec, red);
  if (cf.sign == 0) return;
  float alpha = p.epi.alpha, beta = p.epi.beta, gamma = p.epi.gamma;
  if (p.dec.mode != 0) {
    const int cn = p.epi.centring;
    alpha = cf.a;
    beta = (cn & (kCentredSquare | kCentredPair)) ? cf.b + 2.0f * kPlaneCentre * cf.a : cf.b;
    gamma = (cn & kCentredSquare) ? cf.c - kPlaneCentre * kPlaneCentre * cf.a : cf.c;
  }
  const int64_t np = p.epi.np;
  const int KT = static_cast<int>(np / BK);
  int tile, ti, tj, kb, ke, tail, piece;
  work_of(p.dc, KT * p.nseg / 2, tile, ti, tj, kb, ke, tail, piece);
  kb *= 2;
  ke *= 2;
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int wm = w >> 1, wn = w & 1;

  // Copies: this wave moves rows w * 64 + lane of both panels, chunks
  // c = 0..3 (slot bytes c * 4096 + w * 1024 + lane * 16).
  uint32_t voff[4];
#pragma clang loop unroll(full)
  for (int c = 0; c < 4; ++c) voff[c] = static_cast<uint32_t>((w * 64 + lane) * np * 4 + c * 16);
  const int64_t offa = int64_t(ti) * 256 * np, offb = int64_t(tj) * 256 * np;
  const uint32_t lds0 = static_cast<uint32_t>(
      reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) float*)(lds)));
  // Panel sources of K step IT_ (segment IT_ / KT).
#define SP2_F32_SRC(IT_, GA, GB)                                                          \
  const int it_ = (IT_);                                                                  \
  const int sg_ = (it_ >= KT) + (it_ >= 2 * KT) + (it_ >= 3 * KT);                        \
  const int64_t ko_ = int64_t(it_ - sg_ * KT) * BK;                                       \
  const float* GA = (sg_ == 0 ? p.a[0] : sg_ == 1 ? p.a[1] : sg_ == 2 ? p.a[2] : p.a[3]) + offa + ko_; \
  const float* GB = (sg_ == 0 ? p.b[0] : sg_ == 1 ? p.b[1] : sg_ == 2 ? p.b[2] : p.b[3]) + offb + ko_;
#define SP2_F32_STAGE(SLOT, IT_)                                                          \
  {                                                                                       \
    SP2_F32_SRC(IT_, ga_, gb_)                                                            \
    const uint32_t m0s_ = lds0 + (SLOT) * SLOT_B + w * 1024;                              \
    _Pragma("clang loop unroll(full)") for (int c = 0; c < 4; ++c) {                      \
      dma_chunk(voff[c], ga_, m0s_ + c * 4096);                                           \
      dma_chunk(voff[c], gb_, m0s_ + PANEL_B + c * 4096);                                 \
    }                                                                                     \
  }

  const int r = lane & 31, h = lane >> 5;
  const int fa = 2 * h * 4096 + (wm * TM + r) * 16;
  const int fb = PANEL_B + 2 * h * 4096 + (wn * TN + r) * 16;
  const char* L = reinterpret_cast<const char*>(lds);

  f32x16 acc[MI][NI];
#pragma clang loop unroll(full)
  for (int mi = 0; mi < MI; ++mi)
#pragma clang loop unroll(full)
    for (int ni = 0; ni < NI; ++ni)
#pragma clang loop unroll(full)
      for (int q = 0; q < 16; ++q) acc[mi][ni][q] = 0.0f;
  f32x4 A0[MI][2], B0[NI][2], A1[MI][2], B1[NI][2];

#define SP2_F32_FRAG(AF, BF, SLOT)                                                        \
  {                                                                                       \
    const char* S_ = L + (SLOT) * SLOT_B;                                                 \
    _Pragma("clang loop unroll(full)") for (int u = 0; u < 2; ++u) {                      \
      _Pragma("clang loop unroll(full)") for (int mi = 0; mi < MI; ++mi)                  \
        AF[mi][u] = *reinterpret_cast<const f32x4*>(S_ + fa + u * 4096 + mi * 512);       \
      _Pragma("clang loop unroll(full)") for (int ni = 0; ni < NI; ++ni)                  \
        BF[ni][u] = *reinterpret_cast<const f32x4*>(S_ + fb + u * 4096 + ni * 512);       \
    }                                                                                     \
  }
#define SP2_F32_MFMA(AF, BF, SB)                                                          \
  _Pragma("clang loop unroll(full)") for (int mi = 0; mi < MI; ++mi)                      \
  _Pragma("clang loop unroll(full)") for (int ni = 0; ni < NI; ++ni)                      \
    acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(AF[mi][(SB) >> 2][(SB) & 3],       \
                                                       BF[ni][(SB) >> 2][(SB) & 3], acc[mi][ni], 0, 0, 0);
  // One K step: the first eight-k sub-step's 16 MFMAs carry the copies of
  // K step k + 4 (one after every second MFMA, clamped to the range as in
  // k_sym_split); the LDS reads of step k + 1 go between the other 112.
#define SP2_F32_STEP(K, CA, CB, NA, NB)                                                   \
  {                                                                                       \
    const int k_ = (K);                                                                   \
    wait_ring<kCopies>(2);                                                                \
    __syncthreads();                                                                      \
    {                                                                                     \
      SP2_F32_SRC(min(k_ + 4, ke - 1), ga_, gb_)                                          \
      const uint32_t m0s_ = lds0 + ((k_ - kb) & (NS - 1)) * SLOT_B + w * 1024;            \
      _Pragma("clang loop unroll(full)") for (int mi = 0; mi < MI; ++mi)                  \
      _Pragma("clang loop unroll(full)") for (int ni = 0; ni < NI; ++ni) {                \
        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(CA[mi][0][0], CB[ni][0][0],    \
                                                           acc[mi][ni], 0, 0, 0);         \
        const int j_ = mi * NI + ni;                                                      \
        if (j_ & 1) {                                                                     \
          const int c_ = j_ >> 2;                                                         \
          if (j_ & 2) dma_chunk(voff[c_], gb_, m0s_ + PANEL_B + c_ * 4096);               \
          else dma_chunk(voff[c_], ga_, m0s_ + c_ * 4096);                                \
        }                                                                                 \
        __builtin_amdgcn_sched_barrier(0);                                                \
      }                                                                                   \
    }                                                                                     \
    SP2_F32_FRAG(NA, NB, (k_ + 1 - kb) & (NS - 1));                                       \
    _Pragma("clang loop unroll(full)") for (int sb = 1; sb < 8; ++sb) {                   \
      SP2_F32_MFMA(CA, CB, sb);                                                           \
    }                                                                                     \
    _Pragma("clang loop unroll(full)") for (int g = 0; g < 16; ++g) {                    \
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);                                  \
      __builtin_amdgcn_sched_group_barrier(0x008, 7, 0);                                  \
    }                                                                                     \
  }

  // K ranges are whole pairs of K steps; copies run four steps ahead.
#pragma clang loop unroll(full)
  for (int s = 0; s < NS; ++s) SP2_F32_STAGE(s, min(kb + s, ke - 1));
  wait_ring<kCopies>(3);
  __syncthreads();
  SP2_F32_FRAG(A0, B0, 0);
  for (int kt = kb; kt < ke; kt += 2) {
    SP2_F32_STEP(kt, A0, B0, A1, B1);
    SP2_F32_STEP(kt + 1, A1, B1, A0, B0);
  }
  wait_vmem_all();
  __syncthreads();
#undef SP2_F32_SRC
#undef SP2_F32_STAGE
#undef SP2_F32_FRAG
#undef SP2_F32_MFMA
#undef SP2_F32_STEP
  if (tail >= 0) {   // summed and finished by k_split_tail
    store_piece<NT, MI, NI>(acc, p.dc, tail, piece);
    return;
  }
  sym_epilogue_lds<NT, MI, NI>(acc, p.epi, alpha, beta, gamma, ti, tj, wm, wn, lane, red, tile, lds);
}

}  // namespace sp2
