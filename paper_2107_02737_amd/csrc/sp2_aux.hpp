// Bandwidth-bound kernels around the layer products: Gershgorin bounds,
// the input layer with its fused 16-bit split and trace partials, the plain
// split, output copies and the one-work-group control steps.
#pragma once

#include "sp2_common.hpp"

namespace sp2 {

constexpr int kRowThreads = 256;     // threads per Gershgorin block
constexpr int kRowsPerBlock = 4;     // one wave per row

// Per-row Gershgorin discs in FP64 for rows [0, n) of H: block b writes
// (min_i lower, max_i upper, any non-finite) over its rows.  A wave sums
// |H_ij| over its whole row, diagonal included, and takes |H_ii| off at
// the end: the loop is a convert and an add per element, with four 16-byte
// loads per lane issued before any of them is used.  A NaN or Inf anywhere
// in the row makes the sum non-finite (an FP64 sum of FP32 magnitudes
// cannot overflow: it would take more than 2^890 terms), which is the flag.
__global__ __launch_bounds__(kRowThreads) void k_gershgorin_rows(const float* __restrict__ H,
                                                                 int64_t n, int64_t ld,
                                                                 double* __restrict__ part) {
  __shared__ double red[3 * kRowsPerBlock];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t row = int64_t(blockIdx.x) * kRowsPerBlock + w;
  double lo = INFINITY, hi = -INFINITY, bad = 0.0;
  if (row < n) {
    const float* r = H + row * ld;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t j0 = 0;
    if ((ld % 4 == 0) && ((reinterpret_cast<uintptr_t>(H) & 15) == 0)) {
      constexpr int U = 4;
      const int64_t n4 = n & ~int64_t(3);
      int64_t c = 4 * lane;
      for (; c + 4 * kWave * (U - 1) < n4; c += 4 * kWave * U) {
        f32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = *reinterpret_cast<const f32x4*>(r + c + 4 * kWave * u);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          s0 += fabs(static_cast<double>(v[u][0]));
          s1 += fabs(static_cast<double>(v[u][1]));
          s2 += fabs(static_cast<double>(v[u][2]));
          s3 += fabs(static_cast<double>(v[u][3]));
        }
      }
      for (; c < n4; c += 4 * kWave) {
        const f32x4 v = *reinterpret_cast<const f32x4*>(r + c);
        s0 += fabs(static_cast<double>(v[0]));
        s1 += fabs(static_cast<double>(v[1]));
        s2 += fabs(static_cast<double>(v[2]));
        s3 += fabs(static_cast<double>(v[3]));
      }
      j0 = n4;
    }
    for (int64_t j = j0 + lane; j < n; j += kWave) s0 += fabs(static_cast<double>(r[j]));
    const double s = wave_sum((s0 + s1) + (s2 + s3));
    const double d = static_cast<double>(r[row]);
    const double off = s - fabs(d);
    lo = d - off;
    hi = d + off;
    bad = !isfinite(s) ? 1.0 : 0.0;
  }
  if (lane == 0) {
    red[w] = lo;
    red[kRowsPerBlock + w] = hi;
    red[2 * kRowsPerBlock + w] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = red[0], b = red[kRowsPerBlock], c = red[2 * kRowsPerBlock];
    for (int i = 1; i < kRowsPerBlock; ++i) {
      a = fmin(a, red[i]);
      b = fmax(b, red[kRowsPerBlock + i]);
      c = fmax(c, red[2 * kRowsPerBlock + i]);
    }
    part[3 * blockIdx.x + 0] = a;
    part[3 * blockIdx.x + 1] = b;
    part[3 * blockIdx.x + 2] = c;
  }
}

// One work-group: reduce the per-block discs into the bounds, flag NaN/Inf
// and a degenerate spectrum, and reset the stop state.  `trivial` marks
// n_occ in {0, n}: nothing to iterate.
__global__ __launch_bounds__(256) void k_bounds_final(const double* __restrict__ part, int nblocks,
                                                      Ctrl* ctrl, int trivial) {
  __shared__ double red[3 * 4];
  double lo = INFINITY, hi = -INFINITY, bad = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += 256) {
    lo = fmin(lo, part[3 * i]);
    hi = fmax(hi, part[3 * i + 1]);
    bad = fmax(bad, part[3 * i + 2]);
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  bad = wave_max(bad);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & 63) == 0) {
    red[w] = lo;
    red[4 + w] = hi;
    red[8 + w] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 4; ++i) {
      red[0] = fmin(red[0], red[i]);
      red[4] = fmax(red[4], red[4 + i]);
      red[8] = fmax(red[8], red[8 + i]);
    }
    const double emin = red[0], emax = red[4];
    const int nonfinite = red[8] != 0.0 || !isfinite(emin) || !isfinite(emax);
    const int degenerate = !nonfinite && !(emax > emin);
    ctrl->eps_min = emin;
    ctrl->eps_max = emax;
    ctrl->inv_range = (nonfinite || degenerate) ? 0.0 : 1.0 / (emax - emin);
    ctrl->nonfinite = nonfinite;
    ctrl->degenerate = degenerate;
    ctrl->n_iter = 0;
    ctrl->acc_len = 0;
    ctrl->acc_failed = 0;
    ctrl->stall_from = 0;
    ctrl->converged = (trivial && !nonfinite) ? 1 : 0;
    ctrl->stopped = (nonfinite || degenerate || trivial) ? 1 : 0;
    ctrl->final_t1 = 0.0;
    ctrl->final_t2 = 0.0;
  }
}

constexpr int kEwThreads = 256;

// Input layer (Section II.D): S_0 = (eps_max I - H) / (eps_max - eps_min),
// computed in FP64 per entry and rounded once to FP32, zero on the padding;
// also the hi/lo planes of S_0 - centre I (split: 1 bf16, 2 fp16 scaled;
// the centre taken off the real diagonal) and FP64 partials of
// Tr S_0 and ||S_0||_F^2 per work-group.  Work-groups stride over tiles of
// 32 rows x 256 columns: the tile is read and S_0 written a row at a time
// (1 KB per wave access), then the tile, staged in LDS, is written as planes
// a thread per row, so that every 16-byte chunk store of 32 consecutive rows
// forms one 512-byte run of the K-tiled layout.  A degenerate spectrum
// (eps_max = eps_min) gives S_0 = I/2.
constexpr int kInRows = 32, kInCols = 256, kInLd = 260;   // odd LDS row stride in 16-byte units

// Hi/lo planes of one 32 x 256 tile staged in LDS (row stride kInLd) at
// rows R0.., columns C0.. of an np x np matrix in the K-tiled layout: a
// thread per row, 8 columns (one 16-byte chunk) per store, so that the
// stores of 32 consecutive rows form one 512-byte run.
__device__ __forceinline__ void tile_planes(const float* tile, int64_t R0, int64_t C0, int64_t np,
                                            int split, uint16_t* __restrict__ hi,
                                            uint16_t* __restrict__ lo) {
  const int t = threadIdx.x, r = t % kInRows;
  const int64_t row = R0 + r;
#pragma unroll
  for (int m = 0; m < kInCols / 8 / (kEwThreads / kInRows); ++m) {
    const int ch = t / kInRows + (kEwThreads / kInRows) * m;
    const f32x4 a = *reinterpret_cast<const f32x4*>(tile + r * kInLd + ch * 8);
    const f32x4 b = *reinterpret_cast<const f32x4*>(tile + r * kInLd + ch * 8 + 4);
    const float x8[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    uint16_t h8[8], l8[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      if (split == 1)
        split_bf16(x8[e], h8[e], l8[e]);
      else
        split_fp16s(x8[e], h8[e], l8[e]);
    }
    const int64_t o = plane_off(row, C0 + ch * 8, np);   // 8 columns = one 16-byte chunk
    u32x4 hv, lv;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      hv[e] = uint32_t(h8[2 * e]) | (uint32_t(h8[2 * e + 1]) << 16);
      lv[e] = uint32_t(l8[2 * e]) | (uint32_t(l8[2 * e + 1]) << 16);
    }
    *reinterpret_cast<u32x4*>(hi + o) = hv;
    *reinterpret_cast<u32x4*>(lo + o) = lv;
  }
}

__global__ __launch_bounds__(kEwThreads) void k_input_layer(const float* __restrict__ H, int64_t n,
                                                            int64_t ld, int64_t np,
                                                            const Ctrl* __restrict__ ctrl,
                                                            float* __restrict__ S,
                                                            uint16_t* __restrict__ hi,
                                                            uint16_t* __restrict__ lo, int split,
                                                            float centre,
                                                            double* __restrict__ parts) {
  static_assert(kEwThreads == 256, "tile mapping");
  __shared__ __attribute__((aligned(16))) float tile[kInRows * kInLd];
  __shared__ double red[2 * (kEwThreads / kWave)];
  const double emax = ctrl->eps_max;
  const double inv = ctrl->inv_range;
  const bool degenerate = ctrl->degenerate != 0;
  const bool vec = (ld % 4 == 0) && ((reinterpret_cast<uintptr_t>(H) & 15) == 0);
  const int64_t tiles_c = np / kInCols, ntiles = (np / kInRows) * tiles_c;
  const int t = threadIdx.x, q = t & (kWave - 1), rsub = t / kWave;
  double t1 = 0.0, t2 = 0.0;
  for (int64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int64_t R0 = (tl / tiles_c) * kInRows, C0 = (tl % tiles_c) * kInCols;
    const int64_t j0 = C0 + 4 * q;
#pragma unroll 2
    for (int k = 0; k < kInRows / 4; ++k) {
      const int r = rsub + 4 * k;
      const int64_t i = R0 + r;
      float h4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      if (i < n) {
        if (vec && j0 + 3 < n) {
          const f32x4 h = *reinterpret_cast<const f32x4*>(H + i * ld + j0);
          h4[0] = h[0]; h4[1] = h[1]; h4[2] = h[2]; h4[3] = h[3];
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (j0 + c < n) h4[c] = H[i * ld + j0 + c];
        }
      }
      float v[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t j = j0 + c;
        float x = 0.0f;
        if (i < n && j < n) {
          if (degenerate)
            x = (i == j) ? 0.5f : 0.0f;
          else
            x = static_cast<float>(((i == j ? emax : 0.0) - static_cast<double>(h4[c])) * inv);
        }
        v[c] = x;
        const double xd = static_cast<double>(x);
        t2 += xd * xd;
        if (i == j) t1 += xd;
      }
      *reinterpret_cast<f32x4*>(S + i * np + j0) = f32x4{v[0], v[1], v[2], v[3]};
      // the planes hold S_0 - centre I (real diagonal)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (i < n && i == j0 + c) v[c] -= centre;
      *reinterpret_cast<f32x4*>(tile + r * kInLd + 4 * q) = f32x4{v[0], v[1], v[2], v[3]};
    }
    if (split) {
      __syncthreads();
      tile_planes(tile, R0, C0, np, split, hi, lo);
      __syncthreads();   // the next tile reuses the LDS
    }
  }
  block_sum2<kEwThreads>(t1, t2, red);
  if (threadIdx.x == 0) {
    parts[2 * blockIdx.x] = t1;
    parts[2 * blockIdx.x + 1] = t2;
  }
}

// Dual representation of an n x n FP32 matrix (leading dimension ld) into
// row-major hi/lo planes (leading dimension ldo); rows/cols in [n, np) are
// zero.  split: 1 bf16, 2 fp16 scaled.  (The K-tiled planes of the solver
// come from k_split_tiled.)
__global__ __launch_bounds__(kEwThreads) void k_split(const float* __restrict__ X, int64_t n,
                                                      int64_t ld, int64_t np, int64_t ldo,
                                                      uint16_t* __restrict__ hi,
                                                      uint16_t* __restrict__ lo, int split) {
  const int64_t total = np * np;
  for (int64_t q = int64_t(blockIdx.x) * kEwThreads + threadIdx.x; q < total;
       q += int64_t(gridDim.x) * kEwThreads) {
    const int64_t i = q / np, j = q % np;
    const float x = (i < n && j < n) ? X[i * ld + j] : 0.0f;
    uint16_t h, l;
    if (split == 1)
      split_bf16(x, h, l);
    else
      split_fp16s(x, h, l);
    const int64_t o = i * ldo + j;
    hi[o] = h;
    lo[o] = l;
  }
}

// Dual representation of X - centre I for an n x n FP32 matrix X (leading
// dimension ld; the centre is taken off the first nd diagonal entries, the
// real ones of a padded matrix) into the K-tiled hi/lo planes of an np x np
// matrix (np a multiple of 256; rows and columns in [n, np) are zero):
// work-groups stride over 32 x 256 tiles, read a row at a time and written
// as planes from LDS (tile_planes).
__global__ __launch_bounds__(kEwThreads) void k_split_tiled(const float* __restrict__ X, int64_t n,
                                                            int64_t ld, int64_t np,
                                                            uint16_t* __restrict__ hi,
                                                            uint16_t* __restrict__ lo, int split,
                                                            float centre, int64_t nd) {
  __shared__ __attribute__((aligned(16))) float tile[kInRows * kInLd];
  const bool vec = (ld % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  const int64_t tiles_c = np / kInCols, ntiles = (np / kInRows) * tiles_c;
  const int t = threadIdx.x, q = t & (kWave - 1), rsub = t / kWave;
  for (int64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int64_t R0 = (tl / tiles_c) * kInRows, C0 = (tl % tiles_c) * kInCols;
    const int64_t j0 = C0 + 4 * q;
#pragma unroll 2
    for (int k = 0; k < kInRows / 4; ++k) {
      const int r = rsub + 4 * k;
      const int64_t i = R0 + r;
      f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
      if (i < n) {
        if (vec && j0 + 3 < n) {
          v = *reinterpret_cast<const f32x4*>(X + i * ld + j0);
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (j0 + c < n) v[c] = X[i * ld + j0 + c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (i == j0 + c && i < nd) v[c] -= centre;
      }
      *reinterpret_cast<f32x4*>(tile + r * kInLd + 4 * q) = v;
    }
    __syncthreads();
    tile_planes(tile, R0, C0, np, split, hi, lo);
    __syncthreads();   // the next tile reuses the LDS
  }
}

// Y[i, j] = alpha * X[i, j] for i, j < n, with independent leading dimensions
// (pads, unpads and scales a matrix); padding of a larger Y is zeroed when
// np > n.
__global__ __launch_bounds__(kEwThreads) void k_copy_scaled(const float* __restrict__ X, int64_t ldx,
                                                            float* __restrict__ Y, int64_t ldy,
                                                            int64_t n, int64_t np, float alpha,
                                                            int symmetrize) {
  const int64_t total = np * np;
  for (int64_t q = int64_t(blockIdx.x) * kEwThreads + threadIdx.x; q < total;
       q += int64_t(gridDim.x) * kEwThreads) {
    const int64_t i = q / np, j = q % np;
    float v = 0.0f;
    if (i < n && j < n) {
      v = X[i * ldx + j];
      if (symmetrize) v = 0.5f * (v + X[j * ldx + i]);
      v *= alpha;
    }
    Y[i * ldy + j] = v;
  }
}

// Y = X with the strict lower triangle taken from the upper one
// (Y_ij = X_ji for i > j), np x np with leading dimension np (a multiple of
// 64, rows 16-byte aligned); Y may be X.  64 x 64 blocks, transposed through
// LDS so that both the reads and the writes are row-contiguous; every thread
// moves 16 floats as four 16-byte loads, all issued before the first store.
// lower_only (for Y = X): the grid holds only the nb (nb + 1) / 2 blocks on
// or below the diagonal, block b = bi (bi + 1) / 2 + bj; otherwise all
// nb^2 blocks, the upper ones copied.
constexpr int kMirrorTile = 64;
__global__ __launch_bounds__(256) void k_mirror_upper(const float* X, float* Y, int64_t np,
                                                      int lower_only) {
  __shared__ float t[kMirrorTile][kMirrorTile + 1];
  const int nb = static_cast<int>(np / kMirrorTile);
  int bi, bj;   // output block (bi, bj)
  if (lower_only) {
    const int b = blockIdx.x;
    bi = static_cast<int>((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while (bi * (bi + 1) / 2 > b) --bi;
    while ((bi + 1) * (bi + 2) / 2 <= b) ++bi;
    bj = b - bi * (bi + 1) / 2;
  } else {
    bi = blockIdx.x / nb;
    bj = blockIdx.x % nb;
  }
  const int cq = (threadIdx.x & 15) * 4, rq = threadIdx.x >> 4;   // 16 x float4 columns, 16 rows
  const int64_t r0 = int64_t(bi) * kMirrorTile, c0 = int64_t(bj) * kMirrorTile;
  f32x4 v[4];
  if (bi < bj) {   // upper block (Y != X only): plain copy
#pragma unroll
    for (int k = 0; k < 4; ++k)
      v[k] = *reinterpret_cast<const f32x4*>(X + (r0 + rq + 16 * k) * np + c0 + cq);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      *reinterpret_cast<f32x4*>(Y + (r0 + rq + 16 * k) * np + c0 + cq) = v[k];
    return;
  }
  // source block (bj, bi) of the upper triangle: t[r][c] = X[c0 + r][r0 + c]
#pragma unroll
  for (int k = 0; k < 4; ++k)
    v[k] = *reinterpret_cast<const f32x4*>(X + (c0 + rq + 16 * k) * np + r0 + cq);
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int e = 0; e < 4; ++e) t[rq + 16 * k][cq + e] = v[k][e];
  __syncthreads();
  // Y[r0 + r][c0 + c] = X[c0 + c][r0 + r] = t[c][r]; on a diagonal block the
  // elements on or above the diagonal keep X[r0 + r][r0 + c] = t[r][c]
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = rq + 16 * k;
    f32x4 o;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = cq + e;
      o[e] = (bi > bj || r > c) ? t[c][r] : t[r][c];
    }
    *reinterpret_cast<f32x4*>(Y + (r0 + r) * np + c0 + cq) = o;
  }
}

// P = 0 (value 0) or P = I (value 1), n x n with leading dimension ld.
__global__ __launch_bounds__(kEwThreads) void k_fill_diag(float* __restrict__ P, int64_t n,
                                                          int64_t ld, float value) {
  const int64_t total = n * n;
  for (int64_t q = int64_t(blockIdx.x) * kEwThreads + threadIdx.x; q < total;
       q += int64_t(gridDim.x) * kEwThreads) {
    const int64_t i = q / n, j = q % n;
    P[i * ld + j] = (i == j) ? value : 0.0f;
  }
}

// One work-group after the layer loop: when the network did not stop within
// max_iter layers, evaluate the stop test on S_{max_iter} and record it.
__global__ __launch_bounds__(256) void k_finish_loop(Ctrl* ctrl, Hist* hist,
                                                     const double* __restrict__ parts, int nparts,
                                                     int max_iter, double n_occ, double tol,
                                                     int stop_rule, double stall_gate) {
  __shared__ double red[8];
  if (ctrl->stopped) return;
  double t1 = 0.0, t2 = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) {
    t1 += parts[2 * i];
    t2 += parts[2 * i + 1];
  }
  block_sum2<256>(t1, t2, red);
  if (threadIdx.x == 0) {
    const int n = max_iter;
    const double e = fabs(t1 - t2);
    const bool stop = stop_test(t1, e, n, hist->err, n_occ, tol, stop_rule, stall_gate,
                                ctrl->stall_from);
    hist->t1[n] = t1;
    hist->t2[n] = t2;
    hist->err[n] = e;
    ctrl->n_iter = n;
    ctrl->converged = stop ? 1 : 0;
    ctrl->stopped = 1;
  }
}

// ---------------------------------------------------------------------------
// Accelerated schedule (Section II.E: with estimates of the HOMO and the
// LUMO the network needs fewer layers).  The mapped interval ends
// l = (eps_max - lumo)/(eps_max - eps_min) (top of the virtual eigenvalues)
// and h = (eps_max - homo)/(eps_max - eps_min) (bottom of the occupied ones)
// fix the whole schedule: while max(l, 1 - h) >= kAccEnd, the wider of the
// two intervals is folded about kAccFold of its width, s = kAccFold l with
// the layer ((x - s)/(1 - s))^2 when l >= 1 - h, else s = kAccFold (1 - h)
// with 1 - ((1 - x - s)/(1 - s))^2, and the ends follow the same maps (the
// folded end to the larger of the images of its two ends).  A fold of 0.4
// rather than 1/2 (the smallest folded image) keeps the gap between the two
// intervals growing fast enough that early rounding is not amplified beyond
// the plain network's.  The stagnation test may compare errors from the
// first iterate whose tracked width is below kStallWidth (the remaining
// shifts are then below 0.4 kStallWidth and the layers act as plain ones;
// before that the schedule itself can raise e), or from the end of the
// schedule.  One thread, FP64, every operation rounded as
// written (no contraction), so the coefficients are those of the same
// recursion evaluated anywhere else in IEEE double.  Layers past the
// schedule use the trace-driven sign.
// ---------------------------------------------------------------------------
constexpr double kAccEnd = 1e-14;
constexpr double kAccFold = 0.4;
constexpr double kStallWidth = 1e-4;

__global__ void k_acc_schedule(Ctrl* ctrl, Hist* hist, double homo, double lumo, int max_len) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  ctrl->acc_len = 0;
  ctrl->stall_from = 0;
  if (ctrl->stopped) return;   // NaN/Inf, no spread, or a trivial occupation
  const double r = ctrl->eps_max - ctrl->eps_min;
  double l = fmin(fmax((ctrl->eps_max - lumo) / r, 0.0), 1.0);
  double h = fmin(fmax((ctrl->eps_max - homo) / r, 0.0), 1.0);
  int n = 0, quiet = -1;
  if (l < h) {
    while (n < max_len && fmax(l, 1.0 - h) >= kAccEnd) {
      if (quiet < 0 && fmax(l, 1.0 - h) < kStallWidth) quiet = n;
      double a, b, c;
      int sign;
      if (l >= 1.0 - h) {
        const double s = kAccFold * l, d = 1.0 - s;
        const double q = fmax(s, l - s) / d, t = (h - s) / d;
        l = q * q;
        h = t * t;
        a = 1.0 / (d * d);
        b = -2.0 * s / (d * d);
        c = s * s / (d * d);
        sign = 1;
      } else {
        const double s = kAccFold * (1.0 - h), d = 1.0 - s;
        const double q = (1.0 - l - s) / d, t = fmax(s, 1.0 - h - s) / d;
        l = 1.0 - q * q;
        h = 1.0 - t * t;
        a = -1.0 / (d * d);
        b = 2.0 / d;
        c = 0.0;
        sign = -1;
      }
      hist->coef[n][0] = a;
      hist->coef[n][1] = b;
      hist->coef[n][2] = c;
      hist->branch[n] = sign;
      ++n;
    }
  }
  ctrl->acc_len = n;
  ctrl->stall_from = n == 0 ? 0 : (quiet >= 0 ? quiet : n);
}

// One work-group: sum (Tr, ||.||_F^2) partials of the returned P into ctrl.
__global__ __launch_bounds__(256) void k_sum_parts(Ctrl* ctrl, const double* __restrict__ parts,
                                                   int nparts) {
  __shared__ double red[8];
  double t1 = 0.0, t2 = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) {
    t1 += parts[2 * i];
    t2 += parts[2 * i + 1];
  }
  block_sum2<256>(t1, t2, red);
  if (threadIdx.x == 0) {
    ctrl->final_t1 = t1;
    ctrl->final_t2 = t2;
  }
}

// (Tr, ||.||_F^2) partials of an np x np FP32 matrix, one pair per block.
__global__ __launch_bounds__(kEwThreads) void k_trace_parts(const float* __restrict__ S, int64_t np,
                                                            double* __restrict__ parts) {
  __shared__ double red[2 * (kEwThreads / kWave)];
  double t1 = 0.0, t2 = 0.0;
  const int64_t total = np * np;
  for (int64_t q = int64_t(blockIdx.x) * kEwThreads + threadIdx.x; q < total;
       q += int64_t(gridDim.x) * kEwThreads) {
    const double v = static_cast<double>(S[q]);
    t2 += v * v;
    if (q / np == q % np) t1 += v;
  }
  block_sum2<kEwThreads>(t1, t2, red);
  if (threadIdx.x == 0) {
    parts[2 * blockIdx.x] = t1;
    parts[2 * blockIdx.x + 1] = t2;
  }
}

}  // namespace sp2
