// Shared device-side definitions of the gfx950 DNN-SP2 kernels: vector
// types, the device control block, reductions and the 16-bit split.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sp2.h"

namespace sp2 {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;
typedef __attribute__((ext_vector_type(2))) uint32_t u32x2;

constexpr int kWave = 64;
constexpr int kMaxIter = SP2_MAX_ITER;
constexpr int kFp16ScaleLog2 = 14;   // 2^14 X keeps the FP16 residual normal
// The split planes of a network iterate S hold S - kPlaneCentre I.  Every
// eigenvalue of S lies in [0, 1], so the centred matrix has eigenvalues in
// [-1/2, 1/2] and much smaller diagonal entries (those of a density matrix
// sit near 0 or 1): the FP32 partial sums of the MFMA K loop and the 16-bit
// roundings of the operands shrink with them, and the layer restores
// S^2 = (S - I/2)^2 + S - I/4 exactly in its epilogue.
constexpr float kPlaneCentre = 0.5f;

// Device control block: one per workspace.  Written by the bound pass, the
// layer kernels (work-group 0 only) and the one-work-group control kernels.
struct Ctrl {
  double eps_min, eps_max;   // Gershgorin bounds of H
  double inv_range;          // 1 / (eps_max - eps_min)
  double final_t1, final_t2; // traces of the returned P
  int32_t nonfinite;         // H holds NaN/Inf
  int32_t degenerate;        // eps_max == eps_min
  int32_t stopped;           // stop test passed (or nothing to iterate)
  int32_t n_iter;            // layers applied when stopped
  int32_t converged;
  int32_t acc_len;           // layers 0 .. acc_len-1 follow the accelerated schedule
  int32_t acc_failed;        // the trace check at the end of the schedule failed
  int32_t stall_from;        // the stagnation test compares e_n with e_{n-2} only for n-2 >= this
  int32_t pad[4];
};

// Per-layer history: traces of every examined approximation S_k, the sign
// of every applied layer (+1: the S^2 family, -1: the 2S - S^2 family) and
// its coefficients (a, b, c): S_{k+1} = a S_k^2 + b S_k + c I.
struct Hist {
  double t1[kMaxIter + 1];
  double t2[kMaxIter + 1];
  double err[kMaxIter + 1];
  double coef[kMaxIter][3];
  int32_t branch[kMaxIter];
};

// Coefficients of one layer S_{n+1} = a S_n^2 + b S_n + c I: the DNN layer
// of Eq. 19 with W_n = a I and B_n = b S_n + c I.  Plain SP2 layers are
// (1, 0, 0) and (-1, 2, 0); the accelerated ones shift and scale them.
// sign 0: the network has stopped.
struct LayerCoef {
  int sign;
  float a, b, c;
};

__device__ __forceinline__ LayerCoef plain_coef(int sign) {
  return sign > 0 ? LayerCoef{1, 1.0f, 0.0f, 0.0f} : LayerCoef{-1, -1.0f, 2.0f, 0.0f};
}

// Recorded coefficients of layer n; with_c = false drops c (the derivative
// of the layer map is dS -> a (S dS + dS S) + b dS).
__device__ __forceinline__ LayerCoef hist_coef(const Hist* h, int n, bool with_c) {
  const double a = h->coef[n][0];
  return LayerCoef{a > 0.0 ? 1 : -1, static_cast<float>(a), static_cast<float>(h->coef[n][1]),
                   with_c ? static_cast<float>(h->coef[n][2]) : 0.0f};
}

// Parameters of the trace-driven stop / branch decision (Section II.D-E).
struct Decide {
  Ctrl* ctrl;
  Hist* hist;
  const double* parts_in;   // (Tr, ||.||_F^2) partial pairs of S_n
  int nparts_in;
  int layer;                // n: this launch turns S_n into S_{n+1}
  int mode;                 // 0: fixed coefficients, 1: decide, 2: replay the recorded
                            // layer (a, b, c), 3: its derivative map (a, b, 0)
  double n_occ, tol, stall_gate;
  int stop_rule;
  int quiet;                // 1: decide without recording (a second kernel of the same layer)
};

// ---------------------------------------------------------------------------
// Reductions (fixed order, so every work-group and every run agrees bitwise)
// ---------------------------------------------------------------------------

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline double wave_min(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, kWave));
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Block-wide sum of two doubles; every thread receives the totals.  `red`
// must hold 2 * (blockDim / 64) doubles of LDS.
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
  constexpr int NW = NT / kWave;
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) {
    red[w] = a;
    red[NW + w] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    sa += red[i];
    sb += red[NW + i];
  }
  a = sa;
  b = sb;
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Branch and stop decision, taken redundantly (and identically) by every
// work-group of a layer launch before it multiplies.  Returns the layer's
// coefficients, sign 0 when the network has stopped.  Mode 0 returns sign 1
// and leaves the coefficients to the launch.
// ---------------------------------------------------------------------------

// Stop test on the traces of S_n (Section II.E: idempotency estimated from
// traces), e = |t1 - t2|.  No stop while |t1 - n_occ| >= 1/2: S_n does not
// yet hold n_occ eigenvalues near 1 (an occupied eigenvalue can pass close to
// 0 on the way, which makes e small long before convergence).  Then rule 0:
// e < tol; rule 1 also stops once e < stall_gate and the last two layers did
// not reduce e as exact arithmetic would: e >= e_{n-2}, or
// e >= kQuadFactor e_{n-2}^2.  Below the gate (every eigenvalue within 1/4
// of 0 or 1) a pair of layers of opposite sign maps each eigenvalue's share
// x(1 - x) of e to at most 64/9 times its square (4 times in the limit), and
// the trace-closest sign squares the side that dominates the trace, so
// e_n <= (64/9) e_{n-2}^2 in exact arithmetic: an e_n of 16 e_{n-2}^2 or
// more is mostly rounding.  The
// comparisons start at n - 2 >= stall_from (inside an accelerated schedule e
// can rise, or fall less than quadratically, by itself until the tracked
// interval width is small).
constexpr double kQuadFactor = 16.0;

__device__ __forceinline__ bool stop_test(double t1, double e, int n, const double* err_hist,
                                          double n_occ, double tol, int stop_rule,
                                          double stall_gate, int stall_from) {
  if (!(fabs(t1 - n_occ) < 0.5)) return false;
  if (e < tol) return true;
  if (!(stop_rule == 1 && n >= 2 && n - 2 >= stall_from && e < stall_gate)) return false;
  const double ep = err_hist[n - 2];
  return e >= fmin(ep, kQuadFactor * ep * ep);
}

template <int NT>
__device__ __forceinline__ LayerCoef decide_layer(const Decide& d, double* red) {
  if (d.mode == 2 || d.mode == 3) return hist_coef(d.hist, d.layer, d.mode == 2);
  if (d.mode != 1) return LayerCoef{1, 1.0f, 0.0f, 0.0f};
  // One read of the stop flag per work-group, shared through LDS, so that
  // all of its waves take the same exit -- before the partial sums, so that
  // launches queued after the stop leave at once.
  __shared__ int s_stopped;
  if (threadIdx.x == 0) s_stopped = __atomic_load_n(&d.ctrl->stopped, __ATOMIC_RELAXED);
  __syncthreads();
  if (s_stopped) return LayerCoef{0, 0.0f, 0.0f, 0.0f};
  double t1 = 0.0, t2 = 0.0;
  for (int i = threadIdx.x; i < d.nparts_in; i += NT) {
    t1 += d.parts_in[2 * i];
    t2 += d.parts_in[2 * i + 1];
  }
  block_sum2<NT>(t1, t2, red);
  const int n = d.layer;
  const double e = fabs(t1 - t2);
  const bool stop = stop_test(t1, e, n, d.hist->err, d.n_occ, d.tol, d.stop_rule, d.stall_gate,
                              d.ctrl->stall_from);
  // Layers of the accelerated schedule (written before the first layer)
  // take their recorded coefficients; the others the trace-closest sign:
  // Tr(S^2) = t2 versus Tr(2S - S^2) = 2 t1 - t2; ties take S^2.  At the
  // end of a schedule every eigenvalue sits on its side, so a trace more
  // than 1/2 from n_occ means the estimates were wrong: the network ends
  // unconverged (acc_failed) and the host runs the plain network instead.
  const int acc_len = d.ctrl->acc_len;
  const bool scheduled = n < acc_len;
  const bool failed = !stop && acc_len > 0 && n == acc_len && !(fabs(t1 - d.n_occ) < 0.5);
  const int sign = (fabs(t2 - d.n_occ) <= fabs(2.0 * t1 - t2 - d.n_occ)) ? 1 : -1;
  if (!d.quiet && blockIdx.x == 0 && threadIdx.x == 0) {
    d.hist->t1[n] = t1;
    d.hist->t2[n] = t2;
    d.hist->err[n] = e;
    if (stop || failed) {
      d.ctrl->n_iter = n;
      d.ctrl->converged = stop ? 1 : 0;
      d.ctrl->acc_failed = failed ? 1 : 0;
      __atomic_store_n(&d.ctrl->stopped, 1, __ATOMIC_RELAXED);
    } else if (!scheduled) {
      d.hist->branch[n] = sign;
      d.hist->coef[n][0] = sign > 0 ? 1.0 : -1.0;
      d.hist->coef[n][1] = sign > 0 ? 0.0 : 2.0;
      d.hist->coef[n][2] = 0.0;
    }
  }
  if (stop || failed) return LayerCoef{0, 0.0f, 0.0f, 0.0f};
  return scheduled ? hist_coef(d.hist, n, true) : plain_coef(sign);
}

// The coefficients of a layer as recorded by that layer's product launch,
// for a kernel that follows it on the stream: sign 0 once the network has
// stopped.
__device__ __forceinline__ LayerCoef recorded_coef(const Decide& d) {
  if (d.mode == 2 || d.mode == 3) return hist_coef(d.hist, d.layer, d.mode == 2);
  if (d.mode != 1) return LayerCoef{1, 1.0f, 0.0f, 0.0f};
  if (__atomic_load_n(&d.ctrl->stopped, __ATOMIC_RELAXED)) return LayerCoef{0, 0.0f, 0.0f, 0.0f};
  return hist_coef(d.hist, d.layer, true);
}

// ---------------------------------------------------------------------------
// 16-bit dual representation X = X0 + X1 (Eq. 20-21), round to nearest even.
// ---------------------------------------------------------------------------

__device__ inline void split_bf16(float x, uint16_t& hi, uint16_t& lo) {
  const __bf16 h = static_cast<__bf16>(x);
  const __bf16 l = static_cast<__bf16>(x - static_cast<float>(h));
  hi = __builtin_bit_cast(uint16_t, h);
  lo = __builtin_bit_cast(uint16_t, l);
}

__device__ inline void split_fp16s(float x, uint16_t& hi, uint16_t& lo) {
  // ldexp keeps the sign of zero (a contracted multiply-add with +0 would not)
  const float xs = ldexpf(x, kFp16ScaleLog2);
  const _Float16 h = static_cast<_Float16>(xs);
  const _Float16 l = static_cast<_Float16>(xs - static_cast<float>(h));
  hi = __builtin_bit_cast(uint16_t, h);
  lo = __builtin_bit_cast(uint16_t, l);
}

// ---------------------------------------------------------------------------
// K-tiled layout of the 16-bit planes.  The plane of an np x np matrix is
// stored as blocks of 256 rows x 16 columns (8 KB each), block (I, K) at
// element (I * np/16 + K) * 4096; inside a block, columns 0-7 of all 256
// rows come first (16 bytes per row), then columns 8-15.  One K step of a
// 256-row panel is then one contiguous 8 KB block that the product kernel
// copies verbatim into LDS, where an MFMA fragment read (consecutive lanes
// reading 16 bytes of consecutive rows) is bank-conflict free, and the
// epilogue writes a chunk of 64 consecutive rows as one contiguous 1 KB
// store.
// ---------------------------------------------------------------------------

constexpr int kPlaneRows = 256;
constexpr int kPlaneCols = 16;

// Element offset of (i, k) in the tiled plane of an np x np matrix.
__device__ __forceinline__ int64_t plane_off(int64_t i, int64_t k, int64_t np) {
  const int64_t blk = (i >> 8) * (np >> 4) + (k >> 4);
  return blk * 4096 + ((k >> 3) & 1) * 2048 + (i & 255) * 8 + (k & 7);
}

// ---------------------------------------------------------------------------
// Upper-triangle tile schedule.  Work-group b runs on XCD (b mod 8); the
// remap gives each XCD a contiguous run of logical tiles, and the logical
// order walks bands of `band` tile-rows column by column so that tiles that
// run together on one XCD share row panels in its L2.
// ---------------------------------------------------------------------------

__device__ inline int xcd_remap(int b, int ntiles) {
  const int xcd = b & 7, local = b >> 3;
  const int per = ntiles >> 3, rem = ntiles & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

__device__ __forceinline__ void tile_of(int logical, int nb, int band, int& ti, int& tj) {
  int r0 = 0;
  for (;;) {
    if (r0 >= nb) {   // out of range: cannot happen with grid == tile count
      ti = tj = 0;
      return;
    }
    const int r1 = min(r0 + band, nb) - 1;
    int count = 0;
    for (int j = r0; j < nb; ++j) count += min(r1, j) - r0 + 1;
    if (logical < count) {
      for (int j = r0; j < nb; ++j) {
        const int c = min(r1, j) - r0 + 1;
        if (logical < c) {
          ti = r0 + logical;
          tj = j;
          return;
        }
        logical -= c;
      }
    }
    logical -= count;
    r0 += band;
  }
}

}  // namespace sp2
