// Optional tightening of the spectral bounds before the input layer.
//
// The network needs an interval holding the spectrum of H (Section II.D);
// Gershgorin discs always hold it but are loose, which shrinks the mapped
// HOMO-LUMO gap and costs layers.  Here k steps of the symmetric Lanczos
// recurrence with full reorthogonalisation (Golub and Van Loan, Matrix
// Computations, Sections 10.1 and 10.3) run on the device in FP64 from a
// SplitMix64 start vector (Steele, Lea and Flood, OOPSLA 2014); the extreme eigenvalues of the k x k tridiagonal matrix
// (Sturm-count bisection), widened by their Ritz residual norms
// |beta_k s_k| (inverse iteration) and a relative margin, replace the
// Gershgorin bounds wherever they are tighter.  Nothing returns to the host.
#pragma once

#include "sp2_common.hpp"

namespace sp2 {

constexpr int kLzMaxSteps = 64;
constexpr int kLzThreads = 1024;     // start kernel
constexpr int kLzMvThreads = 512;    // matrix-vector work-group: 8 waves
constexpr int kLzRowsPerWave = 2;
constexpr int kLzRowsPerBlock = (kLzMvThreads / 64) * kLzRowsPerWave;
constexpr int kLzChunk = 256;        // rows per work-group of the vector kernels
constexpr int kLzCoef = kLzMaxSteps + 1;
constexpr double kLzMargin = 0.01;   // relative widening of the Ritz interval

struct LzState {
  double alpha[kLzMaxSteps];
  double beta[kLzMaxSteps];
  int32_t steps;    // recorded alpha values
  int32_t broke;    // beta vanished: invariant subspace, later steps skipped
  int32_t pad[2];
  double ritz[4];   // HOMO/LUMO estimator: (th_max, r_max) of the occupied run,
                    // (th_min, r_min) of the virtual run
};

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <int NT>
__device__ __forceinline__ double block_sum1(double a, double* red) {
  constexpr int NW = NT / kWave;
  a = wave_sum(a);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = a;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += red[i];
  return s;
}

// Sums of the per-chunk partials part[b * stride + i] over the chunks b for
// i < count (count * 4 <= blockDim.x), into out[i] (LDS), in a fixed order:
// thread (i, g) adds chunks g, g + 4, g + 8, ... in turn, then the four
// results are added in order g = 0..3.  Every work-group that needs a sum
// computes it identically.  The partials reach the LDS buffer (cap doubles)
// a batch of chunks at a time, each thread keeping eight loads in flight.
__device__ __forceinline__ void ordered_sums(const double* __restrict__ part, int nchunks,
                                             int stride, int count, double* buf, int cap,
                                             double* out) {
  constexpr int G = 4, U = 8;
  const int batch = (cap / count) / G * G;
  const int i = threadIdx.x / G, g = threadIdx.x % G;
  double s = 0.0;
  for (int b0 = 0; b0 < nchunks; b0 += batch) {
    const int nb = min(batch, nchunks - b0), total = nb * count;
    for (int q0 = threadIdx.x; q0 < total; q0 += U * blockDim.x) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u * blockDim.x;
        v[u] = q < total ? part[int64_t(b0 + q / count) * stride + q % count] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u * blockDim.x;
        if (q < total) buf[(q % count) * batch + q / count] = v[u];
      }
    }
    __syncthreads();
    if (i < count)
      for (int b = g; b < nb; b += G) s += buf[i * batch + b];
    __syncthreads();
  }
  // the four interleaved partial sums of coefficient i, in order
  if (i < count) buf[i * G + g] = s;
  __syncthreads();
  if (threadIdx.x < count) {
    const double* r = buf + threadIdx.x * G;
    out[threadIdx.x] = ((r[0] + r[1]) + r[2]) + r[3];
  }
  __syncthreads();
}

// Partial products of kLzRowsPerWave rows of an FP32 matrix (row pointers
// mrow) with an FP64 vector x scaled by xs, over this lane's columns c = 4
// lane + 256 k.  Four 256-column chunks per step with every load issued
// before the arithmetic, then a chunk at a time; each row's FMA chain runs
// over its columns in increasing order whatever the chunking.
__device__ __forceinline__ void rows_dot(const float* const (&mrow)[kLzRowsPerWave],
                                         const double* __restrict__ x, double xs, int64_t n,
                                         int64_t ld, bool vec, int lane,
                                         double (&acc)[kLzRowsPerWave]) {
  constexpr int U = 4, R = kLzRowsPerWave;
  int64_t c_done = 0;
  if (vec) {
    const int64_t n4 = n & ~int64_t(3);
    int64_t c = 4 * lane;
    for (; c + (U - 1) * 4 * kWave < n4; c += U * 4 * kWave) {
      f32x4 h[U][R];
      double xv[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
          h[u][rr] = *reinterpret_cast<const f32x4*>(mrow[rr] + c + u * 4 * kWave);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) xv[u][e] = x[c + u * 4 * kWave + e];
      // every load above is issued before any of the arithmetic below
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            acc[rr] = fma(static_cast<double>(h[u][rr][e]), xv[u][e] * xs, acc[rr]);
    }
    for (; c < n4; c += 4 * kWave) {
      double xv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) xv[e] = x[c + e] * xs;
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const f32x4 h = *reinterpret_cast<const f32x4*>(mrow[rr] + c);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[rr] = fma(static_cast<double>(h[e]), xv[e], acc[rr]);
      }
    }
    c_done = n4;
  }
  for (int64_t c = c_done + lane; c < n; c += kWave) {
    const double xc = x[c] * xs;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) acc[rr] = fma(static_cast<double>(mrow[rr][c]), xc, acc[rr]);
  }
}

// rows_dot for two vectors x0, x1 at once (xs = 1): every matrix load
// serves both; each vector's FMA chain runs in the same order as rows_dot's.
__device__ __forceinline__ void rows_dot2(const float* const (&mrow)[kLzRowsPerWave],
                                          const double* __restrict__ x0,
                                          const double* __restrict__ x1, int64_t n, int64_t ld,
                                          bool vec, int lane, double (&acc0)[kLzRowsPerWave],
                                          double (&acc1)[kLzRowsPerWave]) {
  constexpr int U = 4, R = kLzRowsPerWave;
  int64_t c_done = 0;
  if (vec) {
    const int64_t n4 = n & ~int64_t(3);
    int64_t c = 4 * lane;
    for (; c + (U - 1) * 4 * kWave < n4; c += U * 4 * kWave) {
      f32x4 h[U][R];
      double xa[U][4], xb[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
          h[u][rr] = *reinterpret_cast<const f32x4*>(mrow[rr] + c + u * 4 * kWave);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          xa[u][e] = x0[c + u * 4 * kWave + e];
          xb[u][e] = x1[c + u * 4 * kWave + e];
        }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const double hv = static_cast<double>(h[u][rr][e]);
            acc0[rr] = fma(hv, xa[u][e] * 1.0, acc0[rr]);
            acc1[rr] = fma(hv, xb[u][e] * 1.0, acc1[rr]);
          }
    }
    for (; c < n4; c += 4 * kWave) {
      double xa[4], xb[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        xa[e] = x0[c + e] * 1.0;
        xb[e] = x1[c + e] * 1.0;
      }
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const f32x4 h = *reinterpret_cast<const f32x4*>(mrow[rr] + c);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc0[rr] = fma(static_cast<double>(h[e]), xa[e], acc0[rr]);
          acc1[rr] = fma(static_cast<double>(h[e]), xb[e], acc1[rr]);
        }
      }
    }
    c_done = n4;
  }
  for (int64_t c = c_done + lane; c < n; c += kWave) {
    const double xa = x0[c] * 1.0, xb = x1[c] * 1.0;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      acc0[rr] = fma(static_cast<double>(mrow[rr][c]), xa, acc0[rr]);
      acc1[rr] = fma(static_cast<double>(mrow[rr][c]), xb, acc1[rr]);
    }
  }
}

// V_0 = u / |u|, u_i = (z_i >> 11) 2^-53 - 1/2; state reset.  V holds the
// Lanczos vectors as consecutive rows of n doubles.
__global__ __launch_bounds__(kLzThreads) void k_lz_start(double* __restrict__ V, int64_t n,
                                                         uint64_t seed, LzState* st) {
  __shared__ double red[kLzThreads / kWave];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kLzThreads) {
    const double u = static_cast<double>(splitmix64(seed, static_cast<uint64_t>(i)) >> 11) *
                         0x1.0p-53 - 0.5;
    V[i] = u;
    s += u * u;
  }
  const double nrm = sqrt(block_sum1<kLzThreads>(s, red));
  for (int64_t i = threadIdx.x; i < n; i += kLzThreads) V[i] = V[i] / nrm;
  if (threadIdx.x == 0) {
    st->steps = 0;
    st->broke = 0;
  }
}

// Step j: wout = H v_j (FP32 H, FP64 products and sums), each wave taking 2
// consecutive rows (every v load serves both; many waves keep the H stream
// at full bandwidth), 8 waves per work-group.  For j >= 1, v_j is
// formed on the fly as win * (1 / beta_{j-1}), beta_{j-1} = sqrt of the
// summed squared-norm partials of step j-1, and stored into V row j by the
// work-group owning each row; block 0 records beta_{j-1}.  Each work-group
// also writes the partial dot products of its rows of wout with
// v_0 .. v_j (the first Gram-Schmidt pass): dot_part[block * kLzCoef + i].
__global__ __launch_bounds__(kLzMvThreads) void k_lz_matvec(const float* __restrict__ H, int64_t n,
                                                   int64_t ld, double* __restrict__ V,
                                                   const double* __restrict__ win,
                                                   double* __restrict__ wout,
                                                   const double* __restrict__ norm_part,
                                                   int nchunks, double* __restrict__ dot_part,
                                                   LzState* st, int j) {
  __shared__ double sbuf[256];
  __shared__ double snorm;
  if (st->broke) return;
  const double* v = V + int64_t(j) * n;
  double inv = 1.0;
  if (j > 0) {
    ordered_sums(norm_part, nchunks, 1, 1, sbuf, 256, &snorm);
    const double beta = sqrt(snorm);
    if (!(beta > 1e-300)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->beta[j - 1] = beta;
        st->broke = 1;
      }
      return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st->beta[j - 1] = beta;
    inv = 1.0 / beta;
    v = win;
  }
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t r0 = int64_t(blockIdx.x) * kLzRowsPerBlock + wv * kLzRowsPerWave;
  double acc[kLzRowsPerWave];
  const float* hrow[kLzRowsPerWave];
  // rows past n read row 0 instead (in bounds; their sums are discarded),
  // so the column loop carries no per-row branch and its loads overlap
#pragma unroll
  for (int rr = 0; rr < kLzRowsPerWave; ++rr) {
    acc[rr] = 0.0;
    hrow[rr] = H + (r0 + rr < n ? r0 + rr : 0) * ld;
  }
  const bool vec = (ld % 4 == 0) && ((reinterpret_cast<uintptr_t>(H) & 15) == 0);
  rows_dot(hrow, v, inv, n, ld, vec, lane, acc);
  double ws[kLzRowsPerWave];
#pragma unroll
  for (int rr = 0; rr < kLzRowsPerWave; ++rr) {
    const double s = wave_sum(acc[rr]);
    const int64_t row = r0 + rr;
    ws[rr] = row < n ? s : 0.0;
    if (lane == 0 && row < n) {
      wout[row] = s;
      if (j > 0) V[int64_t(j) * n + row] = win[row] * inv;
    }
  }
  // lane i: this wave's part of v_i . wout (i <= j < 64), then the waves in order
  __shared__ double dred[kLzMvThreads / kWave][kWave];
  double d = 0.0;
  if (lane <= j) {
#pragma unroll
    for (int rr = 0; rr < kLzRowsPerWave; ++rr) {
      const int64_t row = r0 + rr;
      if (row < n) {
        const double vi = lane < j ? V[int64_t(lane) * n + row] : (j > 0 ? win[row] * inv : V[row]);
        d = fma(vi, ws[rr], d);
      }
    }
  }
  dred[wv][lane] = d;
  __syncthreads();
  if (threadIdx.x <= j) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kLzMvThreads / kWave; ++q) t += dred[q][threadIdx.x];
    dot_part[int64_t(blockIdx.x) * kLzCoef + threadIdx.x] = t;
  }
}

// Partial dot products of w with v_0 .. v_j over one chunk of 256 rows:
// part[chunk * kLzCoef + i].
__device__ __forceinline__ void chunk_dots(const double* V, double wr, int64_t row, int64_t n, int j,
                                           double* part, double* red) {
  constexpr int NW = kLzChunk / kWave, B = 8;
  // eight wave reductions side by side (each the butterfly of wave_sum)
  for (int i0 = 0; i0 <= j; i0 += B) {
    double p[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int i = i0 + b;
      p[b] = (row < n && i <= j) ? V[int64_t(i) * n + row] * wr : 0.0;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
      for (int b = 0; b < B; ++b) p[b] += __shfl_xor(p[b], off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
      for (int b = 0; b < B; ++b)
        if (i0 + b <= j) red[(threadIdx.x / kWave) * kLzCoef + i0 + b] = p[b];
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j; i += kLzChunk) {
    double s = 0.0;
    for (int k = 0; k < NW; ++k) s += red[k * kLzCoef + i];
    part[blockIdx.x * kLzCoef + i] = s;
  }
}

// Coefficient i = blockIdx.x of a Gram-Schmidt pass from many partials
// (one per matrix-vector work-group): thread t adds partials t, t + 256, ...
// in turn, then a fixed-order tree over the work-group.
__device__ __forceinline__ void lz_coef_body(const double* __restrict__ part, int nparts,
                                             double* __restrict__ coef, const LzState* st) {
  __shared__ double red[kLzChunk / kWave];
  if (st->broke) return;
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kLzChunk) s += part[int64_t(b) * kLzCoef + i];
  s = block_sum1<kLzChunk>(s, red);
  if (threadIdx.x == 0) coef[i] = s;
}

__global__ __launch_bounds__(kLzChunk) void k_lz_coef(const double* __restrict__ part, int nparts,
                                                      double* __restrict__ coef,
                                                      const LzState* st) {
  lz_coef_body(part, nparts, coef, st);
}

// A Gram-Schmidt update: c from coef_in (the first pass, reduced by
// k_lz_coef) or summed here from the chunk partials part_in (the second
// pass), w -= V c on this chunk; then either the partial dots of the second
// pass (last = 0; block 0 records alpha_j = c_j of the first pass) or the
// partial |w|^2 (last = 1).
__device__ __forceinline__ void lz_apply_body(const double* __restrict__ V, double* __restrict__ w,
                                              int64_t n, int j, const double* __restrict__ coef_in,
                                              const double* __restrict__ part_in, int nchunks,
                                              double* __restrict__ part_out, LzState* st, int last) {
  constexpr int kBuf = 64 * kLzCoef;
  __shared__ double red[(kLzChunk / kWave) * kLzCoef];
  __shared__ double coef[kLzCoef];
  __shared__ double buf[kBuf];
  if (st->broke) return;
  if (coef_in) {
    if (threadIdx.x <= j) coef[threadIdx.x] = coef_in[threadIdx.x];
    __syncthreads();
  } else {
    ordered_sums(part_in, nchunks, kLzCoef, j + 1, buf, kBuf, coef);
  }
  const int64_t row = int64_t(blockIdx.x) * kLzChunk + threadIdx.x;
  double wr = 0.0;
  if (row < n) {
    wr = w[row];
    for (int i = 0; i <= j; ++i) wr = fma(-coef[i], V[int64_t(i) * n + row], wr);
    w[row] = wr;
  }
  if (!last) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->alpha[j] = coef[j];
      st->steps = j + 1;
    }
    chunk_dots(V, wr, row, n, j, part_out, red);
  } else {
    const double s = block_sum1<kLzChunk>(wr * wr, red);
    if (threadIdx.x == 0) part_out[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(kLzChunk) void k_lz_apply(const double* __restrict__ V,
                                                       double* __restrict__ w, int64_t n, int j,
                                                       const double* __restrict__ coef_in,
                                                       const double* __restrict__ part_in,
                                                       int nchunks, double* __restrict__ part_out,
                                                       LzState* st, int last) {
  lz_apply_body(V, w, n, j, coef_in, part_in, nchunks, part_out, st, last);
}

// Eigenvalues of the symmetric tridiagonal T (diagonal a, off-diagonal b)
// below x: negative pivots of the LDL^T factorisation of T - x I.
__device__ inline int sturm_count(const double* a, const double* b, int k, double x, double pivmin) {
  int cnt = 0;
  double d = a[0] - x;
  if (fabs(d) < pivmin) d = -pivmin;
  cnt += d < 0.0;
  for (int i = 1; i < k; ++i) {
    d = (a[i] - x) - b[i - 1] * b[i - 1] / d;
    if (fabs(d) < pivmin) d = -pivmin;
    cnt += d < 0.0;
  }
  return cnt;
}

// The eigenvalue of index `idx` (0-based, ascending) of T in [lo, hi] by
// multisection across the 64 lanes of one wave: every round each lane counts
// at one of 64 interior points and the interval shrinks to the first gap
// whose right end holds more than idx eigenvalues below it.
__device__ inline double tridiag_eig(const double* a, const double* b, int k, int idx, double lo,
                                     double hi, double pivmin) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int round = 0; round < 16; ++round) {
    const double step = (hi - lo) / (kWave + 1);
    const double x = lo + (lane + 1) * step;
    const bool above = sturm_count(a, b, k, x, pivmin) > idx;
    const unsigned long long m = __ballot(above);
    double nlo, nhi;
    if (m == 0ull) {
      nlo = __shfl(x, kWave - 1, kWave);
      nhi = hi;
    } else {
      const int f = __ffsll(static_cast<long long>(m)) - 1;
      nhi = __shfl(x, f, kWave);
      nlo = f == 0 ? lo : __shfl(x, f - 1, kWave);
    }
    if (!(nhi - nlo < hi - lo)) break;   // no representable progress left
    lo = nlo;
    hi = nhi;
  }
  return 0.5 * (lo + hi);
}

// |last entry| of the normalised eigenvector of T for the eigenvalue th:
// two steps of inverse iteration from the all-ones vector, with the LU
// factorisation with partial pivoting of the tridiagonal T - th I (the
// scheme of LAPACK's dgttrf / dgttrs; pivots below pivmin replaced by
// pivmin).  Work arrays of length k (in LDS).
__device__ inline double tridiag_last_component(const double* a, const double* b, int k, double th,
                                                double pivmin, double* x, double* dl, double* dd,
                                                double* du, double* du2, int* swp) {
  for (int i = 0; i < k; ++i) {
    dd[i] = a[i] - th;
    du[i] = i + 1 < k ? b[i] : 0.0;
    dl[i] = i + 1 < k ? b[i] : 0.0;
    du2[i] = 0.0;
    swp[i] = 0;
  }
  for (int i = 0; i + 1 < k; ++i) {
    if (fabs(dd[i]) >= fabs(dl[i])) {
      if (fabs(dd[i]) < pivmin) dd[i] = pivmin;
      const double f = dl[i] / dd[i];
      dl[i] = f;
      dd[i + 1] -= f * du[i];
    } else {
      swp[i] = 1;
      const double f = dd[i] / dl[i];
      dd[i] = dl[i];
      dl[i] = f;
      const double t = du[i];
      du[i] = dd[i + 1];
      dd[i + 1] = t - f * dd[i + 1];
      if (i + 2 < k) {
        du2[i] = du[i + 1];
        du[i + 1] = -f * du[i + 1];
      }
    }
  }
  if (fabs(dd[k - 1]) < pivmin) dd[k - 1] = pivmin;
  for (int i = 0; i < k; ++i) x[i] = 1.0;
  for (int iter = 0; iter < 2; ++iter) {
    for (int i = 0; i + 1 < k; ++i) {   // L
      if (swp[i]) {
        const double t = x[i];
        x[i] = x[i + 1];
        x[i + 1] = t - dl[i] * x[i];
      } else {
        x[i + 1] -= dl[i] * x[i];
      }
    }
    x[k - 1] /= dd[k - 1];   // U
    if (k >= 2) x[k - 2] = (x[k - 2] - du[k - 2] * x[k - 1]) / dd[k - 2];
    for (int i = k - 3; i >= 0; --i) x[i] = (x[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / dd[i];
    double nrm = 0.0;
    for (int i = 0; i < k; ++i) nrm = fmax(nrm, fabs(x[i]));
    for (int i = 0; i < k; ++i) x[i] /= nrm;
  }
  double s2 = 0.0;
  for (int i = 0; i < k; ++i) s2 += x[i] * x[i];
  return fabs(x[k - 1]) / sqrt(s2);
}

// Replace the Gershgorin bounds in ctrl by the Ritz interval where tighter.
// One thread does the O(k^2) work.
// The last beta (coupling to the next, unused vector) comes from the norm
// partials of the last step unless the recurrence broke down.
// Two waves: wave 0 finds the smallest Ritz value and its residual, wave 1
// the largest, at the same time; thread 0 then widens and clips.
__global__ __launch_bounds__(2 * kWave) void k_lz_bounds(LzState* st, Ctrl* ctrl, double margin,
                                                         const double* __restrict__ norm_part,
                                                         int nchunks) {
  __shared__ double x[2][kLzMaxSteps], dl[2][kLzMaxSteps], dd[2][kLzMaxSteps],
      du[2][kLzMaxSteps], du2[2][kLzMaxSteps];
  __shared__ int swp[2][kLzMaxSteps];
  __shared__ double sa[kLzMaxSteps], sb[kLzMaxSteps], sbuf[256], snorm, sth[2], sr[2];
  const int k = st->steps;
  if (k <= 0) return;
  if (!st->broke) {
    ordered_sums(norm_part, nchunks, 1, 1, sbuf, 256, &snorm);
    if (threadIdx.x == 0) st->beta[k - 1] = sqrt(snorm);
  }
  __syncthreads();
  if (ctrl->nonfinite || ctrl->degenerate) return;
  // T in LDS: the bisection reads it many times
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    sa[i] = st->alpha[i];
    sb[i] = st->beta[i];
  }
  __syncthreads();
  const double* a = sa;
  const double* b = sb;
  double lo = INFINITY, hi = -INFINITY, scale = 0.0;
  for (int i = 0; i < k; ++i) {
    const double off = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < k ? fabs(b[i]) : 0.0);
    lo = fmin(lo, a[i] - off);
    hi = fmax(hi, a[i] + off);
    scale = fmax(scale, fabs(a[i]) + off);
  }
  scale = fmax(scale, 1e-300);
  const double pivmin = 1e-280 * fmax(1.0, scale * scale);
  const double pad = 1e-14 * (hi - lo) + 1e-14 * scale;
  lo -= pad;
  hi += pad;
  const int wv = threadIdx.x / kWave;   // 0: lowest, 1: highest
  const double th = tridiag_eig(a, b, k, wv == 0 ? 0 : k - 1, lo, hi, pivmin);
  const double tiny = 1e-13 * scale;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sth[wv] = th;
    sr[wv] = fabs(b[k - 1]) * tridiag_last_component(a, b, k, wv == 0 ? th - tiny : th + tiny, tiny,
                                                     x[wv], dl[wv], dd[wv], du[wv], du2[wv],
                                                     swp[wv]);
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double th_lo = sth[0], th_hi = sth[1], r_lo = sr[0], r_hi = sr[1];
  const double m = margin * (th_hi - th_lo);
  const double e_lo = fmax(ctrl->eps_min, th_lo - r_lo - m);
  const double e_hi = fmin(ctrl->eps_max, th_hi + r_hi + m);
  if (isfinite(e_lo) && isfinite(e_hi) && e_hi > e_lo) {
    ctrl->eps_min = e_lo;
    ctrl->eps_max = e_hi;
    ctrl->inv_range = 1.0 / (e_hi - e_lo);
  }
}

// ---------------------------------------------------------------------------
// HOMO/LUMO estimates from a density matrix P (input of the accelerated
// network, Section II.E): the same Lanczos recurrence on the projected
// operator v -> Q ((H - shift I) v), Q = P (occupied side) or I - P (virtual
// side), started from Q u / |Q u|.  For a projector commuting with H the
// vectors stay in the range of Q, where the operator is H - shift I on the
// occupied (virtual) eigenstates; the shift (eps_min, resp. eps_max) keeps
// the zero eigenvalue of the complement on the inner side.  The two sides
// run together.  Each step: y = (H - shift) v_j (k_hl_matvec2, mode 0),
// w = Q y with the first Gram-Schmidt dot partials (mode 1 or 2), the two
// Gram-Schmidt passes of the bound refinement (k_hl_coef2, k_hl_apply2: the
// bodies of k_lz_coef and k_lz_apply), then v_{j+1} = w / |w| (k_hl_next2).
// ---------------------------------------------------------------------------

// The two sides of the estimator at once: out_s = M x_s (mode 0: minus
// shift_s x_s, the shifts eps_min (side 0) and eps_max (side 1) from ctrl;
// mode 1: as is; mode 2: x_s - M x_s) for s = 0, 1, reading M once for
// both; with V_s (rows 0 .. j) and dot_part_s, the partial dots of out_s
// with those rows per work-group (FP32 M, FP64 vectors and sums, 2 rows
// per wave as in k_lz_matvec).  A side whose recurrence broke down is
// skipped.
struct HlTwo {
  const double* x[2];
  double* out[2];
  const double* V[2];       // null: no dot partials
  double* dot_part[2];
  const LzState* st[2];
  int mode[2];
};

__global__ __launch_bounds__(kLzMvThreads) void k_hl_matvec2(const float* __restrict__ M, int64_t n,
                                                    int64_t ld, HlTwo a, const Ctrl* ctrl, int j) {
  __shared__ double dred[2][kLzMvThreads / kWave][kWave];
  const bool live[2] = {!a.st[0]->broke, !a.st[1]->broke};
  if (!live[0] && !live[1]) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t r0 = int64_t(blockIdx.x) * kLzRowsPerBlock + wv * kLzRowsPerWave;
  double acc[2][kLzRowsPerWave];
  const float* mrow[kLzRowsPerWave];
#pragma unroll
  for (int rr = 0; rr < kLzRowsPerWave; ++rr) {
    acc[0][rr] = 0.0;
    acc[1][rr] = 0.0;
    mrow[rr] = M + (r0 + rr < n ? r0 + rr : 0) * ld;
  }
  const bool vec = (ld % 4 == 0) && ((reinterpret_cast<uintptr_t>(M) & 15) == 0);
  rows_dot2(mrow, a.x[0], a.x[1], n, ld, vec, lane, acc[0], acc[1]);
  const double shift[2] = {ctrl->eps_min, ctrl->eps_max};
  double ws[2][kLzRowsPerWave];
#pragma unroll
  for (int sd = 0; sd < 2; ++sd)
#pragma unroll
    for (int rr = 0; rr < kLzRowsPerWave; ++rr) {
      const double sum = wave_sum(acc[sd][rr]);
      const int64_t row = r0 + rr;
      const int mode = a.mode[sd];
      double v = 0.0;
      if (row < n)
        v = mode == 0 ? sum - shift[sd] * a.x[sd][row] : (mode == 1 ? sum : a.x[sd][row] - sum);
      ws[sd][rr] = v;
      if (live[sd] && lane == 0 && row < n) a.out[sd][row] = v;
    }
  if (!a.V[0]) return;
#pragma unroll
  for (int sd = 0; sd < 2; ++sd) {
    double d = 0.0;
    if (lane <= j) {
#pragma unroll
      for (int rr = 0; rr < kLzRowsPerWave; ++rr) {
        const int64_t row = r0 + rr;
        if (row < n) d = fma(a.V[sd][int64_t(lane) * n + row], ws[sd][rr], d);
      }
    }
    dred[sd][wv][lane] = d;
  }
  __syncthreads();
  if (threadIdx.x <= j) {
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      if (!live[sd]) continue;
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < kLzMvThreads / kWave; ++q) t += dred[sd][q][threadIdx.x];
      a.dot_part[sd][int64_t(blockIdx.x) * kLzCoef + threadIdx.x] = t;
    }
  }
}

// Squared-norm partials of w per chunk of 256 rows.
__device__ __forceinline__ void hl_norm_parts_body(const double* __restrict__ w, int64_t n,
                                                   double* __restrict__ part, const LzState* st) {
  __shared__ double red[kLzChunk / kWave];
  if (st->broke) return;
  const int64_t row = int64_t(blockIdx.x) * kLzChunk + threadIdx.x;
  const double v = row < n ? w[row] : 0.0;
  const double s = block_sum1<kLzChunk>(v * v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// v_row = w / |w| with |w|^2 the ordered sum of the chunk partials; records
// beta[row - 1] for row >= 1.  A vanishing norm ends the recurrence (broke;
// with row 0, no step is recorded).  Every work-group sums the partials
// identically.
__device__ __forceinline__ void hl_next_body(double* __restrict__ V, const double* __restrict__ w,
                                             int64_t n, int row, const double* __restrict__ part,
                                             int nchunks, LzState* st) {
  __shared__ double sbuf[256];
  __shared__ double snorm;
  if (st->broke) return;
  ordered_sums(part, nchunks, 1, 1, sbuf, 256, &snorm);
  const double nrm = sqrt(snorm);
  if (!(nrm > 1e-300)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (row > 0) st->beta[row - 1] = nrm;
      st->broke = 1;
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && row > 0) st->beta[row - 1] = nrm;
  const int64_t i = int64_t(blockIdx.x) * kLzChunk + threadIdx.x;
  if (i < n) V[int64_t(row) * n + i] = w[i] * (1.0 / nrm);
}

// The estimator's two recurrences (side 0: occupied, side 1: virtual) share
// every launch of their vector steps: side = blockIdx.y, each with its own
// basis, residual, partials and state, the same arithmetic as one side alone.
struct HlVecs {
  double* V[2];       // basis, (steps + 1) x n
  double* w[2];       // residual
  double* p1[2];      // first Gram-Schmidt pass: partials per matrix-vector work-group
  double* p2[2];      // second pass: partials per chunk
  double* pn[2];      // |w|^2 partials per chunk
  double* pc[2];      // first-pass coefficients
  LzState* st[2];
};

__global__ __launch_bounds__(kLzChunk) void k_hl_norm_parts2(HlVecs a, int64_t n) {
  const int sd = blockIdx.y;
  hl_norm_parts_body(a.w[sd], n, a.pn[sd], a.st[sd]);
}

__global__ __launch_bounds__(kLzChunk) void k_hl_next2(HlVecs a, int64_t n, int row, int nchunks) {
  const int sd = blockIdx.y;
  hl_next_body(a.V[sd], a.w[sd], n, row, a.pn[sd], nchunks, a.st[sd]);
}

__global__ __launch_bounds__(kLzChunk) void k_hl_coef2(HlVecs a, int nparts) {
  const int sd = blockIdx.y;
  lz_coef_body(a.p1[sd], nparts, a.pc[sd], a.st[sd]);
}

// Both Gram-Schmidt passes of step j: pass 0 takes the first-pass
// coefficients and leaves the second pass's partials, pass 1 sums those and
// leaves the |w|^2 partials.
__global__ __launch_bounds__(kLzChunk) void k_hl_apply2(HlVecs a, int64_t n, int j, int nchunks,
                                                      int pass) {
  const int sd = blockIdx.y;
  if (pass == 0)
    lz_apply_body(a.V[sd], a.w[sd], n, j, a.pc[sd], nullptr, 0, a.p2[sd], a.st[sd], 0);
  else
    lz_apply_body(a.V[sd], a.w[sd], n, j, nullptr, a.p2[sd], nchunks, a.pn[sd], a.st[sd], 1);
}

// Extreme Ritz value of the recorded tridiagonal matrix and its residual
// norm |beta_k s_k|: the largest (side 0, into ritz[0..1]) or the smallest
// (side 1, into ritz[2..3]).  One wave.  NaN when no step was recorded.
__global__ __launch_bounds__(kWave) void k_hl_ritz(LzState* st, int side) {
  __shared__ double x[kLzMaxSteps], dl[kLzMaxSteps], dd[kLzMaxSteps], du[kLzMaxSteps],
      du2[kLzMaxSteps], sa[kLzMaxSteps], sb[kLzMaxSteps];
  __shared__ int swp[kLzMaxSteps];
  const int k = st->steps;
  if (k <= 0) {
    if (threadIdx.x == 0) st->ritz[2 * side] = st->ritz[2 * side + 1] = NAN;
    return;
  }
  for (int i = threadIdx.x; i < k; i += kWave) {
    sa[i] = st->alpha[i];
    sb[i] = st->beta[i];
  }
  __syncthreads();
  // an early breakdown leaves beta[k - 1] = 0: the Ritz pair is exact
  double lo = INFINITY, hi = -INFINITY, scale = 0.0;
  for (int i = 0; i < k; ++i) {
    const double off = (i > 0 ? fabs(sb[i - 1]) : 0.0) + (i + 1 < k ? fabs(sb[i]) : 0.0);
    lo = fmin(lo, sa[i] - off);
    hi = fmax(hi, sa[i] + off);
    scale = fmax(scale, fabs(sa[i]) + off);
  }
  scale = fmax(scale, 1e-300);
  const double pivmin = 1e-280 * fmax(1.0, scale * scale);
  const double pad = 1e-14 * (hi - lo) + 1e-14 * scale;
  const double th = tridiag_eig(sa, sb, k, side == 0 ? k - 1 : 0, lo - pad, hi + pad, pivmin);
  if (threadIdx.x == 0) {
    const double tiny = 1e-13 * scale;
    const double bk = st->broke ? 0.0 : sb[k - 1];
    st->ritz[2 * side] = th;
    st->ritz[2 * side + 1] =
        fabs(bk) * tridiag_last_component(sa, sb, k, side == 0 ? th + tiny : th - tiny, tiny, x, dl,
                                          dd, du, du2, swp);
  }
}

}  // namespace sp2
