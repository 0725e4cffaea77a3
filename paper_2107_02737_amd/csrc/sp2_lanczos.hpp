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
constexpr int kLzThreads = 1024;     // one-work-group kernels
constexpr int kLzRowsPerWave = 4;
constexpr int kLzRowsPerBlock = 4 * kLzRowsPerWave;
constexpr double kLzMargin = 0.01;   // relative widening of the Ritz interval

struct LzState {
  double alpha[kLzMaxSteps];
  double beta[kLzMaxSteps];
  int32_t steps;    // recorded (alpha, beta) pairs
  int32_t broke;    // beta vanished: invariant subspace, later steps skipped
  int32_t pad[2];
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

// w = H v (FP32 H, FP64 products and sums); each wave takes 4 consecutive
// rows so that every v load serves 4 rows.  Block b writes the partial
// sum over its 16 rows of v_i w_i (rows in order).
__global__ __launch_bounds__(256) void k_lz_matvec(const float* __restrict__ H, int64_t n,
                                                   int64_t ld, const double* __restrict__ v,
                                                   double* __restrict__ w,
                                                   double* __restrict__ part, const LzState* st) {
  __shared__ double red[kLzRowsPerBlock];
  if (st->broke) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int64_t r0 = int64_t(blockIdx.x) * kLzRowsPerBlock + wv * kLzRowsPerWave;
  double acc[kLzRowsPerWave] = {0.0, 0.0, 0.0, 0.0};
  const bool vec = (ld % 4 == 0) && ((reinterpret_cast<uintptr_t>(H) & 15) == 0);
  int64_t c_done = 0;
  if (vec) {
    const int64_t n4 = n & ~int64_t(3);
    for (int64_t c = 4 * lane; c < n4; c += 4 * kWave) {
      const double v0 = v[c], v1 = v[c + 1], v2 = v[c + 2], v3 = v[c + 3];
#pragma unroll
      for (int rr = 0; rr < kLzRowsPerWave; ++rr) {
        const int64_t row = r0 + rr;
        if (row < n) {
          const f32x4 h = *reinterpret_cast<const f32x4*>(H + row * ld + c);
          double a = acc[rr];
          a = fma(static_cast<double>(h[0]), v0, a);
          a = fma(static_cast<double>(h[1]), v1, a);
          a = fma(static_cast<double>(h[2]), v2, a);
          a = fma(static_cast<double>(h[3]), v3, a);
          acc[rr] = a;
        }
      }
    }
    c_done = n4;
  }
  for (int64_t c = c_done + lane; c < n; c += kWave) {
    const double vc = v[c];
#pragma unroll
    for (int rr = 0; rr < kLzRowsPerWave; ++rr) {
      const int64_t row = r0 + rr;
      if (row < n) acc[rr] = fma(static_cast<double>(H[row * ld + c]), vc, acc[rr]);
    }
  }
#pragma unroll
  for (int rr = 0; rr < kLzRowsPerWave; ++rr) {
    const double s = wave_sum(acc[rr]);
    const int64_t row = r0 + rr;
    if (lane == 0) {
      double d = 0.0;
      if (row < n) {
        w[row] = s;
        d = v[row] * s;
      }
      red[wv * kLzRowsPerWave + rr] = d;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < kLzRowsPerBlock; ++i) s += red[i];
    part[blockIdx.x] = s;
  }
}

// One Lanczos step after w = H v_j (j = step): alpha_j = sum of the
// partials; w -= alpha_j v_j + beta_{j-1} v_{j-1}; then full
// reorthogonalisation against v_0 .. v_j by two passes of classical
// Gram-Schmidt (c = V^T w, w -= V c), which keeps the recurrence free of
// spurious copies of converged Ritz values and reproducible to rounding;
// beta_j = |w|, v_{j+1} = w / beta_j.
__global__ __launch_bounds__(kLzThreads) void k_lz_update(double* __restrict__ w,
                                                          double* __restrict__ V,
                                                          const double* __restrict__ part,
                                                          int nparts, int64_t n, LzState* st,
                                                          int step) {
  constexpr int NW = kLzThreads / kWave, G = 8;
  __shared__ double red[NW * G];
  __shared__ double coef[kLzMaxSteps + G];
  if (st->broke) return;
  double a = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kLzThreads) a += part[i];
  const double alpha = block_sum1<kLzThreads>(a, red);
  const double bprev = step > 0 ? st->beta[step - 1] : 0.0;
  const double* vj = V + int64_t(step) * n;
  const double* vm = step > 0 ? V + int64_t(step - 1) * n : vj;
  for (int64_t i = threadIdx.x; i < n; i += kLzThreads) w[i] = w[i] - alpha * vj[i] - bprev * vm[i];
  for (int pass = 0; pass < 2; ++pass) {
    for (int g = 0; g <= step; g += G) {
      double c[G];
#pragma unroll
      for (int q = 0; q < G; ++q) c[q] = 0.0;
      for (int64_t i = threadIdx.x; i < n; i += kLzThreads) {
        const double wi = w[i];
#pragma unroll
        for (int q = 0; q < G; ++q)
          if (g + q <= step) c[q] = fma(V[int64_t(g + q) * n + i], wi, c[q]);
      }
#pragma unroll
      for (int q = 0; q < G; ++q) c[q] = wave_sum(c[q]);
      __syncthreads();
      if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
        for (int q = 0; q < G; ++q) red[(threadIdx.x / kWave) * G + q] = c[q];
      }
      __syncthreads();
      if (threadIdx.x < G) {
        double s = 0.0;
        for (int k = 0; k < NW; ++k) s += red[k * G + threadIdx.x];
        coef[g + threadIdx.x] = s;
      }
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += kLzThreads) {
      double s = w[i];
      for (int q = 0; q <= step; ++q) s = fma(-coef[q], V[int64_t(q) * n + i], s);
      w[i] = s;
    }
    __syncthreads();
  }
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kLzThreads) s += w[i] * w[i];
  const double beta = sqrt(block_sum1<kLzThreads>(s, red));
  if (threadIdx.x == 0) {
    st->alpha[step] = alpha;
    st->beta[step] = beta;
    st->steps = step + 1;
    if (!(beta > 1e-300)) st->broke = 1;
  }
  if (!(beta > 1e-300)) return;
  double* vn = V + int64_t(step + 1) * n;
  for (int64_t i = threadIdx.x; i < n; i += kLzThreads) vn[i] = w[i] / beta;
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

// The eigenvalue of index `idx` (0-based, ascending) by bisection.
__device__ inline double tridiag_eig(const double* a, const double* b, int k, int idx, double lo,
                                     double hi, double pivmin) {
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(a, b, k, mid, pivmin) > idx)
      hi = mid;
    else
      lo = mid;
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
__global__ __launch_bounds__(64) void k_lz_bounds(const LzState* st, Ctrl* ctrl, double margin) {
  __shared__ double x[kLzMaxSteps], dl[kLzMaxSteps], dd[kLzMaxSteps], du[kLzMaxSteps],
      du2[kLzMaxSteps];
  __shared__ int swp[kLzMaxSteps];
  if (threadIdx.x != 0) return;
  if (ctrl->nonfinite || ctrl->degenerate) return;
  const int k = st->steps;
  if (k <= 0) return;
  const double* a = st->alpha;
  const double* b = st->beta;
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
  const double th_lo = tridiag_eig(a, b, k, 0, lo, hi, pivmin);
  const double th_hi = tridiag_eig(a, b, k, k - 1, lo, hi, pivmin);
  const double tiny = 1e-13 * scale;
  const double r_lo = fabs(b[k - 1]) *
      tridiag_last_component(a, b, k, th_lo - tiny, tiny, x, dl, dd, du, du2, swp);
  const double r_hi = fabs(b[k - 1]) *
      tridiag_last_component(a, b, k, th_hi + tiny, tiny, x, dl, dd, du, du2, swp);
  const double m = margin * (th_hi - th_lo);
  const double e_lo = fmax(ctrl->eps_min, th_lo - r_lo - m);
  const double e_hi = fmin(ctrl->eps_max, th_hi + r_hi + m);
  if (isfinite(e_lo) && isfinite(e_hi) && e_hi > e_lo) {
    ctrl->eps_min = e_lo;
    ctrl->eps_max = e_hi;
    ctrl->inv_range = 1.0 / (e_hi - e_lo);
  }
}

}  // namespace sp2
