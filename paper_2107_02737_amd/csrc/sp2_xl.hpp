// XL-BOMD kernel building block (Section III, Eq. 27-28): charge-space
// pieces around the density-matrix response.
//
//   k_mulliken        q_I = z_I - 2 sum_{mu in I} P_mu,mu - sub_I
//   k_atom_matvec     y = alpha A x for an n_atoms x n_atoms FP64 matrix
//   k_atom_scale      y = alpha x
//   k_potential_diag  diagonal of H1 = diag(B u) (atom potentials u)
//   k_xl_init / k_xl_step / k_xl_finish
//                     single-work-group bookkeeping of the preconditioned
//                     Krylov (minimal-residual) approximation of K f: the
//                     orthonormal basis, the QR of the responses, the
//                     residual and the final small triangular solve.
//
// Everything is FP64 and every sum runs in a fixed order, so repeated calls
// agree bitwise.  The charge vectors are short (one entry per atom), so the
// bookkeeping runs in one work-group; the cost of a Krylov step is the
// density-matrix response (sp2_jvp) it needs.
#pragma once

#include "sp2_common.hpp"

namespace sp2 {

constexpr int kXlMaxRank = SP2_XL_MAX_RANK;
constexpr int kXlThreads = 1024;

struct XlState {
  double rho[kXlMaxRank + 1];          // minimal residual with k basis vectors
  double R[kXlMaxRank][kXlMaxRank];    // R[l][k]: QR of the responses K0 J v_k
  double t[kXlMaxRank];                // (Q^T K0 f)_k
  int used;                            // basis vectors with a response
  int stop;                            // the next direction vanished
};

// Orbital range of atom i, clamped to [0, n].
__device__ __forceinline__ void atom_range(const int64_t* __restrict__ ptr, int64_t i, int64_t n,
                                           int64_t& lo, int64_t& hi) {
  lo = ptr[i];
  hi = ptr[i + 1];
  lo = lo < 0 ? 0 : (lo > n ? n : lo);
  hi = hi < lo ? lo : (hi > n ? n : hi);
}

// q_I = z_I - 2 sum_{mu in I} P_mu,mu - sub_I  (z, sub optional: 0).
__global__ __launch_bounds__(256) void k_mulliken(const float* __restrict__ P, int64_t n,
                                                  int64_t ld, int64_t na,
                                                  const int64_t* __restrict__ ptr,
                                                  const double* __restrict__ z,
                                                  const double* __restrict__ sub,
                                                  double* __restrict__ q) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= na) return;
  int64_t lo, hi;
  atom_range(ptr, i, n, lo, hi);
  double s = 0.0;
  for (int64_t m = lo; m < hi; ++m) s += static_cast<double>(P[m * ld + m]);
  q[i] = (z ? z[i] : 0.0) - 2.0 * s - (sub ? sub[i] : 0.0);
}

// y = alpha A x, A row-major na x na; one wave per row (lane-strided sums,
// then a butterfly over the wave).
__global__ __launch_bounds__(256) void k_atom_matvec(const double* __restrict__ A,
                                                     const double* __restrict__ x, int64_t na,
                                                     double alpha, double* __restrict__ y) {
  const int64_t row = int64_t(blockIdx.x) * (256 / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= na) return;   // whole waves
  const double* a = A + row * na;
  double s = 0.0;
  for (int64_t j = lane; j < na; j += kWave) s += a[j] * x[j];
  s = wave_sum(s);
  if (lane == 0) y[row] = alpha * s;
}

// y = alpha x.
__global__ __launch_bounds__(256) void k_atom_scale(const double* __restrict__ x, int64_t na,
                                                    double alpha, double* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < na) y[i] = alpha * x[i];
}

// H1_mu,mu = u_I for every orbital mu of atom I (the off-diagonal entries and
// orbitals of no atom are kept zero by the caller).
__global__ __launch_bounds__(256) void k_potential_diag(const double* __restrict__ u,
                                                        const int64_t* __restrict__ ptr,
                                                        int64_t na, int64_t n,
                                                        float* __restrict__ H1, int64_t ld) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= na) return;
  int64_t lo, hi;
  atom_range(ptr, i, n, lo, hi);
  const float v = static_cast<float>(u[i]);
  for (int64_t m = lo; m < hi; ++m) H1[m * ld + m] = v;
}

// Sum over the work-group of one value per thread (fixed order).
__device__ __forceinline__ double xl_block_sum(double a, double* red) {
  constexpr int NW = kXlThreads / kWave;
  a = wave_sum(a);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = a;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += red[i];
  return s;
}

// Dot products of w with rows 0..rows-1 of M (rows of na doubles) into d[].
__device__ __forceinline__ void xl_dots(const double* __restrict__ M, int rows,
                                        const double* __restrict__ w, int64_t na, double* d,
                                        double* red) {
  for (int l = 0; l < rows; ++l) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < na; i += kXlThreads) s += M[l * na + i] * w[i];
    s = xl_block_sum(s, red);
    if (threadIdx.x == 0) d[l] = s;
  }
  __syncthreads();
}

// w <- w - sum_l d_l M_l (rows 0..rows-1).
__device__ __forceinline__ void xl_subtract(const double* __restrict__ M, int rows,
                                            const double* d, double* __restrict__ w, int64_t na) {
  for (int64_t i = threadIdx.x; i < na; i += kXlThreads) {
    double x = w[i];
    for (int l = 0; l < rows; ++l) x -= d[l] * M[l * na + i];
    w[i] = x;
  }
  __syncthreads();
}

// Two-pass classical Gram-Schmidt of w against rows 0..rows-1 of M; the
// coefficients of both passes are added into coef[] when given.  Returns |w|.
__device__ __forceinline__ double xl_orthogonalise(const double* __restrict__ M, int rows,
                                                   double* __restrict__ w, int64_t na,
                                                   double* coef, double* d, double* red) {
  for (int pass = 0; pass < 2; ++pass) {
    xl_dots(M, rows, w, na, d, red);
    if (coef && threadIdx.x == 0)
      for (int l = 0; l < rows; ++l) coef[l] += d[l];
    xl_subtract(M, rows, d, w, na);
  }
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < na; i += kXlThreads) s += w[i] * w[i];
  return sqrt(xl_block_sum(s, red));
}

// v_1 = r0 / |r0|, res = r0, rho_0 = |r0|.
__global__ __launch_bounds__(kXlThreads) void k_xl_init(const double* __restrict__ r0, int64_t na,
                                                        double* __restrict__ V,
                                                        double* __restrict__ res, XlState* st) {
  __shared__ double red[kXlThreads / kWave];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < na; i += kXlThreads) s += r0[i] * r0[i];
  const double nrm = sqrt(xl_block_sum(s, red));
  for (int64_t i = threadIdx.x; i < na; i += kXlThreads) {
    V[i] = nrm > 0.0 ? r0[i] / nrm : 0.0;
    res[i] = r0[i];
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k <= kXlMaxRank; ++k) st->rho[k] = nrm;
    for (int a = 0; a < kXlMaxRank; ++a) {
      st->t[a] = 0.0;
      for (int b = 0; b < kXlMaxRank; ++b) st->R[a][b] = 0.0;
    }
    st->used = 0;
    st->stop = nrm > 0.0 ? 0 : 1;
  }
}

// Step k with the response fk = K0 J v_k: extend the QR of the responses
// (q_k, column k of R), take the component t_k of the residual along q_k,
// and unless `last`, the next basis vector v_{k+1} = fk orthonormalised
// against v_1..v_k (stop when it vanishes).  w1: scratch vector.
__global__ __launch_bounds__(kXlThreads) void k_xl_step(const double* __restrict__ fk, int k,
                                                        int last, int64_t na,
                                                        double* __restrict__ V,
                                                        double* __restrict__ Q,
                                                        double* __restrict__ res,
                                                        double* __restrict__ w1, XlState* st) {
  __shared__ double red[kXlThreads / kWave];
  __shared__ double d[kXlMaxRank];
  __shared__ double coef[kXlMaxRank];
  if (st->stop) return;
  double fs = 0.0;
  for (int64_t i = threadIdx.x; i < na; i += kXlThreads) {
    w1[i] = fk[i];
    fs += fk[i] * fk[i];
  }
  const double fnorm = sqrt(xl_block_sum(fs, red));
  if (threadIdx.x < kXlMaxRank) coef[threadIdx.x] = 0.0;
  __syncthreads();
  // QR of the responses: q_k = (fk - sum_l R_lk q_l) / R_kk
  const double rkk = xl_orthogonalise(Q, k, w1, na, coef, d, red);
  if (!(rkk > 1e-14 * fnorm)) {   // response dependent on the previous ones
    if (threadIdx.x == 0) st->stop = 1;
    return;
  }
  double ts = 0.0;
  for (int64_t i = threadIdx.x; i < na; i += kXlThreads) {
    const double q = w1[i] / rkk;
    Q[int64_t(k) * na + i] = q;
    ts += q * res[i];
  }
  const double tk = xl_block_sum(ts, red);
  double rs = 0.0;
  for (int64_t i = threadIdx.x; i < na; i += kXlThreads) {
    const double r = res[i] - tk * Q[int64_t(k) * na + i];
    res[i] = r;
    rs += r * r;
  }
  const double rho = sqrt(xl_block_sum(rs, red));
  if (threadIdx.x == 0) {
    for (int l = 0; l < k; ++l) st->R[l][k] = coef[l];
    st->R[k][k] = rkk;
    st->t[k] = tk;
    for (int j = k + 1; j <= kXlMaxRank; ++j) st->rho[j] = rho;
    st->used = k + 1;
  }
  if (last) return;
  // next basis vector
  for (int64_t i = threadIdx.x; i < na; i += kXlThreads) w1[i] = fk[i];
  __syncthreads();
  const double beta = xl_orthogonalise(V, k + 1, w1, na, nullptr, d, red);
  if (!(beta > 1e-12 * fnorm)) {
    if (threadIdx.x == 0) st->stop = 1;
    return;
  }
  for (int64_t i = threadIdx.x; i < na; i += kXlThreads) V[int64_t(k + 1) * na + i] = w1[i] / beta;
}

// kf = V c with R c = t (back substitution over the basis vectors used).
__global__ __launch_bounds__(kXlThreads) void k_xl_finish(const double* __restrict__ V, int64_t na,
                                                          const XlState* st,
                                                          double* __restrict__ kf) {
  __shared__ double c[kXlMaxRank];
  const int m = st->used;
  if (threadIdx.x == 0) {
    for (int k = m - 1; k >= 0; --k) {
      double s = st->t[k];
      for (int l = k + 1; l < m; ++l) s -= st->R[k][l] * c[l];
      c[k] = s / st->R[k][k];
    }
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < na; i += kXlThreads) {
    double s = 0.0;
    for (int l = 0; l < m; ++l) s += c[l] * V[int64_t(l) * na + i];
    kf[i] = s;
  }
}

}  // namespace sp2
