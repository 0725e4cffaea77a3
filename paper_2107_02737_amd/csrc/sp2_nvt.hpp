// Canonical integration with the force noise as the heat bath (Section IV,
// Eq. 31-33, and the variant of the Supporting Information), one thread per
// scalar coordinate, FP64.
//
//   k_nvt_first   R_k, V_k, F_k, eta_k -> R_{k+1} and the velocity W before
//                 the last half kick (V_{k+3/4} of Eq. 31, V_{k+4/5} of the
//                 variant), in place
//   k_nvt_second  W, F_{k+1} -> V_{k+1}; Eq. 31 solves its last sub-step,
//                 which holds V_{k+1} on both sides
//
// Coefficients per coordinate of mass M: h = dt / (2M); sigma_L =
// sqrt(kT (1 - c_L^2) / M) with c_L = (1 - gamma_L dt/2) / (1 + gamma_L dt/2)
// (host); the variant's friction factor c_TC = (1 - gamma_TC h) /
// (1 + gamma_TC h), gamma_TC a force per velocity.  Every operation is
// written in the order of the formulas, without contraction into fused
// multiply-adds, so the result is the correctly rounded evaluation of
// exactly those formulas.  Every array is streamed once: loads and stores
// are non-temporal, and the launch gives each thread one coordinate.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

namespace sp2 {

constexpr int kNvtThreads = 256;

__global__ __launch_bounds__(kNvtThreads) void k_nvt_first(double* __restrict__ R,
                                                           double* __restrict__ V,
                                                           const double* __restrict__ F,
                                                           const double* __restrict__ eta,
                                                           const double* __restrict__ mass,
                                                           int64_t n, double dt, double kt,
                                                           double gamma_tc, double c_l,
                                                           int scheme) {
#pragma clang fp contract(off)
  const int64_t stride = int64_t(gridDim.x) * kNvtThreads;
  for (int64_t i = int64_t(blockIdx.x) * kNvtThreads + threadIdx.x; i < n; i += stride) {
    const double m = __builtin_nontemporal_load(mass + i);
    const double v = __builtin_nontemporal_load(V + i);
    const double f = __builtin_nontemporal_load(F + i);
    const double r0 = __builtin_nontemporal_load(R + i);
    const double h = dt / (2.0 * m);
    const double sigma_l = sqrt(kt * (1.0 - c_l * c_l) / m);
    const double noise = eta ? sigma_l * __builtin_nontemporal_load(eta + i) : 0.0;
    const double half = 0.5 * dt;
    double w;
    double r;
    if (scheme == 0) {
      const double v1 = v + h * (f - gamma_tc * v);         // V_{k+1/4}
      r = r0 + half * v1;                                   // R_{k+1/2}
      w = c_l * v1 + noise;                                 // V_{k+3/4}
    } else {
      const double a = gamma_tc * dt / (2.0 * m);
      const double s = sqrt((1.0 - a) / (1.0 + a));        // sqrt(c_TC)
      const double v1 = v + h * f;                          // V_{k+1/5}
      r = r0 + half * v1;                                   // R_{k+1/2}
      w = s * (c_l * (s * v1) + noise);                     // V_{k+4/5}
    }
    __builtin_nontemporal_store(r + half * w, R + i);       // R_{k+1}
    __builtin_nontemporal_store(w, V + i);
  }
}

__global__ __launch_bounds__(kNvtThreads) void k_nvt_second(double* __restrict__ V,
                                                            const double* __restrict__ F,
                                                            const double* __restrict__ mass,
                                                            int64_t n, double dt,
                                                            double gamma_tc, int scheme) {
#pragma clang fp contract(off)
  const int64_t stride = int64_t(gridDim.x) * kNvtThreads;
  for (int64_t i = int64_t(blockIdx.x) * kNvtThreads + threadIdx.x; i < n; i += stride) {
    const double m = __builtin_nontemporal_load(mass + i);
    const double kick = __builtin_nontemporal_load(V + i) +
                        dt / (2.0 * m) * __builtin_nontemporal_load(F + i);
    __builtin_nontemporal_store(scheme == 0 ? kick / (1.0 + gamma_tc * dt / (2.0 * m)) : kick,
                                V + i);
  }
}

}  // namespace sp2
