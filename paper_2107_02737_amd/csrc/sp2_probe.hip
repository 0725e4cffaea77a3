// Matrix-core rate probe (libsp2_probe.so): the layer product's instruction
// sequence on register-resident fragments, with no memory traffic in the
// loop, to measure what the matrix cores reach under the board's power limit
// for operands of given statistics.  Not used by the solver.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sp2_probe.h"

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 pbf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 pf16x8;
typedef __attribute__((ext_vector_type(16))) float pf32x16;
typedef __attribute__((ext_vector_type(4))) uint32_t pu32x4;

constexpr int kMI = 4, kNI = 4;

template <bool FP16>
__device__ __forceinline__ void mma(pf32x16& acc, pu32x4 a, pu32x4 b) {
  if constexpr (FP16)
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(pf16x8, a),
                                                 __builtin_bit_cast(pf16x8, b), acc, 0, 0, 0);
  else
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(pbf16x8, a),
                                                  __builtin_bit_cast(pbf16x8, b), acc, 0, 0, 0);
}

// One K step of the layer kernel per wave: hi*hi for every block, then
// hi*lo, then lo*hi.
template <bool FP16>
__device__ __forceinline__ void step(pf32x16 (&acc)[kMI][kNI], const pu32x4 (&ah)[kMI],
                                     const pu32x4 (&al)[kMI], const pu32x4 (&bh)[kNI],
                                     const pu32x4 (&bl)[kNI]) {
#pragma unroll
  for (int mi = 0; mi < kMI; ++mi)
#pragma unroll
    for (int ni = 0; ni < kNI; ++ni) mma<FP16>(acc[mi][ni], ah[mi], bh[ni]);
#pragma unroll
  for (int mi = 0; mi < kMI; ++mi)
#pragma unroll
    for (int ni = 0; ni < kNI; ++ni) mma<FP16>(acc[mi][ni], ah[mi], bl[ni]);
#pragma unroll
  for (int mi = 0; mi < kMI; ++mi)
#pragma unroll
    for (int ni = 0; ni < kNI; ++ni) mma<FP16>(acc[mi][ni], al[mi], bh[ni]);
}

// Fragment of rows row0 .. row0 + 31 of panel p, K step kt: lane (r, h)
// holds the 8 values of column chunk h of row row0 + r (K-tiled planes:
// 256 x 16 blocks, block (p, kt) at element (p * KT + kt) * 4096, chunk h
// at + h * 2048, row r at + r * 8).
__device__ __forceinline__ pu32x4 frag(const uint16_t* plane, int64_t KT, int p, int kt, int row0,
                                       int lane) {
  const int r = lane & 31, h = lane >> 5;
  const int64_t off = (int64_t(p) * KT + kt) * 4096 + h * 2048 + (row0 + r) * 8;
  return *reinterpret_cast<const pu32x4*>(plane + off);
}

template <bool FP16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_probe_mfma(const uint16_t* __restrict__ hi, const uint16_t* __restrict__ lo, int64_t np,
                  int iters, float* __restrict__ sink, uint64_t* __restrict__ clocks) {
  const int npan = static_cast<int>(np / 256);
  const int64_t KT = np / 16;
  const int b = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int pa = b % npan, pb = (b / npan) % npan;
  pu32x4 ah0[kMI], al0[kMI], bh0[kNI], bl0[kNI], ah1[kMI], al1[kMI], bh1[kNI], bl1[kNI];
#pragma unroll
  for (int mi = 0; mi < kMI; ++mi) {
    ah0[mi] = frag(hi, KT, pa, 0, wm * 128 + mi * 32, lane);
    al0[mi] = frag(lo, KT, pa, 0, wm * 128 + mi * 32, lane);
    ah1[mi] = frag(hi, KT, pa, 1, wm * 128 + mi * 32, lane);
    al1[mi] = frag(lo, KT, pa, 1, wm * 128 + mi * 32, lane);
  }
#pragma unroll
  for (int ni = 0; ni < kNI; ++ni) {
    bh0[ni] = frag(hi, KT, pb, 0, wn * 128 + ni * 32, lane);
    bl0[ni] = frag(lo, KT, pb, 0, wn * 128 + ni * 32, lane);
    bh1[ni] = frag(hi, KT, pb, 1, wn * 128 + ni * 32, lane);
    bl1[ni] = frag(lo, KT, pb, 1, wn * 128 + ni * 32, lane);
  }
  pf32x16 acc[kMI][kNI];
#pragma unroll
  for (int mi = 0; mi < kMI; ++mi)
#pragma unroll
    for (int ni = 0; ni < kNI; ++ni)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[mi][ni][q] = 0.0f;
  __syncthreads();
  const uint64_t c0 = clock64(), t0 = wall_clock64();
  for (int it = 0; it < iters; ++it) {
    step<FP16>(acc, ah0, al0, bh0, bl0);
    step<FP16>(acc, ah1, al1, bh1, bl1);
  }
  __syncthreads();
  const uint64_t c1 = clock64(), t1 = wall_clock64();
  float s = 0.0f;
#pragma unroll
  for (int mi = 0; mi < kMI; ++mi)
#pragma unroll
    for (int ni = 0; ni < kNI; ++ni) s += acc[mi][ni][(mi * kNI + ni) & 15];
  sink[int64_t(b) * 256 + threadIdx.x] = s;
  if (threadIdx.x == 0) {
    clocks[4 * int64_t(b) + 0] = c0;
    clocks[4 * int64_t(b) + 1] = t0;
    clocks[4 * int64_t(b) + 2] = c1;
    clocks[4 * int64_t(b) + 3] = t1;
  }
}

}  // namespace

extern "C" int32_t sp2_probe_mfma(const uint16_t* hi, const uint16_t* lo, int64_t np,
                                  int32_t precision, int32_t iters, int32_t nblocks, float* sink,
                                  uint64_t* clocks, double* wall_hz, void* stream) {
  if (!hi || !lo || !sink || !clocks) return 1;
  if (np < 256 || np % 256 != 0 || np > (int64_t(1) << 17)) return 1;
  if (precision != 2 && precision != 3) return 1;
  if (iters < 1 || iters > 10000000 || nblocks < 1 || nblocks > 65536) return 1;
  if (wall_hz) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
      return 5;
    *wall_hz = 1e3 * khz;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (precision == 3)
    k_probe_mfma<true><<<nblocks, 256, 0, st>>>(hi, lo, np, iters, sink, clocks);
  else
    k_probe_mfma<false><<<nblocks, 256, 0, st>>>(hi, lo, np, iters, sink, clocks);
  return hipGetLastError() == hipSuccess ? 0 : 5;
}
