// Host driver and C ABI of the gfx950 DNN-SP2 solver (declared in sp2.h).
//
// One solve: Gershgorin bounds -> input layer (fused split + trace
// partials) -> layer loop -> optional McWeeny refinement -> P.  Every layer
// launch decides its own branch and stop from the FP64 trace partials left
// by the previous launch, so the host never waits between layers; it polls
// the device stop flag once per chunk of layers while the next chunk is
// already queued.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <string>
#include <vector>

#include "sp2_aux.hpp"
#include "sp2_common.hpp"
#include "sp2_gemm.hpp"
#include "sp2_lanczos.hpp"
#include "sp2_nvt.hpp"
#include "sp2_xl.hpp"

using namespace sp2;

// Library-owned workspace of sp2_density_noalloc, for callers that cannot
// allocate device memory.  Each device that runs the library holds its own
// copy until the process ends; every sp2_density_noalloc call on a device
// uses that device's copy (calls that overlap in time on one device race).
// Host code reaches it only through the address hipGetSymbolAddress returns.
static constexpr size_t kNoAllocScratchBytes = SP2_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_err;

sp2_status fail(sp2_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(SP2_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

#define LAUNCH_TRY()                                                                    \
  do {                                                                                  \
    hipError_t e_ = hipGetLastError();                                                  \
    if (e_ != hipSuccess)                                                               \
      return fail(SP2_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e_));   \
  } while (0)

constexpr int64_t kPad = 256;          // matrices are padded to a multiple of this
constexpr int kBand = 4;               // tile-rows per band of the tile schedule
// Layers launched between stop-flag polls: 8, or 2 once a layer is long
// (np >= 4096: ~0.5 ms and more), so that few launches run after the stop
// while the queued chunk still covers the host's poll.
constexpr int kChunk = 8;
constexpr int kChunkLarge = 2;
constexpr int64_t kChunkLargeNp = 4096;
constexpr int kInitBlocksMax = 1024;   // partial pairs written by the input layer
constexpr size_t kPartialBytes = size_t(64) << 20;   // split-K tail accumulators
constexpr int kMaxTailTiles = 1024;                   // split-K tail tiles per launch

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Tape description kept in the workspace for sp2_jvp / sp2_vjp.  The
// bounds of the recorded network are copied here when the forward call
// seals the tape, so that a later bound computation on the same workspace
// (which rewrites the control block) cannot rescale the derivative; such
// calls also clear `valid`.
struct Meta {
  int64_t n, np;
  int32_t precision, refine, every, n_iter;
  int32_t valid;       // 1: tape usable, 2: trivial occupation (P independent of H), 0: none
  int32_t max_iter;
  int32_t flags;       // options flags of the forward call (SP2_FLAG_SPLIT_DERIVATIVES)
  int32_t reserved;
  double eps_min, eps_max, inv_range;   // spectral bounds of the recorded network
  int64_t magic;
};
constexpr int64_t kMetaMagic = 0x5350324d45544131LL;

// Workspace layout (byte offsets), derived from n and the options only.
struct Layout {
  int64_t n, np;
  int nb_split, ntiles_split;
  int init_blocks, gersh_blocks, max_parts;
  size_t off_ctrl, off_hist, off_meta, off_parts0, off_parts1, off_gersh, off_partial;
  size_t off_lz, off_lzvec, off_lzpart;   // Lanczos state, vectors, chunk partials
  size_t off_lz1, off_lzvec1, off_lzpart1;   // the same for the estimator's second side
  int lz_blocks, lz_chunks;
  size_t off_slot0;     // first matrix slot
  size_t slot_bytes;
  int nslots, ntape, every;
  size_t total;
};

int ntiles_of(int nb) { return nb * (nb + 1) / 2; }

bool make_layout(int64_t n, const sp2_options& o, Layout& L) {
  if (n <= 0 || n > (int64_t(1) << 20)) return false;
  L.n = n;
  L.np = round_up(n, kPad);
  L.nb_split = static_cast<int>(L.np / 256);
  L.ntiles_split = ntiles_of(L.nb_split);
  // input layer: work-groups striding over its 32 x 256 tiles
  L.init_blocks = static_cast<int>(std::min<int64_t>(kInitBlocksMax, (L.np / kInRows) * (L.np / kInCols)));
  L.gersh_blocks = static_cast<int>((n + kRowsPerBlock - 1) / kRowsPerBlock);
  // product layers: whole tiles + 8 strips per split-K tail tile
  L.max_parts = std::max({L.ntiles_split + kTailStrips * std::min(L.ntiles_split, kMaxTailTiles),
                          L.init_blocks, kInitBlocksMax});
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o2 = off;
    off = round_up(off + bytes, 256);
    return o2;
  };
  L.off_ctrl = take(sizeof(Ctrl));
  L.off_hist = take(sizeof(Hist));
  L.off_meta = take(sizeof(Meta));
  L.off_parts0 = take(size_t(L.max_parts) * 16);
  L.off_parts1 = take(size_t(L.max_parts) * 16);
  L.off_gersh = take(size_t(L.gersh_blocks) * 24);
  L.off_partial = take(kPartialBytes);
  L.lz_blocks = static_cast<int>((n + kLzRowsPerBlock - 1) / kLzRowsPerBlock);
  L.lz_chunks = static_cast<int>((n + kLzChunk - 1) / kLzChunk);
  L.off_lz = take(sizeof(LzState));
  // Lanczos vectors v_0 .. v_kmax and two w buffers, sized for the largest
  // k so that the layout does not depend on the bound option (the tape
  // reader rebuilds it)
  L.off_lzvec = take(size_t(kLzMaxSteps + 3) * size_t(n) * 8);
  // first-pass dot partials per matvec work-group, second-pass partials and
  // squared-norm partials per 256-row chunk, first-pass coefficients
  L.off_lzpart = take((size_t(L.lz_blocks + L.lz_chunks) * kLzCoef + size_t(L.lz_chunks) + kLzCoef) * 8);
  // the HOMO/LUMO estimator runs its two sides together: a second set
  L.off_lz1 = take(sizeof(LzState));
  L.off_lzvec1 = take(size_t(kLzMaxSteps + 3) * size_t(n) * 8);
  L.off_lzpart1 = take((size_t(L.lz_blocks + L.lz_chunks) * kLzCoef + size_t(L.lz_chunks) + kLzCoef) * 8);
  L.slot_bytes = size_t(L.np) * size_t(L.np) * 4;
  L.every = o.checkpoint_every;
  // slots 0-3: S (FP32), two hi/lo plane pairs (or FP32 ping-pong), S^2 for
  // the refinement.  With a tape: 4 derivative work slots, `every` segment
  // slots and the checkpoints S_0, S_k, S_2k, ...
  L.ntape = L.every > 0 ? o.max_iter / L.every + 1 : 0;
  L.nslots = 4 + (L.every > 0 ? 4 + L.every + L.ntape : 0);
  L.off_slot0 = off;
  L.total = off + L.slot_bytes * size_t(L.nslots);
  return true;
}

struct WS {
  Layout L;
  char* base;
  Ctrl* ctrl;
  Hist* hist;
  Meta* meta;
  double* parts[2];
  double* gersh;
  float* partial;
  LzState* lz;
  double* lzv;      // Lanczos vectors v_0 .. v_kmax, then two w buffers: n doubles each
  double* lzpart;
  LzState* lz1;     // the estimator's second side
  double* lzv1;
  double* lzpart1;
  float* slotf(int i) const { return reinterpret_cast<float*>(base + L.off_slot0 + L.slot_bytes * size_t(i)); }
  uint16_t* hi(int pair) const { return reinterpret_cast<uint16_t*>(slotf(1 + pair)); }
  uint16_t* lo(int pair) const { return hi(pair) + L.np * L.np; }
  // derivative work slots and tape
  float* work(int i) const { return slotf(4 + i); }
  float* seg(int i) const { return slotf(8 + i); }
  float* tape(int i) const { return slotf(8 + L.every + i); }
};

void bind(WS& w, void* ws, const Layout& L) {
  w.L = L;
  w.base = static_cast<char*>(ws);
  w.ctrl = reinterpret_cast<Ctrl*>(w.base + L.off_ctrl);
  w.hist = reinterpret_cast<Hist*>(w.base + L.off_hist);
  w.meta = reinterpret_cast<Meta*>(w.base + L.off_meta);
  w.parts[0] = reinterpret_cast<double*>(w.base + L.off_parts0);
  w.parts[1] = reinterpret_cast<double*>(w.base + L.off_parts1);
  w.gersh = reinterpret_cast<double*>(w.base + L.off_gersh);
  w.partial = reinterpret_cast<float*>(w.base + L.off_partial);
  w.lz = reinterpret_cast<LzState*>(w.base + L.off_lz);
  w.lzv = reinterpret_cast<double*>(w.base + L.off_lzvec);
  w.lzpart = reinterpret_cast<double*>(w.base + L.off_lzpart);
  w.lz1 = reinterpret_cast<LzState*>(w.base + L.off_lz1);
  w.lzv1 = reinterpret_cast<double*>(w.base + L.off_lzvec1);
  w.lzpart1 = reinterpret_cast<double*>(w.base + L.off_lzpart1);
}

// Lanczos tightening of the Gershgorin bounds already in ctrl (no host
// round trip; a NaN H or a degenerate spectrum leaves ctrl as it is).
sp2_status refine_bounds(const WS& w, const float* H, int64_t n, int64_t ld, int steps,
                         int32_t seed, hipStream_t st) {
  const int nc = w.L.lz_chunks;
  double* V = w.lzv;
  double* wb[2] = {w.lzv + int64_t(kLzMaxSteps + 1) * n, w.lzv + int64_t(kLzMaxSteps + 2) * n};
  const int nb = w.L.lz_blocks;
  double* p1 = w.lzpart;                  // first-pass dot partials (per matvec work-group)
  double* p2 = p1 + size_t(nb) * kLzCoef;  // second-pass dot partials
  double* pn = p2 + size_t(nc) * kLzCoef;  // squared-norm partials
  double* pc = pn + nc;                    // first-pass coefficients
  steps = static_cast<int>(std::min<int64_t>(steps, n));
  k_lz_start<<<1, kLzThreads, 0, st>>>(V, n, static_cast<uint64_t>(static_cast<uint32_t>(seed)),
                                       w.lz);
  LAUNCH_TRY();
  for (int j = 0; j < steps; ++j) {
    double* wj = wb[j & 1];
    k_lz_matvec<<<nb, kLzMvThreads, 0, st>>>(H, n, ld, V, wb[(j + 1) & 1], wj, pn, nc, p1, w.lz, j);
    LAUNCH_TRY();
    k_lz_coef<<<j + 1, kLzChunk, 0, st>>>(p1, nb, pc, w.lz);
    LAUNCH_TRY();
    k_lz_apply<<<nc, kLzChunk, 0, st>>>(V, wj, n, j, pc, nullptr, 0, p2, w.lz, 0);
    LAUNCH_TRY();
    k_lz_apply<<<nc, kLzChunk, 0, st>>>(V, wj, n, j, nullptr, p2, nc, pn, w.lz, 1);
    LAUNCH_TRY();
  }
  k_lz_bounds<<<1, 2 * kWave, 0, st>>>(w.lz, w.ctrl, kLzMargin, pn, nc);
  LAUNCH_TRY();
  return SP2_OK;
}

// Compute units of the current device (cached per device and thread, so
// that concurrent callers never share a write).
int device_cus() {
  thread_local int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cache[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    cache[dev] = cus;
  }
  return cache[dev];
}

// Split-K tail plan for ntiles tiles on `slots` concurrent work-groups:
// whole rounds of tiles run unsplit; the tiles of the last partial round are
// split along K so that their pieces fill the machine.
Decomp plan_decomp(const WS& w, int nb, int slots, int ksteps, size_t piece_bytes) {
  Decomp d;
  memset(&d, 0, sizeof(d));
  d.nb = nb;
  d.ntiles = nb * (nb + 1) / 2;
  d.band = kBand;
  d.nfull = d.ntiles;
  d.nsplit = 1;
  d.partial = w.partial;
  if (const char* e = getenv("SP2_NO_SPLITK"))
    if (atoi(e)) return d;
  const int r = slots > 0 ? d.ntiles % slots : 0;
  if (r == 0) return d;
  int s = std::min(slots / r, ksteps / 4);
  s = std::min<int64_t>(s, int64_t(kPartialBytes / piece_bytes) / r);
  if (s < 2 || r > kMaxTailTiles) return d;
  d.nfull = d.ntiles - r;
  d.nsplit = s;
  return d;
}

bool options_ok(const sp2_options& o) {
  return o.precision >= SP2_FP32 && o.precision <= SP2_FP16X3 && o.refine >= SP2_REFINE_NONE &&
         o.refine <= SP2_REFINE_SPLIT && o.max_iter >= 1 && o.max_iter <= SP2_MAX_ITER &&
         (o.stop_rule == 0 || o.stop_rule == 1) && o.checkpoint_every >= 0 &&
         o.checkpoint_every <= SP2_MAX_ITER && o.tol >= 0.0 && o.stall_gate == o.stall_gate &&
         (o.flags & ~(SP2_FLAG_TIME_LAYERS | SP2_FLAG_SPLIT_DERIVATIVES | SP2_FLAG_ACCELERATE)) == 0 &&
         (!(o.flags & SP2_FLAG_ACCELERATE) ||
          (std::isfinite(o.homo) && std::isfinite(o.lumo) && o.homo < o.lumo)) &&
         (o.bound_steps == 0 ||
          (o.bound_steps >= SP2_MIN_BOUND_STEPS && o.bound_steps <= SP2_MAX_BOUND_STEPS));
}

// Stagnation gate of stop rule 1: the caller's, or (stall_gate < 0) the
// larger of 3/16 and n u / 16, u the unit roundoff of the layer operands.
// Below 3/16 every eigenvalue of S_n lies within 1/4 of 0 or 1; the second
// term keeps the gate above the rounding floor of the error estimate, which
// grows with n u.
// Unit roundoff of the layer operands: 8 significant bits for single
// BF16, 16 for the BF16 pair, 22 for the scaled FP16 pair, 24 for FP32.
double unit_roundoff_of(int precision) {
  return precision == SP2_BF16X1   ? 0x1p-8
         : precision == SP2_BF16X3 ? 0x1p-16
         : precision == SP2_FP16X3 ? 0x1p-22
                                   : 0x1p-24;
}

double stall_gate_of(const sp2_options& o, int precision, int64_t n) {
  if (o.stall_gate >= 0.0) return o.stall_gate;
  return std::max(3.0 / 16.0, static_cast<double>(n) * unit_roundoff_of(precision) / 16.0);
}

int split_kind_of(int precision) {
  switch (precision) {
    case SP2_BF16X1: return kBF16X1;
    case SP2_BF16X3: return kBF16X3;
    case SP2_FP16X3: return kFP16X3;
    default: return -1;
  }
}

// Split code used by the epilogue / split kernels: 1 bf16, 2 scaled fp16.
int split_code_of(int precision) {
  if (precision == SP2_FP16X3) return 2;
  if (precision == SP2_BF16X1 || precision == SP2_BF16X3) return 1;
  return 0;
}

float out_scale_of(int precision) {
  return precision == SP2_FP16X3 ? 1.0f / float(1u << (2 * kFp16ScaleLog2)) : 1.0f;
}

// Pinned host mirror of the control block and history, one per thread.
struct HostMirror {
  Ctrl ctrl[2];
  Hist hist;
  Meta meta;
  XlState xl;
  int xl_stop;
  double ritz[4];
};
thread_local HostMirror* g_host = nullptr;

sp2_status host_mirror(HostMirror** out) {
  if (!g_host) {
    void* p = nullptr;
    HIP_TRY(hipHostMalloc(&p, sizeof(HostMirror), hipHostMallocDefault));
    g_host = static_cast<HostMirror*>(p);
  }
  *out = g_host;
  return SP2_OK;
}

Epi make_epi(const Layout& L) {
  Epi e;
  memset(&e, 0, sizeof(e));
  e.np = static_cast<int>(L.np);
  e.ld_out = L.np;
  e.n_valid = static_cast<int>(L.np);
  e.vec_ok = 1;
  e.alpha = 1.0f;
  e.beta = 0.0f;
  e.oscale = 1.0f;
  e.mirror_out = 1;
  return e;
}

Decide make_decide(const WS& w, int mode, int layer) {
  Decide d;
  memset(&d, 0, sizeof(d));
  d.ctrl = w.ctrl;
  d.hist = w.hist;
  d.mode = mode;
  d.layer = layer;
  return d;
}

// Resident work-groups per CU of a kernel (cached per kernel and thread).
template <class K>
int wgs_per_cu(K kernel, int threads) {
  struct Entry { const void* k; int n; };
  thread_local Entry cache[32];
  thread_local int used = 0;
  const void* key = reinterpret_cast<const void*>(kernel);
  for (int i = 0; i < used; ++i)
    if (cache[i].k == key) return cache[i].n;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess || n <= 0)
    n = 1;
  if (used < 32) cache[used++] = Entry{key, n};
  return n;
}

// Work decomposition of a split launch (the same on every call for a
// given layout and device).
template <int KIND>
Decomp split_decomp(const WS& w) {
  constexpr size_t piece = size_t(256) * 4 * 4 * 16 * 4;   // one 256x256 FP32 accumulator
  const int slots = device_cus() * wgs_per_cu(k_sym_split<KIND>, 256);
  return plan_decomp(w, static_cast<int>(w.L.np / 256), slots, static_cast<int>(w.L.np / 32), piece);
}

Decomp split_decomp_of(const WS& w, int precision) {
  const int kind = split_kind_of(precision);
  if (kind == kBF16X3) return split_decomp<kBF16X3>(w);
  if (kind == kBF16X1) return split_decomp<kBF16X1>(w);
  return split_decomp<kFP16X3>(w);
}

// Trace partial pairs written by one split launch: one per whole tile, one
// per strip of every split-K tail tile.
int split_nparts(const Decomp& d) { return d.nfull + kTailStrips * (d.ntiles - d.nfull); }

template <int KIND>
sp2_status launch_split_t(const WS& w, SplitArgs a, hipStream_t st) {
  a.dc = split_decomp<KIND>(w);
  const int ntail = a.dc.ntiles - a.dc.nfull;
  const int grid = a.dc.nfull + ntail * a.dc.nsplit;
  k_sym_split<KIND><<<grid, 256, 0, st>>>(a);
  LAUNCH_TRY();
  if (ntail > 0) {
    a.dec.quiet = 1;   // the product launch already recorded this layer's decision
    k_split_tail<<<ntail * kTailStrips, 256, 0, st>>>(a);
    LAUNCH_TRY();
  }
  return SP2_OK;
}

// Launch a 16-bit split product of planes (a_hi, a_lo) x (b_hi, b_lo)^T
// (planes in the K-tiled layout).
sp2_status launch_split(const WS& w, int precision, const uint16_t* ah, const uint16_t* al,
                        const uint16_t* bh, const uint16_t* bl, const Epi& epi, const Decide& dec,
                        hipStream_t st) {
  SplitArgs a;
  memset(&a, 0, sizeof(a));
  a.a_hi = ah;
  a.a_lo = al;
  a.b_hi = bh;
  a.b_lo = bl;
  a.epi = epi;
  a.epi.oscale = out_scale_of(precision);
  a.dec = dec;
  const int kind = split_kind_of(precision);
  if (kind == kBF16X3) return launch_split_t<kBF16X3>(w, a, st);
  if (kind == kBF16X1) return launch_split_t<kBF16X1>(w, a, st);
  return launch_split_t<kFP16X3>(w, a, st);
}

// BF16X3 two-segment product out = alpha (X Y + Y X) + beta C of two
// symmetric matrices given by their K-tiled planes: A = [X|Y], B = [Y|X].
sp2_status launch_split_pair(const WS& w, const uint16_t* xh, const uint16_t* xl,
                             const uint16_t* yh, const uint16_t* yl, const Epi& epi,
                             const Decide& dec, hipStream_t st) {
  SplitArgs a;
  memset(&a, 0, sizeof(a));
  a.a_hi = xh;
  a.a_lo = xl;
  a.b_hi = yh;
  a.b_lo = yl;
  a.a2_hi = yh;
  a.a2_lo = yl;
  a.b2_hi = xh;
  a.b2_lo = xl;
  a.epi = epi;
  a.epi.oscale = 1.0f;
  a.dec = dec;
  constexpr size_t piece = size_t(256) * 4 * 4 * 16 * 4;
  const int slots = device_cus() * wgs_per_cu(k_sym_split<kBF16X3, 2>, 256);
  a.dc = plan_decomp(w, static_cast<int>(w.L.np / 256), slots, static_cast<int>(w.L.np / 32) * 2,
                     piece);
  const int ntail = a.dc.ntiles - a.dc.nfull;
  k_sym_split<kBF16X3, 2><<<a.dc.nfull + ntail * a.dc.nsplit, 256, 0, st>>>(a);
  LAUNCH_TRY();
  if (ntail > 0) {
    a.dec.quiet = 1;
    k_split_tail<<<ntail * kTailStrips, 256, 0, st>>>(a);
    LAUNCH_TRY();
  }
  return SP2_OK;
}

// Work decomposition of an FP32 product over nseg K segments.
Decomp f32_decomp(const WS& w, int nseg) {
  constexpr size_t piece = size_t(256) * 4 * 4 * 16 * 4;   // one 256x256 FP32 accumulator
  const int slots = device_cus() * wgs_per_cu(k_sym_f32, 256);
  return plan_decomp(w, static_cast<int>(w.L.np / 256), slots,
                     static_cast<int>(w.L.np / 32) * nseg, piece);
}

// Launch an FP32 product sum_s A_s B_s^T (nseg <= 4; row-major operands,
// leading dimension np), then the strip kernel for its split-K tail tiles.
sp2_status launch_f32(const WS& w, int nseg, const float* const* A, const float* const* B,
                      const Epi& epi, const Decide& dec, hipStream_t st) {
  F32Args a;
  memset(&a, 0, sizeof(a));
  for (int s = 0; s < nseg; ++s) {
    a.a[s] = A[s];
    a.b[s] = B[s];
  }
  a.nseg = nseg;
  a.epi = epi;
  a.dec = dec;
  a.dc = f32_decomp(w, nseg);
  const int ntail = a.dc.ntiles - a.dc.nfull;
  k_sym_f32<<<a.dc.nfull + ntail * a.dc.nsplit, 256, 0, st>>>(a);
  LAUNCH_TRY();
  if (ntail > 0) {
    SplitArgs t;
    memset(&t, 0, sizeof(t));
    t.epi = a.epi;
    t.dc = a.dc;
    t.dec = a.dec;
    t.dec.quiet = 1;   // the product launch already recorded this layer's decision
    k_split_tail<<<ntail * kTailStrips, 256, 0, st>>>(t);
    LAUNCH_TRY();
  }
  return SP2_OK;
}

int nparts_of_layer(const WS& w, int precision, int layer) {
  if (layer == 0) return w.L.init_blocks;
  return split_nparts(precision == SP2_FP32 ? f32_decomp(w, 1) : split_decomp_of(w, precision));
}

// Where S_n lives in the forward network (FP32 value and hi/lo planes).
float* s_f32(const WS& w, int precision, int n) {
  return precision == SP2_FP32 ? w.slotf(n & 1) : w.slotf(0);
}

// One forward layer S_n -> S_{n+1}.  mode 1: device decision; mode 2: replay
// the recorded layer.  src/dst FP32 buffers may alias (split modes only).
sp2_status launch_layer(const WS& w, int precision, int n, int mode, const float* src, float* dst,
                        int pair_in, int pair_out, double* parts_out, hipStream_t st,
                        const sp2_options* o, int64_t n_occ, bool full_out = true) {
  Decide d = make_decide(w, mode, n);
  if (mode == 1) {
    d.parts_in = w.parts[n & 1];
    d.nparts_in = nparts_of_layer(w, precision, n);
    d.n_occ = static_cast<double>(n_occ);
    d.tol = o->tol;
    d.stall_gate = stall_gate_of(*o, precision, w.L.n);
    d.stop_rule = o->stop_rule;
  }
  Epi e = make_epi(w.L);
  e.c = src;
  e.out = dst;
  e.parts_out = parts_out;
  e.n_diag = static_cast<int>(w.L.n);   // the c I term of a shifted layer: real rows only
  if (precision == SP2_FP32) {
    const float* A[1] = {src};
    return launch_f32(w, 1, A, A, e, d, st);
  }
  e.split_out = split_code_of(precision);
  e.hi_out = w.hi(pair_out);
  e.lo_out = w.lo(pair_out);
  // Planes of S_n - I/2 in, planes of S_{n+1} - I/2 out (kPlaneCentre):
  // S^2 = (S - I/2)^2 + S - I/4, so every layer reads C = S_n.
  e.centring = kCentredSquare | kCentredOut;
  // The next split layer reads only the planes and the upper triangle of C.
  e.mirror_out = full_out ? 1 : 0;
  return launch_split(w, precision, w.hi(pair_in), w.lo(pair_in), w.hi(pair_in), w.lo(pair_in), e,
                      d, st);
}

// Complete an FP32 iterate that split layers left upper-triangle-only.
sp2_status mirror_upper(const WS& w, const float* X, float* Y, hipStream_t st) {
  const int nb = static_cast<int>(w.L.np / kMirrorTile);
  const bool in_place = X == Y;
  k_mirror_upper<<<in_place ? nb * (nb + 1) / 2 : nb * nb, 256, 0, st>>>(X, Y, w.L.np,
                                                                       in_place ? 1 : 0);
  LAUNCH_TRY();
  return SP2_OK;
}

sp2_status check_ws(const Layout& L, void* ws, size_t ws_bytes) {
  if (!ws) return fail(SP2_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(SP2_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(SP2_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  return SP2_OK;
}

int ew_grid(int64_t elems) {
  return static_cast<int>(std::min<int64_t>(8192, std::max<int64_t>(1, (elems + kEwThreads - 1) / kEwThreads)));
}

__global__ void k_write_meta(Meta* m, Meta v) { *m = v; }

// Seal the tape of a finished forward call: the description `v` with the
// bounds the input layer used, usable only for a converged, non-degenerate
// network (the derivative of an unconverged one is not that of P).
__global__ void k_seal_tape(Meta* m, Meta v, const Ctrl* c) {
  v.eps_min = c->eps_min;
  v.eps_max = c->eps_max;
  v.inv_range = c->inv_range;
  if (v.valid == 1 && !(c->converged && !c->degenerate)) v.valid = 0;
  *m = v;
}

// A call that reuses the workspace header for other work drops the tape.
__global__ void k_drop_tape(Meta* m) { m->valid = 0; }

// Events of this thread on the current device, created on first use and
// kept until the process ends (a solve records into them; creating and
// destroying hundreds of events per solve would cost more than the
// records).  Timing events for SP2_FLAG_TIME_LAYERS; two untimed events for
// the stop-flag polls.
struct EventPool {
  int dev = -1;
  std::vector<hipEvent_t> timed;
  hipEvent_t poll[2] = {nullptr, nullptr};
};

hipError_t event_pool(EventPool** out, size_t timed) {
  thread_local EventPool pools[16];
  int dev = 0;
  hipError_t r = hipGetDevice(&dev);
  if (r != hipSuccess) return r;
  if (dev < 0 || dev >= 16) return hipErrorInvalidDevice;
  EventPool& p = pools[dev];
  if (!p.poll[0]) {
    for (auto& e : p.poll)
      if ((r = hipEventCreateWithFlags(&e, hipEventDisableTiming)) != hipSuccess) return r;
  }
  while (p.timed.size() < timed) {
    hipEvent_t e = nullptr;
    if ((r = hipEventCreate(&e)) != hipSuccess) return r;
    p.timed.push_back(e);
  }
  *out = &p;
  return hipSuccess;
}

// Timing events for SP2_FLAG_TIME_LAYERS: a start and an end event around
// every layer launch and around the refinement.
struct LayerTimer {
  hipEvent_t* ev = nullptr;
  bool on = false;
  hipError_t init(int max_iter) {
    EventPool* p = nullptr;
    hipError_t r = event_pool(&p, size_t(2 * max_iter + 2));
    if (r != hipSuccess) return r;
    ev = p->timed.data();
    on = true;
    return hipSuccess;
  }
  hipError_t mark(int idx, hipStream_t st) { return on ? hipEventRecord(ev[idx], st) : hipSuccess; }
  // summed milliseconds of pairs (2k, 2k+1) for k in [k0, k1)
  double sum(int k0, int k1) const {
    double t = 0.0;
    for (int k = k0; k < k1; ++k) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]) == hipSuccess) t += ms;
    }
    return t;
  }
};

// McWeeny refinement P = 3 S^2 - 2 S^3 into `out` (leading dimension ld,
// n valid rows/cols); writes trace partials into parts[0].
sp2_status refine(const WS& w, int precision, int refine_mode, int n_iter, const float* S,
                  float* out, int64_t ld, int64_t n, bool vec_ok, hipStream_t st) {
  const Layout& L = w.L;
  float* S2 = w.slotf(3);
  Epi e1 = make_epi(L);
  e1.out = S2;
  Epi e2 = make_epi(L);
  e2.c = S2;
  e2.out = out;
  e2.ld_out = ld;
  e2.n_valid = static_cast<int>(n);
  e2.vec_ok = vec_ok;
  e2.alpha = -2.0f;
  e2.beta = 3.0f;
  e2.parts_out = w.parts[0];
  const Decide d0 = make_decide(w, 0, 0);
  sp2_status s;
  if (refine_mode == SP2_REFINE_FP32) {
    const float* A[1] = {S};
    if ((s = launch_f32(w, 1, A, A, e1, d0, st))) return s;
    const float* B[1] = {S2};
    if ((s = launch_f32(w, 1, A, B, e2, d0, st))) return s;
    return SP2_OK;
  }
  // FP16X3 split refinement with S's planes centred (c = kPlaneCentre, pair
  // p): Q = S^2 = (S - cI)^2 + 2c S - c^2 I, its plain planes in pair 1-p,
  // then P = 3Q - 2SQ = -2 (S - cI) Q + (3 - 2c) Q.
  constexpr float c = kPlaneCentre;
  const int p = precision == SP2_FP32 ? 0 : (n_iter & 1);
  if (precision != SP2_FP16X3) {
    k_split_tiled<<<L.init_blocks, kEwThreads, 0, st>>>(S, L.np, L.np, L.np, w.hi(p), w.lo(p), 2,
                                                        c, L.n);
    LAUNCH_TRY();
  }
  Epi f1 = e1;
  f1.c = S;
  f1.beta = 2.0f * c;
  f1.gamma = -c * c;
  f1.n_diag = static_cast<int>(L.n);
  f1.mirror_out = 0;   // the second product reads only the upper triangle of Q
  f1.split_out = 2;
  f1.hi_out = w.hi(1 - p);
  f1.lo_out = w.lo(1 - p);
  if ((s = launch_split(w, SP2_FP16X3, w.hi(p), w.lo(p), w.hi(p), w.lo(p), f1, d0, st))) return s;
  Epi f2 = e2;
  f2.beta = 3.0f - 2.0f * c;
  return launch_split(w, SP2_FP16X3, w.hi(p), w.lo(p), w.hi(1 - p), w.lo(1 - p), f2, d0, st);
}

sp2_status read_back(const WS& w, HostMirror* hm, bool with_hist, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(&hm->ctrl[0], w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
  if (with_hist) HIP_TRY(hipMemcpyAsync(&hm->hist, w.hist, sizeof(Hist), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SP2_OK;
}

constexpr int kMaxDevices = 64;

sp2_status check_density_args(const float* H, int64_t n, int64_t ld, int64_t n_occ,
                              const sp2_options& o, const float* P, const uint8_t* branches,
                              int32_t branches_cap, Layout& L);
sp2_status noalloc_scratch(void** out);
sp2_status density_impl(const float* H, int64_t n, int64_t ld, int64_t n_occ, const sp2_options& o,
                        const Layout& L, float* P, sp2_info* info, uint8_t* branches,
                        int32_t branches_cap, void* workspace, hipStream_t st, HostMirror* hm,
                        bool pinned);

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

void sp2_default_options(sp2_options* opt) {
  if (!opt) return;
  memset(opt, 0, sizeof(*opt));
  opt->precision = SP2_BF16X3;
  opt->refine = SP2_REFINE_FP32;
  opt->max_iter = 100;
  opt->stop_rule = 1;
  opt->checkpoint_every = 0;
  opt->tol = 1e-5;
  opt->stall_gate = -1.0;
}

const char* sp2_last_error(void) { return g_err.c_str(); }

size_t sp2_workspace_bytes(int64_t n, const sp2_options* opt) {
  sp2_options o;
  sp2_default_options(&o);
  if (opt) o = *opt;
  if (!options_ok(o)) return 0;
  Layout L;
  if (!make_layout(n, o, L)) return 0;
  return L.total;
}

sp2_status sp2_density_ex(const float* H, int64_t n, int64_t ld, int64_t n_occ,
                          const sp2_options* opt, float* P, sp2_info* info, uint8_t* branches,
                          int32_t branches_cap, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  sp2_options o;
  sp2_default_options(&o);
  if (opt) o = *opt;
  Layout L;
  if (sp2_status s = check_density_args(H, n, ld, n_occ, o, P, branches, branches_cap, L)) return s;
  if (sp2_status s = check_ws(L, workspace, ws_bytes)) return s;
  HostMirror* hm;
  if (sp2_status s = host_mirror(&hm)) return s;
  return density_impl(H, n, ld, n_occ, o, L, P, info, branches, branches_cap, workspace,
                      static_cast<hipStream_t>(stream), hm, true);
}

sp2_status sp2_density_noalloc(const float* H, int64_t n, int64_t ld, int64_t n_occ,
                               const sp2_options* opt, float* P, sp2_info* info,
                               uint8_t* branches, int32_t branches_cap, void* stream) {
  g_err.clear();
  sp2_options o;
  sp2_default_options(&o);
  if (opt) o = *opt;
  Layout L;
  if (sp2_status s = check_density_args(H, n, ld, n_occ, o, P, branches, branches_cap, L)) return s;
  if (o.checkpoint_every != 0)
    return fail(SP2_ERR_INVALID_ARG, "sp2_density_noalloc keeps no derivative tape");
  if (o.flags & SP2_FLAG_TIME_LAYERS)
    return fail(SP2_ERR_INVALID_ARG, "sp2_density_noalloc does not time layers");
  if (L.total > kNoAllocScratchBytes)
    return fail(SP2_ERR_INVALID_ARG, "n = %lld needs %zu bytes of scratch; the static scratch holds %zu",
                static_cast<long long>(n), L.total, kNoAllocScratchBytes);
  void* ws = nullptr;
  if (sp2_status s = noalloc_scratch(&ws)) return s;
  thread_local HostMirror pageable;   // plain host memory: no pinned allocation
  return density_impl(H, n, ld, n_occ, o, L, P, info, branches, branches_cap, ws,
                      static_cast<hipStream_t>(stream), &pageable, false);
}

}  // extern "C"

namespace {

sp2_status check_density_args(const float* H, int64_t n, int64_t ld, int64_t n_occ,
                              const sp2_options& o, const float* P, const uint8_t* branches,
                              int32_t branches_cap, Layout& L) {
  if (!H || !P) return fail(SP2_ERR_INVALID_ARG, "H and P must be non-NULL");
  if (n <= 0 || ld < n) return fail(SP2_ERR_INVALID_ARG, "need n > 0 and ld >= n");
  if (n_occ < 0 || n_occ > n) return fail(SP2_ERR_INVALID_ARG, "n_occ must lie in [0, n]");
  if (!options_ok(o)) return fail(SP2_ERR_INVALID_ARG, "invalid options");
  if (branches_cap < 0 || (branches_cap > 0 && !branches))
    return fail(SP2_ERR_INVALID_ARG, "branches buffer missing");
  if (!make_layout(n, o, L)) return fail(SP2_ERR_INVALID_ARG, "matrix order out of range");
  return SP2_OK;
}

// Device address of the static scratch array on the current device, looked
// up once per device (each device holds its own copy of the array).
sp2_status noalloc_scratch(void** out) {
  static std::atomic<void*> table[kMaxDevices];
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SP2_ERR_DEVICE, "device index %d out of range", dev);
  void* p = table[dev].load(std::memory_order_acquire);
  if (!p) {
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || reinterpret_cast<uintptr_t>(p) % 256)
      return fail(SP2_ERR_DEVICE, "static scratch missing or misaligned");
    table[dev].store(p, std::memory_order_release);
  }
  *out = p;
  return SP2_OK;
}

// One solve on a bound workspace.  `pinned`: hm is pinned host memory, and
// the layer loop polls the stop flag of chunk c asynchronously (events)
// while chunk c+1 runs; otherwise (plain host memory) it synchronises the
// stream after every chunk.
sp2_status density_impl(const float* H, int64_t n, int64_t ld, int64_t n_occ, const sp2_options& o,
                        const Layout& L, float* P, sp2_info* info, uint8_t* branches,
                        int32_t branches_cap, void* workspace, hipStream_t st, HostMirror* hm,
                        bool pinned) {
  WS w;
  bind(w, workspace, L);
  const int prec = o.precision;
  const bool trivial = n_occ == 0 || n_occ == n;
  const bool vec_ok = (ld % 4 == 0) && (reinterpret_cast<uintptr_t>(P) % 16 == 0);
  sp2_status s;

  {
    Meta none{n, L.np, prec, o.refine, 0, 0, 0, o.max_iter, 0, 0, 0.0, 0.0, 0.0, kMetaMagic};
    k_write_meta<<<1, 1, 0, st>>>(w.meta, none);
    LAUNCH_TRY();
  }
  // Spectral bounds (FP64 Gershgorin discs) and control reset.
  k_gershgorin_rows<<<L.gersh_blocks, kRowThreads, 0, st>>>(H, n, ld, w.gersh);
  LAUNCH_TRY();
  k_bounds_final<<<1, 256, 0, st>>>(w.gersh, L.gersh_blocks, w.ctrl, trivial ? 1 : 0);
  LAUNCH_TRY();
  if (!trivial && o.bound_steps > 0)
    if ((s = refine_bounds(w, H, n, ld, o.bound_steps, o.bound_seed, st))) return s;
  if (!trivial && (o.flags & SP2_FLAG_ACCELERATE)) {
    k_acc_schedule<<<1, 1, 0, st>>>(w.ctrl, w.hist, o.homo, o.lumo, o.max_iter);
    LAUNCH_TRY();
  }

  int n_iter = 0;
  bool n_iter_even_for_refine = false;
  if (trivial) {
    k_fill_diag<<<ew_grid(n * n), kEwThreads, 0, st>>>(P, n, ld, n_occ == 0 ? 0.0f : 1.0f);
    LAUNCH_TRY();
    if ((s = read_back(w, hm, false, st))) return s;
    if (hm->ctrl[0].nonfinite) return fail(SP2_ERR_NONFINITE, "H holds NaN or Inf");
    if (o.checkpoint_every > 0) {
      Meta m{n, L.np, prec, o.refine, o.checkpoint_every, 0, 2, o.max_iter, o.flags, 0,
             0.0, 0.0, 0.0, kMetaMagic};
      k_seal_tape<<<1, 1, 0, st>>>(w.meta, m, w.ctrl);
      LAUNCH_TRY();
    }
    if (info) {
      memset(info, 0, sizeof(*info));
      info->converged = 1;
      info->eps_min = hm->ctrl[0].eps_min;
      info->eps_max = hm->ctrl[0].eps_max;
      info->trace = static_cast<double>(n_occ);
    }
    return SP2_OK;
  }

  // Input layer S_0 with its split planes (pair 0) and trace partials.
  k_input_layer<<<L.init_blocks, kEwThreads, 0, st>>>(H, n, ld, L.np, w.ctrl, w.slotf(0), w.hi(0),
                                                      w.lo(0), split_code_of(prec), kPlaneCentre,
                                                      w.parts[0]);
  LAUNCH_TRY();
  if (o.checkpoint_every > 0) HIP_TRY(hipMemcpyAsync(w.tape(0), w.slotf(0), L.slot_bytes, hipMemcpyDeviceToDevice, st));

  LayerTimer timer;
  if (o.flags & SP2_FLAG_TIME_LAYERS) HIP_TRY(timer.init(o.max_iter));
  const int refine_ev = o.max_iter;   // event pair index of the refinement

  // Layer loop in chunks; poll the stop flag of chunk c while chunk c+1 runs.
  hipEvent_t* ev = nullptr;
  if (pinned) {
    EventPool* pool = nullptr;
    HIP_TRY(event_pool(&pool, 0));
    ev = pool->poll;
  }
  int launched = 0, chunk = 0;
  bool stopped = false;
  int stop_slot = -1;   // host copy of the control block that showed the stop
  sp2_status err = SP2_OK;
  while (!stopped && launched < o.max_iter && err == SP2_OK) {
    const int end = std::min(o.max_iter, launched + (L.np >= kChunkLargeNp ? kChunkLarge : kChunk));
    for (int k = launched; k < end && err == SP2_OK; ++k) {
      const float* src = s_f32(w, prec, k);
      float* dst = s_f32(w, prec, k + 1);
      if (timer.mark(2 * k, st) != hipSuccess) err = fail(SP2_ERR_DEVICE, "event record failed");
      if (err == SP2_OK)
        err = launch_layer(w, prec, k, 1, src, dst, k & 1, (k + 1) & 1, w.parts[(k + 1) & 1], st, &o,
                           n_occ, prec == SP2_FP32);
      if (err == SP2_OK && timer.mark(2 * k + 1, st) != hipSuccess)
        err = fail(SP2_ERR_DEVICE, "event record failed");
      if (err == SP2_OK && o.checkpoint_every > 0 && (k + 1) % o.checkpoint_every == 0) {
        if (prec == SP2_FP32) {
          hipError_t e = hipMemcpyAsync(w.tape((k + 1) / o.checkpoint_every), dst, L.slot_bytes,
                                        hipMemcpyDeviceToDevice, st);
          if (e != hipSuccess) err = fail(SP2_ERR_DEVICE, "tape copy: %s", hipGetErrorString(e));
        } else {
          err = mirror_upper(w, dst, w.tape((k + 1) / o.checkpoint_every), st);
        }
      }
    }
    launched = end;
    if (err != SP2_OK) break;
    const int slot = chunk & 1;
    hipError_t e = hipMemcpyAsync(&hm->ctrl[slot], w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st);
    if (!pinned) {
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) { err = fail(SP2_ERR_DEVICE, "poll: %s", hipGetErrorString(e)); break; }
      if (hm->ctrl[slot].stopped) {
        stopped = true;
        stop_slot = slot;
      }
      ++chunk;
      continue;
    }
    if (e == hipSuccess) e = hipEventRecord(ev[slot], st);
    if (e != hipSuccess) { err = fail(SP2_ERR_DEVICE, "poll: %s", hipGetErrorString(e)); break; }
    if (chunk > 0) {
      e = hipEventSynchronize(ev[slot ^ 1]);
      if (e != hipSuccess) { err = fail(SP2_ERR_DEVICE, "poll sync: %s", hipGetErrorString(e)); break; }
      if (hm->ctrl[slot ^ 1].stopped) {
        stopped = true;
        stop_slot = slot ^ 1;
      }
    }
    ++chunk;
  }
  if (err != SP2_OK) return err;
  // Once the stop flag is set the control block no longer changes (later
  // layer launches exit at entry), so the host copy that showed it is final
  // and the rest of the solve is queued behind those launches without
  // waiting.  (A copy of the last chunk may still be landing in the other
  // host slot.)  At the layer cap: the freshest copy after the queue drains.
  if (!stopped) {
    if ((s = read_back(w, hm, false, st))) return s;
    stop_slot = 0;
  }
  const Ctrl cl = hm->ctrl[stop_slot];
  if (cl.nonfinite) {
    HIP_TRY(hipStreamSynchronize(st));   // nothing of this call lands after it returns
    return fail(SP2_ERR_NONFINITE, "H holds NaN or Inf");
  }
  if (cl.acc_failed) {
    // The estimates did not bracket the gap (trace check at the end of the
    // schedule): run the plain network from the start.
    sp2_options plain = o;
    plain.flags &= ~SP2_FLAG_ACCELERATE;
    const sp2_status r = density_impl(H, n, ld, n_occ, plain, L, P, info, branches, branches_cap,
                                      workspace, st, hm, pinned);
    if (info) info->fallback = 1;
    return r;
  }
  if (!cl.stopped) {
    k_finish_loop<<<1, 256, 0, st>>>(w.ctrl, w.hist, w.parts[o.max_iter & 1],
                                     nparts_of_layer(w, prec, o.max_iter), o.max_iter,
                                     static_cast<double>(n_occ), o.tol, o.stop_rule,
                                     stall_gate_of(o, prec, n));
    LAUNCH_TRY();
    n_iter = o.max_iter;
  } else {
    n_iter = cl.n_iter;
  }
  const float* S = s_f32(w, prec, n_iter);
  // split layers wrote the FP32 iterate's upper triangle only
  if (prec != SP2_FP32 && n_iter > 0)
    if ((s = mirror_upper(w, S, const_cast<float*>(S), st))) return s;
  if (o.refine == SP2_REFINE_SPLIT && prec == SP2_FP32 && (n_iter & 1)) {
    // S sits in slot 1, which the split refinement uses for hi/lo planes.
    HIP_TRY(hipMemcpyAsync(w.slotf(0), S, L.slot_bytes, hipMemcpyDeviceToDevice, st));
    S = w.slotf(0);
    n_iter_even_for_refine = true;
  }

  if (o.refine != SP2_REFINE_NONE && !cl.degenerate) {
    HIP_TRY(timer.mark(2 * refine_ev, st));
    if ((s = refine(w, prec, o.refine, n_iter_even_for_refine ? 0 : n_iter, S, P, ld, n, vec_ok, st)))
      return s;
    HIP_TRY(timer.mark(2 * refine_ev + 1, st));
    k_sum_parts<<<1, 256, 0, st>>>(w.ctrl, w.parts[0],
                                   split_nparts(o.refine == SP2_REFINE_FP32
                                                    ? f32_decomp(w, 1)
                                                    : split_decomp_of(w, SP2_FP16X3)));
    LAUNCH_TRY();
  } else {
    k_copy_scaled<<<ew_grid(n * n), kEwThreads, 0, st>>>(S, L.np, P, ld, n, n, 1.0f, 0);
    LAUNCH_TRY();
  }
  if (o.checkpoint_every > 0) {
    Meta m{n, L.np, prec, o.refine, o.checkpoint_every, n_iter, 1, o.max_iter, o.flags, 0,
           0.0, 0.0, 0.0, kMetaMagic};
    k_seal_tape<<<1, 1, 0, st>>>(w.meta, m, w.ctrl);
    LAUNCH_TRY();
  }
  if ((s = read_back(w, hm, true, st))) return s;
  const Ctrl& c = hm->ctrl[0];
  const bool refined = o.refine != SP2_REFINE_NONE && !c.degenerate;
  const int32_t nit = c.n_iter;
  const double t1 = refined ? c.final_t1 : hm->hist.t1[nit];
  const double t2 = refined ? c.final_t2 : hm->hist.t2[nit];
  const bool converged = c.converged && !c.degenerate;
  if (info) {
    info->n_iter = nit;
    info->converged = converged ? 1 : 0;
    info->eps_min = c.eps_min;
    info->eps_max = c.eps_max;
    info->trace = t1;
    info->idem_err = fabs(t1 - t2);
    info->fallback = 0;
    info->layer_ms = timer.on ? timer.sum(0, nit) : 0.0;
    info->refine_ms = (timer.on && refined) ? timer.sum(refine_ev, refine_ev + 1) : 0.0;
  }
  for (int k = 0; k < std::min<int32_t>(nit, branches_cap); ++k)
    branches[k] = hm->hist.branch[k] > 0 ? 1 : 0;
  sp2_status ret = SP2_OK;
  if (c.degenerate) ret = fail(SP2_ERR_NOT_CONVERGED, "degenerate spectrum (eps_max == eps_min): no gap");
  else if (!converged) ret = fail(SP2_ERR_NOT_CONVERGED, "stop test not met within %d layers", o.max_iter);
  if (info) info->status = ret;
  return ret;
}

}  // namespace

extern "C" {

sp2_status sp2_density(const float* H, int64_t n, int64_t n_occ, double tol, float* P,
                       int32_t* n_iter, uint8_t* branches, int32_t branches_cap, void* workspace,
                       size_t ws_bytes, void* stream) {
  sp2_options o;
  sp2_default_options(&o);
  o.tol = tol;
  sp2_info info;
  const sp2_status s = sp2_density_ex(H, n, n, n_occ, &o, P, &info, branches, branches_cap,
                                      workspace, ws_bytes, stream);
  if (n_iter) *n_iter = (s == SP2_OK || s == SP2_ERR_NOT_CONVERGED) ? info.n_iter : 0;
  return s;
}

sp2_status sp2_bounds(const float* H, int64_t n, int64_t ld, double* eps_min, double* eps_max,
                      void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!H || !eps_min || !eps_max) return fail(SP2_ERR_INVALID_ARG, "NULL argument");
  if (n <= 0 || ld < n) return fail(SP2_ERR_INVALID_ARG, "need n > 0 and ld >= n");
  sp2_options o;
  sp2_default_options(&o);
  Layout L;
  if (!make_layout(n, o, L)) return fail(SP2_ERR_INVALID_ARG, "matrix order out of range");
  // only the header part of the workspace is used
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 || ws_bytes < L.off_slot0)
    return fail(SP2_ERR_WORKSPACE, "workspace missing, misaligned or too small");
  HostMirror* hm;
  if (sp2_status s = host_mirror(&hm)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  WS w;
  bind(w, workspace, L);
  k_drop_tape<<<1, 1, 0, st>>>(w.meta);
  LAUNCH_TRY();
  k_gershgorin_rows<<<L.gersh_blocks, kRowThreads, 0, st>>>(H, n, ld, w.gersh);
  LAUNCH_TRY();
  k_bounds_final<<<1, 256, 0, st>>>(w.gersh, L.gersh_blocks, w.ctrl, 1);
  LAUNCH_TRY();
  if (sp2_status s = read_back(w, hm, false, st)) return s;
  *eps_min = hm->ctrl[0].eps_min;
  *eps_max = hm->ctrl[0].eps_max;
  if (hm->ctrl[0].nonfinite) return fail(SP2_ERR_NONFINITE, "H holds NaN or Inf");
  return SP2_OK;
}

sp2_status sp2_spectral_bounds(const float* H, int64_t n, int64_t ld, int32_t steps,
                               int32_t seed, double* eps_min, double* eps_max, void* workspace,
                               size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!H || !eps_min || !eps_max) return fail(SP2_ERR_INVALID_ARG, "NULL argument");
  if (n <= 0 || ld < n) return fail(SP2_ERR_INVALID_ARG, "need n > 0 and ld >= n");
  if (steps < SP2_MIN_BOUND_STEPS || steps > SP2_MAX_BOUND_STEPS)
    return fail(SP2_ERR_INVALID_ARG, "steps must lie in [%d, %d]", SP2_MIN_BOUND_STEPS,
                SP2_MAX_BOUND_STEPS);
  sp2_options o;
  sp2_default_options(&o);
  o.bound_steps = steps;
  Layout L;
  if (!make_layout(n, o, L)) return fail(SP2_ERR_INVALID_ARG, "matrix order out of range");
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 || ws_bytes < L.off_slot0)
    return fail(SP2_ERR_WORKSPACE, "workspace missing, misaligned or too small");
  HostMirror* hm;
  if (sp2_status s = host_mirror(&hm)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  WS w;
  bind(w, workspace, L);
  k_drop_tape<<<1, 1, 0, st>>>(w.meta);
  LAUNCH_TRY();
  k_gershgorin_rows<<<L.gersh_blocks, kRowThreads, 0, st>>>(H, n, ld, w.gersh);
  LAUNCH_TRY();
  k_bounds_final<<<1, 256, 0, st>>>(w.gersh, L.gersh_blocks, w.ctrl, 1);
  LAUNCH_TRY();
  if (sp2_status s = refine_bounds(w, H, n, ld, steps, seed, st)) return s;
  if (sp2_status s = read_back(w, hm, false, st)) return s;
  *eps_min = hm->ctrl[0].eps_min;
  *eps_max = hm->ctrl[0].eps_max;
  if (hm->ctrl[0].nonfinite) return fail(SP2_ERR_NONFINITE, "H holds NaN or Inf");
  return SP2_OK;
}

sp2_status sp2_homo_lumo(const float* H, const float* P, int64_t n, int64_t ld, int32_t steps,
                         int32_t seed, double margin, double* homo, double* lumo, void* workspace,
                         size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!H || !P || !homo || !lumo) return fail(SP2_ERR_INVALID_ARG, "NULL argument");
  if (n <= 0 || ld < n) return fail(SP2_ERR_INVALID_ARG, "need n > 0 and ld >= n");
  if (steps < SP2_MIN_BOUND_STEPS || steps > SP2_MAX_BOUND_STEPS)
    return fail(SP2_ERR_INVALID_ARG, "steps must lie in [%d, %d]", SP2_MIN_BOUND_STEPS,
                SP2_MAX_BOUND_STEPS);
  if (!(margin >= 0.0 && margin < 0.5)) return fail(SP2_ERR_INVALID_ARG, "margin must lie in [0, 1/2)");
  sp2_options o;
  sp2_default_options(&o);
  Layout L;
  if (!make_layout(n, o, L)) return fail(SP2_ERR_INVALID_ARG, "matrix order out of range");
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 || ws_bytes < L.off_slot0)
    return fail(SP2_ERR_WORKSPACE, "workspace missing, misaligned or too small");
  HostMirror* hm;
  if (sp2_status s = host_mirror(&hm)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  WS w;
  bind(w, workspace, L);
  k_drop_tape<<<1, 1, 0, st>>>(w.meta);
  LAUNCH_TRY();
  k_gershgorin_rows<<<L.gersh_blocks, kRowThreads, 0, st>>>(H, n, ld, w.gersh);
  LAUNCH_TRY();
  k_bounds_final<<<1, 256, 0, st>>>(w.gersh, L.gersh_blocks, w.ctrl, 1);
  LAUNCH_TRY();
  const int nb = L.lz_blocks, nc = L.lz_chunks;
  const int k = static_cast<int>(std::min<int64_t>(steps, n));
  // side 0: occupied (Q = P), side 1: virtual (Q = I - P); both run
  // together: each matrix is read once per step for the two (k_hl_matvec2)
  // and their vector steps share launches (k_hl_*2, side = blockIdx.y)
  LzState* lz[2] = {w.lz, w.lz1};
  double *V[2], *wv[2], *yv[2], *p1[2], *p2[2], *pn[2], *pc[2];
  double* lzv[2] = {w.lzv, w.lzv1};
  double* lzp[2] = {w.lzpart, w.lzpart1};
  for (int sd = 0; sd < 2; ++sd) {
    V[sd] = lzv[sd];
    wv[sd] = lzv[sd] + int64_t(kLzMaxSteps + 1) * n;   // w
    yv[sd] = lzv[sd] + int64_t(kLzMaxSteps + 2) * n;   // (H - shift) v_j
    p1[sd] = lzp[sd];
    p2[sd] = p1[sd] + size_t(nb) * kLzCoef;
    pn[sd] = p2[sd] + size_t(nc) * kLzCoef;
    pc[sd] = pn[sd] + nc;
  }
  const uint64_t seed64 = static_cast<uint64_t>(static_cast<uint32_t>(seed));
  for (int sd = 0; sd < 2; ++sd) {
    k_lz_start<<<1, kLzThreads, 0, st>>>(V[sd], n, seed64, lz[sd]);
    LAUNCH_TRY();
  }
  HlTwo a;
  memset(&a, 0, sizeof(a));
  for (int sd = 0; sd < 2; ++sd) {
    a.st[sd] = lz[sd];
    a.x[sd] = V[sd];
    a.out[sd] = wv[sd];
    a.mode[sd] = sd == 0 ? 1 : 2;   // Q = P, or I - P
  }
  HlVecs vs;
  for (int sd = 0; sd < 2; ++sd) {
    vs.V[sd] = V[sd];
    vs.w[sd] = wv[sd];
    vs.p1[sd] = p1[sd];
    vs.p2[sd] = p2[sd];
    vs.pn[sd] = pn[sd];
    vs.pc[sd] = pc[sd];
    vs.st[sd] = lz[sd];
  }
  k_hl_matvec2<<<nb, kLzMvThreads, 0, st>>>(P, n, ld, a, w.ctrl, 0);
  LAUNCH_TRY();
  k_hl_norm_parts2<<<dim3(nc, 2), kLzChunk, 0, st>>>(vs, n);
  LAUNCH_TRY();
  k_hl_next2<<<dim3(nc, 2), kLzChunk, 0, st>>>(vs, n, 0, nc);
  LAUNCH_TRY();
  for (int j = 0; j < k; ++j) {
    HlTwo sh = a;   // y = (H - shift) v_j
    HlTwo q = a;    // w = Q y with the first Gram-Schmidt partials
    for (int sd = 0; sd < 2; ++sd) {
      sh.x[sd] = V[sd] + int64_t(j) * n;
      sh.out[sd] = yv[sd];
      sh.mode[sd] = 0;
      q.x[sd] = yv[sd];
      q.V[sd] = V[sd];
      q.dot_part[sd] = p1[sd];
    }
    k_hl_matvec2<<<nb, kLzMvThreads, 0, st>>>(H, n, ld, sh, w.ctrl, j);
    LAUNCH_TRY();
    k_hl_matvec2<<<nb, kLzMvThreads, 0, st>>>(P, n, ld, q, w.ctrl, j);
    LAUNCH_TRY();
    k_hl_coef2<<<dim3(j + 1, 2), kLzChunk, 0, st>>>(vs, nb);
    LAUNCH_TRY();
    k_hl_apply2<<<dim3(nc, 2), kLzChunk, 0, st>>>(vs, n, j, nc, 0);
    LAUNCH_TRY();
    k_hl_apply2<<<dim3(nc, 2), kLzChunk, 0, st>>>(vs, n, j, nc, 1);
    LAUNCH_TRY();
    k_hl_next2<<<dim3(nc, 2), kLzChunk, 0, st>>>(vs, n, j + 1, nc);
    LAUNCH_TRY();
  }
  for (int sd = 0; sd < 2; ++sd) {
    k_hl_ritz<<<1, kWave, 0, st>>>(lz[sd], sd);
    LAUNCH_TRY();
  }
  HIP_TRY(hipMemcpyAsync(hm->ritz, w.lz->ritz, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(hm->ritz + 2, w.lz1->ritz + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  if (sp2_status s = read_back(w, hm, false, st)) return s;
  const Ctrl& c = hm->ctrl[0];
  if (c.nonfinite) return fail(SP2_ERR_NONFINITE, "H holds NaN or Inf");
  if (c.degenerate) return fail(SP2_ERR_NOT_CONVERGED, "degenerate spectrum (eps_max == eps_min): no gap");
  const double h_est = hm->ritz[0] + c.eps_min + hm->ritz[1];
  const double l_est = hm->ritz[2] + c.eps_max - hm->ritz[3];
  const double gap = l_est - h_est;
  if (!(gap > 0.0))
    return fail(SP2_ERR_NOT_CONVERGED, "no gap between the estimates (HOMO %.6g, LUMO %.6g)", h_est,
                l_est);
  *homo = h_est + margin * gap;
  *lumo = l_est - margin * gap;
  return SP2_OK;
}

sp2_status sp2_split(const float* X, int64_t n, int64_t ld, int32_t precision, uint16_t* hi,
                     uint16_t* lo, void* stream) {
  g_err.clear();
  if (!X || !hi || !lo) return fail(SP2_ERR_INVALID_ARG, "NULL argument");
  if (n <= 0 || ld < n) return fail(SP2_ERR_INVALID_ARG, "need n > 0 and ld >= n");
  const int code = split_code_of(precision);
  if (!code) return fail(SP2_ERR_INVALID_ARG, "precision has no 16-bit split");
  hipStream_t st = static_cast<hipStream_t>(stream);
  k_split<<<ew_grid(n * n), kEwThreads, 0, st>>>(X, n, ld, n, n, hi, lo, code);
  LAUNCH_TRY();
  return SP2_OK;
}

sp2_status sp2_layer(const float* X, int64_t n, int64_t ld, int32_t precision, int32_t sign,
                     float* Y, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!X || !Y || X == Y) return fail(SP2_ERR_INVALID_ARG, "X and Y must be distinct non-NULL buffers");
  if (n <= 0 || ld < n) return fail(SP2_ERR_INVALID_ARG, "need n > 0 and ld >= n");
  if (sign != 1 && sign != -1) return fail(SP2_ERR_INVALID_ARG, "sign must be +1 or -1");
  sp2_options o;
  sp2_default_options(&o);
  o.precision = precision;
  o.refine = SP2_REFINE_NONE;
  if (!options_ok(o)) return fail(SP2_ERR_INVALID_ARG, "invalid precision");
  Layout L;
  if (!make_layout(n, o, L)) return fail(SP2_ERR_INVALID_ARG, "matrix order out of range");
  if (sp2_status s = check_ws(L, workspace, ws_bytes)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  WS w;
  bind(w, workspace, L);
  k_drop_tape<<<1, 1, 0, st>>>(w.meta);
  LAUNCH_TRY();
  float* Xp = w.slotf(0);
  k_copy_scaled<<<ew_grid(L.np * L.np), kEwThreads, 0, st>>>(X, ld, Xp, L.np, n, L.np, 1.0f, 0);
  LAUNCH_TRY();
  Epi e = make_epi(L);
  e.c = Xp;
  e.out = Y;
  e.ld_out = ld;
  e.n_valid = static_cast<int>(n);
  e.vec_ok = (ld % 4 == 0) && (reinterpret_cast<uintptr_t>(Y) % 16 == 0);
  e.alpha = sign > 0 ? 1.0f : -1.0f;
  e.beta = sign > 0 ? 0.0f : 2.0f;
  const Decide d0 = make_decide(w, 0, 0);
  sp2_status s;
  if (precision == SP2_FP32) {
    const float* A[1] = {Xp};
    s = launch_f32(w, 1, A, A, e, d0, st);
  } else {
    // as in the network: the planes hold X - cI, X^2 = (X - cI)^2 + 2c X - c^2 I
    k_split_tiled<<<L.init_blocks, kEwThreads, 0, st>>>(Xp, L.np, L.np, L.np, w.hi(0), w.lo(0),
                                                        split_code_of(precision), kPlaneCentre, L.n);
    LAUNCH_TRY();
    e.beta += 2.0f * kPlaneCentre * e.alpha;
    e.gamma = -kPlaneCentre * kPlaneCentre * e.alpha;
    e.n_diag = static_cast<int>(n);
    s = launch_split(w, precision, w.hi(0), w.lo(0), w.hi(0), w.lo(0), e, d0, st);
  }
  if (s) return s;
  HIP_TRY(hipStreamSynchronize(st));
  return SP2_OK;
}

sp2_status sp2_history(void* workspace, size_t ws_bytes, int32_t cap, double* t1, double* t2,
                       double* err, double* coef, int32_t* count, void* stream) {
  g_err.clear();
  if (cap < 0 || (cap > 0 && !t1 && !t2 && !err && !coef))
    return fail(SP2_ERR_INVALID_ARG, "bad cap or outputs");
  sp2_options d;
  sp2_default_options(&d);
  Layout L0;
  make_layout(256, d, L0);   // header offsets do not depend on n
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 || ws_bytes < L0.off_meta)
    return fail(SP2_ERR_WORKSPACE, "workspace missing, misaligned or too small");
  HostMirror* hm;
  if (sp2_status s = host_mirror(&hm)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  WS w;
  bind(w, workspace, L0);
  if (sp2_status s = read_back(w, hm, true, st)) return s;
  const int32_t nk = std::min(std::max(hm->ctrl[0].n_iter, 0), kMaxIter) + 1;
  for (int32_t k = 0; k < std::min(nk, cap); ++k) {
    if (t1) t1[k] = hm->hist.t1[k];
    if (t2) t2[k] = hm->hist.t2[k];
    if (err) err[k] = hm->hist.err[k];
  }
  if (coef)
    for (int32_t k = 0; k < std::min(nk - 1, cap); ++k)
      for (int q = 0; q < 3; ++q)
        coef[3 * k + q] = hm->hist.coef[k][q];
  if (count) *count = nk;
  return SP2_OK;
}

}  // extern "C"

namespace {

// Load the tape description, control block and history written by the last
// forward call on this workspace.
sp2_status open_tape(void* workspace, size_t ws_bytes, hipStream_t st, WS& w, HostMirror*& hm,
                     sp2_options& o) {
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(SP2_ERR_WORKSPACE, "workspace missing or misaligned");
  sp2_options d;
  sp2_default_options(&d);
  Layout L0;
  make_layout(256, d, L0);   // header offsets do not depend on n
  if (ws_bytes < L0.off_parts0) return fail(SP2_ERR_WORKSPACE, "workspace too small");
  if (sp2_status s = host_mirror(&hm)) return s;
  HIP_TRY(hipMemcpyAsync(&hm->meta, static_cast<char*>(workspace) + L0.off_meta, sizeof(Meta),
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const Meta m = hm->meta;
  if (m.magic != kMetaMagic || m.valid == 0 || m.every <= 0)
    return fail(SP2_ERR_TAPE, "no derivative tape: run sp2_density_ex with checkpoint_every > 0 first");
  o = d;
  o.precision = m.precision;
  o.refine = m.refine;
  o.checkpoint_every = m.every;
  o.max_iter = m.max_iter;
  o.flags = m.flags;
  Layout L;
  if (!make_layout(m.n, o, L)) return fail(SP2_ERR_TAPE, "corrupt tape description");
  if (sp2_status s = check_ws(L, workspace, ws_bytes)) return s;
  bind(w, workspace, L);
  return read_back(w, hm, true, st);
}

// Symmetric two-operand product  out = alpha (X Y + Y X) + beta C  or the
// branch-coefficient form (mode 2, layer n) of one derivative layer.
sp2_status sym_pair(const WS& w, const float* X, const float* Y, const float* C, float* out,
                    float alpha, float beta, int mode, int layer, hipStream_t st) {
  const float* A[2] = {X, Y};
  const float* B[2] = {Y, X};
  Epi e = make_epi(w.L);
  e.c = C;
  e.out = out;
  e.alpha = alpha;
  e.beta = beta;
  return launch_f32(w, 2, A, B, e, make_decide(w, mode, layer), st);
}

// Split derivatives (SP2_FLAG_SPLIT_DERIVATIVES with BF16X3 layers): the
// BF16X3 planes of a derivative iterate live in work slot 2 + i (hi, then lo).
bool split_derivatives(const sp2_options& o) {
  return (o.flags & SP2_FLAG_SPLIT_DERIVATIVES) && o.precision == SP2_BF16X3;
}
uint16_t* dhi(const WS& w, int i) { return reinterpret_cast<uint16_t*>(w.work(2 + i)); }
uint16_t* dlo(const WS& w, int i) { return dhi(w, i) + w.L.np * w.L.np; }

// Split form of sym_pair: out = alpha (X Y + Y X) + beta C from the planes
// of X and Y (in mode 3 the recorded a, b of layer `layer`), with the
// planes of out written to pair `op` of the derivative planes.
sp2_status sym_pair_split(const WS& w, const uint16_t* xh, const uint16_t* xl, int yp,
                          const float* C, float* out, int op, int mode, int layer,
                          hipStream_t st) {
  Epi e = make_epi(w.L);
  e.c = C;
  e.out = out;
  e.split_out = split_code_of(SP2_BF16X3);
  e.hi_out = dhi(w, op);
  e.lo_out = dlo(w, op);
  // X's planes are centred: (X - cI) Y + Y (X - cI) = X Y + Y X - 2c Y
  e.centring = kCentredPair;
  return launch_split_pair(w, xh, xl, dhi(w, yp), dlo(w, yp), e, make_decide(w, mode, layer), st);
}

// BF16X3 planes of an FP32 derivative iterate (np x np) into pair `op`.
sp2_status split_derivative(const WS& w, const float* X, int op, hipStream_t st) {
  k_split_tiled<<<w.L.init_blocks, kEwThreads, 0, st>>>(X, w.L.np, w.L.np, w.L.np, dhi(w, op),
                                                        dlo(w, op), split_code_of(SP2_BF16X3), 0.0f,
                                                        0);
  LAUNCH_TRY();
  return SP2_OK;
}

// Derivative of the McWeeny step at S in direction D (JVP) or its adjoint
// (identical map): 3(SD + DS) - 2(S^2 D + S D S + D S^2)
//   = 3M - (S M + M S) - (S^2 D + D S^2)  with  M = SD + DS.
sp2_status refine_derivative(const WS& w, const float* S, const float* D, float* out, int64_t ld,
                             int64_t n, bool vec_ok, hipStream_t st) {
  float* M = w.work(2);
  float* S2 = w.work(3);
  sp2_status s;
  if ((s = sym_pair(w, S, D, nullptr, M, 1.0f, 0.0f, 0, 0, st))) return s;
  {
    const float* A[1] = {S};
    Epi e = make_epi(w.L);
    e.out = S2;
    if ((s = launch_f32(w, 1, A, A, e, make_decide(w, 0, 0), st))) return s;
  }
  const float* A[4] = {S, M, S2, D};
  const float* B[4] = {M, S, D, S2};
  Epi e = make_epi(w.L);
  e.c = M;
  e.out = out;
  e.ld_out = ld;
  e.n_valid = static_cast<int>(n);
  e.vec_ok = vec_ok;
  e.alpha = -1.0f;
  e.beta = 3.0f;
  return launch_f32(w, 4, A, B, e, make_decide(w, 0, 0), st);
}

// The same map in BF16X3 products (split derivatives): S given by its
// centred planes (S - cI, c = kPlaneCentre) in forward pair ps and its FP32
// value S32, D by its planes in derivative pair qd and its FP32 copy in
// work(qd) (overwritten).  Four products: M = SD + DS = [(S - cI) D +
// D (S - cI)] + 2c D (planes in derivative pair 1 - qd), S^2 = (S - cI)^2 +
// 2c S - c^2 I (plain planes in forward pair 1 - ps), T = (3 - 2c) M -
// (S^2 D + D S^2) into work(qd), out = T - [(S - cI) M + M (S - cI)]
// (= 3M - (SM + MS) - (S^2 D + D S^2)).
sp2_status refine_derivative_split(const WS& w, int ps, int qd, const float* S32, float* out,
                                   int64_t ld, int64_t n, bool vec_ok, hipStream_t st) {
  constexpr float c = kPlaneCentre;
  const int bf = split_code_of(SP2_BF16X3);
  const Decide d0 = make_decide(w, 0, 0);
  float* M = w.work(1 - qd);
  float* T = w.work(qd);
  sp2_status s;
  {
    Epi e = make_epi(w.L);
    e.c = w.work(qd);
    e.beta = 2.0f * c;
    e.out = M;
    e.split_out = bf;
    e.hi_out = dhi(w, 1 - qd);
    e.lo_out = dlo(w, 1 - qd);
    if ((s = launch_split_pair(w, w.hi(ps), w.lo(ps), dhi(w, qd), dlo(w, qd), e, d0, st))) return s;
  }
  {
    Epi e = make_epi(w.L);
    e.c = S32;
    e.beta = 2.0f * c;
    e.gamma = -c * c;
    e.n_diag = static_cast<int>(w.L.n);
    e.out = w.slotf(3);
    e.split_out = bf;
    e.hi_out = w.hi(1 - ps);
    e.lo_out = w.lo(1 - ps);
    if ((s = launch_split(w, SP2_BF16X3, w.hi(ps), w.lo(ps), w.hi(ps), w.lo(ps), e, d0, st))) return s;
  }
  {
    Epi e = make_epi(w.L);
    e.c = M;
    e.out = T;
    e.alpha = -1.0f;
    e.beta = 3.0f - 2.0f * c;
    if ((s = launch_split_pair(w, w.hi(1 - ps), w.lo(1 - ps), dhi(w, qd), dlo(w, qd), e, d0, st)))
      return s;
  }
  Epi e = make_epi(w.L);
  e.c = T;
  e.out = out;
  e.ld_out = ld;
  e.n_valid = static_cast<int>(n);
  e.vec_ok = vec_ok;
  e.alpha = -1.0f;
  e.beta = 1.0f;
  return launch_split_pair(w, w.hi(ps), w.lo(ps), dhi(w, 1 - qd), dlo(w, 1 - qd), e, d0, st);
}

// Bring checkpoint `slot` into the forward buffers as iterate S_c (FP32 at
// dst, the centred hi/lo planes of S_c - I/2 in pair 0 for the split
// precisions).
sp2_status load_checkpoint(const WS& w, int prec, int slot, float* dst, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(dst, w.tape(slot), w.L.slot_bytes, hipMemcpyDeviceToDevice, st));
  if (prec != SP2_FP32) {
    k_split_tiled<<<w.L.init_blocks, kEwThreads, 0, st>>>(dst, w.L.np, w.L.np, w.L.np, w.hi(0),
                                                          w.lo(0), split_code_of(prec), kPlaneCentre,
                                                          w.L.n);
    LAUNCH_TRY();
  }
  return SP2_OK;
}

// Forward derivative P1 = dP/dH [H1] of the taped network (open tape).
sp2_status jvp_run(const WS& w, const HostMirror* hm, const sp2_options& o, const float* H1,
                   int64_t ld, float* P1, hipStream_t st) {
  const Layout& L = w.L;
  const int64_t n = L.n;
  const bool vec_ok = (ld % 4 == 0) && (reinterpret_cast<uintptr_t>(P1) % 16 == 0);
  if (hm->meta.valid == 2) {   // n_occ in {0, n}: P does not depend on H
    k_fill_diag<<<ew_grid(n * n), kEwThreads, 0, st>>>(P1, n, ld, 0.0f);
    LAUNCH_TRY();
    HIP_TRY(hipStreamSynchronize(st));
    return SP2_OK;
  }
  const int prec = o.precision;
  const int nl = hm->meta.n_iter;
  const float inv = static_cast<float>(hm->meta.inv_range);
  // dS_0 = -H1 / (eps_max - eps_min)  (H1 symmetrised)
  k_copy_scaled<<<ew_grid(L.np * L.np), kEwThreads, 0, st>>>(H1, ld, w.work(0), L.np, n, L.np, -inv, 1);
  LAUNCH_TRY();
  sp2_status s;
  const bool sd = split_derivatives(o);
  if (sd && (s = split_derivative(w, w.work(0), 0, st))) return s;
  if ((s = load_checkpoint(w, prec, 0, s_f32(w, prec, 0), st))) return s;
  for (int k = 0; k < nl; ++k) {
    const float* S = s_f32(w, prec, k);
    if (sd)
      s = sym_pair_split(w, w.hi(k & 1), w.lo(k & 1), k & 1, w.work(k & 1), w.work((k + 1) & 1),
                         (k + 1) & 1, 3, k, st);
    else
      s = sym_pair(w, S, w.work(k & 1), w.work(k & 1), w.work((k + 1) & 1), 1.0f, 0.0f, 3, k, st);
    if (s) return s;
    if (k + 1 < nl || o.refine != SP2_REFINE_NONE)
      if ((s = launch_layer(w, prec, k, 2, S, s_f32(w, prec, k + 1), k & 1, (k + 1) & 1, nullptr, st,
                            &o, 0)))
        return s;
  }
  const float* Y = w.work(nl & 1);
  if (o.refine != SP2_REFINE_NONE) {
    // S_nl's planes are in forward pair nl & 1, Y's in derivative pair nl & 1
    if (sd)
      s = refine_derivative_split(w, nl & 1, nl & 1, s_f32(w, prec, nl), P1, ld, n, vec_ok, st);
    else
      s = refine_derivative(w, s_f32(w, prec, nl), Y, P1, ld, n, vec_ok, st);
    if (s) return s;
  } else {
    k_copy_scaled<<<ew_grid(n * n), kEwThreads, 0, st>>>(Y, L.np, P1, ld, n, n, 1.0f, 0);
    LAUNCH_TRY();
  }
  HIP_TRY(hipStreamSynchronize(st));
  return SP2_OK;
}

}  // namespace

extern "C" {

sp2_status sp2_jvp(void* workspace, size_t ws_bytes, const float* H1, int64_t ld, float* P1,
                   void* stream) {
  g_err.clear();
  if (!H1 || !P1) return fail(SP2_ERR_INVALID_ARG, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  WS w;
  HostMirror* hm;
  sp2_options o;
  if (sp2_status s = open_tape(workspace, ws_bytes, st, w, hm, o)) return s;
  if (ld < w.L.n) return fail(SP2_ERR_INVALID_ARG, "ld < n");
  return jvp_run(w, hm, o, H1, ld, P1, st);
}

sp2_status sp2_vjp(void* workspace, size_t ws_bytes, const float* W, int64_t ld, float* G,
                   void* stream) {
  g_err.clear();
  if (!W || !G) return fail(SP2_ERR_INVALID_ARG, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  WS w;
  HostMirror* hm;
  sp2_options o;
  if (sp2_status s = open_tape(workspace, ws_bytes, st, w, hm, o)) return s;
  const Layout& L = w.L;
  const int64_t n = L.n;
  if (ld < n) return fail(SP2_ERR_INVALID_ARG, "ld < n");
  if (hm->meta.valid == 2) {
    k_fill_diag<<<ew_grid(n * n), kEwThreads, 0, st>>>(G, n, ld, 0.0f);
    LAUNCH_TRY();
    HIP_TRY(hipStreamSynchronize(st));
    return SP2_OK;
  }
  const int prec = o.precision;
  const int nl = hm->meta.n_iter;
  const int k = L.every;
  const float inv = static_cast<float>(hm->meta.inv_range);
  sp2_status s;
  // G_L = sym(W)
  k_copy_scaled<<<ew_grid(L.np * L.np), kEwThreads, 0, st>>>(W, ld, w.work(0), L.np, n, L.np, 1.0f, 1);
  LAUNCH_TRY();
  int cur = 0;
  const bool sd = split_derivatives(o);
  if (o.refine != SP2_REFINE_NONE) {
    // recompute S_L from its last checkpoint, then apply the refinement adjoint
    const int c = (nl / k) * k;
    if ((s = load_checkpoint(w, prec, c / k, s_f32(w, prec, c), st))) return s;
    for (int m = c; m < nl; ++m)
      if ((s = launch_layer(w, prec, m, 2, s_f32(w, prec, m), s_f32(w, prec, m + 1), (m - c) & 1,
                            (m - c + 1) & 1, nullptr, st, &o, 0)))
        return s;
    if (sd) {
      // S_L's planes are in forward pair (nl - c) & 1; G's go to derivative pair 0
      if ((s = split_derivative(w, w.work(0), 0, st))) return s;
      s = refine_derivative_split(w, (nl - c) & 1, 0, s_f32(w, prec, nl), w.work(1), L.np, L.np,
                                  true, st);
    } else {
      s = refine_derivative(w, s_f32(w, prec, nl), w.work(0), w.work(1), L.np, L.np, true, st);
    }
    if (s) return s;
    cur = 1;
  }
  if (sd && (s = split_derivative(w, w.work(cur), cur, st))) return s;
  const int nseg = (nl + k - 1) / k;
  for (int j = nseg - 1; j >= 0; --j) {
    const int c = j * k, e = std::min(c + k, nl);
    if ((s = load_checkpoint(w, prec, j, w.seg(0), st))) return s;
    for (int m = 1; m < e - c; ++m)
      if ((s = launch_layer(w, prec, c + m - 1, 2, w.seg(m - 1), w.seg(m), (m - 1) & 1, m & 1, nullptr,
                            st, &o, 0)))
        return s;
    for (int nn = e - 1; nn >= c; --nn) {
      if (sd) {
        // centred planes of S_nn into pair 0 (the recomputation has moved on)
        k_split_tiled<<<L.init_blocks, kEwThreads, 0, st>>>(w.seg(nn - c), L.np, L.np, L.np, w.hi(0),
                                                            w.lo(0), split_code_of(SP2_BF16X3),
                                                            kPlaneCentre, L.n);
        LAUNCH_TRY();
        s = sym_pair_split(w, w.hi(0), w.lo(0), cur, w.work(cur), w.work(1 - cur), 1 - cur, 3, nn,
                           st);
      } else {
        s = sym_pair(w, w.seg(nn - c), w.work(cur), w.work(cur), w.work(1 - cur), 1.0f, 0.0f, 3, nn,
                     st);
      }
      if (s) return s;
      cur = 1 - cur;
    }
  }
  // dTr(WP)/dH = -G_0 / (eps_max - eps_min)
  k_copy_scaled<<<ew_grid(n * n), kEwThreads, 0, st>>>(w.work(cur), L.np, G, ld, n, n, -inv, 0);
  LAUNCH_TRY();
  HIP_TRY(hipStreamSynchronize(st));
  return SP2_OK;
}

}  // extern "C"

namespace {

// Scratch of the XL-BOMD building block (offsets from a 256-aligned base):
// H1 and P1 (n x n FP32, leading dimension n), the basis V and the response
// QR factor Q (rank rows of n_atoms doubles each), five charge vectors and
// the Krylov state.
struct XlScratch {
  float* h1;
  float* p1;
  double *V, *Q, *r0, *res, *u, *jv, *fk;
  XlState* st;
  size_t total;
};

size_t xl_layout(int64_t n, int64_t na, int rank, char* base, XlScratch* x) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o2 = off;
    off = round_up(off + bytes, 256);
    return base ? base + o2 : nullptr;
  };
  const size_t mat = size_t(n) * size_t(n) * 4, vec = size_t(na) * 8;
  char* h1 = take(mat);
  char* p1 = take(mat);
  char* V = take(vec * size_t(rank));
  char* Q = take(vec * size_t(rank));
  char* r0 = take(vec);
  char* res = take(vec);
  char* u = take(vec);
  char* jv = take(vec);
  char* fk = take(vec);
  char* st = take(sizeof(XlState));
  if (x) {
    x->h1 = reinterpret_cast<float*>(h1);
    x->p1 = reinterpret_cast<float*>(p1);
    x->V = reinterpret_cast<double*>(V);
    x->Q = reinterpret_cast<double*>(Q);
    x->r0 = reinterpret_cast<double*>(r0);
    x->res = reinterpret_cast<double*>(res);
    x->u = reinterpret_cast<double*>(u);
    x->jv = reinterpret_cast<double*>(jv);
    x->fk = reinterpret_cast<double*>(fk);
    x->st = reinterpret_cast<XlState*>(st);
    x->total = off;
  }
  return off;
}

int atom_grid(int64_t na) { return static_cast<int>((na + 255) / 256); }

// Common argument checks and set-up of sp2_xl_response / sp2_xl_kernel:
// open the tape, bind the scratch and clear H1.
sp2_status xl_open(void* workspace, size_t ws_bytes, int64_t na, const int64_t* atom_ptr,
                   const double* gamma, int rank, void* scratch, size_t scratch_bytes,
                   hipStream_t st, WS& w, HostMirror*& hm, sp2_options& o, XlScratch& x) {
  if (!atom_ptr || !gamma) return fail(SP2_ERR_INVALID_ARG, "NULL atom_ptr or gamma");
  if (na <= 0 || na > (int64_t(1) << 24)) return fail(SP2_ERR_INVALID_ARG, "n_atoms out of range");
  if (!scratch || reinterpret_cast<uintptr_t>(scratch) % 256)
    return fail(SP2_ERR_INVALID_ARG, "scratch missing or not 256-byte aligned");
  if (sp2_status s = open_tape(workspace, ws_bytes, st, w, hm, o)) return s;
  const int64_t n = w.L.n;
  if (scratch_bytes < xl_layout(n, na, rank, nullptr, nullptr))
    return fail(SP2_ERR_INVALID_ARG, "scratch smaller than sp2_xl_scratch_bytes");
  xl_layout(n, na, rank, static_cast<char*>(scratch), &x);
  k_fill_diag<<<ew_grid(n * n), kEwThreads, 0, st>>>(x.h1, n, n, 0.0f);
  LAUNCH_TRY();
  return SP2_OK;
}

// jv = J v = dq0/dn v - v: u = gamma v, H1 = diag(B u), P1 = JVP(H1),
// jv_I = -2 sum_{mu in I} P1_mu,mu - v_I.  Blocks (the JVP does).
sp2_status xl_apply_j(const WS& w, const HostMirror* hm, const sp2_options& o, const XlScratch& x,
                      int64_t na, const int64_t* atom_ptr, const double* gamma, const double* v,
                      double* jv, hipStream_t st) {
  const int64_t n = w.L.n;
  k_atom_matvec<<<static_cast<int>((na + 3) / 4), 256, 0, st>>>(gamma, v, na, 1.0, x.u);
  LAUNCH_TRY();
  k_potential_diag<<<atom_grid(na), 256, 0, st>>>(x.u, atom_ptr, na, n, x.h1, n);
  LAUNCH_TRY();
  if (sp2_status s = jvp_run(w, hm, o, x.h1, n, x.p1, st)) return s;
  k_mulliken<<<atom_grid(na), 256, 0, st>>>(x.p1, n, n, na, atom_ptr, nullptr, v, jv);
  LAUNCH_TRY();
  return SP2_OK;
}

}  // namespace

extern "C" {

sp2_status sp2_mulliken(const float* P, int64_t n, int64_t ld, int64_t n_atoms,
                        const int64_t* atom_ptr, const double* z, const double* sub, double* q,
                        void* stream) {
  g_err.clear();
  if (!P || !atom_ptr || !z || !q) return fail(SP2_ERR_INVALID_ARG, "NULL argument");
  if (n <= 0 || ld < n) return fail(SP2_ERR_INVALID_ARG, "need n > 0 and ld >= n");
  if (n_atoms <= 0 || n_atoms > (int64_t(1) << 24))
    return fail(SP2_ERR_INVALID_ARG, "n_atoms out of range");
  hipStream_t st = static_cast<hipStream_t>(stream);
  k_mulliken<<<atom_grid(n_atoms), 256, 0, st>>>(P, n, ld, n_atoms, atom_ptr, z, sub, q);
  LAUNCH_TRY();
  return SP2_OK;
}

size_t sp2_xl_scratch_bytes(int64_t n, int64_t n_atoms, int32_t rank) {
  if (n <= 0 || n_atoms <= 0 || rank < 1 || rank > SP2_XL_MAX_RANK) return 0;
  return xl_layout(n, n_atoms, rank, nullptr, nullptr);
}

sp2_status sp2_xl_response(void* workspace, size_t ws_bytes, int64_t n_atoms,
                           const int64_t* atom_ptr, const double* gamma, const double* v,
                           double* jv, void* scratch, size_t scratch_bytes, void* stream) {
  g_err.clear();
  if (!v || !jv) return fail(SP2_ERR_INVALID_ARG, "NULL v or jv");
  hipStream_t st = static_cast<hipStream_t>(stream);
  WS w;
  HostMirror* hm;
  sp2_options o;
  XlScratch x;
  if (sp2_status s = xl_open(workspace, ws_bytes, n_atoms, atom_ptr, gamma, 1, scratch,
                             scratch_bytes, st, w, hm, o, x))
    return s;
  if (sp2_status s = xl_apply_j(w, hm, o, x, n_atoms, atom_ptr, gamma, v, jv, st)) return s;
  HIP_TRY(hipStreamSynchronize(st));
  return SP2_OK;
}

sp2_status sp2_xl_kernel(void* workspace, size_t ws_bytes, int64_t n_atoms,
                         const int64_t* atom_ptr, const double* gamma, const double* k0,
                         const double* f, int32_t rank, double* kf, double* rho,
                         int32_t* rank_used, void* scratch, size_t scratch_bytes, void* stream) {
  g_err.clear();
  if (!f || !kf) return fail(SP2_ERR_INVALID_ARG, "NULL f or kf");
  if (rank < 1 || rank > SP2_XL_MAX_RANK) return fail(SP2_ERR_INVALID_ARG, "rank out of range");
  hipStream_t st = static_cast<hipStream_t>(stream);
  WS w;
  HostMirror* hm;
  sp2_options o;
  XlScratch x;
  if (sp2_status s = xl_open(workspace, ws_bytes, n_atoms, atom_ptr, gamma, rank, scratch,
                             scratch_bytes, st, w, hm, o, x))
    return s;
  const int64_t na = n_atoms;
  const int mv_grid = static_cast<int>((na + 3) / 4);
  // r0 = K0 f
  if (k0)
    k_atom_matvec<<<mv_grid, 256, 0, st>>>(k0, f, na, 1.0, x.r0);
  else
    k_atom_scale<<<atom_grid(na), 256, 0, st>>>(f, na, -1.0, x.r0);
  LAUNCH_TRY();
  k_xl_init<<<1, kXlThreads, 0, st>>>(x.r0, na, x.V, x.res, x.st);
  LAUNCH_TRY();
  for (int k = 0; k < rank; ++k) {
    HIP_TRY(hipMemcpyAsync(&hm->xl_stop, &x.st->stop, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hm->xl_stop) break;
    const double* vk = x.V + int64_t(k) * na;
    if (sp2_status s = xl_apply_j(w, hm, o, x, na, atom_ptr, gamma, vk, x.jv, st)) return s;
    if (k0)
      k_atom_matvec<<<mv_grid, 256, 0, st>>>(k0, x.jv, na, 1.0, x.fk);
    else
      k_atom_scale<<<atom_grid(na), 256, 0, st>>>(x.jv, na, -1.0, x.fk);
    LAUNCH_TRY();
    k_xl_step<<<1, kXlThreads, 0, st>>>(x.fk, k, k + 1 == rank, na, x.V, x.Q, x.res, x.u, x.st);
    LAUNCH_TRY();
  }
  k_xl_finish<<<1, kXlThreads, 0, st>>>(x.V, na, x.st, kf);
  LAUNCH_TRY();
  HIP_TRY(hipMemcpyAsync(&hm->xl, x.st, sizeof(XlState), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (rho)
    for (int k = 0; k <= rank; ++k) rho[k] = hm->xl.rho[k];
  if (rank_used) *rank_used = hm->xl.used;
  return SP2_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Canonical integration (Section IV, Eq. 31-33)
// ---------------------------------------------------------------------------
namespace {

bool finite_nonneg(double x) { return x >= 0.0 && x <= 1.7976931348623157e308; }

sp2_status nvt_check(const sp2_nvt_params* p, int64_t n) {
  if (!p) return fail(SP2_ERR_INVALID_ARG, "NULL params");
  if (p->scheme != 0 && p->scheme != 1) return fail(SP2_ERR_INVALID_ARG, "scheme must be 0 or 1");
  if (!(finite_nonneg(p->dt) && p->dt > 0.0) || !finite_nonneg(p->kt) ||
      !finite_nonneg(p->gamma_tc) || !finite_nonneg(p->gamma_l))
    return fail(SP2_ERR_INVALID_ARG, "need dt > 0 and kt, gamma_tc, gamma_l >= 0, all finite");
  if (n < 0) return fail(SP2_ERR_INVALID_ARG, "n < 0");
  return SP2_OK;
}

// One coordinate per thread (all loads of a thread issued at once); the
// kernels' grid-stride loop only runs past the first pass beyond 2^31 - 1
// work-groups.
int nvt_grid(int64_t n) {
  return static_cast<int>(std::min<int64_t>(0x7fffffff, (n + kNvtThreads - 1) / kNvtThreads));
}

}  // namespace

extern "C" {

double sp2_nvt_gamma_tc(double sigma_tc, double kt, double dt) {
#pragma clang fp contract(off)
  if (!(finite_nonneg(sigma_tc) && finite_nonneg(kt) && kt > 0.0 && finite_nonneg(dt) && dt > 0.0))
    return __builtin_nan("");
  return sigma_tc * sigma_tc * dt / (2.0 * kt);
}

sp2_status sp2_nvt_first_half(double* R, double* V, const double* F, const double* eta,
                              const double* mass, int64_t n, const sp2_nvt_params* p,
                              void* stream) {
#pragma clang fp contract(off)
  g_err.clear();
  if (sp2_status s = nvt_check(p, n)) return s;
  if (n == 0) return SP2_OK;
  if (!R || !V || !F || !mass) return fail(SP2_ERR_INVALID_ARG, "NULL R, V, F or mass");
  if (p->gamma_l > 0.0 && !eta) return fail(SP2_ERR_INVALID_ARG, "gamma_l > 0 needs eta");
  const double c_l = (1.0 - 0.5 * p->gamma_l * p->dt) / (1.0 + 0.5 * p->gamma_l * p->dt);
  k_nvt_first<<<nvt_grid(n), kNvtThreads, 0, static_cast<hipStream_t>(stream)>>>(
      R, V, F, p->gamma_l > 0.0 ? eta : nullptr, mass, n, p->dt, p->kt, p->gamma_tc, c_l,
      p->scheme);
  LAUNCH_TRY();
  return SP2_OK;
}

sp2_status sp2_nvt_second_half(double* V, const double* F, const double* mass, int64_t n,
                               const sp2_nvt_params* p, void* stream) {
  g_err.clear();
  if (sp2_status s = nvt_check(p, n)) return s;
  if (n == 0) return SP2_OK;
  if (!V || !F || !mass) return fail(SP2_ERR_INVALID_ARG, "NULL V, F or mass");
  k_nvt_second<<<nvt_grid(n), kNvtThreads, 0, static_cast<hipStream_t>(stream)>>>(
      V, F, mass, n, p->dt, p->gamma_tc, p->scheme);
  LAUNCH_TRY();
  return SP2_OK;
}

}  // extern "C"
