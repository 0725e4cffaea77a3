/*
 * sp2.h -- C ABI of the MI355X (gfx950) density-matrix solver.
 *
 * Computes the zero-temperature density matrix D = theta(mu I - H) of a
 * symmetric Hamiltonian H in an orthogonal basis (Section II.C, Eq. 18 of
 * Finkelstein et al., arXiv 2107.02737) with the recursive second-order
 * spectral projection written as a deep network, DNN-SP2 (Section II.D,
 * Eq. 19 and Fig. 1): S_0 maps the spectrum of H linearly onto [0, 1] in
 * reverse order, and each layer is S_n = S_{n-1}^2 or 2 S_{n-1} - S_{n-1}^2.
 * The matrix squares run on MFMA matrix cores, optionally in the dual 16-bit
 * representation X = X0 + X1 of Eq. (20)-(22).  Around the solver: its
 * forward derivative and adjoint (sp2_jvp, sp2_vjp), the charge-space pieces
 * of the XL-BOMD kernel K f (Section III, sp2_mulliken, sp2_xl_*) and one
 * step of the canonical integration scheme that treats force noise as a
 * heat bath (Section IV, sp2_nvt_*).
 *
 * Conventions shared by every entry point:
 *   - Matrix pointers are DEVICE pointers (HIP device memory) owned by the
 *     caller.  Matrices are square, FP32, row-major with leading dimension
 *     `ld` (elements, ld >= n).  Because every matrix here is symmetric,
 *     row- and column-major agree.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     All device work is ordered on it.
 *   - `workspace` is caller-owned device memory of at least
 *     sp2_workspace_bytes(n, opt) bytes, 256-byte aligned.  The library
 *     never allocates device matrix memory; it only allocates a few KB of
 *     pinned host memory once per thread for status read-back.
 *   - Functions never throw; they return an sp2_status.  On failure
 *     sp2_last_error() gives a thread-local description.
 *   - Calls that share a workspace must not overlap in time.
 */
#ifndef SP2_H
#define SP2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SP2_OK = 0,
  SP2_ERR_INVALID_ARG = 1,   /* bad size, pointer, option or n_occ outside [0, n] */
  SP2_ERR_NONFINITE = 2,     /* H holds NaN or Inf (found by the bound pass) */
  SP2_ERR_NOT_CONVERGED = 3, /* stop test not met within max_iter layers, or H = cI
                                with 0 < n_occ < n (no gap); P holds the last iterate */
  SP2_ERR_WORKSPACE = 4,     /* workspace missing, too small or misaligned */
  SP2_ERR_DEVICE = 5,        /* a HIP runtime call failed */
  SP2_ERR_TAPE = 6           /* derivative requested but the workspace holds no tape */
} sp2_status;

/* Arithmetic of the layer products S^2 (Section II.D, Eq. 20-22).  All modes
 * accumulate in FP32; traces, bounds and branch decisions are FP64.
 *   SP2_FP32   one FP32 MFMA product per layer.
 *   SP2_BF16X1 one bfloat16 product (X0 X0 only; single pass).
 *   SP2_BF16X3 X0 X0 + X0 X1 + X1 X0 with X0 = BF16[X], X1 = BF16[X - X0].
 *   SP2_FP16X3 the same with IEEE half on 2^14 X (exact power-of-two scale
 *              that keeps the residual X1 out of the half subnormal range).
 * In the three split modes X is the centred iterate S - I/2 (FP32), and
 * each layer restores S^2 = X^2 + S - I/4 in FP32: a S^2 + b S + c I is
 * formed as a X^2 + (a + b) S + (c - a/4) I.  The centred matrix has far
 * smaller entries than S near a projector, which shrinks both the FP32
 * accumulation and the 16-bit rounding errors. */
typedef enum { SP2_FP32 = 0, SP2_BF16X1 = 1, SP2_BF16X3 = 2, SP2_FP16X3 = 3 } sp2_precision;

/* Refinement after the last layer: the McWeeny purification 3 S^2 - 2 S^3
 * (the refinement step that closes Section II.D).
 *   SP2_REFINE_NONE  no refinement.
 *   SP2_REFINE_FP32  both products in FP32 MFMA.
 *   SP2_REFINE_SPLIT both products in the FP16X3 split representation:
 *                    Q = S^2 from the centred S - I/2, then
 *                    P = -2 (S - I/2) Q + 2Q. */
typedef enum { SP2_REFINE_NONE = 0, SP2_REFINE_FP32 = 1, SP2_REFINE_SPLIT = 2 } sp2_refine;

#define SP2_MAX_ITER 256
#define SP2_MIN_BOUND_STEPS 8
#define SP2_MAX_BOUND_STEPS 64
#define SP2_FLAG_TIME_LAYERS 1
#define SP2_FLAG_SPLIT_DERIVATIVES 2
#define SP2_FLAG_ACCELERATE 4

typedef struct {
  int32_t precision;        /* sp2_precision (default SP2_BF16X3) */
  int32_t refine;           /* sp2_refine (default SP2_REFINE_FP32) */
  int32_t max_iter;         /* layer cap, 1..SP2_MAX_ITER (default 100) */
  int32_t stop_rule;        /* 0: stop when e_n < tol; 1 (default): also stop when
                               e_n < stall_gate and e_n >= min(e_{n-2}, 16 e_{n-2}^2): two
                               more layers no longer reduced e_n as exact arithmetic would
                               (there e_n <= (64/9) e_{n-2}^2 below the gate), so rounding
                               dominates.  Either rule stops only while
                               |Tr S_n - n_occ| < 1/2 */
  int32_t checkpoint_every; /* 0 (default): no tape.  k > 0: keep S_0 and every k-th
                               iterate in the workspace for sp2_jvp / sp2_vjp */
  int32_t flags;            /* bit SP2_FLAG_TIME_LAYERS: time every layer launch with HIP
                               events on `stream` (fills sp2_info.layer_ms/refine_ms).
                               bit SP2_FLAG_SPLIT_DERIVATIVES (precision SP2_BF16X3 with a
                               tape): sp2_jvp / sp2_vjp run the per-layer derivative
                               products S dS + dS S in the same BF16X3 split arithmetic as
                               the layers (one two-segment product [S|dS][dS|S]^T per layer)
                               instead of FP32, and the refinement's derivative
                               3M - (SM + MS) - (S^2 dS + dS S^2), M = S dS + dS S, in four
                               BF16X3 products */
  int32_t bound_steps;      /* 0 (default): Gershgorin bounds.  k in SP2_MIN_BOUND_STEPS..
                               SP2_MAX_BOUND_STEPS: tighten them with k Lanczos steps (see
                               sp2_spectral_bounds) */
  int32_t bound_seed;       /* SplitMix64 state of the Lanczos start vector (default 0) */
  double tol;               /* stop when e_n = |Tr S_n - ||S_n||_F^2| < tol (default 1e-5) */
  double stall_gate;        /* gate of the stagnation test; < 0 (default -1): automatic,
                               max(3/16, n u / 16) with u the unit roundoff of the layer
                               operands (2^-8 BF16X1, 2^-16 BF16X3, 2^-22 FP16X3, 2^-24
                               FP32).  Below 3/16 every eigenvalue of S_n is within 1/4 of
                               0 or 1; n u / 16 stays above the rounding floor of e_n.
                               NaN is rejected */
  double homo, lumo;        /* with SP2_FLAG_ACCELERATE: estimates of the highest occupied
                               and the lowest unoccupied eigenvalue of H (energies, finite,
                               homo < lumo; default 0).  Section II.E: such estimates allow an
                               accelerated network with fewer layers.  With the bounds mapped
                               to l = (eps_max - lumo)/(eps_max - eps_min) (top of the
                               virtual eigenvalues) and h = (eps_max - homo)/(eps_max -
                               eps_min) (bottom of the occupied ones), clipped to [0, 1], the
                               first layers follow a schedule fixed by (l, h): while
                               max(l, 1 - h) >= 1e-14 the wider interval is folded about
                               0.4 of its width, S <- ((S - sI)/(1 - s))^2 with s = 0.4 l when
                               l >= 1 - h, else S <- I - ((I - S - sI)/(1 - s))^2 with
                               s = 0.4 (1 - h), the ends following the same maps; later layers
                               take the trace-driven sign.  Inside the schedule the stagnation
                               test of stop_rule 1 waits until the tracked width is below
                               1e-4 (the schedule itself can raise e_n before that).  Estimates must bracket part of the
                               true gap (homo >= HOMO, lumo <= LUMO).  At the end of the
                               schedule every eigenvalue has reached its side, so
                               |Tr S - n_occ| >= 1/2 there means the estimates were wrong: the
                               scheduled iterate is dropped and the plain network runs from
                               the start (sp2_info.fallback = 1; the schedule's layers are
                               lost time).  sp2_homo_lumo computes estimates from a P */
} sp2_options;

typedef struct {
  int32_t n_iter;      /* layers applied (refinement not counted) */
  int32_t converged;   /* 1 if the stop test passed */
  int32_t status;      /* sp2_status of the call */
  int32_t fallback;    /* 1: SP2_FLAG_ACCELERATE was set but the trace check at the end of
                          the schedule failed (the estimates do not bracket the HOMO-LUMO
                          gap), so the plain network was run instead and produced P */
  double eps_min;      /* lower spectral bound used by the input layer, FP64 */
  double eps_max;      /* upper spectral bound */
  double trace;        /* Tr P of the returned P, FP64 sum of FP32 entries */
  double idem_err;     /* |Tr P - ||P||_F^2| of the returned P */
  double layer_ms;     /* with SP2_FLAG_TIME_LAYERS: summed event time of the n_iter applied
                          layer launches (each from the previous launch's end to its own end) */
  double refine_ms;    /* with SP2_FLAG_TIME_LAYERS: event time of the refinement */
} sp2_info;

/* Fills *opt with the defaults listed above. */
void sp2_default_options(sp2_options* opt);

/* Bytes of device workspace needed by sp2_density / sp2_density_ex /
 * sp2_layer / sp2_jvp / sp2_vjp for matrices of order n with options opt
 * (NULL = defaults).  Includes the derivative tape when
 * opt->checkpoint_every > 0.  Returns 0 for invalid arguments. */
size_t sp2_workspace_bytes(int64_t n, const sp2_options* opt);

/* Density matrix P = theta(mu I - H) with the n_occ lowest states occupied
 * (Eq. 17-19), default options and tolerance tol.  H and P: n x n, ld = n.
 * On return (the call blocks until the solve is done):
 *   *n_iter   layers applied;
 *   branches  min(n_iter, branches_cap) bytes: 1 for S^2 (W_n = +I),
 *             0 for 2S - S^2 (W_n = -I); may be NULL when branches_cap = 0.
 * Special cases: n_occ = 0 gives P = 0 and n_occ = n gives P = I, with no
 * layers.  Returns SP2_OK, or an error as listed in sp2_status. */
sp2_status sp2_density(const float* H, int64_t n, int64_t n_occ, double tol, float* P,
                       int32_t* n_iter, uint8_t* branches, int32_t branches_cap,
                       void* workspace, size_t ws_bytes, void* stream);

/* Full form of sp2_density: leading dimension ld for H and P, explicit
 * options (NULL = defaults; opt->tol is used), and an info record (may be
 * NULL).  With opt->checkpoint_every > 0 the workspace keeps the tape used
 * by sp2_jvp / sp2_vjp (and the spectral bounds of the recorded network)
 * until the next call on the same workspace.  The tape is kept only for a
 * converged solve: after SP2_ERR_NOT_CONVERGED the derivative entry points
 * return SP2_ERR_TAPE.  sp2_bounds, sp2_spectral_bounds and sp2_layer on the
 * same workspace drop it as well. */
sp2_status sp2_density_ex(const float* H, int64_t n, int64_t ld, int64_t n_occ,
                          const sp2_options* opt, float* P, sp2_info* info,
                          uint8_t* branches, int32_t branches_cap,
                          void* workspace, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of sp2_density_ex without a caller workspace.  The library keeps its
 * workspace in a static device array of SP2_NOALLOC_SCRATCH_BYTES (136 MiB),
 * one copy per device, held until the process ends; this call runs no
 * allocating routine (no hipMalloc/hipFree, no pinned host memory, no event
 * creation) and reads its status back through plain host memory,
 * synchronising the stream once per chunk of layers.  Arguments, layout and results are those of
 * sp2_density_ex; the caller still owns H and P.
 * Limits: no derivative tape (opt->checkpoint_every must be 0) and no layer
 * timing (SP2_FLAG_TIME_LAYERS must be clear); n must satisfy
 * sp2_workspace_bytes(n, opt) <= SP2_NOALLOC_SCRATCH_BYTES (n <= 2048 with
 * default options).  Violations return SP2_ERR_INVALID_ARG before any work.
 * Every call on a device shares that device's array and overwrites what the
 * previous call left there, so calls that overlap in time on one device
 * (several host threads or streams) race; serialise them. */
#define SP2_NOALLOC_SCRATCH_BYTES ((size_t)136 << 20)
sp2_status sp2_density_noalloc(const float* H, int64_t n, int64_t ld, int64_t n_occ,
                               const sp2_options* opt, float* P, sp2_info* info,
                               uint8_t* branches, int32_t branches_cap, void* stream);

/* Forward derivative (density-matrix response, as needed for the XL-BOMD
 * kernel of Section III): P1 = dP/dH [H1] of the network recorded by the
 * last sp2_density_ex call on this workspace, with the spectral bounds and
 * the branch signs held fixed.  dS_0 = -H1 / (eps_max - eps_min); each layer
 * maps dS -> S dS + dS S (sign +) or 2 dS - (S dS + dS S) (sign -), using the
 * recomputed forward iterates; the refinement contributes its own
 * derivative.  The derivative products run in FP32 MFMA.  H1 (symmetric) and
 * P1: n x n with leading dimension ld.  Returns SP2_ERR_TAPE when the
 * workspace holds no usable tape (the forward kept none, did not converge,
 * or another call has reused the workspace since). */
sp2_status sp2_jvp(void* workspace, size_t ws_bytes, const float* H1, int64_t ld, float* P1,
                   void* stream);

/* Reverse derivative: the symmetric G with Tr(G H1) = Tr(W P1) for every
 * symmetric H1, i.e. dTr(W P)/dH of the recorded network (bounds and
 * branches fixed; W is symmetrised).  Replays the branch sequence backwards;
 * each layer maps G -> S G + G S (sign +) or 2 G - (S G + G S) (sign -); the
 * iterates S_n are recomputed segment by segment from the checkpoints.
 * Products in FP32 MFMA.  W and G: n x n with leading dimension ld. */
sp2_status sp2_vjp(void* workspace, size_t ws_bytes, const float* W, int64_t ld, float* G,
                   void* stream);

/* Estimates of the highest occupied and the lowest unoccupied eigenvalue of
 * H from a density matrix P of it (for the accelerated network of Section
 * II.E, SP2_FLAG_ACCELERATE; in molecular dynamics P comes from the previous
 * step).  HOMO = largest eigenvalue of H on the range of P, LUMO = smallest
 * on the range of I - P, each from `steps` (SP2_MIN_BOUND_STEPS ..
 * SP2_MAX_BOUND_STEPS) steps of the Lanczos recurrence (FP64 vectors, full
 * reorthogonalisation, as sp2_spectral_bounds) on v -> Q((H - s I) v),
 * Q = P or I - P, started from Q u / |Q u| with the SplitMix64 vector u of
 * `seed`; s = the Gershgorin eps_min (occupied side) or eps_max (virtual
 * side), so that the complement's zero eigenvalue cannot be the extreme
 * one.  Each extreme Ritz value is moved outwards by its residual norm
 * |beta_k s_k| (HOMO up, LUMO down), then the interval between them is
 * shrunk by margin (0 <= margin < 1/2) of its width on each side.  H and P:
 * n x n FP32, leading dimension ld, DEVICE; P symmetric (not checked).
 * Outputs are host doubles; blocks until done.  Reuses the workspace
 * header and Lanczos area (drops a derivative tape).  Returns
 * SP2_ERR_NONFINITE for NaN/Inf in H, SP2_ERR_NOT_CONVERGED when no gap
 * separates the two estimates (P empty or full, or not a density matrix of
 * H). */
sp2_status sp2_homo_lumo(const float* H, const float* P, int64_t n, int64_t ld, int32_t steps,
                         int32_t seed, double margin, double* homo, double* lumo, void* workspace,
                         size_t ws_bytes, void* stream);

/* Gershgorin enclosure of the spectrum of H (the linear map of the input
 * layer needs spectral bounds; Section II.D): eps_min = min_i(H_ii -
 * sum_{j!=i}|H_ij|), eps_max = max_i(H_ii + sum_{j!=i}|H_ij|), FP64 sums of
 * the FP32 entries.  Outputs are host doubles; blocks until done.  Returns
 * SP2_ERR_NONFINITE when H holds NaN/Inf. */
sp2_status sp2_bounds(const float* H, int64_t n, int64_t ld, double* eps_min, double* eps_max,
                      void* workspace, size_t ws_bytes, void* stream);

/* Tightened spectral bounds (the paper maps the spectrum onto [0, 1] in
 * Section II.D without fixing how the bounds are estimated).  Starting from
 * the Gershgorin interval of sp2_bounds, `steps` (SP2_MIN_BOUND_STEPS..SP2_MAX_BOUND_STEPS)
 * steps of the symmetric Lanczos recurrence run in FP64 (products of the
 * FP32 H with FP64 vectors) from the start vector u / |u|,
 * u_i = (z_i >> 11) 2^-53 - 1/2, z_i the SplitMix64 output of state
 * seed + (i+1) 0x9E3779B97F4A7C15.  The extreme eigenvalues th of the
 * Lanczos tridiagonal matrix, widened by their Ritz residual norms
 * |beta_k s_k| and by 1% of th_max - th_min, replace the Gershgorin bounds
 * where tighter.  This is what sp2_density_ex runs when opt->bound_steps > 0.
 * The widened Ritz interval is an estimate, not a proof: a Ritz value that
 * has not converged can sit inside the spectrum by more than its residual,
 * which is why fewer than SP2_MIN_BOUND_STEPS steps are refused (16 or more
 * are advisable for broad spectra).  A layer sequence started from an
 * interval that misses part of the spectrum ends in SP2_ERR_NOT_CONVERGED
 * rather than in a silently wrong P.
 * Outputs are host doubles; blocks until done.  Returns SP2_ERR_NONFINITE
 * when H holds NaN/Inf, SP2_ERR_INVALID_ARG for steps outside the range. */
sp2_status sp2_spectral_bounds(const float* H, int64_t n, int64_t ld, int32_t steps,
                               int32_t seed, double* eps_min, double* eps_max, void* workspace,
                               size_t ws_bytes, void* stream);

/* Dual representation of Eq. (20)-(21): hi = R[X], lo = R[X - hi] with
 * round-to-nearest-even R into bfloat16 (precision SP2_BF16X3/SP2_BF16X1)
 * or IEEE half of 2^14 X (SP2_FP16X3).  X: n x n FP32 with leading
 * dimension ld; hi, lo: n x n raw 16-bit patterns, leading dimension n.
 * Asynchronous on stream. */
sp2_status sp2_split(const float* X, int64_t n, int64_t ld, int32_t precision,
                     uint16_t* hi, uint16_t* lo, void* stream);

/* One expansion layer (Eq. 19, Fig. 1): Y = X^2 (sign = +1) or
 * Y = 2X - X^2 (sign = -1) for a symmetric X, computed by the same
 * symmetric-output MFMA kernels (and arithmetic `precision`) as the solver's
 * layers; in the split modes the product is that of the centred X - I/2
 * with the square restored as described for sp2_precision.  X, Y: n x n,
 * leading dimension ld, distinct buffers.  Blocks until done. */
sp2_status sp2_layer(const float* X, int64_t n, int64_t ld, int32_t precision, int32_t sign,
                     float* Y, void* workspace, size_t ws_bytes, void* stream);

/* Per-layer trace history of the last sp2_density_ex / sp2_density call on
 * this workspace: the traces of every examined approximation S_k, which
 * decide each branch and the stop (Section II.D-E: idempotency estimated
 * from traces), for k = 0 .. n_iter:
 *   t1[k] = Tr S_k, t2[k] = ||S_k||_F^2 (= Tr S_k^2), err[k] = |t1[k] - t2[k]|,
 * FP64 sums over the FP32 iterate as the layer kernels formed them.  Host
 * arrays of `cap` entries (any of them may be NULL; all NULL only with
 * cap = 0); min(cap, n_iter + 1) entries are written and *count (may be
 * NULL) receives n_iter + 1.  After a trivial occupation (n_occ in {0, n}),
 * a bound error, or another call that reuses the workspace (sp2_bounds,
 * sp2_spectral_bounds, sp2_layer), the history holds one meaningless entry.
 * coef (may be NULL): 3 * min(cap, n_iter) doubles, the coefficients
 * (a, b, c) of every applied layer S_{k+1} = a S_k^2 + b S_k + c I, in
 * FP64 as recorded (the layer kernels apply them rounded to FP32): (1, 0, 0)
 * and (-1, 2, 0) for plain layers, the scheduled ones with
 * SP2_FLAG_ACCELERATE.
 * Blocks until the copy is done. */
sp2_status sp2_history(void* workspace, size_t ws_bytes, int32_t cap, double* t1, double* t2,
                       double* err, double* coef, int32_t* count, void* stream);

/* ---- XL-BOMD kernel building block (Section III, Eq. 27-28) ----------------
 * Extended-Lagrangian dynamics propagates one net charge n_I per atom and
 * drives it towards the ground-state charges q0[n] of H(n) through the
 * kernel K = J^-1, J = dq0/dn - I the Jacobian of the residual
 * f(n) = q0[n] - n; the paper approximates K f in a preconditioned Krylov
 * subspace.  The charge model is given by its pieces:
 *   atom_ptr: DEVICE int64[n_atoms + 1]; atom I owns orbitals
 *             atom_ptr[I] .. atom_ptr[I+1]-1 (non-decreasing, at most n;
 *             orbitals past atom_ptr[n_atoms] belong to no atom).  Indices
 *             are clamped to [0, n], so a malformed array gives meaningless
 *             charges but no access outside the matrices.
 *   gamma:    DEVICE double[n_atoms * n_atoms], row-major, symmetric: the
 *             charge coupling, H(n) = H0 + diag(B gamma n) with B the
 *             orbital-to-atom incidence (every orbital of atom I shifted by
 *             (gamma n)_I).
 * Charge vectors are DEVICE double[n_atoms]. */
#define SP2_XL_MAX_RANK 32

/* Net Mulliken charges of a density matrix in an orthogonal basis with doubly
 * occupied states: q_I = z_I - 2 sum_{mu in I} P_mu,mu, minus sub_I when sub
 * is not NULL (with sub = the dynamical charges n, q is the residual f(n)).
 * P: n x n, leading dimension ld (only the diagonal is read); z, sub, q:
 * DEVICE double[n_atoms].  Asynchronous on stream. */
sp2_status sp2_mulliken(const float* P, int64_t n, int64_t ld, int64_t n_atoms,
                        const int64_t* atom_ptr, const double* z, const double* sub, double* q,
                        void* stream);

/* Device scratch (bytes, 256-aligned) of sp2_xl_response / sp2_xl_kernel for
 * matrices of order n, n_atoms atoms and Krylov rank `rank`. */
size_t sp2_xl_scratch_bytes(int64_t n, int64_t n_atoms, int32_t rank);

/* Charge-space Jacobian-vector product jv = J v = dq0/dn v - v at the H of
 * the last sp2_density_ex call on `workspace` (which must hold a derivative
 * tape: opt->checkpoint_every > 0): dq0/dn v = -2 B^T diag(P1) with P1 the
 * sp2_jvp response to H1 = diag(B gamma v).  v, jv: DEVICE double[n_atoms].
 * Blocks until done.  SP2_ERR_TAPE without a tape. */
sp2_status sp2_xl_response(void* workspace, size_t ws_bytes, int64_t n_atoms,
                           const int64_t* atom_ptr, const double* gamma, const double* v,
                           double* jv, void* scratch, size_t scratch_bytes, void* stream);

/* Rank-`rank` (1..SP2_XL_MAX_RANK) Krylov approximation kf ~ K f = J^-1 f at
 * the H of the last sp2_density_ex call on `workspace` (derivative tape
 * required).  With the preconditioner K0 (DEVICE double[n_atoms^2],
 * row-major; NULL means K0 = -I): v_1 = K0 f / |K0 f|; each further basis
 * vector is K0 J v_k (one sp2_xl_response) orthonormalised against the
 * previous ones (classical Gram-Schmidt, two passes); kf = V c with c
 * minimising |K0 J V c - K0 f| (QR of the K0 J v_k, two-pass Gram-Schmidt).
 * This is the minimal-residual (GMRES) form of the preconditioned Krylov
 * approximation; at full rank it is exact.  The basis stops early when a new
 * direction vanishes (invariant subspace: the result is then exact).
 * Outputs: kf (DEVICE double[n_atoms]); rho (HOST double[rank + 1] or NULL):
 * rho[0] = |K0 f|, rho[k] the minimal residual with k basis vectors (entries
 * past the rank used are repeated); rank_used (HOST or NULL).  Blocks until
 * done.  SP2_ERR_INVALID_ARG for a rank outside the range or too small a
 * scratch; SP2_ERR_TAPE without a tape. */
sp2_status sp2_xl_kernel(void* workspace, size_t ws_bytes, int64_t n_atoms,
                         const int64_t* atom_ptr, const double* gamma, const double* k0,
                         const double* f, int32_t rank, double* kf, double* rho,
                         int32_t* rank_used, void* scratch, size_t scratch_bytes, void* stream);

/* ---- Canonical integration with force noise as the heat bath (Section IV) ----
 * One time step of Eq. 31 (scheme 0) or of the variant in the Supporting
 * Information (scheme 1) for n independent scalar coordinates (x, y, z of
 * every atom), FP64, split where the force is evaluated:
 *   sp2_nvt_first_half:  R_k, V_k, F_k, eta_k -> R <- R_{k+1} and V <- W, the
 *                        velocity before the last half kick;
 *   (caller: F_{k+1} = force at R_{k+1}, including its noise sigma_TC xi)
 *   sp2_nvt_second_half: W, F_{k+1} -> V <- V_{k+1}.
 * Scheme 0: V' = V + h (F - gamma_tc V); R' = R + dt/2 V';
 * W = c_L V' + sigma_L eta; R_{k+1} = R' + dt/2 W; V_{k+1} solves
 * V_{k+1} = W + h (F_{k+1} - gamma_tc V_{k+1}).  Scheme 1: V' = V + h F;
 * R' = R + dt/2 V'; W = s (c_L (s V') + sigma_L eta) with
 * s = sqrt((1 - gamma_tc h) / (1 + gamma_tc h)); R_{k+1} = R' + dt/2 W;
 * V_{k+1} = W + h F_{k+1}.  Here h = dt / (2M), c_L = (1 - gamma_l dt/2) /
 * (1 + gamma_l dt/2), sigma_L = sqrt(kt (1 - c_L^2) / M) (Eq. 32).
 * gamma_tc is a force per velocity (mass per time); Eq. 33 balances force
 * noise of standard deviation sigma_TC with gamma_tc = sigma_TC^2 dt / (2 kT)
 * (sp2_nvt_gamma_tc).  Scheme 1 needs gamma_tc dt < 2M for every coordinate
 * (else its friction factor is imaginary and V becomes NaN).
 * Arrays are DEVICE double[n]: R, V updated in place; F the force at the
 * positions the step starts from (first half) or ends at (second half);
 * eta standard normal Langevin noise, may be NULL when gamma_l = 0; mass the
 * mass of every coordinate.  Units are the caller's, consistent (e.g. eV,
 * Angstrom, fs, eV fs^2 / Angstrom^2).  Every operation is the correctly
 * rounded FP64 evaluation of these formulas in the order written (no fused
 * multiply-adds).  Asynchronous on stream; n = 0 is a no-op. */
typedef struct {
  double dt;          /* time step, > 0 */
  double kt;          /* k_B T, >= 0 */
  double gamma_tc;    /* friction balancing the force noise, force per velocity, >= 0 */
  double gamma_l;     /* Langevin friction, per time, >= 0 (0: no Langevin term) */
  int32_t scheme;     /* 0: Eq. 31; 1: the Supporting Information's variant */
  int32_t reserved;   /* 0 */
} sp2_nvt_params;

/* gamma_tc = sigma_tc^2 dt / (2 kt) (Eq. 33); NaN unless sigma_tc >= 0,
 * kt > 0 and dt > 0. */
double sp2_nvt_gamma_tc(double sigma_tc, double kt, double dt);

sp2_status sp2_nvt_first_half(double* R, double* V, const double* F, const double* eta,
                              const double* mass, int64_t n, const sp2_nvt_params* p,
                              void* stream);

sp2_status sp2_nvt_second_half(double* V, const double* F, const double* mass, int64_t n,
                               const sp2_nvt_params* p, void* stream);

/* Thread-local text describing the last error of this thread ("" if none). */
const char* sp2_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SP2_H */
