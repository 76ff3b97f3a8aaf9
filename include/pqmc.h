/*
 * pqmc.h -- C ABI of the MI355X (gfx950) ground-state AFQMC field-update sweep.
 *
 * The library runs one projector-QMC Markov chain (one "walker") of a
 * spin-1/2 lattice model with on-site Hubbard interaction, following
 * H. Du and Y.-Y. He, "Accelerating ground-state auxiliary-field quantum
 * Monte Carlo simulations by delayed update and block force-bias update",
 * arXiv:2506.09611:
 *
 *   weight      W(X) = prod_s det(P_s^+ B_M ... B_1 P_s)          Sec. II B, Eq. (8)
 *   propagator  B_l^s = diag(e^{alpha f_s x_l}) e^{-dtau H0}      Eqs. (9), (13)-(14)
 *   state       U_R, U_L, T = (U_L U_R)^{-1}; G = 1 - U_R T U_L   Sec. II B, Eq. (15)
 *   updates     local (Eqs. (20)-(21)), delayed (Sec. III A, Eqs. (27)-(30)),
 *               block force-bias (Sec. III B, Eqs. (31)-(36))
 *
 * U > 0 uses the real coupling alpha = arccosh(e^{dtau U/2}) with two real
 * float64 spin sectors (f_up = +1, f_dn = -1); U = 0 gives alpha = 0.
 * U < 0 is the paper's own convention (Sec. II B, Eqs. (13)-(14)):
 * alpha = i gamma, gamma = arccos(e^{dtau U/2}), so B_dn = conj(B_up) and
 * only the spin-up sector is simulated, in complex128, with
 * R = r_up r_dn = |r_up|^2.  It needs n_dn = n_up and trial_dn = trial_up,
 * runs the local (as groups of one site), delayed (k <= 64) and block
 * force-bias (b <= 64) schemes with the LOG and TIMING flags, and returns
 * complex G from pqmc_get_green; batches of U < 0 walkers run one walker
 * after the other.
 *
 * Memory: the library allocates no device memory.  The caller obtains the
 * size from pqmc_workspace_bytes() and passes one device buffer of at least
 * that many bytes, 256-byte aligned, which must stay valid until
 * pqmc_destroy().  Host inputs are copied during pqmc_create(); the caller
 * keeps ownership of every pointer it passes.
 *
 * Streams: every call enqueues work on the HIP stream given to pqmc_create()
 * (NULL = the null stream).  pqmc_sweep() returns after its work completes;
 * the getters synchronise the stream before they copy.
 *
 * Errors: every function returns a pqmc_status; a message for the calling
 * thread's last failure is available from pqmc_last_error().  After
 * PQMC_ESINGULAR or PQMC_ENONFINITE the context refuses further sweeps
 * (PQMC_ESTATE) until pqmc_set_fields() rebuilds its state.  No C++
 * exception crosses this interface.
 */
#ifndef PQMC_H
#define PQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pqmc_ctx pqmc_ctx;

typedef enum {
  PQMC_OK = 0,
  PQMC_EINVAL = -1,      /* bad argument or unsupported problem             */
  PQMC_ENOMEM = -2,      /* workspace too small                             */
  PQMC_EDEVICE = -3,     /* a HIP runtime call failed                       */
  PQMC_ESINGULAR = -4,   /* a stabilisation factorisation broke down        */
  PQMC_ENONFINITE = -5,  /* a determinant ratio was not finite              */
  PQMC_ESTATE = -6       /* context is in a failed state                    */
} pqmc_status;

/* Update schemes.
 *   PQMC_LOCAL    sites i = 1..N of a slice one by one, Sherman-Morrison
 *                 rank-1 upgrade of T per accepted flip (Sec. II D,
 *                 Eqs. (20)-(21)).  A single walker runs it as one
 *                 cooperative launch per slice with T held in registers
 *                 across the GPU and one grid barrier per site (N_up, N_dn
 *                 <= 1024); batches of walkers, or PQMC_FLAG_SITE_LAUNCHES,
 *                 run one launch per site.
 *   PQMC_DELAYED  groups of delay_k consecutive sites; ratios from the
 *                 delayed recursion and one rank-n_A flush of T per group
 *                 (Sec. III A, first strategy: n_d = proposals).
 *   PQMC_BLOCK_FB blocks of block_b consecutive sites proposed together from
 *                 the force-bias heat-bath prior, one Metropolis test per
 *                 block and a rank-n_F Woodbury upgrade (Sec. III B).
 *   PQMC_LOCAL_G  the local update on the equal-time Green's function
 *                 itself: r_s = 1 + Delta_s (1 - G_s,ii) and
 *                 G <- G - (Delta / r) G[:, i] (e_i^T - G[i, :]), O(N^2) per
 *                 site (the G-form that Sec. III A contrasts with the
 *                 T-form); G is propagated as B G B^{-1} between slices and
 *                 rebuilt from U_L, U_R at every stabilisation.  Same
 *                 decisions as PQMC_LOCAL.  One cooperative launch per slice
 *                 with G held in registers (N_s <= 2048); the context must be
 *                 created with this scheme (G is sized in the workspace).  */
typedef enum { PQMC_LOCAL = 0, PQMC_DELAYED = 1, PQMC_BLOCK_FB = 2,
               PQMC_LOCAL_G = 3 } pqmc_scheme;

/* flags of pqmc_update_opts */
#define PQMC_FLAG_LOG    1u  /* record every decision of the last pqmc_sweep call */
#define PQMC_FLAG_TIMING 2u  /* time propagation / update / stabilisation phases  */
#define PQMC_FLAG_KTIME  4u  /* time every launch of the kernel classes below      */
/* Precision form (delayed and block force-bias with k, b <= 64): between
 * stabilisations T is kept in float32 and the group flush and panel products
 * run on FP32 MFMA with FP32 accumulation.  The panel sums, W0, every
 * acceptance ratio and decision, the propagation, the QR and the inverse
 * stay float64, and T is recomputed in float64 from U_L, U_R at every
 * stabilisation, which discards the float32 drift.  Decisions can differ
 * from the float64 chain where a ratio lies within the float32 error of u. */
#define PQMC_FLAG_FP32   8u
/* PQMC_LOCAL with one launch per site (the form batches use) instead of the
 * persistent kernel, for comparisons. */
#define PQMC_FLAG_SITE_LAUNCHES 16u
/* Graph-captured sweeps (delayed and block force-bias): the first sweep of
 * a batch records its whole forward and backward pass -- every propagation,
 * panel, decision, flush and stabilisation launch -- into one HIP graph, and
 * every sweep (that one included) is one graph launch; the Philox sweep
 * counter is read from device memory.  The graph is kept by the batch's
 * first context and captured again when the batch or any walker's options,
 * fields or position change.  Needs a non-null stream; phase and kernel
 * timers are off; with n_sweeps > 1 the decision log holds the last sweep.
 * Results are bit for bit those of the sweeps launched one by one.  While a
 * capture runs (the first graph sweep of a batch, or the first after a
 * change), no other thread of the process may use the legacy (null) stream
 * or synchronise the device; the library's own calls copy on the contexts'
 * streams, so concurrent batches of pqmc_multi_sweep are safe. */
#define PQMC_FLAG_GRAPH  32u
/* Propagate with the dense K = e^{-dtau H0} and K^{-1} (GEMMs) even when H0
 * is sparse.  By default a walker whose H0 has at most 8 nonzeros per row,
 * N <= 4096 and ||dtau H0||_1 <= 1 applies e^{-+dtau H0} as the Taylor series
 * of the sparse H0 (degree J with a dropped term below 2^-60; the same
 * operator to rounding), which costs 2 J nnz(H0) N_sigma flops per product
 * instead of 2 N^2 N_sigma.  The same holds for the complex 2N x 2N H0 of
 * pqmc_soc_create (and the U < 0 model), where this flag is also accepted. */
#define PQMC_FLAG_DENSE_PROP 64u

/* kernel classes of pqmc_get_kernel_times() */
enum {
  PQMC_K_PROPAGATE = 0,  /* batched B-matrix propagation GEMM (one per slice visit)  */
  PQMC_K_LOCAL = 1,      /* local update: a site step, or a whole persistent slice   */
  PQMC_K_TILE = 2,       /* group flush + next group's panel products (MFMA)        */
  PQMC_K_REDUCE = 3,     /* panel partial sums and W0                                */
  PQMC_K_DECIDE = 4,     /* delayed / block force-bias decision kernel              */
  PQMC_K_COUNT = 5
};

typedef struct {
  int32_t n_sites;            /* N_s: number of lattice sites                          */
  int32_t n_up, n_dn;         /* N_up, N_dn: particles per spin, 1 <= N_s <= n_sites   */
  const double *hopping;      /* H0, N_s x N_s row-major, real symmetric (Sec. II B)   */
  const double *trial_up;     /* P_up, N_s x N_up row-major, orthonormal columns       */
  const double *trial_dn;     /* P_dn, N_s x N_dn row-major, orthonormal columns       */
  double U;                   /* on-site interaction (U < 0: see above)                */
  double dtau;                /* imaginary-time step                                   */
  int32_t n_slices;           /* M = 2 Theta / dtau                                     */
  int32_t stab_every;         /* k_tau: QR stabilisation period, must divide M         */
  uint64_t seed;              /* Philox key word 0                                     */
  uint64_t walker_id;         /* Philox key word 1                                     */
} pqmc_problem;

typedef struct {
  int32_t scheme;             /* pqmc_scheme                                           */
  int32_t delay_k;            /* n_d for PQMC_DELAYED, 1 <= k <= 128 (clipped to N_s)   */
  int32_t block_b;            /* n_b for PQMC_BLOCK_FB, 1 <= b <= 64 (clipped to N_s)   */
  uint32_t flags;             /* PQMC_FLAG_*                                           */
  int32_t tile_chunks;        /* column chunks per 64-row strip of T in the fused flush
                                 kernel (delayed / block): 0 = 2, suited to batches of
                                 several walkers; larger values give shorter chunks and
                                 more workgroups (a value >= N_s/64 gives one 64 x 64
                                 tile each, suited to one walker).  The summation order
                                 of the panel partials, and hence G to rounding, depends
                                 on it and on nothing else of the batch.              */
} pqmc_update_opts;

typedef struct {
  uint64_t proposed;          /* Metropolis tests (sites, or blocks for block FB)      */
  uint64_t accepted;          /* accepted tests                                        */
  uint64_t flips;             /* fields changed                                        */
  uint64_t low_margin;        /* decisions with | |A| - u | < 1e-12 (incl. heat bath)  */
  uint64_t negative;          /* accepted-or-not tests with a negative weight ratio    */
  uint64_t field_updates;     /* single-site field visits (2 M N per sweep)            */
  double t_total_s;           /* wall time of the call (stream-synchronised)           */
  double t_update_s;          /* with PQMC_FLAG_TIMING: field-update phase             */
  double t_prop_s;            /* with PQMC_FLAG_TIMING: B-matrix propagation phase     */
  double t_stab_s;            /* with PQMC_FLAG_TIMING: QR + inverse phase             */
  double max_stab_drift;      /* largest |G_running - G_fresh| entry that a QR
                                 stabilisation corrected (Sec. II B), over 16 sampled
                                 columns of G per stabilisation and spin: how far the
                                 updated state had drifted from the recomputed one   */
} pqmc_stats;

/* Size of the device workspace for this problem and the largest delay_k /
 * block_b the context will be asked to run (opts->delay_k, opts->block_b
 * are upper bounds for later pqmc_set_opts calls).  Validates the problem. */
pqmc_status pqmc_workspace_bytes(const pqmc_problem *prob, const pqmc_update_opts *opts,
                                 size_t *bytes);

/* Build a context: copies H0 and P_s to the device, computes
 * K = e^{-dtau H0} and K^{-1} (Taylor series with scaling and squaring),
 * draws the initial fields x_{l,i} = +1 iff u(INIT; 0, l-1, i) < 1/2, builds
 * the stack of row-orthonormalised U_L at every k_tau (Sec. II B) and sets
 * the walker at position 0 with U_R = P, T = (U_L U_R)^{-1}.
 * workspace: device pointer, >= pqmc_workspace_bytes(), 256-byte aligned. */
pqmc_status pqmc_create(const pqmc_problem *prob, const pqmc_update_opts *opts,
                        void *hip_stream, void *workspace, size_t workspace_bytes,
                        pqmc_ctx **out);

/* Change scheme / k / b / flags (k and b within the workspace bounds). */
pqmc_status pqmc_set_opts(pqmc_ctx *ctx, const pqmc_update_opts *opts);

/* Replace the field configuration (host, M x N_s int8 row-major, entries
 * +1 or -1) and rebuild the stack and position-0 state; clears a failed state. */
pqmc_status pqmc_set_fields(pqmc_ctx *ctx, const int8_t *fields);

/* Copy the current fields to host memory (M x N_s int8). */
pqmc_status pqmc_get_fields(pqmc_ctx *ctx, int8_t *fields);

/* Run n_sweeps sweeps.  One sweep is the forward pass l = 1..M (propagate,
 * update slice l, stabilise when k_tau divides l) followed by the backward
 * pass l = M..1 (update slice l, propagate back, stabilise when k_tau
 * divides l-1) -- Sec. II B and the efficiency measurements of Sec. IV.
 * Metropolis test of Eq. (16): accept iff u < |A|, u from Philox4x64-10 at
 * counter (sweep, dir*M + l-1, site, purpose).  out may be NULL. */
pqmc_status pqmc_sweep(pqmc_ctx *ctx, int32_t n_sweeps, pqmc_stats *out);

/* Run only the forward pass over slices 1..n_slices (a window of a sweep;
 * leaves the walker at position n_slices).  Used for windowed comparisons
 * at sizes where a whole sweep is long; the next pqmc_sweep is refused. */
pqmc_status pqmc_forward_window(pqmc_ctx *ctx, int32_t n_slices, pqmc_stats *out);

/* Batched walkers: run the sweeps of n contexts (1 <= n <= 8) in lockstep,
 * every kernel launch covering all of them (independent Markov chains, each
 * with its own Philox key, fields, stack and statistics).  The contexts must
 * share n_slices, stab_every, scheme, delay_k, block_b, the precision form
 * and the stream, and their workspace group bounds (the larger of
 * min(delay_k, n_sites) and min(block_b, n_sites) at creation) must lie on
 * the same side of 64 (PQMC_EINVAL otherwise).  With the local scheme they
 * must also share n_sites, n_up and n_dn; with the delayed and block
 * force-bias schemes the lattices may differ in size (n_sites, n_up, n_dn):
 * the batch walks the groups of the largest lattice and a walker takes part
 * in those that hold its own sites.  Hopping matrices, U and seeds may
 * differ.  Each walker's decisions, fields and G are the ones pqmc_sweep
 * would give it alone, bit for bit.  out: n entries or
 * NULL; the timing fields of every entry are those of the whole batch.  The
 * phase and kernel timers are those of ctxs[0]. */
pqmc_status pqmc_batch_sweep(pqmc_ctx *const *ctxs, int32_t n, int32_t n_sweeps,
                             pqmc_stats *out);

/* pqmc_forward_window for a batch of walkers (same rules as pqmc_batch_sweep). */
pqmc_status pqmc_batch_forward_window(pqmc_ctx *const *ctxs, int32_t n, int32_t n_slices,
                                      pqmc_stats *out);

/* Walkers on several streams: the n contexts (1 <= n <= 128) are split by
 * their stream, in order of first appearance (at most 16 streams); the
 * walkers of one stream form one pqmc_batch_sweep batch (same rules, at most
 * 8 walkers), and the batches run concurrently, each driven by its own host
 * thread, so that the serial phases of one batch (decisions, panel sums)
 * overlap the MFMA work of another.  Independent chains as in
 * pqmc_batch_sweep: each walker's decisions, fields and G are the ones it
 * gets alone.  out: n entries in ctxs order, or NULL; timing fields are
 * those of the walker's own batch.  Errors: PQMC_EINVAL or PQMC_ESTATE from
 * the checks, before any work starts; otherwise the status and message of
 * the first failing batch in stream order (the other batches still finish,
 * and the failing batch's contexts need pqmc_set_fields).  The calling
 * thread's current HIP device is used by every worker thread. */
pqmc_status pqmc_multi_sweep(pqmc_ctx *const *ctxs, int32_t n, int32_t n_sweeps,
                             pqmc_stats *out);

/* Replay: one sweep (forward then backward, as pqmc_sweep) in which every
 * outcome is forced instead of drawn.  flips: host, 2 M x N_s int8, row
 * v = dir*M + l-1 (dir 0 forward, 1 backward) for the visit of slice l;
 * flips[v*N_s + i] != 0 means that the field of site i flips on that visit.
 *   PQMC_LOCAL, PQMC_DELAYED: the Metropolis test of site i is accepted iff
 *     listed (its ratio is still computed, logged and checked for NaN);
 *   PQMC_BLOCK_FB: each block's heat-bath proposal is the listed flip set
 *     and the block's Metropolis test is accepted (an empty set is the usual
 *     no-op).
 * The same list through the three schemes yields the same fields and, in
 * exact arithmetic, the same G: the cross-scheme invariant of the updates
 * (Secs. II D, III A, III B all apply Eq. (19) to the accepted flips).
 * Forced outcomes are implemented as uniforms u = -0 (take) and u = +inf
 * (do not take) in place of the Philox draws, so the log's margin field
 * holds |A| itself for a taken outcome and -inf otherwise.  The walker must be at position 0 (PQMC_ESTATE
 * otherwise); the sweep counter advances as after pqmc_sweep. */
pqmc_status pqmc_replay(pqmc_ctx *ctx, const int8_t *flips, pqmc_stats *out);

/* G^s = 1 - U_R T U_L at the walker's current position (Eq. (15)),
 * written to host memory as N_s x N_s row-major float64.  spin: 0 up, 1 down.
 * U < 0: complex128, (re, im) interleaved (2 N_s^2 doubles); spin 1 is the
 * complex conjugate of spin 0. */
pqmc_status pqmc_get_green(pqmc_ctx *ctx, int32_t spin, double *out);

/* pqmc_get_green for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same G, bit for bit, with its two device temporaries (U_R T, N x N_s,
 * and G, N x N) taken from a static device array of the library instead of
 * the context's workspace.  The array holds 4194304 doubles (32 MiB) on every
 * GPU the library runs on, until the process ends; problems with
 * N_s (N_s + N_sigma) (rounded up to 32) above that are refused with
 * PQMC_EINVAL.  Calls no hipMalloc, hipFree or allocating library routine
 * (its device address is looked up once per device, on the first call).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (several host threads or streams at once) race and must be
 * serialised by the caller.  U < 0 contexts are refused (PQMC_EINVAL). */
pqmc_status pqmc_get_green_static(pqmc_ctx *ctx, int32_t spin, double *out);

/* Decisions of the last pqmc_sweep / pqmc_forward_window call made with
 * PQMC_FLAG_LOG, in order: meta[3*n] = (dir*M + l-1, site, accepted) and
 * margin[n] = |A| - u.  For block FB, site is the block's first site and the
 * heat-bath draws are not included.  cap: capacity of the host arrays; *n
 * receives the number of entries (copied: min(cap, count)). */
pqmc_status pqmc_get_decisions(pqmc_ctx *ctx, int32_t *meta, double *margin, size_t cap,
                               size_t *n);

/* Heat-bath draws of the last block-FB call made with PQMC_FLAG_LOG:
 * meta[3*n] = (dir*M + l-1, site, proposed x'), margin[n] = p(+1) - u. */
pqmc_status pqmc_get_heat_bath(pqmc_ctx *ctx, int32_t *meta, double *margin, size_t cap,
                               size_t *n);

/* With PQMC_FLAG_KTIME set for the last pqmc_sweep / pqmc_forward_window
 * call: total device time (seconds, from HIP events bracketing each launch
 * on the context's stream) and launch count per kernel class PQMC_K_*.
 * totals and counts: host arrays of PQMC_K_COUNT entries. */
pqmc_status pqmc_get_kernel_times(pqmc_ctx *ctx, double *totals, uint64_t *counts);

/* Release the context (the workspace stays the caller's). */
pqmc_status pqmc_destroy(pqmc_ctx *ctx);

/* Message of the calling thread's last failure ("" if none). */
const char *pqmc_last_error(void);

/* ------------------------------------------------------------------------
 * Spin-orbit coupled Hubbard model (Eq. (2), Appendix A): one complex
 * sector in the basis (c_1up .. c_Nup, c_1dn .. c_Ndn), 2N orbitals, N_e
 * fermions, complex128 throughout.  The interaction is decoupled in the
 * spin-s^y channel, Eq. (A4): gamma = arccos(e^{dtau U/2}) (U <= 0), and
 * e^{H_I(x)} mixes the row pair (i, N+i) by A(x_i) = e^{gamma x_i i sigma_y},
 * Eq. (A6).  B_l = e^{H_I(x_l)} e^{-dtau H0}; U_R is 2N x N_e, U_L N_e x 2N,
 * T = (U_L U_R)^{-1} N_e x N_e, G = 1 - U_R T U_L (2N x 2N).
 * Updates: PQMC_LOCAL (rank-two Sherman-Morrison per site, Eqs. (A7)-(A9)),
 * PQMC_DELAYED (delay_k <= 32 sites per flush, the x_m, y_m of
 * Eqs. (28)-(30) grown to N_e x 2 and 2 x N_e blocks) and PQMC_BLOCK_FB
 * (block_b <= 32 sites per block, Sec. III B with the force bias
 * s_i = gamma <c+_{i up} c_{i dn} - c+_{i dn} c_{i up}> of the spin-s^y
 * channel, the block's own fields removed; one decision and one log entry
 * per block, at its first site).  Metropolis: accept iff u < |R| (times the
 * prior ratio for blocks), R = det(1 + Y V), with the uniforms of the
 * spin-decoupled path (same Philox counters).  Flags: LOG, TIMING.  Same
 * workspace, stream and error rules as pqmc_create.
 * ------------------------------------------------------------------------ */
typedef struct pqmc_soc_ctx pqmc_soc_ctx;

typedef struct {
  int32_t n_sites;            /* N (the matrices are 2N x 2N)                          */
  int32_t n_e;                /* N_e fermions, 1 <= N_e <= min(2N, 1024)                */
  const double *hopping;      /* 2N x 2N complex128 row-major, (re, im) interleaved,
                                 Hermitian (copied)                                      */
  const double *trial;        /* 2N x N_e complex128 row-major, orthonormal columns    */
  double U;                   /* <= 0                                                  */
  double dtau;
  int32_t n_slices;           /* M                                                     */
  int32_t stab_every;         /* k_tau, divides M                                      */
  uint64_t seed;
  uint64_t walker_id;
} pqmc_soc_problem;

/* Workspace size for this problem (opts->delay_k <= 32 when delayed). */
pqmc_status pqmc_soc_workspace_bytes(const pqmc_soc_problem *prob, const pqmc_update_opts *opts,
                                     size_t *bytes);

/* Build a context: e^{-dtau H0} and e^{dtau H0} on the device (Taylor
 * series with scaling and squaring), Philox fields, the stack of U_L and
 * the position-0 state.  workspace: device, 256-byte aligned. */
pqmc_status pqmc_soc_create(const pqmc_soc_problem *prob, const pqmc_update_opts *opts,
                            void *hip_stream, void *workspace, size_t workspace_bytes,
                            pqmc_soc_ctx **out);

/* n_sweeps sweeps (forward l = 1..M, backward l = M..1, stabilising every
 * k_tau slices as pqmc_sweep).  out may be NULL. */
pqmc_status pqmc_soc_sweep(pqmc_soc_ctx *ctx, int32_t n_sweeps, pqmc_stats *out);

/* Forward pass over slices 1..n_slices only; the context then refuses
 * further sweeps. */
pqmc_status pqmc_soc_forward_window(pqmc_soc_ctx *ctx, int32_t n_slices, pqmc_stats *out);

/* pqmc_soc_sweep / pqmc_soc_forward_window for a batch of n <= 8 walkers
 * (Appendix A model, independent Markov chains) in lockstep: every launch
 * (complex GEMMs, decisions, eliminations) serves all of them.  The walkers
 * need the same lattice, N_e, M, k_tau, scheme, k (or b) and stream; each
 * takes exactly the decisions and reaches the G it reaches alone.  out: n
 * entries or NULL.  Errors mark every walker of the batch failed. */
pqmc_status pqmc_soc_batch_sweep(pqmc_soc_ctx *const *ctxs, int32_t n, int32_t n_sweeps,
                                 pqmc_stats *out);
pqmc_status pqmc_soc_batch_forward_window(pqmc_soc_ctx *const *ctxs, int32_t n,
                                          int32_t n_slices, pqmc_stats *out);

/* G = 1 - U_R T U_L at the current position, 2N x 2N complex128 row-major
 * interleaved, to host memory. */
pqmc_status pqmc_soc_get_green(pqmc_soc_ctx *ctx, double *out);

/* Current fields, M x N int8. */
pqmc_status pqmc_soc_get_fields(pqmc_soc_ctx *ctx, int8_t *fields);

/* Decisions of the last call (PQMC_FLAG_LOG), as pqmc_get_decisions. */
pqmc_status pqmc_soc_get_decisions(pqmc_soc_ctx *ctx, int32_t *meta, double *margin,
                                   size_t cap, size_t *n);

/* Release the context (not the workspace). */
pqmc_status pqmc_soc_destroy(pqmc_soc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* PQMC_H */
