/*
 * mvmc.h -- C ABI of libmvmc, the MI355X (gfx950) many-variable variational
 * Monte Carlo hot path: batched Metropolis sampling of a Pfaffian x Jastrow x
 * Gutzwiller (optionally x RBM) wave function, local energies and
 * log-derivatives, and the stochastic-reconfiguration (SR) update.
 *
 * The operations follow arXiv:1711.11418 ("mVMC -- open-source software for
 * many-variable variational Monte Carlo method"):
 *   wave function   psi = P_G P_J phi_AP-Pf      section 3.2 (Eqs. Pf, AP-Pf,
 *                                                 Gutzwiller/Jastrow factors)
 *   <x|phi_Pf>      proportional to Pf(X), X_IJ = F_IJ - F_JI   section 3.2.1
 *   sampling        Metropolis over rho(x) = |<x|psi>|^2, hopping update
 *                   and Sherman-Morrison-type fast update   section 3.1
 *   estimators      Eq. MC (local energy); O_k = d ln<x|psi>/d alpha_k with
 *                   Eq. DiffPf for the pair amplitudes      section 3.3.1
 *   SR              Delta alpha = -dtau S^-1 g (Eq. SR_equation_system),
 *                   Cholesky or the CG method of Algorithm 1   sections 3.3.1-3.3.2
 * plus an RBM factor exp(sum_v a_v s_v) prod_h 2 cosh(b_h + sum_v W_hv s_v),
 * s_v = 2 n_v - 1 over the 2 Ns spin-orbitals (not in the paper).
 *
 * Conventions for every function:
 *   - Returns an mvmc_status; MVMC_OK == 0.  Nothing throws across the ABI.
 *   - Arguments are checked before anything is enqueued; on an argument error
 *     the context is unchanged.  mvmc_last_error() describes the last failure.
 *   - Pointers named d_* are device pointers, h_* host pointers.  The caller
 *     owns every buffer it passes, including the workspace; the library owns
 *     only the host-side context and never allocates device memory.
 *   - All device work is enqueued on the stream given to init, in order.
 *     Calls that fill h_* outputs synchronise that stream before returning.
 *   - Spin-orbital index I = i + Ns*sigma (sigma = 0 up, 1 down); electron
 *     a < n_up is up, a >= n_up is down (section 3.2.1).
 */
#ifndef MVMC_H
#define MVMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mvmc_ctx mvmc_ctx;

typedef enum {
  MVMC_OK = 0,
  MVMC_E_ARG = 1,        /* bad pointer, value or index map */
  MVMC_E_SHAPE = 2,      /* inconsistent sizes (odd N_e, n_up != n_dn, ...) */
  MVMC_E_WORKSPACE = 3,  /* workspace too small or misaligned */
  MVMC_E_HIP = 4,        /* a HIP runtime call or kernel launch failed */
  MVMC_E_SINGULAR = 5,   /* X (or the regularised S) could not be factorised */
  MVMC_E_NONFINITE = 6,  /* NaN/Inf parameter or result */
  MVMC_E_STATE = 7       /* call out of order (e.g. sr_update before build_sr) */
} mvmc_status;

typedef enum { MVMC_FP64 = 0, MVMC_MIXED = 1 } mvmc_precision;
typedef enum { MVMC_SOLVE_CHOL = 0, MVMC_SOLVE_CG = 1 } mvmc_solver;

/*
 * One lattice instance (host pointers, copied at init).  Hamiltonian
 * H = -sum_bonds,sigma t (c+_i c_j + h.c.) + sum_i U_i n_iup n_idn
 * (section 2.3, Eq. GHam with H_U).  Index maps name the parameter slot of
 * each pair amplitude f_ij, Gutzwiller g_i and Jastrow v_ij (the Orbital,
 * Gutzwiller and Jastrow keyword files of Table 1), -1 = held at zero.
 * Instance parameter vector: [f (n_f) | g (n_g) | v (n_v) | RBM a (2Ns) |
 * RBM b (M) | RBM W (M x 2Ns row-major)], the RBM blocks only when M > 0.
 */
typedef struct {
  int32_t n_sites;            /* Ns, 3..1024 */
  int32_t n_up, n_dn;         /* n_up == n_dn >= 1 (anti-parallel pairing, Eq. AP-Pf) */
  int32_t n_bonds;            /* unordered nearest-neighbour bonds */
  const int32_t *bond_i;      /* [n_bonds] */
  const int32_t *bond_j;      /* [n_bonds] */
  const double *bond_t;       /* [n_bonds] hopping amplitude t_ij */
  const double *U;            /* [Ns] on-site interaction */
  int32_t n_f;                /* pair-amplitude slots */
  const int32_t *f_idx;       /* [Ns*Ns] row-major, f_ij slot or -1 */
  int32_t n_g;
  const int32_t *g_idx;       /* [Ns] */
  int32_t n_v;
  const int32_t *v_idx;       /* [Ns*Ns] symmetric, diagonal -1 */
  int32_t n_hidden;           /* RBM hidden units M; 0 = no RBM factor */
  int32_t n_walkers;          /* independent Markov chains for this instance */
  /* Quantum-number projection of the pair-product part (section 3.2.2, Eqs.
   * momP and pointP): <x|psi> = P_G P_J [RBM] sum_p w_p Pf(X(q_p(x))), where
   * q_p(x) puts every electron on the image q_p(i) of its site i (spin and
   * electron order kept), i.e. term p is the AP Pfaffian with
   * f_p(i, j) = f(q_p(i), q_p(j)).  A translation or point-group operation
   * with a real character (momentum K with K.R in {0, pi}) is one term; the
   * 1/N_g normalisation is dropped.  n_proj = 0: no projection.  Projected
   * instances run their own sweep (hopping updates, all N_P inverses M_p^-1
   * in LDS, rank-1 updates of each) and refresh; they need exchange_per64 = 0
   * and MVMC_SCHED_BUCKETS, and sweep_variant / sweep_threads do not apply
   * to them.  Every M_p must be invertible at every visited configuration: a
   * proposal whose acceptance would make one singular stops the walker like
   * a non-finite ratio. */
  int32_t n_proj;             /* N_P, 0..MVMC_MAX_PROJ */
  const int32_t *proj_map;    /* [N_P * Ns] row-major: q_p(i); each row a permutation */
  const double *proj_weight;  /* [N_P] real weights w_p, finite, not all zero */
} mvmc_instance_desc;

#define MVMC_MAX_PROJ 32

typedef struct {
  int32_t precision;          /* MVMC_FP64: double sweeps and S.  MVMC_MIXED: single-
                                 precision sweeps/O, split-bf16 S with FP32 accumulation;
                                 inverse refresh and SR solve stay double */
  int32_t refresh_every;      /* proposals (or applied updates, see refresh_unit) between
                                 full double recomputations of X^-1 (0 = only at init,
                                 set_state and parameter updates) */
  uint64_t seed;              /* Philox4x32-10 key (proposal stream and initial draw) */
  int32_t n_instances;
  const mvmc_instance_desc *inst;
  int32_t n_slots;            /* sample slots per SR step: rows of O per walker */
  int32_t solver;             /* MVMC_SOLVE_CHOL reserves the double factor; CG does not */
  int32_t build_s;            /* 1 = explicit S is built (reserves its scratch); 0 = CG only */
  int32_t sweep_threads;      /* 0 = automatic, else 64, 128 or 256 threads per walker of
                                 the kernels that keep the full X^-1 (LDS, else HBM) */
  int32_t sweep_variant;      /* 0 = automatic; 1 + v forces sweep variant v (below) for
                                 every instance (MVMC_E_SHAPE where it does not fit) */
  int32_t exchange_per64;     /* 0..64: a proposal is an exchange update (section 3.1.2,
                                 Fig. 5b) with probability exchange_per64/64, else a hop;
                                 needs the register or anti-parallel-block sweep */
  int32_t schedule;           /* MVMC_SCHED_BUCKETS: one launch per group of instances that
                                 share a sweep variant and LDS class, refresh launches at
                                 every multiple of refresh_every.  MVMC_SCHED_QUEUE: one
                                 persistent launch per mvmc_sample_sweeps call for every
                                 instance, walkers taken longest first (cost ~ N_e^2) from
                                 a device queue; the register tier (variant 0) where it
                                 fits, else the anti-parallel-block sweep with 256 threads
                                 (variant 9, N_e <= 256), both refreshing inside the launch;
                                 sweep_variant may force 1 or 10, sweep_threads must be 0 */
  int32_t refresh_unit;       /* MVMC_REFRESH_PROPOSALS: refresh_every counts proposals (the
                                 walker's counter; bit-exact across get/set_state).
                                 MVMC_REFRESH_UPDATES: it counts applied updates (accepted
                                 hops and exchanges, the only steps that change X^-1), from
                                 the context's creation or the last mvmc_set_state, which
                                 starts that count again.  A walker that reaches a multiple
                                 stops for the refresh (bucket schedule: a launch takes at
                                 most refresh_every proposals per walker, 8 refresh_every in
                                 the update unit). */
} mvmc_config;

#define MVMC_REFRESH_PROPOSALS 0
#define MVMC_REFRESH_UPDATES 1

#define MVMC_SCHED_BUCKETS 0
#define MVMC_SCHED_QUEUE 1

/* Sizes of the caller-owned buffers for a configuration. */
typedef struct {
  int64_t n_walkers;          /* total walkers */
  int64_t n_params;           /* total parameters (length of params, g, dparams) */
  int64_t eloc_elems;         /* doubles in the local-energy buffer */
  int64_t O_elems;            /* elements of O (double for FP64, float for MIXED) */
  int64_t S_elems;            /* elements of S (same type as O); 0 when build_s == 0 */
  int64_t Y_elems;            /* doubles returned by mvmc_get_inverse */
  int64_t pos_elems;          /* int16 configuration entries of mvmc_get_state */
  int64_t empty_elems;        /* int16 empty-list entries of mvmc_get_state */
  int64_t workspace_bytes;    /* device workspace, 256-byte aligned */
  int32_t O_elem_bytes;       /* 8 (FP64) or 4 (MIXED) */
  int32_t pad;
} mvmc_sizes;

/* Where instance k lives inside the caller buffers (element offsets). */
typedef struct {
  int64_t walker_off, n_walkers;   /* global walker ids [walker_off, walker_off+n_walkers) */
  int64_t param_off, n_params;     /* block of params / g / dparams */
  int64_t eloc_off;                /* eloc[eloc_off + slot*n_walkers + w] */
  int64_t O_off, O_ld;             /* O row (slot*n_walkers + w) at O_off + row*O_ld;
                                      O_ld = n_params rounded up to 64 (to 128 when
                                      n_params > 3968) */
  int64_t S_off;                   /* S block [n_params][n_params] at S_off (full square) */
  int64_t Y_off;                   /* get_inverse: walker w at Y_off + w*Y_ld; X^-1 row-major
                                      (n_elec^2 entries), or for a projected instance the
                                      N_P blocks M_p^-1 (n x n each, n = n_elec/2, block p at
                                      p*n^2, entry [b][a] at b*n + a for down electron b and
                                      up electron a: X(q_p(x))^-1[n + b][a]) */
  int64_t pos_off;                 /* get/set_state: walker w at pos_off + w*n_elec */
  int64_t empty_off;               /* get/set_state: walker w at empty_off + w*2*n_sites,
                                      [spin][n_sites], n_sites - n_sigma sites then -1 */
  int32_t n_elec, n_sites;
  int64_t Y_ld;                    /* entries per walker of get_inverse: n_elec^2, or
                                      max(n_elec^2, N_P n^2) for a projected instance */
} mvmc_instance_layout;

/* Sizes for cfg; touches no device.  Errors: MVMC_E_ARG / MVMC_E_SHAPE. */
int mvmc_query_sizes(const mvmc_config *cfg, mvmc_sizes *out);

/* Layout of instance k for cfg; touches no device. */
int mvmc_query_layout(const mvmc_config *cfg, int32_t k, mvmc_instance_layout *out);

/*
 * Create a context for psi = P_G P_J phi_AP-Pf (section 3.2; Eqs. Pf and
 * AP-Pf of section 3.2.1, the Gutzwiller and Jastrow factors of section
 * 3.2.3): copies the descriptors, lays out the workspace, expands d_params
 * (device, double, n_params) into the skew table A = F - F^T (so that
 * X_ab = A[I_a][I_b], section 3.2.1), v_ij, g_i and the RBM weights, draws a
 * uniform real-space configuration per walker (the fixed-S^z basis of
 * section 3.1.1; redrawn while X is singular) and computes X^-1, log|Pf X|
 * and its sign in double.
 * d_workspace: device memory of at least workspace_bytes, 256-byte aligned,
 * owned by the caller and untouched by anything else until mvmc_destroy.
 * hip_stream: hipStream_t (NULL = default stream).  Synchronises the stream.
 * Errors: MVMC_E_ARG, MVMC_E_SHAPE, MVMC_E_WORKSPACE (ws_bytes below
 * workspace_bytes, or d_workspace not 256-byte aligned), MVMC_E_HIP,
 * MVMC_E_NONFINITE (a NaN/Inf parameter), MVMC_E_SINGULAR (no invertible
 * initial configuration in 100 draws).  On error *out is NULL.
 */
int mvmc_init_wavefunction(mvmc_ctx **out, const mvmc_config *cfg, void *d_workspace,
                           size_t ws_bytes, const double *d_params, void *hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * context as mvmc_init_wavefunction, with the workspace taken from a static
 * array of MVMC_STATIC_WORKSPACE_BYTES in the library's device memory (one
 * per device, held until the process ends) instead of a caller buffer.  The
 * call allocates no device memory and no pinned host memory.
 * Every static context on a device shares that device's array: creating a
 * second one overwrites the first, and calls on two static contexts of one
 * device race.  The array keeps the last context's contents; this call
 * rewrites everything the context reads before use.
 * Errors: those of mvmc_init_wavefunction; MVMC_E_WORKSPACE when the
 * configuration needs more than MVMC_STATIC_WORKSPACE_BYTES (workspace_bytes
 * of mvmc_query_sizes).
 */
#define MVMC_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int mvmc_init_wavefunction_static(mvmc_ctx **out, const mvmc_config *cfg, const double *d_params,
                                  void *hip_stream);

/*
 * n_sweeps sweeps of every walker; one sweep is N_e hopping proposals
 * (section 3.1.2), each accepted with probability min(1, R^2), R = psi(x')/psi(x)
 * from a row of X^-1 and the correlator ratios, followed on acceptance by the
 * rank-2 update of X^-1.  h_accepted (may be NULL): [n_instances] accepted
 * proposals since the last call that returned them (the counters are then
 * cleared; with NULL they keep accumulating).  With h_accepted == NULL the
 * call only enqueues kernels on the context's stream, so it can be captured
 * into a HIP graph (as can mvmc_measure_energy_and_O).
 * Guard: a ratio that is not finite (NaN or Inf) triggers an immediate
 * double-precision recomputation of the walker's X^-1 and correlator state,
 * and the same proposal is tried again; if it is still not finite the walker
 * stops there (its counter stays at that proposal) until the next
 * mvmc_refresh, mvmc_set_state, mvmc_set_params or mvmc_sr_update.  Calls
 * that synchronise (this one with h_accepted, mvmc_build_sr with host
 * outputs) then return MVMC_E_NONFINITE with the instance, walker and
 * proposal in mvmc_last_error.
 * Errors: MVMC_E_ARG, MVMC_E_HIP, MVMC_E_NONFINITE (with h_accepted only).
 */
int mvmc_sample_sweeps(mvmc_ctx *ctx, int32_t n_sweeps, int64_t *h_accepted);

/* Sweep kernel variants (same proposals and decisions, different residency
 * of X^-1): 0 registers (one wavefront per walker, N_e <= 64), 1-3 the full
 * X^-1 in LDS with 64/128/256 threads per walker, 4-6 the full X^-1 in HBM
 * with 64/128/256, 7-9 the anti-parallel block alone (M^-1, n x n with
 * n = N_e/2, Eq. AP-Pf) in LDS with 64/128/256 threads: rank-1
 * Sherman-Morrison updates of M^-1 (a quarter of the state of 1-6).
 * Automatic choice: 0 where it fits, else 7-9 (threads by n), else 6.
 * mvmc_sweep_variants reports MVMC_N_SWEEP_VARIANTS for a projected instance
 * (its own sweep; the autotuner leaves it alone). */
enum { MVMC_N_SWEEP_VARIANTS = 10 };

/*
 * Autotuner for the ragged batch (section 3.1.2 sweeps, any mix of lattice
 * sizes): times n_sweeps >= 1 sweeps of every instance with each variant
 * that fits it (register tier; full-X^-1 kernel in LDS or HBM and
 * anti-parallel-block kernel, each at three thread counts), the refresh
 * launches between launches included, and keeps the
 * fastest per instance for all later calls.  The timed sweeps advance the
 * chains exactly like mvmc_sample_sweeps (they count as warm-up); the
 * accepted counters are cleared at the end.  cache_path (may be NULL): text
 * file of earlier choices, one line per (precision, N_e, N_s, M, walkers);
 * matching instances are not timed, new choices are appended.  h_ms (may be
 * NULL): [n_instances][MVMC_N_SWEEP_VARIANTS] measured milliseconds, NaN for
 * variants not timed.  Synchronises the stream; not capturable.
 * With MVMC_MIXED and build_s it also arms the tile tuner of the split-bf16
 * S build (section 3.3.1 S_km): the next mvmc_build_sr times the instances
 * with wide parameter sets (at least 512 upper-triangle tiles of 128) at
 * tile sides 128, 192 and 256 on that call's own data and keeps the fastest;
 * that call synchronises the stream.
 * With MVMC_SCHED_QUEUE the variants are fixed: MVMC_E_ARG.
 * Errors: MVMC_E_ARG, MVMC_E_HIP.
 */
int mvmc_autotune(mvmc_ctx *ctx, int32_t n_sweeps, const char *cache_path, double *h_ms);

/* Current sweep variant of every instance ([n_instances], host). */
int mvmc_sweep_variants(const mvmc_ctx *ctx, int32_t *h_variant);

/*
 * Tile side of the split-bf16 S build of every instance (h_tile,
 * [n_instances], host): 0 for the 64-tile kernel (narrow parameter sets, or
 * no split-bf16 build), else 128, 192 or 256 (default 256 until tuned or set).
 * h_ms (may be NULL): [n_instances][3] milliseconds of the last tuning at
 * sides 128, 192, 256 (NaN where not timed).
 * Errors: MVMC_E_ARG.
 */
int mvmc_s_tiles(const mvmc_ctx *ctx, int32_t *h_tile, double *h_ms);

/*
 * Sets the tile side (128, 192 or 256) of the split-bf16 S build for every
 * instance that uses the direct-to-LDS kernel (those with 64 in
 * mvmc_s_tiles are unchanged) and cancels a pending tile tuning.  S does
 * not depend on the side except in the order of FP32 partial sums.
 * Synchronises the stream.  Errors: MVMC_E_ARG, MVMC_E_HIP.
 */
int mvmc_set_s_tile(mvmc_ctx *ctx, int32_t side);

/*
 * Measurement aid for the roofline report (not a step of the method):
 * attainable throughput of the instructions the path relies on, timed on
 * register-only loops with non-zero data at two wavefronts per SIMD over
 * every compute unit.  kind: 0 bf16 MFMA 32x32x16 (FP32 accumulate),
 * 1 FP64 MFMA 16x16x4, 2 FP64 vector FMA.  d_scratch: device buffer of at
 * least mvmc_peak_probe_bytes() bytes (overwritten, caller-owned).  Runs on
 * hip_stream (NULL: the null stream) and synchronises it; *h_tflops receives
 * TFLOP/s.  Errors: MVMC_E_ARG, MVMC_E_HIP.
 */
size_t mvmc_peak_probe_bytes(void);
int mvmc_peak_probe(int32_t kind, void *d_scratch, void *hip_stream, double *h_tflops);

/*
 * Local energy E_loc(x) (Eq. MC, H of section 2.3) and the row of
 * O_k = d ln<x|psi>/d alpha_k (section 3.3.1) of every walker's current
 * configuration into sample slot `slot` (0 <= slot < n_slots):
 * d_eloc[eloc_off + slot*W + w] and O row slot*W + w (layout above); columns
 * n_params..O_ld-1 are written as zero.
 */
int mvmc_measure_energy_and_O(mvmc_ctx *ctx, int32_t slot, double *d_eloc, void *d_O);

/*
 * First-step power-Lanczos (section 3.4), local values: for every walker's
 * current configuration x, F(x, H) = E_loc(x) into d_f1 and
 * F(x, H^2) = <x|H^2|psi>/<x|psi> into d_f2 (each [eloc_elems] doubles,
 * device, caller-owned, written at eloc_off + slot*W + w like d_eloc above).
 * F(x, H^2) sums every two-step path of the Hamiltonian; the Pfaffian ratios
 * of the one- and two-electron moves come from M^-1 (Eq. AP-Pf) and its
 * products with the pair amplitudes, formed per walker in LDS in double.
 * Pfaffian-Jastrow-Gutzwiller states only: an instance with an RBM factor
 * or a quantum-number projection gives MVMC_E_ARG; MVMC_E_SHAPE where N_s, N_e do not fit the LDS budget
 * (about N_s <= 90 at half filling).  Enqueues only (capturable).
 * Errors: MVMC_E_ARG, MVMC_E_SHAPE, MVMC_E_HIP.
 */
int mvmc_measure_h2(mvmc_ctx *ctx, int32_t slot, double *d_f1, double *d_f2);

/*
 * First-step power-Lanczos (section 3.4), energy of (1 + alpha_1 H)|psi>: per
 * instance the sample means over the first n_slots_used slots
 *   h1 = <F(x,H)>, h11 = <F(x,H)^2>, h20 = <F(x,H^2)>, h12 = <F(x,H) F(x,H^2)>,
 * E_1(a) = (h1 + a (h20 + h11) + a^2 h12) / (1 + 2 a h1 + a^2 h11), and
 * alpha_1 the root of dE_1/da = 0 with the lower E_1 (0 when the quadratic
 * has no real root).  h_out (host): [n_instances][7] = h1, h11, h20, h12,
 * alpha_1, E_1(alpha_1), number of real roots.  Synchronises the stream.
 * Errors: MVMC_E_ARG, MVMC_E_HIP.
 */
int mvmc_lanczos_first_step(mvmc_ctx *ctx, int32_t n_slots_used, const double *d_f1,
                            const double *d_f2, double *h_out);

/*
 * SR quantities over the first n_slots_used slots (section 3.3.1, with the
 * sample means of section 3.3.2): E_bar = <E_loc>; o_k = <O_k>; O is centred
 * in place (O <- O - o); d_g = O~^T(E-E_bar)/N (double, n_params); d_S (may be
 * NULL) = O~^T O~ / N, both triangles of each instance block.
 * Host outputs, each [n_instances] and each may be NULL:
 *   h_E     E_bar;
 *   h_Eerr  its statistical error, the walkers being independent chains:
 *           sigma = std(walker means) / sqrt(W) with the unbiased std
 *           (NaN for a single walker);
 *   h_Evar  the sample variance <(E_loc - E_bar)^2>.
 * Any host output synchronises the stream.
 * Errors: MVMC_E_ARG (NULL buffer, n_slots_used outside [1, n_slots]),
 * MVMC_E_STATE (d_S given to a context built with build_s = 0), MVMC_E_HIP.
 */
int mvmc_build_sr(mvmc_ctx *ctx, int32_t n_slots_used, const double *d_eloc, void *d_O, void *d_S,
                  double *d_g, double *h_E, double *h_Eerr, double *h_Evar);

/*
 * Solve S_reg x = g with S_reg = S + diag(eps_rel S_kk + eps_abs) (parameters
 * with S_kk < 1e-12 frozen) by Cholesky (needs d_S from build_sr) or by CG
 * (Algorithm 1, matrix-free over the centred d_O, stop when
 * |r|^2 < cg_tol^2 |g|^2 or after cg_maxit iterations); then
 * d_params += d_dparams = -dtau x (Eq. SR_equation_system), re-expands the
 * tables and recomputes every walker's X^-1 in double.
 * Cholesky: when S_reg is not numerically positive definite (possible when S
 * has fewer samples than parameters and is built in reduced precision), the
 * shift eps_rel is raised tenfold and the factorisation repeated, at most 4
 * times, for every instance of the context.
 * h_cg_iters (may be NULL): [n_instances] CG iterations, or for the Cholesky
 * solver the number of tenfold raises of eps_rel (0: the caller's value).
 * d_dparams may be NULL.
 * Errors: MVMC_E_STATE (build_sr not called), MVMC_E_SINGULAR (Cholesky failed
 * after the raises, or a walker's X became singular), MVMC_E_NONFINITE (the
 * updated parameters hold a NaN/Inf: d_params keeps that update, the walkers
 * keep the previous tables).
 */
int mvmc_sr_update(mvmc_ctx *ctx, const void *d_S, const void *d_O, const double *d_g, double dtau,
                   double eps_rel, double eps_abs, int32_t solver, double cg_tol, int32_t cg_maxit,
                   double *d_params, double *d_dparams, int32_t *h_cg_iters);

/* Replace the parameters (device, double, n_params) and recompute every
 * walker in double (X^-1 and Pf X of section 3.2.1).  Synchronises.
 * Errors: MVMC_E_ARG, MVMC_E_NONFINITE (nothing changed),
 * MVMC_E_SINGULAR (a walker's X is singular for the new parameters). */
int mvmc_set_params(mvmc_ctx *ctx, const double *d_params);

/* Checkpoint of the Markov chains (section 3.1.1): walker configurations as
 * int16 spin-orbital indices I = i + Ns*sigma (section 3.2.1; walker w of
 * instance k at pos_off + w*n_elec, up electrons first), the Philox proposal
 * counters [n_walkers], and the per-spin lists of empty sites in the order
 * the hopping proposals index them (they are reordered as the chain moves;
 * layout at empty_off, pos_elems / empty_elems entries in all).  Device
 * buffers, caller-owned; any may be NULL.  Enqueued only. */
int mvmc_get_state(mvmc_ctx *ctx, int16_t *d_pos, uint64_t *d_counter, int16_t *d_empty);

/* Resume from a checkpoint: load configurations (int16, layout of
 * mvmc_get_state), counters (equal within an instance) and, when d_empty is
 * not NULL, the empty-site lists (each must list exactly the empty sites of
 * its spin); with d_empty NULL the lists are rebuilt in ascending order.
 * Every walker is then recomputed in double.  With the lists given, the
 * chains continue bit for bit as a context that called mvmc_refresh at the
 * checkpoint would.  Synchronises.
 * Errors: MVMC_E_ARG (bad configuration, counters or lists; state
 * unchanged), MVMC_E_SINGULAR (a loaded X is singular), MVMC_E_HIP. */
int mvmc_set_state(mvmc_ctx *ctx, const int16_t *d_pos, const uint64_t *d_counter,
                   const int16_t *d_empty);

/* Every walker's current X^-1 as double (Y_elems, layout above; the N_P
 * inverses M_p^-1 for a projected instance). */
int mvmc_get_inverse(mvmc_ctx *ctx, double *d_Y);

/* log|Pf(X)| and sign of every walker from the last full recomputation
 * (log|sum_p w_p Pf(X(q_p(x)))| and its sign for a projected instance, kept
 * current by its sweep). */
int mvmc_get_pfaffian(mvmc_ctx *ctx, double *d_logabs, double *d_sign);

/* Full double recomputation of every walker now (X^-1, log|Pf X| and sign,
 * section 3.2.1; Jastrow field and RBM angles); clears the non-finite
 * guard.  Synchronises.  Errors: MVMC_E_SINGULAR, MVMC_E_HIP. */
int mvmc_refresh(mvmc_ctx *ctx);

/*
 * Record every proposal into d_trace (40-byte records
 * {int64 n; int32 walker; int32 a; int32 i_new; int32 accepted; double ratio;
 *  int32 b; int32 pad}: a the moved electron (the up one of an exchange),
 * i_new its proposed spin-orbital (-1 when no move was possible), b the down
 * electron of an exchange (-1 for a hop)); the record for proposal n of
 * walker w at w*capacity + (n - n_at_enable).  d_trace NULL or capacity 0
 * disables.
 */
int mvmc_trace_enable(mvmc_ctx *ctx, void *d_trace, int64_t per_walker_capacity);

/*
 * Kernel timing with HIP events on the context's stream.  enable = 1 starts
 * (and clears) collection, 0 stops; when h_ms/h_calls are not NULL the
 * totals so far are returned for categories
 * [0 sweep, 1 refresh, 2 measure, 3 SR statistics, 4 S build, 5 SR solve].
 */
int mvmc_timing(mvmc_ctx *ctx, int32_t enable, double *h_ms, int64_t *h_calls);

int mvmc_destroy(mvmc_ctx *ctx);
const char *mvmc_last_error(const mvmc_ctx *ctx);
const char *mvmc_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* MVMC_H */
