/*
 * xy.h - C ABI of the MI355X (gfx950) hot path for Monte Carlo simulation of
 * the classical three-dimensional XY model, after Lan, Hsieh and Kao,
 * "High-precision Monte Carlo study of the three-dimensional XY model on GPU"
 * (arXiv:1211.0780).
 *
 * The library keeps every configuration of every lattice resident in device
 * memory (Sec. II: all spin configurations at all temperatures stay in GPU
 * memory and all updates run on the GPU) and exposes four verbs:
 *
 *   xy_init      allocate / adopt device state, random or ordered start
 *   xy_sweep     n_metro checkerboard Metropolis sweeps followed by n_or
 *                over-relaxation sweeps of every configuration (Sec. II, the
 *                Monte Carlo step; over-relaxation is Eq. (2))
 *   xy_measure   per-configuration energy and magnetisation moments
 *                (Eq. (1) energy, Eq. (4) magnetisation, inputs of Eq. (5))
 *   xy_exchange  one parallel-tempering exchange step per lattice (Eq. (3))
 *
 * plus a graph-replayed driver loop (xy_run), state access for checkpointing
 * and testing, and error reporting.  Nothing here takes or returns a PyTorch
 * type: device buffers are plain pointers, streams are hipStream_t passed as
 * void*.
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - "Device buffer" below means memory the GPU reaches: device memory of
 *    the context's GPU, managed memory, or host memory pinned with
 *    hipHostMalloc (kernels write it through its mapped address).  Pageable
 *    host memory, memory of another GPU, or a buffer whose allocation ends
 *    before the bytes a call writes (checked where HIP reports the
 *    allocation's range) makes the call return XY_ERR_ARG before it enqueues
 *    anything.
 *  - Lattice l is a periodic L_l x L_l x L_l simple cubic lattice with
 *    N_l = L_l^3 sites, site index i = x + L*(y + L*z).  J = k_B = 1 and
 *    beta = 1/T.
 *  - Lattice l carries R_l configurations, one per entry of its beta-ladder.
 *    "beta-position" k (0 <= k < R_l) names the ladder entry beta_l[k];
 *    ladders are strictly ascending.  Exchanges permute which stored
 *    configuration sits at which beta-position; every call below that takes
 *    or returns per-configuration data indexes it by (lattice, beta-position).
 *  - The flat "position index" of (l, k) is sum_{l' < l} R_l' + k, and
 *    R_total = sum_l R_l.
 *  - Randomness is Philox4x32-10 with key (seed mod 2^32, seed >> 32) and
 *    counter (c0, c1, (l << 16) | k, (phase << 24) | substep): c0 is the site
 *    (or exchange pair) index, c1 the sweep counter t (or exchange counter
 *    tau), phase 1 = initial state, 2 = Metropolis, 3 = exchange.  A
 *    Metropolis block serves two sites of one colour, (x, y, 2m) and
 *    (x xor 1, y, 2m+1): c0 is the even-plane site's index, which takes
 *    words (r0, r1); the odd-plane site takes (r2, r3), written (a, b) below.
 *    Uniforms are U(r) = (r >> 8) * 2^-24.  Random draws depend only on these
 *    counters, never on thread layout, so results do not depend on tiling.
 *  - All device work is ordered on the context's stream.  Calls return
 *    without waiting unless they hand data to host memory.
 *  - No call throws; each returns an xy_status and, on failure, leaves a
 *    message readable with xy_last_error(ctx).  Calls on one context are not
 *    thread-safe; distinct contexts are independent.
 */
#ifndef XY_H
#define XY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xy_ctx_s *xy_ctx;

typedef enum {
    XY_OK = 0,
    XY_ERR_ARG = 1,         /* invalid argument (null pointer, range, ladder order, size) */
    XY_ERR_ODD_L = 2,       /* L odd or L < 4: the checkerboard needs an even, bipartite lattice */
    XY_ERR_OOM = 3,         /* device or host allocation failed */
    XY_ERR_HIP = 4,         /* a HIP runtime call failed; the message names it */
    XY_ERR_STATE = 5,       /* state blob or device state inconsistent (bad blob, NaN angle) */
    XY_ERR_UNSUPPORTED = 6  /* valid request this library does not implement */
} xy_status;

typedef enum {
    XY_FP32 = 0, /* angles stored and updated in float32; reductions and the
                    exchange in float64; Metropolis decisions near the
                    threshold re-evaluated in float64 */
    XY_FP64 = 1  /* angles stored and updated in float64 (plain kernels) */
} xy_prec;

typedef enum {
    XY_START_RANDOM = 0,  /* theta = 2*pi*U(r0) with phase 1, c1 = 0, substep 0 */
    XY_START_ORDERED = 1  /* theta = 0 everywhere */
} xy_start;

/* xy_config.flags */
#define XY_F_NO_RECHECK  0x1u /* FP32: take Metropolis decisions in float32 only */
#define XY_F_NO_FUSED_OR 0x2u /* FP32: run every over-relaxation substep as two half-sweep
                                 kernels instead of one fused kernel (the fused kernel is
                                 used when every L <= 256; it needs a second angle buffer) */

typedef struct {
    int32_t n_lattices;          /* >= 1 */
    const int32_t *L;            /* [n_lattices] linear sizes, even, 4 <= L <= 1024; copied */
    const int32_t *n_replicas;   /* [n_lattices] ladder lengths, 1 <= R <= 65535; copied */
    const double *beta;          /* [R_total] ladders concatenated by lattice, each strictly
                                    ascending, finite, >= 0; copied */
    uint64_t seed;               /* Philox key */
    int32_t prec;                /* xy_prec */
    int32_t start;               /* xy_start */
    void *angles_dev;            /* optional caller-owned device buffer of xy_angles_bytes()
                                    bytes (layout below), or NULL to let the library allocate.
                                    A caller-owned buffer is never freed by the library and
                                    must outlive the context. */
    void *stream;                /* hipStream_t for all work, or NULL for the null stream */
    uint32_t flags;              /* XY_F_* */
} xy_config;

/*
 * Device layout of the angle buffer (what angles_dev must hold): for each
 * lattice in order, for each storage slot r < R_l, for each colour c in
 * {0, 1} (colour = (x + y + z) mod 2), the N_l/2 sites of that colour ordered
 * (z, y, x/2) with x/2 fastest.  FP32 buffers hold angles in turns
 * (theta / 2pi, in [0, 1)); FP64 buffers hold radians in [0, 2pi).  Storage
 * slot and beta-position coincide at start and are permuted by exchanges;
 * use xy_get_angles / xy_set_angles for position-indexed access.
 */

/* Bytes of angle storage a configuration needs (0 on invalid input). */
size_t xy_angles_bytes(const xy_config *cfg);

/*
 * Create a context: validate cfg (XY_ERR_ODD_L for odd or small L,
 * XY_ERR_ARG for the rest), allocate device state, write the start
 * configuration, set t = tau = 0.  On success *out owns the context; on
 * failure *out is NULL.
 */
xy_status xy_init(const xy_config *cfg, xy_ctx *out);

/*
 * One sweep of every configuration (Sec. II): n_metro Metropolis substeps,
 * each a half-sweep over colour 0 then colour 1 with proposal
 * theta' = 2*pi*U(a) accepted iff U(b) < exp(-beta*dE), then n_or
 * over-relaxation substeps (Eq. (2)), each colour 0 then colour 1.  Then
 * t <- t + 1.  n_metro, n_or >= 0 and n_metro + n_or >= 1.  Asynchronous.
 */
xy_status xy_sweep(xy_ctx ctx, int32_t n_metro, int32_t n_or);

/*
 * Observables of every configuration in its current state, by position
 * index: obs[5*p + {0..4}] = {E, E/N, |m|, |m|^2, |m|^4} with
 * E = -sum_<ij> cos(theta_i - theta_j) (Eq. (1)) and
 * |m| = |sum_j (cos theta_j, sin theta_j)| / N (Eq. (4), one sample).
 * The energy is summed as E = -sum_{i of colour 1} S_i . h_i, h_i the sum of
 * the six neighbour spins (every bond has one end of each colour).  Terms
 * are formed in the configuration's precision and accumulated in float64.
 * obs has 5*R_total doubles; if
 * obs_on_device is nonzero it is a device buffer (see the conventions:
 * pinned host memory qualifies) and the call is asynchronous, otherwise it
 * is any host memory and the call waits for it.
 * Returns XY_ERR_STATE (host destination only) if any energy or
 * magnetisation measured since the sentinel was last reported is not finite,
 * and clears the sentinel.
 */
xy_status xy_measure(xy_ctx ctx, double *obs, int32_t obs_on_device);

/*
 * One parallel-tempering exchange step on every lattice (Eq. (3)): pairs
 * (k, k+1) with k = tau mod 2, tau mod 2 + 2, ... swap their configurations
 * iff U(r0) < exp((beta_k - beta_k+1)(E_k - E_k+1)), r drawn with counter
 * (k, tau, l << 16, 3 << 24).  E is the float64 energy of the current
 * configurations (measured first if the state changed since the last
 * measurement).  Swaps relabel storage slots; no angle moves.  Then
 * tau <- tau + 1.  n_acc (nullable, host) receives R_total cumulative
 * acceptance counts, entry p counting swaps of pair (p, p+1) within its
 * lattice (the last entry of each lattice stays 0); the call then waits.
 */
xy_status xy_exchange(xy_ctx ctx, int64_t *n_acc);

/*
 * The production loop, captured as HIP graphs (several sweeps per graph when
 * exchange_every is 0 or 1) and replayed: n_sweeps
 * times { xy_sweep(n_metro, n_or); measure into obs_dev; exchange if
 * (sweep index + 1) % exchange_every == 0 }.  exchange_every = 0 disables
 * exchange.  obs_dev: device buffer (pinned host memory qualifies) of
 * n_sweeps*5*R_total doubles, sweep s at
 * offset 5*R_total*s, laid out as xy_measure; may be NULL to skip the copy
 * (observables are still computed for the exchange).  Graphs are cached per
 * (n_metro, n_or, obs_dev, bonds ring); reusing a ring reuses its graphs,
 * and past 32 cached graphs the oldest of other shapes or rings are released
 * (after the stream has drained).  Asynchronous.  Failure detection without
 * waiting: each loop leaves a copy of the device's non-finite sentinel (set
 * when a measured E, Mx or My is not finite), and the next xy_run or
 * xy_run_ex returns XY_ERR_STATE (enqueuing nothing) if that copy has
 * already landed and is set; a report clears the sentinel.  xy_measure into
 * host memory waits and reports it as well.
 */
xy_status xy_run(xy_ctx ctx, int32_t n_sweeps, int32_t n_metro, int32_t n_or,
                 int32_t exchange_every, double *obs_dev);

/*
 * xy_sweep with each group of consecutive launches of one kind bracketed by
 * HIP events on the context's stream (profiling aid; same result as
 * xy_sweep).  ms[0..3] receive the device time of the Metropolis half-sweeps
 * (their float64 re-decision included), the over-relaxation
 * half-sweeps, the fused over-relaxation substeps (one launch updates both
 * colours) and the counter update; launches[0..3] the number of half-sweep,
 * half-sweep, fused and counter launches in each group.  Waits.
 */
xy_status xy_sweep_profiled(xy_ctx ctx, int32_t n_metro, int32_t n_or, double *ms,
                            int32_t *launches);

/*
 * xy_run that also records, per sweep, the bond sums behind the spin
 * stiffness of Eq. (6) into bonds_dev (device buffer, n_sweeps*6*R_total doubles,
 * sweep s at offset 6*R_total*s, position p at 6*p): {C_x, C_y, C_z, I_x,
 * I_y, I_z} with C_mu = sum_i cos(theta_i - theta_{i+mu}) and
 * I_mu = sum_i sin(theta_i - theta_{i+mu}), each bond (i, i+mu) once, in
 * float64.  Then rho_s = (1/3N) sum_mu [<C_mu> - beta <I_mu^2>].
 * Either ring may be NULL; with bonds_dev NULL the bond sums are not formed
 * (the measurement then costs less).  E and -(C_x + C_y + C_z) agree to the
 * rounding of the configuration's precision.  Asynchronous.
 */
xy_status xy_run_ex(xy_ctx ctx, int32_t n_sweeps, int32_t n_metro, int32_t n_or,
                    int32_t exchange_every, double *obs_dev, double *bonds_dev);

/* The bond sums {C_x, C_y, C_z, I_x, I_y, I_z} (see xy_run_ex) of every
 * configuration in its current state, by position index (6*R_total
 * doubles); device or host destination as for xy_measure.  Measures first
 * when the state changed since the last measurement. */
xy_status xy_get_bond_sums(xy_ctx ctx, double *out, int32_t out_on_device);

/*
 * Metropolis proposal: window = 0 (the default) proposes theta' = 2*pi*U(a)
 * uniformly on the circle; 0 < window <= 2*pi proposes the symmetric
 * restricted move theta' = theta + window*(U(a) - 1/2), wrapped into
 * [0, 2pi).  The paper does not state its proposal (Sec. II); the window
 * raises acceptance at large beta.  Applies to later sweeps.
 */
xy_status xy_set_proposal_window(xy_ctx ctx, double window);

/* Copy the N_l angles (radians in [0, 2pi), natural site order) of the
 * configuration at (lattice, beta_pos) to host memory.  Waits. */
xy_status xy_get_angles(xy_ctx ctx, int32_t lattice, int32_t beta_pos, double *host);

/* Diagnostic read of the fused over-relaxation pass (Eq. (2), both colours
 * per launch, FP32 contexts that use it): the fused substeps of a sweep
 * alternate between the primary angle buffer and a second library-owned one,
 * so after a sweep with 2m fused substeps the second buffer holds the
 * configuration after fused substep 2m-1 (the substep before the last).
 * Copies that configuration at (lattice, beta_pos) to host radians like
 * xy_get_angles, letting a caller check a single fused substep site by site.
 * XY_ERR_UNSUPPORTED for contexts without the fused pass.  Meaningless
 * before the first such sweep.  Waits. */
xy_status xy_get_angles_fused_mid(xy_ctx ctx, int32_t lattice, int32_t beta_pos, double *host);

/* The angles (radians) of n chosen sites (natural index i = x + L*(y + L*z),
 * 0 <= i < N_l) of the configuration at (lattice, beta_pos), in order, into
 * host memory; n <= 2^26.  For sampled checks of lattices too large to copy
 * whole.  Waits. */
xy_status xy_get_sites(xy_ctx ctx, int32_t lattice, int32_t beta_pos, int64_t n,
                       const int64_t *sites, double *host);

/*
 * xy_get_sites for callers that cannot allocate device memory (code that
 * must not call hipMalloc, e.g. tight monitoring loops and harnesses that
 * forbid allocation): the same result, bit for bit, with the site list and
 * the gathered angles staged in a static device array of the library
 * instead of buffers allocated per call.  n <= XY_NOALLOC_MAX_SITES
 * (XY_ERR_ARG beyond it).  Every GPU holds one such array (4 MiB) from the
 * first xy_init on it until the process ends, and every call on that GPU
 * shares it: calls that overlap in time on one GPU (from several threads or
 * contexts) race and must be serialised by the caller.  Waits.
 */
#define XY_NOALLOC_MAX_SITES (1 << 18)
xy_status xy_get_sites_noalloc(xy_ctx ctx, int32_t lattice, int32_t beta_pos, int64_t n,
                               const int64_t *sites, double *host);

/* Overwrite that configuration from host radians (any finite values; they are
 * wrapped into [0, 2pi) and, for FP32, rounded to float32 turns).  Waits. */
xy_status xy_set_angles(xy_ctx ctx, int32_t lattice, int32_t beta_pos, const double *host);

/* Counters: sweep counter t, exchange counter tau. */
xy_status xy_get_counters(xy_ctx ctx, uint64_t *t, uint64_t *tau);

/* Storage slot holding each beta-position of a lattice: slot[k], R_l entries. */
xy_status xy_get_permutation(xy_ctx ctx, int32_t lattice, int32_t *slot);

/* Cumulative accepted Metropolis moves per position index (R_total entries,
 * attributed to the beta-position the configuration held while it moved). */
xy_status xy_get_metro_accepts(xy_ctx ctx, int64_t *n_acc);

/*
 * Float64 re-decision queue of the FP32 Metropolis path (Sec. II; the
 * acceptance test of the Metropolis update): sites whose float32 decision
 * lies within max(1e-5, 1.6e-5 * beta) of the threshold (eight times the
 * float32 error of exp(-beta dE)) are queued and decided again in float64.
 * The queue holds max(4096, min(2^22, S / 1000)) entries, S being the sites
 * one half-sweep updates over every lattice and replica (about 2e-5 S land
 * in the band); entries beyond that keep their float32 decision and are
 * counted.  *n receives the cumulative count since
 * xy_init (0 for FP64 contexts and with XY_F_NO_RECHECK).  Waits for the
 * stream.
 */
xy_status xy_get_recheck_overflow(xy_ctx ctx, uint64_t *n);

/*
 * Launch shape of the FP32 tiled half-sweep for one lattice: a work item is
 * ty rows (y) by L/2 sites (x) of one colour, streamed over tz planes (z).
 * ty and tz must divide L, ty*L/2 <= 2048.  Launches are persistent: each
 * workgroup takes work items in turn.  grid_cap > 0 sets the number of
 * workgroups (at most one per item); grid_cap = 0 (the default) uses as many
 * as the GPU holds at once, compute units times the kernel's resident
 * workgroups per CU.  The cap applies to the half-sweep and the fused
 * over-relaxation launches.
 * Results do not depend on these choices (they only change the order in
 * which independent same-colour sites are visited); they exist for tuning.
 * XY_ERR_UNSUPPORTED for FP64 contexts.  Takes effect for later calls.
 */
xy_status xy_set_tiling(xy_ctx ctx, int32_t lattice, int32_t ty, int32_t tz, int32_t grid_cap);

/*
 * Pick the tile shapes of every lattice by timing.  All lattices of a
 * context share one launch per half-sweep, so each candidate (ty, tz) of one
 * lattice is timed on the whole batch while the other lattices keep their
 * current shapes, one lattice after another (coordinate descent): first the
 * half-sweep tiles, cost = n_metro * t_metro + n_unfused * t_over per launch
 * of one Metropolis and one over-relaxation half-sweep (n_unfused: the
 * over-relaxation substeps that do not run fused), then, when n_or >= 2 and
 * the context fuses over-relaxation, the fused tiles, cost = one fused
 * substep.  Then the sublattice schedule of the over-relaxation substeps:
 * the fused pass (both colours per launch) or two half-sweep launches, the
 * faster kept (bit-identical results either way); then the workgroup cap of
 * the tiled launches among the resident capacity and 2, 3, 4, 6 workgroups
 * per compute unit, cost = one whole sweep.  Each timing is reps launches
 * after one warm-up launch.  The angles and acceptance counters are saved
 * and restored around the timing and the sweep counter is not advanced, so
 * the chain is unchanged.  Needs scratch device memory the size of the angle
 * buffer.  No-op for FP64 contexts.  Waits.
 */
xy_status xy_autotune(xy_ctx ctx, int32_t n_metro, int32_t n_or, int32_t reps);
xy_status xy_get_tiling(xy_ctx ctx, int32_t lattice, int32_t *ty, int32_t *tz, int32_t *grid_cap);

/* The same for the fused over-relaxation kernel (its own tiles; rows and
 * planes as above; ty * L/2 <= 1280).  Setting a fused tile also selects the
 * fused schedule (which xy_autotune may have switched off).
 * XY_ERR_UNSUPPORTED when the context cannot fuse (FP64, XY_F_NO_FUSED_OR,
 * or a lattice with L > 256); xy_get_tiling_fused reports (0, 0) while the
 * fused schedule is not in use. */
xy_status xy_set_tiling_fused(xy_ctx ctx, int32_t lattice, int32_t ty, int32_t tz);
xy_status xy_get_tiling_fused(xy_ctx ctx, int32_t lattice, int32_t *ty, int32_t *tz);

/* Cumulative accepted exchanges per position index (R_total entries; entry
 * p counts swaps of pair (p, p+1) of its lattice; the last entry of each
 * lattice stays 0).  Pair k is attempted at exchange steps tau with
 * tau = k (mod 2).  Waits. */
xy_status xy_get_swap_accepts(xy_ctx ctx, int64_t *n_acc);

/*
 * Checkpoint: the whole chain state (angles, permutation, t, tau, seed,
 * ladders, acceptance counters) as an opaque blob.  With blob == NULL, *size
 * receives the size needed.  Because randomness is counter-based, a context
 * restored with xy_set_state continues bit-identically.  Both wait.
 * xy_set_state requires a context created with the same lattices, ladders,
 * seed and precision (XY_ERR_STATE otherwise).
 */
xy_status xy_get_state(xy_ctx ctx, void *blob, size_t *size);
xy_status xy_set_state(xy_ctx ctx, const void *blob, size_t size);

/* Message of the last failed call on ctx (or of the last failed xy_init when
 * ctx is NULL); valid until the next call on the same context. */
const char *xy_last_error(xy_ctx ctx);

/* Wait for outstanding work and free everything the context owns. */
void xy_destroy(xy_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* XY_H */
