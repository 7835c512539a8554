/*
 * gsbs.h -- C ABI of the MI355X step-by-step (SBS) diffusion-reaction engine
 * for water-radiolysis species in periodic cubes.
 *
 * The method (arXiv 2509.03313, "Advancements in Monte Carlo simulations with
 * gMicroMC ..."): molecules of the chemical stage make Brownian jumps, re-enter
 * the cube through the opposite face (PBC 1, Eq. 1), and react with a partner
 * found through the minimum image (PBC 2, Eq. 2) when the pair comes within the
 * reaction radius R derived from the rate constants of Table 1 (supplement,
 * reaction-radius derivation; 2k for self-recombination).  Fresh molecules
 * are injected at the times radiation events arrive (Sec. "Workflow of
 * gMicroMC extension"); species counts give G-values (molecules per 100 eV).
 *
 * Units: nm, ns, nm^2/ns (= 1e-9 m^2/s), rate constants in 1e10 L/mol/s.
 *
 * Conventions
 *   - Every function returns 0 (GSBS_OK) or a negative GSBS_E* code; the
 *     message of the last failure on the calling thread is gsbs_last_error().
 *   - Host arrays passed in are read during the call only; the caller keeps
 *     ownership.  Device arrays passed in (flag device_ptrs) are read in
 *     stream order on the context's stream and must stay valid until the
 *     next synchronising call (gsbs_advance_to, gsbs_get_*, gsbs_sync).
 *   - The context owns every device allocation it makes and frees them in
 *     gsbs_destroy.  All work runs on the HIP stream given to gsbs_create.
 *   - One context is used by one host thread at a time.
 *   - Instances are independent periodic cubes simulated together: instance
 *     i uses the Philox4x64-10 key (seed, i).
 */
#ifndef GSBS_H
#define GSBS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSBS_OK 0
#define GSBS_EINVAL (-1)     /* bad argument */
#define GSBS_ESTATE (-2)     /* call not valid now (e.g. time before the present) */
#define GSBS_EMINIMAGE (-3)  /* reaction radius or cutoff too large for the cube */
#define GSBS_ECAPACITY (-4)  /* molecule, pair or cell capacity exceeded */
#define GSBS_EHIP (-5)       /* HIP runtime error, or a device-side stall (cell-scan look-back) */
#define GSBS_ENOMEM (-6)     /* host or device allocation failed */

#define GSBS_MAX_SPECIES 16
#define GSBS_MAX_REACTIONS 32

typedef struct gsbs_ctx gsbs_ctx;

/* One periodic cube. */
typedef struct {
    double L_nm;          /* edge length; positions live in [-L/2, L/2)^3 */
    int64_t capacity;     /* molecules this instance may hold at once (0: grow on demand) */
} gsbs_box;

/* One reaction of Table 1: a + b -> products. */
typedef struct {
    int32_t a, b;            /* reactant species indices */
    double k_in;             /* rate constant as printed (for a == b the printed 2k) */
    int32_t n_products;      /* 0..3 */
    int32_t products[3];     /* species of the products */
    int32_t keep_b;          /* 1: the reactant of species b survives unchanged (sink, tests) */
} gsbs_reaction;

/* Method and schedule parameters (gsbs_default_params fills the defaults). */
typedef struct {
    double c_cut;            /* candidate cutoff r_c = R + c_cut * sqrt(2 D_AB dt); 5 */
    int32_t rounds;          /* mutual-best partner matching rounds per step; 4 */
    int32_t contact_only;    /* 1: react only pairs within R at the start or end of a step */
    double dt0_ns;           /* first step end after an injection; 1e-3 */
    double ratio;            /* step end times after an injection: dt0 * ratio^j; 10^(6/1999) */
    double dt_max_ns;        /* cap of a step; 0 = largest step keeping every r_c below L/2 */
    int32_t grid_config;     /* -1: search grid chosen per step by the autotuner (default);
                                k >= 0: always grid configuration k (see gsbs_get_tuning) */
    int32_t autotune;        /* 1: try untried configurations on live steps (default); 0: use
                                the process-wide table as it is, defaults where it is empty */
    int32_t search_split;    /* species-bin search: slices of each partner stream, one wave
                                each; 0 = chosen from the work per box (default), 1..16 */
    int32_t search_box;      /* species-bin search: edge in cells of the box of molecules a
                                wave holds; 0 = chosen per species (default), 1..8 */
    int32_t step_graph;      /* 1: the launches of each uploaded chunk of steps (up to the next
                                injection) are captured into a HIP graph and launched as one;
                                0: launched one by one (default).  Off while profiling, while
                                the autotuner explores, and on the null stream (which cannot be
                                captured).  Results are identical either way. */
} gsbs_params;

/* Counters since the context was created. */
typedef struct {
    int64_t steps;           /* global steps launched */
    int64_t molecule_steps;  /* sum over active instances and steps of the live molecules */
    int64_t reactions;       /* reactions performed */
    int64_t pair_candidates; /* candidate pairs tested (end separation below r_c) */
    int64_t max_live;        /* largest live count seen at a synchronisation point */
} gsbs_stats;

/* ---------------------------------------------------------------- setup --- */

/* Fill p with the defaults listed above.  Host only. */
int gsbs_default_params(gsbs_params* p);

/* Create a context of n_instances cubes (boxes[i]) on `stream` (a hipStream_t,
 * NULL for the null stream) of the current HIP device.  seed keys every Philox
 * stream.  *out receives the context. */
int gsbs_create(const gsbs_box* boxes, int32_t n_instances, uint64_t seed, void* stream,
                gsbs_ctx** out);

/* Free the context and all its device memory. NULL is accepted. */
int gsbs_destroy(gsbs_ctx* ctx);

/* Message of the last failure on this thread (never NULL). */
const char* gsbs_last_error(void);

/* Species diffusion coefficients D[0..n) in nm^2/ns (Table S2), n <= 16. Must be
 * called before the first injection. */
int gsbs_set_species(gsbs_ctx* ctx, int32_t n, const double* D);

/* Reactions (Table 1), n <= 32, at most one reaction per unordered species pair.
 * The engine derives each radius from the steady state of the supplement's
 * k_diff(t): R = k_in / (4 pi (D_a + D_b) N_A).  Fails with GSBS_EMINIMAGE if
 * 2R >= L for some cube (PBC 2). */
int gsbs_set_reactions(gsbs_ctx* ctx, int32_t n, const gsbs_reaction* r);

/* A first-order channel: a molecule of species a turns into its products at
 * k_per_ns per ns (scavenging by a solute held at a fixed concentration,
 * e.g. e_aq + O2 at k [O2]).  An extension of Table 1. */
typedef struct {
    int32_t a;
    int32_t n_products; /* 0..2: 0 removes the molecule */
    int32_t products[2];
    double k_per_ns;
} gsbs_first_order;

/* Replace the first-order channels (at most one per species; 0 clears them).
 * SBS: after each step's pair reactions, every molecule that took part in the
 * step and is not one of its products converts with probability
 * 1 - exp(-k dt), decided by the top 24 bits k24 of Philox word 0 at counter
 * (uid, step, 3, 0): converts iff (2 k24 + 1) 2^-25 < p; product 1 keeps the
 * molecule's place and uid, product 2 appears at the same point with uid
 * = word 1 | 2^63.  Rate equations: k [a]; Gillespie runs: propensity k n_a,
 * after the reactions and before the sources, in species order.  Fails with
 * GSBS_EINVAL for a species outside the table, two channels of one species,
 * a rate <= 0 or not finite, or more than two products; GSBS_ESTATE before
 * gsbs_set_species. */
int gsbs_set_first_order(gsbs_ctx* ctx, int32_t n, const gsbs_first_order* ch);

/* A zero-order reaction: its products appear at rate_M_per_ns mol/L/ns
 * anywhere in the volume.  Extension of Table 1, which prints R9 as an
 * equilibrium: R9's reverse, the water autoionisation H2O -> H3O+ + OH- at
 * k9 Kw, keeps [H3O+][OH-] at Kw (pH 7 water). */
typedef struct {
    double rate_M_per_ns;
    int32_t n_products; /* 1..3 */
    int32_t products[3];
} gsbs_source;

/* Replace the zero-order sources (n <= 4; 0 clears them).  They act in the
 * homogeneous solvers (gsbs_numodes, gsbs_ssa); the SBS steps of
 * gsbs_advance_to do not create molecules from them.  Fails with GSBS_EINVAL
 * for a negative or non-finite rate or a product outside the species table,
 * GSBS_ESTATE before gsbs_set_species. */
int gsbs_set_sources(gsbs_ctx* ctx, int32_t n, const gsbs_source* src);

/* Replace the method parameters.  The search fields (grid_config, autotune,
 * search_split, search_box) and step_graph change only speed, never a result,
 * and may change between advances; the others before the first one. */
int gsbs_set_params(gsbs_ctx* ctx, const gsbs_params* p);

/* Reaction radii R[0..n_reactions) in nm. */
int gsbs_get_radii(gsbs_ctx* ctx, double* R);

/* Largest step of instance inst (ns) after the params' cap is applied. */
int gsbs_get_dt_max(gsbs_ctx* ctx, int32_t inst, double* dt);

/* ------------------------------------------------------------- injection --- */

/* Queue n molecules for instance inst at time t_ns (>= the instance's time).
 * xyz: n x 3 float32 positions inside [-L/2, L/2)^3; species: n uint8.  With
 * device_ptrs = 1 both arrays are device pointers, else host pointers.  The
 * molecules enter at the step boundary at t_ns (every injection time is a
 * step boundary and restarts the step ramp), get uids in array order from the
 * instance's counter, and add edep_eV to the deposited energy used by the
 * G-values.  The arrays are copied before the call returns (device arrays in
 * stream order). */
int gsbs_inject(gsbs_ctx* ctx, int32_t inst, double t_ns, int64_t n, const float* xyz,
                const uint8_t* species, double edep_eV, int32_t device_ptrs);

/* A pulse generated on the device from a counter-based spur model (the input
 * side: it stands in for the paper's physical and physico-chemical stages).
 * n_tracks straight tracks parallel to z through the cube; along each, spur
 * centres at exponential spacing (mean spacing_nm), a Poisson number of
 * molecules per spur (mean mol_per_spur, at most 30; at most 64 drawn), the
 * species from frac[0..n_species-1] (>= 0, summing to 1), Gaussian offsets of
 * sigma_nm per axis.  Draws: Philox4x64-10, key (the context seed,
 * 0x53505552534D4F44), u = (top 53 bits + 1/2) 2^-53; track k: block
 * (stream, k, 0, 0), x = -L/2 + L u0, y = -L/2 + L u1; spur j: block
 * (stream, k, j+1, 0), z_j = z_{j-1} - spacing ln u0 from z = -L/2 until
 * z_j >= L/2, count by inverting the Poisson CDF at u1; molecule m: block
 * (stream, k, j+1, 2m+1) for the offsets sigma sqrt(-2 ln u0)(cos, sin)(2 pi
 * u1) on x, y and sigma sqrt(-2 ln u2) cos(2 pi u3) on z, block
 * (stream, k, j+1, 2m+2) for the species (first s with u0 below the running
 * sum of the fractions).  FP64, wrapped into the cube, stored as FP32.  The
 * molecules are queued like gsbs_inject's at t_ns, with deposited energy
 * n_tracks * L * let_kev_per_um eV; *n_injected (may be NULL) receives their
 * number.  Fails with GSBS_EINVAL for bad parameters, GSBS_ESTATE for a time
 * before the instance's present or before the species are set. */
typedef struct {
    double t_ns;
    int32_t n_tracks;
    int32_t reserved;
    double spacing_nm;
    double mol_per_spur;
    double sigma_nm;
    double let_kev_per_um;
    uint64_t stream;
    double frac[16];
} gsbs_pulse;

int gsbs_inject_pulse(gsbs_ctx* ctx, int32_t inst, const gsbs_pulse* pulse, int64_t* n_injected);

/* Record times of instance inst (ns, ascending); counts are taken at each
 * record time after that boundary's injection.  Replaces earlier records. */
int gsbs_set_records(gsbs_ctx* ctx, int32_t inst, int32_t n, const double* t_ns);

/* ---------------------------------------------------------------- advance --- */

#define GSBS_PLAIN 0      /* every interval by SBS steps */
#define GSBS_SURROGATE 1  /* inter-pulse intervals by the network where its error estimate allows */

/* Advance every instance i to t_target[i] (>= its current time) by SBS steps:
 * Brownian jump + PBC 1, cell binning, minimum-image candidate search, radial
 * Brownian-bridge contact probability, mutual-best single-partner matching,
 * products.  Returns after the device work has completed.
 *
 * mode GSBS_SURROGATE (after gsbs_set_surrogate) replaces the long
 * homogeneous evolution between pulses (the paper's beam-off stage, Eq. 3-4)
 * by the network where its held-out error estimate allows.  A hand-over
 * point of an instance is settle_ns after one of its injections at a_k when
 * its next injection a_(k+1) comes later than a_k + settle_ns + min_gap_ns;
 * there the instance stops, its features are computed (gsbs_features with the
 * configuration's mu, sd), and the interval [a_k + settle_ns, a_(k+1)] is
 * handed to the network when
 *   - the table entry of its bin (log10 of the interval length in ns, log10 of
 *     the total concentration in mol/L) is at most tol (outside the table's
 *     edges: never),
 *   - every normalised feature lies within [lo - m (hi - lo) - 1e-3,
 *     hi + m (hi - lo) + 1e-3], m = guard_margin, and
 *   - with budget > 0, the entries of the intervals the instance has handed
 *     over since gsbs_set_surrogate, this one included, sum to at most budget.
 * A handed-over instance is re-populated at a_(k+1) from the network's output
 * as the change of the log10 concentrations (gsbs_repopulate with relative = 1,
 * mu_y, sd_y); else it continues by SBS steps.  While a surrogate is set,
 * hand-over points are step ends in both modes, so that an advance in which
 * the network takes no interval is the GSBS_PLAIN advance bit for bit.
 * Fails with GSBS_ESTATE for GSBS_SURROGATE without a surrogate, GSBS_EINVAL
 * for another mode. */
int gsbs_advance_to(gsbs_ctx* ctx, const double* t_target, int32_t mode);

typedef struct gsbs_mlp gsbs_mlp;

/* Surrogate hand-over configuration (arrays are copied). */
typedef struct {
    double settle_ns;          /* hand-over this long after an injection (1000) */
    double min_gap_ns;         /* shortest interval handed over (0) */
    double tol;                /* largest table entry of an interval handed over (0.01) */
    double budget;             /* > 0: largest sum of the entries handed over per instance */
    double guard_margin;       /* fraction of the training span the features may exceed (0.1) */
    double r_max_nm;           /* pair-correlation shells reach min(L/2, r_max_nm) (200) */
    double c_floor_M;          /* added to concentrations before log10 (1e-10) */
    int32_t n_ref_max;         /* references per species of the pair correlations (1024) */
    int32_t n_dt, n_c;         /* table bins, 1..16 each */
    int32_t reserved;
    const float* mu;           /* [296] feature centres */
    const float* sd;           /* [296] feature scales */
    const float* lo;           /* [296] smallest normalised training feature (NULL: no guard) */
    const float* hi;           /* [296] largest normalised training feature */
    const float* mu_y;         /* [7] output centres (a calibration offset folded in) */
    const float* sd_y;         /* [7] output scales */
    const double* dt_edges;    /* [n_dt + 1] ascending, log10 ns */
    const double* c_edges;     /* [n_c + 1] ascending, log10 mol/L */
    const double* table;       /* [n_dt][n_c] held-out error estimate (relative H2O2 error) */
} gsbs_surrogate;

/* Set (cfg and net non-NULL) or clear (both NULL) the surrogate of the
 * context: net is borrowed (it must outlive the context's advances and hold
 * at least as many batch rows as the context has instances); every instance's
 * spent budget and hand-over log restart.  The table needs the 7-species,
 * 9-reaction chemistry of gsbs_features.  Fails with GSBS_EINVAL for
 * non-positive scales, non-ascending edges or a bin count outside 1..16. */
int gsbs_set_surrogate(gsbs_ctx* ctx, gsbs_mlp* net, const gsbs_surrogate* cfg);

/* Hand-over points instance inst met in GSBS_SURROGATE advances since
 * gsbs_set_surrogate (host arrays of capacity max_n, any may be NULL): the
 * hand-over time, the next injection time, the table entry (+inf when the
 * guard or the table's edges refused it) and whether the network took the
 * interval; *n the count. */
int gsbs_get_handover_log(gsbs_ctx* ctx, int32_t inst, int64_t max_n, double* t_switch, double* t_next,
                          double* estimate, int32_t* taken, int64_t* n);

/* Pair-correlation function of instance inst in its present state: out[r][k]
 * for the 9 reactions and 32 shells, as defined for gsbs_features (features
 * 7..294 unnormalised).  Synchronises. */
int gsbs_pair_corr(gsbs_ctx* ctx, int32_t inst, double r_max_nm, int32_t n_ref_max, float* out);

/* Block until all queued work on the context's stream has finished. */
int gsbs_sync(gsbs_ctx* ctx);

/* -------------------------------------------------------------- results --- */

/* Species counts of instance inst at its record times: out[n_records][n_species]
 * (int64); records not reached yet hold -1. */
int gsbs_get_counts(gsbs_ctx* ctx, int32_t inst, int64_t* out);

/* G-values at the record times: out[n_records][n_species] in molecules per
 * 100 eV of the energy deposited up to that record (NaN before any energy). */
int gsbs_get_gvalues(gsbs_ctx* ctx, int32_t inst, double* out);

/* Current species counts of instance inst: out[n_species]. */
int gsbs_get_current_counts(gsbs_ctx* ctx, int32_t inst, int64_t* out);

/* Current time (ns) and live molecule count of an instance. */
int gsbs_get_time(gsbs_ctx* ctx, int32_t inst, double* t_ns);
int gsbs_get_n(gsbs_ctx* ctx, int32_t inst, int64_t* n);

int gsbs_get_stats(gsbs_ctx* ctx, gsbs_stats* out);

/* The autotuner's process-wide table.  A step's search grid is one of a few
 * configurations (search mode, cells per cutoff, molecules per cell); the
 * grid never changes which pairs are candidates, only the speed, so the
 * tuner times configurations on live steps (keyed by the occupancy of a
 * cutoff-sized grid and the molecule count, both in octaves) and reuses the
 * fastest.  For k < *n (at most max_k entries): keys[2k], keys[2k+1] = the two
 * octaves, best[k] = the chosen configuration, best_ms[k] = its mean step
 * time. */
int gsbs_get_tuning(int32_t max_k, int32_t* keys, int32_t* best, double* best_ms, int32_t* n);

/* Per-kernel timing with HIP events recorded around every step kernel on the
 * context's stream (on = 1).  Profiling drains the stream after each step, so
 * it is for measurement passes, not for production runs. */
int gsbs_set_profiling(gsbs_ctx* ctx, int32_t on);

/* Live per-kernel timing: while kernel_mask != 0, gsbs_advance_to records a
 * HIP event at every boundary between the kernels of each step (slots as
 * named by gsbs_get_profile: 0 k_bin, 1 k_scan, 2 k_scatter, 3 k_pairs,
 * 4 k_pairs_sp, 5 k_react with the first-order kernel), on the context's
 * stream, without draining it: a chunk of steps' events are read once its
 * last kernel has finished.  A slot's time runs from its boundary to the
 * next.  Times and launches of the slots whose bit is set accumulate into
 * gsbs_get_profile's totals, and its work units then come from device-side
 * counters: molecule-steps of the stepped instances (k_bin, k_scatter,
 * k_react), of the instances searched by whole cells (k_pairs) or species bins
 * (k_pairs_sp), bins (k_scan).  Switching (also to 0) drains the stream and
 * clears the totals.  Not combined with gsbs_set_profiling or step graphs.
 * Fails with GSBS_EINVAL for mask bits above 5. */
int gsbs_set_live_timing(gsbs_ctx* ctx, uint32_t kernel_mask);

/* Device memory the context holds now, in bytes: molecule arrays at their
 * capacity, search grid, pair list, records, queued injections. */
int gsbs_get_device_bytes(gsbs_ctx* ctx, int64_t* bytes);

/* Accumulated profile: for k < *n (at most max_k) the kernel name (NUL-padded
 * in names[k*32 .. k*32+31]), total milliseconds, number of launches, work
 * units processed (bins for the scan, live molecules for every other kernel)
 * and candidate pairs found (end separation below r_c; non-zero for the two
 * pair-search kernels only).  Any output pointer may be NULL. */
int gsbs_get_profile(gsbs_ctx* ctx, int32_t max_k, char* names, double* total_ms, int64_t* launches,
                     int64_t* work, int64_t* candidates, int32_t* n);

/* Per-step log of the profiled steps of gsbs_advance_to (instance 0): Philox
 * step index, step time in ms (first to last kernel), grid (nc, reach,
 * species-bin search flag, configuration) as 4 ints, live-count estimate. */
int gsbs_get_step_log(gsbs_ctx* ctx, int64_t max_n, int64_t* step, double* ms, int32_t* grid, int64_t* n_est,
                      int64_t* n);

/* ------------------------------------------------- schedule (host only) --- */

/* Step end times in (t_start, t_end] for ramp anchors (injection times) and
 * events (records, injections; t_end is always one): after each anchor the
 * lattice anchor + dt0 * ratio^j, j >= 0, up to the next anchor; lattice points
 * within 1e-9 (relative) of an event are dropped; gaps above dt_max are cut in
 * equal sub-steps.  Writes min(count, max_out) times to out (may be NULL) and
 * returns the count in *n_out.  Needs no device. */
int gsbs_plan_schedule(double t_start, double t_end, int32_t n_anchor, const double* anchors,
                       int32_t n_events, const double* events, double dt0, double ratio,
                       double dt_max, double* out, int64_t max_out, int64_t* n_out);

/* ---------------------------------------------------------------- debug --- */

/* Copy instance inst's live molecules out (host arrays of capacity max_n):
 * positions xyz (n x 3), species, uids; *n receives the live count. */
int gsbs_debug_get_state(gsbs_ctx* ctx, int32_t inst, int64_t max_n, float* xyz, uint8_t* species,
                         uint64_t* uid, int64_t* n);

/* Replace the whole state of a single-instance context: n molecules with
 * positions xyz, species and uids (host arrays); `step` is the index the next
 * step uses in its Philox counters; next_uid the next fresh uid. */
int gsbs_debug_set_state(gsbs_ctx* ctx, int64_t n, const float* xyz, const uint8_t* species,
                         const uint64_t* uid, int64_t step, uint64_t next_uid);

/* One step of length dt_ns on a single-instance context.  flags bit 0: skip the
 * Brownian jump and treat xyz0 (n x 3, host) as the start positions of the
 * current state (pairs are then searched on fixed positions).  flags bit 1:
 * log every candidate pair, not only accepted ones.  flags bit 2: stop after
 * the pair search (no matching, no reactions, state unchanged).  flags bit 3 /
 * bit 4: force the species-bin / whole-cell search.  nc_force > 0 forces the
 * search grid to nc_force^3 cells (the stencil widens to cover the cutoff). */
int gsbs_debug_step(gsbs_ctx* ctx, double dt_ns, int32_t flags, const float* xyz0, int32_t nc_force);

/* Pair log of the last debug step (host arrays of capacity max_n): uid pairs
 * (lower, higher), contact probability P (FP32), the pair uniform's 24-bit
 * integer, reaction index, flags (bit0 accepted, bit1 reacted); *n the size. */
int gsbs_debug_get_pairs(gsbs_ctx* ctx, int64_t max_n, uint64_t* uid2, float* P, uint32_t* u24,
                         int32_t* rx, int32_t* flags, int64_t* n);

/* Search grid of the last debug step: *nc cells per axis, and for every live
 * molecule (same order as gsbs_debug_get_state after that step's sort) its
 * cell index (ix*nc + iy)*nc + iz and uid. */
int gsbs_debug_get_cells(gsbs_ctx* ctx, int64_t max_n, int32_t* cell, uint64_t* uid, int32_t* nc,
                         int64_t* n);

/* ---------------------------------------- surrogate state (features) --- */
/* Input features of the surrogate for instance inst in its present state
 * (7 species and 9 reactions required), 296 floats:
 *   [0..7)    log10(C_s + c_floor_M), C_s the concentration in mol/L;
 *   [7..295)  g_r(k), reaction r = 0..8, shell k = 0..31: the pair-correlation
 *             function of the reactants (a, b) of reaction r, i.e. the count of
 *             b molecules in shell k around reference a molecules divided by
 *             its ideal-gas expectation n_ref (N_b - [a == b]) / L^3 V_k.
 *             Shells are log-spaced, edges e_k = R_r (r_m / R_r)^(k/32),
 *             r_m = min(L/2, r_max_nm), R_r the reaction radius; shell 0 also
 *             holds r < R_r; distances are FP32 minimum-image (Eq. 2).  The
 *             references are the molecules of species a with uid % m_a == 0,
 *             m_a = ceil(N_a / n_ref_max) (1 when no reference or partner);
 *   [295]     log10(dt_next_ns).
 * Each feature f is returned as (f - mu[f]) / sd[f] clamped to [-8, 8] (mu,
 * sd: host arrays of 296); with both NULL the raw value, unclamped.  out is a
 * device pointer when out_is_device = 1,
 * else a host array.  Synchronises the context's stream. */
int gsbs_features(gsbs_ctx* ctx, int32_t inst, double dt_next_ns, double r_max_nm, int32_t n_ref_max,
                  double c_floor_M, const float* mu, const float* sd, float* out, int32_t out_is_device);

/* Replace every molecule of instance inst by a homogeneous population and
 * move the instance's clock to t_new_ns (>= its present time, before any of
 * its queued injections): y[7] (device pointer when y_is_device, else host)
 * holds normalised log10 concentrations, C_s = 10^(y_s sd_y[s] + mu_y[s]) -
 * c_floor_M (mol/L, clipped at 0), or with relative = 1 their change from the
 * present state, C_s = 10^(y_s sd_y[s] + mu_y[s] + log10(C_s,now + c_floor_M))
 * - c_floor_M; the mean count C_s N_A L^3 is rounded
 * down or up with the Philox uniform at counter (s, step, 0, 3); positions
 * are uniform in the cube from the Philox words at counter (uid, step, 1, 3),
 * key (seed, inst); uids continue the instance's counter.  Records strictly
 * between the old and the new time are left unrecorded.  Synchronises. */
int gsbs_repopulate(gsbs_ctx* ctx, int32_t inst, double t_new_ns, const float* y, int32_t y_is_device,
                    const float* mu_y, const float* sd_y, double c_floor_M, int32_t relative);

/* ------------------------------------------------------- checkpoint --- */
/* Checkpoint and resume: the whole state of a context between calls --
 * chemistry, parameters, seed, every instance's time, step counter, next uid,
 * deposited energy, record times and results, pending injections, and the
 * molecule array with its counters.  Random numbers are counter-based (seed,
 * instance, uid, step), so a run resumed from a checkpoint continues exactly
 * as the uninterrupted run would (same steps, same outcomes), provided both
 * stop at the same step ends.
 *
 * gsbs_save writes the checkpoint into buf (host, cap bytes) and its length
 * into *size; with buf NULL it only reports the length.  Fails with
 * GSBS_ECAPACITY when cap is too small, GSBS_ESTATE before the chemistry is
 * set.  The format is private to this library version. */
int gsbs_save(gsbs_ctx* ctx, void* buf, int64_t cap, int64_t* size);

/* Restore a checkpoint of gsbs_save into ctx, which must have been created
 * with the same number of instances and the same cube edges (its seed and
 * chemistry are replaced).  Fails with GSBS_EINVAL for anything else or a
 * truncated or inconsistent buffer (ctx unchanged up to the chemistry). */
int gsbs_load(gsbs_ctx* ctx, const void* buf, int64_t size);

/* ------------------------------------------------- rate equations --- */
/* The homogeneous beam-off stage of the paper (its "NumODEs", Eq. 3-4): the
 * mass-action rate equations of the context's reaction table for n
 * independent well-mixed solutions.  Reaction r between species a and b runs
 * at the event rate k [a][b] (k [a]^2 / 2 when a == b: the table prints 2k for
 * self-recombinations, so that d[a]/dt = -k [a]^2, the paper's equation for the
 * OH recombination), k = 10 * k_in L/mol/ns; each event removes its reactants
 * (not b when keep_b) and adds its products; each first-order channel of
 * gsbs_set_first_order runs at k [a], and each zero-order source of
 * gsbs_set_sources adds its rate to its products.  c0 and c1 are [n][n_species]
 * concentrations in mol/L (row-major; n_species must equal the table's
 * species count, else GSBS_EINVAL), dt_ns[n] the time of each solution;
 * c1 receives the concentrations after dt_ns (negative entries of c0 are
 * taken as 0; a dt_ns of 0 or below returns them so).  Integration: FP64, the
 * four-stage third-order stiffly accurate Rosenbrock method RODAS3 with step
 * control by its embedded second-order solution, relative tolerance rtol
 * (0 < rtol <= 0.1) and absolute tolerance 1e-10 * rtol mol/L; one device
 * thread per solution.  on_device = 1: c0, dt_ns, c1 are device pointers;
 * 0: host arrays.  steps (host, may be NULL) receives the accepted steps of
 * every solution.  Returns after c1 is written.  Fails with GSBS_ESTATE before
 * the reaction table is set or when a solution needs more than 200000 steps
 * (its steps entry is then -1), and with GSBS_EINVAL when the table has more
 * than 8 species (a mixture's state is held in registers). */
int gsbs_numodes(gsbs_ctx* ctx, int32_t n, int32_t n_species, const double* c0, const double* dt_ns, double* c1,
                 double rtol, int32_t* steps, int32_t on_device);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * computation of gsbs_numodes on device arrays only, with no allocation.
 * c0, dt_ns, c1 are device pointers (as gsbs_numodes with on_device = 1);
 * steps (host, n entries, required) receives the accepted steps.  The step
 * counts are staged in a file-scope device array of the library (1048576
 * int32 = 4 MiB per GPU, held until the process ends), so n is at most
 * 1048576 (else GSBS_EINVAL); every call on one GPU uses that GPU's array,
 * so calls that overlap on one GPU race (serialise them, e.g. on one
 * stream).  Call with the context's device current.  Returns after c1 and
 * steps are written; errors as gsbs_numodes. */
int gsbs_numodes_noalloc(gsbs_ctx* ctx, int32_t n, int32_t n_species, const double* c0, const double* dt_ns,
                         double* c1, double rtol, int32_t* steps);

/* --------------------------------------------- stochastic kinetics --- */
/* Homogeneous stochastic kinetics of the context's reaction table in n
 * independent well-mixed volumes: Gillespie's direct method (Gillespie 1977),
 * the stochastic reference the paper checks SBS + PBCs and its rate
 * equations against (section on the verification of periodic boundary
 * conditions).  Volume m (volume_L[m] litres) starts from the counts
 * n0[m][n_species] (n_species must equal the table's species count).
 * Reaction r between a and b has the propensity c_r h_r, c_r = k_r / (N_A V)
 * (k_r = 10 * k_in L/mol/ns, the printed constant: 2k for a
 * self-recombination), h_r = n_a n_b or n_a (n_a - 1) / 2 when a == b; each
 * event removes the reactants (not b when keep_b) and adds the products.  The
 * first-order channels of gsbs_set_first_order (a = k n_a, species order) and
 * then the zero-order sources of gsbs_set_sources (a_q = rate_q N_A V) follow
 * the reactions in the propensity list.
 * Random numbers: Philox4x64-10, key (seed, 0x4753534153534131), counter
 * (stream0 + m, j / 2, 0, 0) for events j (even; words 0, 1) and j + 1
 * (words 2, 3); waiting time -ln(u1) / a_0, reaction = first r whose running
 * sum of propensities (table order) exceeds u2 a_0, u = (top 53 bits of the
 * word + 1/2) 2^-53.  A stream's event sequence
 * is therefore fixed bit for bit; event times carry the rounding of ln.
 * t_rec_ns[n_rec] (host, finite, >= 0, ascending) are the record times:
 * out[m][k][s] receives the counts after every event at a time <= t_rec_ns[k].
 * A volume stops once its last record is taken or no reaction can happen.
 * events (host, may be NULL) receives the number of events of each volume.
 * on_device = 1: n0, volume_L and out are device pointers (volumes and counts
 * are then not checked); 0: host arrays.  Returns after out is written.
 * Fails with GSBS_EINVAL for bad arguments, a table beyond 8 species or 16
 * reactions, a volume <= 0 or a negative count (host arrays); GSBS_ESTATE
 * before the reaction table is set or when a volume needs more than
 * max_events events before its last record (its events entry is then -1).
 * One device thread per volume; its run time grows with the event count, so
 * callers bound max_events. */
int gsbs_ssa(gsbs_ctx* ctx, int32_t n, int32_t n_species, const int32_t* n0, const double* volume_L, int32_t n_rec,
             const double* t_rec_ns, uint64_t seed, uint64_t stream0, int64_t max_events, int32_t* out,
             int64_t* events, int32_t on_device);

/* ------------------------------------------- inter-pulse surrogate MLP --- */
/* A perceptron that maps the state at the end of a pulse's SBS segment
 * (species concentrations, binned pair-correlation features, log of the time
 * to the next pulse: 296 inputs) to the 7 log-concentrations at the next
 * pulse, standing in for the long homogeneous evolution between pulses that
 * the paper integrates with rate equations (its Eq. 3-4, "NumODEs").  Layers
 * 296-256-256-256-256-7, erf-GELU after each hidden layer, BF16 weights and
 * activations, FP32 accumulation, FP32 master weights updated by Adam.  All
 * x / t / y arrays are device pointers, row-major [batch][width], read and
 * written in order on the stream given at creation; every call returns after
 * queueing its kernels unless it returns host data. */
/* Number of parameters of the flat FP32 layout used by set/get: per layer the
 * weight matrix W[n_out][n_in] row-major, then the bias b[n_out]. */
int gsbs_mlp_param_count(int64_t* n);

/* Allocate a network for batches of up to max_batch rows on `stream` (a
 * hipStream_t, NULL for the null stream).  Weights start at zero. */
int gsbs_mlp_create(int32_t max_batch, void* stream, gsbs_mlp** out);
int gsbs_mlp_destroy(gsbs_mlp* m);

/* Replace / read the FP32 master weights (host arrays of n = param_count
 * floats).  Setting resets the Adam moments and step counter and refreshes
 * the BF16 copies (round to nearest even). */
int gsbs_mlp_set_weights(gsbs_mlp* m, const float* w, int64_t n);
int gsbs_mlp_get_weights(gsbs_mlp* m, float* w, int64_t n);

/* y[batch][7] = network(x[batch][296]); x is rounded to BF16 on entry. */
int gsbs_mlp_forward(gsbs_mlp* m, const float* x, int32_t batch, float* y);

/* BF16 activations entering layer `layer` (0: the rounded input, 1..4: the
 * hidden outputs) of the last forward pass, as FP32 host array
 * out[batch][width] (width 296 for layer 0, else 256). */
int gsbs_mlp_get_activation(gsbs_mlp* m, int32_t layer, int32_t batch, float* out);

/* Forward and backward pass of the mean squared error over the batch x 7
 * outputs against t[batch][7]; keeps the FP32 gradients (read them with
 * gsbs_mlp_get_grads, same layout as the weights); *loss (host, may be NULL)
 * receives the mean squared error.  The product operands (activations,
 * output gradients, weights) are BF16, accumulation FP32. */
int gsbs_mlp_backward(gsbs_mlp* m, const float* x, const float* t, int32_t batch, float* loss);
int gsbs_mlp_get_grads(gsbs_mlp* m, float* g, int64_t n);

/* One Adam step (bias-corrected, step counter inside the network) on the FP32
 * master weights with the last gradients, then the BF16 copies refresh. */
int gsbs_mlp_adam(gsbs_mlp* m, float lr, float beta1, float beta2, float eps);

/* gsbs_mlp_backward followed by gsbs_mlp_adam. */
int gsbs_mlp_train_step(gsbs_mlp* m, const float* x, const float* t, int32_t batch, float lr, float beta1,
                        float beta2, float eps, float* loss);

#ifdef __cplusplus
}
#endif

#endif /* GSBS_H */
