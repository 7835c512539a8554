// engine.h -- structures shared by the host scheduler (api.cpp) and the HIP
// kernels (kernels.hip) of the SBS diffusion-reaction engine.  Internal: not
// part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsbs {

constexpr int kMaxSpecies = 16;
constexpr int kMaxReactions = 32;
constexpr int kDead = 0xFF;          // species byte of a removed molecule
constexpr uint32_t kNoCell = 0xFFFFFFFFu;

// Chemistry tables (constant during a run).
// Reaction table of the rate equations (passed by value to the integrator):
// reaction r runs at the event rate kr[r] [a][b] (kr = k for a != b, k / 2 for
// a == b; k in L/mol/ns), or kr[r] [a] for a first-order channel (rb = -1, kr
// per ns), and changes species s by nu[r][s] per event.  The
// integrator keeps a mixture's state in registers: at most kOdeMaxSpecies.
constexpr int kOdeMaxSpecies = 8;
struct OdeTable {
    int32_t ns, nr;
    int32_t ra[kMaxReactions], rb[kMaxReactions];
    double kr[kMaxReactions];
    double nu[kMaxReactions][kOdeMaxSpecies];
    double src[kOdeMaxSpecies];  // zero-order production, mol/L/ns per species
};

// Reaction table of the stochastic kinetics (Gillespie's direct method):
// reaction r between ra and rb has the macroscopic constant k10[r] L/mol/ns
// (the printed value, 2k for a self-recombination) and changes species s by
// the signed byte s of dn[r] per event.
constexpr int kSsaMaxReactions = 16;
constexpr int kMaxSources = 4;
// propensity slots: reactions, first-order channels, sources
constexpr int kSsaSlots = kSsaMaxReactions + kOdeMaxSpecies + kMaxSources;
struct SsaTable {
    int32_t ns, nr, nfo, nsrc;
    int32_t ra[kSsaMaxReactions], rb[kSsaMaxReactions];
    uint64_t dn[kSsaSlots];
    double k10[kSsaMaxReactions];
    int32_t fo_a[kOdeMaxSpecies];                  // first-order channels: species, rate per ns
    double fo_k[kOdeMaxSpecies];
    double src_rate[kMaxSources];                  // zero-order sources, mol/L/ns
};

// Counter-based spur model of a pulse (device generator of gsbs_inject_pulse).
struct SpurParams {
    double L, spacing, mean, sigma;
    double cum[kMaxSpecies];  // running sums of the species fractions
    int32_t ns, last, n_tracks, pad;
    uint64_t seed, stream;
};

struct ChemDev {
    int32_t rmap[kMaxSpecies][kMaxSpecies];  // reaction index of a species pair or -1
    float D[kMaxSpecies];                    // nm^2/ns
    int32_t nprod[kMaxReactions];
    int32_t prod[kMaxReactions][3];
    int32_t keep_b[kMaxReactions];
    int32_t rb[kMaxReactions];
    uint32_t reactive_mask;                  // bit s: species s takes part in a reaction
    uint32_t pmask[kMaxSpecies];             // bit t of pmask[s]: pair (s, t), t >= s, is searched from s
    int32_t n_species;
    int32_t rounds;
    int32_t contact_only;
    // first-order channels: species s -> fo_prod[s][0] (+ fo_prod[s][1]);
    // removed when fo_nprod[s] == 0; bit s of fo_mask: s has a channel
    uint32_t fo_mask;
    int32_t fo_nprod[kMaxSpecies];
    int32_t fo_prod[kMaxSpecies][2];
};

// Everything one instance needs for one step; rebuilt by the host per step.
// The search grid has nc^3 cells of edge h = L/nc per instance.  Molecules are
// sorted by bin: in the species-bin search bins are species-major (bin =
// bin_base + species * nc^3 + cell), in the whole-cell search a cell is one
// bin (bin = bin_base + cell); cell = (ix*nc + iy)*nc + iz.  A candidate of a molecule
// lies at most `reach` cells away along each axis (reach * h >= the largest
// cutoff).
struct alignas(16) InstStep {
    float sigma[kMaxSpecies];      // sqrt(2 D dt) per species
    float rc2[kMaxReactions];      // squared candidate cutoff (FP32 of the FP64 square)
    float R[kMaxReactions];        // reaction radius
    float inv_s[kMaxReactions];    // 1 / (D_AB * dt), 0 when D_AB = 0
    float cull2[kMaxReactions];    // squared cutoff widened for cell culling
    float cull2_sp[kMaxSpecies];   // largest cull2 over the pairs searched from a species (species bins)
    float cull2_all[kMaxSpecies];  // largest cull2 over every reaction of a species (whole cells)
    float L, halfL, invL, inv_h;   // edge, L/2, 1/L, nc/L (all FP32)
    float h, cull_eps;             // cell edge L/nc, slack of the cell-distance bound
    int32_t nc;                    // cells per axis of the search grid
    int32_t reach;                 // stencil half-width in cells
    int32_t bin_base;              // first global bin index of this instance
    int32_t active;                // 1: this instance takes a step now
    int32_t by_species;            // 1: search partner-species bins, 0: whole cells
    int32_t unit_base;             // species-bin search: first global work item of this instance
    int32_t pad1;
    int32_t pad0;
    // species-bin search: partner species searched from each species (the more
    // abundant side of every pair), A-box size in cells of each species
    // (kx | ky << 8 | kz << 16), and the first work item of each species inside
    // the instance
    uint32_t pm_dir[kMaxSpecies];
    int32_t kdim_sp[kMaxSpecies];
    int32_t unit_off_sp[kMaxSpecies + 4];
    // species-bin search: work items (stream slices) per A box of each species,
    // and (host planning only) the partner molecules a box of that species streams
    int32_t nsplit_sp[kMaxSpecies];
    float work_sp[kMaxSpecies];
    uint64_t step;                 // Philox step counter word
    uint64_t key0, key1;           // Philox key (seed, instance)
    double fo_p[kMaxSpecies];      // first-order conversion probability 1 - exp(-k dt) per species
};

// Accepted (or, in debug logging, candidate) pair of sorted indices.
struct PairRec {
    int32_t i, j;         // sorted indices, i < j in enumeration order
    uint32_t u24;         // pair uniform, integer part
    int32_t rx;           // reaction index
    float P;              // contact probability (FP32)
    int32_t flags;        // bit0 accepted, bit1 reacted, bit2 matched in the current round
};

// Device-wide counters and flags.
struct DevCounters {
    int32_t n_in;              // molecules in the current input array (incl. removed)
    int32_t n_live;            // live molecules after the sort
    uint32_t n_pairs;          // pairs appended this step
    uint32_t err;              // bit0 molecule overflow, bit1 pair overflow, bit2 key tie
    unsigned long long cand;   // candidate pairs tested (cumulative)
    unsigned long long reactions;
    // molecule-steps of the instances stepped with the whole-cell / species-bin
    // search (cumulative), and the species-bin search's share of cand
    unsigned long long msteps_mode[2];
    unsigned long long cand_sp;
    unsigned long long pad;
};

constexpr uint32_t kErrMolOverflow = 1u;
constexpr uint32_t kErrPairOverflow = 2u;
constexpr uint32_t kErrTie = 4u;
constexpr uint32_t kErrScanStall = 16u;  // a scan tile waited too long for its predecessors

struct RecordList {
    int32_t n;
    int32_t inst[32];
    int32_t rec[32];
};

// Kernel launch helpers (kernels.hip).
struct StepBuffers {
    float4* pos_in;       // current molecules: x, y, z, meta = (instance << 8) | species
    uint64_t* uid_in;
    float4* pos_out;      // sorted molecules after the jump
    float4* pos0_out;     // sorted start-of-step positions; .w carries the global bin index
    uint64_t* uid_out;
    uint2* cellrank;      // per input molecule: (global bin, rank inside the bin)
    float4* xnew;         // per input molecule: end position of the step (meta in .w)
    uint32_t* cell_count; // per bin, zero between steps
    uint32_t* cell_start; // per bin exclusive prefix sums, one extra entry at the end
    unsigned long long* scan_status;  // per scan tile: look-back status word
    uint32_t scan_epoch;              // 1 .. 2^31 - 1, one per step
    PairRec* pairs;
    uint32_t pair_cap;
    unsigned long long* claim;  // per sorted index, all ones between steps
    int32_t* mate;              // per sorted index, -1 between steps
    long long* counts;          // [n_inst][kMaxSpecies] current species counts
    unsigned long long* msteps; // [n_inst] molecule-steps
    DevCounters* ctr;
    int32_t cap;
    const float4* x0_override;  // debug: start positions in input order, or nullptr
};

void launch_inject(hipStream_t st, float4* pos, uint64_t* uid, long long* counts, DevCounters* ctr,
                   const float* xyz, const uint8_t* sp, int32_t n, int32_t inst, uint64_t uid_base,
                   int32_t cap);
// Kernels of one step, in launch order; ev (optional) holds 2 events per kernel.
constexpr int kStepKernels = 6;
extern const char* const kStepKernelNames[kStepKernels];
// ev_mask: bit k set records the two events of kernel slot k (ev[2k], ev[2k+1]);
// with kEvChain set, ev[0 .. kStepKernels] mark the boundaries between the slots.
constexpr uint32_t kEvChain = 0x80000000u;
void launch_step(hipStream_t st, const StepBuffers& b, const InstStep* P, const ChemDev* chem,
                 int32_t n_inst, int32_t total_bins, int32_t total_units, int32_t n_species, int32_t grid,
                 int32_t flags, hipEvent_t* ev = nullptr, uint32_t ev_mask = 0xFFFFFFFFu);
// bins up to which k_bin counts in an LDS histogram (larger grids use global atomics)
constexpr int32_t kLdsBins = 12288;
void launch_record(hipStream_t st, const long long* counts, long long* rec, int32_t max_rec,
                   const RecordList& list);

// Sets the message gsbs_last_error returns and passes the code through.
int set_error(int code, const char* msg);

// Surrogate state kernels (surrogate.hip): pair-correlation shells per reaction,
// reference subsample stride per species, error flag of a reference overflow.
constexpr int kSurBins = 32;
constexpr uint32_t kErrRefOverflow = 8u;
struct SurStrides {
    int32_t s[kMaxSpecies];
};
void launch_collect_refs(hipStream_t st, const float4* pos, const uint64_t* uid, const DevCounters* ctr, int inst,
                         const SurStrides& strides, int cap, int32_t* ref_idx, int32_t* ref_cnt, uint32_t* err,
                         int grid);
void launch_pair_corr(hipStream_t st, const float4* pos, const DevCounters* ctr, int inst, const int32_t* ref_idx,
                      const int32_t* ref_cnt, int cap, const int32_t* pair_ab, const float* edges2, int n_pairs,
                      float L, unsigned long long* hist, int64_t n_est);
void launch_features(hipStream_t st, const long long* counts, int inst, int ns, const unsigned long long* hist,
                     const int32_t* ref_cnt, int cap, const int32_t* pair_ab, const double* shell_vol, int n_pairs,
                     double L, double dt_next, double c_floor, const float* mu, const float* sd, int clamp,
                     float* out);
void launch_repop_counts(hipStream_t st, const float* y, const float* mu, const float* sd, int ns, double c_floor,
                         double vol_litre, uint64_t seed, int inst, uint64_t step, int relative,
                         const long long* counts, long long* out);
// Rate equations of n mixtures (c0, c1: [n][tb.ns] mol/L, dt: [n] ns, device).
void launch_spur_count(hipStream_t st, const SpurParams& P, int64_t* cnt);
void launch_spur_emit(hipStream_t st, const SpurParams& P, const int64_t* off, float* xyz, uint8_t* sp);
void launch_ssa(hipStream_t st, const int32_t* n0, const double* vol, const double* t_rec, int32_t n_rec,
                int32_t* out, long long* events, int32_t n, const SsaTable& tb, uint64_t seed, uint64_t stream0,
                long long max_events);
void launch_numodes(hipStream_t st, const double* c0, const double* dt, double* c1, int32_t* steps, int32_t n,
                    const OdeTable& tb, double rtol, double atol, int32_t max_steps);
// Mixtures of one gsbs_numodes_noalloc call at most, and the device address of
// its step-count array on the current device (numodes.hip).
constexpr int32_t kNoAllocMaxMixtures = 1 << 20;
int numodes_scratch(int32_t** out);
void launch_repop(hipStream_t st, float4* pos, uint64_t* uid, DevCounters* ctr, const long long* newc, int ns,
                  int n_new, int inst, uint64_t uid_base, uint64_t seed, uint64_t step, float L, int cap,
                  long long* counts, int grid);

// debug flags of launch_step
constexpr int32_t kStepLogAll = 2;
constexpr int32_t kStepSearchOnly = 4;
constexpr int32_t kStepFixed = 1;
constexpr int32_t kStepBySpecies = 8;   // debug: force the species-bin search
constexpr int32_t kStepWholeCells = 16;  // debug: force the whole-cell search
constexpr int32_t kStepHasWhole = 32;    // some instance uses the whole-cell search this step
constexpr int32_t kStepHasSpecies = 64;  // some instance uses the species-bin search this step
constexpr int32_t kStepFirstOrder = 128; // the chemistry has first-order channels

}  // namespace gsbs
