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
struct ChemDev {
    int32_t rmap[kMaxSpecies][kMaxSpecies];  // reaction index of a species pair or -1
    float D[kMaxSpecies];                    // nm^2/ns
    int32_t nprod[kMaxReactions];
    int32_t prod[kMaxReactions][3];
    int32_t keep_b[kMaxReactions];
    int32_t rb[kMaxReactions];
    uint32_t reactive_mask;                  // bit s: species s takes part in a reaction
    int32_t n_species;
    int32_t rounds;
    int32_t contact_only;
};

// Everything one instance needs for one step; rebuilt by the host per step.
struct alignas(16) InstStep {
    float sigma[kMaxSpecies];      // sqrt(2 D dt) per species
    float rc2[kMaxReactions];      // squared candidate cutoff (FP32 of the FP64 square)
    float R[kMaxReactions];        // reaction radius
    float inv_s[kMaxReactions];    // 1 / (D_AB * dt), 0 when D_AB = 0
    float L, halfL, invL, inv_h;   // edge, L/2, 1/L, nc/L (all FP32)
    int32_t nc;                    // cells per axis of the search grid
    int32_t cell_base;             // first global cell index of this instance
    int32_t active;                // 1: this instance takes a step now
    int32_t pad0;
    uint64_t step;                 // Philox step counter word
    uint64_t key0, key1;           // Philox key (seed, instance)
    uint64_t pad1;
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
    unsigned long long pad[4];
};

constexpr uint32_t kErrMolOverflow = 1u;
constexpr uint32_t kErrPairOverflow = 2u;
constexpr uint32_t kErrTie = 4u;

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
    float4* pos0_out;     // sorted start-of-step positions; .w carries the global cell index
    uint64_t* uid_out;
    uint2* cellrank;      // per input molecule: (global cell, rank inside the cell)
    uint32_t* cell_count; // zero between steps
    uint32_t* cell_start; // exclusive prefix sums, one extra entry at the end
    uint32_t* block_sums;
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
void launch_step(hipStream_t st, const StepBuffers& b, const InstStep* P, const ChemDev* chem,
                 int32_t n_inst, int32_t total_cells, int32_t grid, int32_t flags, hipEvent_t* ev = nullptr);
void launch_record(hipStream_t st, const long long* counts, long long* rec, int32_t max_rec,
                   const RecordList& list);

// debug flags of launch_step
constexpr int32_t kStepLogAll = 2;
constexpr int32_t kStepSearchOnly = 4;
constexpr int32_t kStepFixed = 1;

}  // namespace gsbs
