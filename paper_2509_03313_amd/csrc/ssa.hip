// ssa.hip -- homogeneous stochastic kinetics for many independent well-mixed
// volumes at once: Gillespie's direct method (Gillespie, J. Phys. Chem. 81,
// 1977), the stochastic reference against which the paper checks SBS + PBCs
// and its rate equations (section on the verification of periodic boundary
// conditions, and the discussion of its figure).  One lane per volume; the
// constants and propensities live in registers, the counts in LDS.
//
// Propensity of reaction r: a_r = c_r h_r, c_r = k_r / (N_A V) with k_r the
// printed constant in L/mol/ns, h_r = n_a n_b (a != b) or n_a (n_a - 1) / 2
// (a == b), the number of distinct reactant pairs.  A step draws u1, u2 from
// Philox4x64-10 (key (seed, 0x4753534153534131), counter (stream, j / 2, 0,
// 0): words 0 and 1 for an even event j, 2 and 3 for the odd one after it;
// u = (top 53 bits + 1/2) 2^-53), waits -ln(u1) / a_0
// (a_0 summed in table order) and fires the first reaction whose running sum
// of propensities exceeds u2 a_0 (the last one with a_r > 0 if rounding leaves
// none).  The reaction choice is exact integer-derived FP64 arithmetic in a
// fixed order, so the event sequence of a stream is reproducible bit for bit.
// First-order channels (a = k n_s, in species order) and then zero-order
// sources (a_q = rate_q N_A V, rate in mol/L/ns) follow the reactions in the
// propensity list.
#include "device_common.h"
#include "engine.h"

namespace gsbs {

namespace {

constexpr double kNA = 6.02214076e23;
constexpr uint64_t kSsaKey = 0x4753534153534131ull;

__device__ __forceinline__ double u53(uint64_t w) {
    return ((double)(w >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// kExtra: the table has first-order channels or sources (more propensity slots)
template <int S, bool kExtra>
__global__ __launch_bounds__(64) void k_ssa(const int32_t* __restrict__ n0, const double* __restrict__ vol,
                                            const double* __restrict__ t_rec, int32_t n_rec,
                                            int32_t* __restrict__ out, long long* __restrict__ events, int32_t n,
                                            SsaTable tb, uint64_t seed, uint64_t stream0, long long max_events) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const int ns = tb.ns, nr = tb.nr;
    // the counts live in LDS, one column per lane: a reactant's count is read
    // at an offset that is the same for every lane
    __shared__ int32_t cnt_lds[S][64];
    const int lane = threadIdx.x;
#pragma unroll
    for (int s = 0; s < S; ++s) cnt_lds[s][lane] = s < ns ? n0[(size_t)m * ns + s] : 0;
    const double nav = kNA * vol[m];
    constexpr int kA = kExtra ? kSsaSlots : kSsaMaxReactions;  // reactions, first-order channels, sources
    constexpr int kF = kSsaMaxReactions, kQ = kSsaMaxReactions + kOdeMaxSpecies;
    double c[kSsaMaxReactions];
#pragma unroll
    for (int r = 0; r < kSsaMaxReactions; ++r) c[r] = r < nr ? tb.k10[r] / nav : 0.0;
    const uint64_t stream = stream0 + (uint64_t)m;
    int32_t* o = out + (size_t)m * n_rec * ns;
    double t = 0.0;
    long long j = 0;
    int rec = 0;
    double t_r = t_rec[0];
    uint64_t w[4] = {0, 0, 0, 0};
    for (;;) {
        double a[kA];
        double a0 = 0.0;
#pragma unroll
        for (int r = 0; r < kSsaMaxReactions; ++r) {
            if (r < nr) {
                const int32_t na = cnt_lds[tb.ra[r]][lane], nb = cnt_lds[tb.rb[r]][lane];
                const double h = tb.ra[r] == tb.rb[r] ? (double)na * (double)(na - 1) * 0.5
                                                      : (double)na * (double)nb;
                a[r] = c[r] * h;
                a0 += a[r];
            } else {
                a[r] = 0.0;
            }
        }
        if (kExtra) {
#pragma unroll
            for (int q = 0; q < kOdeMaxSpecies; ++q) {
                a[kF + q] = q < tb.nfo ? tb.fo_k[q] * (double)cnt_lds[q < tb.nfo ? tb.fo_a[q] : 0][lane] : 0.0;
                if (q < tb.nfo) a0 += a[kF + q];
            }
#pragma unroll
            for (int q = 0; q < kMaxSources; ++q) {
                a[kQ + q] = q < tb.nsrc ? tb.src_rate[q] * nav : 0.0;
                if (q < tb.nsrc) a0 += a[kQ + q];
            }
        }
        double t_next = __builtin_huge_val(), u2 = 0.0;
        if (a0 > 0.0) {
            // every live lane is at the same event index, so this branch is uniform
            if ((j & 1) == 0) philox(stream, (uint64_t)j >> 1, 0, 0, seed, kSsaKey, w);
            const bool odd = (j & 1) != 0;
            t_next = t + (-log(u53(odd ? w[2] : w[0])) / a0);
            u2 = u53(odd ? w[3] : w[1]);
        }
        while (rec < n_rec && t_r < t_next) {
            int32_t* orow = o + (size_t)rec * ns;
#pragma unroll
            for (int s = 0; s < S; ++s)
                if (s < ns) orow[s] = cnt_lds[s][lane];
            ++rec;
            t_r = rec < n_rec ? t_rec[rec] : 0.0;
        }
        if (rec == n_rec) break;
        if (j == max_events) {
            j = -1;
            break;
        }
        const double target = u2 * a0;
        double cum = 0.0;
        int mu = -1, last = -1;
#pragma unroll
        for (int r = 0; r < kA; ++r) {
            if (r < nr || (r >= kF && r < kQ && r - kF < tb.nfo) || (r >= kQ && r - kQ < tb.nsrc)) {
                cum += a[r];
                last = (mu < 0 && a[r] > 0.0) ? r : last;
                mu = (mu < 0 && target < cum) ? r : mu;
            }
        }
        mu = mu < 0 ? last : mu;
        uint64_t d = 0;
#pragma unroll
        for (int r = 0; r < kA; ++r)
            if (r < nr || (r >= kF && r < kQ && r - kF < tb.nfo) || (r >= kQ && r - kQ < tb.nsrc))
                d = r == mu ? tb.dn[r] : d;
#pragma unroll
        for (int s = 0; s < S; ++s) cnt_lds[s][lane] += (int32_t)(int8_t)(uint8_t)(d >> (8 * s));
        t = t_next;
        ++j;
    }
    events[m] = j;
}

}  // namespace

void launch_ssa(hipStream_t st, const int32_t* n0, const double* vol, const double* t_rec, int32_t n_rec,
                int32_t* out, long long* events, int32_t n, const SsaTable& tb, uint64_t seed, uint64_t stream0,
                long long max_events) {
    if (n <= 0 || n_rec <= 0 || tb.ns > kOdeMaxSpecies || tb.nr > kSsaMaxReactions) return;
    const dim3 grid((n + 63) / 64), block(64);
    const bool extra = tb.nfo + tb.nsrc > 0;
#define GSBS_SSA_LAUNCH(SL, EX)                                                                                   \
    hipLaunchKernelGGL((k_ssa<SL, EX>), grid, block, 0, st, n0, vol, t_rec, n_rec, out, events, n, tb, seed, stream0, \
                       max_events)
    if (tb.ns <= 4) {
        if (extra) GSBS_SSA_LAUNCH(4, true); else GSBS_SSA_LAUNCH(4, false);
    } else if (tb.ns <= 7) {
        if (extra) GSBS_SSA_LAUNCH(7, true); else GSBS_SSA_LAUNCH(7, false);
    } else {
        if (extra) GSBS_SSA_LAUNCH(kOdeMaxSpecies, true); else GSBS_SSA_LAUNCH(kOdeMaxSpecies, false);
    }
#undef GSBS_SSA_LAUNCH
}

}  // namespace gsbs
