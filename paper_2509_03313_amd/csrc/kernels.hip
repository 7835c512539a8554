// kernels.hip -- gfx950 kernels of one SBS step of the diffusion-reaction
// method of arXiv 2509.03313 (multi-pulse gMicroMC extension):
//
//   k_bin      Brownian jump (Philox4x64-10 + Box-Muller, FP32) and PBC 1
//              (Eq. 1), (cell, species) bin of the moved position, per-bin
//              count and rank (LDS histogram for small grids); the moved
//              position is kept for the scatter
//   k_scan     exclusive scan of the cell counts (one pass, decoupled look-back)
//   k_scatter  molecules into cell order
//   k_pairs    stencil minimum-image (Eq. 2) candidate search against the
//              per-reaction cutoff, radial Brownian-bridge contact
//              probability, pair uniform, accepted pairs appended
//   k_pairs_sp the same search over species bins (late, large cutoffs)
//   k_react    mutual-best single-partner matching by 64-bit atomic min,
//              products of Table 1 appended, reactants removed, species
//              counts updated
//
// All molecules of all instances live in one array; the sort groups them by
// instance (each instance owns a contiguous range of global cells).  Removed
// molecules stay in the array, flagged, until the next sort drops them.
#include <type_traits>

#include "device_common.h"
#include "engine.h"

namespace gsbs {

#define GSBS_BLOCK 256

// ln(u) for u = (k + 1/2) 2^-24, k = top 24 bits of w, to a few FP32 ulps
// relative.  Below the midpoint u = (2k+1) 2^-25 is exact in FP32.  Above it u
// needs 25 bits, but 1 - u = (2^25 - 2k - 1) 2^-25 is exact; u is split as
// w + d with w = fl(1 - (1 - u)) and d = (1 - w) - (1 - u), both differences
// exact (Sterbenz; |d| <= 2^-25), and ln(u) = ln(w) + ln(1 + d/w), where
// ln(1 + d/w) = d/w to within 2^-51.  One logf per value, no log1pf.
__device__ __forceinline__ float ln_u24(uint64_t w) {
    const uint32_t k = (uint32_t)(w >> 40);
    const bool lower = k < (1u << 23);
    const float v = (float)((1u << 25) - 2u * k - 1u) * 0x1p-25f;  // 1 - u (exact above the midpoint)
    const float wu = lower ? (float)(2u * k + 1u) * 0x1p-25f : __fsub_rn(1.0f, v);
    const float d = lower ? 0.0f : __fsub_rn(__fsub_rn(1.0f, wu), v);
    return __fadd_rn(logf(wu), __fmul_rn(d, __builtin_amdgcn_rcpf(wu)));
}

// sin and cos of 2 pi u, u = (k + 1/2) 2^-24: 2 pi u = pi x with x = (2k+1) 2^-24;
// above the midpoint x is folded to 2 - x so the sincospi argument stays exact.
__device__ __forceinline__ void sincos_2pi_u24(uint64_t w, float* s, float* c) {
    const uint32_t k = (uint32_t)(w >> 40);
    const bool lower = k < (1u << 23);  // selected, not branched: one call for the wave
    const uint32_t m = lower ? 2u * k + 1u : (1u << 25) - 2u * k - 1u;
    float ss, cc;
    sincospif((float)m * 0x1p-24f, &ss, &cc);
    *s = lower ? ss : -ss;
    *c = cc;
}

// Position after this step's Brownian jump: Gaussian of variance 2 D dt per
// axis from the Philox block at counter (uid, step, 0, 0), key (seed, instance).
__device__ __forceinline__ float3 jump(float4 p, uint64_t uid, const InstStep& S, int sp) {
    float3 x = make_float3(p.x, p.y, p.z);
    if (!S.active) return x;
    uint64_t w[4];
    philox(uid, S.step, 0ull, 0ull, S.key0, S.key1, w);
    // the hardware root (1 ulp): -2 ln u >= 6e-8, no denormal argument
    const float ra = __builtin_amdgcn_sqrtf(-2.0f * ln_u24(w[0]));
    const float rb = __builtin_amdgcn_sqrtf(-2.0f * ln_u24(w[2]));
    float s1, c1, s3, c3;
    sincos_2pi_u24(w[1], &s1, &c1);
    sincos_2pi_u24(w[3], &s3, &c3);
    const float sg = S.sigma[sp];
    x.x = wrap_f(__fadd_rn(x.x, __fmul_rn(sg, __fmul_rn(ra, c1))), S.L, S.halfL, S.invL);
    x.y = wrap_f(__fadd_rn(x.y, __fmul_rn(sg, __fmul_rn(ra, s1))), S.L, S.halfL, S.invL);
    x.z = wrap_f(__fadd_rn(x.z, __fmul_rn(sg, __fmul_rn(rb, c3))), S.L, S.halfL, S.invL);
    return x;
}

// Cell of a wrapped position: i = min(nc-1, floor((x + L/2) * (nc/L))) per axis,
// FP32 round-to-nearest, no contraction (the oracle emulates it bit for bit).
__device__ __forceinline__ int cell_axis(float x, const InstStep& S) {
    int q = (int)floorf(__fmul_rn(__fadd_rn(x, S.halfL), S.inv_h));
    q = q > S.nc - 1 ? S.nc - 1 : q;
    return q < 0 ? 0 : q;
}

__device__ __forceinline__ int local_cell(float3 x, const InstStep& S) {
    return (cell_axis(x.x, S) * S.nc + cell_axis(x.y, S)) * S.nc + cell_axis(x.z, S);
}

// ------------------------------------------------------------ injection ---
__global__ __launch_bounds__(GSBS_BLOCK) void k_inject(float4* __restrict__ pos, uint64_t* __restrict__ uid,
                                                     long long* __restrict__ counts,
                                                     const DevCounters* __restrict__ ctr,
                                                     const float* __restrict__ xyz,
                                                     const uint8_t* __restrict__ sp, int32_t n,
                                                     int32_t inst, uint64_t uid_base, int32_t cap,
                                                     uint32_t* __restrict__ err) {
    __shared__ int hist[kMaxSpecies];
    if (threadIdx.x < kMaxSpecies) hist[threadIdx.x] = 0;
    __syncthreads();
    const int base = ctr->n_in;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const int s = sp[k];
        const int dst = base + k;
        if (dst >= cap) {
            atomicOr(err, kErrMolOverflow);
            continue;
        }
        pos[dst] = make_float4(xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2], __int_as_float((inst << 8) | s));
        uid[dst] = uid_base + (uint64_t)k;
        atomicAdd(&hist[s & (kMaxSpecies - 1)], 1);
    }
    __syncthreads();
    if (threadIdx.x < kMaxSpecies && hist[threadIdx.x])
        atomicAdd((unsigned long long*)&counts[inst * kMaxSpecies + threadIdx.x],
                  (unsigned long long)hist[threadIdx.x]);
}

__global__ void k_add_n(DevCounters* ctr, int32_t n, int32_t cap) {
    int v = ctr->n_in + n;
    ctr->n_in = v > cap ? cap : v;
}

// ------------------------------------------------------------------ bin ---
constexpr int kScanItems = 16;
constexpr int kScanTile = GSBS_BLOCK * kScanItems;
// Global bin of a moved molecule.
__device__ __forceinline__ uint32_t bin_of(float3 x, const InstStep& S, int sp, int ns) {
    const int c = local_cell(x, S);
    return (uint32_t)(S.bin_base + (S.by_species ? sp * S.nc * S.nc * S.nc + c : c));
}

// Bin of molecule i after its jump; the end position is kept in xnew[i] so
// that the scatter does not draw the jump a second time.
__device__ __forceinline__ uint32_t molecule_bin(const float4* __restrict__ pos, const uint64_t* __restrict__ uid,
                                                 const InstStep* __restrict__ P, int i, int fixed, int ns,
                                                 float4* __restrict__ xnew) {
    const float4 p = pos[i];
    const int meta = __float_as_int(p.w);
    const int sp = meta & 0xFF;
    if (sp == kDead) return kNoCell;
    const InstStep& S = P[meta >> 8];
    const float3 x = fixed ? make_float3(p.x, p.y, p.z) : jump(p, uid[i], S, sp);
    xnew[i] = make_float4(x.x, x.y, x.z, p.w);
    return bin_of(x, S, sp, ns);
}

// Few bins (late, large steps): count in an LDS histogram, one global atomic
// per block and non-empty bin.  Each block owns `per_block` consecutive
// molecules, handled in rounds of GSBS_BLOCK (at most kBinRounds).
constexpr int kBinRounds = 8;

__global__ __launch_bounds__(GSBS_BLOCK) void k_bin_lds(const float4* __restrict__ pos,
                                                      const uint64_t* __restrict__ uid,
                                                      DevCounters* __restrict__ ctr,
                                                      const InstStep* __restrict__ P,
                                                      uint32_t* __restrict__ cell_count,
                                                      uint2* __restrict__ cellrank, float4* __restrict__ xnew,
                                                      int32_t fixed, int32_t total_bins, int32_t ns) {
    extern __shared__ uint32_t hist[];
    for (int b = threadIdx.x; b < total_bins; b += GSBS_BLOCK) hist[b] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->n_pairs = 0u;  // read by k_pairs, after this kernel
    __syncthreads();
    const int n = ctr->n_in;
    const int per_block = ((n + gridDim.x - 1) / gridDim.x + GSBS_BLOCK - 1) / GSBS_BLOCK * GSBS_BLOCK;
    const int first = blockIdx.x * per_block;
    uint32_t bin[kBinRounds], lr[kBinRounds];
#pragma unroll
    for (int r = 0; r < kBinRounds; ++r) {
        const int i = first + r * GSBS_BLOCK + threadIdx.x;
        bin[r] = kNoCell;
        lr[r] = 0u;
        if (r * GSBS_BLOCK < per_block && i < n) {
            bin[r] = molecule_bin(pos, uid, P, i, fixed, ns, xnew);
            if (bin[r] != kNoCell) lr[r] = atomicAdd(&hist[bin[r]], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < total_bins; b += GSBS_BLOCK) {
        const uint32_t c = hist[b];
        if (c) hist[b] = atomicAdd(&cell_count[b], c);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kBinRounds; ++r) {
        const int i = first + r * GSBS_BLOCK + threadIdx.x;
        if (r * GSBS_BLOCK < per_block && i < n)
            cellrank[i] = make_uint2(bin[r], bin[r] == kNoCell ? 0u : hist[bin[r]] + lr[r]);
    }
}

// Many bins (early, small steps): one global atomic per run of equal bins among
// consecutive lanes (the input is still sorted from the previous step, so a
// spur's molecules mostly form one run).
__global__ __launch_bounds__(GSBS_BLOCK) void k_bin(const float4* __restrict__ pos,
                                                  const uint64_t* __restrict__ uid,
                                                  DevCounters* __restrict__ ctr,
                                                  const InstStep* __restrict__ P,
                                                  uint32_t* __restrict__ cell_count,
                                                  uint2* __restrict__ cellrank, float4* __restrict__ xnew,
                                                  int32_t fixed, int32_t ns) {
    const int n = ctr->n_in;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->n_pairs = 0u;  // read by k_pairs, after this kernel
    const int lane = threadIdx.x & 63;
    const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int i = base + threadIdx.x;
        const bool valid = i < n;
        const uint32_t bin = valid ? molecule_bin(pos, uid, P, i, fixed, ns, xnew) : kNoCell;
        const uint32_t prev = wave_prev(bin, kNoCell);
        const bool head = (lane == 0) || (prev != bin);
        const unsigned long long heads = __ballot(head);
        const int start = 63 - __clzll(heads & upto);
        const unsigned long long above = heads & ~upto;
        const int next = above ? __ffsll((long long)above) - 1 : 64;
        uint32_t b0 = 0u;
        if (head && bin != kNoCell) b0 = atomicAdd(&cell_count[bin], (uint32_t)(next - lane));
        b0 = __shfl(b0, start, 64);
        if (valid) cellrank[i] = make_uint2(bin, bin == kNoCell ? 0u : b0 + (uint32_t)(lane - start));
    }
}

// ----------------------------------------------------------------- scan ---


// exclusive scan of one value per thread over the block; *total gets the sum
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t wsum[GSBS_BLOCK / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < GSBS_BLOCK / 64; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// Single-pass scan with decoupled look-back: each tile publishes its total,
// then wave 0 walks back over the status words of the tiles before it (64 at a
// time) until it meets one that carries an inclusive prefix.  A status word is
// (epoch: 31 bits, inclusive flag, value: 32 bits); words of other steps never
// match the epoch, so the array is not cleared between steps.  Tiles wait only
// on tiles with lower indices, which are dispatched first.
__device__ __forceinline__ unsigned long long scan_word(uint32_t epoch, uint32_t incl, uint32_t v) {
    return ((unsigned long long)((epoch << 1) | incl) << 32) | v;
}

__global__ __launch_bounds__(GSBS_BLOCK) void k_scan(uint32_t* __restrict__ cnt, int32_t total,
                                                   unsigned long long* __restrict__ status, uint32_t epoch,
                                                   uint32_t* __restrict__ start, DevCounters* __restrict__ ctr) {
    __shared__ uint32_t s_prefix;
    const int b = blockIdx.x;
    const int base = b * kScanTile + threadIdx.x * kScanItems;
    const bool whole = base + kScanItems <= total;  // 16-byte vector accesses (the arrays are 256-byte aligned)
    uint32_t v[kScanItems];
    uint32_t sum = 0;
    if (whole) {
#pragma unroll
        for (int k = 0; k < kScanItems; k += 4) {
            const uint4 q = *reinterpret_cast<const uint4*>(cnt + base + k);
            v[k] = q.x, v[k + 1] = q.y, v[k + 2] = q.z, v[k + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = base + k < total ? cnt[base + k] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) sum += v[k];
    uint32_t blk_total;
    const uint32_t excl = block_excl_scan(sum, &blk_total);
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        uint32_t prefix = 0;
        if (b > 0) {
            if (lane == 0)
                __hip_atomic_store(&status[b], scan_word(epoch, 0u, blk_total), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            for (int j0 = b - 1;; j0 -= 64) {
                const int j = j0 - lane;
                unsigned long long w = scan_word(epoch, 1u, 0u);  // before tile 0: an inclusive zero
                if (j >= 0) {
                    // bounded: a stall is reported instead of hanging the device
                    for (int spin = 0;; ++spin) {
                        w = __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if ((uint32_t)(w >> 33) == epoch) break;
                        if (spin > (1 << 20)) {
                            atomicOr(&ctr->err, kErrScanStall);
                            w = scan_word(epoch, 1u, 0u);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                const unsigned long long incl = __ballot(((w >> 32) & 1ull) != 0ull);
                const int stop = incl ? __ffsll((long long)incl) - 1 : 64;  // nearest inclusive word
                const uint32_t part = lane <= stop ? (uint32_t)w : 0u;
                prefix += (uint32_t)wave_last((int)wave_incl_scan(part));
                if (incl) break;
            }
        }
        if (lane == 0) {
            __hip_atomic_store(&status[b], scan_word(epoch, 1u, prefix + blk_total), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            s_prefix = prefix;
        }
    }
    __syncthreads();
    const uint32_t tile_off = s_prefix;
    uint32_t run = tile_off + excl;
    if (whole) {
#pragma unroll
        for (int k = 0; k < kScanItems; k += 4) {
            uint4 q;
            q.x = run;
            run += v[k];
            q.y = run;
            run += v[k + 1];
            q.z = run;
            run += v[k + 2];
            q.w = run;
            run += v[k + 3];
            *reinterpret_cast<uint4*>(start + base + k) = q;
            *reinterpret_cast<uint4*>(cnt + base + k) = make_uint4(0u, 0u, 0u, 0u);
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int c = base + k;
            if (c < total) {
                start[c] = run;
                cnt[c] = 0u;
            }
            run += v[k];
        }
    }
    if (b == gridDim.x - 1 && threadIdx.x == 0) {
        start[total] = tile_off + blk_total;
        ctr->n_live = (int32_t)(tile_off + blk_total);
    }
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int32_t n, unsigned long long v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// -------------------------------------------------------------- scatter ---
__global__ __launch_bounds__(GSBS_BLOCK) void k_scatter(const float4* __restrict__ pos,
                                                      const uint64_t* __restrict__ uid,
                                                      const DevCounters* __restrict__ ctr,
                                                      const float4* __restrict__ xnew,
                                                      const uint2* __restrict__ cellrank,
                                                      const uint32_t* __restrict__ start,
                                                      float4* __restrict__ pos_out,
                                                      float4* __restrict__ pos0_out,
                                                      uint64_t* __restrict__ uid_out,
                                                      const float4* __restrict__ x0_override) {
    const int n = ctr->n_in;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint2 cr = cellrank[i];
        if (cr.x == kNoCell) continue;
        const float4 p = pos[i];
        const uint64_t u = uid[i];
        const uint32_t dst = start[cr.x] + cr.y;
        const float4 x = xnew[i];
        const float4 p0 = x0_override ? x0_override[i] : p;
        pos_out[dst] = x;
        pos0_out[dst] = make_float4(p0.x, p0.y, p0.z, __uint_as_float(cr.x));  // bin index
        uid_out[dst] = u;
    }
}

// ---------------------------------------------------------- pair search ---
// Orders LDS accesses of the lanes of one wave (no workgroup barrier needed).
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Probability that the pair touched R during the step given start/end
// separations r0, r1 (radial Brownian bridge; method of images for the pair
// density of the supplement), inv_s = 1 / (D_AB dt).
__device__ __forceinline__ float bridge_f(float r0, float r1, float R, float inv_s) {
    if (r0 <= R || r1 <= R) return 1.0f;
    const float a = (r0 - R) * (r1 - R) * inv_s;
    const float b = R * (r0 + r1 - R) * inv_s;
    const float c = r0 * r1 * inv_s;
    return expf(-a) * (expm1f(-b) / expm1f(-c));
}

// One candidate pair (i, j) of reaction rx: minimum-image end separation
// below the cutoff (FP32, fixed operation order), contact probability, pair
// uniform, accepted pairs appended.
// Squared minimum-image end separation in FP32 with a fixed operation order
// (the oracle emulates it bit for bit).
__device__ __forceinline__ float end_d2(const float4& pj, const float4& pi, float L, float hL) {
    const float dx = minimg_f(__fsub_rn(pj.x, pi.x), L, hL);
    const float dy = minimg_f(__fsub_rn(pj.y, pi.y), L, hL);
    const float dz = minimg_f(__fsub_rn(pj.z, pi.z), L, hL);
    return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

// A candidate (end separation below the cutoff): start separation, contact
// probability, pair uniform, accepted pair appended.
__device__ __forceinline__ void eval_candidate(int i, int j, float d2, const float4* __restrict__ pos0,
                                               const uint64_t* __restrict__ uid, const InstStep& S, int rx,
                                               int contact_only, int log_all, DevCounters* __restrict__ ctr,
                                               PairRec* __restrict__ pairs, uint32_t pair_cap) {
    const float L = S.L, hL = S.halfL;
    const float4 qi = pos0[i];
    const float4 qj = pos0[j];
    const float ex = minimg_f(qj.x - qi.x, L, hL);
    const float ey = minimg_f(qj.y - qi.y, L, hL);
    const float ez = minimg_f(qj.z - qi.z, L, hL);
    const float r1 = sqrtf(d2);
    const float r0 = sqrtf(ex * ex + ey * ey + ez * ez);
    const float R = S.R[rx];
    float Pc;
    if (contact_only) {
        Pc = (r0 <= R || r1 <= R) ? 1.0f : 0.0f;
    } else {
        // exp(-a) bounds P; below 1.5e-8 no 24-bit uniform can fall under P
        const float a = (r0 - R) * (r1 - R) * S.inv_s[rx];
        if (!log_all && r0 > R && r1 > R && a > 18.0f) return;
        Pc = bridge_f(r0, r1, R, S.inv_s[rx]);
    }
    if (!log_all && !(Pc > 0x1p-25f)) return;
    const uint64_t ui = uid[i], uj = uid[j];
    const uint64_t lo = ui < uj ? ui : uj, hi = ui < uj ? uj : ui;
    uint64_t w[4];
    philox(lo, hi, S.step, 1ull, S.key0, S.key1, w);
    const uint32_t u24 = (uint32_t)(w[0] >> 40);
    // u = (2 u24 + 1) 2^-25 < P, compared exactly in FP64
    const bool acc = (double)(2u * u24 + 1u) * 0x1p-25 < (double)Pc;
    if (acc || log_all) {
        const uint32_t k = atomicAdd(&ctr->n_pairs, 1u);
        if (k < pair_cap) {
            PairRec r;
            r.i = i;
            r.j = j;
            r.u24 = u24;
            r.rx = rx;
            r.P = Pc;
            r.flags = acc ? 1 : 0;
            pairs[k] = r;
        } else {
            atomicOr(&ctr->err, kErrPairOverflow);
        }
    }
}

__device__ __forceinline__ void test_pair(int i, int j, const float4& pi, const float4* __restrict__ pos,
                                          const float4* __restrict__ pos0, const uint64_t* __restrict__ uid,
                                          const InstStep& S, int rx, float rc2, int contact_only, int log_all,
                                          DevCounters* __restrict__ ctr, PairRec* __restrict__ pairs,
                                          uint32_t pair_cap, unsigned long long& ncand) {
    const float d2 = end_d2(pos[j], pi, S.L, S.halfL);
    if (!(d2 < rc2)) return;
    ++ncand;
    eval_candidate(i, j, d2, pos0, uid, S, rx, contact_only, log_all, ctr, pairs, pair_cap);
}

// Lower bound of the distance along one axis from x to the cell `o` cells away
// from its own cell q (unwrapped), minus a slack for FP32 binning.
__device__ __forceinline__ float cell_gap(float x, int q, int o, float h, float hL, float eps) {
    float g = 0.0f;
    if (o > 0) g = (float)(q + o) * h - hL - x;
    else if (o < 0) g = x - ((float)(q + o + 1) * h - hL);
    g -= eps;
    return g > 0.0f ? g : 0.0f;
}

// Offsets [lo, hi] within +-m along one axis whose cells can hold a partner of
// x (cell q) within reach_d: the slab k cells below starts (k - 1) h beyond the
// distance from x to its cell's lower face, likewise above.
__device__ __forceinline__ void stencil_range(float x, int q, float h, float inv_h, float hL, float reach_d, int m,
                                              int& lo, int& hi) {
    const float a = x - ((float)q * h - hL);        // to the lower face
    const float b = ((float)(q + 1) * h - hL) - x;  // to the upper face
    const float ta = reach_d - a, tb = reach_d - b;
    lo = ta < 0.0f ? 0 : -min(m, (int)floorf(ta * inv_h) + 1);
    hi = tb < 0.0f ? 0 : min(m, (int)floorf(tb * inv_h) + 1);
}

__device__ __forceinline__ int wrap_cell(int c, int nc) { return c < 0 ? c + nc : (c >= nc ? c - nc : c); }

// Out of line: candidates are rare in the whole-cell search and the
// evaluation's registers would otherwise cap the occupancy of its loops.
__device__ __noinline__ void eval_candidate_call(int i, int j, float d2, const float4* __restrict__ pos0,
                                                 const uint64_t* __restrict__ uid, const InstStep& S, int rx,
                                                 int contact_only, int log_all, DevCounters* __restrict__ ctr,
                                                 PairRec* __restrict__ pairs, uint32_t pair_cap) {
    eval_candidate(i, j, d2, pos0, uid, S, rx, contact_only, log_all, ctr, pairs, pair_cap);
}

// Molecules [j0, j1) of one cell against molecule i, four loads in flight at a time.
// The same without Eq. 2, for two molecules known to be less than L/2 apart
// along every axis (Eq. 2 is then the identity): identical FP32 result.
__device__ __forceinline__ float sep2(const float4& pj, const float4& pi) {
    const float dx = __fsub_rn(pj.x, pi.x), dy = __fsub_rn(pj.y, pi.y), dz = __fsub_rn(pj.z, pi.z);
    return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

// Molecules j0 .. j1-1 of the sorted array against molecule i.  cpre bounds
// every cutoff of i's species from above, so the per-partner cutoff lookups
// (dependent loads) run only for the rare pairs that pass it.
template <bool kEq2 = true>
__device__ __forceinline__ void scan_run(int i, const float4& pi, int j0, int j1, float cpre, float L, float hL,
                                         const float4* __restrict__ pos, const float4* __restrict__ pos0,
                                         const uint64_t* __restrict__ uid, const InstStep& S, const int* row,
                                         int contact_only, int log_all, DevCounters* __restrict__ ctr,
                                         PairRec* __restrict__ pairs, uint32_t pair_cap, unsigned long long& ncand) {
    for (int j = j0; j < j1; j += 4) {
        float4 q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = (j + u < j1) ? pos[j + u] : make_float4(0.f, 0.f, 0.f, 0.f);
        float d2v[4];
        int rxv[4];
        uint32_t m = 0u;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            d2v[u] = kEq2 ? end_d2(q[u], pi, L, hL) : sep2(q[u], pi);
            rxv[u] = -1;
            if (j + u < j1 && d2v[u] < cpre) {
                rxv[u] = row[__float_as_int(q[u].w) & 0xFF];
                if (rxv[u] >= 0 && d2v[u] < S.rc2[rxv[u]]) m |= 1u << u;
            }
        }
        while (m) {  // one evaluation site for the (rare) candidates
            const int u = __ffs(m) - 1;
            m &= m - 1u;
            const float d2 = u == 0 ? d2v[0] : (u == 1 ? d2v[1] : (u == 2 ? d2v[2] : d2v[3]));
            const int rx = u == 0 ? rxv[0] : (u == 1 ? rxv[1] : (u == 2 ? rxv[2] : rxv[3]));
            ++ncand;
            eval_candidate_call(i, j + u, d2, pos0, uid, S, rx, contact_only, log_all, ctr, pairs, pair_cap);
        }
    }
}

// Whole-cell search (small cells, few molecules each): one thread per sorted
// molecule; a pair is searched from the molecule in the lower cell (or with the
// lower index in one cell).  Each wave first stages the 128 sorted molecules
// from its first one into LDS, so the partners in a molecule's own cell --
// contiguous in sorted order, and most of the work when the cutoff is small
// against the cell -- are read from LDS; the rest of a very full cell and the
// stencil cells come from global memory.  Cells whose distance from the
// molecule exceeds the largest cutoff of its species are skipped.
constexpr int kWin = 128;

constexpr int kNbrQ = 256;  // neighbour-cell items queued per wave


__global__ __launch_bounds__(GSBS_BLOCK, 4) void k_pairs(const float4* __restrict__ pos,
                                                       const float4* __restrict__ pos0,
                                                       const uint64_t* __restrict__ uid,
                                                       DevCounters* __restrict__ ctr,
                                                       const InstStep* __restrict__ P,
                                                       const ChemDev* __restrict__ chem,
                                                       const uint32_t* __restrict__ start,
                                                       PairRec* __restrict__ pairs, uint32_t pair_cap,
                                                       int32_t log_all, int32_t ns) {
    __shared__ int32_t rmap[kMaxSpecies * kMaxSpecies];
    __shared__ unsigned long long s_cand;
    __shared__ float4 wpos_all[GSBS_BLOCK / 64][kWin];
    __shared__ uint32_t wbin_all[GSBS_BLOCK / 64][kWin];
    __shared__ unsigned long long nq_all[GSBS_BLOCK / 64][kNbrQ];  // (global bin << 7) | (needs Eq. 2 << 6) | lane
    __shared__ int2 qinfo_all[GSBS_BLOCK / 64][kNbrQ];  // queued item: first partner, inclusive end of its tests
    __shared__ int4 cq_all[GSBS_BLOCK / 64][128];       // candidates: i, j, bits of d2, (instance << 6) | reaction
    __shared__ float rc2s[kMaxSpecies * kMaxSpecies];  // squared cutoffs of the home instance, -1: no reaction
    __shared__ float hs_f[5 + kMaxSpecies];            // home instance: L, L/2, h, cull_eps, 1/h, cull2_all[]
    __shared__ int hs_i[4];                            // home instance: nc, reach, bin_base, searched here
    __shared__ int home_s;
    for (int k = threadIdx.x; k < kMaxSpecies * kMaxSpecies; k += blockDim.x)
        rmap[k] = chem->rmap[k / kMaxSpecies][k % kMaxSpecies];
    if (threadIdx.x == 0) s_cand = 0ull;
    __syncthreads();
    const uint32_t reactive = chem->reactive_mask;
    const int contact_only = chem->contact_only;
    const int n = ctr->n_live;
    const int lane = threadIdx.x & 63;
    float4* wpos = wpos_all[threadIdx.x >> 6];
    uint32_t* wbin = wbin_all[threadIdx.x >> 6];
    unsigned long long* nq = nq_all[threadIdx.x >> 6];
    int2* qinfo = qinfo_all[threadIdx.x >> 6];
    int4* cq = cq_all[threadIdx.x >> 6];
    int cqn = 0;  // wave-uniform length of the candidate queue
    unsigned long long ncand = 0;
    // Candidates of the balanced walks are queued and evaluated 64 at a time, one
    // per lane (start separation, bridge probability, Philox pair uniform), so
    // that the evaluation does not run once per candidate with the other lanes
    // idle.  Every lane of the wave calls these.
    auto cand_flush = [&](bool all) {
        while (cqn >= 64 || (all && cqn > 0)) {
            wave_sync_lds();
            const int take = cqn < 64 ? cqn : 64;
            const int rest = cqn - take;
            int4 e = make_int4(0, 0, 0, 0), r = make_int4(0, 0, 0, 0);
            if (lane < take) e = cq[lane];
            if (lane < rest) r = cq[64 + lane];
            wave_sync_lds();
            if (lane < rest) cq[lane] = r;
            cqn = rest;
            if (lane < take)
                eval_candidate_call(e.x, e.y, __int_as_float(e.z), pos0, uid, P[e.w >> 6], e.w & 63, contact_only,
                                    log_all, ctr, pairs, pair_cap);
        }
    };
    auto cand_push = [&](bool c, int ci, int cj, float d2, int inst_c, int rx) {
        const unsigned long long m = __ballot(c);
        if (m == 0ull) return;
        if (c) cq[cqn + (int)__popcll(m & ((1ull << lane) - 1ull))] = make_int4(ci, cj, __float_as_int(d2), (inst_c << 6) | rx);
        cqn += (int)__popcll(m);
        if (cqn >= 64) cand_flush(false);
    };
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int i0 = base + (threadIdx.x & ~63);
        const int i = i0 + lane;
        // the wave's window of 128 sorted molecules, loaded before anything that
        // depends on it; the block's home instance (that of its first molecule, the
        // first window entry of thread 0) gets its step parameters and cutoffs in
        // LDS, so that molecules of that instance -- nearly all -- read no step
        // parameters from global memory
        float4 wv[kWin / 64];
        uint32_t wb[kWin / 64];
#pragma unroll
        for (int h2 = 0; h2 < kWin / 64; ++h2) {
            const int j = i0 + 64 * h2 + lane;
            wv[h2] = make_float4(0.f, 0.f, 0.f, 0.f);
            wb[h2] = kNoCell;
            if (j < n) {
                wv[h2] = pos[j];
                wb[h2] = __float_as_uint(pos0[j].w);
            }
        }
        __syncthreads();  // the previous iteration is done with the block's tables
        if (threadIdx.x == 0) home_s = __float_as_int(wv[0].w) >> 8;
        __syncthreads();
        const int home = home_s;
        {
            const InstStep& H = P[home];
            const int t = threadIdx.x;
            if (t < kMaxSpecies * kMaxSpecies) rc2s[t] = rmap[t] >= 0 ? H.rc2[rmap[t]] : -1.0f;
            if (t >= 64 && t < 64 + kMaxSpecies) hs_f[5 + t - 64] = H.cull2_all[t - 64];
            if (t == 128) {
                hs_f[0] = H.L;
                hs_f[1] = H.halfL;
                hs_f[2] = H.h;
                hs_f[3] = H.cull_eps;
                hs_f[4] = H.inv_h;
            }
            if (t == 192) {
                hs_i[0] = H.nc;
                hs_i[1] = H.reach;
                hs_i[2] = H.bin_base;
                hs_i[3] = (H.active && !H.by_species) ? 1 : 0;
            }
        }
#pragma unroll
        for (int h2 = 0; h2 < kWin / 64; ++h2) {
            wpos[64 * h2 + lane] = wv[h2];
            wbin[64 * h2 + lane] = wb[h2];
        }
        __syncthreads();
        // lanes without work stay in the loop: the neighbour queue below works in lockstep
        const float4 pi = wpos[lane];
        const int mi = __float_as_int(pi.w);
        const int si = mi & 0xFF;
        const int inst = i < n ? (mi >> 8) : home;
        const InstStep& S = P[inst];
        float sL, sHL, sH, sEps, sInvH, cmax;
        int sNc, sReach, sBase;
        bool sOk;
        if (inst == home) {
            sL = hs_f[0], sHL = hs_f[1], sH = hs_f[2], sEps = hs_f[3], sInvH = hs_f[4];
            cmax = hs_f[5 + (si & (kMaxSpecies - 1))];
            sNc = hs_i[0], sReach = hs_i[1], sBase = hs_i[2], sOk = hs_i[3] != 0;
        } else {
            sL = S.L, sHL = S.halfL, sH = S.h, sEps = S.cull_eps, sInvH = S.inv_h;
            cmax = S.cull2_all[si & (kMaxSpecies - 1)];
            sNc = S.nc, sReach = S.reach, sBase = S.bin_base, sOk = S.active && !S.by_species;
        }
        const bool act = i < n && ((reactive >> si) & 1u) && sOk;
        if (!act) cmax = -1.0f;  // bounds every cutoff of the species
        const int* row = rmap + (si & (kMaxSpecies - 1)) * kMaxSpecies;
        const uint32_t bi = wbin[lane];
        const int cg = (int)bi - sBase;  // local cell
        // End of this lane's bin inside the window: the first position q >= lane whose
        // successor lies in another bin (position kWin - 1 always ends a run)
        const unsigned long long ends_lo = __ballot(wbin[lane] != wbin[lane + 1]);
        const unsigned long long ends_hi = __ballot(lane == 63 || wbin[lane + 64] != wbin[min(lane + 65, kWin - 1)]);
        const unsigned long long mine = ends_lo & (~0ull << lane);
        const int run_end = 1 + (mine ? __ffsll((long long)mine) - 1 : 64 + __ffsll((long long)ends_hi) - 1);
        // Own-cell pairs.  Among the lanes of one run (a bin, possibly begun in the
        // wave before) each pair is taken once, cyclically: lane r of c takes the
        // members r+1 .. r+(c-1)/2 (mod c), and for even c the first c/2 lanes also
        // take r + c/2 -- every lane does about c/2 tests instead of c-1-r.  Members
        // after the lanes (window positions 64 .. run_end-1, then beyond the window)
        // are taken by every lane of the run.
        const unsigned long long heads = __ballot(lane == 0 || wbin[lane] != wbin[max(lane - 1, 0)]);
        const int run_beg = 63 - __clzll(heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull)));
        const int run_lanes = min(run_end, 64) - run_beg;
        const int rel = lane - run_beg;
        const int ncyc = (run_lanes - 1) / 2 + (((run_lanes & 1) == 0 && rel < run_lanes / 2) ? 1 : 0);
        const int nown = ncyc + (run_end > 64 ? run_end - 64 : 0);
        auto own_partner = [&](int t) {
            const int q = rel + 1 + t;
            const int kc = run_beg + (q >= run_lanes ? q - run_lanes : q);
            return t >= ncyc ? 64 + (t - ncyc) : kc;
        };
        // Own-cell pairs of the home instance's molecules: each lane takes its
        // nown cyclic partners in its run (then the run's members at window
        // positions 64 ..), four at a time with their LDS reads in flight
        // together, in a loop as long as the wave's longest list; candidates go
        // to the wave's queue.  The largest cutoff of the owner's species screens
        // each partner before its own cutoff is looked up.  Two molecules of one
        // cell are less than a cell width apart, below L/2 once an edge holds 3
        // cells: Eq. 2 then changes nothing and is skipped.
        {
            const int mown = (act && inst == home) ? nown : 0;
            const int wmax = wave_max_i(mown);
            if (wmax > 0) {
                const float* rcrow = rc2s + (si & (kMaxSpecies - 1)) * kMaxSpecies;
                auto own_loop = [&](auto plain_tag) {
                    constexpr bool kPlain = decltype(plain_tag)::value;
                    for (int t0 = 0; t0 < wmax; t0 += 4) {
                        float4 pj[4];
                        int kk[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            kk[u] = own_partner(min(t0 + u, max(mown - 1, 0)));
                            pj[u] = wpos[kk[u]];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const float d2 = kPlain ? sep2(pj[u], pi) : end_d2(pj[u], pi, sL, sHL);
                            bool cnd = false;
                            int crx = 0;
                            if (t0 + u < mown && d2 < cmax) {  // rare
                                const int sj = __float_as_int(pj[u].w) & 0xFF;
                                if (d2 < rcrow[sj]) {
                                    ++ncand;
                                    cnd = true;
                                    crx = row[sj];
                                }
                            }
                            cand_push(cnd, i, i0 + kk[u], d2, home, crx);
                        }
                    }
                };
                if (hs_i[0] >= 3) own_loop(std::true_type{});
                else own_loop(std::false_type{});
            }
        }
        if (act) {
            if (inst != home) {  // a block straddling two instances: per-lane loop
                for (int t = 0; t < nown; ++t) {
                    const int k = own_partner(t);
                    const float4 pj = wpos[k];
                    const float d2 = end_d2(pj, pi, sL, sHL);
                    if (!(d2 < cmax)) continue;
                    const int rx = row[__float_as_int(pj.w) & 0xFF];
                    if (rx < 0 || !(d2 < S.rc2[rx])) continue;
                    ++ncand;
                    eval_candidate_call(i, i0 + k, d2, pos0, uid, S, rx, contact_only, log_all, ctr, pairs,
                                        pair_cap);
                }
            }
            if (run_end == kWin)  // the bin may continue past the window
                scan_run<true>(i, pi, i0 + kWin, (int)start[bi + 1], cmax, sL, sHL, pos, pos0, uid, S, row,
                               contact_only, log_all, ctr, pairs, pair_cap, ncand);
        }
        // stencil cells after the own cell in cell order: along each axis only the
        // offsets whose slab can lie within the species' largest cutoff; every lane
        // walks its own offsets (the wave as long as its longest list) and queues
        // (molecule, cell) items, then the queued cells are scanned one item per lane
        const int nc = sNc, m = sReach;
        // the molecule's cell, by the binning's own arithmetic on the same position
        auto axis_cell = [&](float x) {
            const int q = (int)floorf(__fmul_rn(__fadd_rn(x, sHL), sInvH));
            return q > nc - 1 ? nc - 1 : (q < 0 ? 0 : q);
        };
        const int ix = axis_cell(pi.x), iy = axis_cell(pi.y), iz = axis_cell(pi.z);
        const bool full = nc < 2 * m + 1;  // the stencil covers each axis entirely
        const float h = sH, hL = sHL, eps = sEps;
        int xlo = 1, xhi = 0, ylo = 1, yhi = 0, zlo = 1, zhi = 0;  // empty for idle lanes
        if (act) {
            if (full) {  // every cell along each axis, as offsets 0 .. nc-1 taken modulo nc
                xlo = ylo = zlo = 0;
                xhi = yhi = zhi = nc - 1;
            } else {
                // generous (hardware root, quotients by a product): the gap tests decide
                const float reach_d = __builtin_amdgcn_sqrtf(cmax) + eps + 1e-3f * h;
                stencil_range(pi.x, ix, h, sInvH, hL, reach_d, m, xlo, xhi);
                stencil_range(pi.y, iy, h, sInvH, hL, reach_d, m, ylo, yhi);
                stencil_range(pi.z, iz, h, sInvH, hL, reach_d, m, zlo, zhi);
            }
        }
        const int nxr = xhi - xlo + 1, nyr = yhi - ylo + 1, nzr = zhi - zlo + 1;
        const int nitem = act ? nxr * nyr * nzr : 0;
        const int witem = wave_max_i(nitem);
        int qn = 0;
        // The queued (molecule, cell) items, scanned with the work spread evenly
        // over the wave: item e holds the tests of its molecule against every
        // molecule of its cell; the tests of all items are cut into 64 contiguous
        // chunks, one per lane, walked four at a time (their loads in flight
        // together), the item changing where its range ends.  Eq. 2 is applied
        // when some item needs it (a wrapped cell, or a grid too small for
        // neighbour cells to stay within L/2): elsewhere it is the identity.
        auto drain = [&]() {
            wave_sync_lds();
            int carry = 0;
            bool eq2 = false;
            for (int e0 = 0; e0 < qn; e0 += 64) {
                const bool has = e0 + lane < qn;
                const unsigned long long it = has ? nq[e0 + lane] : 0ull;
                int j0 = 0, cnt = 0;
                if (has) {
                    const int b = (int)(it >> 7);
                    j0 = (int)start[b];
                    cnt = (int)start[b + 1] - j0;
                }
                eq2 = eq2 || __ballot(has && ((it >> 6) & 1ull)) != 0ull;
                const int inc = (int)wave_incl_scan((uint32_t)cnt) + carry;
                if (has) qinfo[e0 + lane] = make_int2(j0, inc);
                carry = wave_last(inc);
            }
            const int T = carry;
            wave_sync_lds();
            auto walk = [&](auto eq2_tag) {
                constexpr bool kEq2 = decltype(eq2_tag)::value;
                const int c0 = (int)(((long long)T * lane) >> 6), c1 = (int)(((long long)T * (lane + 1)) >> 6);
                const int iters = ((T + 63) / 64 + 1) / 2;  // pairs of tests in the longest chunk
                int e = 0, ebeg = 0, t = 0;
                int2 qi = make_int2(0, 0);
                if (c0 < c1) {
                    int lo = 0, hi = qn - 1;  // the first item whose range ends after c0
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (qinfo[mid].y > c0) hi = mid;
                        else lo = mid + 1;
                    }
                    e = lo;
                    qi = qinfo[e];
                    ebeg = e ? qinfo[e - 1].y : 0;  // first test of item e
                    t = c0 - ebeg;
                }
                int ecur = -1;  // item whose molecule data are loaded
                float4 pm = make_float4(0.f, 0.f, 0.f, 0.f);
                float cm = 0.0f, Lm = 0.0f, hLm = 0.0f;
                int im = 0, rowo = 0, ml = 0;
                for (int it = 0; it < iters; ++it) {
                    const int g0 = c0 + 2 * it;
                    int eu[2], ju[2];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        eu[u] = -1;
                        ju[u] = 0;
                        if (g0 + u < c1) {
                            while (ebeg + t >= qi.y) {  // next item with tests
                                ebeg = qi.y;
                                ++e;
                                qi = qinfo[e];
                                t = 0;
                            }
                            eu[u] = e;
                            ju[u] = qi.x + t;
                            ++t;
                        }
                    }
                    float4 pj[2];
#pragma unroll
                    for (int u = 0; u < 2; ++u) pj[u] = eu[u] >= 0 ? pos[ju[u]] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        bool cnd = false;
                        int crx = 0;
                        float cd2 = 0.0f;
                        if (eu[u] >= 0) {
                            if (eu[u] != ecur) {
                                ecur = eu[u];
                                ml = (int)(nq[ecur] & 63ull);
                                pm = wpos[ml];
                                const int mm = __float_as_int(pm.w);
                                const int sm = mm & (kMaxSpecies - 1);
                                im = mm >> 8;
                                rowo = sm * kMaxSpecies;
                                if (im == home) {
                                    cm = hs_f[5 + sm], Lm = hs_f[0], hLm = hs_f[1];
                                } else {
                                    cm = P[im].cull2_all[sm], Lm = P[im].L, hLm = P[im].halfL;
                                }
                            }
                            const float d2 = kEq2 ? end_d2(pj[u], pm, Lm, hLm) : sep2(pj[u], pm);
                            if (d2 < cm) {  // rare
                                const int rx = rmap[rowo + (__float_as_int(pj[u].w) & 0xFF)];
                                if (rx >= 0 && d2 < P[im].rc2[rx]) {
                                    ++ncand;
                                    cnd = true;
                                    crx = rx;
                                    cd2 = d2;
                                }
                            }
                        }
                        cand_push(cnd, i0 + ml, ju[u], cd2, im, crx);
                    }
                }
            };
            if (T > 0) {
                if (eq2) walk(std::true_type{});
                else walk(std::false_type{});
            }
            wave_sync_lds();
            qn = 0;
        };
        int ox = xlo, oy = ylo, oz = zlo;  // this lane's item it, counted up without divisions
        // neighbour cells that are not wrapped lie within (m + 1) cells along every
        // axis: less than L/2 apart once an edge holds 2m + 3 cells
        const bool near_ok = !full && nc >= 2 * m + 3;
        for (int it = 0; it < witem; ++it) {
            bool need = false, wrapped = false;
            int c2 = 0;
            if (it < nitem) {
                const int qx = wrap_cell(ix + ox, nc), qy = wrap_cell(iy + oy, nc), qz = wrap_cell(iz + oz, nc);
                wrapped = qx != ix + ox || qy != iy + oy || qz != iz + oz;
                const float gx = full ? 0.0f : cell_gap(pi.x, ix, ox, h, hL, eps);
                const float gy = full ? 0.0f : cell_gap(pi.y, iy, oy, h, hL, eps);
                const float gz = full ? 0.0f : cell_gap(pi.z, iz, oz, h, hL, eps);
                c2 = (qx * nc + qy) * nc + qz;
                need = !(gx * gx + gy * gy + gz * gz > cmax) && c2 > cg;
                if (++oz > zhi) {
                    oz = zlo;
                    if (++oy > yhi) {
                        oy = ylo;
                        ++ox;
                    }
                }
            }
            const unsigned long long bal = __ballot(need);
            if (bal) {
                if (need)
                    nq[qn + __popcll(bal & ((1ull << lane) - 1ull))] =
                        ((unsigned long long)(uint32_t)(sBase + c2) << 7) |
                        ((wrapped || !near_ok) ? 64ull : 0ull) | (unsigned long long)lane;
                qn += __popcll(bal);
            }
            // one call site of the drain: when the queue is nearly full, and after the last item
            if (qn > kNbrQ - 64 || (it + 1 == witem && qn > 0)) drain();
        }
        cand_flush(true);  // the window and its wave's tables are reused by the next iteration
    }
    for (int d = 32; d >= 1; d >>= 1) ncand += __shfl_xor(ncand, d, 64);
    if (lane == 0 && ncand) atomicAdd(&s_cand, ncand);
    __syncthreads();
    if (threadIdx.x == 0 && s_cand) atomicAdd(&ctr->cand, s_cand);
}

// ------------------------------------------------ species-bin pair search ---
// Large cells (many molecules per cell).  Bins are species-major (bin =
// bin_base + species * nc^3 + cell, cell = (ix*nc + iy)*nc + iz), so the
// molecules of one species along a z-run of cells are contiguous.
//
// Work item: species s, a box of kx*ky*kz cells (the A unit, about 50
// molecules of s) and one of nsplit slices of the partner stream.  A wave
// holds the A molecules one per lane and takes their bounding box.  For every
// partner species t searched from s, the box widened by the pair's cutoff
// gives a rectangle of (x, y) cell rows; 64 rows at a time are culled in
// parallel (one per lane) by their distance from the box, each kept row gets
// the z-window that the rest of the cutoff allows, and its z-runs of cells
// (two when the window wraps) become segments of the partner stream.  The
// wave takes its slice of the concatenated stream and stages it 64 molecules
// at a time through LDS (the next stage's loads are in flight while one is
// tested).  Every lane tests its A molecule against every staged B in a fully
// unrolled loop (64-bit candidate mask); the candidates are then compacted into
// an LDS list and evaluated with every lane busy.
//
// Minimum image (Eq. 2): for each segment the range of x_B - x_A over the box
// and the segment's cells is known, so when it lies inside one branch of Eq. 2
// the branch is a per-segment shift of 0 or -+L, added after the subtraction
// exactly as Eq. 2 adds it -- the FP32 result is the same.  A stage that holds
// a segment whose range straddles L/2 evaluates Eq. 2 per pair instead.
// A pair of one species is tested from the molecule with the lower sorted index.

constexpr int kSegCap = 128;   // segments of 64 rows (at most two z-runs per row)
constexpr int kListCap = 256;  // candidates compacted per pass (4 per lane)
constexpr int kLaneQuota = kListCap / 64;
constexpr float kFar = 3.0e38f;

// Shift of one axis from its code (0: none, 1: +L, 2: -L).
__device__ __forceinline__ float shift_of(int code, float L) { return code == 1 ? L : (code == 2 ? -L : 0.0f); }

struct SpWave {
    float4 bp[64];   // staged B end position, .w = bits of the sorted index (-1: padding)
    float4 bs[64];   // staged B end position moved by its shift (screening only), .w = sorted index
    float4 bq[64];   // staged B start position, .w = bits of its shift code
    float4 ap[64];   // A end position, .w = bits of the sorted index
    float4 aq[64];   // A start position
    int32_t seg_j0[kSegCap];
    int32_t seg_pre[kSegCap + 1];
    int32_t seg_code[kSegCap];
    uint16_t list[kListCap];
    int4 qe[128];    // queued for evaluation: i, j, rx, bits of r0^2
    float qr[128];   // queued r1^2
};

// Contact probability, pair uniform and acceptance of one pair.
__device__ __forceinline__ void eval_pair(int i, int j, int rx, float r0, float r1, const uint64_t* __restrict__ uid,
                                          const InstStep& S, int contact_only, int log_all,
                                          DevCounters* __restrict__ ctr, PairRec* __restrict__ pairs,
                                          uint32_t pair_cap) {
    const float R = S.R[rx];
    float Pc;
    if (contact_only) Pc = (r0 <= R || r1 <= R) ? 1.0f : 0.0f;
    else Pc = bridge_f(r0, r1, R, S.inv_s[rx]);
    if (!log_all && !(Pc > 0x1p-25f)) return;
    const uint64_t ui = uid[i], uj = uid[j];
    const uint64_t lo = ui < uj ? ui : uj, hi = ui < uj ? uj : ui;
    uint64_t w[4];
    philox(lo, hi, S.step, 1ull, S.key0, S.key1, w);
    const uint32_t u24 = (uint32_t)(w[0] >> 40);
    const bool acc = (double)(2u * u24 + 1u) * 0x1p-25 < (double)Pc;
    if (acc || log_all) {
        const uint32_t k = atomicAdd(&ctr->n_pairs, 1u);
        if (k < pair_cap) {
            PairRec r;
            r.i = i;
            r.j = j;
            r.u24 = u24;
            r.rx = rx;
            r.P = Pc;
            r.flags = acc ? 1 : 0;
            pairs[k] = r;
        } else {
            atomicOr(&ctr->err, kErrPairOverflow);
        }
    }
}

// Append the lanes' entries (need) to the wave's queue and, once 64 are
// queued -- or, with force, whatever is queued -- evaluate up to 64 of them,
// one per lane.  The only evaluation site, so it is inlined once.  All lanes
// of the wave call it together.
__device__ __forceinline__ void qpush(SpWave& w, int& qn, int lane, bool need, const int4& e, float r1, bool force,
                                      const uint64_t* __restrict__ uid, const InstStep& S, int contact_only,
                                      int log_all, DevCounters* __restrict__ ctr, PairRec* __restrict__ pairs,
                                      uint32_t pair_cap) {
    const unsigned long long m = __ballot(need);
    if (m != 0ull) {
        if (need) {
            const int k = qn + (int)__popcll(m & ((1ull << lane) - 1ull));
            w.qe[k] = e;
            w.qr[k] = r1;
        }
        qn += (int)__popcll(m);
    }
    if (qn < 64 && !(force && qn > 0)) return;
    wave_sync_lds();
    const int take = qn < 64 ? qn : 64;
    const bool mine = lane < take;
    int4 v = make_int4(0, 0, 0, 0);
    float vr = 0.0f;
    if (mine) {
        v = w.qe[lane];
        vr = w.qr[lane];
    }
    const int rest = qn - take;
    int4 rv = make_int4(0, 0, 0, 0);
    float rr = 0.0f;
    if (lane < rest) {
        rv = w.qe[64 + lane];
        rr = w.qr[64 + lane];
    }
    wave_sync_lds();
    if (lane < rest) {
        w.qe[lane] = rv;
        w.qr[lane] = rr;
    }
    qn = rest;
    if (mine)
        eval_pair(v.x, v.y, v.z, sqrtf(__int_as_float(v.w)), sqrtf(vr), uid, S, contact_only, log_all, ctr, pairs,
                  pair_cap);
}

// m = 2 m + (d2 < rc2): one compare into VCC and one add-with-carry per test
// (NaN compares false).  A VALU read of VCC written by the previous VALU
// instruction needs two wait states on this target (the compiler inserts the
// same s_nop between a compare and a select).
__device__ __forceinline__ void mask_push(uint32_t& m, float d2, float rc2) {
    asm("v_cmp_lt_f32 vcc, %1, %2\n\ts_nop 1\n\tv_addc_co_u32 %0, vcc, %0, %0, vcc"
        : "+v"(m)
        : "v"(d2), "v"(rc2)
        : "vcc");
}

// Candidate mask of one stage: bit t set when staged B t may lie within the
// cutoff of this lane's A (a superset: rc2 comes with a relative margin of
// 2^-19 over the exact FP32 test, which the candidate stage applies).  The
// tests run from t = 31 down so that doubling the mask lands bit t at t.
// Entries from nb on are padding (their bits are 0): blocks of 8 that hold
// only padding are skipped, which leaves every bit where it was since they
// are the first blocks of their half to run.
template <bool kShift, bool kSame>
__device__ __forceinline__ void stage_mask(const SpWave& w, const float4& pa, int ia, float rc2, float L, float hL,
                                           int nb, uint32_t& mlo, uint32_t& mhi) {
    uint32_t half[2];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        uint32_t m = 0u;
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            if (32 * g + 24 - 8 * blk >= nb) continue;  // only padding (wave-uniform)
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
            const int t = 32 * g + 31 - 8 * blk - kk;
            float dx, dy, dz;
            // a stage whose shifts are exact screens the staged positions moved by
            // their shift (equal to the unmoved ones where the shift is 0)
            const float4 p = kShift ? w.bs[t] : w.bp[t];
            if (kShift) {
                dx = __fsub_rn(p.x, pa.x);
                dy = __fsub_rn(p.y, pa.y);
                dz = __fsub_rn(p.z, pa.z);
            } else {
                dx = minimg_f(__fsub_rn(p.x, pa.x), L, hL);
                dy = minimg_f(__fsub_rn(p.y, pa.y), L, hL);
                dz = minimg_f(__fsub_rn(p.z, pa.z), L, hL);
            }
            // screening value with fused multiply-adds (3 operations instead of 5);
            // rc2 carries a margin above the exact rounding differences, and the
            // candidate stage repeats the exact test
            float d2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __fmul_rn(dz, dz)));
            if (kSame) d2 = (__float_as_int(p.w) > ia) ? d2 : INFINITY;  // each pair once
            mask_push(m, d2, rc2);
            }
        }
        half[g] = m;
    }
    const uint32_t lo = half[0], hi = half[1];
    mlo = lo;
    mhi = hi;
}

// Compact the stage's candidates (lane l, staged t) into the LDS list, at most
// kLaneQuota per lane and pass, and evaluate the list with every lane busy:
// start separation, bridge-exponent bound, queue.
template <bool kShift>
__device__ __forceinline__ void stage_candidates(SpWave& w, uint32_t mlo, uint32_t mhi, int lane, int rx, float R,
                                                 float inv_s, float rc2, float L, float hL, int& qn,
                                                 const uint64_t* __restrict__ uid, const InstStep& S,
                                                 int contact_only, int log_all, DevCounters* __restrict__ ctr,
                                                 PairRec* __restrict__ pairs, uint32_t pair_cap,
                                                 unsigned long long& ncand) {
    while (__ballot((mlo | mhi) != 0u)) {
        const int have = __popc(mlo) + __popc(mhi);
        const int mine = have < kLaneQuota ? have : kLaneQuota;
        const int incl = (int)wave_incl_scan((uint32_t)mine);
        const int total = wave_last(incl);
        const int at = incl - mine;
        for (int k = 0; k < mine; ++k) {
            int t;
            if (mlo) {
                t = __ffs(mlo) - 1;
                mlo &= mlo - 1u;
            } else {
                t = 32 + __ffs(mhi) - 1;
                mhi &= mhi - 1u;
            }
            w.list[at + k] = (uint16_t)((lane << 6) | t);
        }
        wave_sync_lds();
        for (int e0 = 0; e0 < total; e0 += 64) {
            bool need = false;
            int4 e = make_int4(0, 0, 0, 0);
            float r1 = 0.0f;
            if (e0 + lane < total) {
                const int code = w.list[e0 + lane];
                const int l = code >> 6, t = code & 63;
                const float4 pa = w.ap[l], qa = w.aq[l];
                const float4 p = w.bp[t], q = w.bq[t];
                float dx, dy, dz;
                if (kShift) {
                    const int sc = __float_as_int(q.w);  // shift code of the staged molecule
                    dx = __fadd_rn(__fsub_rn(p.x, pa.x), shift_of(sc & 3, L));
                    dy = __fadd_rn(__fsub_rn(p.y, pa.y), shift_of((sc >> 2) & 3, L));
                    dz = __fadd_rn(__fsub_rn(p.z, pa.z), shift_of((sc >> 4) & 3, L));
                } else {
                    dx = minimg_f(__fsub_rn(p.x, pa.x), L, hL);
                    dy = minimg_f(__fsub_rn(p.y, pa.y), L, hL);
                    dz = minimg_f(__fsub_rn(p.z, pa.z), L, hL);
                }
                const float d2 = __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
                const float ex = minimg_f(q.x - qa.x, L, hL);
                const float ey = minimg_f(q.y - qa.y, L, hL);
                const float ez = minimg_f(q.z - qa.z, L, hL);
                const float e2 = ex * ex + ey * ey + ez * ez;
                // exp(-a) bounds P; below 1.5e-8 no 24-bit uniform can fall under P.
                // The test runs on the hardware square root (within 1 ulp) with
                // margins that keep every pair the correctly rounded roots keep:
                // the error of a is below 3e-4 once both separations exceed 1.01 R.
                const float r1a = __builtin_amdgcn_sqrtf(d2), r0a = __builtin_amdgcn_sqrtf(e2);
                const float aexp = (r0a - R) * (r1a - R) * inv_s;
                // (the end separation is tested again: padding, whose positions lie
                // far outside the cube, never reaches the evaluation)
                ncand += d2 < rc2 ? 1ull : 0ull;  // the exact test: candidates as the oracle counts them
                need = d2 < rc2 &&
                       (log_all || contact_only || r0a <= 1.01f * R || r1a <= 1.01f * R || !(aexp > 18.01f));
                r1 = d2;
                e = make_int4(__float_as_int(pa.w), __float_as_int(p.w), rx, __float_as_int(e2));
            }
            qpush(w, qn, lane, need, e, r1, false, uid, S, contact_only, log_all, ctr, pairs, pair_cap);
        }
        wave_sync_lds();
    }
}


// Cells [c0, c1] (unwrapped, may leave [0, nc)) whose extent meets [lo, hi];
// eps covers the FP32 rounding of the binning.  Returns false (and the whole
// axis) when the span would reach nc cells.
__device__ __forceinline__ bool cell_span(float lo, float hi, float hL, float inv_h, float eps, int nc, int& c0,
                                          int& c1) {
    c0 = (int)floorf((lo - eps + hL) * inv_h);
    c1 = (int)floorf((hi + eps + hL) * inv_h);
    if (c1 - c0 + 1 >= nc) {
        c0 = 0;
        c1 = nc - 1;
        return false;
    }
    return true;
}

// Cells [qlo, qhi] (wrapped) against the box [blo, bhi] along one axis: the
// range of x_B - x_A lies in [dlo, dhi].  Picks the Eq. 2 branch that holds for
// the whole range (code 0: none, 1: +L, 2: -L; valid false when the range
// straddles +-L/2) and the smallest |minimum-image separation| over it (0 when
// it straddles).
__device__ __forceinline__ void axis_shift(int qlo, int qhi, float blo, float bhi, float h, float hL, float eps,
                                           int& code, bool& valid, float& gap) {
    const float dlo = (float)qlo * h - hL - bhi - eps;
    const float dhi = (float)(qhi + 1) * h - hL - blo + eps;
    if (dlo >= hL) {
        code = 2;
        valid = true;
    } else if (dhi < -hL) {
        code = 1;
        valid = true;
    } else {
        code = 0;
        valid = dlo >= -hL && dhi < hL;
    }
    const float s = code == 1 ? 2.0f * hL : (code == 2 ? -2.0f * hL : 0.0f);
    const float a = dlo + s, b = dhi + s;
    gap = valid ? fmaxf(0.0f, fmaxf(a, -b)) : 0.0f;
}


__global__ __launch_bounds__(GSBS_BLOCK) void k_pairs_sp(const float4* __restrict__ pos,
                                                       const float4* __restrict__ pos0,
                                                       const uint64_t* __restrict__ uid,
                                                       DevCounters* __restrict__ ctr,
                                                       const InstStep* __restrict__ P,
                                                       const ChemDev* __restrict__ chem,
                                                       const uint32_t* __restrict__ start,
                                                       PairRec* __restrict__ pairs, uint32_t pair_cap,
                                                       int32_t log_all, int32_t n_inst, int32_t total_units) {
    __shared__ int32_t rmap[kMaxSpecies * kMaxSpecies];
    __shared__ unsigned long long s_cand;
    __shared__ SpWave wall[GSBS_BLOCK / 64];
    for (int k = threadIdx.x; k < kMaxSpecies * kMaxSpecies; k += blockDim.x)
        rmap[k] = chem->rmap[k / kMaxSpecies][k % kMaxSpecies];
    if (threadIdx.x == 0) s_cand = 0ull;
    __syncthreads();
    const int contact_only = chem->contact_only;
    const int ns = chem->n_species;
    const int lane = threadIdx.x & 63;
    const int waves = GSBS_BLOCK / 64;
    SpWave& w = wall[threadIdx.x >> 6];
    int qn = 0;  // wave-uniform queue length
    unsigned long long ncand = 0;
    const InstStep* Sq = nullptr;
    // first work item of each instance, one per lane (up to 64 instances)
    const int ub_lane = lane < n_inst ? P[lane].unit_base : 0x7FFFFFFF;
    for (int u = blockIdx.x * waves + (threadIdx.x >> 6); u < total_units; u += gridDim.x * waves) {
        // instance owning work item u (instances own consecutive ranges, in order):
        // the last one whose first item is at most u
        int lo_i = 0;
        if (n_inst <= 64) {
            lo_i = __popcll(__ballot(ub_lane <= u)) - 1;
        } else {
            int hi_i = n_inst - 1;
            while (lo_i < hi_i) {
                const int mid = (lo_i + hi_i + 1) >> 1;
                if (P[mid].unit_base <= u) lo_i = mid;
                else hi_i = mid - 1;
            }
        }
        const InstStep& S = P[lo_i];
        if (!S.active || !S.by_species) continue;
        if (Sq != &S && qn > 0) {  // queued pairs belong to the previous instance's step data
            while (qn > 0)
                qpush(w, qn, lane, false, make_int4(0, 0, 0, 0), 0.0f, true, uid, *Sq, contact_only, log_all, ctr,
                      pairs, pair_cap);
        }
        Sq = &S;
        const int lu = u - S.unit_base;
        if (lu >= S.unit_off_sp[ns]) continue;
        int si = 0;
        while (si + 1 < ns && S.unit_off_sp[si + 1] <= lu) ++si;
        const uint32_t pm = S.pm_dir[si];
        if (pm == 0u) continue;
        const int nc = S.nc, nsplit = S.nsplit_sp[si];
        const int kx = S.kdim_sp[si] & 0xFF, ky = (S.kdim_sp[si] >> 8) & 0xFF, kz = (S.kdim_sp[si] >> 16) & 0xFF;
        const int nbx = (nc + kx - 1) / kx, nby = (nc + ky - 1) / ky, nbz = (nc + kz - 1) / kz;
        const int r = lu - S.unit_off_sp[si];
        const int split = r % nsplit, unit = r / nsplit;
        const int bx = unit / (nby * nbz), by = (unit / nbz) % nby, bz = unit % nbz;
        const int x0 = bx * kx, x1 = min(x0 + kx, nc), y0 = by * ky, y1 = min(y0 + ky, nc);
        const int z0 = bz * kz, z1 = min(z0 + kz, nc);
        const int ncell = nc * nc * nc;
        const int sbase = S.bin_base + si * ncell;
        // A: the box's rows (x, y) over z-cells [z0, z1); kx * ky <= 64 rows
        const int nyA = y1 - y0;
        const int nrowsA = (x1 - x0) * nyA;
        int cntA = 0, begA = 0;
        if (lane < nrowsA) {
            const int b0 = sbase + ((x0 + lane / nyA) * nc + y0 + lane % nyA) * nc;
            begA = (int)start[b0 + z0];
            cntA = (int)start[b0 + z1] - begA;
        }
        const int inclA = (int)wave_incl_scan((uint32_t)cntA);
        const int nA = wave_last(inclA);
        if (nA == 0) continue;
        // first A index of each row, one row per lane (non-decreasing; past the rows: never reached)
        const int exclA = lane < nrowsA ? inclA - cntA : 0x7FFFFFFF;
        const float h = S.h, eps = S.cull_eps, L = S.L, hL = S.halfL, inv_h = S.inv_h;
        const int* rrow = rmap + si * kMaxSpecies;
        for (int ab = 0; ab < nA; ab += 64) {
            const int k = ab + lane;
            const bool va = k < nA;
            // row of this lane's molecule: the last row whose first index is at most k
            // (rows read from the lanes that hold them; every lane takes part)
            int row = 0;
#pragma unroll
            for (int st = 32; st >= 1; st >>= 1) {
                const int nx = row + st;
                const int ex = __shfl(exclA, nx < 64 ? nx : 63, 64);
                if (nx < 64 && ex <= k) row = nx;
            }
            const int rb0 = __shfl(begA, row, 64), rx0 = __shfl(exclA, row, 64);
            const int ia = va ? rb0 + (k - rx0) : -1;
            float4 pa = make_float4(kFar, kFar, kFar, __int_as_float(-1));
            float4 qa = make_float4(0.f, 0.f, 0.f, 0.f);
            if (va) {
                pa = pos[ia];
                pa.w = __int_as_float(ia);
                qa = pos0[ia];
            }
            wave_sync_lds();
            w.ap[lane] = pa;
            w.aq[lane] = qa;
            // sorted index of the chunk's first molecule, the lowest of the chunk (rows
            // and cells are listed in bin order)
            const int ia_first = __builtin_amdgcn_readfirstlane(ia);
            // bounding box of the chunk's end positions (the box does not cross the cube faces)
            const float blx = wave_min_f(va ? pa.x : kFar), bhx = wave_max_f(va ? pa.x : -kFar);
            const float bly = wave_min_f(va ? pa.y : kFar), bhy = wave_max_f(va ? pa.y : -kFar);
            const float blz = wave_min_f(va ? pa.z : kFar), bhz = wave_max_f(va ? pa.z : -kFar);
            uint32_t mm = pm;
            while (mm) {
                const int sj = __ffs(mm) - 1;
                mm &= mm - 1u;
                const int rx = rrow[sj];
                const float c2 = S.cull2[rx];
                const float rcu = sqrtf(c2);
                const float rc2 = S.rc2[rx];
                // screening cutoff: a relative margin for the fused arithmetic and an
                // absolute one for the rounding of a position moved by +-L
                const float rcs = __builtin_amdgcn_sqrtf(rc2) * (1.0f + 0x1p-19f) + 1e-6f * L;
                const float rc2m = rcs * rcs;
                const float Rr = S.R[rx], inv_s = S.inv_s[rx];
                const bool same = (sj == si);
                int cx0, cx1, cy0, cy1, czl, czh;
                cell_span(blx - rcu, bhx + rcu, hL, inv_h, eps, nc, cx0, cx1);
                cell_span(bly - rcu, bhy + rcu, hL, inv_h, eps, nc, cy0, cy1);
                const bool cullz = cell_span(blz - rcu, bhz + rcu, hL, inv_h, eps, nc, czl, czh);
                const int sbB = S.bin_base + sj * ncell;
                const int ny = cy1 - cy0 + 1;
                const int nrows = (cx1 - cx0 + 1) * ny;
                for (int rb = 0; rb < nrows; rb += 64) {
                    // --- rows rb .. rb+63, one per lane: culling, z-window, segments
                    const int rr = rb + lane;
                    int n1 = 0, n2 = 0, j1 = 0, j2 = 0, code1 = 0, code2 = 0;
                    if (rr < nrows) {
                        const int cx = cx0 + rr / ny, cy = cy0 + rr % ny;
                        const int qx = cx < 0 ? cx + nc : (cx >= nc ? cx - nc : cx);
                        const int qy = cy < 0 ? cy + nc : (cy >= nc ? cy - nc : cy);
                        int sxc, syc;
                        bool vx, vy;
                        float gx, gy;
                        axis_shift(qx, qx, blx, bhx, h, hL, eps, sxc, vx, gx);
                        axis_shift(qy, qy, bly, bhy, h, hL, eps, syc, vy, gy);
                        const float gxy2 = gx * gx + gy * gy;
                        if (gxy2 <= c2) {
                            int cz0 = czl, cz1 = czh;
                            if (cullz) {
                                const float rz = sqrtf(c2 - gxy2);
                                cell_span(blz - rz, bhz + rz, hL, inv_h, eps, nc, cz0, cz1);
                            }
                            const int rowB = sbB + (qx * nc + qy) * nc;
                            // main run inside [0, nc) and the wrapped run, if any
                            const int ml = cz0 < 0 ? 0 : cz0, mh = cz1 >= nc ? nc - 1 : cz1;
                            int wl = 1, wh = 0;
                            if (cz0 < 0) {
                                wl = cz0 + nc;
                                wh = nc - 1;
                            } else if (cz1 >= nc) {
                                wl = 0;
                                wh = cz1 - nc;
                            }
                            const int base_code = sxc | (syc << 2);
                            const bool vxy = vx && vy;
                            if (ml <= mh) {
                                j1 = (int)start[rowB + ml];
                                n1 = (int)start[rowB + mh + 1] - j1;
                                int szc;
                                bool vz;
                                float gz;
                                axis_shift(ml, mh, blz, bhz, h, hL, eps, szc, vz, gz);
                                code1 = base_code | (szc << 4) | ((vxy && vz) ? 64 : 0);
                            }
                            if (wl <= wh) {
                                j2 = (int)start[rowB + wl];
                                n2 = (int)start[rowB + wh + 1] - j2;
                                int szc;
                                bool vz;
                                float gz;
                                axis_shift(wl, wh, blz, bhz, h, hL, eps, szc, vz, gz);
                                code2 = base_code | (szc << 4) | ((vxy && vz) ? 64 : 0);
                            }
                            if (same) {
                                // a pair of one species is taken from its lower sorted
                                // index: partners below the chunk's first molecule would
                                // all be masked, so they are not streamed
                                auto trim = [&](int& j, int& nn) {
                                    const int e = j + nn;
                                    if (e <= ia_first) nn = 0;
                                    else if (j < ia_first) {
                                        nn = e - ia_first;
                                        j = ia_first;
                                    }
                                };
                                trim(j1, n1);
                                trim(j2, n2);
                            }
                        }
                    }
                    // segments whose exact shift is 0 on every axis go first in the
                    // stream (stages of one kind)
                    const bool z1 = n1 > 0 && (code1 & 127) == 64, z2 = n2 > 0 && (code2 & 127) == 64;
                    const int nz_l = (z1 ? 1 : 0) + (z2 ? 1 : 0);
                    const int no_l = (n1 > 0 ? 1 : 0) + (n2 > 0 ? 1 : 0) - nz_l;
                    const int mz_l = (z1 ? n1 : 0) + (z2 ? n2 : 0), mo_l = n1 + n2 - mz_l;
                    const int sz = (int)wave_incl_scan((uint32_t)nz_l), so = (int)wave_incl_scan((uint32_t)no_l);
                    const int mz = (int)wave_incl_scan((uint32_t)mz_l), mo = (int)wave_incl_scan((uint32_t)mo_l);
                    const int NZ = wave_last(sz), NO = wave_last(so);
                    const int MZ = wave_last(mz), MO = wave_last(mo);
                    const int nseg = NZ + NO, T = MZ + MO;
                    if (T == 0) continue;
                    wave_sync_lds();
                    {
                        int atz = sz - nz_l, ato = NZ + so - no_l;
                        int mpz = mz - mz_l, mpo = MZ + mo - mo_l;
                        if (n1 > 0) {
                            int& at = z1 ? atz : ato;
                            int& mp = z1 ? mpz : mpo;
                            w.seg_j0[at] = j1;
                            w.seg_pre[at] = mp;
                            w.seg_code[at] = code1;
                            ++at;
                            mp += n1;
                        }
                        if (n2 > 0) {
                            int& at = z2 ? atz : ato;
                            int& mp = z2 ? mpz : mpo;
                            w.seg_j0[at] = j2;
                            w.seg_pre[at] = mp;
                            w.seg_code[at] = code2;
                        }
                        if (lane == 0) w.seg_pre[nseg] = T;
                    }
                    wave_sync_lds();
                    // --- this wave's slice of the stream, 64 molecules per stage
                    const int p0 = (int)(((long long)T * split) / nsplit);
                    const int p1 = (int)(((long long)T * (split + 1)) / nsplit);
                    auto fetch = [&](int b, float4& fp, float4& fq, int& fj, int& fc) {
                        const int p = b + lane;
                        fj = -1;
                        fc = 64;
                        fp = make_float4(-kFar, -kFar, -kFar, 0.f);
                        fq = make_float4(0.f, 0.f, 0.f, 0.f);
                        if (p < p1) {
                            int lo = 0, hi = nseg - 1;
                            while (lo < hi) {
                                const int mid = (lo + hi + 1) >> 1;
                                if (w.seg_pre[mid] <= p) lo = mid;
                                else hi = mid - 1;
                            }
                            fj = w.seg_j0[lo] + (p - w.seg_pre[lo]);
                            fc = w.seg_code[lo];
                            fp = pos[fj];
                            fq = pos0[fj];
                        }
                    };
                    float4 fp, fq;
                    int fj, fc;
                    if (p0 < p1) fetch(p0, fp, fq, fj, fc);
                    for (int b = p0; b < p1; b += 64) {
                        wave_sync_lds();
                        w.bp[lane] = make_float4(fp.x, fp.y, fp.z, __int_as_float(fj));
                        w.bq[lane] = make_float4(fq.x, fq.y, fq.z, __int_as_float(fc & 63));
                        w.bs[lane] = make_float4(fp.x + shift_of(fc & 3, L), fp.y + shift_of((fc >> 2) & 3, L),
                                                 fp.z + shift_of((fc >> 4) & 3, L), __int_as_float(fj));
                        const bool exact = __ballot((fc & 64) == 0) == 0ull;
                        wave_sync_lds();
                        if (b + 64 < p1) fetch(b + 64, fp, fq, fj, fc);
                        uint32_t mlo, mhi;
                        const int nbs = p1 - b;  // staged entries that are partners (the rest is padding)
                        if (exact) {
                            if (same) stage_mask<true, true>(w, pa, ia, rc2m, L, hL, nbs, mlo, mhi);
                            else stage_mask<true, false>(w, pa, ia, rc2m, L, hL, nbs, mlo, mhi);
                            stage_candidates<true>(w, mlo, mhi, lane, rx, Rr, inv_s, rc2, L, hL, qn, uid, S, contact_only,
                                                   log_all, ctr, pairs, pair_cap, ncand);
                        } else {
                            if (same) stage_mask<false, true>(w, pa, ia, rc2m, L, hL, nbs, mlo, mhi);
                            else stage_mask<false, false>(w, pa, ia, rc2m, L, hL, nbs, mlo, mhi);
                            stage_candidates<false>(w, mlo, mhi, lane, rx, Rr, inv_s, rc2, L, hL, qn, uid, S,
                                                    contact_only, log_all, ctr, pairs, pair_cap, ncand);
                        }
                    }
                }
            }
        }
    }
    while (qn > 0)
        qpush(w, qn, lane, false, make_int4(0, 0, 0, 0), 0.0f, true, uid, *Sq, contact_only, log_all, ctr, pairs,
              pair_cap);
    for (int d = 32; d >= 1; d >>= 1) ncand += __shfl_xor(ncand, d, 64);
    if (lane == 0 && ncand) atomicAdd(&s_cand, ncand);
    __syncthreads();
    if (threadIdx.x == 0 && s_cand) {
        atomicAdd(&ctr->cand, s_cand);
        atomicAdd(&ctr->cand_sp, s_cand);
    }
}

// --------------------------------------------------------------- react ---
// One work-group: the accepted pairs are few compared with the molecules.
constexpr int kReactBlock = 1024;

__device__ __forceinline__ unsigned long long match_key(uint32_t u24, uint64_t partner) {
    return ((unsigned long long)u24 << 40) | (partner & 0xFFFFFFFFFFull);
}

__device__ __forceinline__ int ld_mate(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_mate(int32_t* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Outcome of one reacted pair: reactants flagged removed, products of Table 1
// appended after the live molecules at the weighted position, counts updated.
__device__ __forceinline__ void apply_reaction(const PairRec& r, float4* __restrict__ pos, uint64_t* __restrict__ uid,
                                               DevCounters* __restrict__ ctr, const InstStep* __restrict__ P,
                                               const ChemDev* __restrict__ chem, long long* __restrict__ counts,
                                               int n_live, int cap, int* n_prod, int* n_react) {
    int a = r.i, b = r.j;
    uint64_t ua = uid[a], ub = uid[b];
    if (ub < ua) {
        const int t = a; a = b; b = t;
        const uint64_t tu = ua; ua = ub; ub = tu;
    }
    const float4 pa = pos[a], pb = pos[b];
    const int ma = __float_as_int(pa.w), mb = __float_as_int(pb.w);
    const int inst = ma >> 8;
    const int sa = ma & 0xFF, sb = mb & 0xFF;
    const int rx = r.rx;
    long long* cnt = counts + inst * kMaxSpecies;
    atomicAdd(n_react, 1);
    if (chem->keep_b[rx]) {
        const int gone = (sa == chem->rb[rx]) ? b : a;
        const int sg = (gone == a) ? sa : sb;
        pos[gone].w = __int_as_float((inst << 8) | kDead);
        atomicAdd((unsigned long long*)&cnt[sg], (unsigned long long)(-1ll));
        return;
    }
    pos[a].w = __int_as_float((inst << 8) | kDead);
    pos[b].w = __int_as_float((inst << 8) | kDead);
    atomicAdd((unsigned long long*)&cnt[sa], (unsigned long long)(-1ll));
    atomicAdd((unsigned long long*)&cnt[sb], (unsigned long long)(-1ll));
    const int npr = chem->nprod[rx];
    if (npr == 0) return;
    const InstStep& S = P[inst];
    const float Da = chem->D[sa], Db = chem->D[sb];
    const float wgt = (Da + Db > 0.0f) ? Da / (Da + Db) : 0.5f;
    const float px = wrap_f(pa.x + wgt * minimg_f(pb.x - pa.x, S.L, S.halfL), S.L, S.halfL, S.invL);
    const float py = wrap_f(pa.y + wgt * minimg_f(pb.y - pa.y, S.L, S.halfL), S.L, S.halfL, S.invL);
    const float pz = wrap_f(pa.z + wgt * minimg_f(pb.z - pa.z, S.L, S.halfL), S.L, S.halfL, S.invL);
    const int base = atomicAdd(n_prod, npr);
    for (int k = 0; k < npr; ++k) {
        const int dst = n_live + base + k;
        if (dst >= cap) {
            atomicOr(&ctr->err, kErrMolOverflow);
            continue;
        }
        uint64_t u;
        if (k == 0) u = ua;
        else if (k == 1) u = ub;
        else {
            uint64_t w[4];
            philox(ua, ub, S.step, 2ull, S.key0, S.key1, w);
            u = w[0] | 0x8000000000000000ull;
        }
        const int ps = chem->prod[rx][k];
        pos[dst] = make_float4(px, py, pz, __int_as_float((inst << 8) | ps));
        uid[dst] = u;
        atomicAdd((unsigned long long*)&cnt[ps], 1ull);
    }
}

// Slot of molecule `mol` in the block's open-addressing table (inserted when
// absent).  The table holds at most two molecules per pair and is at most
// half full, so the probe ends.
constexpr int kReactHashBits = 12;
constexpr int kReactHash = 1 << kReactHashBits;
constexpr int kReactFast = kReactHash / 4;  // pairs handled in LDS (one per thread)
static_assert(kReactFast <= kReactBlock, "one pair per thread");
__device__ __forceinline__ int react_slot(int* key, int mol) {
    int h = (int)(((uint32_t)mol * 2654435761u) >> (32 - kReactHashBits));
    while (true) {
        const int prev = atomicCAS(&key[h], -1, mol);
        if (prev == -1 || prev == mol) return h;
        h = (h + 1) & (kReactHash - 1);
    }
}

__global__ __launch_bounds__(kReactBlock) void k_react(float4* __restrict__ pos, uint64_t* __restrict__ uid,
                                                     DevCounters* __restrict__ ctr,
                                                     const InstStep* __restrict__ P,
                                                     const ChemDev* __restrict__ chem,
                                                     PairRec* __restrict__ pairs, uint32_t pair_cap,
                                                     unsigned long long* __restrict__ claim,
                                                     int32_t* __restrict__ mate,
                                                     long long* __restrict__ counts,
                                                     unsigned long long* __restrict__ msteps,
                                                     int32_t n_inst, int32_t cap, int32_t search_only) {
    __shared__ int n_new, n_wait, n_prod, n_react;
    __shared__ int ht_key[kReactHash];
    __shared__ unsigned long long ht_claim[kReactHash];
    __shared__ int ht_mate[kReactHash];
    const int tid = threadIdx.x;
    // molecule-steps of the instances that stepped (counts before this step's reactions)
    unsigned long long mm[2] = {0ull, 0ull};
    for (int t = tid; t < n_inst; t += kReactBlock) {
        if (!P[t].active) continue;
        long long s = 0;
        for (int k = 0; k < chem->n_species; ++k) s += counts[t * kMaxSpecies + k];
        msteps[t] += (unsigned long long)s;
        mm[P[t].by_species ? 1 : 0] += (unsigned long long)s;
    }
    if (mm[0]) atomicAdd(&ctr->msteps_mode[0], mm[0]);
    if (mm[1]) atomicAdd(&ctr->msteps_mode[1], mm[1]);
    const uint32_t np_raw = ctr->n_pairs;
    const int np = (int)(np_raw < pair_cap ? np_raw : pair_cap);
    const int n_live = ctr->n_live;
    if (tid == 0) {
        n_prod = 0;
        n_react = 0;
    }
    __syncthreads();
    if (search_only) {
        if (tid == 0) ctr->n_in = n_live;
        return;
    }
    if (np <= kReactFast) {
        // Few pairs (every step but debug logging): one pair per thread, claims
        // and mates in an LDS table instead of the per-molecule global arrays.
        for (int k = tid; k < kReactHash; k += kReactBlock) {
            ht_key[k] = -1;
            ht_claim[k] = ~0ull;
            ht_mate[k] = -1;
        }
        __syncthreads();
        PairRec r{};
        bool acc = false;
        int si = 0, sj = 0;
        unsigned long long ki = 0, kj = 0;  // claim keys written to i and to j
        if (tid < np) {
            r = pairs[tid];
            acc = (r.flags & 1) != 0;
            if (acc) {
                si = react_slot(ht_key, r.i);
                sj = react_slot(ht_key, r.j);
                ki = match_key(r.u24, uid[r.j]);
                kj = match_key(r.u24, uid[r.i]);
            }
        }
        bool reacted = false;
        for (int round = 0; round < chem->rounds; ++round) {
            if (tid == 0) {
                n_new = 0;
                n_wait = 0;
            }
            __syncthreads();
            const bool open = acc && !reacted && ht_mate[si] < 0 && ht_mate[sj] < 0;
            if (open) {
                atomicMin(&ht_claim[si], ki);
                atomicMin(&ht_claim[sj], kj);
            }
            __syncthreads();
            bool matched = false;
            if (open) {
                matched = ht_claim[si] == ki && ht_claim[sj] == kj;
                atomicAdd(matched ? &n_new : &n_wait, 1);
            }
            __syncthreads();
            if (acc) {
                ht_claim[si] = ~0ull;
                ht_claim[sj] = ~0ull;
            }
            if (matched) {
                // a molecule in two mutual pairs needs two pairs with equal keys
                if (atomicCAS(&ht_mate[si], -1, r.j) != -1) atomicOr(&ctr->err, kErrTie);
                if (atomicCAS(&ht_mate[sj], -1, r.i) != -1) atomicOr(&ctr->err, kErrTie);
                reacted = true;
            }
            __syncthreads();
            // eligible pairs only lose eligibility: with none left waiting, later rounds find nothing
            const bool stop = n_new == 0 || n_wait == 0;
            __syncthreads();  // every thread has read the counters before the next round resets them
            if (stop) break;
        }
        if (tid < np && acc) {
            if (reacted) pairs[tid].flags = r.flags | 2;
            if (reacted) apply_reaction(r, pos, uid, ctr, P, chem, counts, n_live, cap, &n_prod, &n_react);
        }
    } else {
        for (int round = 0; round < chem->rounds; ++round) {
            for (int p = tid; p < np; p += kReactBlock) {
                const PairRec r = pairs[p];
                if (!(r.flags & 1) || ld_mate(&mate[r.i]) >= 0 || ld_mate(&mate[r.j]) >= 0) continue;
                atomicMin(&claim[r.i], match_key(r.u24, uid[r.j]));
                atomicMin(&claim[r.j], match_key(r.u24, uid[r.i]));
            }
            if (tid == 0) {
                n_new = 0;
                n_wait = 0;
            }
            __syncthreads();
            for (int p = tid; p < np; p += kReactBlock) {
                const PairRec r = pairs[p];
                if (!(r.flags & 1) || ld_mate(&mate[r.i]) >= 0 || ld_mate(&mate[r.j]) >= 0) continue;
                const unsigned long long ci =
                    __hip_atomic_load(&claim[r.i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned long long cj =
                    __hip_atomic_load(&claim[r.j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (ci == match_key(r.u24, uid[r.j]) && cj == match_key(r.u24, uid[r.i])) {
                    pairs[p].flags = r.flags | 4;
                    atomicAdd(&n_new, 1);
                } else {
                    atomicAdd(&n_wait, 1);
                }
            }
            __syncthreads();
            for (int p = tid; p < np; p += kReactBlock) {
                const PairRec r = pairs[p];
                if (!(r.flags & 1)) continue;
                __hip_atomic_store(&claim[r.i], ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&claim[r.j], ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (r.flags & 4) {
                    // a molecule in two mutual pairs needs two pairs with equal keys
                    if (atomicCAS(&mate[r.i], -1, r.j) != -1) atomicOr(&ctr->err, kErrTie);
                    if (atomicCAS(&mate[r.j], -1, r.i) != -1) atomicOr(&ctr->err, kErrTie);
                    pairs[p].flags = (r.flags & ~4) | 2;
                }
            }
            __syncthreads();
            // eligible pairs only lose eligibility: with none left waiting, later rounds find nothing
            if (n_new == 0 || n_wait == 0) break;
            __syncthreads();
        }
        // products, removals, counts
        for (int p = tid; p < np; p += kReactBlock) {
            const PairRec r = pairs[p];
            if (!(r.flags & 2)) continue;
            st_mate(&mate[r.i], -1);
            st_mate(&mate[r.j], -1);
            apply_reaction(r, pos, uid, ctr, P, chem, counts, n_live, cap, &n_prod, &n_react);
        }
    }
    __syncthreads();
    if (tid == 0) {
        const int nn = n_live + n_prod;
        ctr->n_in = nn > cap ? cap : nn;
        ctr->reactions += (unsigned long long)n_react;
    }
}

// First-order channels (an extension: scavenging by a solute held at a fixed
// concentration).  After the step's pair reactions every live molecule of
// the sorted array (not this step's products, which sit at n_live and beyond)
// whose species has a channel converts with probability p = 1 - exp(-k dt)
// (FP64, from the host): the top 24 bits k24 of word 0 of the Philox block
// (uid, step, 3, 0) decide, converting iff (2 k24 + 1) 2^-25 < p (exact in
// FP64).  Product 1 takes the molecule's place and uid; product 2 is appended
// at the same point with uid = word 1 | 2^63; no product removes it.
__global__ __launch_bounds__(GSBS_BLOCK) void k_first_order(float4* __restrict__ pos, uint64_t* __restrict__ uid,
                                                          DevCounters* __restrict__ ctr,
                                                          const InstStep* __restrict__ P,
                                                          const ChemDev* __restrict__ chem,
                                                          long long* __restrict__ counts, int32_t cap) {
    const int n = ctr->n_live;
    const uint32_t mask = chem->fo_mask;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float4 p = pos[i];
        const int meta = __float_as_int(p.w);
        const int sp = meta & 0xFF;
        if (sp == kDead || !((mask >> sp) & 1u)) continue;
        const int inst = meta >> 8;
        const InstStep& S = P[inst];
        if (!S.active) continue;
        uint64_t w[4];
        const uint64_t u = uid[i];
        philox(u, S.step, 3ull, 0ull, S.key0, S.key1, w);
        if (!((double)(2u * (uint32_t)(w[0] >> 40) + 1u) * 0x1p-25 < S.fo_p[sp])) continue;
        long long* cnt = counts + inst * kMaxSpecies;
        atomicAdd((unsigned long long*)&cnt[sp], (unsigned long long)(-1ll));
        const int np = chem->fo_nprod[sp];
        if (np == 0) {
            pos[i].w = __int_as_float((inst << 8) | kDead);
            continue;
        }
        const int p0 = chem->fo_prod[sp][0];
        pos[i].w = __int_as_float((inst << 8) | p0);
        atomicAdd((unsigned long long*)&cnt[p0], 1ull);
        if (np < 2) continue;
        // append product 2: a slot below cap, else flag the overflow
        int dst = __hip_atomic_load(&ctr->n_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (dst < cap) {
            const int prev = atomicCAS(&ctr->n_in, dst, dst + 1);
            if (prev == dst) break;
            dst = prev;
        }
        if (dst >= cap) {
            atomicOr(&ctr->err, kErrMolOverflow);
            continue;
        }
        const int p1 = chem->fo_prod[sp][1];
        pos[dst] = make_float4(p.x, p.y, p.z, __int_as_float((inst << 8) | p1));
        uid[dst] = w[1] | 0x8000000000000000ull;
        atomicAdd((unsigned long long*)&cnt[p1], 1ull);
    }
}

// -------------------------------------------------------------- records ---
__global__ void k_record(const long long* __restrict__ counts, long long* __restrict__ rec, int32_t max_rec,
                         RecordList list) {
    const int e = blockIdx.x;
    const int k = threadIdx.x;
    if (e >= list.n || k >= kMaxSpecies) return;
    const int inst = list.inst[e];
    rec[((long long)inst * max_rec + list.rec[e]) * kMaxSpecies + k] = counts[inst * kMaxSpecies + k];
}

// ------------------------------------------------------------- launches ---
void launch_inject(hipStream_t st, float4* pos, uint64_t* uid, long long* counts, DevCounters* ctr,
                   const float* xyz, const uint8_t* sp, int32_t n, int32_t inst, uint64_t uid_base,
                   int32_t cap) {
    if (n <= 0) return;
    int grid = (n + GSBS_BLOCK - 1) / GSBS_BLOCK;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_inject, dim3(grid), dim3(GSBS_BLOCK), 0, st, pos, uid, counts, ctr, xyz, sp, n,
                       inst, uid_base, cap, &ctr->err);
    hipLaunchKernelGGL(k_add_n, dim3(1), dim3(1), 0, st, ctr, n, cap);
}

const char* const kStepKernelNames[kStepKernels] = {"k_bin", "k_scan", "k_scatter", "k_pairs", "k_pairs_sp", "k_react"};

void launch_step(hipStream_t st, const StepBuffers& b, const InstStep* P, const ChemDev* chem,
                 int32_t n_inst, int32_t total_bins, int32_t total_units, int32_t ns, int32_t grid, int32_t flags,
                 hipEvent_t* ev, uint32_t ev_mask) {
    const int fixed = (flags & kStepFixed) ? 1 : 0;
    const int nb = (total_bins + kScanTile - 1) / kScanTile;
    // every kernel slot in the mask gets its two events, also when the kernel is not
    // launched; with kEvChain, ev[k] marks the start of slot k and ev[kStepKernels]
    // the end of the last one (one event per boundary)
    const bool chain = (ev_mask & kEvChain) != 0u;
    auto mark = [&](int slot, int end) {
        if (!ev) return;
        if (chain) {
            if (end == 0) (void)hipEventRecord(ev[slot], st);
            else if (slot == kStepKernels - 1) (void)hipEventRecord(ev[kStepKernels], st);
            return;
        }
        if ((ev_mask >> slot) & 1u) (void)hipEventRecord(ev[2 * slot + end], st);
    };
    mark(0, 0);
    if (total_bins <= kLdsBins) {
        // enough blocks that no block owns more than kBinRounds * GSBS_BLOCK molecules
        const int g = grid > (b.cap + kBinRounds * GSBS_BLOCK - 1) / (kBinRounds * GSBS_BLOCK)
                          ? grid
                          : (b.cap + kBinRounds * GSBS_BLOCK - 1) / (kBinRounds * GSBS_BLOCK);
        hipLaunchKernelGGL(k_bin_lds, dim3(g), dim3(GSBS_BLOCK), total_bins * sizeof(uint32_t), st, b.pos_in,
                           b.uid_in, b.ctr, P, b.cell_count, b.cellrank, b.xnew, fixed, total_bins, ns);
    } else {
        hipLaunchKernelGGL(k_bin, dim3(grid), dim3(GSBS_BLOCK), 0, st, b.pos_in, b.uid_in, b.ctr, P,
                           b.cell_count, b.cellrank, b.xnew, fixed, ns);
    }
    mark(0, 1);
    mark(1, 0);
    if (b.scan_epoch == 1u)  // first step, or the epoch counter wrapped: no stale word may match
        hipLaunchKernelGGL(k_fill_u64, dim3((nb + 255) / 256), dim3(256), 0, st, b.scan_status, nb, 0ull);
    hipLaunchKernelGGL(k_scan, dim3(nb), dim3(GSBS_BLOCK), 0, st, b.cell_count, total_bins, b.scan_status,
                       b.scan_epoch, b.cell_start, b.ctr);
    mark(1, 1);
    mark(2, 0);
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(GSBS_BLOCK), 0, st, b.pos_in, b.uid_in, b.ctr, b.xnew,
                       b.cellrank, b.cell_start, b.pos_out, b.pos0_out, b.uid_out,
                       fixed ? b.x0_override : nullptr);
    mark(2, 1);
    mark(3, 0);
    if (flags & kStepHasWhole)
        hipLaunchKernelGGL(k_pairs, dim3(grid), dim3(GSBS_BLOCK), 0, st, b.pos_out, b.pos0_out, b.uid_out,
                           b.ctr, P, chem, b.cell_start, b.pairs, b.pair_cap, (flags & kStepLogAll) ? 1 : 0, ns);
    mark(3, 1);
    mark(4, 0);
    if (flags & kStepHasSpecies) {
        int gb = (total_units + GSBS_BLOCK / 64 - 1) / (GSBS_BLOCK / 64);
        gb = gb < 1 ? 1 : (gb > 65536 ? 65536 : gb);
        hipLaunchKernelGGL(k_pairs_sp, dim3(gb), dim3(GSBS_BLOCK), 0, st, b.pos_out, b.pos0_out, b.uid_out,
                           b.ctr, P, chem, b.cell_start, b.pairs, b.pair_cap, (flags & kStepLogAll) ? 1 : 0, n_inst,
                           total_units);
    }
    mark(4, 1);
    mark(5, 0);
    hipLaunchKernelGGL(k_react, dim3(1), dim3(kReactBlock), 0, st, b.pos_out, b.uid_out, b.ctr, P, chem,
                       b.pairs, b.pair_cap, b.claim, b.mate, b.counts, b.msteps, n_inst, b.cap,
                       (flags & kStepSearchOnly) ? 1 : 0);
    if ((flags & kStepFirstOrder) && !(flags & kStepSearchOnly))
        hipLaunchKernelGGL(k_first_order, dim3(grid), dim3(GSBS_BLOCK), 0, st, b.pos_out, b.uid_out, b.ctr, P, chem,
                           b.counts, b.cap);
    mark(5, 1);
}

void launch_record(hipStream_t st, const long long* counts, long long* rec, int32_t max_rec,
                   const RecordList& list) {
    if (list.n <= 0) return;
    hipLaunchKernelGGL(k_record, dim3(list.n), dim3(kMaxSpecies), 0, st, counts, rec, max_rec, list);
}

}  // namespace gsbs
