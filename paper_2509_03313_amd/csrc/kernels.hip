// kernels.hip -- gfx950 kernels of one SBS step of the diffusion-reaction
// method of arXiv 2509.03313 (multi-pulse gMicroMC extension):
//
//   k_bin      Brownian jump (Philox4x64-10 + Box-Muller, FP32) and PBC 1
//              (Eq. 1), cell of the moved position, per-cell count and rank
//   k_scan_*   exclusive scan of the cell counts (wave64 shuffles + LDS)
//   k_scatter  molecules into cell order (jump recomputed from the counter)
//   k_pairs    27-cell minimum-image (Eq. 2) candidate search against the
//              per-reaction cutoff, radial Brownian-bridge contact
//              probability, pair uniform, accepted pairs appended
//   k_react    mutual-best single-partner matching by 64-bit atomic min,
//              products of Table 1 appended, reactants removed, species
//              counts updated
//
// All molecules of all instances live in one array; the sort groups them by
// instance (each instance owns a contiguous range of global cells).  Removed
// molecules stay in the array, flagged, until the next sort drops them.
#include "engine.h"

namespace gsbs {

#define GSBS_BLOCK 256

// --------------------------------------------------------------- Philox ---
// Philox4x64-10 (Salmon et al., SC'11): multipliers 0xD2E7470EE14C6C93 and
// 0xCA5A826395121157, Weyl increments 0x9E3779B97F4A7C15 and 0xBB67AE8584CAA73B.
__device__ __forceinline__ void philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                       uint64_t k0, uint64_t k1, uint64_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        const uint64_t lo0 = 0xD2E7470EE14C6C93ull * c0;
        const uint64_t hi0 = __umul64hi(0xD2E7470EE14C6C93ull, c0);
        const uint64_t lo1 = 0xCA5A826395121157ull * c2;
        const uint64_t hi1 = __umul64hi(0xCA5A826395121157ull, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// ln(u) for u = (k + 1/2) 2^-24, k = top 24 bits of w.  Both branches feed an
// exactly representable FP32 argument: 2k+1 < 2^24 below the midpoint, and
// 1 - u = (2^25 - 2k - 1) 2^-25 above it (log1p keeps it accurate near u = 1).
__device__ __forceinline__ float ln_u24(uint64_t w) {
    const uint32_t k = (uint32_t)(w >> 40);
    if (k < (1u << 23)) return logf((float)(2u * k + 1u) * 0x1p-25f);
    return log1pf(-(float)((1u << 25) - 2u * k - 1u) * 0x1p-25f);
}

// sin and cos of 2 pi u, u = (k + 1/2) 2^-24: 2 pi u = pi x with x = (2k+1) 2^-24;
// above the midpoint x is folded to 2 - x so the sincospi argument stays exact.
__device__ __forceinline__ void sincos_2pi_u24(uint64_t w, float* s, float* c) {
    const uint32_t k = (uint32_t)(w >> 40);
    float ss, cc;
    if (k < (1u << 23)) {
        sincospif((float)(2u * k + 1u) * 0x1p-24f, &ss, &cc);
        *s = ss;
        *c = cc;
    } else {
        sincospif((float)((1u << 25) - 2u * k - 1u) * 0x1p-24f, &ss, &cc);
        *s = -ss;
        *c = cc;
    }
}

// PBC 1 (Eq. 1); a jump may exceed one edge, so whole edges are removed first.
__device__ __forceinline__ float wrap_f(float x, float L, float hL, float invL) {
    const float k = floorf(__fmul_rn(__fadd_rn(x, hL), invL));
    x = __fsub_rn(x, __fmul_rn(k, L));
    if (x >= hL) x = __fsub_rn(x, L);
    if (x < -hL) x = __fadd_rn(x, L);
    return x;
}

// PBC 2 (Eq. 2).
__device__ __forceinline__ float minimg_f(float d, float L, float hL) {
    if (d >= hL) return __fsub_rn(d, L);
    if (d < -hL) return __fadd_rn(d, L);
    return d;
}

// Position after this step's Brownian jump: Gaussian of variance 2 D dt per
// axis from the Philox block at counter (uid, step, 0, 0), key (seed, instance).
__device__ __forceinline__ float3 jump(float4 p, uint64_t uid, const InstStep& S, int sp) {
    float3 x = make_float3(p.x, p.y, p.z);
    if (!S.active) return x;
    uint64_t w[4];
    philox(uid, S.step, 0ull, 0ull, S.key0, S.key1, w);
    const float ra = sqrtf(-2.0f * ln_u24(w[0]));
    const float rb = sqrtf(-2.0f * ln_u24(w[2]));
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
__global__ __launch_bounds__(GSBS_BLOCK) void k_bin(const float4* __restrict__ pos,
                                                  const uint64_t* __restrict__ uid,
                                                  DevCounters* __restrict__ ctr,
                                                  const InstStep* __restrict__ P,
                                                  uint32_t* __restrict__ cell_count,
                                                  uint2* __restrict__ cellrank, int32_t fixed) {
    const int n = ctr->n_in;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->n_pairs = 0u;  // read by k_pairs, after this kernel
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float4 p = pos[i];
        const int meta = __float_as_int(p.w);
        const int sp = meta & 0xFF;
        if (sp == kDead) {
            cellrank[i] = make_uint2(kNoCell, 0u);
            continue;
        }
        const InstStep& S = P[meta >> 8];
        const float3 x = fixed ? make_float3(p.x, p.y, p.z) : jump(p, uid[i], S, sp);
        const uint32_t c = (uint32_t)(S.cell_base + local_cell(x, S));
        const uint32_t r = atomicAdd(&cell_count[c], 1u);
        cellrank[i] = make_uint2(c, r);
    }
}

// ----------------------------------------------------------------- scan ---
constexpr int kScanItems = 16;
constexpr int kScanTile = GSBS_BLOCK * kScanItems;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

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

__global__ __launch_bounds__(GSBS_BLOCK) void k_scan_reduce(const uint32_t* __restrict__ cnt, int32_t total,
                                                          uint32_t* __restrict__ block_sums) {
    const int base = blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int c = base + k * GSBS_BLOCK + threadIdx.x;
        if (c < total) s += cnt[c];
    }
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(GSBS_BLOCK) void k_scan_apply(uint32_t* __restrict__ cnt, int32_t total,
                                                         const uint32_t* __restrict__ block_sums,
                                                         uint32_t* __restrict__ start,
                                                         DevCounters* __restrict__ ctr) {
    // offset of this tile: sum of the block sums before it
    uint32_t part = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += GSBS_BLOCK) part += block_sums[b];
    uint32_t off_total;
    block_excl_scan(part, &off_total);
    const uint32_t tile_off = off_total;

    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int c = base + k;
        v[k] = c < total ? cnt[c] : 0u;
        sum += v[k];
    }
    uint32_t blk_total;
    uint32_t run = tile_off + block_excl_scan(sum, &blk_total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int c = base + k;
        if (c < total) {
            start[c] = run;
            cnt[c] = 0u;
        }
        run += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        start[total] = tile_off + blk_total;
        ctr->n_live = (int32_t)(tile_off + blk_total);
    }
}

// -------------------------------------------------------------- scatter ---
__global__ __launch_bounds__(GSBS_BLOCK) void k_scatter(const float4* __restrict__ pos,
                                                      const uint64_t* __restrict__ uid,
                                                      const DevCounters* __restrict__ ctr,
                                                      const InstStep* __restrict__ P,
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
        const int meta = __float_as_int(p.w);
        const uint64_t u = uid[i];
        const uint32_t dst = start[cr.x] + cr.y;
        float3 x;
        float4 p0;
        if (x0_override) {
            x = make_float3(p.x, p.y, p.z);
            p0 = x0_override[i];
        } else {
            x = jump(p, u, P[meta >> 8], meta & 0xFF);
            p0 = p;
        }
        pos_out[dst] = make_float4(x.x, x.y, x.z, p.w);
        pos0_out[dst] = make_float4(p0.x, p0.y, p0.z, __uint_as_float(cr.x));
        uid_out[dst] = u;
    }
}

// ---------------------------------------------------------- pair search ---
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

__global__ __launch_bounds__(GSBS_BLOCK) void k_pairs(const float4* __restrict__ pos,
                                                    const float4* __restrict__ pos0,
                                                    const uint64_t* __restrict__ uid,
                                                    DevCounters* __restrict__ ctr,
                                                    const InstStep* __restrict__ P,
                                                    const ChemDev* __restrict__ chem,
                                                    const uint32_t* __restrict__ start,
                                                    PairRec* __restrict__ pairs, uint32_t pair_cap,
                                                    int32_t log_all) {
    __shared__ int32_t rmap[kMaxSpecies * kMaxSpecies];
    for (int k = threadIdx.x; k < kMaxSpecies * kMaxSpecies; k += blockDim.x)
        rmap[k] = chem->rmap[k / kMaxSpecies][k % kMaxSpecies];
    __syncthreads();
    const uint32_t reactive = chem->reactive_mask;
    const int contact_only = chem->contact_only;
    const int n = ctr->n_live;
    unsigned long long ncand = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float4 pi = pos[i];
        const int mi = __float_as_int(pi.w);
        const int si = mi & 0xFF;
        if (!((reactive >> si) & 1u)) continue;
        const InstStep& S = P[mi >> 8];
        if (!S.active) continue;
        const float4 qi = pos0[i];
        const int ci = (int)__float_as_uint(qi.w);
        const int nc = S.nc;
        const int loc = ci - S.cell_base;
        const int ix = loc / (nc * nc), iy = (loc / nc) % nc, iz = loc % nc;
        const uint64_t ui = uid[i];
        const int* row = rmap + si * kMaxSpecies;
        const float L = S.L, hL = S.halfL;
        for (int ox = -1; ox <= 1; ++ox) {
            if ((nc == 1 && ox != 0) || (nc == 2 && ox == 1)) continue;
            const int qx = (ix + ox + nc) % nc;
            for (int oy = -1; oy <= 1; ++oy) {
                if ((nc == 1 && oy != 0) || (nc == 2 && oy == 1)) continue;
                const int qy = (iy + oy + nc) % nc;
                for (int oz = -1; oz <= 1; ++oz) {
                    if ((nc == 1 && oz != 0) || (nc == 2 && oz == 1)) continue;
                    const int qz = (iz + oz + nc) % nc;
                    const int c2 = S.cell_base + (qx * nc + qy) * nc + qz;
                    if (c2 < ci) continue;  // each unordered pair of cells once
                    int j = (c2 == ci) ? i + 1 : (int)start[c2];
                    const int j1 = (int)start[c2 + 1];
                    for (; j < j1; ++j) {
                        const float4 pj = pos[j];
                        const int rx = row[__float_as_int(pj.w) & 0xFF];
                        if (rx < 0) continue;
                        const float dx = minimg_f(__fsub_rn(pj.x, pi.x), L, hL);
                        const float dy = minimg_f(__fsub_rn(pj.y, pi.y), L, hL);
                        const float dz = minimg_f(__fsub_rn(pj.z, pi.z), L, hL);
                        const float d2 = __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
                        if (!(d2 < S.rc2[rx])) continue;
                        ++ncand;
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
                            if (!log_all && r0 > R && r1 > R && a > 18.0f) continue;
                            Pc = bridge_f(r0, r1, R, S.inv_s[rx]);
                        }
                        if (!log_all && !(Pc > 0x1p-25f)) continue;
                        const uint64_t uj = uid[j];
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
                }
            }
        }
    }
    if (ncand) atomicAdd(&ctr->cand, ncand);
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
    __shared__ int n_new, n_prod, n_react;
    const int tid = threadIdx.x;
    // molecule-steps of the instances that stepped (counts before this step's reactions)
    for (int t = tid; t < n_inst; t += kReactBlock) {
        if (!P[t].active) continue;
        long long s = 0;
        for (int k = 0; k < chem->n_species; ++k) s += counts[t * kMaxSpecies + k];
        msteps[t] += (unsigned long long)s;
    }
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
    for (int round = 0; round < chem->rounds; ++round) {
        for (int p = tid; p < np; p += kReactBlock) {
            const PairRec r = pairs[p];
            if (!(r.flags & 1) || ld_mate(&mate[r.i]) >= 0 || ld_mate(&mate[r.j]) >= 0) continue;
            atomicMin(&claim[r.i], match_key(r.u24, uid[r.j]));
            atomicMin(&claim[r.j], match_key(r.u24, uid[r.i]));
        }
        if (tid == 0) n_new = 0;
        __syncthreads();
        for (int p = tid; p < np; p += kReactBlock) {
            const PairRec r = pairs[p];
            if (!(r.flags & 1) || ld_mate(&mate[r.i]) >= 0 || ld_mate(&mate[r.j]) >= 0) continue;
            const unsigned long long ci = __hip_atomic_load(&claim[r.i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long cj = __hip_atomic_load(&claim[r.j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ci == match_key(r.u24, uid[r.j]) && cj == match_key(r.u24, uid[r.i])) {
                pairs[p].flags = r.flags | 4;
                atomicAdd(&n_new, 1);
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
        if (n_new == 0) break;
        __syncthreads();
    }
    // products, removals, counts
    for (int p = tid; p < np; p += kReactBlock) {
        const PairRec r = pairs[p];
        if (!(r.flags & 2)) continue;
        int a = r.i, b = r.j;
        uint64_t ua = uid[a], ub = uid[b];
        if (ub < ua) {
            const int t = a; a = b; b = t;
            const uint64_t tu = ua; ua = ub; ub = tu;
        }
        st_mate(&mate[a], -1);
        st_mate(&mate[b], -1);
        const float4 pa = pos[a], pb = pos[b];
        const int ma = __float_as_int(pa.w), mb = __float_as_int(pb.w);
        const int inst = ma >> 8;
        const int sa = ma & 0xFF, sb = mb & 0xFF;
        const int rx = r.rx;
        long long* cnt = counts + inst * kMaxSpecies;
        atomicAdd(&n_react, 1);
        if (chem->keep_b[rx]) {
            const int gone = (sa == chem->rb[rx]) ? b : a;
            const int sg = (gone == a) ? sa : sb;
            pos[gone].w = __int_as_float((inst << 8) | kDead);
            atomicAdd((unsigned long long*)&cnt[sg], (unsigned long long)(-1ll));
            continue;
        }
        pos[a].w = __int_as_float((inst << 8) | kDead);
        pos[b].w = __int_as_float((inst << 8) | kDead);
        atomicAdd((unsigned long long*)&cnt[sa], (unsigned long long)(-1ll));
        atomicAdd((unsigned long long*)&cnt[sb], (unsigned long long)(-1ll));
        const int npr = chem->nprod[rx];
        if (npr == 0) continue;
        const InstStep& S = P[inst];
        const float Da = chem->D[sa], Db = chem->D[sb];
        const float wgt = (Da + Db > 0.0f) ? Da / (Da + Db) : 0.5f;
        const float px = wrap_f(pa.x + wgt * minimg_f(pb.x - pa.x, S.L, S.halfL), S.L, S.halfL, S.invL);
        const float py = wrap_f(pa.y + wgt * minimg_f(pb.y - pa.y, S.L, S.halfL), S.L, S.halfL, S.invL);
        const float pz = wrap_f(pa.z + wgt * minimg_f(pb.z - pa.z, S.L, S.halfL), S.L, S.halfL, S.invL);
        const int base = atomicAdd(&n_prod, npr);
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
    __syncthreads();
    if (tid == 0) {
        const int nn = n_live + n_prod;
        ctr->n_in = nn > cap ? cap : nn;
        ctr->reactions += (unsigned long long)n_react;
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

const char* const kStepKernelNames[kStepKernels] = {"k_bin", "k_scan_reduce", "k_scan_apply",
                                                     "k_scatter", "k_pairs", "k_react"};

void launch_step(hipStream_t st, const StepBuffers& b, const InstStep* P, const ChemDev* chem,
                 int32_t n_inst, int32_t total_cells, int32_t grid, int32_t flags, hipEvent_t* ev) {
    const int fixed = (flags & kStepFixed) ? 1 : 0;
    const int nb = (total_cells + kScanTile - 1) / kScanTile;
    int k = 0;
    auto mark = [&](int end) {
        if (ev) (void)hipEventRecord(ev[2 * k + end], st);
        if (end) ++k;
    };
    mark(0);
    hipLaunchKernelGGL(k_bin, dim3(grid), dim3(GSBS_BLOCK), 0, st, b.pos_in, b.uid_in, b.ctr, P,
                       b.cell_count, b.cellrank, fixed);
    mark(1);
    mark(0);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(GSBS_BLOCK), 0, st, b.cell_count, total_cells,
                       b.block_sums);
    mark(1);
    mark(0);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(GSBS_BLOCK), 0, st, b.cell_count, total_cells,
                       b.block_sums, b.cell_start, b.ctr);
    mark(1);
    mark(0);
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(GSBS_BLOCK), 0, st, b.pos_in, b.uid_in, b.ctr, P,
                       b.cellrank, b.cell_start, b.pos_out, b.pos0_out, b.uid_out,
                       fixed ? b.x0_override : nullptr);
    mark(1);
    mark(0);
    hipLaunchKernelGGL(k_pairs, dim3(grid), dim3(GSBS_BLOCK), 0, st, b.pos_out, b.pos0_out, b.uid_out,
                       b.ctr, P, chem, b.cell_start, b.pairs, b.pair_cap,
                       (flags & kStepLogAll) ? 1 : 0);
    mark(1);
    mark(0);
    hipLaunchKernelGGL(k_react, dim3(1), dim3(kReactBlock), 0, st, b.pos_out, b.uid_out, b.ctr, P, chem,
                       b.pairs, b.pair_cap, b.claim, b.mate, b.counts, b.msteps, n_inst, b.cap,
                       (flags & kStepSearchOnly) ? 1 : 0);
    mark(1);
}

void launch_record(hipStream_t st, const long long* counts, long long* rec, int32_t max_rec,
                   const RecordList& list) {
    if (list.n <= 0) return;
    hipLaunchKernelGGL(k_record, dim3(list.n), dim3(kMaxSpecies), 0, st, counts, rec, max_rec, list);
}

}  // namespace gsbs
