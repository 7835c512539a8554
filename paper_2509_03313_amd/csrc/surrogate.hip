// surrogate.hip -- gfx950 kernels that connect the SBS state with the
// inter-pulse surrogate: reference sampling and binned pair correlations
// g_ab(r), the 296 input features of the perceptron, and re-population of an
// instance with uniformly placed molecules at predicted counts.
#include "device_common.h"
#include "engine.h"

namespace gsbs {

constexpr int kSurBlock = 256;
constexpr int kPcTile = 1024;  // molecules staged per LDS tile in the pair-correlation kernel
constexpr double kFeatureClamp = 8.0;  // |normalised feature| limit

// Reference molecules of each species: live molecules of instance `inst` with
// uid % stride[s] == 0 (a subsample that depends on the state only), at most
// cap per species (the count keeps counting past cap).
__global__ __launch_bounds__(kSurBlock) void k_collect_refs(const float4* __restrict__ pos,
                                                          const uint64_t* __restrict__ uid,
                                                          const DevCounters* __restrict__ ctr, int32_t inst,
                                                          SurStrides strides, int32_t cap,
                                                          int32_t* __restrict__ ref_idx,
                                                          int32_t* __restrict__ ref_cnt, uint32_t* __restrict__ err) {
    const int n = ctr->n_in;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int meta = __float_as_int(pos[i].w);
        const int s = meta & 0xFF;
        if ((meta >> 8) != inst || s == kDead || s >= kMaxSpecies) continue;
        if (uid[i] % (uint64_t)strides.s[s] != 0ull) continue;
        const int k = atomicAdd(&ref_cnt[s], 1);
        if (k < cap) ref_idx[s * cap + k] = i;  // the host checks ref_cnt <= cap
    }
}

// Pair counts in log-spaced shells: blockIdx.y = pair p (species a, b), one
// thread per reference of species a; every molecule of the instance is staged
// through LDS and those of species b (other than the reference) are binned by
// their FP32 minimum-image distance (Eq. 2, fixed operation order) against the
// squared FP32 shell edges edges2[p][0..32]: bin k for edges2[k] <= d2 <
// edges2[k+1], bin 0 also below edges2[0], nothing from edges2[32] on.
__global__ __launch_bounds__(kSurBlock) void k_pair_corr(const float4* __restrict__ pos,
                                                       const DevCounters* __restrict__ ctr, int32_t inst,
                                                       const int32_t* __restrict__ ref_idx,
                                                       const int32_t* __restrict__ ref_cnt, int32_t cap,
                                                       const int32_t* __restrict__ pair_ab,
                                                       const float* __restrict__ edges2, float L,
                                                       unsigned long long* __restrict__ hist) {
    __shared__ float4 tile[kPcTile];
    __shared__ float e2[kSurBins + 1];
    __shared__ unsigned int h[kSurBins];
    const int p = blockIdx.y;
    const int a = pair_ab[2 * p], b = pair_ab[2 * p + 1];
    if (threadIdx.x <= kSurBins) e2[threadIdx.x] = edges2[p * (kSurBins + 1) + threadIdx.x];
    if (threadIdx.x < kSurBins) h[threadIdx.x] = 0u;
    const int nref = min(ref_cnt[a], cap);
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const bool has = r < nref;
    const int ia = has ? ref_idx[a * cap + r] : -1;
    float4 pa = make_float4(0.f, 0.f, 0.f, 0.f);
    if (has) pa = pos[ia];
    const float hL = 0.5f * L;
    // blockIdx.z takes one contiguous share of the molecule array
    const int n = ctr->n_in;
    const int share = (n + gridDim.z - 1) / gridDim.z;
    const int m0 = blockIdx.z * share, m1 = min(n, m0 + share);
    const int want = (inst << 8) | b;
    __syncthreads();
    if (blockIdx.x * blockDim.x >= nref) return;  // the whole block has no reference (uniform)
    for (int t0 = m0; t0 < m1; t0 += kPcTile) {
        const int cnt = min(kPcTile, m1 - t0);
        for (int k = threadIdx.x; k < cnt; k += blockDim.x) tile[k] = pos[t0 + k];
        __syncthreads();
        if (has) {
            for (int k = 0; k < cnt; ++k) {
                const float4 q = tile[k];
                if (__float_as_int(q.w) != want || t0 + k == ia) continue;
                const float dx = minimg_f(__fsub_rn(q.x, pa.x), L, hL);
                const float dy = minimg_f(__fsub_rn(q.y, pa.y), L, hL);
                const float dz = minimg_f(__fsub_rn(q.z, pa.z), L, hL);
                const float d2 = __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
                if (!(d2 < e2[kSurBins])) continue;
                int lo = 0, hi = kSurBins - 1;  // largest k with e2[k] <= d2 (0 when below e2[0])
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (e2[mid] <= d2) lo = mid;
                    else hi = mid - 1;
                }
                atomicAdd(&h[lo], 1u);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < kSurBins && h[threadIdx.x])
        atomicAdd(&hist[p * kSurBins + threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// The 296 features of the perceptron for one instance, normalised as
// (f - mu) / sd (clamped to +-8 when clamp is set): log10(C_s + c_floor) of the 7 species (C in mol/L), the
// pair correlations g_p(k) = hist / (n_ref rho_b V_k) of the 9 reactions x 32
// shells (1 where a pair has no reference or no partner), log10(dt_next / ns).
__global__ void k_features(const long long* __restrict__ counts, int32_t inst, int32_t ns,
                           const unsigned long long* __restrict__ hist, const int32_t* __restrict__ ref_cnt,
                           int32_t cap, const int32_t* __restrict__ pair_ab, const double* __restrict__ shell_vol,
                           int32_t n_pairs, double L, double dt_next, double c_floor, const float* __restrict__ mu,
                           const float* __restrict__ sd, int32_t clamp, float* __restrict__ out) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = ns + n_pairs * kSurBins + 1;
    if (f >= nf) return;
    const double vol_nm3 = L * L * L;
    double v;
    if (f < ns) {
        const double conc = (double)counts[inst * kMaxSpecies + f] / (6.02214076e23 * vol_nm3 * 1e-24);
        v = log10(conc + c_floor);
    } else if (f < ns + n_pairs * kSurBins) {
        const int p = (f - ns) / kSurBins, k = (f - ns) % kSurBins;
        const int a = pair_ab[2 * p], b = pair_ab[2 * p + 1];
        const double nref = (double)min(ref_cnt[a], cap);
        const double nb = (double)counts[inst * kMaxSpecies + b] - (a == b ? 1.0 : 0.0);
        const double expect = nref * (nb / vol_nm3) * shell_vol[p * kSurBins + k];
        v = (nref > 0 && nb > 0) ? (double)hist[p * kSurBins + k] / expect : 1.0;
    } else {
        v = log10(dt_next);
    }
    // normalised, and clamped so that a feature far outside the training range
    // cannot drive the network into extrapolation without bound
    const double z = (v - (double)mu[f]) / (double)sd[f];
    out[f] = (float)(clamp ? fmin(kFeatureClamp, fmax(-kFeatureClamp, z)) : z);
}

// Counts of the re-populated instance: the network output y (normalised
// log10 concentrations, or their change from the present state) back to
// mol/L, to a mean count in the cube, rounded stochastically with the Philox
// word at counter (species, step, 0, 3).
__global__ void k_repop_counts(const float* __restrict__ y, const float* __restrict__ mu,
                               const float* __restrict__ sd, int32_t ns, double c_floor, double vol_litre,
                               uint64_t seed, int32_t inst, uint64_t step, int32_t relative,
                               const long long* __restrict__ counts, long long* __restrict__ out) {
    const int s = threadIdx.x;
    if (s >= ns) return;
    double lc = (double)y[s] * (double)sd[s] + (double)mu[s];
    // relative: y encodes the change of log10(C + c_floor) from the present state
    if (relative) lc += log10((double)counts[inst * kMaxSpecies + s] / (6.02214076e23 * vol_litre) + c_floor);
    const double conc = fmax(0.0, pow(10.0, lc) - c_floor);
    const double mean = conc * 6.02214076e23 * vol_litre;
    uint64_t w[4];
    philox((uint64_t)s, step, 0ull, 3ull, seed, (uint64_t)inst, w);
    const double u = ((double)(w[0] >> 11) + 0.5) * 0x1p-53;
    const double fl = floor(mean);
    out[s] = (long long)fl + ((u < mean - fl) ? 1 : 0);
}

// Remove every molecule of instance inst (flagged; the next sort drops them)
// and zero its species counts.
__global__ void k_repop_clear(float4* __restrict__ pos, const DevCounters* __restrict__ ctr, int32_t inst,
                              long long* __restrict__ counts) {
    const int n = ctr->n_in;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int meta = __float_as_int(pos[i].w);
        if ((meta >> 8) == inst) pos[i].w = __int_as_float((inst << 8) | kDead);
    }
    if (blockIdx.x == 0 && threadIdx.x < kMaxSpecies) counts[inst * kMaxSpecies + threadIdx.x] = 0;
}

// Append n_new molecules at uniform positions: molecule k has uid uid_base + k,
// species by the prefix sums of the new counts, and coordinates from the
// Philox word at counter (uid, step, 1, 3), key (seed, inst).
__global__ __launch_bounds__(kSurBlock) void k_repop_place(float4* __restrict__ pos, uint64_t* __restrict__ uid,
                                                         const DevCounters* __restrict__ ctr,
                                                         const long long* __restrict__ newc, int32_t ns,
                                                         int32_t n_new, int32_t inst, uint64_t uid_base,
                                                         uint64_t seed, uint64_t step, float L, int32_t cap,
                                                         long long* __restrict__ counts,
                                                         uint32_t* __restrict__ err) {
    const int base = ctr->n_in;
    const float hL = 0.5f * L, invL = 1.0f / L;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_new; k += gridDim.x * blockDim.x) {
        const int dst = base + k;
        if (dst >= cap) {
            atomicOr(err, kErrMolOverflow);
            continue;
        }
        int s = 0;
        long long acc = newc[0];
        while (s + 1 < ns && k >= acc) acc += newc[++s];
        const uint64_t u = uid_base + (uint64_t)k;
        uint64_t w[4];
        philox(u, step, 1ull, 3ull, seed, (uint64_t)inst, w);
        const float x = wrap_f((u24_f(w[0]) - 0.5f) * L, L, hL, invL);
        const float y = wrap_f((u24_f(w[1]) - 0.5f) * L, L, hL, invL);
        const float z = wrap_f((u24_f(w[2]) - 0.5f) * L, L, hL, invL);
        pos[dst] = make_float4(x, y, z, __int_as_float((inst << 8) | s));
        uid[dst] = u;
    }
    if (blockIdx.x == 0 && threadIdx.x < ns)
        atomicAdd((unsigned long long*)&counts[inst * kMaxSpecies + threadIdx.x],
                  (unsigned long long)newc[threadIdx.x]);
}

void launch_collect_refs(hipStream_t st, const float4* pos, const uint64_t* uid, const DevCounters* ctr, int inst,
                         const SurStrides& strides, int cap, int32_t* ref_idx, int32_t* ref_cnt, uint32_t* err,
                         int grid) {
    hipLaunchKernelGGL(k_collect_refs, dim3(grid), dim3(kSurBlock), 0, st, pos, uid, ctr, inst, strides, cap, ref_idx,
                       ref_cnt, err);
}
void launch_pair_corr(hipStream_t st, const float4* pos, const DevCounters* ctr, int inst, const int32_t* ref_idx,
                      const int32_t* ref_cnt, int cap, const int32_t* pair_ab, const float* edges2, int n_pairs,
                      float L, unsigned long long* hist, int64_t n_est) {
    int64_t z = (n_est + 32767) / 32768;
    z = z < 1 ? 1 : (z > 64 ? 64 : z);
    hipLaunchKernelGGL(k_pair_corr, dim3((cap + kSurBlock - 1) / kSurBlock, n_pairs, (unsigned)z), dim3(kSurBlock), 0,
                       st, pos, ctr, inst, ref_idx, ref_cnt, cap, pair_ab, edges2, L, hist);
}
void launch_features(hipStream_t st, const long long* counts, int inst, int ns, const unsigned long long* hist,
                     const int32_t* ref_cnt, int cap, const int32_t* pair_ab, const double* shell_vol, int n_pairs,
                     double L, double dt_next, double c_floor, const float* mu, const float* sd, int clamp,
                     float* out) {
    const int nf = ns + n_pairs * kSurBins + 1;
    hipLaunchKernelGGL(k_features, dim3((nf + kSurBlock - 1) / kSurBlock), dim3(kSurBlock), 0, st, counts, inst, ns,
                       hist, ref_cnt, cap, pair_ab, shell_vol, n_pairs, L, dt_next, c_floor, mu, sd, clamp, out);
}
void launch_repop_counts(hipStream_t st, const float* y, const float* mu, const float* sd, int ns, double c_floor,
                         double vol_litre, uint64_t seed, int inst, uint64_t step, int relative,
                         const long long* counts, long long* out) {
    hipLaunchKernelGGL(k_repop_counts, dim3(1), dim3(kMaxSpecies), 0, st, y, mu, sd, ns, c_floor, vol_litre, seed,
                       inst, step, relative, counts, out);
}
__global__ void k_sur_add_n(DevCounters* ctr, int32_t n, int32_t cap) {
    const int v = ctr->n_in + n;
    ctr->n_in = v > cap ? cap : v;
}

void launch_repop(hipStream_t st, float4* pos, uint64_t* uid, DevCounters* ctr, const long long* newc, int ns,
                  int n_new, int inst, uint64_t uid_base, uint64_t seed, uint64_t step, float L, int cap,
                  long long* counts, int grid) {
    hipLaunchKernelGGL(k_repop_clear, dim3(grid), dim3(kSurBlock), 0, st, pos, ctr, inst, counts);
    const int g2 = n_new > 0 ? (n_new + kSurBlock - 1) / kSurBlock : 1;
    hipLaunchKernelGGL(k_repop_place, dim3(g2 < 65535 ? g2 : 65535), dim3(kSurBlock), 0, st, pos, uid, ctr, newc, ns,
                       n_new, inst, uid_base, seed, step, L, cap, counts, &ctr->err);
    hipLaunchKernelGGL(k_sur_add_n, dim3(1), dim3(1), 0, st, ctr, n_new, cap);
}

}  // namespace gsbs
