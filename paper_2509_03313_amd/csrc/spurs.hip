// spurs.hip -- a pulse of spurs generated on the device (the input side: this
// counter-based spur model stands in for the paper's physical and
// physico-chemical stages, which are out of scope).  Straight tracks parallel
// to z through the cube, spur centres at exponential spacing along each
// track, a Poisson number of molecules per spur, species from fixed
// fractions, Gaussian offsets per axis.  Every draw comes from a Philox4x64-10
// block keyed by (stream, track, spur, molecule), so the two passes (count,
// then emit) see the same pulse and a host implementation can reproduce it:
//   track k, block (stream, k, 0, 0): x = -L/2 + L u0, y = -L/2 + L u1;
//   spur j, block (stream, k, j + 1, 0): z_j = z_{j-1} - spacing ln u0
//     (z_{-1} = -L/2; the track ends at the first z_j >= L/2), molecule count
//     by inversion of the Poisson CDF at u1 (at most 64);
//   molecule m, block (stream, k, j + 1, 2m + 1): offsets
//     sigma sqrt(-2 ln u0) (cos, sin)(2 pi u1) on x, y and
//     sigma sqrt(-2 ln u2) cos(2 pi u3) on z; block (stream, k, j + 1, 2m + 2):
//     species = first s with u0 < cum[s] (the last species with a positive
//     fraction otherwise);
// u = (top 53 bits + 1/2) 2^-53, key (seed, 0x53505552534D4F44).  FP64
// arithmetic, positions wrapped into [-L/2, L/2) and stored as FP32.
#include "device_common.h"
#include "engine.h"

namespace gsbs {

namespace {

constexpr uint64_t kSpurKey = 0x53505552534D4F44ull;
constexpr uint64_t kMaxSpurs = 1ull << 20;

__device__ __forceinline__ double u53s(uint64_t w) {
    return ((double)(w >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ double wrap_d(double x, double L) {
    x -= L * floor((x + 0.5 * L) / L);
    if (x >= 0.5 * L) x -= L;
    if (x < -0.5 * L) x += L;
    return x;
}

__device__ __forceinline__ float to_box(double x, double L) {
    const float f = (float)x, hL = (float)(0.5 * L);
    return f >= hL ? f - (float)L : f;  // FP32 rounding may reach L/2
}

// One track's spurs: with out == nullptr only counts its molecules.
__device__ int64_t walk_track(const SpurParams& P, int k, float* __restrict__ xyz, uint8_t* __restrict__ sp) {
    uint64_t w[4];
    philox(P.stream, (uint64_t)k, 0ull, 0ull, P.seed, kSpurKey, w);
    const double L = P.L;
    const double x = -0.5 * L + L * u53s(w[0]), y = -0.5 * L + L * u53s(w[1]);
    const double two_pi = 6.283185307179586476925286766559;
    double z = -0.5 * L;
    int64_t n = 0;
    for (uint64_t j = 0; j < kMaxSpurs; ++j) {
        philox(P.stream, (uint64_t)k, j + 1, 0ull, P.seed, kSpurKey, w);
        z = z - P.spacing * log(u53s(w[0]));
        if (z >= 0.5 * L) break;
        const double u = u53s(w[1]);
        int cnt = 0;
        double p = exp(-P.mean), F = p;
        while (u > F && cnt < 64) {
            ++cnt;
            p *= P.mean / cnt;
            F += p;
        }
        if (xyz) {
            for (int m = 0; m < cnt; ++m) {
                uint64_t v[4];
                philox(P.stream, (uint64_t)k, j + 1, (uint64_t)(2 * m + 1), P.seed, kSpurKey, v);
                const double r1 = P.sigma * sqrt(-2.0 * log(u53s(v[0])));
                const double a1 = two_pi * u53s(v[1]);
                const double r2 = P.sigma * sqrt(-2.0 * log(u53s(v[2])));
                const double a2 = two_pi * u53s(v[3]);
                philox(P.stream, (uint64_t)k, j + 1, (uint64_t)(2 * m + 2), P.seed, kSpurKey, v);
                const double us = u53s(v[0]);
                int s_pick = P.last;
                for (int s = 0; s < P.ns; ++s)
                    if (us < P.cum[s]) {
                        s_pick = s;
                        break;
                    }
                const int64_t o = n + m;
                xyz[3 * o + 0] = to_box(wrap_d(x + r1 * cos(a1), L), L);
                xyz[3 * o + 1] = to_box(wrap_d(y + r1 * sin(a1), L), L);
                xyz[3 * o + 2] = to_box(wrap_d(z + r2 * cos(a2), L), L);
                sp[o] = (uint8_t)s_pick;
            }
        }
        n += cnt;
    }
    return n;
}

__global__ __launch_bounds__(64) void k_spur_count(SpurParams P, int64_t* __restrict__ cnt) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < P.n_tracks) cnt[k] = walk_track(P, k, nullptr, nullptr);
}

__global__ __launch_bounds__(64) void k_spur_emit(SpurParams P, const int64_t* __restrict__ off,
                                                  float* __restrict__ xyz, uint8_t* __restrict__ sp) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < P.n_tracks) (void)walk_track(P, k, xyz + 3 * off[k], sp + off[k]);
}

}  // namespace

void launch_spur_count(hipStream_t st, const SpurParams& P, int64_t* cnt) {
    if (P.n_tracks <= 0) return;
    hipLaunchKernelGGL(k_spur_count, dim3((P.n_tracks + 63) / 64), dim3(64), 0, st, P, cnt);
}

void launch_spur_emit(hipStream_t st, const SpurParams& P, const int64_t* off, float* xyz, uint8_t* sp) {
    if (P.n_tracks <= 0) return;
    hipLaunchKernelGGL(k_spur_emit, dim3((P.n_tracks + 63) / 64), dim3(64), 0, st, P, off, xyz, sp);
}

}  // namespace gsbs
