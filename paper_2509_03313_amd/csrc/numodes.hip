// numodes.hip -- the homogeneous rate equations of the beam-off stage (the
// paper's NumODEs, Eq. 3-4, with the self-recombination factor of its
// rate-equation appendix), integrated for many independent mixtures at once:
// one thread per mixture, FP64, the four-stage, third-order, stiffly accurate
// Rosenbrock method RODAS3 (Sandu, Verwer, Blom, Spee, Carmichael and Potra,
// Atmos. Environ. 31, 1997; Hairer and Wanner, Solving ODEs II) with its
// embedded second-order solution for step control.
//
// Stages, with gamma = 1/2 and W = I/(gamma h) - J:
//   W K1 = f(y)
//   W K2 = f(y) + 4 K1 / h
//   W K3 = f(y + 2 K1) + (K1 - K2) / h
//   W K4 = f(y + 2 K1 + K3) + (K1 - K2 - 8/3 K3) / h
//   y1 = y + 2 K1 + K3 + K4, local error estimate K4.
// One Jacobian and one LU per step serve all four stages.
//
// Event rate of reaction r between a and b: k_r [a][b] (a != b), k_r [a]^2 / 2
// (a == b; the table prints 2k for self-recombinations), k_r in L/mol/ns;
// d[X]/dt = sum_r nu_rX rate_r with nu_rX the net change of X per event
// (products minus reactants).  The stage matrix is factored in registers.
#include <mutex>
#include <string>

#include "engine.h"
#include "gsbs.h"

namespace gsbs {

namespace {

// The table's species indices are the same for every lane, so the gathers of
// y[a], y[b] and the column updates below are uniform (scalar) selections.
template <int S>
__device__ __forceinline__ void gather2(const double* y, int a, int b, double& ya, double& yb) {
    ya = 0.0;
    yb = b < 0 ? 1.0 : 0.0;  // b < 0: first-order channel, rate kr [a]
#pragma unroll
    for (int s = 0; s < S; ++s) {
        ya = s == a ? y[s] : ya;
        yb = s == b ? y[s] : yb;
    }
}

template <int S>
__device__ __forceinline__ void ode_rhs(const double* y, const OdeTable& tb, double* f) {
#pragma unroll
    for (int s = 0; s < S; ++s) f[s] = tb.src[s];  // zero-order sources
#pragma unroll 3
    for (int r = 0; r < tb.nr; ++r) {
        double ya, yb;
        gather2<S>(y, tb.ra[r], tb.rb[r], ya, yb);
        const double rho = tb.kr[r] * ya * yb;
#pragma unroll
        for (int s = 0; s < S; ++s) f[s] = fma(tb.nu[r][s], rho, f[s]);
    }
}

// J[i][j] = d f_i / d y_j = sum_r nu[r][i] d rate_r / d y_j; the rate of r
// depends on y_a and y_b only: kr y_b and kr y_a, or 2 kr y_a when a == b, or
// kr for a first-order channel (b < 0).
template <int S>
__device__ __forceinline__ void ode_jac(const double* y, const OdeTable& tb, double (*J)[S]) {
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j < S; ++j) J[i][j] = 0.0;
#pragma unroll 3
    for (int r = 0; r < tb.nr; ++r) {
        const int a = tb.ra[r], b = tb.rb[r];
        double ya, yb;
        gather2<S>(y, a, b, ya, yb);
        const double ga = (a == b ? 2.0 : 1.0) * tb.kr[r] * yb, gb = tb.kr[r] * ya;
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (j == a || j == b) {
                const double g = j == a ? ga : gb;
#pragma unroll
                for (int i = 0; i < S; ++i) J[i][j] = fma(tb.nu[r][i], g, J[i][j]);
            }
        }
    }
}

// 1/x from the hardware estimate refined by two Newton steps (each squares
// the relative error), for x normal and finite.
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// In-place LU of M.  kPivot: partial pivoting, rows exchanged by selects and
// recorded in perm for solve_lu.  Without it the diagonal is taken as the
// pivot, and the result says whether every pivot was at least a tenth of the
// largest entry below it (threshold pivoting; for mass-action stage matrices
// the diagonal, 1/(gamma h) plus the species' own loss rate, is normally the
// largest).  The diagonal receives the pivots' reciprocals.
template <int S, bool kPivot>
__device__ __forceinline__ bool factor(double (*M)[S], int* perm) {
    bool ok = true;
    if (kPivot) {
#pragma unroll
        for (int i = 0; i < S; ++i) perm[i] = i;
    }
#pragma unroll
    for (int k = 0; k < S; ++k) {
        int p = k;
        double best = fabs(M[k][k]), below = 0.0;
#pragma unroll
        for (int i = k + 1; i < S; ++i) {
            const double v = fabs(M[i][k]);
            below = fmax(below, v);
            if (kPivot && v > best) {
                best = v;
                p = i;
            }
        }
        if (kPivot) {
#pragma unroll
            for (int i = k + 1; i < S; ++i) {
                const bool sw = i == p;
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    const double a = M[k][j], b = M[i][j];
                    M[k][j] = sw ? b : a;
                    M[i][j] = sw ? a : b;
                }
                const int pa = perm[k], pb = perm[i];
                perm[k] = sw ? pb : pa;
                perm[i] = sw ? pa : pb;
            }
        } else {
            ok = ok && best >= 0.1 * below && best > 0.0;
        }
        const double inv = recip(M[k][k]);
        M[k][k] = inv;
#pragma unroll
        for (int i = k + 1; i < S; ++i) {
            const double l = M[i][k] * inv;
            M[i][k] = l;
#pragma unroll
            for (int j = k + 1; j < S; ++j) M[i][j] -= l * M[k][j];
        }
    }
    return ok;
}

template <int S, bool kPivot>
__device__ __forceinline__ void solve_lu(const double (*M)[S], const int* perm, const double* b, double* x) {
    double z[S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
        double v = b[i];
        if (kPivot) {
#pragma unroll
            for (int s = 0; s < S; ++s) v = perm[i] == s ? b[s] : v;
        }
        z[i] = v;
    }
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) z[i] -= M[i][j] * z[j];
#pragma unroll
    for (int i = S - 1; i >= 0; --i) {
#pragma unroll
        for (int j = i + 1; j < S; ++j) z[i] -= M[i][j] * z[j];
        z[i] *= M[i][i];
    }
#pragma unroll
    for (int i = 0; i < S; ++i) x[i] = z[i];
}

// W = I / (gamma h) - J at y
template <int S>
__device__ __forceinline__ void stage_matrix(const double* y, const OdeTable& tb, double dg, double (*M)[S]) {
    ode_jac<S>(y, tb, M);
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j < S; ++j) M[i][j] = (i == j ? dg : 0.0) - M[i][j];
}

template <int S>
__global__ __launch_bounds__(64) void k_numodes(const double* __restrict__ c0, const double* __restrict__ dt,
                                                double* __restrict__ c1, int32_t* __restrict__ steps, int32_t n,
                                                OdeTable tb, double rtol, double atol, int32_t max_steps) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const int ns = tb.ns;
    double y[S];
#pragma unroll
    for (int s = 0; s < S; ++s) y[s] = s < ns ? fmax(c0[(size_t)m * ns + s], 0.0) : 0.0;
    const double T = dt[m];
    const double gam = 0.5;
    double t = 0.0;
    int nstep = 0, nrej = 0;
    double f[S];
    ode_rhs<S>(y, tb, f);
    // first step: a small fraction of the fastest relative rate's time scale
    double rmax = 1.0 / fmax(T, 1e-300);
#pragma unroll
    for (int s = 0; s < S; ++s) rmax = fmax(rmax, fabs(f[s]) / (fabs(y[s]) + atol));
    double h = fmin(T, 1e-2 / rmax);
    bool ok = true;
    while (T - t > 1e-12 * T && T > 0.0) {
        if (nstep + nrej >= max_steps) {
            ok = false;
            break;
        }
        h = fmin(h, T - t);
        const double ih = 1.0 / h;
        double M[S][S];
        int perm[S];
        stage_matrix<S>(y, tb, ih / gam, M);
        // threshold-pivoted LU; a wave with any lane below the threshold
        // refactors with partial pivoting (wave-uniform branch)
        const bool piv = __builtin_amdgcn_ballot_w64(!factor<S, false>(M, perm)) != 0;
        if (piv) {
            stage_matrix<S>(y, tb, ih / gam, M);
            factor<S, true>(M, perm);
        }
        auto solve = [&](const double* rhs_, double* x_) {
            if (piv)
                solve_lu<S, true>(M, perm, rhs_, x_);
            else
                solve_lu<S, false>(M, perm, rhs_, x_);
        };
        double k1[S], d[S], k3[S], k4[S], r[S], ys[S], fs[S];
        solve(f, k1);
#pragma unroll
        for (int s = 0; s < S; ++s) r[s] = f[s] + 4.0 * ih * k1[s];
        solve(r, d);  // K2
#pragma unroll
        for (int s = 0; s < S; ++s) {
            d[s] = k1[s] - d[s];  // K1 - K2
            ys[s] = y[s] + 2.0 * k1[s];
        }
        ode_rhs<S>(ys, tb, fs);
#pragma unroll
        for (int s = 0; s < S; ++s) r[s] = fs[s] + ih * d[s];
        solve(r, k3);
#pragma unroll
        for (int s = 0; s < S; ++s) ys[s] += k3[s];
        ode_rhs<S>(ys, tb, fs);
#pragma unroll
        for (int s = 0; s < S; ++s) r[s] = fs[s] + ih * (d[s] - (8.0 / 3.0) * k3[s]);
        solve(r, k4);
        double err = 0.0, yn[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            yn[s] = ys[s] + k4[s];
            const double e = fabs(k4[s]) * recip(atol + rtol * fmax(fabs(y[s]), fabs(yn[s])));
            err = (e > err || isnan(e)) ? e : err;  // a NaN stays and rejects the step
        }
        if (err <= 1.0 && isfinite(err)) {
            t += h;
#pragma unroll
            for (int s = 0; s < S; ++s) y[s] = fmax(yn[s], 0.0);
            ode_rhs<S>(y, tb, f);
            ++nstep;
        } else {
            ++nrej;
        }
        // embedded solution of order 2: the error scales as h^3
        const double fac = !isfinite(err) ? 0.2 : err == 0.0 ? 5.0 : 0.9 * cbrt(1.0 / err);
        h *= fmin(5.0, fmax(0.2, fac));
    }
    for (int s = 0; s < ns; ++s) c1[(size_t)m * ns + s] = y[s];
    steps[m] = ok ? nstep : -1;
}

}  // namespace

// Step counts of gsbs_numodes_noalloc: a file-scope device array instead of an
// allocation (each GPU the library runs on holds its own copy until the
// process ends).  Host code never passes the array's name to a kernel: the
// per-device address from hipGetSymbolAddress, taken once per device, is
// what the launches and copies use.
static __device__ __align__(256) int32_t scratch[kNoAllocMaxMixtures];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int numodes_scratch(int32_t** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return set_error(GSBS_EHIP, "no current HIP device for the rate-equation scratch array");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(GSBS_EHIP, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
        g_scratch_ptr[dev] = static_cast<int32_t*>(p);
    }
    *out = g_scratch_ptr[dev];
    return GSBS_OK;
}

void launch_numodes(hipStream_t st, const double* c0, const double* dt, double* c1, int32_t* steps, int32_t n,
                    const OdeTable& tb, double rtol, double atol, int32_t max_steps) {
    if (n <= 0 || tb.ns > kOdeMaxSpecies) return;
    // species slots: the table's species padded with inert ones (zero rows of
    // the Jacobian) to one of three register layouts
    const dim3 grid((n + 63) / 64), block(64);
    if (tb.ns <= 4)
        hipLaunchKernelGGL(k_numodes<4>, grid, block, 0, st, c0, dt, c1, steps, n, tb, rtol, atol, max_steps);
    else if (tb.ns <= 7)
        hipLaunchKernelGGL(k_numodes<7>, grid, block, 0, st, c0, dt, c1, steps, n, tb, rtol, atol, max_steps);
    else
        hipLaunchKernelGGL(k_numodes<kOdeMaxSpecies>, grid, block, 0, st, c0, dt, c1, steps, n, tb, rtol, atol,
                           max_steps);
}

}  // namespace gsbs
