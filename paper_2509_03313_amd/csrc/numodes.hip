// numodes.hip -- the homogeneous rate equations of the beam-off stage (the
// paper's NumODEs, Eq. 3-4, with the self-recombination factor of its
// rate-equation appendix), integrated for many independent mixtures at once:
// one thread per mixture, FP64, two-stage L-stable Rosenbrock method (ROS2:
// gamma = 1 + 1/sqrt 2; Verwer, Spee, Blom and Hundsdorfer, SIAM J. Sci.
// Comput. 20, 1999) with the embedded first-order solution for step control.
//
// Event rate of reaction r between a and b: k_r [a][b] (a != b), k_r [a]^2 / 2
// (a == b; the table prints 2k for self-recombinations), k_r in L/mol/ns;
// d[X]/dt = sum_r rate_r (products X - reactants X).  The 8 x 8 stage matrix
// I - gamma h J (unused species padded with the identity) is factored in
// registers with partial pivoting done by selects.
#include "engine.h"

namespace gsbs {

namespace {

constexpr int kOS = 8;  // species slots of the integrator (kMaxSpecies)

__device__ __forceinline__ void ode_rhs(const double* y, const OdeTable& tb, double* f) {
#pragma unroll
    for (int s = 0; s < kOS; ++s) f[s] = 0.0;
    for (int r = 0; r < tb.nr; ++r) {
        const int a = tb.ra[r], b = tb.rb[r];
        double ya = 0.0, yb = 0.0;
#pragma unroll
        for (int s = 0; s < kOS; ++s) {
            ya = s == a ? y[s] : ya;
            yb = s == b ? y[s] : yb;
        }
        const double rho = (a == b ? 0.5 : 1.0) * tb.k[r] * ya * yb;
        const double da = -rho, db = tb.keep_b[r] ? 0.0 : -rho;
        const int p0 = tb.nprod[r] > 0 ? tb.prod[r][0] : -1;
        const int p1 = tb.nprod[r] > 1 ? tb.prod[r][1] : -1;
        const int p2 = tb.nprod[r] > 2 ? tb.prod[r][2] : -1;
#pragma unroll
        for (int s = 0; s < kOS; ++s) {
            double d = (s == a ? da : 0.0) + (s == b ? db : 0.0);
            d += (s == p0 ? rho : 0.0) + (s == p1 ? rho : 0.0) + (s == p2 ? rho : 0.0);
            f[s] += d;
        }
    }
}

// J[i][j] = d f_i / d y_j
__device__ __forceinline__ void ode_jac(const double* y, const OdeTable& tb, double (*J)[kOS]) {
#pragma unroll
    for (int i = 0; i < kOS; ++i)
#pragma unroll
        for (int j = 0; j < kOS; ++j) J[i][j] = 0.0;
    for (int r = 0; r < tb.nr; ++r) {
        const int a = tb.ra[r], b = tb.rb[r];
        double ya = 0.0, yb = 0.0;
#pragma unroll
        for (int s = 0; s < kOS; ++s) {
            ya = s == a ? y[s] : ya;
            yb = s == b ? y[s] : yb;
        }
        // d rate / d y_j: k y_a (j = a, a == b); k y_b (j = a), k y_a (j = b)
        double g[kOS];
#pragma unroll
        for (int j = 0; j < kOS; ++j) {
            g[j] = a == b ? (j == a ? tb.k[r] * ya : 0.0)
                          : ((j == a ? tb.k[r] * yb : 0.0) + (j == b ? tb.k[r] * ya : 0.0));
        }
        const int p0 = tb.nprod[r] > 0 ? tb.prod[r][0] : -1;
        const int p1 = tb.nprod[r] > 1 ? tb.prod[r][1] : -1;
        const int p2 = tb.nprod[r] > 2 ? tb.prod[r][2] : -1;
        const bool kb = tb.keep_b[r] != 0;
#pragma unroll
        for (int i = 0; i < kOS; ++i) {
            const double w = (i == a ? -1.0 : 0.0) + (i == b && !kb ? -1.0 : 0.0) + (i == p0 ? 1.0 : 0.0) +
                             (i == p1 ? 1.0 : 0.0) + (i == p2 ? 1.0 : 0.0);
            if (w != 0.0) {
#pragma unroll
                for (int j = 0; j < kOS; ++j) J[i][j] += w * g[j];
            }
        }
    }
}

// In-place LU of M with partial pivoting; the row exchanges are applied to
// the right-hand sides by solve_lu through perm.
__device__ __forceinline__ void factor(double (*M)[kOS], int* perm) {
#pragma unroll
    for (int i = 0; i < kOS; ++i) perm[i] = i;
#pragma unroll
    for (int k = 0; k < kOS; ++k) {
        // pivot: the largest |M[i][k]|, i >= k; rows exchanged by selects
        int p = k;
        double best = fabs(M[k][k]);
#pragma unroll
        for (int i = k + 1; i < kOS; ++i) {
            const double v = fabs(M[i][k]);
            if (v > best) {
                best = v;
                p = i;
            }
        }
#pragma unroll
        for (int i = k + 1; i < kOS; ++i) {
            const bool sw = i == p;
#pragma unroll
            for (int j = 0; j < kOS; ++j) {
                const double a = M[k][j], b = M[i][j];
                M[k][j] = sw ? b : a;
                M[i][j] = sw ? a : b;
            }
            const int pa = perm[k], pb = perm[i];
            perm[k] = sw ? pb : pa;
            perm[i] = sw ? pa : pb;
        }
        const double inv = 1.0 / M[k][k];
#pragma unroll
        for (int i = k + 1; i < kOS; ++i) {
            const double l = M[i][k] * inv;
            M[i][k] = l;
#pragma unroll
            for (int j = k + 1; j < kOS; ++j) M[i][j] -= l * M[k][j];
        }
    }
}

__device__ __forceinline__ void solve_lu(const double (*M)[kOS], const int* perm, const double* b, double* x) {
    double z[kOS];
#pragma unroll
    for (int i = 0; i < kOS; ++i) {
        double v = 0.0;
#pragma unroll
        for (int s = 0; s < kOS; ++s) v = perm[i] == s ? b[s] : v;
        z[i] = v;
    }
#pragma unroll
    for (int i = 0; i < kOS; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) z[i] -= M[i][j] * z[j];
#pragma unroll
    for (int i = kOS - 1; i >= 0; --i) {
#pragma unroll
        for (int j = i + 1; j < kOS; ++j) z[i] -= M[i][j] * z[j];
        z[i] /= M[i][i];
    }
#pragma unroll
    for (int i = 0; i < kOS; ++i) x[i] = z[i];
}

__global__ __launch_bounds__(64) void k_numodes(const double* __restrict__ c0, const double* __restrict__ dt,
                                                double* __restrict__ c1, int32_t* __restrict__ steps, int32_t n,
                                                OdeTable tb, double rtol, double atol, int32_t max_steps) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const int ns = tb.ns;
    double y[kOS];
#pragma unroll
    for (int s = 0; s < kOS; ++s) y[s] = s < ns ? fmax(c0[(size_t)m * ns + s], 0.0) : 0.0;
    const double T = dt[m];
    const double gam = 1.0 + 0.70710678118654752440;
    double t = 0.0;
    int nstep = 0, nrej = 0;
    double f[kOS];
    ode_rhs(y, tb, f);
    // first step: a small fraction of the fastest relative rate's time scale
    double rmax = 1.0 / fmax(T, 1e-300);
#pragma unroll
    for (int s = 0; s < kOS; ++s) rmax = fmax(rmax, fabs(f[s]) / (fabs(y[s]) + atol));
    double h = fmin(T, 1e-2 / rmax);
    bool ok = true;
    while (T - t > 1e-12 * T && T > 0.0) {
        if (nstep + nrej >= max_steps) {
            ok = false;
            break;
        }
        h = fmin(h, T - t);
        double J[kOS][kOS];
        ode_jac(y, tb, J);
        double M[kOS][kOS];
#pragma unroll
        for (int i = 0; i < kOS; ++i)
#pragma unroll
            for (int j = 0; j < kOS; ++j) M[i][j] = (i == j ? 1.0 : 0.0) - gam * h * J[i][j];
        int perm[kOS];
        factor(M, perm);
        double k1[kOS], k2[kOS], y2[kOS], f2[kOS], r2[kOS];
        solve_lu(M, perm, f, k1);
#pragma unroll
        for (int s = 0; s < kOS; ++s) y2[s] = y[s] + h * k1[s];
        ode_rhs(y2, tb, f2);
#pragma unroll
        for (int s = 0; s < kOS; ++s) r2[s] = f2[s] - 2.0 * k1[s];
        solve_lu(M, perm, r2, k2);
        double err = 0.0, yn[kOS];
#pragma unroll
        for (int s = 0; s < kOS; ++s) {
            yn[s] = y[s] + 1.5 * h * k1[s] + 0.5 * h * k2[s];
            const double e = 0.5 * h * (k1[s] + k2[s]);
            err = fmax(err, fabs(e) / (atol + rtol * fmax(fabs(y[s]), fabs(yn[s]))));
        }
        if (err <= 1.0 && isfinite(err)) {
            t += h;
#pragma unroll
            for (int s = 0; s < kOS; ++s) y[s] = fmax(yn[s], 0.0);
            ode_rhs(y, tb, f);
            ++nstep;
        } else {
            ++nrej;
        }
        const double fac = isfinite(err) ? 0.9 / sqrt(fmax(err, 1e-10)) : 0.2;
        h *= fmin(5.0, fmax(0.2, fac));
    }
    for (int s = 0; s < ns; ++s) c1[(size_t)m * ns + s] = y[s];
    steps[m] = ok ? nstep : -1;
}

}  // namespace

void launch_numodes(hipStream_t st, const double* c0, const double* dt, double* c1, int32_t* steps, int32_t n,
                    const OdeTable& tb, double rtol, double atol, int32_t max_steps) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_numodes, dim3((n + 63) / 64), dim3(64), 0, st, c0, dt, c1, steps, n, tb, rtol, atol,
                       max_steps);
}

}  // namespace gsbs
