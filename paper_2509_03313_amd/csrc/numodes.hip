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
// d[X]/dt = sum_r rate_r (products X - reactants X).  The stage matrix is factored in registers with
// partial pivoting done by selects.
#include "engine.h"

namespace gsbs {

namespace {

template <int S>
__device__ __forceinline__ void ode_rhs(const double* y, const OdeTable& tb, double* f) {
#pragma unroll
    for (int s = 0; s < S; ++s) f[s] = 0.0;
    for (int r = 0; r < tb.nr; ++r) {
        const int a = tb.ra[r], b = tb.rb[r];
        double ya = 0.0, yb = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            ya = s == a ? y[s] : ya;
            yb = s == b ? y[s] : yb;
        }
        const double rho = (a == b ? 0.5 : 1.0) * tb.k[r] * ya * yb;
        const double da = -rho, db = tb.keep_b[r] ? 0.0 : -rho;
        const int p0 = tb.nprod[r] > 0 ? tb.prod[r][0] : -1;
        const int p1 = tb.nprod[r] > 1 ? tb.prod[r][1] : -1;
        const int p2 = tb.nprod[r] > 2 ? tb.prod[r][2] : -1;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            double d = (s == a ? da : 0.0) + (s == b ? db : 0.0);
            d += (s == p0 ? rho : 0.0) + (s == p1 ? rho : 0.0) + (s == p2 ? rho : 0.0);
            f[s] += d;
        }
    }
}

// J[i][j] = d f_i / d y_j
template <int S>
__device__ __forceinline__ void ode_jac(const double* y, const OdeTable& tb, double (*J)[S]) {
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j < S; ++j) J[i][j] = 0.0;
    for (int r = 0; r < tb.nr; ++r) {
        const int a = tb.ra[r], b = tb.rb[r];
        double ya = 0.0, yb = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            ya = s == a ? y[s] : ya;
            yb = s == b ? y[s] : yb;
        }
        // d rate / d y_j: k y_a (j = a, a == b); k y_b (j = a), k y_a (j = b)
        double g[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            g[j] = a == b ? (j == a ? tb.k[r] * ya : 0.0)
                          : ((j == a ? tb.k[r] * yb : 0.0) + (j == b ? tb.k[r] * ya : 0.0));
        }
        const int p0 = tb.nprod[r] > 0 ? tb.prod[r][0] : -1;
        const int p1 = tb.nprod[r] > 1 ? tb.prod[r][1] : -1;
        const int p2 = tb.nprod[r] > 2 ? tb.prod[r][2] : -1;
        const bool kb = tb.keep_b[r] != 0;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const double w = (i == a ? -1.0 : 0.0) + (i == b && !kb ? -1.0 : 0.0) + (i == p0 ? 1.0 : 0.0) +
                             (i == p1 ? 1.0 : 0.0) + (i == p2 ? 1.0 : 0.0);
            if (w != 0.0) {
#pragma unroll
                for (int j = 0; j < S; ++j) J[i][j] += w * g[j];
            }
        }
    }
}

// In-place LU of M with partial pivoting; the row exchanges are applied to
// the right-hand sides by solve_lu through perm.
template <int S>
__device__ __forceinline__ void factor(double (*M)[S], int* perm) {
#pragma unroll
    for (int i = 0; i < S; ++i) perm[i] = i;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        // pivot: the largest |M[i][k]|, i >= k; rows exchanged by selects
        int p = k;
        double best = fabs(M[k][k]);
#pragma unroll
        for (int i = k + 1; i < S; ++i) {
            const double v = fabs(M[i][k]);
            if (v > best) {
                best = v;
                p = i;
            }
        }
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
        const double inv = 1.0 / M[k][k];
#pragma unroll
        for (int i = k + 1; i < S; ++i) {
            const double l = M[i][k] * inv;
            M[i][k] = l;
#pragma unroll
            for (int j = k + 1; j < S; ++j) M[i][j] -= l * M[k][j];
        }
    }
}

template <int S>
__device__ __forceinline__ void solve_lu(const double (*M)[S], const int* perm, const double* b, double* x) {
    double z[S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
        double v = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) v = perm[i] == s ? b[s] : v;
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
        z[i] /= M[i][i];
    }
#pragma unroll
    for (int i = 0; i < S; ++i) x[i] = z[i];
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
        ode_jac<S>(y, tb, M);
        const double dg = 1.0 / (gam * h);
#pragma unroll
        for (int i = 0; i < S; ++i)
#pragma unroll
            for (int j = 0; j < S; ++j) M[i][j] = (i == j ? dg : 0.0) - M[i][j];
        int perm[S];
        factor<S>(M, perm);
        double k1[S], d[S], k3[S], k4[S], r[S], ys[S], fs[S];
        solve_lu<S>(M, perm, f, k1);
#pragma unroll
        for (int s = 0; s < S; ++s) r[s] = f[s] + 4.0 * ih * k1[s];
        solve_lu<S>(M, perm, r, d);  // K2
#pragma unroll
        for (int s = 0; s < S; ++s) {
            d[s] = k1[s] - d[s];  // K1 - K2
            ys[s] = y[s] + 2.0 * k1[s];
        }
        ode_rhs<S>(ys, tb, fs);
#pragma unroll
        for (int s = 0; s < S; ++s) r[s] = fs[s] + ih * d[s];
        solve_lu<S>(M, perm, r, k3);
#pragma unroll
        for (int s = 0; s < S; ++s) ys[s] += k3[s];
        ode_rhs<S>(ys, tb, fs);
#pragma unroll
        for (int s = 0; s < S; ++s) r[s] = fs[s] + ih * (d[s] - (8.0 / 3.0) * k3[s]);
        solve_lu<S>(M, perm, r, k4);
        double err = 0.0, yn[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            yn[s] = ys[s] + k4[s];
            err = fmax(err, fabs(k4[s]) / (atol + rtol * fmax(fabs(y[s]), fabs(yn[s]))));
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
