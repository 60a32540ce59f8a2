// Vector kernels of the FP64 flexible CG, the Chebyshev-Jacobi preconditioner
// in FP32 or FP64, and the Lanczos eigenvalue estimate (Sec. 5.3).
//
// Reductions are deterministic: each of kRedBlocks blocks reduces a fixed
// grid-stride subset with a fixed tree and writes one partial; a one-block
// "scalar" kernel sums the partials in a fixed order and updates the solve
// state (alpha, beta, convergence flags) on the device, so iterations can be
// enqueued without host round trips.  Every kernel of an iteration returns at
// once when the state's skip flag is set (the solve has finished).

#include "device_common.h"
#include "solver_kernels.h"

namespace sipg {

template <int NS>
__device__ __forceinline__ void block_reduce_store(double (&v)[NS], double* partials) {
    __shared__ double sh[NS][kRedThreads];
#pragma unroll
    for (int k = 0; k < NS; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < NS; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NS; ++k) partials[k * kRedBlocks + blockIdx.x] = sh[k][0];
}

#define GRID_STRIDE(i, n) for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < (n); \
                               i += (long long)gridDim.x * blockDim.x)

// SplitMix64 (Steele, Lea and Flood 2014): counter-based U(-1, 1)
__device__ inline double splitmix_uniform(unsigned long long seed, unsigned long long i) {
    unsigned long long z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}

__global__ void k_lz_start(double* v, long long n, unsigned long long seed, double* partials) {
    double acc[1] = {0.0};
    GRID_STRIDE(i, n) {
        const double u = splitmix_uniform(seed, (unsigned long long)i);
        v[i] = u;
        acc[0] += u * u;
    }
    block_reduce_store<1>(acc, partials);
}

// v *= scale (Lanczos normalisation) and vprev = 0
__global__ void k_lz_normalize(double* v, double* vprev, long long n, const SolveState* st) {
    const double sc = st->scale;
    GRID_STRIDE(i, n) {
        v[i] *= sc;
        vprev[i] = 0.0;
    }
}

// t = sqrt(dinv) * v
__global__ void k_lz_pre(double* t, const double* v, const double* dinv, long long n) {
    GRID_STRIDE(i, n) t[i] = sqrt(dinv[i]) * v[i];
}

// w = sqrt(dinv) * w; partial w.v
__global__ void k_lz_post(double* w, const double* v, const double* dinv, long long n, double* partials) {
    double acc[1] = {0.0};
    GRID_STRIDE(i, n) {
        const double x = sqrt(dinv[i]) * w[i];
        w[i] = x;
        acc[0] += x * v[i];
    }
    block_reduce_store<1>(acc, partials);
}

// w -= alpha_m v + beta_m vprev; partial w.w
__global__ void k_lz_orth(double* w, const double* v, const double* vprev, long long n, const SolveState* st,
                          double* partials) {
    const int m = st->lz_m;
    const double a = st->lz_alpha[m], b = st->lz_beta[m];
    double acc[1] = {0.0};
    GRID_STRIDE(i, n) {
        const double x = w[i] - a * v[i] - b * vprev[i];
        w[i] = x;
        acc[0] += x * x;
    }
    block_reduce_store<1>(acc, partials);
}

// vnew = w / beta_{m}  (after the scalar step advanced m)
__global__ void k_lz_next(double* vnew, const double* w, long long n, const SolveState* st) {
    const double b = st->lz_beta[st->lz_m];
    const double inv = b > 0.0 ? 1.0 / b : 0.0;
    GRID_STRIDE(i, n) vnew[i] = w[i] * inv;
}

// Largest eigenvalue of the Lanczos tridiagonal (Sturm-sequence bisection),
// then the Chebyshev interval [lam_hi/ratio, lam_hi], lam_hi = safety * lam,
// and the coefficients of the three-term recurrence (Saad, Alg. 12.1):
// theta = (hi+lo)/2, delta = (hi-lo)/2, sigma = theta/delta, rho_0 = 1/sigma,
// rho_j = 1/(2 sigma - rho_{j-1}), c1_j = rho_j rho_{j-1}, c2_j = 2 rho_j / delta.
__global__ void k_lz_finish(SolveState* st, double safety, double ratio, int degree) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int m = st->lz_m;
    double lam;
    if (m <= 0) {
        lam = 1.0;
    } else {
        double lo = 1e300, hi = -1e300;
        for (int i = 0; i < m; ++i) {
            const double r = (i > 0 ? fabs(st->lz_beta[i]) : 0.0) + (i + 1 < m ? fabs(st->lz_beta[i + 1]) : 0.0);
            lo = fmin(lo, st->lz_alpha[i] - r);
            hi = fmax(hi, st->lz_alpha[i] + r);
        }
        // count(x) = number of eigenvalues < x
        auto count = [&](double x) {
            int cnt = 0;
            double q = 1.0;
            for (int i = 0; i < m; ++i) {
                const double b2 = i > 0 ? st->lz_beta[i] * st->lz_beta[i] : 0.0;
                q = st->lz_alpha[i] - x - (i > 0 ? b2 / q : 0.0);
                if (q == 0.0) q = -1e-300;
                if (q < 0.0) ++cnt;
            }
            return cnt;
        };
        hi += 1e-12 * fabs(hi) + 1e-300;
        for (int it = 0; it < 200 && hi - lo > 1e-15 * fabs(hi); ++it) {
            const double mid = 0.5 * (lo + hi);
            if (count(mid) >= m) hi = mid;  // all eigenvalues below mid
            else lo = mid;
        }
        lam = hi;
    }
    st->lam_max = lam;
    const double lhi = safety * lam, llo = lhi / ratio;
    const double theta = 0.5 * (lhi + llo), delta = 0.5 * (lhi - llo);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    st->theta_inv = 1.0 / theta;
    for (int j = 1; j < degree && j < 64; ++j) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        st->cheb[j][0] = rn * rho;
        st->cheb[j][1] = 2.0 * rn / delta;
        rho = rn;
    }
}

// One-block reduction of the partials in a fixed order, then the scalar step.
__global__ void k_scalar(SolveState* st, const double* partials, int nslots, int op, long long n,
                         int respect_skip) {
    if (respect_skip && st->skip) return;
    __shared__ double sh[2][kRedThreads];
    for (int k = 0; k < 2; ++k) {
        double s = 0.0;
        if (k < nslots)
            for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) s += partials[k * kRedBlocks + i];
        sh[k][threadIdx.x] = s;
    }
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double s0 = sh[0][0], s1 = sh[1][0];
    switch (op) {
        case SC_LZ_NORM:
            st->scale = s0 > 0.0 ? 1.0 / sqrt(s0) : 0.0;
            st->lz_m = 0;
            st->lz_beta[0] = 0.0;
            break;
        case SC_LZ_ALPHA:
            st->lz_alpha[st->lz_m] = s0;
            break;
        case SC_LZ_BETA:
            st->lz_m += 1;
            st->lz_beta[st->lz_m] = sqrt(s0);
            break;
        case SC_PCG_INIT:
            st->bnorm2 = s0;
            st->iter = 0;
            st->done = !isfinite(s0) ? 2 : (s0 > 0.0 ? 0 : 1);   // NaN/Inf in b: breakdown
            st->skip = st->done != 0;
            st->rr = s0;
            break;
        case SC_RZ:
            st->rz = s0;
            break;
        case SC_ALPHA:
            if (!(s0 > 0.0) || !isfinite(s0)) {
                st->done = 2;
                st->skip = 1;
            } else {
                st->alpha = st->rz / s0;
            }
            break;
        case SC_RESID:
            st->rr = s0;
            st->iter += 1;
            if (!isfinite(s0)) st->done = 2;
            else if (s0 <= st->tol2 * st->bnorm2) st->done = 1;
            else if (st->iter >= st->max_iter) st->done = 3;
            st->skip = st->done != 0;
            break;
        case SC_BETA:
            st->beta = (s0 - s1) / st->rz;
            st->rz = s0;
            break;
        case SC_MEAN:
            st->mean = s0 / (double)n;
            break;
        case SC_TRUE:
            st->rr_true = s0;
            break;
    }
}

__device__ __forceinline__ bool skipped(const SolveState* st) { return st != nullptr && st->skip; }

// partial sums of x (slot 0)
__global__ void k_sum(const double* x, long long n, double* partials, const SolveState* st) {
    if (skipped(st)) return;
    double acc[1] = {0.0};
    GRID_STRIDE(i, n) acc[0] += x[i];
    block_reduce_store<1>(acc, partials);
}

// x -= mean (from state)
__global__ void k_sub_mean(double* x, long long n, const SolveState* st, const SolveState* skip_st) {
    if (skipped(skip_st)) return;
    const double m = st->mean;
    GRID_STRIDE(i, n) x[i] -= m;
}

// partials a.b (slot 0) and a.c (slot 1, if c)
__global__ void k_dot2(const double* a, const double* b, const double* c, long long n, double* partials,
                       const SolveState* st) {
    if (skipped(st)) return;
    double acc[2] = {0.0, 0.0};
    GRID_STRIDE(i, n) {
        acc[0] += a[i] * b[i];
        if (c) acc[1] += a[i] * c[i];
    }
    block_reduce_store<2>(acc, partials);
}

// r = b - mean, x = 0, partial r.r   (mean from state when mean_zero)
__global__ void k_pcg_start(const double* b, double* r, double* x, long long n, int mean_zero,
                            const SolveState* st, double* partials) {
    const double m = mean_zero ? st->mean : 0.0;
    double acc[1] = {0.0};
    GRID_STRIDE(i, n) {
        const double v = b[i] - m;
        r[i] = v;
        x[i] = 0.0;
        acc[0] += v * v;
    }
    block_reduce_store<1>(acc, partials);
}

// r = b - Ax (q holds Ax); partial r.r  (restart / true residual)
__global__ void k_residual(const double* b, const double* q, double* r, long long n, int mean_zero,
                           const SolveState* st, double* partials) {
    const double m = mean_zero ? st->mean : 0.0;
    double acc[1] = {0.0};
    GRID_STRIDE(i, n) {
        const double v = (b[i] - m) - q[i];
        r[i] = v;
        acc[0] += v * v;
    }
    block_reduce_store<1>(acc, partials);
}

// x += alpha p, r -= alpha q; partial r.r
__global__ void k_pcg_update(double* x, double* r, const double* p, const double* q, long long n,
                             const SolveState* st, double* partials) {
    if (skipped(st)) return;
    const double a = st->alpha;
    double acc[1] = {0.0};
    GRID_STRIDE(i, n) {
        x[i] += a * p[i];
        const double v = r[i] - a * q[i];
        r[i] = v;
        acc[0] += v * v;
    }
    block_reduce_store<1>(acc, partials);
}

// p = z + beta p (beta from state, or 0 when first)
__global__ void k_pcg_direction(double* p, const double* z, long long n, int first, const SolveState* st) {
    if (skipped(st)) return;
    const double b = first ? 0.0 : st->beta;
    GRID_STRIDE(i, n) p[i] = first ? z[i] : z[i] + b * p[i];
}

// Chebyshev start: rT = (T) r, z = theta^-1 dinv rT, d = z
template <typename T>
__global__ void k_cheb_start(const double* r, T* rT, T* z, T* d, const T* dinv, long long n, const SolveState* st) {
    if (skipped(st)) return;
    const T ti = T(st->theta_inv);
    GRID_STRIDE(i, n) {
        const T rv = T(r[i]);
        rT[i] = rv;
        const T zv = ti * dinv[i] * rv;
        z[i] = zv;
        d[i] = zv;
    }
}

// Chebyshev end: z64 = (double) zT; partial sum(z64) when mean_zero
template <typename T>
__global__ void k_cheb_end(const T* zT, double* z, long long n, const SolveState* st, double* partials,
                           int want_sum) {
    if (skipped(st)) return;
    double acc[1] = {0.0};
    GRID_STRIDE(i, n) {
        const double v = (double)zT[i];
        z[i] = v;
        acc[0] += v;
    }
    if (want_sum) block_reduce_store<1>(acc, partials);
}

__global__ void k_copy(double* dst, const double* src, long long n) { GRID_STRIDE(i, n) dst[i] = src[i]; }
__global__ void k_cast(float* dst, const double* src, long long n) { GRID_STRIDE(i, n) dst[i] = (float)src[i]; }
__global__ void k_fill(double* dst, double v, long long n) { GRID_STRIDE(i, n) dst[i] = v; }

// set scalar fields of the state from the host without a memcpy
__global__ void k_state_init(SolveState* st, double tol2, int max_iter) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->tol2 = tol2;
    st->max_iter = max_iter;
    st->done = 0;
    st->skip = 0;
    st->iter = 0;
}
__global__ void k_state_resume(SolveState* st, int max_iter) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->done = 0;
    st->skip = 0;
    st->max_iter = max_iter;
}

// ---------------------------------------------------------------- launchers

static inline dim3 red_grid() { return dim3(kRedBlocks); }
static inline dim3 red_block() { return dim3(kRedThreads); }

#define L(kern, ...) hipLaunchKernelGGL(kern, red_grid(), red_block(), 0, s, __VA_ARGS__)

void sk_lz_start(double* v, long long n, unsigned long long seed, double* partials, hipStream_t s) {
    L(k_lz_start, v, n, seed, partials);
}
void sk_lz_normalize(double* v, double* vprev, long long n, const SolveState* st, hipStream_t s) {
    L(k_lz_normalize, v, vprev, n, st);
}
void sk_lz_pre(double* t, const double* v, const double* dinv, long long n, hipStream_t s) { L(k_lz_pre, t, v, dinv, n); }
void sk_lz_post(double* w, const double* v, const double* dinv, long long n, double* partials, hipStream_t s) {
    L(k_lz_post, w, v, dinv, n, partials);
}
void sk_lz_orth(double* w, const double* v, const double* vprev, long long n, const SolveState* st,
                double* partials, hipStream_t s) {
    L(k_lz_orth, w, v, vprev, n, st, partials);
}
void sk_lz_next(double* vnew, const double* w, long long n, const SolveState* st, hipStream_t s) {
    L(k_lz_next, vnew, w, n, st);
}
void sk_lz_finish(SolveState* st, double safety, double ratio, int degree, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_finish, dim3(1), dim3(1), 0, s, st, safety, ratio, degree);
}
void sk_scalar(SolveState* st, const double* partials, int nslots, int op, long long n, hipStream_t s,
               int respect_skip) {
    hipLaunchKernelGGL(k_scalar, dim3(1), dim3(kRedThreads), 0, s, st, partials, nslots, op, n, respect_skip);
}
void sk_sum(const double* x, long long n, double* partials, const SolveState* st, hipStream_t s) {
    L(k_sum, x, n, partials, st);
}
void sk_sub_mean(double* x, long long n, const SolveState* st, const SolveState* skip_st, hipStream_t s) {
    L(k_sub_mean, x, n, st, skip_st);
}
void sk_dot2(const double* a, const double* b, const double* c, long long n, double* partials, const SolveState* st,
             hipStream_t s) {
    L(k_dot2, a, b, c, n, partials, st);
}
void sk_pcg_start(const double* b, double* r, double* x, long long n, int mean_zero, const SolveState* st,
                  double* partials, hipStream_t s) {
    L(k_pcg_start, b, r, x, n, mean_zero, st, partials);
}
void sk_residual(const double* b, const double* q, double* r, long long n, int mean_zero, const SolveState* st,
                 double* partials, hipStream_t s) {
    L(k_residual, b, q, r, n, mean_zero, st, partials);
}
void sk_pcg_update(double* x, double* r, const double* p, const double* q, long long n, const SolveState* st,
                   double* partials, hipStream_t s) {
    L(k_pcg_update, x, r, p, q, n, st, partials);
}
void sk_pcg_direction(double* p, const double* z, long long n, int first, const SolveState* st, hipStream_t s) {
    L(k_pcg_direction, p, z, n, first, st);
}
template <typename T>
void sk_cheb_start(const double* r, T* rT, T* z, T* d, const T* dinv, long long n, const SolveState* st,
                   hipStream_t s) {
    L(k_cheb_start<T>, r, rT, z, d, dinv, n, st);
}
template <typename T>
void sk_cheb_end(const T* zT, double* z, long long n, const SolveState* st, double* partials, int want_sum,
                 hipStream_t s) {
    L(k_cheb_end<T>, zT, z, n, st, partials, want_sum);
}
template void sk_cheb_start<double>(const double*, double*, double*, double*, const double*, long long,
                                    const SolveState*, hipStream_t);
template void sk_cheb_start<float>(const double*, float*, float*, float*, const float*, long long, const SolveState*,
                                   hipStream_t);
template void sk_cheb_end<double>(const double*, double*, long long, const SolveState*, double*, int, hipStream_t);
template void sk_cheb_end<float>(const float*, double*, long long, const SolveState*, double*, int, hipStream_t);

void sk_copy(double* dst, const double* src, long long n, hipStream_t s) { L(k_copy, dst, src, n); }
void sk_cast(float* dst, const double* src, long long n, hipStream_t s) { L(k_cast, dst, src, n); }
void sk_fill(double* dst, double v, long long n, hipStream_t s) { L(k_fill, dst, v, n); }
void sk_state_init(SolveState* st, double tol2, int max_iter, hipStream_t s) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, st, tol2, max_iter);
}
void sk_state_resume(SolveState* st, int max_iter, hipStream_t s) {
    hipLaunchKernelGGL(k_state_resume, dim3(1), dim3(1), 0, s, st, max_iter);
}

}  // namespace sipg
