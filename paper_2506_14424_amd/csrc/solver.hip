// Vector kernels of the FP64 flexible CG, the Chebyshev-Jacobi preconditioner
// in FP32 or FP64, and the Lanczos eigenvalue estimate (Sec. 5.3).
//
// Reductions are deterministic: each of kRedBlocks blocks reduces a fixed
// grid-stride subset with a fixed tree and writes one partial; the partials
// are then summed in a fixed order, either by a one-block "scalar" kernel or,
// in the CG iteration, by the last block of the same kernel to finish, which
// also updates the solve state (alpha, beta, convergence flags) on the
// device, so iterations are enqueued without host round trips.  Every kernel
// of an iteration returns at once when the state's skip flag is set (the
// solve has finished).
//
// One CG iteration is: A p (FP64 apply), alpha, update + first Chebyshev
// step, degree-1 Chebyshev applies, beta, direction.

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
// The largest eigenvalue of the Lanczos tridiagonal by Sturm counts, with
// the bracket [lo, hi] (count(lo) < m <= count(hi), Gershgorin start)
// narrowed by multisection: the 64 lanes of one wavefront each count at one
// of 64 interior points, the bracket shrinks 65-fold per round, until its
// width is below 1e-15 |hi|; lambda = hi.
constexpr int kEigLanes = 64;

__global__ void __launch_bounds__(kEigLanes) k_lz_eig(SolveState* st) {
    __shared__ double sa[64], sb2[64];
    __shared__ int cnt[kEigLanes];
    __shared__ double br[2];
    const int m = st->lz_m;
    const int l = threadIdx.x;
    if (m <= 0) {
        if (l == 0) st->lam_max = 1.0;
        return;
    }
    if (l < m) {
        sa[l] = st->lz_alpha[l];
        sb2[l] = l > 0 ? st->lz_beta[l] * st->lz_beta[l] : 0.0;
    }
    if (l == 0) {
        double lo = 1e300, hi = -1e300;
        for (int i = 0; i < m; ++i) {
            const double r = (i > 0 ? fabs(st->lz_beta[i]) : 0.0) + (i + 1 < m ? fabs(st->lz_beta[i + 1]) : 0.0);
            lo = fmin(lo, st->lz_alpha[i] - r);
            hi = fmax(hi, st->lz_alpha[i] + r);
        }
        br[0] = lo;
        br[1] = hi + (1e-12 * fabs(hi) + 1e-300);
    }
    __syncthreads();
    for (int round = 0; round < 40; ++round) {
        const double lo = br[0], hi = br[1];
        if (!(hi - lo > 1e-15 * fabs(hi))) break;  // uniform: every lane reads the same bracket
        const double x = lo + (hi - lo) * (double)(l + 1) / (double)(kEigLanes + 1);
        int c = 0;
        double q = 1.0;
        for (int i = 0; i < m; ++i) {
            q = sa[i] - x - (i > 0 ? sb2[i] / q : 0.0);
            if (q == 0.0) q = -1e-300;
            if (q < 0.0) ++c;
        }
        cnt[l] = c;
        __syncthreads();
        if (l == 0) {
            // first point with every eigenvalue below it
            int k = kEigLanes;
            for (int j = 0; j < kEigLanes; ++j)
                if (cnt[j] >= m) { k = j; break; }
            const double w = hi - lo;
            const double nlo = k == 0 ? lo : lo + w * (double)k / (double)(kEigLanes + 1);
            const double nhi = k == kEigLanes ? hi : lo + w * (double)(k + 1) / (double)(kEigLanes + 1);
            br[0] = nlo;
            br[1] = nhi;
        }
        __syncthreads();
    }
    if (l == 0) st->lam_max = br[1];
}

// Chebyshev interval and coefficients from the cached estimate (cheap; once
// per solve and level): lambda_hi = safety * lambda, lambda_lo =
// lambda_hi / ratio, and the coefficients of the three-term recurrence
// (Saad, Alg. 12.1): theta = (hi+lo)/2, delta = (hi-lo)/2, sigma =
// theta/delta, rho_0 = 1/sigma, rho_j = 1/(2 sigma - rho_{j-1}),
// c1_j = rho_j rho_{j-1}, c2_j = 2 rho_j / delta.
__global__ void k_lz_coef(SolveState* st, double safety, double ratio, int degree) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double lam = st->lam_max;
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

// The scalar step that follows a reduction (s0, s1: the first two sums).
__device__ void scalar_step(SolveState* st, int op, double s0, double s1, long long n) {
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

// One-block reduction of the partials in a fixed order, then the scalar step.
__global__ void k_scalar(SolveState* st, const double* partials, int nslots, int nblocks, int op, long long n,
                         int respect_skip) {
    if (respect_skip && st->skip) return;
    __shared__ double sh[2][kRedThreads];
    for (int k = 0; k < 2; ++k) {
        double s = 0.0;
        if (k < nslots)
            for (int i = threadIdx.x; i < nblocks; i += kRedThreads) s += partials[k * kRedBlocks + i];
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
    scalar_step(st, op, sh[0][0], sh[1][0], n);
}

// Fused reduction: every block stores its NS partial sums; the last block to
// arrive (device-scope counter in the state) adds the partials of all blocks
// in the same fixed order as k_scalar, so the totals do not depend on which
// block finishes last.  Returns true in (all threads of) the last block, with
// the totals in tot for thread 0; that block also clears the counter for the
// next fused kernel on the stream.
template <int NS>
__device__ bool reduce_last(double (&v)[NS], double* partials, SolveState* st, double (&tot)[NS]) {
    block_reduce_store<NS>(v, partials);
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        const unsigned prev = __hip_atomic_fetch_add(&st->arrive, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __shared__ double sh[NS][kRedThreads];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        double s = 0.0;
        for (int i = threadIdx.x; i < (int)gridDim.x; i += kRedThreads) s += partials[k * kRedBlocks + i];
        sh[k][threadIdx.x] = s;
    }
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < NS; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) tot[k] = sh[k][0];
    if (threadIdx.x == 0) __hip_atomic_store(&st->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
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

// r = b - mean, x = 0; |r|^2 -> bnorm2 and the start flags (mean from state when mean_zero)
__global__ void k_pcg_start(const double* b, double* r, double* x, long long n, int mean_zero, SolveState* st,
                            double* partials) {
    const double m = mean_zero ? st->mean : 0.0;
    double acc[1] = {0.0}, tot[1];
    GRID_STRIDE(i, n) {
        const double v = b[i] - m;
        r[i] = v;
        x[i] = 0.0;
        acc[0] += v * v;
    }
    if (reduce_last<1>(acc, partials, st, tot) && threadIdx.x == 0) scalar_step(st, SC_PCG_INIT, tot[0], 0.0, n);
}

// r = b - Ax (q holds Ax); |r|^2 -> rr_true  (restart / final defect check)
__global__ void k_residual(const double* b, const double* q, double* r, long long n, int mean_zero, SolveState* st,
                           double* partials) {
    const double m = mean_zero ? st->mean : 0.0;
    double acc[1] = {0.0}, tot[1];
    GRID_STRIDE(i, n) {
        const double v = (b[i] - m) - q[i];
        r[i] = v;
        acc[0] += v * v;
    }
    if (reduce_last<1>(acc, partials, st, tot) && threadIdx.x == 0) scalar_step(st, SC_TRUE, tot[0], 0.0, n);
}

// Lanczos step with the scalar steps fused (same fixed-order sums as the
// separate kernels): w = sqrt(dinv) w with alpha_m = w.v, ...
__global__ void k_lz_post_alpha(double* w, const double* v, const double* dinv, long long n, SolveState* st,
                                double* partials) {
    double acc[1] = {0.0}, tot[1];
    GRID_STRIDE(i, n) {
        const double x = sqrt(dinv[i]) * w[i];
        w[i] = x;
        acc[0] += x * v[i];
    }
    if (reduce_last<1>(acc, partials, st, tot) && threadIdx.x == 0) scalar_step(st, SC_LZ_ALPHA, tot[0], 0.0, n);
}

// ... w -= alpha_m v + beta_m vprev with beta_{m+1} = |w| (m advances), ...
__global__ void k_lz_orth_beta(double* w, const double* v, const double* vprev, long long n, SolveState* st,
                               double* partials) {
    const int m = st->lz_m;
    const double a = st->lz_alpha[m], b = st->lz_beta[m];
    double acc[1] = {0.0}, tot[1];
    GRID_STRIDE(i, n) {
        const double x = w[i] - a * v[i] - b * vprev[i];
        w[i] = x;
        acc[0] += x * x;
    }
    if (reduce_last<1>(acc, partials, st, tot) && threadIdx.x == 0) scalar_step(st, SC_LZ_BETA, tot[0], 0.0, n);
}

// ... and the next vector vnew = w / beta with the next step's input
// t = sqrt(dinv) vnew.
__global__ void k_lz_next_pre(double* vnew, double* t, const double* w, const double* dinv, long long n,
                              const SolveState* st) {
    const double b = st->lz_beta[st->lz_m];
    const double inv = b > 0.0 ? 1.0 / b : 0.0;
    GRID_STRIDE(i, n) {
        const double x = w[i] * inv;
        vnew[i] = x;
        t[i] = sqrt(dinv[i]) * x;
    }
}

// alpha = (r.z) / (p.Ap), breakdown when p.Ap is not positive
__global__ void k_cg_alpha(const double* p, const double* q, long long n, SolveState* st, double* partials) {
    if (skipped(st)) return;
    double acc[1] = {0.0}, tot[1];
    GRID_STRIDE(i, n) acc[0] += p[i] * q[i];
    if (reduce_last<1>(acc, partials, st, tot) && threadIdx.x == 0) scalar_step(st, SC_ALPHA, tot[0], 0.0, n);
}

// x += alpha p, r -= alpha q, convergence test on |r|^2, and the first
// Chebyshev step from the new residual: rT = (T) r, z = theta^-1 dinv rT, d = z.
template <typename T>
__global__ void k_cg_update(double* x, double* r, const double* p, const double* q, T* rT, T* z, T* d,
                            const T* dinv, long long n, SolveState* st, double* partials) {
    if (skipped(st)) return;
    const double a = st->alpha;
    const T ti = T(st->theta_inv);
    double acc[1] = {0.0}, tot[1];
    GRID_STRIDE(i, n) {
        x[i] += a * p[i];
        const double v = r[i] - a * q[i];
        r[i] = v;
        acc[0] += v * v;
        const T rv = T(v);
        rT[i] = rv;
        const T zv = ti * dinv[i] * rv;
        z[i] = zv;
        d[i] = zv;
    }
    if (reduce_last<1>(acc, partials, st, tot) && threadIdx.x == 0) scalar_step(st, SC_RESID, tot[0], 0.0, n);
}

// Chebyshev start from r without a CG update (first iteration, restarts)
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

// End of the preconditioner and the flexible-CG beta:
//   z = (double) zT;  with mean_zero the mean of z is removed (the
//   subtraction itself happens in k_cg_direction; r.(z - m 1) = r.z - m sum r);
//   first: rz = r.z;  else beta = (r.z - r.zold) / rz, rz = r.z.
template <typename T>
__global__ void k_cg_beta(const T* zT, double* z, const double* r, const double* zold, long long n, int mean_zero,
                          int first, SolveState* st, double* partials) {
    if (skipped(st)) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0}, tot[4];
    GRID_STRIDE(i, n) {
        const double v = (double)zT[i];
        const double ri = r[i];
        z[i] = v;
        acc[0] += ri * v;
        if (!first) acc[1] += ri * zold[i];
        acc[2] += v;
        acc[3] += ri;
    }
    if (reduce_last<4>(acc, partials, st, tot) && threadIdx.x == 0) {
        const double m = mean_zero ? tot[2] / (double)n : 0.0;
        const double rzn = mean_zero ? tot[0] - m * tot[3] : tot[0];
        st->mean = m;
        if (!first) st->beta = (rzn - tot[1]) / st->rz;
        st->rz = rzn;
    }
}

// z -= mean (mean_zero), p = z + beta p  (p = z when first)
__global__ void k_cg_direction(double* p, double* z, long long n, int mean_zero, int first, const SolveState* st) {
    if (skipped(st)) return;
    const double b = first ? 0.0 : st->beta;
    const double m = st->mean;
    GRID_STRIDE(i, n) {
        double zz = z[i];
        if (mean_zero) {
            zz -= m;
            z[i] = zz;
        }
        p[i] = first ? zz : zz + b * p[i];
    }
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
    st->arrive = 0;
}
__global__ void k_state_resume(SolveState* st, int max_iter) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->done = 0;
    st->skip = 0;
    st->max_iter = max_iter;
}

// ---------------------------------------------------------------- launchers

// Reduction grids shrink with the vector (at least 4 elements per thread) so
// that small solves do not pay for hundreds of idle blocks per kernel.
static inline int red_blocks(long long n) {
    const long long b = (n + 4 * kRedThreads - 1) / (4 * kRedThreads);
    return (int)(b < 1 ? 1 : b > kRedBlocks ? kRedBlocks : b);
}
static inline dim3 red_grid(long long n) { return dim3(red_blocks(n)); }
static inline dim3 red_block() { return dim3(kRedThreads); }

#define L(kern, ...) hipLaunchKernelGGL(kern, red_grid(n), red_block(), 0, s, __VA_ARGS__)

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
void sk_lz_post_alpha(double* w, const double* v, const double* dinv, long long n, SolveState* st, double* partials,
                      hipStream_t s) {
    L(k_lz_post_alpha, w, v, dinv, n, st, partials);
}
void sk_lz_orth_beta(double* w, const double* v, const double* vprev, long long n, SolveState* st, double* partials,
                     hipStream_t s) {
    L(k_lz_orth_beta, w, v, vprev, n, st, partials);
}
void sk_lz_next_pre(double* vnew, double* t, const double* w, const double* dinv, long long n, const SolveState* st,
                    hipStream_t s) {
    L(k_lz_next_pre, vnew, t, w, dinv, n, st);
}
void sk_lz_eig(SolveState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_eig, dim3(1), dim3(kEigLanes), 0, s, st);
}
void sk_lz_coef(SolveState* st, double safety, double ratio, int degree, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_coef, dim3(1), dim3(1), 0, s, st, safety, ratio, degree);
}
void sk_scalar(SolveState* st, const double* partials, int nslots, int op, long long n, hipStream_t s,
               int respect_skip) {
    hipLaunchKernelGGL(k_scalar, dim3(1), dim3(kRedThreads), 0, s, st, partials, nslots, red_blocks(n), op, n,
                       respect_skip);
}
void sk_sum(const double* x, long long n, double* partials, const SolveState* st, hipStream_t s) {
    L(k_sum, x, n, partials, st);
}
void sk_sub_mean(double* x, long long n, const SolveState* st, const SolveState* skip_st, hipStream_t s) {
    L(k_sub_mean, x, n, st, skip_st);
}
void sk_pcg_start(const double* b, double* r, double* x, long long n, int mean_zero, SolveState* st,
                  double* partials, hipStream_t s) {
    L(k_pcg_start, b, r, x, n, mean_zero, st, partials);
}
void sk_residual(const double* b, const double* q, double* r, long long n, int mean_zero, SolveState* st,
                 double* partials, hipStream_t s) {
    L(k_residual, b, q, r, n, mean_zero, st, partials);
}
void sk_cg_alpha(const double* p, const double* q, long long n, SolveState* st, double* partials, hipStream_t s) {
    L(k_cg_alpha, p, q, n, st, partials);
}
template <typename T>
void sk_cg_update(double* x, double* r, const double* p, const double* q, T* rT, T* z, T* d, const T* dinv,
                  long long n, SolveState* st, double* partials, hipStream_t s) {
    L(k_cg_update<T>, x, r, p, q, rT, z, d, dinv, n, st, partials);
}
template <typename T>
void sk_cheb_start(const double* r, T* rT, T* z, T* d, const T* dinv, long long n, const SolveState* st,
                   hipStream_t s) {
    L(k_cheb_start<T>, r, rT, z, d, dinv, n, st);
}
template <typename T>
void sk_cg_beta(const T* zT, double* z, const double* r, const double* zold, long long n, int mean_zero, int first,
                SolveState* st, double* partials, hipStream_t s) {
    L(k_cg_beta<T>, zT, z, r, zold, n, mean_zero, first, st, partials);
}
void sk_cg_direction(double* p, double* z, long long n, int mean_zero, int first, const SolveState* st,
                     hipStream_t s) {
    L(k_cg_direction, p, z, n, mean_zero, first, st);
}
#define INST(T)                                                                                             \
    template void sk_cg_update<T>(double*, double*, const double*, const double*, T*, T*, T*, const T*,       \
                                  long long, SolveState*, double*, hipStream_t);                            \
    template void sk_cheb_start<T>(const double*, T*, T*, T*, const T*, long long, const SolveState*,         \
                                   hipStream_t);                                                             \
    template void sk_cg_beta<T>(const T*, double*, const double*, const double*, long long, int, int,         \
                                SolveState*, double*, hipStream_t);
INST(double)
INST(float)
#undef INST

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
