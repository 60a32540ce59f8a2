// Host-callable launchers of the solver's vector kernels (solver.hip).
#pragma once

#include "sipg_internal.h"

namespace sipg {

enum ScalarOp {
    SC_LZ_NORM = 0, SC_LZ_ALPHA, SC_LZ_BETA, SC_PCG_INIT, SC_RZ, SC_ALPHA, SC_RESID, SC_BETA, SC_MEAN, SC_TRUE
};

void sk_lz_start(double* v, long long n, unsigned long long seed, double* partials, hipStream_t s);
void sk_lz_normalize(double* v, double* vprev, long long n, const SolveState* st, hipStream_t s);
void sk_lz_pre(double* t, const double* v, const double* dinv, long long n, hipStream_t s);
void sk_lz_post(double* w, const double* v, const double* dinv, long long n, double* partials, hipStream_t s);
void sk_lz_orth(double* w, const double* v, const double* vprev, long long n, const SolveState* st,
                double* partials, hipStream_t s);
void sk_lz_next(double* vnew, const double* w, long long n, const SolveState* st, hipStream_t s);
// fused Lanczos step: post-scaling with alpha, orthogonalisation with beta, next vector with its pre-scaling
void sk_lz_post_alpha(double* w, const double* v, const double* dinv, long long n, SolveState* st, double* partials,
                      hipStream_t s);
void sk_lz_orth_beta(double* w, const double* v, const double* vprev, long long n, SolveState* st, double* partials,
                     hipStream_t s);
void sk_lz_next_pre(double* vnew, double* t, const double* w, const double* dinv, long long n, const SolveState* st,
                    hipStream_t s);
void sk_lz_eig(SolveState* st, hipStream_t s);   // lambda_max of the Lanczos tridiagonal
void sk_lz_coef(SolveState* st, double safety, double ratio, int degree, hipStream_t s);  // Chebyshev coefficients
void sk_scalar(SolveState* st, const double* partials, int nslots, int op, long long n, hipStream_t s,
               int respect_skip = 0);
void sk_sum(const double* x, long long n, double* partials, const SolveState* st, hipStream_t s);
void sk_sub_mean(double* x, long long n, const SolveState* st, const SolveState* skip_st, hipStream_t s);
void sk_pcg_start(const double* b, double* r, double* x, long long n, int mean_zero, SolveState* st,
                  double* partials, hipStream_t s);
void sk_residual(const double* b, const double* q, double* r, long long n, int mean_zero, SolveState* st,
                 double* partials, hipStream_t s);
void sk_cg_alpha(const double* p, const double* q, long long n, SolveState* st, double* partials, hipStream_t s);
template <typename T>
void sk_cg_update(double* x, double* r, const double* p, const double* q, T* rT, T* z, T* d, const T* dinv,
                  long long n, SolveState* st, double* partials, hipStream_t s);
template <typename T>
void sk_cheb_start(const double* r, T* rT, T* z, T* d, const T* dinv, long long n, const SolveState* st,
                   hipStream_t s);
template <typename T>
void sk_cg_beta(const T* zT, double* z, const double* r, const double* zold, long long n, int mean_zero, int first,
                SolveState* st, double* partials, hipStream_t s);
void sk_cg_direction(double* p, double* z, long long n, int mean_zero, int first, const SolveState* st,
                     hipStream_t s);
void sk_copy(double* dst, const double* src, long long n, hipStream_t s);
void sk_cast(float* dst, const double* src, long long n, hipStream_t s);
void sk_fill(double* dst, double v, long long n, hipStream_t s);
void sk_state_init(SolveState* st, double tol2, int max_iter, hipStream_t s);
void sk_state_resume(SolveState* st, int max_iter, hipStream_t s);

}  // namespace sipg
