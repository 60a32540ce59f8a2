// Picard update of the viscosity from the velocity (Sec. 4.1, eq.
// viscosity_pointwise: nu = eta(gdot(grad^S u)) at every integration point)
// and the vector kernels of the Aitken-relaxed fixed-point iteration
// (Sec. 5.1, Alg. 1).
//
// The shear rate gdot = sqrt(2 eps:eps) is that of the finest level's DG
// velocity, evaluated at the quadrature points of any multigrid level: a
// point xi of a level cell e lies in the fine cell r e + min(floor(r xi),
// r - 1) at the fine reference point r xi - that, per direction (r = 2^L
// after L mesh steps, 1 for degree steps).  At a face point the symmetric
// gradients of the two adjacent fine cells' traces are averaged (the
// interior trace alone on the boundary), so every face point carries one
// viscosity, as the operator kernel expects.  One thread per point; the
// fine velocity is evaluated with the 1D Lagrange values and derivatives at
// the fine reference point (O(n^3) per point, cache-resident cell values).

#include "device_common.h"

namespace sipg {

namespace {

constexpr int kThreads = 256;

// 1D Lagrange basis on the fine level's Gauss points and its derivative at x.
__device__ __forceinline__ void lagrange_1d(const FineVelocity& F, double x, double* v, double* dv) {
    const int n = F.n;
    for (int j = 0; j < n; ++j) {
        double val = F.inv_den[j], der = 0.0;
        // l_j(x) = inv_den_j prod_{m != j} (x - g_m); l_j' by the product rule
        for (int m = 0; m < n; ++m) {
            if (m == j) continue;
            const double f = x - F.g[m];
            der = der * f + val;
            val *= f;
        }
        v[j] = val;
        dv[j] = der;
    }
}

// Physical velocity gradient G[c][i] = d u_c / d x_i of fine cell (fx, fy, fz)
// at fine reference point xi.
__device__ void velocity_gradient(const FineVelocity& F, int fx, int fy, int fz, const double xi[3],
                                  double G[3][3]) {
    double lv[3][kMaxN], ld[3][kMaxN];
    for (int d = 0; d < 3; ++d) lagrange_1d(F, xi[d], lv[d], ld[d]);
    const int n = F.n, n3 = n * n * n;
    const long long cell = ((long long)fz * F.ny + fy) * F.nx + fx;
    double gref[3][3];
    for (int c = 0; c < 3; ++c) {
        const double* U = F.u + (cell * 3 + c) * n3;
        double g0 = 0.0, g1 = 0.0, g2 = 0.0;
        for (int j3 = 0; j3 < n; ++j3)
            for (int j2 = 0; j2 < n; ++j2) {
                const double* row = U + (j3 * n + j2) * n;
                double sd = 0.0, sv = 0.0;
                for (int j1 = 0; j1 < n; ++j1) {
                    sd += ld[0][j1] * row[j1];
                    sv += lv[0][j1] * row[j1];
                }
                g0 += (lv[1][j2] * lv[2][j3]) * sd;
                g1 += (ld[1][j2] * lv[2][j3]) * sv;
                g2 += (lv[1][j2] * ld[2][j3]) * sv;
            }
        gref[c][0] = g0; gref[c][1] = g1; gref[c][2] = g2;
    }
    double Ji[3][3];
    if (F.verts != nullptr) {
        double geo[8][3], gi[8];
        for (int i = 0; i < 3; ++i) {
            trilinear_coeffs(F.verts, F.nx, F.ny, fx, fy, fz, i, gi);
            for (int k = 0; k < 8; ++k) geo[k][i] = gi[k];
        }
        double det;
        jacobian_inverse<double>(geo, xi[0], xi[1], xi[2], Ji, det);
    } else {
        for (int d = 0; d < 3; ++d)
            for (int i = 0; i < 3; ++i) Ji[d][i] = d == i ? double(d == 0 ? F.nx : d == 1 ? F.ny : F.nz) : 0.0;
    }
    for (int c = 0; c < 3; ++c)
        for (int i = 0; i < 3; ++i) G[c][i] = gref[c][0] * Ji[0][i] + gref[c][1] * Ji[1][i] + gref[c][2] * Ji[2][i];
}

// eps:eps of the symmetric part of G (times `scale` squared)
__device__ __forceinline__ double sym_square(const double G[3][3]) {
    double ee = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double e = 0.5 * (G[i][j] + G[j][i]);
            ee += e * e;
        }
    return ee;
}

__device__ __forceinline__ double eta(const LawDev& L, double gdot) {
    return L.mu_inf + (L.mu0 - L.mu_inf) * pow(L.kappa + pow(L.lam * gdot, L.a_exp), (L.n_exp - 1.0) / L.a_exp);
}

// fine cell index and fine reference coordinate along one direction
__device__ __forceinline__ void locate(int r, int e, double xi, int& f, double& xf) {
    const double t = r * xi;
    int k = (int)floor(t);
    k = k > r - 1 ? r - 1 : k;
    f = r * e + k;
    xf = t - k;
}

__global__ void k_picard_cell(FineVelocity F, LevelPoints Lv, LawDev law, double* mu64, float* mu32) {
    const int n = Lv.n, n3 = n * n * n;
    const long long total = (long long)Lv.nx * Lv.ny * Lv.nz * n3;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int q = (int)(idx % n3);
        const int e = (int)(idx / n3);
        const int ex = e % Lv.nx, ey = (e / Lv.nx) % Lv.ny, ez = e / (Lv.nx * Lv.ny);
        const int q1 = q % n, q2 = (q / n) % n, q3 = q / (n * n);
        int fx, fy, fz;
        double xi[3];
        locate(Lv.r, ex, Lv.g[q1], fx, xi[0]);
        locate(Lv.r, ey, Lv.g[q2], fy, xi[1]);
        locate(Lv.r, ez, Lv.g[q3], fz, xi[2]);
        double G[3][3];
        velocity_gradient(F, fx, fy, fz, xi, G);
        const double m = eta(law, sqrt(2.0 * sym_square(G)));
        mu64[idx] = m;
        mu32[idx] = (float)m;
    }
}

__global__ void k_picard_face(FineVelocity F, LevelPoints Lv, LawDev law, long long nface, double* mu64,
                              float* mu32) {
    const int n = Lv.n, n2 = n * n;
    const long long total = nface * n2;
    const long long nfx = (long long)(Lv.nx + 1) * Lv.ny * Lv.nz, nfy = (long long)Lv.nx * (Lv.ny + 1) * Lv.nz;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int p = (int)(idx % n2);
        long long f = idx / n2;
        int d, pos[3];  // pos[d] = face position 0..N_d, the others the cell indices
        if (f < nfx) {
            d = 0;
            pos[0] = (int)(f % (Lv.nx + 1)); pos[1] = (int)((f / (Lv.nx + 1)) % Lv.ny);
            pos[2] = (int)(f / ((long long)(Lv.nx + 1) * Lv.ny));
        } else if (f < nfx + nfy) {
            f -= nfx;
            d = 1;
            pos[0] = (int)(f % Lv.nx); pos[1] = (int)((f / Lv.nx) % (Lv.ny + 1));
            pos[2] = (int)(f / ((long long)Lv.nx * (Lv.ny + 1)));
        } else {
            f -= nfx + nfy;
            d = 2;
            pos[0] = (int)(f % Lv.nx); pos[1] = (int)((f / Lv.nx) % Lv.ny);
            pos[2] = (int)(f / ((long long)Lv.nx * Lv.ny));
        }
        const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        const int N[3] = {Lv.nx, Lv.ny, Lv.nz};
        double acc[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        int sides = 0;
        for (int side = 1; side >= 0; --side) {  // side 1: the lower cell's face xi_d = 1
            const int ed = side == 1 ? pos[d] - 1 : pos[d];
            if (ed < 0 || ed >= N[d]) continue;
            int fc[3];
            double xi[3];
            locate(Lv.r, pos[t1], Lv.g[p % n], fc[t1], xi[t1]);
            locate(Lv.r, pos[t2], Lv.g[p / n], fc[t2], xi[t2]);
            fc[d] = Lv.r * ed + (side == 1 ? Lv.r - 1 : 0);
            xi[d] = (double)side;
            double G[3][3];
            velocity_gradient(F, fc[0], fc[1], fc[2], xi, G);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) acc[i][j] += G[i][j];
            ++sides;
        }
        const double s = 1.0 / sides;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) acc[i][j] *= s;
        const double m = eta(law, sqrt(2.0 * sym_square(acc)));
        mu64[idx] = m;
        mu32[idx] = (float)m;
    }
}

// Per-block partial sums of |R|^2, Rp.(R - Rp), |R - Rp|^2 (fixed order).
__global__ void k_picard_sums(const double* R, const double* Rp, long long n, double* partials) {
    __shared__ double sh[3][kThreads];
    double a = 0.0, b = 0.0, c = 0.0;
    for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const double r = R[i];
        a += r * r;
        if (Rp != nullptr) {
            const double rp = Rp[i], dr = r - rp;
            b += rp * dr;
            c += dr * dr;
        }
    }
    sh[0][threadIdx.x] = a; sh[1][threadIdx.x] = b; sh[2][threadIdx.x] = c;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) partials[threadIdx.x * gridDim.x + blockIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_picard_finish(const double* partials, int nblocks, double* out) {
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partials[threadIdx.x * nblocks + b];
        out[threadIdx.x] = s;
    }
}

__global__ void k_axpy(double* x, const double* d, double omega, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] += omega * d[i];
}

inline int grid_for(long long work) {
    const long long b = (work + kThreads - 1) / kThreads;
    return (int)(b < 1 ? 1 : b > 65535 ? 65535 : b);
}

}  // namespace

hipError_t launch_picard_viscosity(const FineVelocity& F, const LevelPoints& Lv, const LawDev& law, long long nface,
                                   double* mu_cell64, float* mu_cell32, double* mu_face64, float* mu_face32,
                                   hipStream_t s) {
    const long long nc = (long long)Lv.nx * Lv.ny * Lv.nz * Lv.n * Lv.n * Lv.n;
    hipLaunchKernelGGL(k_picard_cell, dim3(grid_for(nc)), dim3(kThreads), 0, s, F, Lv, law, mu_cell64, mu_cell32);
    const long long nf = nface * Lv.n * Lv.n;
    hipLaunchKernelGGL(k_picard_face, dim3(grid_for(nf)), dim3(kThreads), 0, s, F, Lv, law, nface, mu_face64,
                       mu_face32);
    return hipGetLastError();
}

hipError_t launch_picard_sums(const double* R, const double* Rp, long long n, double* partials, double* out,
                              hipStream_t s) {
    const int nb = kPicardBlocks;
    hipLaunchKernelGGL(k_picard_sums, dim3(nb), dim3(kThreads), 0, s, R, Rp, n, partials);
    hipLaunchKernelGGL(k_picard_finish, dim3(1), dim3(64), 0, s, partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_axpy(double* x, const double* d, double omega, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(kThreads), 0, s, x, d, omega, n);
    return hipGetLastError();
}

}  // namespace sipg
