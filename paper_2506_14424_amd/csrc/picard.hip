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
// the fine reference point (O(n^3) per point).  On the levels that share
// the fine mesh (r = 1) a block handles one cell or one face and stages the
// cells' values in LDS once; coarser levels read them through the caches.

#include "device_common.h"

namespace sipg {

namespace {

constexpr int kThreads = 256;

// 1D Lagrange basis on the fine level's NF Gauss points and its derivative at x.
template <int NF>
__device__ __forceinline__ void lagrange_1d(const FineVelocity& F, double x, double* v, double* dv) {
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        double val = F.inv_den[j], der = 0.0;
        // l_j(x) = inv_den_j prod_{m != j} (x - g_m); l_j' by the product rule
#pragma unroll
        for (int m = 0; m < NF; ++m) {
            if (m == j) continue;
            const double f = x - F.g[m];
            der = der * f + val;
            val *= f;
        }
        v[j] = val;
        dv[j] = der;
    }
}

// l_j(x) and l_j'(x) for one (runtime) j on the NF fine Gauss points.
template <int NF>
__device__ __forceinline__ void lagrange_one(const FineVelocity& F, double x, int j, double& v, double& dv) {
    double val = F.inv_den[j], der = 0.0;
#pragma unroll
    for (int m = 0; m < NF; ++m) {
        const double f = m == j ? 1.0 : x - F.g[m];
        der = m == j ? der : der * f + val;
        val *= f;
    }
    v = val;
    dv = der;
}

// G = gref J^-1 for fine cell (fx, fy, fz) at fine reference point xi
// (gref[c][d] = d u_c / d xi_d).
__device__ __forceinline__ void physical_gradient(const FineVelocity& F, int fx, int fy, int fz, const double xi[3],
                                  const double gref[3][3], double G[3][3]) {
    double Ji[3][3];
    if (F.verts != nullptr) {
        double geo[8][3], gi[8];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            trilinear_coeffs(F.verts, F.nx, F.ny, fx, fy, fz, i, gi);
#pragma unroll
            for (int k = 0; k < 8; ++k) geo[k][i] = gi[k];
        }
        double det;
        jacobian_inverse<double>(geo, xi[0], xi[1], xi[2], Ji, det);
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int i = 0; i < 3; ++i) Ji[d][i] = d == i ? double(d == 0 ? F.nx : d == 1 ? F.ny : F.nz) : 0.0;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < 3; ++i) G[c][i] = gref[c][0] * Ji[0][i] + gref[c][1] * Ji[1][i] + gref[c][2] * Ji[2][i];
}

// Physical velocity gradient G[c][i] = d u_c / d x_i of fine cell (fx, fy, fz)
// at fine reference point xi; U: that cell's 3 NF^3 values (global memory or
// a copy in LDS).  The xi_1 and xi_2 contractions are unrolled with their
// 1D tables in registers; the xi_3 loop computes its factor in place.
template <int NF>
__device__ void velocity_gradient(const FineVelocity& F, const double* U, int fx, int fy, int fz, const double xi[3],
                                  double G[3][3]) {
    double lv[2][NF], ld[2][NF];
    lagrange_1d<NF>(F, xi[0], lv[0], ld[0]);
    lagrange_1d<NF>(F, xi[1], lv[1], ld[1]);
    constexpr int n3 = NF * NF * NF;
    double gref[3][3];
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        double g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll 1
        for (int j3 = 0; j3 < NF; ++j3) {
            double v3, d3;
            lagrange_one<NF>(F, xi[2], j3, v3, d3);
            const double* slab = U + c * n3 + j3 * NF * NF;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0;  // sums over (j1, j2) of the slab
#pragma unroll
            for (int j2 = 0; j2 < NF; ++j2) {
                double sd = 0.0, sv = 0.0;
#pragma unroll
                for (int j1 = 0; j1 < NF; ++j1) {
                    const double u = slab[j2 * NF + j1];
                    sd += ld[0][j1] * u;
                    sv += lv[0][j1] * u;
                }
                a0 += lv[1][j2] * sd;
                a1 += ld[1][j2] * sv;
                a2 += lv[1][j2] * sv;
            }
            g0 += v3 * a0;
            g1 += v3 * a1;
            g2 += d3 * a2;
        }
        gref[c][0] = g0; gref[c][1] = g1; gref[c][2] = g2;
    }
    physical_gradient(F, fx, fy, fz, xi, gref, G);
}

// eps:eps of the symmetric part of G
__device__ __forceinline__ double sym_square(const double G[3][3]) {
    double ee = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
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

// Face f of a level: its normal direction (returned) and position, pos[d] =
// 0..N_d along the normal, the other two the cell indices.
__device__ __forceinline__ int decode_face(const LevelPoints& Lv, long long f, int pos[3]) {
    const long long nfx = (long long)(Lv.nx + 1) * Lv.ny * Lv.nz, nfy = (long long)Lv.nx * (Lv.ny + 1) * Lv.nz;
    if (f < nfx) {
        pos[0] = (int)(f % (Lv.nx + 1)); pos[1] = (int)((f / (Lv.nx + 1)) % Lv.ny);
        pos[2] = (int)(f / ((long long)(Lv.nx + 1) * Lv.ny));
        return 0;
    }
    if (f < nfx + nfy) {
        f -= nfx;
        pos[0] = (int)(f % Lv.nx); pos[1] = (int)((f / Lv.nx) % (Lv.ny + 1));
        pos[2] = (int)(f / ((long long)Lv.nx * (Lv.ny + 1)));
        return 1;
    }
    f -= nfx + nfy;
    pos[0] = (int)(f % Lv.nx); pos[1] = (int)((f / Lv.nx) % Lv.ny);
    pos[2] = (int)(f / ((long long)Lv.nx * Lv.ny));
    return 2;
}

__device__ __forceinline__ void store_mu(double* mu64, float* mu32, long long idx, const LawDev& law, double ee) {
    const double m = eta(law, sqrt(2.0 * ee));
    mu64[idx] = m;
    mu32[idx] = (float)m;
}

// Any level (fine cells found by locate): one thread per point, the fine
// cell's values read through the caches.
template <int NF>
__global__ void __launch_bounds__(kThreads) k_picard_cell(FineVelocity F, LevelPoints Lv, LawDev law, double* mu64, float* mu32) {
    const int n = Lv.n, n3 = n * n * n;
    const long long total = (long long)Lv.nx * Lv.ny * Lv.nz * n3;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int q = (int)(idx % n3);
        const int e = (int)(idx / n3);
        const int ex = e % Lv.nx, ey = (e / Lv.nx) % Lv.ny, ez = e / (Lv.nx * Lv.ny);
        int fx, fy, fz;
        double xi[3];
        locate(Lv.r, ex, Lv.g[q % n], fx, xi[0]);
        locate(Lv.r, ey, Lv.g[(q / n) % n], fy, xi[1]);
        locate(Lv.r, ez, Lv.g[q / (n * n)], fz, xi[2]);
        double G[3][3];
        const long long fc = ((long long)fz * F.ny + fy) * F.nx + fx;
        velocity_gradient<NF>(F, F.u + fc * 3 * NF * NF * NF, fx, fy, fz, xi, G);
        store_mu(mu64, mu32, idx, law, sym_square(G));
    }
}

template <int NF>
__global__ void __launch_bounds__(kThreads) k_picard_face(FineVelocity F, LevelPoints Lv, LawDev law, long long nface, double* mu64,
                              float* mu32) {
    const int n = Lv.n, n2 = n * n;
    const long long total = nface * n2;
    const int N[3] = {Lv.nx, Lv.ny, Lv.nz};
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int p = (int)(idx % n2);
        int pos[3];
        const int d = decode_face(Lv, idx / n2, pos);
        const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
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
            const long long cid = ((long long)fc[2] * F.ny + fc[1]) * F.nx + fc[0];
            velocity_gradient<NF>(F, F.u + cid * 3 * NF * NF * NF, fc[0], fc[1], fc[2], xi, G);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) acc[i][j] += G[i][j];
            ++sides;
        }
        const double sc = 1.0 / sides;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) acc[i][j] *= sc;
        store_mu(mu64, mu32, idx, law, sym_square(acc));
    }
}

// Levels on the fine mesh (r = 1: the finest level and the degree steps):
// a block of kSame threads takes `per` consecutive cells (or faces), stages
// their fine values in LDS once and gives each level point one thread.
constexpr int kSame = 256;

template <int NF>
__global__ void __launch_bounds__(kSame) k_picard_cell_same(FineVelocity F, LevelPoints Lv, LawDev law, int per,
                                                            double* mu64, float* mu32) {
    extern __shared__ double su[];  // [per][3 NF^3]
    constexpr int nv = 3 * NF * NF * NF;
    const int n = Lv.n, n3 = n * n * n;
    const long long ncell = (long long)Lv.nx * Lv.ny * Lv.nz;
    const int g = threadIdx.x / n3, q = threadIdx.x % n3;
    for (long long c0 = (long long)blockIdx.x * per; c0 < ncell; c0 += (long long)gridDim.x * per) {
        __syncthreads();
        const long long lim = (ncell - c0 < per ? ncell - c0 : per) * nv;
        for (int i = threadIdx.x; i < lim; i += kSame) su[i] = F.u[c0 * nv + i];
        __syncthreads();
        const long long e = c0 + g;
        if (g < per && e < ncell) {
            const int ex = (int)(e % Lv.nx), ey = (int)((e / Lv.nx) % Lv.ny), ez = (int)(e / ((long long)Lv.nx * Lv.ny));
            const double xi[3] = {Lv.g[q % n], Lv.g[(q / n) % n], Lv.g[q / (n * n)]};
            double G[3][3];
            velocity_gradient<NF>(F, su + g * nv, ex, ey, ez, xi, G);
            store_mu(mu64, mu32, e * n3 + q, law, sym_square(G));
        }
    }
}

// Faces of a level on the fine mesh: a face point lies on the fine face, so
// each side's gradient there factors into the trace and the normal
// derivative on the face's NF x NF grid of fine tangential nodes (one
// contraction along the normal per grid node, done once per face and side
// into LDS) and a 2D interpolation of those to the point (values and
// tangential derivatives of the fine 1D basis): O(NF^2) per point instead
// of O(NF^3).
template <int NF>
__global__ void __launch_bounds__(kSame) k_picard_face_same(FineVelocity F, LevelPoints Lv, LawDev law,
                                                            long long nface, int per, double* mu64, float* mu32) {
    constexpr int nv = 3 * NF * NF * NF, NF2 = NF * NF, tw = 2 * 3 * NF2;  // per face side: trace, d/dxi_d
    extern __shared__ double st[];  // [per][2 sides][tw]
    __shared__ int meta[kSame][6];  // per face: d, pos[3], have lower, have upper
    const int n = Lv.n, n2 = n * n;
    const int g = threadIdx.x / n2, p = threadIdx.x % n2;
    // the fine 1D basis and its derivative at the lower cell's face (xi_d = 1, side 0) and the upper's (0)
    double fv[2][NF], fd[2][NF];
    lagrange_1d<NF>(F, 1.0, fv[0], fd[0]);
    lagrange_1d<NF>(F, 0.0, fv[1], fd[1]);
    for (long long f0 = (long long)blockIdx.x * per; f0 < nface; f0 += (long long)gridDim.x * per) {
        __syncthreads();
        if ((int)threadIdx.x < per && f0 + threadIdx.x < nface) {
            int pos[3];
            const int d = decode_face(Lv, f0 + threadIdx.x, pos);
            meta[threadIdx.x][0] = d;
            meta[threadIdx.x][1] = pos[0]; meta[threadIdx.x][2] = pos[1]; meta[threadIdx.x][3] = pos[2];
            const int pd = d == 0 ? pos[0] : d == 1 ? pos[1] : pos[2];
            meta[threadIdx.x][4] = pd > 0;
            meta[threadIdx.x][5] = pd < (d == 0 ? Lv.nx : d == 1 ? Lv.ny : Lv.nz);
        }
        __syncthreads();
        const int nf = (int)(nface - f0 < per ? nface - f0 : per);
        for (int i = threadIdx.x; i < nf * 2 * 3 * NF2; i += kSame) {
            const int gg = i / (2 * 3 * NF2), rem = i % (2 * 3 * NF2), s = rem / (3 * NF2), c = (rem / NF2) % 3,
                      jab = rem % NF2;
            if (!meta[gg][4 + s]) continue;
            const int d = meta[gg][0];
            const int lo = s == 0 ? 1 : 0;  // the lower cell lies one step down along d
            const int cx = meta[gg][1] - (d == 0 ? lo : 0), cy = meta[gg][2] - (d == 1 ? lo : 0),
                      cz = meta[gg][3] - (d == 2 ? lo : 0);
            const long long cell = ((long long)cz * Lv.ny + cy) * Lv.nx + cx;
            const double* U = F.u + cell * nv + c * NF * NF2;
            // node strides along the normal and the two tangential directions (t1 < t2)
            const int sd = d == 0 ? 1 : d == 1 ? NF : NF2, s1 = d == 0 ? NF : 1, s2 = d == 2 ? NF : NF2;
            const int base = (jab % NF) * s1 + (jab / NF) * s2;
            double tv = 0.0, nd = 0.0;
#pragma unroll
            for (int jd = 0; jd < NF; ++jd) {
                const double u = U[base + jd * sd];
                tv += (s == 0 ? fv[0][jd] : fv[1][jd]) * u;
                nd += (s == 0 ? fd[0][jd] : fd[1][jd]) * u;
            }
            double* T = st + (gg * 2 + s) * tw;
            T[c * NF2 + jab] = tv;
            T[3 * NF2 + c * NF2 + jab] = nd;
        }
        __syncthreads();
        if (g < nf) {
            const int d = meta[g][0];
            double la[NF], da[NF], lb[NF], db[NF];  // fine basis at the point's tangential coordinates
            lagrange_1d<NF>(F, Lv.g[p % n], la, da);
            lagrange_1d<NF>(F, Lv.g[p / n], lb, db);
            double acc[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            int sides = 0;
            for (int s = 0; s < 2; ++s) {  // s = 0: the lower cell (its face xi_d = 1)
                if (!meta[g][4 + s]) continue;
                const int lo = s == 0 ? 1 : 0;
                const int cx = meta[g][1] - (d == 0 ? lo : 0), cy = meta[g][2] - (d == 1 ? lo : 0),
                          cz = meta[g][3] - (d == 2 ? lo : 0);
                // (t1, t2) = the tangential directions in increasing order
                const double xa = Lv.g[p % n], xb = Lv.g[p / n], xn = s == 0 ? 1.0 : 0.0;
                const double xi[3] = {d == 0 ? xn : xa, d == 0 ? xa : (d == 1 ? xn : xb), d == 2 ? xn : xb};
                const double* T = st + (g * 2 + s) * tw;
                double gref[3][3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double g1 = 0.0, g2 = 0.0, g3 = 0.0;
#pragma unroll 1
                    for (int jb = 0; jb < NF; ++jb) {
                        double sd = 0.0, sv = 0.0, sn = 0.0;
#pragma unroll
                        for (int ja = 0; ja < NF; ++ja) {
                            const double tv = T[c * NF2 + jb * NF + ja], nd = T[3 * NF2 + c * NF2 + jb * NF + ja];
                            sd += da[ja] * tv;
                            sv += la[ja] * tv;
                            sn += la[ja] * nd;
                        }
                        g1 += lb[jb] * sd;
                        g2 += db[jb] * sv;
                        g3 += lb[jb] * sn;
                    }
                    gref[c][0] = d == 0 ? g3 : g1;
                    gref[c][1] = d == 0 ? g1 : (d == 1 ? g3 : g2);
                    gref[c][2] = d == 2 ? g3 : g2;
                }
                double G[3][3];
                physical_gradient(F, cx, cy, cz, xi, gref, G);
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int jj = 0; jj < 3; ++jj) acc[i][jj] += G[i][jj];
                ++sides;
            }
            const double sc = 1.0 / sides;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) acc[i][jj] *= sc;
            store_mu(mu64, mu32, (f0 + g) * n2 + p, law, sym_square(acc));
        }
    }
}

constexpr int kLdsCap = 56 * 1024;  // dynamic LDS per block of the same-mesh kernels (plus 6 KB of face data)

template <int NF>
hipError_t launch_nf(const FineVelocity& F, const LevelPoints& Lv, const LawDev& law, long long nface,
                     double* mu_cell64, float* mu_cell32, double* mu_face64, float* mu_face32, hipStream_t s) {
    constexpr int nvb = 3 * NF * NF * NF * (int)sizeof(double);
    const int n = Lv.n;
    if (Lv.r == 1) {
        const long long ncell = (long long)Lv.nx * Lv.ny * Lv.nz;
        constexpr int ftb = 2 * 2 * 3 * NF * NF * (int)sizeof(double);  // per face: both sides' traces
        int pc = kSame / (n * n * n), pf = kSame / (n * n);
        pc = pc < kLdsCap / nvb ? pc : kLdsCap / nvb;
        pf = pf < kLdsCap / ftb ? pf : kLdsCap / ftb;
        const long long bc = (ncell + pc - 1) / pc, bf = (nface + pf - 1) / pf;
        hipLaunchKernelGGL(k_picard_cell_same<NF>, dim3((unsigned)(bc < 65535 ? bc : 65535)), dim3(kSame),
                           (size_t)pc * nvb, s, F, Lv, law, pc, mu_cell64, mu_cell32);
        hipLaunchKernelGGL(k_picard_face_same<NF>, dim3((unsigned)(bf < 65535 ? bf : 65535)), dim3(kSame),
                           (size_t)pf * ftb, s, F, Lv, law, nface, pf, mu_face64, mu_face32);
        return hipGetLastError();
    }
    auto grid = [](long long work) {
        const long long b = (work + kThreads - 1) / kThreads;
        return (unsigned)(b < 1 ? 1 : b > 65535 ? 65535 : b);
    };
    const long long nc = (long long)Lv.nx * Lv.ny * Lv.nz * n * n * n;
    hipLaunchKernelGGL(k_picard_cell<NF>, dim3(grid(nc)), dim3(kThreads), 0, s, F, Lv, law, mu_cell64, mu_cell32);
    hipLaunchKernelGGL(k_picard_face<NF>, dim3(grid(nface * n * n)), dim3(kThreads), 0, s, F, Lv, law, nface,
                       mu_face64, mu_face32);
    return hipGetLastError();
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
    switch (F.n) {
        case 2: return launch_nf<2>(F, Lv, law, nface, mu_cell64, mu_cell32, mu_face64, mu_face32, s);
        case 3: return launch_nf<3>(F, Lv, law, nface, mu_cell64, mu_cell32, mu_face64, mu_face32, s);
        case 4: return launch_nf<4>(F, Lv, law, nface, mu_cell64, mu_cell32, mu_face64, mu_face32, s);
        case 5: return launch_nf<5>(F, Lv, law, nface, mu_cell64, mu_cell32, mu_face64, mu_face32, s);
        case 6: return launch_nf<6>(F, Lv, law, nface, mu_cell64, mu_cell32, mu_face64, mu_face32, s);
    }
    return hipErrorInvalidValue;
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
