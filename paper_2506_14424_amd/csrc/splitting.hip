// Operators of one dual-splitting time step that are not linear solves
// (Sec. 3 "Splitting Scheme"; weak forms of Sec. 4.1; order of Alg. 1):
//
//   convective step   uhat = sum_i (alpha_i/gamma_0) u^{n-i} + (dt/gamma_0)(b - sum_i beta_i M^-1 c_h(u^{n-i}; u^{n-i}))
//                     (eqs. convective_step_weak, convective_term_weak: (w.grad)u
//                     in the cell, upwind flux on the faces, mirror principle
//                     with g_u = 0 on the walls, where {w} = 0 removes the term)
//   pressure rhs      f_q = (gamma_0/dt)[(grad q, uhat) - (q, {uhat}.n)] + (q, h_p)_walls
//                     (eq. pressure_step_weak; on the walls {uhat} = g_uhat of
//                     eq. guhat_consistent_BC from the interior traces of u^n, b,
//                     grad u^n, and h_p of eq. pressure_Neumann_BC)
//   projection        uhh = uhat + (dt/gamma_0) M^-1 [(div v, p) - (v, {p} n)]
//                     (eq. projection_step_weak; {p} = p- on the walls) and the
//                     viscous step's right-hand side (gamma_0/dt) M uhh
//   mass              y = s M x
//   penalty factors   tau_div = zeta |u_e| h_e dt/(k+1), tau_cont = zeta |u_e| dt,
//                     |u_e| the volume mean of |u| over the cell
//
// BDF1 (gamma_0 = alpha_0 = beta_0 = 1; m_p = 0 leaves no extrapolated
// terms in h_p) or BDF2 (gamma_0 = 3/2, alpha = (2, -1/2), beta = (2, -1);
// m_p = 1: h_p takes -n.((grad u^n) u^n) - nu n.curl(omega) +
// 2 n.(grad^S u^n . grad nu) with omega = curl u^n and nu = eta(gdot(u^n))
// projected onto DG_k, i.e. their values at the Gauss nodes; the
// coefficients come in SplitGeo).  Velocity DG_k nodal at its n = k+1 Gauss
// points, pressure DG_{k-1} at its n-1; all integrals on the velocity's
// n-point rule.  One workgroup per cell: thread q < n^3 owns a velocity
// node (or a quadrature point), thread t < 6 n^2 a face point, thread
// j < (n-1)^3 a pressure node; the cell's data are staged in LDS.  FP64.

#include <algorithm>

#include "device_common.h"

namespace sipg {

namespace {

// Workgroup sizes: a multiple of the 64-wide wavefront covering a cell's
// n^3 nodes (kCellThreads, a power of two for the tree sums) or also its
// 6 n^2 face points (kFaceThreads).
template <int N>
constexpr int kCellThreads = N * N * N <= 64 ? 64 : N * N * N <= 128 ? 128 : 256;
template <int N>
constexpr int kFaceThreads = ((N * N * N > 6 * N * N ? N * N * N : 6 * N * N) + 63) / 64 * 64;

struct CellMap {
    bool curved;
    double geo[8][3];
    double h[3], hinv[3];
};

__device__ __forceinline__ void cell_map(const SplitGeo& S, int ex, int ey, int ez, CellMap& m) {
    m.curved = S.verts != nullptr;
    if (m.curved) {
        double g[8];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            trilinear_coeffs(S.verts, S.nx, S.ny, ex, ey, ez, i, g);
#pragma unroll
            for (int k = 0; k < 8; ++k) m.geo[k][i] = g[k];
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        m.h[d] = S.h[d];
        m.hinv[d] = S.hinv[d];
    }
}

__device__ __forceinline__ void point_geo(const CellMap& m, double x1, double x2, double x3, double Ji[3][3],
                                          double& det) {
    if (m.curved) {
        jacobian_inverse<double>(m.geo, x1, x2, x3, Ji, det);
        return;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int i = 0; i < 3; ++i) Ji[d][i] = d == i ? m.hinv[d] : 0.0;
    det = m.h[0] * m.h[1] * m.h[2];
}

// The face xi_d = s of a cell: its tangential axes (t1 < t2), the unit
// normal out of the cell and ds at the face point (g_a, g_b).
struct FacePoint {
    int t1, t2;
    double n[3], ds;
    double Ji[3][3];
};

__device__ __forceinline__ void face_point(const SplitGeo& S, const CellMap& m, int d, int s, int a, int b,
                                           FacePoint& fp) {
    fp.t1 = d == 0 ? 1 : 0;
    fp.t2 = d == 2 ? 1 : 2;
    double xi[3];
    xi[d] = s;
    xi[fp.t1] = S.tab.x[a];
    xi[fp.t2] = S.tab.x[b];
    double det;
    point_geo(m, xi[0], xi[1], xi[2], fp.Ji, det);
    const double v0 = fp.Ji[d][0], v1 = fp.Ji[d][1], v2 = fp.Ji[d][2];
    const double nv = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    const double sg = s ? 1.0 : -1.0;
    fp.n[0] = sg * v0 / nv;
    fp.n[1] = sg * v1 / nv;
    fp.n[2] = sg * v2 / nv;
    fp.ds = det * nv * S.tab.w[a] * S.tab.w[b];
}

__device__ __forceinline__ void cell_ijk(const SplitGeo& S, int e, int ijk[3]) {
    ijk[0] = e % S.nx;
    ijk[1] = (e / S.nx) % S.ny;
    ijk[2] = e / (S.nx * S.ny);
}

// neighbour across face (d, s), or -1 on the boundary
__device__ __forceinline__ int neighbour(const SplitGeo& S, int e, const int ijk[3], int d, int s) {
    const int lim = d == 0 ? S.nx : d == 1 ? S.ny : S.nz;
    const int stride = d == 0 ? 1 : d == 1 ? S.nx : S.nx * S.ny;
    if (s == 1) return ijk[d] < lim - 1 ? e + stride : -1;
    return ijk[d] > 0 ? e - stride : -1;
}

// Row of the wall data for the face (d, s) of a boundary cell: sides -x,
// +x, -y, +y, -z, +z, each in the order of its cells' tangential indices.
__device__ __forceinline__ int wall_row(const SplitGeo& S, const int ijk[3], int d, int s) {
    const int nx = S.nx, ny = S.ny, nz = S.nz;
    const int sz[3] = {ny * nz, nx * nz, nx * ny};
    int off = 0;
    for (int k = 0; k < 2 * d + s; ++k) off += sz[k >> 1];
    const int in = d == 0 ? ijk[2] * ny + ijk[1] : d == 1 ? ijk[2] * nx + ijk[0] : ijk[1] * nx + ijk[0];
    return off + in;
}

// Global number of the face (d, s) of cell ijk: x-faces, then y-, then z-faces.
__device__ __forceinline__ int face_id(const SplitGeo& S, const int ijk[3], int d, int s) {
    const int nx = S.nx, ny = S.ny, nz = S.nz;
    const int nfx = (nx + 1) * ny * nz, nfy = nx * (ny + 1) * nz;
    if (d == 0) return (ijk[2] * ny + ijk[1]) * (nx + 1) + ijk[0] + s;
    if (d == 1) return nfx + (ijk[2] * (ny + 1) + ijk[1] + s) * nx + ijk[0];
    return nfx + nfy + ((ijk[2] + s) * ny + ijk[1]) * nx + ijk[0];
}

// ds ({w}.n) (u+ - u-) at face point ab of face FC if {w}.n < 0 (inflow:
// u_dag = u+), else 0; zero on a wall ({w} = g_u = 0).  U: the cell's values.
template <int N, int FC>
__device__ __forceinline__ void conv_face(const SplitGeo& S, const CellMap& m, int e, const int ijk[3], int ab,
                                          const double* U, const double* __restrict__ u, double* out) {
    constexpr int N2 = N * N, N3 = N2 * N, d = FC >> 1, s = FC & 1;
    const int str[3] = {1, N, N2};
    out[0] = out[1] = out[2] = 0.0;
    const int ne = neighbour(S, e, ijk, d, s);
    if (ne < 0 && S.gw == nullptr) return;       // no-slip wall: {w} = g_u = 0
    const int a = ab % N, bb = ab / N;
    FacePoint fp;
    face_point(S, m, d, s, a, bb, fp);
    const int line = a * str[fp.t1] + bb * str[fp.t2];
    double um[3], up[3];
    if (ne >= 0) {
        const double* un = u + (long long)ne * 3 * N3;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double sm = 0.0, sp = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) {
                sm += S.tab.S[s][k] * U[c * N3 + line + k * str[d]];
                sp += S.tab.S[1 - s][k] * un[c * N3 + line + k * str[d]];
            }
            um[c] = sm;
            up[c] = sp;
        }
    } else {                                      // wall data: mirror u+ = 2 g_u - u-
        const double* g = S.gw + ((long long)wall_row(S, ijk, d, s) * N2 + ab) * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double sm = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) sm += S.tab.S[s][k] * U[c * N3 + line + k * str[d]];
            um[c] = sm;
            up[c] = 2.0 * g[c] - sm;
        }
    }
    const double wn = 0.5 * ((um[0] + up[0]) * fp.n[0] + (um[1] + up[1]) * fp.n[1] + (um[2] + up[2]) * fp.n[2]);
    if (wn < 0.0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] = fp.ds * wn * (up[c] - um[c]);
    }
}

template <int N>
__global__ void __launch_bounds__(kFaceThreads<N>) k_split_convective(SplitGeo S, const double* __restrict__ u,
                                                                     const double* __restrict__ u1,
                                                                     const double* __restrict__ b, double dt,
                                                                     double* __restrict__ uhat) {
    constexpr int N2 = N * N, N3 = N2 * N;
    __shared__ double U[3 * N3];
    __shared__ double FF[6][N2][3];
    const int e = blockIdx.x, t = threadIdx.x;
    int ijk[3];
    cell_ijk(S, e, ijk);
    CellMap m;
    cell_map(S, ijk[0], ijk[1], ijk[2], m);
    const int qi[3] = {t % N, (t / N) % N, t / N2};
    const int str[3] = {1, N, N2};
    double Ji[3][3], det = 1.0;
    if (t < N3) point_geo(m, S.tab.x[qi[0]], S.tab.x[qi[1]], S.tab.x[qi[2]], Ji, det);
    const double wq = S.tab.w[qi[0] % N] * S.tab.w[qi[1] % N] * S.tab.w[qi[2] % N];
    const double inv_m = 1.0 / (wq * det);
    double cacc[3] = {0.0, 0.0, 0.0}, uacc[3] = {0.0, 0.0, 0.0};
    // sum over the old velocities u^{n-i}: alpha_i u^{n-i} and beta_i M^-1 c_h(u^{n-i}; u^{n-i})
    for (int i = 0; i < S.order; ++i) {
        const double* ui = i == 0 ? u : u1;
        __syncthreads();                              // the previous velocity's readers are done
        const double* ue = ui + (long long)e * 3 * N3;
        for (int k = t; k < 3 * N3; k += blockDim.x) U[k] = ue[k];
        __syncthreads();
        if (t < 6 * N2) {
            const int fc = t / N2, ab = t % N2;
            switch (fc) {
                case 0: conv_face<N, 0>(S, m, e, ijk, ab, U, ui, FF[0][ab]); break;
                case 1: conv_face<N, 1>(S, m, e, ijk, ab, U, ui, FF[1][ab]); break;
                case 2: conv_face<N, 2>(S, m, e, ijk, ab, U, ui, FF[2][ab]); break;
                case 3: conv_face<N, 3>(S, m, e, ijk, ab, U, ui, FF[3][ab]); break;
                case 4: conv_face<N, 4>(S, m, e, ijk, ab, U, ui, FF[4][ab]); break;
                default: conv_face<N, 5>(S, m, e, ijk, ab, U, ui, FF[5][ab]); break;
            }
        }
        __syncthreads();
        if (t < N3) {
            double uq[3], gr[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                uq[c] = U[c * N3 + t];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    double acc = 0.0;
                    const int base = c * N3 + t - qi[d] * str[d];
#pragma unroll
                    for (int k = 0; k < N; ++k) acc += S.tab.D[qi[d]][k] * U[base + k * str[d]];
                    gr[c][d] = acc;
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double a = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    a += (gr[c][0] * Ji[0][k] + gr[c][1] * Ji[1][k] + gr[c][2] * Ji[2][k]) * uq[k];
                double face = 0.0;
#pragma unroll
                for (int fc = 0; fc < 6; ++fc) {
                    const int d = fc >> 1, s = fc & 1;
                    const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;
                    face += S.tab.S[s][qi[d]] * FF[fc][qi[tb] * N + qi[ta]][c];
                }
                cacc[c] += S.beta[i] * (a + face * inv_m);
                uacc[c] += S.alpha[i] * uq[c];
            }
        }
    }
    if (t >= N3) return;
    double* out = uhat + (long long)e * 3 * N3;
    const double* be = b ? b + (long long)e * 3 * N3 : nullptr;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double bq = be ? be[c * N3 + t] : 0.0;
        out[c * N3 + t] = uacc[c] / S.gamma0 + dt / S.gamma0 * (bq - cacc[c]);
    }
}

__device__ __forceinline__ double eta_split(const SplitGeo& S, double gdot) {
    return S.eta[1] + (S.eta[0] - S.eta[1]) * pow(S.eta[4] + pow(S.eta[2] * gdot, S.eta[5]), (S.eta[3] - 1.0) / S.eta[5]);
}

// Trace and reference gradient (d/dxi_1, d/dxi_2, d/dxi_3) at the face point
// (a, bb) of face (D, SD) of one component's n^3 nodal values P of a cell.
// TB: the 1D tables in LDS, D (n x n), then S (2 x n), then G (2 x n); read
// from LDS rather than the kernel argument, whose runtime-indexed reads made
// the compiler copy the whole argument into scratch.
template <int N, int D, int SD>
__device__ __forceinline__ void face_trace_grad(const double* TB, const double* P, int a, int bb, double& tr,
                                                double gref[3]) {
    constexpr int t1 = D == 0 ? 1 : 0, t2 = D == 2 ? 1 : 2;
    const int str[3] = {1, N, N * N};
    const int line = a * str[t1] + bb * str[t2];
    double v = 0.0, dn = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        v += TB[N * N + SD * N + k] * P[line + k * str[D]];
        dn += TB[N * N + 2 * N + SD * N + k] * P[line + k * str[D]];
    }
#pragma unroll 1
    for (int k2 = 0; k2 < N; ++k2) {
        double t1v = 0.0, t2v = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            t1v += TB[N * N + SD * N + k] * P[k2 * str[t1] + bb * str[t2] + k * str[D]];
            t2v += TB[N * N + SD * N + k] * P[a * str[t1] + k2 * str[t2] + k * str[D]];
        }
        d1 += TB[a * N + k2] * t1v;
        d2 += TB[bb * N + k2] * t2v;
    }
    tr = v;
    gref[D] = dn;
    gref[t1] = d1;
    gref[t2] = d2;
}

// physical gradient G[c][i] of a 3-component field at a face point from its
// trace ut and reference gradients gref[c][d]
__device__ __forceinline__ void phys_grad3(const double gref[3][3], const double Ji[3][3], double G[3][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < 3; ++i) G[c][i] = gref[c][0] * Ji[0][i] + gref[c][1] * Ji[1][i] + gref[c][2] * Ji[2][i];
}

template <int N, int ORDER, int FC>
__device__ __forceinline__ double ppe_face(const SplitGeo& S, const CellMap& m, int e, const int ijk[3], int ab,
                                           const double* __restrict__ uhat, const double* __restrict__ u_old,
                                           const double* __restrict__ u1, const double* __restrict__ b, double dt,
                                           const double* OM, const double* NU, const double* TB) {
    constexpr int N2 = N * N, N3 = N2 * N, d = FC >> 1, s = FC & 1;
    const int str[3] = {1, N, N2};
    const int a = ab % N, bb = ab / N;
    const double* uh = uhat + (long long)e * 3 * N3;
    FacePoint fp;
    face_point(S, m, d, s, a, bb, fp);
    const int line = a * str[fp.t1] + bb * str[fp.t2];     // node (0 along d, a, bb)
    const int ne = neighbour(S, e, ijk, d, s);
    double val;
    if (ne >= 0) {
        const double* un = uhat + (long long)ne * 3 * N3;
        double an = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double sm = 0.0, sp = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) {
                sm += S.tab.S[s][k] * uh[c * N3 + line + k * str[d]];
                sp += S.tab.S[1 - s][k] * un[c * N3 + line + k * str[d]];
            }
            an += 0.5 * (sm + sp) * fp.n[c];
        }
        val = -S.gamma0 / dt * an;
    } else {
        if constexpr (ORDER == 1) {
            // BDF1 wall: g_uhat = (dt/gamma_0)(b - beta_0 (grad u^n) u^n) + (alpha_0/gamma_0) g_u,
            // h_p = n.b (- n.d_t g_u = 0: data constant in time), from the interior traces
            const double* uo = u_old + (long long)e * 3 * N3;
            const double* be = b ? b + (long long)e * 3 * N3 : nullptr;
            double ut[3], bt[3], gref[3][3];
    #pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double* uc = uo + c * N3;
                double tr = 0.0, dn = 0.0, btc = 0.0, d1 = 0.0, d2 = 0.0;
    #pragma unroll
                for (int k = 0; k < N; ++k) {
                    tr += S.tab.S[s][k] * uc[line + k * str[d]];
                    dn += S.tab.G[s][k] * uc[line + k * str[d]];
                    if (be) btc += S.tab.S[s][k] * be[c * N3 + line + k * str[d]];
                }
                // tangential derivatives of the trace
    #pragma unroll 1
                for (int k2 = 0; k2 < N; ++k2) {
                    double t1v = 0.0, t2v = 0.0;
    #pragma unroll
                    for (int k = 0; k < N; ++k) {
                        t1v += S.tab.S[s][k] * uc[k2 * str[fp.t1] + bb * str[fp.t2] + k * str[d]];
                        t2v += S.tab.S[s][k] * uc[a * str[fp.t1] + k2 * str[fp.t2] + k * str[d]];
                    }
                    d1 += S.tab.D[a][k2] * t1v;
                    d2 += S.tab.D[bb][k2] * t2v;
                }
                ut[c] = tr;
                bt[c] = btc;
                gref[c][d] = dn;
                gref[c][fp.t1] = d1;
                gref[c][fp.t2] = d2;
            }
            double gn = 0.0, hp = 0.0;
    #pragma unroll
            for (int c = 0; c < 3; ++c) {
                double conv = 0.0;
    #pragma unroll
                for (int i = 0; i < 3; ++i)
                    conv += (gref[c][0] * fp.Ji[0][i] + gref[c][1] * fp.Ji[1][i] + gref[c][2] * fp.Ji[2][i]) * ut[i];
                const double gu = S.gw ? S.gw[((long long)wall_row(S, ijk, d, s) * N2 + ab) * 3 + c] : 0.0;
                const double guhat = dt / S.gamma0 * (bt[c] - S.beta[0] * conv) + S.alpha[0] / S.gamma0 * gu;
                gn += guhat * fp.n[c];
                hp += fp.n[c] * bt[c];
            }
            val = -S.gamma0 / dt * gn + hp;
        } else {
            // wall, from the interior traces:
            // g_uhat = (dt/gamma_0)(b - sum_i beta_i (grad u^{n-i}) u^{n-i}) + sum_i (alpha_i/gamma_0) g_u,
            // h_p = n.b - n.d_t g_u (= 0: data constant in time) - beta_bar n.((grad u^n) u^n)
            //       - nu n.curl(omega) + 2 n.(grad^S u^n . grad nu)      (BDF2: m_p = 1, u^dd = u^n)
            const double* be = b ? b + (long long)e * 3 * N3 : nullptr;
            double bt[3] = {0.0, 0.0, 0.0};
            if (be) {
    #pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double v = 0.0;
    #pragma unroll
                    for (int k = 0; k < N; ++k) v += S.tab.S[s][k] * be[c * N3 + line + k * str[d]];
                    bt[c] = v;
                }
            }
            double conv_sum[3] = {0.0, 0.0, 0.0}, conv0[3] = {0.0, 0.0, 0.0}, G0[3][3];
    #pragma unroll
            for (int i = 0; i < ORDER; ++i) {
                const double* uo = (i == 0 ? u_old : u1) + (long long)e * 3 * N3;
                double ut[3], gref[3][3], G[3][3];
    #pragma unroll
                for (int c = 0; c < 3; ++c) face_trace_grad<N, d, s>(TB, uo + c * N3, a, bb, ut[c], gref[c]);
                phys_grad3(gref, fp.Ji, G);
    #pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double cv = G[c][0] * ut[0] + G[c][1] * ut[1] + G[c][2] * ut[2];
                    conv_sum[c] += S.beta[i] * cv;
                    if (i == 0) conv0[c] = cv;
                }
                if (ORDER > 1 && i == 0) {
    #pragma unroll
                    for (int c = 0; c < 3; ++c)
    #pragma unroll
                        for (int k = 0; k < 3; ++k) G0[c][k] = G[c][k];
                }
            }
            double gn = 0.0, hp = 0.0;
            const double asum = S.alpha[0] + (ORDER > 1 ? S.alpha[1] : 0.0);
    #pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double gu = S.gw ? S.gw[((long long)wall_row(S, ijk, d, s) * N2 + ab) * 3 + c] : 0.0;
                const double guhat = dt / S.gamma0 * (bt[c] - conv_sum[c]) + asum / S.gamma0 * gu;
                gn += guhat * fp.n[c];
                hp += fp.n[c] * (bt[c] - S.beta_bar * conv0[c]);
            }
            if constexpr (ORDER > 1) {
                double ee = 0.0, Sy[3][3];
    #pragma unroll
                for (int c = 0; c < 3; ++c)
    #pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        Sy[c][k] = 0.5 * (G0[c][k] + G0[k][c]);
                        ee += Sy[c][k] * Sy[c][k];
                    }
                const double nu = eta_split(S, sqrt(2.0 * ee));
                double ot[3], gro[3][3], Go[3][3], nt, gn_ref[3];
    #pragma unroll
                for (int c = 0; c < 3; ++c) face_trace_grad<N, d, s>(TB, OM + c * N3, a, bb, ot[c], gro[c]);
                phys_grad3(gro, fp.Ji, Go);
                const double curl[3] = {Go[2][1] - Go[1][2], Go[0][2] - Go[2][0], Go[1][0] - Go[0][1]};
                face_trace_grad<N, d, s>(TB, NU, a, bb, nt, gn_ref);
                double gnu[3];
    #pragma unroll
                for (int k = 0; k < 3; ++k)
                    gnu[k] = gn_ref[0] * fp.Ji[0][k] + gn_ref[1] * fp.Ji[1][k] + gn_ref[2] * fp.Ji[2][k];
                double ncurl = 0.0, nsg = 0.0;
    #pragma unroll
                for (int c = 0; c < 3; ++c) {
                    ncurl += fp.n[c] * curl[c];
                    nsg += fp.n[c] * (Sy[c][0] * gnu[0] + Sy[c][1] * gnu[1] + Sy[c][2] * gnu[2]);
                }
                hp += -nu * ncurl + 2.0 * nsg;
            }
            val = -S.gamma0 / dt * gn + hp;
        }
    }
    return fp.ds * val;
}

template <int N, int ORDER>
__global__ void __launch_bounds__(kFaceThreads<N>) k_split_ppe_rhs(SplitGeo S, const double* __restrict__ uhat,
                                                                  const double* __restrict__ u_old,
                                                                  const double* __restrict__ u1,
                                                                  const double* __restrict__ b, double dt,
                                                                  double* __restrict__ f) {
    constexpr int N2 = N * N, N3 = N2 * N, NP = N - 1, NP3 = NP * NP * NP;
    __shared__ double GQ[3][N3];
    __shared__ double FF[6][N2];
    // BDF2, wall cells: u^n, its vorticity and viscosity at the nodes
    __shared__ double UO[ORDER > 1 ? 3 * N3 : 1];
    __shared__ double OM[ORDER > 1 ? 3 * N3 : 1];
    __shared__ double NU[ORDER > 1 ? N3 : 1];
    __shared__ double TB[ORDER > 1 ? N2 + 4 * N : 1];   // BDF2 wall cells: D, S, G tables
    static_assert(kFaceThreads<N> >= N2 + 4 * N, "one thread per table entry");
    const int e = blockIdx.x, t = threadIdx.x;
    int ijk[3];
    cell_ijk(S, e, ijk);
    CellMap m;
    cell_map(S, ijk[0], ijk[1], ijk[2], m);
    const int str[3] = {1, N, N2};
    const double* uh = uhat + (long long)e * 3 * N3;
    const bool wall = ijk[0] == 0 || ijk[0] == S.nx - 1 || ijk[1] == 0 || ijk[1] == S.ny - 1 || ijk[2] == 0 ||
                      ijk[2] == S.nz - 1;
    if (ORDER > 1 && wall) {           // uniform over the workgroup
        const double* uo = u_old + (long long)e * 3 * N3;
        for (int k = t; k < 3 * N3; k += blockDim.x) UO[k] = uo[k];
        if (t < N2) TB[t] = S.tab.D[t / N][t % N];
        else if (t < N2 + 2 * N) TB[t] = S.tab.S[(t - N2) / N][(t - N2) % N];
        else if (t < N2 + 4 * N) TB[t] = S.tab.G[(t - N2 - 2 * N) / N][(t - N2 - 2 * N) % N];
        __syncthreads();
        if (t < N3) {
            // omega = curl u and nu = eta(gdot(grad^S u)) at the node: with the
            // nodes at the Gauss points (diagonal mass matrix) these are the
            // element-local L2 projections onto DG_k
            const int qi[3] = {t % N, (t / N) % N, t / N2};
            double Ji[3][3], det, gr[3][3], G[3][3];
            point_geo(m, S.tab.x[qi[0]], S.tab.x[qi[1]], S.tab.x[qi[2]], Ji, det);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    double acc = 0.0;
                    const int base = c * N3 + t - qi[d] * str[d];
#pragma unroll
                    for (int k = 0; k < N; ++k) acc += S.tab.D[qi[d]][k] * UO[base + k * str[d]];
                    gr[c][d] = acc;
                }
            phys_grad3(gr, Ji, G);
            OM[t] = G[2][1] - G[1][2];
            OM[N3 + t] = G[0][2] - G[2][0];
            OM[2 * N3 + t] = G[1][0] - G[0][1];
            double ee = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double sy = 0.5 * (G[c][k] + G[k][c]);
                    ee += sy * sy;
                }
            NU[t] = eta_split(S, sqrt(2.0 * ee));
        }
        __syncthreads();
    }
    if (t < N3) {
        const int q1 = t % N, q2 = (t / N) % N, q3 = t / N2;
        double Ji[3][3], det;
        point_geo(m, S.tab.x[q1], S.tab.x[q2], S.tab.x[q3], Ji, det);
        const double jw = S.tab.w[q1] * S.tab.w[q2] * S.tab.w[q3] * det;
        const double u0 = uh[t], v1 = uh[N3 + t], v2 = uh[2 * N3 + t];
#pragma unroll
        for (int d = 0; d < 3; ++d) GQ[d][t] = jw * (Ji[d][0] * u0 + Ji[d][1] * v1 + Ji[d][2] * v2);
    }
    if (t < 6 * N2) {
        const int fc = t / N2, ab = t % N2;
        double v = 0.0;
        switch (fc) {
            case 0: v = ppe_face<N, ORDER, 0>(S, m, e, ijk, ab, uhat, u_old, u1, b, dt, OM, NU, TB); break;
            case 1: v = ppe_face<N, ORDER, 1>(S, m, e, ijk, ab, uhat, u_old, u1, b, dt, OM, NU, TB); break;
            case 2: v = ppe_face<N, ORDER, 2>(S, m, e, ijk, ab, uhat, u_old, u1, b, dt, OM, NU, TB); break;
            case 3: v = ppe_face<N, ORDER, 3>(S, m, e, ijk, ab, uhat, u_old, u1, b, dt, OM, NU, TB); break;
            case 4: v = ppe_face<N, ORDER, 4>(S, m, e, ijk, ab, uhat, u_old, u1, b, dt, OM, NU, TB); break;
            default: v = ppe_face<N, ORDER, 5>(S, m, e, ijk, ab, uhat, u_old, u1, b, dt, OM, NU, TB); break;
        }
        FF[fc][ab] = v;
    }
    __syncthreads();
    if (t >= NP3) return;
    const int j[3] = {t % NP, (t / NP) % NP, t / (NP * NP)};
    double acc = 0.0;
#pragma unroll 1
    for (int q3 = 0; q3 < N; ++q3) {
        const double v3 = S.PV[q3][j[2]], d3 = S.PD[q3][j[2]];
#pragma unroll
        for (int q2 = 0; q2 < N; ++q2) {
            const double v2 = S.PV[q2][j[1]], d2 = S.PD[q2][j[1]];
#pragma unroll
            for (int q1 = 0; q1 < N; ++q1) {
                const int q = (q3 * N + q2) * N + q1;
                const double v1 = S.PV[q1][j[0]], d1 = S.PD[q1][j[0]];
                acc += d1 * v2 * v3 * GQ[0][q] + v1 * d2 * v3 * GQ[1][q] + v1 * v2 * d3 * GQ[2][q];
            }
        }
    }
    acc *= S.gamma0 / dt;
#pragma unroll
    for (int fc = 0; fc < 6; ++fc) {
        const int d = fc >> 1, s = fc & 1;
        const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        const double cn = S.PS[s][j[d]];
        double fs = 0.0;
#pragma unroll
        for (int bb = 0; bb < N; ++bb) {
            double row = 0.0;
#pragma unroll
            for (int a = 0; a < N; ++a) row += S.PV[a][j[t1]] * FF[fc][bb * N + a];
            fs += S.PV[bb][j[t2]] * row;
        }
        acc += cn * fs;
    }
    f[(long long)e * NP3 + t] = acc;
}

// Penalty-step factors of a coarse mesh-step level: the mean of each coarse
// cell's 8 children (fine mesh fx * fy * fz, children in the order of their
// (z, y, x) offsets), as the multigrid hierarchy is built.
__global__ void k_pen_coarsen(int fx, int fy, int fz, const double* __restrict__ td, const double* __restrict__ tc,
                              double* __restrict__ ctd, double* __restrict__ ctc) {
    const int cx = fx / 2, cy = fy / 2, cz = fz / 2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cx * cy * cz) return;
    const int i = e % cx, j = (e / cx) % cy, k = e / (cx * cy);
    double a = 0.0, b = 0.0;
    for (int c = 0; c < 8; ++c) {
        const long long f = ((long long)(2 * k + (c >> 2)) * fy + 2 * j + ((c >> 1) & 1)) * fx + 2 * i + (c & 1);
        a += td[f];
        b += tc[f];
    }
    ctd[e] = a / 8.0;
    ctc[e] = b / 8.0;
}

__global__ void k_lincomb(long long n, double a, const double* __restrict__ x, double c,
                          const double* __restrict__ z, double* __restrict__ y) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        y[i] = a * x[i] + c * z[i];
}

// pressure of a cell (NP^3 nodal values) at the velocity face point (a, b) of face (d, s)
template <int N>
__device__ __forceinline__ double pressure_at_face(const SplitGeo& S, const double* P, int d, int s, int a, int b) {
    constexpr int NP = N - 1;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const int sp[3] = {1, NP, NP * NP};
    double acc = 0.0;
#pragma unroll
    for (int jd = 0; jd < NP; ++jd) {
        double plane = 0.0;
#pragma unroll
        for (int j2 = 0; j2 < NP; ++j2) {
            double row = 0.0;
#pragma unroll
            for (int j1 = 0; j1 < NP; ++j1) row += S.PV[a][j1] * P[jd * sp[d] + j1 * sp[t1] + j2 * sp[t2]];
            plane += S.PV[b][j2] * row;
        }
        acc += S.PS[s][jd] * plane;
    }
    return acc;
}

// ds {p} n at the face point ab of face FC ({p} = p- on a wall)
template <int N, int FC>
__device__ __forceinline__ void proj_face(const SplitGeo& S, const CellMap& m, int e, const int ijk[3], int ab,
                                          const double* PL, const double* __restrict__ p, double* out) {
    constexpr int NP = N - 1, NP3 = NP * NP * NP, d = FC >> 1, s = FC & 1;
    const int a = ab % N, bb = ab / N;
    FacePoint fp;
    face_point(S, m, d, s, a, bb, fp);
    const int ne = neighbour(S, e, ijk, d, s);
    double pavg = pressure_at_face<N>(S, PL, d, s, a, bb);
    if (ne >= 0) pavg = 0.5 * (pavg + pressure_at_face<N>(S, p + (long long)ne * NP3, d, 1 - s, a, bb));
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = fp.ds * pavg * fp.n[c];
}

template <int N>
__global__ void __launch_bounds__(kFaceThreads<N>) k_split_projection(SplitGeo S, const double* __restrict__ uhat,
                                                               const double* __restrict__ p, double dt,
                                                               double* __restrict__ uhh, double* __restrict__ rhs) {
    constexpr int N2 = N * N, N3 = N2 * N, NP = N - 1, NP3 = NP * NP * NP;
    __shared__ double H[9][N3];
    __shared__ double FP[6][N2][3];
    __shared__ double PL[NP3];
    const int e = blockIdx.x, t = threadIdx.x;
    for (int i = t; i < NP3; i += blockDim.x) PL[i] = p[(long long)e * NP3 + i];
    __syncthreads();
    int ijk[3];
    cell_ijk(S, e, ijk);
    CellMap m;
    cell_map(S, ijk[0], ijk[1], ijk[2], m);
    const int str[3] = {1, N, N2};
    const int qi[3] = {t % N, (t / N) % N, t / N2};
    double jw = 0.0;
    if (t < N3) {
        double Ji[3][3], det;
        point_geo(m, S.tab.x[qi[0]], S.tab.x[qi[1]], S.tab.x[qi[2]], Ji, det);
        jw = S.tab.w[qi[0]] * S.tab.w[qi[1]] * S.tab.w[qi[2]] * det;
        double pq = 0.0;
#pragma unroll 1
        for (int j3 = 0; j3 < NP; ++j3) {
            double plane = 0.0;
#pragma unroll
            for (int j2 = 0; j2 < NP; ++j2) {
                double row = 0.0;
#pragma unroll
                for (int j1 = 0; j1 < NP; ++j1) row += S.PV[qi[0]][j1] * PL[(j3 * NP + j2) * NP + j1];
                plane += S.PV[qi[1]][j2] * row;
            }
            pq += S.PV[qi[2]][j3] * plane;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int c = 0; c < 3; ++c) H[d * 3 + c][t] = jw * Ji[d][c] * pq;
    }
    if (t < 6 * N2) {
        const int fc = t / N2, ab = t % N2;
        switch (fc) {
            case 0: proj_face<N, 0>(S, m, e, ijk, ab, PL, p, FP[0][ab]); break;
            case 1: proj_face<N, 1>(S, m, e, ijk, ab, PL, p, FP[1][ab]); break;
            case 2: proj_face<N, 2>(S, m, e, ijk, ab, PL, p, FP[2][ab]); break;
            case 3: proj_face<N, 3>(S, m, e, ijk, ab, PL, p, FP[3][ab]); break;
            case 4: proj_face<N, 4>(S, m, e, ijk, ab, PL, p, FP[4][ab]); break;
            default: proj_face<N, 5>(S, m, e, ijk, ab, PL, p, FP[5][ab]); break;
        }
    }
    __syncthreads();
    if (t >= N3) return;
    const double* ue = uhat + (long long)e * 3 * N3;
    double* out = uhh + (long long)e * 3 * N3;
    double* ro = rhs ? rhs + (long long)e * 3 * N3 : nullptr;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int base = t - qi[d] * str[d];
#pragma unroll
            for (int k = 0; k < N; ++k) acc += S.tab.D[k][qi[d]] * H[d * 3 + c][base + k * str[d]];
        }
#pragma unroll
        for (int fc = 0; fc < 6; ++fc) {
            const int d = fc >> 1, s = fc & 1;
            const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;
            acc -= S.tab.S[s][qi[d]] * FP[fc][qi[tb] * N + qi[ta]][c];
        }
        const double v = ue[c * N3 + t] + dt / S.gamma0 * acc / jw;
        out[c * N3 + t] = v;
        if (ro) ro[c * N3 + t] = S.gamma0 / dt * jw * v;
    }
}

template <int N>
__global__ void __launch_bounds__(kCellThreads<N>) k_split_mass(SplitGeo S, const double* __restrict__ x, double scale,
                                                         double* __restrict__ y) {
    constexpr int N2 = N * N, N3 = N2 * N;
    const int e = blockIdx.x, t = threadIdx.x;
    if (t >= N3) return;
    int ijk[3];
    cell_ijk(S, e, ijk);
    CellMap m;
    cell_map(S, ijk[0], ijk[1], ijk[2], m);
    const int q1 = t % N, q2 = (t / N) % N, q3 = t / N2;
    double Ji[3][3], det;
    point_geo(m, S.tab.x[q1], S.tab.x[q2], S.tab.x[q3], Ji, det);
    const double jw = scale * S.tab.w[q1] * S.tab.w[q2] * S.tab.w[q3] * det;
    const long long o = (long long)e * 3 * N3 + t;
#pragma unroll
    for (int c = 0; c < 3; ++c) y[o + c * N3] = jw * x[o + c * N3];
}

template <int N>
__global__ void __launch_bounds__(kCellThreads<N>) k_pen_factors(SplitGeo S, const double* __restrict__ u, double dt,
                                                          double zeta, const double* __restrict__ hcell,
                                                          double* __restrict__ tau_div, double* __restrict__ tau_cont) {
    constexpr int N2 = N * N, N3 = N2 * N;
    constexpr int B = kCellThreads<N>;
    __shared__ double sw[B], su[B];
    const int e = blockIdx.x, t = threadIdx.x;
    double jw = 0.0, js = 0.0;
    if (t < N3) {
        int ijk[3];
        cell_ijk(S, e, ijk);
        CellMap m;
        cell_map(S, ijk[0], ijk[1], ijk[2], m);
        const int q1 = t % N, q2 = (t / N) % N, q3 = t / N2;
        double Ji[3][3], det;
        point_geo(m, S.tab.x[q1], S.tab.x[q2], S.tab.x[q3], Ji, det);
        jw = S.tab.w[q1] * S.tab.w[q2] * S.tab.w[q3] * det;
        const double* ue = u + (long long)e * 3 * N3;
        const double a = ue[t], b = ue[N3 + t], c = ue[2 * N3 + t];
        js = jw * sqrt(a * a + b * b + c * c);
    }
    sw[t] = jw;
    su[t] = js;
    __syncthreads();
    for (int w = B / 2; w > 0; w >>= 1) {          // fixed-order tree: deterministic
        if (t < w) {
            sw[t] += sw[t + w];
            su[t] += su[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double ue = su[0] / sw[0];
        tau_div[e] = zeta * ue * hcell[e] * dt / N;
        tau_cont[e] = zeta * ue * dt;
    }
}

// One wall face point of the load: ds a (value part) and ds J^-1 B (gradient
// part, reference frame) of the viscous (a = 2 tau (g + (g.n) n), B = -2 mu
// sym(g (x) n)) or penalty (a = tau_e (g.n) n, B = 0) wall data; zero off the walls.
template <int N, int FC>
__device__ __forceinline__ void load_face(const SplitGeo& S, const CellMap& m, int e, const int ijk[3], int ab,
                                          const double* __restrict__ mu_face, const double* __restrict__ tfac,
                                          int pen, double* va, double* vb) {
    constexpr int N2 = N * N, d = FC >> 1, s = FC & 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) va[c] = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) vb[k] = 0.0;
    if (neighbour(S, e, ijk, d, s) >= 0) return;
    const int a = ab % N, bb = ab / N;
    FacePoint fp;
    face_point(S, m, d, s, a, bb, fp);
    const int fid = face_id(S, ijk, d, s);
    const double* g = S.gw + ((long long)wall_row(S, ijk, d, s) * N2 + ab) * 3;
    const double gn = g[0] * fp.n[0] + g[1] * fp.n[1] + g[2] * fp.n[2];
    if (pen) {
        const double t = tfac[fid] * gn * fp.ds;
#pragma unroll
        for (int c = 0; c < 3; ++c) va[c] = t * fp.n[c];
        return;
    }
    const double mu = mu_face[(long long)fid * N2 + ab];
    const double tau = tfac[fid] * mu;
#pragma unroll
    for (int c = 0; c < 3; ++c) va[c] = fp.ds * 2.0 * tau * (g[c] + gn * fp.n[c]);
    // B = -2 mu sym(g (x) n) = -mu (g_c n_i + g_i n_c); vb[c*3 + r] = ds sum_i Ji[r][i] B[c][i]
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) acc += fp.Ji[r][i] * (-mu * (g[c] * fp.n[i] + g[i] * fp.n[c]));
            vb[c * 3 + r] = fp.ds * acc;
        }
}

template <int N>
__global__ void __launch_bounds__(kFaceThreads<N>) k_wall_load(SplitGeo S, const double* __restrict__ mu_face,
                                                              const double* __restrict__ tfac, int pen,
                                                              double* __restrict__ y) {
    constexpr int N2 = N * N, N3 = N2 * N;
    __shared__ double VA[6][N2][3];
    __shared__ double VB[6][N2][9];
    const int e = blockIdx.x, t = threadIdx.x;
    int ijk[3];
    cell_ijk(S, e, ijk);
    const bool wall = ijk[0] == 0 || ijk[0] == S.nx - 1 || ijk[1] == 0 || ijk[1] == S.ny - 1 || ijk[2] == 0 ||
                      ijk[2] == S.nz - 1;
    if (!wall) return;                            // whole workgroup: interior cells carry no load
    CellMap m;
    cell_map(S, ijk[0], ijk[1], ijk[2], m);
    if (t < 6 * N2) {
        const int fc = t / N2, ab = t % N2;
        switch (fc) {
            case 0: load_face<N, 0>(S, m, e, ijk, ab, mu_face, tfac, pen, VA[0][ab], VB[0][ab]); break;
            case 1: load_face<N, 1>(S, m, e, ijk, ab, mu_face, tfac, pen, VA[1][ab], VB[1][ab]); break;
            case 2: load_face<N, 2>(S, m, e, ijk, ab, mu_face, tfac, pen, VA[2][ab], VB[2][ab]); break;
            case 3: load_face<N, 3>(S, m, e, ijk, ab, mu_face, tfac, pen, VA[3][ab], VB[3][ab]); break;
            case 4: load_face<N, 4>(S, m, e, ijk, ab, mu_face, tfac, pen, VA[4][ab], VB[4][ab]); break;
            default: load_face<N, 5>(S, m, e, ijk, ab, mu_face, tfac, pen, VA[5][ab], VB[5][ab]); break;
        }
    }
    __syncthreads();
    if (t >= N3) return;
    const int qi[3] = {t % N, (t / N) % N, t / N2};
    double* out = y + (long long)e * 3 * N3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int fc = 0; fc < 6; ++fc) {
            const int d = fc >> 1, s = fc & 1;
            const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            const int a = qi[t1], b = qi[t2];
            const double sv = S.tab.S[s][qi[d]];
            // grad phi_i at the face point (k, b) along t1 and (a, k) along t2; l_j'(g_k) = D[k][j]
            double f = sv * VA[fc][b * N + a][c] + S.tab.G[s][qi[d]] * VB[fc][b * N + a][c * 3 + d];
#pragma unroll
            for (int k = 0; k < N; ++k) {
                f += sv * S.tab.D[k][a] * VB[fc][b * N + k][c * 3 + t1];
                f += sv * S.tab.D[k][b] * VB[fc][k * N + a][c * 3 + t2];
            }
            acc += f;
        }
        out[c * N3 + t] += acc;
    }
}

template <int N>
hipError_t launch_n(int which, const SplitGeo& S, const double* a0, const double* a1, const double* a2,
                    const double* a3, double s0, double s1, double* o0, double* o1, hipStream_t s) {
    const dim3 grid((unsigned)(S.nx * S.ny * S.nz)), cb(kCellThreads<N>), fb(kFaceThreads<N>);
    static_assert(kCellThreads<N> >= N * N * N && kFaceThreads<N> >= 6 * N * N && kFaceThreads<N> >= N * N * N,
                  "a workgroup must cover the cell's nodes and face points");
    switch (which) {
        case 0: hipLaunchKernelGGL(k_split_convective<N>, grid, fb, 0, s, S, a0, a1, a2, s0, o0); break;
        case 1:
            if (S.order > 1)
                hipLaunchKernelGGL((k_split_ppe_rhs<N, 2>), grid, fb, 0, s, S, a0, a1, a2, a3, s0, o0);
            else
                hipLaunchKernelGGL((k_split_ppe_rhs<N, 1>), grid, fb, 0, s, S, a0, a1, a2, a3, s0, o0);
            break;
        case 2: hipLaunchKernelGGL(k_split_projection<N>, grid, fb, 0, s, S, a0, a1, s0, o0, o1); break;
        case 3: hipLaunchKernelGGL(k_split_mass<N>, grid, cb, 0, s, S, a0, s0, o0); break;
        case 4: hipLaunchKernelGGL(k_pen_factors<N>, grid, cb, 0, s, S, a0, s0, s1, a1, o0, o1); break;
        case 5: hipLaunchKernelGGL(k_wall_load<N>, grid, fb, 0, s, S, a0, a1, (int)s0, o0); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t dispatch(int n, int which, const SplitGeo& S, const double* a0, const double* a1, const double* a2,
                    double s0, double s1, double* o0, double* o1, hipStream_t s, const double* a3 = nullptr) {
    switch (n) {
        case 3: return launch_n<3>(which, S, a0, a1, a2, a3, s0, s1, o0, o1, s);
        case 4: return launch_n<4>(which, S, a0, a1, a2, a3, s0, s1, o0, o1, s);
        case 5: return launch_n<5>(which, S, a0, a1, a2, a3, s0, s1, o0, o1, s);
        case 6: return launch_n<6>(which, S, a0, a1, a2, a3, s0, s1, o0, o1, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_split_convective(int n, const SplitGeo& S, const double* u, const double* u_prev, const double* b,
                                   double dt, double* uhat, hipStream_t s) {
    return dispatch(n, 0, S, u, u_prev, b, dt, 0.0, uhat, nullptr, s);
}

hipError_t launch_split_ppe_rhs(int n, const SplitGeo& S, const double* uhat, const double* u_old,
                                const double* u_prev, const double* b, double dt, double* f, hipStream_t s) {
    return dispatch(n, 1, S, uhat, u_old, u_prev, dt, 0.0, f, nullptr, s, b);
}

hipError_t launch_pen_coarsen(int fx, int fy, int fz, const double* td, const double* tc, double* ctd, double* ctc,
                              hipStream_t s) {
    const int nc = (fx / 2) * (fy / 2) * (fz / 2);
    hipLaunchKernelGGL(k_pen_coarsen, dim3((nc + 255) / 256), dim3(256), 0, s, fx, fy, fz, td, tc, ctd, ctc);
    return hipGetLastError();
}

hipError_t launch_lincomb(long long n, double a, const double* x, double c, const double* z, double* y, hipStream_t s) {
    const long long blocks = std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_lincomb, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, s, n, a, x, c, z, y);
    return hipGetLastError();
}

hipError_t launch_split_projection(int n, const SplitGeo& S, const double* uhat, const double* p, double dt,
                                   double* uhh, double* rhs, hipStream_t s) {
    return dispatch(n, 2, S, uhat, p, nullptr, dt, 0.0, uhh, rhs, s);
}

hipError_t launch_split_mass(int n, const SplitGeo& S, const double* x, double scale, double* y, hipStream_t s) {
    return dispatch(n, 3, S, x, nullptr, nullptr, scale, 0.0, y, nullptr, s);
}

hipError_t launch_pen_factors(int n, const SplitGeo& S, const double* u, double dt, double zeta, const double* hcell,
                              double* tau_div, double* tau_cont, hipStream_t s) {
    return dispatch(n, 4, S, u, hcell, nullptr, dt, zeta, tau_div, tau_cont, s);
}

hipError_t launch_wall_load(int n, const SplitGeo& S, const double* mu_face, const double* tfac, int pen, double* y,
                            hipStream_t s) {
    if (S.gw == nullptr) return hipSuccess;
    return dispatch(n, 5, S, mu_face, tfac, nullptr, (double)pen, 0.0, y, nullptr, s);
}

}  // namespace sipg
