// Matrix-free SIPG operator application (viscous and Poisson) for gfx950.
//
// One workgroup handles CPB cells; each cell gets n*n threads, thread (i1, i2)
// owning the line of nodes (i1, i2, 0..n-1) along xi_3.  Everything a cell
// needs is computed by its own threads ("cell-centric"): the cell integral
// and all six face integrals for the cell's own test functions.  A face is
// therefore evaluated once from each side, but every output entry is written
// exactly once, with no atomics and no second pass over the output.  The
// neighbour's trace on a shared face is interpolated from the neighbour's
// nodal values, which the XCD-aware block order keeps in the L2.
//
// Sum factorisation (Sec. 5.3): with nodes at the Gauss points, values at
// quadrature points are the nodal values; reference derivatives are 1D
// contractions with D[q][j] = l_j'(g_q) along one axis.  Derivatives along
// xi_3 stay in registers; along xi_1 and xi_2 they go through LDS.
//
// Forms (Sec. 4.1), per quadrature point, written for the test functions of
// the cell that owns the thread (outward unit normal n, [u] = u_own - u_nbr):
//   cell      viscous: sigma = 2 mu eps(u) JxW, mass alpha u JxW
//             poisson: sigma = grad u JxW,      mass alpha u JxW
//   face      viscous: a = -2 {{mu eps(u)}} n + tau([u] + n([u].n)),
//                      B = -mu sym([u] (x) n)
//             poisson: a = -{{grad u}}.n + tau [u],  B = -[u] n / 2
//   and the test integration y_i += sum ds (phi_i a + grad phi_i : B).
// Dirichlet faces use the mirror state u_nbr = -u_own, grad u_nbr = grad u_own;
// Neumann faces contribute nothing.

#include "device_common.h"

namespace sipg {

template <int N, int C, bool DBL>
struct Shape {
    // cells per workgroup: about 64-256 threads, LDS well under 64 KB
    static constexpr int CPB = N == 2 ? 16 : N == 3 ? 7 : N == 4 ? 4 : N == 5 ? 5 : (DBL && C == 3 ? 3 : 7);
    static constexpr int THREADS = CPB * N * N;
};

template <int N, int C, typename T, bool CURVED, int MODE>
__global__ void __launch_bounds__((Shape<N, C, sizeof(T) == 8>::THREADS))
    k_apply(const OpData<T> op, const ApplyIO<T> io) {
    constexpr int NN = N * N, NNN = N * N * N;
    constexpr int CPB = Shape<N, C, sizeof(T) == 8>::CPB;

    if (io.skip != nullptr && *io.skip) return;  // uniform over the grid

    __shared__ T s_u[CPB][C * NNN];      // the cell's nodal values
    __shared__ T s_w[CPB][2 * C * NNN];  // work space of the cell and face passes
    __shared__ T s_geo[CPB][2][8][3];    // own / neighbour trilinear coefficients

    const int lc = threadIdx.x / NN;
    const int t = threadIdx.x - lc * NN;
    const int i1 = t % N, i2 = t / N;
    const int e = xcd_block(blockIdx.x, gridDim.x) * CPB + lc;
    const bool active = e < op.ncell;
    const int ec = active ? e : 0;
    const int ex = ec % op.nx, ey = (ec / op.nx) % op.ny, ez = ec / (op.nx * op.ny);
    const auto& tb = op.tab;
    const int parts = io.parts;

    // ------------------------------------------------------------ load
    const T* xe = io.x + (size_t)ec * (C * NNN);
    T ucol[C][N];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            ucol[c][j] = active ? xe[(c * N + j) * NN + t] : T(0);
            s_u[lc][c * NNN + j * NN + t] = ucol[c][j];
        }
    if constexpr (CURVED) {
        if (t < 3) {
            T g[8];
            trilinear_coeffs(op.verts, op.nx, op.ny, ex, ey, ez, t, g);
#pragma unroll
            for (int k = 0; k < 8; ++k) s_geo[lc][0][k][t] = g[k];
        }
    }
    __syncthreads();

    T y[C][N];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int j = 0; j < N; ++j) y[c][j] = T(0);

    // ------------------------------------------------------------ cell
    if (parts & SIPG_PART_CELL) {
        T f3[C][N];
#pragma unroll
        for (int q3 = 0; q3 < N; ++q3) {
            T gr[C][3];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                T g1 = 0, g2 = 0, g3 = 0;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    g1 += tb.D[i1][j] * s_u[lc][c * NNN + q3 * NN + i2 * N + j];
                    g2 += tb.D[i2][j] * s_u[lc][c * NNN + q3 * NN + j * N + i1];
                    g3 += tb.D[q3][j] * ucol[c][j];
                }
                gr[c][0] = g1; gr[c][1] = g2; gr[c][2] = g3;
            }
            T Ji[3][3], JxW;
            if constexpr (CURVED) {
                T det;
                jacobian_inverse(s_geo[lc][0], tb.x[i1], tb.x[i2], tb.x[q3], Ji, det);
                JxW = det * (tb.w[i1] * tb.w[i2] * tb.w[q3]);
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) Ji[a][b] = a == b ? T(1) / op.h[a] : T(0);
                JxW = op.h[0] * op.h[1] * op.h[2] * (tb.w[i1] * tb.w[i2] * tb.w[q3]);
            }
            // physical gradient G[c][i] = sum_d gr[c][d] Ji[d][i]
            T G[C][3];
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    G[c][i] = gr[c][0] * Ji[0][i] + gr[c][1] * Ji[1][i] + gr[c][2] * Ji[2][i];
            T S[C][3];
            if constexpr (C == 3) {
                const T mu = active ? op.mu_cell[(size_t)ec * NNN + q3 * NN + t] : T(0);
                const T f = mu * JxW;  // 2 mu eps = mu (G + G^T)
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int i = 0; i < 3; ++i) S[c][i] = f * (G[c][i] + G[i][c]);
            } else {
#pragma unroll
                for (int i = 0; i < 3; ++i) S[0][i] = JxW * G[0][i];
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                T Bh[3];
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    Bh[d] = Ji[d][0] * S[c][0] + Ji[d][1] * S[c][1] + Ji[d][2] * S[c][2];
                s_w[lc][(2 * c) * NNN + q3 * NN + t] = Bh[0];
                s_w[lc][(2 * c + 1) * NNN + q3 * NN + t] = Bh[1];
                f3[c][q3] = Bh[2];
                y[c][q3] = op.alpha * JxW * ucol[c][q3];
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int i3 = 0; i3 < N; ++i3) {
                T acc = y[c][i3];
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    acc += tb.D[q][i1] * s_w[lc][(2 * c) * NNN + i3 * NN + i2 * N + q];
                    acc += tb.D[q][i2] * s_w[lc][(2 * c + 1) * NNN + i3 * NN + q * N + i1];
                    acc += tb.D[q][i3] * f3[c][q];
                }
                y[c][i3] = acc;
            }
        __syncthreads();
    }

    // ------------------------------------------------------------ faces
    if (parts & (SIPG_PART_INTERIOR | SIPG_PART_BOUNDARY)) {
        T* FO = &s_w[lc][0];          // own trace values      [C][NN]
        T* FN = &s_w[lc][C * NN];     // neighbour trace values [C][NN]
        T* VV = &s_w[lc][2 * C * NN]; // value coefficients     [C][NN]
        T* VN = &s_w[lc][3 * C * NN]; // normal coefficients    [C][NN]
#pragma unroll
        for (int d = 0; d < 3; ++d) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                const int pos = d == 0 ? ex : d == 1 ? ey : ez;
                const int lim = d == 0 ? op.nx : d == 1 ? op.ny : op.nz;
                const bool has_nb = s == 1 ? pos + 1 < lim : pos > 0;
                const int en = ec + (s == 1 ? 1 : -1) * (d == 0 ? 1 : d == 1 ? op.nx : op.nx * op.ny);
                const bool dir = !has_nb && op.bc[2 * d + s] == 0;
                const bool live = active && (has_nb ? (parts & SIPG_PART_INTERIOR) != 0
                                                    : (dir && (parts & SIPG_PART_BOUNDARY) != 0));
                int fid;
                if (d == 0) fid = (ez * op.ny + ey) * (op.nx + 1) + ex + s;
                else if (d == 1) fid = op.nfx + (ez * (op.ny + 1) + ey + s) * op.nx + ex;
                else fid = op.nfx + op.nfy + ((ez + s) * op.ny + ey) * op.nx + ex;

                // traces at face point (a, b) = (i1, i2): value and d/dxi_d
                T uo[C], uno[C], un[C], unn[C];
                const T* xn = io.x + (size_t)(has_nb ? en : ec) * (C * NNN);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    T v0 = 0, v1 = 0, w0 = 0, w1 = 0;
#pragma unroll
                    for (int j = 0; j < N; ++j) {
                        T own;
                        if (d == 2) own = ucol[c][j];
                        else if (d == 0) own = s_u[lc][c * NNN + i2 * NN + i1 * N + j];
                        else own = s_u[lc][c * NNN + i2 * NN + j * N + i1];
                        v0 += tb.S[s][j] * own;
                        v1 += tb.G[s][j] * own;
                        if (live && has_nb) {
                            T nb;
                            if (d == 2) nb = xn[(c * N + j) * NN + i2 * N + i1];
                            else if (d == 0) nb = xn[(c * N + i2) * NN + i1 * N + j];
                            else nb = xn[(c * N + i2) * NN + j * N + i1];
                            w0 += tb.S[1 - s][j] * nb;
                            w1 += tb.G[1 - s][j] * nb;
                        }
                    }
                    uo[c] = v0; uno[c] = v1; un[c] = w0; unn[c] = w1;
                    FO[c * NN + t] = v0;
                    FN[c * NN + t] = w0;
                }
                if constexpr (CURVED) {
                    if (t < 3 && has_nb && active) {
                        const int nex = en % op.nx, ney = (en / op.nx) % op.ny, nez = en / (op.nx * op.ny);
                        T g[8];
                        trilinear_coeffs(op.verts, op.nx, op.ny, nex, ney, nez, t, g);
#pragma unroll
                        for (int k = 0; k < 8; ++k) s_geo[lc][1][k][t] = g[k];
                    }
                }
                __syncthreads();

                // reference gradients (order xi_1, xi_2, xi_3)
                T gro[C][3], grn[C][3];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    T ta = 0, tbv = 0, na = 0, nbv = 0;
#pragma unroll
                    for (int j = 0; j < N; ++j) {
                        ta += tb.D[i1][j] * FO[c * NN + i2 * N + j];
                        tbv += tb.D[i2][j] * FO[c * NN + j * N + i1];
                        na += tb.D[i1][j] * FN[c * NN + i2 * N + j];
                        nbv += tb.D[i2][j] * FN[c * NN + j * N + i1];
                    }
                    gro[c][t1] = ta; gro[c][t2] = tbv; gro[c][d] = uno[c];
                    grn[c][t1] = na; grn[c][t2] = nbv; grn[c][d] = unn[c];
                }
                // geometry on the face
                T xi[3];
                xi[t1] = tb.x[i1]; xi[t2] = tb.x[i2]; xi[d] = T(s);
                T Jo[3][3], Jn[3][3], nrm[3], ds;
                const T sgn = s == 1 ? T(1) : T(-1);
                if constexpr (CURVED) {
                    T deto, detn;
                    jacobian_inverse(s_geo[lc][0], xi[0], xi[1], xi[2], Jo, deto);
                    T xin[3] = {xi[0], xi[1], xi[2]};
                    xin[d] = T(1 - s);
                    if (has_nb) jacobian_inverse(s_geo[lc][1], xin[0], xin[1], xin[2], Jn, detn);
                    else {
#pragma unroll
                        for (int a = 0; a < 3; ++a)
#pragma unroll
                            for (int b = 0; b < 3; ++b) Jn[a][b] = Jo[a][b];
                    }
                    const T v0 = Jo[d][0], v1 = Jo[d][1], v2 = Jo[d][2];
                    const T nv = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
                    nrm[0] = sgn * v0 / nv; nrm[1] = sgn * v1 / nv; nrm[2] = sgn * v2 / nv;
                    ds = deto * nv * (tb.w[i1] * tb.w[i2]);
                } else {
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) {
                            Jo[a][b] = a == b ? T(1) / op.h[a] : T(0);
                            Jn[a][b] = Jo[a][b];
                        }
                    nrm[0] = nrm[1] = nrm[2] = T(0);
                    nrm[d] = sgn;
                    ds = op.h[t1] * op.h[t2] * (tb.w[i1] * tb.w[i2]);
                }
                T Go[C][3], Gn[C][3];
#pragma unroll
                for (int c = 0; c < C; ++c)
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        Go[c][i] = gro[c][0] * Jo[0][i] + gro[c][1] * Jo[1][i] + gro[c][2] * Jo[2][i];
                        Gn[c][i] = grn[c][0] * Jn[0][i] + grn[c][1] * Jn[1][i] + grn[c][2] * Jn[2][i];
                    }
                if (!has_nb) {  // mirror principle, Dirichlet: u+ = -u-, grad u+ = grad u-
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        un[c] = -uo[c];
#pragma unroll
                        for (int i = 0; i < 3; ++i) Gn[c][i] = Go[c][i];
                    }
                }
                const T mu = (C == 3 && live) ? op.mu_face[(size_t)fid * NN + t] : T(1);
                const T tau = live ? op.tfac[fid] * mu : T(0);
                T av[C], Bh[C][3];
                T ju[C];
#pragma unroll
                for (int c = 0; c < C; ++c) ju[c] = uo[c] - un[c];
                if constexpr (C == 3) {
                    const T jn = ju[0] * nrm[0] + ju[1] * nrm[1] + ju[2] * nrm[2];
                    T B[3][3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        T en_ = 0;  // (eps(u-) + eps(u+)) n, times 1/2 twice folded below
#pragma unroll
                        for (int i = 0; i < 3; ++i)
                            en_ += (Go[c][i] + Go[i][c] + Gn[c][i] + Gn[i][c]) * nrm[i];
                        // -2 {{mu eps}} n = -2 * mu/2 * (eps- + eps+) n = -mu/2 * (G + G^T)- + ...) n
                        av[c] = -T(0.5) * mu * en_ + tau * (ju[c] + nrm[c] * jn);
#pragma unroll
                        for (int i = 0; i < 3; ++i) B[c][i] = -T(0.5) * mu * (ju[c] * nrm[i] + nrm[c] * ju[i]);
                    }
#pragma unroll
                    for (int c = 0; c < 3; ++c)
#pragma unroll
                        for (int dd = 0; dd < 3; ++dd)
                            Bh[c][dd] = ds * (Jo[dd][0] * B[c][0] + Jo[dd][1] * B[c][1] + Jo[dd][2] * B[c][2]);
                } else {
                    const T gn = (Go[0][0] + Gn[0][0]) * nrm[0] + (Go[0][1] + Gn[0][1]) * nrm[1] +
                                 (Go[0][2] + Gn[0][2]) * nrm[2];
                    av[0] = -T(0.5) * gn + tau * ju[0];
                    T B[3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) B[i] = -T(0.5) * ju[0] * nrm[i];
#pragma unroll
                    for (int dd = 0; dd < 3; ++dd)
                        Bh[0][dd] = ds * (Jo[dd][0] * B[0] + Jo[dd][1] * B[1] + Jo[dd][2] * B[2]);
                }
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    av[c] = live ? av[c] * ds : T(0);
#pragma unroll
                    for (int dd = 0; dd < 3; ++dd) Bh[c][dd] = live ? Bh[c][dd] : T(0);
                }
                __syncthreads();  // all reads of FO/FN done
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    FO[c * NN + t] = Bh[c][t1];
                    FN[c * NN + t] = Bh[c][t2];
                }
                __syncthreads();
                T vv[C], vn[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    T acc = av[c];
#pragma unroll
                    for (int q = 0; q < N; ++q) {
                        acc += tb.D[q][i1] * FO[c * NN + i2 * N + q];
                        acc += tb.D[q][i2] * FN[c * NN + q * N + i1];
                    }
                    vv[c] = acc;
                    vn[c] = Bh[c][d];
                }
                if (d == 2) {
#pragma unroll
                    for (int c = 0; c < C; ++c)
#pragma unroll
                        for (int i3 = 0; i3 < N; ++i3) y[c][i3] += tb.S[s][i3] * vv[c] + tb.G[s][i3] * vn[c];
                } else {
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        VV[c * NN + t] = vv[c];
                        VN[c * NN + t] = vn[c];
                    }
                    __syncthreads();
#pragma unroll
                    for (int c = 0; c < C; ++c)
#pragma unroll
                        for (int i3 = 0; i3 < N; ++i3) {
                            // node (i1, i2, i3): d == 0 -> face point (i2, i3), normal index i1
                            //                    d == 1 -> face point (i1, i3), normal index i2
                            const int fp = d == 0 ? i3 * N + i2 : i3 * N + i1;
                            const int ni = d == 0 ? i1 : i2;
                            y[c][i3] += tb.S[s][ni] * VV[c * NN + fp] + tb.G[s][ni] * VN[c * NN + fp];
                        }
                }
                __syncthreads();
            }
        }
    }

    // ------------------------------------------------------------ store
    if (!active) return;
    const size_t base = (size_t)ec * (C * NNN);
    if constexpr (MODE == MODE_APPLY) {
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int j = 0; j < N; ++j) io.y[base + (c * N + j) * NN + t] = y[c][j];
    } else {
        const T c1 = T(io.coef[0]), c2 = T(io.coef[1]);
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const size_t idx = base + (c * N + j) * NN + t;
                const T dn = c1 * io.d[idx] + c2 * io.dinv[idx] * (io.r[idx] - y[c][j]);
                io.d[idx] = dn;
                io.y[idx] = ucol[c][j] + dn;
            }
    }
}

template <int N, int C, typename T, bool CURVED>
static hipError_t launch_nc(const OpData<T>& op, const ApplyIO<T>& io, int mode, hipStream_t s) {
    using Sh = Shape<N, C, sizeof(T) == 8>;
    const int blocks = (op.ncell + Sh::CPB - 1) / Sh::CPB;
    if (mode == MODE_APPLY)
        hipLaunchKernelGGL((k_apply<N, C, T, CURVED, MODE_APPLY>), dim3(blocks), dim3(Sh::THREADS), 0, s, op, io);
    else
        hipLaunchKernelGGL((k_apply<N, C, T, CURVED, MODE_CHEB>), dim3(blocks), dim3(Sh::THREADS), 0, s, op, io);
    return hipGetLastError();
}

template <int C, typename T, bool CURVED>
static hipError_t launch_c(int n, const OpData<T>& op, const ApplyIO<T>& io, int mode, hipStream_t s) {
    switch (n) {
        case 2: return launch_nc<2, C, T, CURVED>(op, io, mode, s);
        case 3: return launch_nc<3, C, T, CURVED>(op, io, mode, s);
        case 4: return launch_nc<4, C, T, CURVED>(op, io, mode, s);
        case 5: return launch_nc<5, C, T, CURVED>(op, io, mode, s);
        case 6: return launch_nc<6, C, T, CURVED>(op, io, mode, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_apply(int n, int C, bool curved, const OpData<T>& op, const ApplyIO<T>& io, int mode,
                        hipStream_t s) {
    if (op.ncell <= 0) return hipSuccess;
    if (C == 3) return curved ? launch_c<3, T, true>(n, op, io, mode, s) : launch_c<3, T, false>(n, op, io, mode, s);
    return curved ? launch_c<1, T, true>(n, op, io, mode, s) : launch_c<1, T, false>(n, op, io, mode, s);
}

template hipError_t launch_apply<double>(int, int, bool, const OpData<double>&, const ApplyIO<double>&, int,
                                         hipStream_t);
template hipError_t launch_apply<float>(int, int, bool, const OpData<float>&, const ApplyIO<float>&, int,
                                        hipStream_t);

}  // namespace sipg
