// Continuous levels of the cph-multigrid preconditioner (Sec. 5.3, paragraph
// on preconditioning the viscous terms: the DG space is first transferred to
// continuous elements of the same degree, then the degree and the mesh are
// coarsened, and the coarsest level is solved directly).
//
// A continuous level of degree j on a mesh of nx*ny*nz cells is nodal at the
// Gauss-Lobatto points of every cell: (j nx + 1)(j ny + 1)(j nz + 1) nodes per
// component, node index (gz My + gy) Mx + gx with g = j * cell + local index,
// component-major.  Its operator is the Galerkin restriction G^T A G of the
// DG operator of the same degree and mesh (the "carrier" plan), where G
// evaluates a cell's Lobatto interpolant at its Gauss nodes; for continuous
// functions every interior-face term vanishes, so the carrier is applied with
// its cell and boundary parts only:
//   y = assemble(local G^T (A_cell+boundary (G x))).
// Kernels here: the per-cell sum factorisations of G and G^T (three 1D
// sweeps in LDS), the node-wise sum of the cells' local contributions (a
// fixed order over the up to 8 cells of a node: deterministic, no atomics),
// 1D sparse transfers along one axis (prolongation between continuous levels
// is a tensor product of 1D matrices), the diagonal of G^T A G from the
// local Lobatto basis functions, and the coarsest level's direct solve: its
// dense matrix from the element matrices of the degree-1 carrier, in-place
// Gauss-Jordan inversion, and a dense matrix-vector product per V-cycle.
// Every kernel used inside a solve returns at once while *skip != 0.

#include <cstring>
#include <type_traits>

#include "device_common.h"

namespace sipg {

namespace {

constexpr int kThreads = 256;

inline int grid_for(long long work) {
    const long long b = (work + kThreads - 1) / kThreads;
    return (int)(b < 1 ? 1 : b > 65535 ? 65535 : b);
}

#define GRID_STRIDE(i, n) for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < (n); \
                               i += (long long)gridDim.x * blockDim.x)

constexpr int kCellThreads = 128;
constexpr int kCellVals = 3 * kMaxN * kMaxN * kMaxN;

// One cell per block (grid-stride over cells), n = j + 1 values per
// direction on both sides.  GATHER: in = continuous vector, out = the DG
// values at the Gauss nodes (ADD: added); else in = DG values, out = the
// cell's local Lobatto contributions G_e^T in (same DG layout; in == out is
// allowed: the cell is read completely before it is written).
template <typename T, bool GATHER, bool ADD>
__global__ void __launch_bounds__(kCellThreads) k_cg_cell(CgGeo g, const CgL<T> tab, const T* in, T* out,
                                                         const int* skip) {
    if (skip != nullptr && *skip) return;
    __shared__ T A[kCellVals], B[kCellVals];
    const int n = g.j + 1, C = g.C, j = g.j;
    const int n3 = n * n * n, nin = C * n3;
    const long long nv = (long long)g.Mx * g.My * g.Mz;
    const int ncell = g.nx * g.ny * g.nz;
    // W(b, a): gather Gauss b <- Lobatto a: L[b][a]; transposed: L[a][b]
    auto W = [&](int b, int a) -> T { return GATHER ? tab.L[b][a] : tab.L[a][b]; };
    for (int e = blockIdx.x; e < ncell; e += gridDim.x) {
        __syncthreads();
        const int ex = e % g.nx, ey = (e / g.nx) % g.ny, ez = e / (g.nx * g.ny);
        for (int i = threadIdx.x; i < nin; i += kCellThreads) {
            if constexpr (GATHER) {
                const int c = i / n3, a = i - c * n3;
                const int a1 = a % n, a2 = (a / n) % n, a3 = a / (n * n);
                A[i] = in[c * nv + ((long long)(ez * j + a3) * g.My + ey * j + a2) * g.Mx + ex * j + a1];
            } else {
                A[i] = in[(long long)e * nin + i];
            }
        }
        __syncthreads();
        // sweep along the first index: B[c][a3][a2][b1] = sum_a1 W(b1, a1) A[c][a3][a2][a1]
        for (int k = threadIdx.x; k < nin; k += kCellThreads) {
            const int b1 = k % n, rest = k / n;
            const T* src = A + rest * n;
            T acc = 0;
            for (int a = 0; a < n; ++a) acc += W(b1, a) * src[a];
            B[k] = acc;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nin; k += kCellThreads) {
            const int b1 = k % n, b2 = (k / n) % n, rest = k / (n * n);
            const T* src = B + rest * n * n + b1;
            T acc = 0;
            for (int a = 0; a < n; ++a) acc += W(b2, a) * src[a * n];
            A[k] = acc;
        }
        __syncthreads();
        const int nn = n * n;
        for (int k = threadIdx.x; k < nin; k += kCellThreads) {
            const int b12 = k % nn, b3 = (k / nn) % n, c = k / (nn * n);
            const T* src = A + c * n3 + b12;
            T acc = 0;
            for (int a = 0; a < n; ++a) acc += W(b3, a) * src[a * nn];
            if (ADD) out[(long long)e * nin + k] += acc;
            else out[(long long)e * nin + k] = acc;
        }
    }
}

// The same for a degree known at compile time (n = N per direction): the
// 1D table in LDS, the index arithmetic by constants and the short loops
// unrolled; the sums are the generic kernel's, in the same order.
template <typename T, bool GATHER, bool ADD, int N>
__global__ void __launch_bounds__(kCellThreads) k_cg_cell_n(CgGeo g, const CgL<T> tab, const T* in, T* out,
                                                           const int* skip) {
    if (skip != nullptr && *skip) return;
    constexpr int n = N, j = N - 1, nn = N * N, n3 = N * N * N;
    __shared__ T A[kCellVals], B[kCellVals];
    __shared__ T Wt[N][N];  // Wt[b][a] = W(b, a)
    const int C = g.C, nin = C * n3;
    const long long nv = (long long)g.Mx * g.My * g.Mz;
    const int ncell = g.nx * g.ny * g.nz;
    if ((int)threadIdx.x < nn) {
        const int b = threadIdx.x / n, a = threadIdx.x - b * n;
        Wt[b][a] = GATHER ? tab.L[b][a] : tab.L[a][b];
    }
    for (int e = blockIdx.x; e < ncell; e += gridDim.x) {
        __syncthreads();
        const int ex = e % g.nx, ey = (e / g.nx) % g.ny, ez = e / (g.nx * g.ny);
        for (int i = threadIdx.x; i < nin; i += kCellThreads) {
            if constexpr (GATHER) {
                const int c = i / n3, a = i - c * n3;
                const int a1 = a % n, a2 = (a / n) % n, a3 = a / nn;
                A[i] = in[c * nv + ((long long)(ez * j + a3) * g.My + ey * j + a2) * g.Mx + ex * j + a1];
            } else {
                A[i] = in[(long long)e * nin + i];
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nin; k += kCellThreads) {
            const int b1 = k % n, rest = k / n;
            const T* src = A + rest * n;
            T acc = 0;
#pragma unroll
            for (int a = 0; a < n; ++a) acc += Wt[b1][a] * src[a];
            B[k] = acc;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nin; k += kCellThreads) {
            const int b1 = k % n, b2 = (k / n) % n, rest = k / nn;
            const T* src = B + rest * nn + b1;
            T acc = 0;
#pragma unroll
            for (int a = 0; a < n; ++a) acc += Wt[b2][a] * src[a * n];
            A[k] = acc;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nin; k += kCellThreads) {
            const int b12 = k % nn, b3 = (k / nn) % n, c = k / n3;
            const T* src = A + c * n3 + b12;
            T acc = 0;
#pragma unroll
            for (int a = 0; a < n; ++a) acc += Wt[b3][a] * src[a * nn];
            if (ADD) out[(long long)e * nin + k] += acc;
            else out[(long long)e * nin + k] = acc;
        }
    }
}

template <typename T, bool GATHER, bool ADD>
void launch_cell_n(const CgGeo& g, const CgL<T>& tab, const T* in, T* out, const int* skip, dim3 grid,
                   hipStream_t s) {
    switch (g.j + 1) {
        case 2: hipLaunchKernelGGL((k_cg_cell_n<T, GATHER, ADD, 2>), grid, dim3(kCellThreads), 0, s, g, tab, in, out, skip); break;
        case 3: hipLaunchKernelGGL((k_cg_cell_n<T, GATHER, ADD, 3>), grid, dim3(kCellThreads), 0, s, g, tab, in, out, skip); break;
        case 4: hipLaunchKernelGGL((k_cg_cell_n<T, GATHER, ADD, 4>), grid, dim3(kCellThreads), 0, s, g, tab, in, out, skip); break;
        case 5: hipLaunchKernelGGL((k_cg_cell_n<T, GATHER, ADD, 5>), grid, dim3(kCellThreads), 0, s, g, tab, in, out, skip); break;
        case 6: hipLaunchKernelGGL((k_cg_cell_n<T, GATHER, ADD, 6>), grid, dim3(kCellThreads), 0, s, g, tab, in, out, skip); break;
        default: hipLaunchKernelGGL((k_cg_cell<T, GATHER, ADD>), grid, dim3(kCellThreads), 0, s, g, tab, in, out, skip); break;
    }
}

// The cells of a continuous node along one direction: node g of a line with
// `cells` cells of degree j lies in cell g / j (local index g % j) and, when
// g % j == 0 and 0 < g < j * cells, also in cell g / j - 1 (local index j).
__device__ inline int node_cells(int g, int j, int cells, int e[2], int a[2]) {
    int m = 0;
    if (g % j == 0 && g > 0) { e[m] = g / j - 1; a[m] = j; ++m; }
    if (g / j < cells) { e[m] = g / j; a[m] = g % j; ++m; }
    return m;
}

// out[node] = sum over the node's cells (in increasing cell order) of their
// local contributions (DG layout), for every component; with the sum t = (A
// z) at the node, mode RESID writes out = r - t and mode CHEB the Chebyshev
// step d <- c1 d + c2 dinv (r - t), out = z + d; mode CHEB_ACC the same step
// added to out (out += z + d: a V-cycle's last post-smoothing step).
enum AssembleMode { ASM_SUM = 0, ASM_RESID = 1, ASM_CHEB = 2, ASM_CHEB_ACC = 3 };

template <typename T>
struct AsmIO {
    const T* r;
    const T* z;
    T* d;
    const T* dinv;
    const double* coef;
};

template <typename T, int MODE>
__global__ void k_cg_assemble(CgGeo g, const T* local, T* out, const AsmIO<T> io, const int* skip) {
    if (skip != nullptr && *skip) return;
    const int n = g.j + 1, n3 = n * n * n;
    const long long nv = (long long)g.Mx * g.My * g.Mz, total = nv * g.C;
    GRID_STRIDE(idx, total) {
        const int c = (int)(idx / nv);
        const long long v = idx - c * nv;
        const int gx = (int)(v % g.Mx), gy = (int)((v / g.Mx) % g.My), gz = (int)(v / ((long long)g.Mx * g.My));
        int ex[2], ax[2], ey[2], ay[2], ez[2], az[2];
        const int mx = node_cells(gx, g.j, g.nx, ex, ax);
        const int my = node_cells(gy, g.j, g.ny, ey, ay);
        const int mz = node_cells(gz, g.j, g.nz, ez, az);
        T acc = 0;
        for (int kz = 0; kz < mz; ++kz)
            for (int ky = 0; ky < my; ++ky)
                for (int kx = 0; kx < mx; ++kx) {
                    const long long e = ((long long)ez[kz] * g.ny + ey[ky]) * g.nx + ex[kx];
                    acc += local[(e * g.C + c) * n3 + (az[kz] * n + ay[ky]) * n + ax[kx]];
                }
        if constexpr (MODE == ASM_SUM) {
            out[idx] = acc;
        } else if constexpr (MODE == ASM_RESID) {
            out[idx] = io.r[idx] - acc;
        } else {
            const T dn = T(io.coef[0]) * io.d[idx] + T(io.coef[1]) * io.dinv[idx] * (io.r[idx] - acc);
            io.d[idx] = dn;
            if constexpr (MODE == ASM_CHEB_ACC) out[idx] = out[idx] + (io.z[idx] + dn);
            else out[idx] = io.z[idx] + dn;
        }
    }
}

// The same sum for a level of degree J known at compile time, one thread per
// node of a (gz, component) plane: grid (ceil(Mx My / 256), Mz C).  Along
// each axis a node has a lower candidate cell (g / J - 1, local index J; it
// exists when g is a positive multiple of J) and an upper one (g / J, local
// index g % J; it exists when g / J < cells).  All eight candidate loads are
// issued together, a missing candidate reading the existing one along its
// axis (in bounds, the same cache line), and the sum takes the existing ones
// in the generic kernel's order (lower before upper, z, then y, then x), so
// the two kernels agree bit for bit.  The generic kernel's run-time trip
// counts issued the up to eight loads one after another, and its 64-bit
// index divisions cost more than the sums.
template <typename T, int MODE, int J>
__global__ void __launch_bounds__(kThreads) k_cg_assemble_j(CgGeo g, const T* local, T* out, const AsmIO<T> io,
                                                            const int* skip) {
    if (skip != nullptr && *skip) return;
    constexpr int n = J + 1, n3 = n * n * n;
    const int plane = g.Mx * g.My;
    const int xy = blockIdx.x * kThreads + threadIdx.x;
    if (xy >= plane) return;
    const int c = blockIdx.y / g.Mz, gz = blockIdx.y - c * g.Mz;  // uniform over the block
    const int gy = xy / g.Mx, gx = xy - gy * g.Mx;
    int ex[2], ax[2], ey[2], ay[2], ez[2], az[2];
    bool vx[2], vy[2], vz[2];
    auto cand = [](int gg, int cells, int e[2], int a[2], bool v[2]) {
        const int q = gg / J, r = gg - q * J;
        v[0] = r == 0 && gg > 0;
        v[1] = q < cells;
        e[1] = v[1] ? q : q - 1;   // the node at the far end has only the lower cell
        a[1] = v[1] ? r : J;
        e[0] = v[0] ? q - 1 : e[1];
        a[0] = v[0] ? J : a[1];
    };
    cand(gx, g.nx, ex, ax, vx);
    cand(gy, g.ny, ey, ay, vy);
    cand(gz, g.nz, ez, az, vz);
    T val[2][2][2];
#pragma unroll
    for (int kz = 0; kz < 2; ++kz)
#pragma unroll
        for (int ky = 0; ky < 2; ++ky)
#pragma unroll
            for (int kx = 0; kx < 2; ++kx) {
                const long long e = ((long long)ez[kz] * g.ny + ey[ky]) * g.nx + ex[kx];
                val[kz][ky][kx] = local[(e * g.C + c) * n3 + (az[kz] * n + ay[ky]) * n + ax[kx]];
            }
    T acc = 0;
#pragma unroll
    for (int kz = 0; kz < 2; ++kz)
#pragma unroll
        for (int ky = 0; ky < 2; ++ky)
#pragma unroll
            for (int kx = 0; kx < 2; ++kx) acc = (vz[kz] && vy[ky] && vx[kx]) ? acc + val[kz][ky][kx] : acc;
    const long long idx = (long long)c * plane * g.Mz + (long long)gz * plane + xy;
    if constexpr (MODE == ASM_SUM) {
        out[idx] = acc;
    } else if constexpr (MODE == ASM_RESID) {
        out[idx] = io.r[idx] - acc;
    } else {
        const T dn = T(io.coef[0]) * io.d[idx] + T(io.coef[1]) * io.dinv[idx] * (io.r[idx] - acc);
        io.d[idx] = dn;
        if constexpr (MODE == ASM_CHEB_ACC) out[idx] = out[idx] + (io.z[idx] + dn);
        else out[idx] = io.z[idx] + dn;
    }
}

// out = M in along one axis of a (C, N2, N1, N0) array: M is a 1D sparse
// matrix (CSR, rows = the axis length of out); ADD: out += M in.
template <typename T, bool ADD>
__global__ void k_axis(AxisMat<T> M, int axis, int C, int n0, int n1, int n2, const T* in, T* out, const int* skip) {
    if (skip != nullptr && *skip) return;
    int o0 = n0, o1 = n1, o2 = n2;  // output extents
    if (axis == 0) o0 = M.rows; else if (axis == 1) o1 = M.rows; else o2 = M.rows;
    const long long total = (long long)C * o0 * o1 * o2;
    GRID_STRIDE(idx, total) {
        const int i0 = (int)(idx % o0), i1 = (int)((idx / o0) % o1);
        const long long r = idx / ((long long)o0 * o1);
        const int i2 = (int)(r % o2), c = (int)(r / o2);
        const int row = axis == 0 ? i0 : axis == 1 ? i1 : i2;
        T acc = 0;
        for (int k = M.rp[row]; k < M.rp[row + 1]; ++k) {
            const int col = M.ci[k];
            const int j0 = axis == 0 ? col : i0, j1 = axis == 1 ? col : i1, j2 = axis == 2 ? col : i2;
            acc += M.v[k] * in[(((long long)c * n2 + j2) * n1 + j1) * n0 + j0];
        }
        if (ADD) out[idx] += acc;
        else out[idx] = acc;
    }
}

// The same with 32-bit indices on a 2D grid: x over the (i0, i1) plane of
// the output, y over (i2, c) (the generic kernel's 64-bit index divisions
// cost more than the few products of a row).
template <typename T, bool ADD>
__global__ void __launch_bounds__(kThreads) k_axis2(AxisMat<T> M, int axis, int n0, int n1, int n2, int o0, int o1,
                                                     int o2, const T* in, T* out, const int* skip) {
    if (skip != nullptr && *skip) return;
    const int plane = o0 * o1;
    const int xy = blockIdx.x * kThreads + threadIdx.x;
    if (xy >= plane) return;
    const int c = blockIdx.y / o2, i2 = blockIdx.y - c * o2;  // uniform over the block
    const int i1 = xy / o0, i0 = xy - i1 * o0;
    const int row = axis == 0 ? i0 : axis == 1 ? i1 : i2;
    T acc = 0;
    for (int k = M.rp[row]; k < M.rp[row + 1]; ++k) {
        const int col = M.ci[k];
        const int j0 = axis == 0 ? col : i0, j1 = axis == 1 ? col : i1, j2 = axis == 2 ? col : i2;
        acc += M.v[k] * in[(((long long)c * n2 + j2) * n1 + j1) * n0 + j0];
    }
    const long long idx = ((long long)c * o2 + i2) * plane + xy;
    if (ADD) out[idx] += acc;
    else out[idx] = acc;
}

// Chebyshev step of a continuous level: d <- c1 d + c2 dinv (r - t),
// zn = z + d (t = A z computed before).
template <typename T>
__global__ void k_cg_cheb(const T* z, T* zn, T* d, const T* r, const T* t, const T* dinv, const double* coef,
                          long long n, const int* skip) {
    if (skip != nullptr && *skip) return;
    const T c1 = T(coef[0]), c2 = T(coef[1]);
    GRID_STRIDE(i, n) {
        const T dn = c1 * d[i] + c2 * dinv[i] * (r[i] - t[i]);
        d[i] = dn;
        zn[i] = z[i] + dn;
    }
}

template <typename T>
__global__ void k_cg_sub(T* y, const T* r, const T* t, long long n, const int* skip) {
    if (skip != nullptr && *skip) return;
    GRID_STRIDE(i, n) y[i] = r[i] - t[i];
}

// Local diagonal of G^T A G: for every cell and local Lobatto function
// psi = l_a1(xi1) l_a2(xi2) l_a3(xi3) e_c, a_cell+boundary(psi, psi) with the
// Gauss rule of the carrier (all n^3 points: psi is not collocated):
//   viscous  sum_q JxW (alpha psi^2 + mu (|g|^2 + g_c^2))
//   poisson  sum_q JxW (alpha psi^2 + |g|^2)
//   penalty  sum_q JxW (alpha psi^2 + tau_div g_c^2)
// plus, on a Dirichlet face of the cell (only nodes on it have a trace;
// there psi = l_a_t1 l_a_t2 at the face point):
//   viscous  ds (-2 mu psi (g.n + n_c g_c) + 2 tau psi^2 (1 + n_c^2))
//   poisson  ds (-2 psi g.n + 2 tau psi^2)
//   penalty  ds tau_e psi^2 n_c^2
// written at the node's local position (DG layout); k_cg_assemble sums the
// cells.  A block holds CPB = 256 / n^3 cells (one thread per node): the
// geometry of every quadrature point (J^-1, JxW, the coefficient) is computed
// once into LDS, then the thread sums over the points for its node; likewise
// per Dirichlet face (each cell of the block checks its own faces).
constexpr int kDiagThreads = 256;
template <int C, int N>
__global__ void __launch_bounds__(kDiagThreads) k_cg_diag_local(const OpData<double> op, const CgDiagTab tab,
                                                                double* local) {
    constexpr int NN = N * N, NNN = NN * N, CPB = kDiagThreads / NNN, J = N - 1;
    __shared__ double sJ[CPB * NNN][9];
    __shared__ double sW[CPB * NNN], sM[CPB * NNN];
    __shared__ double sF[CPB][NN][14];  // face point: J^-1 (9), normal (3), ds, penalty coefficient
    __shared__ double sFm[CPB][NN];     // face point viscosity
    __shared__ double sLV[N][N], sLD[N][N], sLG[2][N];
    const auto& tb = op.tab;
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        sLV[i / N][i % N] = tab.LV[i / N][i % N];
        sLD[i / N][i % N] = tab.LD[i / N][i % N];
    }
    if ((int)threadIdx.x < 2 * N) sLG[threadIdx.x / N][threadIdx.x % N] = tab.LGs[threadIdx.x / N][threadIdx.x % N];
    const int lc = threadIdx.x / NNN, node = threadIdx.x % NNN;  // blockDim = CPB * NNN
    const int a[3] = {node % N, (node / N) % N, node / NN};
    for (long long e0 = (long long)blockIdx.x * CPB; e0 < op.ncell; e0 += (long long)gridDim.x * CPB) {
        const bool act = e0 + lc < op.ncell;
        const int e = act ? (int)(e0 + lc) : 0;  // inactive threads take cell 0: every access in bounds
        const int ex = e % op.nx, ey = (e / op.nx) % op.ny, ez = e / (op.nx * op.ny);
        double geo[8][3];
        cell_geo_full(op, e, geo);
        __syncthreads();  // the previous cells' readers are done
        {
            const int q1 = a[0], q2 = a[1], q3 = a[2];
            double Ji[3][3], det;
            jacobian_inverse<double>(geo, tb.x[q1], tb.x[q2], tb.x[q3], Ji, det);
            for (int u = 0; u < 3; ++u)
                for (int v = 0; v < 3; ++v) sJ[threadIdx.x][u * 3 + v] = Ji[u][v];
            sW[threadIdx.x] = det * tb.w[q1] * tb.w[q2] * tb.w[q3];
            sM[threadIdx.x] = C == 3 ? op.mu_cell[(size_t)e * NNN + node] : 1.0;
        }
        __syncthreads();
        const double(*cJ)[9] = sJ + lc * NNN;
        const double* cW = sW + lc * NNN;
        const double* cM = sM + lc * NNN;
        double acc[C];
        for (int c = 0; c < C; ++c) acc[c] = 0.0;
#pragma unroll 1
        for (int q = 0; q < NNN; ++q) {
            const int q1 = q % N, q2 = (q / N) % N, q3 = q / NN;
            const double v1 = sLV[q1][a[0]], v2 = sLV[q2][a[1]], v3 = sLV[q3][a[2]];
            const double psi = v1 * v2 * v3;
            const double gr[3] = {sLD[q1][a[0]] * v2 * v3, v1 * sLD[q2][a[1]] * v3, v1 * v2 * sLD[q3][a[2]]};
            double g[3];
            for (int k = 0; k < 3; ++k) g[k] = gr[0] * cJ[q][k] + gr[1] * cJ[q][3 + k] + gr[2] * cJ[q][6 + k];
            const double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
            for (int c = 0; c < C; ++c) {
                double v = op.alpha * psi * psi;
                if (C == 3 && op.pen) v += cM[q] * g[c] * g[c];
                else if (C == 3) v += cM[q] * (g2 + g[c] * g[c]);
                else v += g2;
                acc[c] += cW[q] * v;
            }
        }
        for (int d = 0; d < 3; ++d)
            for (int s = 0; s < 2; ++s) {
                const int pos = d == 0 ? ex : d == 1 ? ey : ez;
                const int lim = d == 0 ? op.nx : d == 1 ? op.ny : op.nz;
                const bool boundary = s == 1 ? pos + 1 == lim : pos == 0;
                const bool dface = act && boundary && op.bc[2 * d + s] == 0;  // per cell of the block
                const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                int fid;
                if (d == 0) fid = (ez * op.ny + ey) * (op.nx + 1) + ex + s;
                else if (d == 1) fid = op.nfx + (ez * (op.ny + 1) + ey + s) * op.nx + ex;
                else fid = op.nfx + op.nfy + ((ez + s) * op.ny + ey) * op.nx + ex;
                __syncthreads();  // the previous face's readers are done
                if (dface && node < NN) {
                    const int fp = node, qa = fp % N, qb = fp / N;
                    double xi[3];
                    xi[t1] = tb.x[qa];
                    xi[t2] = tb.x[qb];
                    xi[d] = (double)s;
                    double Ji[3][3], det;
                    jacobian_inverse<double>(geo, xi[0], xi[1], xi[2], Ji, det);
                    const double w0 = Ji[d][0], w1 = Ji[d][1], w2 = Ji[d][2];
                    const double nv = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
                    const double sg = s == 1 ? 1.0 : -1.0;
                    for (int a2 = 0; a2 < 3; ++a2)
                        for (int b = 0; b < 3; ++b) sF[lc][fp][a2 * 3 + b] = Ji[a2][b];
                    sF[lc][fp][9] = sg * w0 / nv; sF[lc][fp][10] = sg * w1 / nv; sF[lc][fp][11] = sg * w2 / nv;
                    sF[lc][fp][12] = det * nv * tb.w[qa] * tb.w[qb];
                    const double mu = (C == 3 && !op.pen) ? op.mu_face[(size_t)fid * NN + fp] : 1.0;
                    sFm[lc][fp] = mu;
                    sF[lc][fp][13] = (C == 3 && !op.pen) ? op.tfac[fid] * mu : op.tfac[fid];
                }
                __syncthreads();
                if (!dface || a[d] != (s == 1 ? J : 0)) continue;   // no trace on this face
#pragma unroll 1
                for (int fp = 0; fp < NN; ++fp) {
                    const int qa = fp % N, qb = fp / N;
                    const double va = sLV[qa][a[t1]], vb = sLV[qb][a[t2]];
                    const double psi = va * vb;
                    double gr[3];
                    gr[t1] = sLD[qa][a[t1]] * vb;
                    gr[t2] = va * sLD[qb][a[t2]];
                    gr[d] = sLG[s][a[d]] * psi;
                    const double* F = sF[lc][fp];
                    double g[3];
                    for (int k = 0; k < 3; ++k) g[k] = gr[0] * F[k] + gr[1] * F[3 + k] + gr[2] * F[6 + k];
                    const double nrm[3] = {F[9], F[10], F[11]};
                    const double ds = F[12], tau = F[13];
                    const double gn = g[0] * nrm[0] + g[1] * nrm[1] + g[2] * nrm[2];
                    if (C == 3 && op.pen) {
                        for (int c = 0; c < 3; ++c) acc[c] += ds * tau * psi * psi * nrm[c] * nrm[c];
                    } else if (C == 3) {
                        const double mu = sFm[lc][fp];
                        for (int c = 0; c < 3; ++c)
                            acc[c] += 2.0 * ds *
                                      (-mu * psi * (gn + nrm[c] * g[c]) + tau * psi * psi * (1.0 + nrm[c] * nrm[c]));
                    } else {
                        acc[0] += 2.0 * ds * (-psi * gn + tau * psi * psi);
                    }
                }
            }
        if (act)
            for (int c = 0; c < C; ++c) local[((size_t)e * C + c) * NNN + node] = acc[c];
    }
}

__global__ void k_cg_invert(const double* diag, double* dinv64, float* dinv32, long long n) {
    GRID_STRIDE(i, n) {
        const double v = 1.0 / diag[i];
        dinv64[i] = v;
        dinv32[i] = (float)v;
    }
}

// Coarsest level (degree 1): probe vector `col` = local DoF (c, Gauss node q)
// of every cell set to one, all else zero (DG_1 layout, 8 nodes per cell).
__global__ void k_cg_probe(double* v, int C, long long ncell, int col) {
    const long long total = ncell * C * 8;
    GRID_STRIDE(i, total) v[i] = (int)(i % (C * 8)) == col ? 1.0 : 0.0;
}

// Dense matrix of the coarsest continuous level from the carrier's element
// matrices K_e (column (c', q') of every cell's K_e = the carrier's cell and
// boundary parts applied to probe c' * 8 + q'): entry (I, J), I = (c, vertex
// vi), J = (c', vertex vj), sums over the cells holding both vertices
// G_e[q][vi] K_e[(c, q), (c', q')] G_e[q'][vj], G_e the trilinear vertex
// basis at the Gauss nodes.  Pure-Neumann Poisson (mean_zero): plus
// mean(diag) / n on every entry (added before the inversion).
__global__ void k_cg_coarse_matrix(CgGeo g, const double* probes, long long dgsize, const CgL<double> tab,
                                   double* A) {
    const long long nv = (long long)g.Mx * g.My * g.Mz, nc = nv * g.C;
    GRID_STRIDE(idx, nc * nc) {
        const long long I = idx / nc, J = idx - I * nc;
        const int cI = (int)(I / nv), cJ = (int)(J / nv);
        const long long vI = I - cI * nv, vJ = J - cJ * nv;
        const int ix = (int)(vI % g.Mx), iy = (int)((vI / g.Mx) % g.My), iz = (int)(vI / ((long long)g.Mx * g.My));
        const int jx = (int)(vJ % g.Mx), jy = (int)((vJ / g.Mx) % g.My), jz = (int)(vJ / ((long long)g.Mx * g.My));
        double acc = 0.0;
        if (abs(ix - jx) <= 1 && abs(iy - jy) <= 1 && abs(iz - jz) <= 1) {
            for (int ez = max(max(iz, jz) - 1, 0); ez <= min(min(iz, jz), g.nz - 1); ++ez)
                for (int ey = max(max(iy, jy) - 1, 0); ey <= min(min(iy, jy), g.ny - 1); ++ey)
                    for (int ex = max(max(ix, jx) - 1, 0); ex <= min(min(ix, jx), g.nx - 1); ++ex) {
                        const long long e = ((long long)ez * g.ny + ey) * g.nx + ex;
                        const int ai[3] = {ix - ex, iy - ey, iz - ez}, aj[3] = {jx - ex, jy - ey, jz - ez};
                        for (int qp = 0; qp < 8; ++qp) {   // column's Gauss node
                            const double gj = tab.L[qp & 1][aj[0]] * tab.L[(qp >> 1) & 1][aj[1]] *
                                              tab.L[qp >> 2][aj[2]];
                            const double* colv = probes + (long long)(cJ * 8 + qp) * dgsize + (e * g.C + cI) * 8;
                            double s = 0.0;
                            for (int q = 0; q < 8; ++q)
                                s += tab.L[q & 1][ai[0]] * tab.L[(q >> 1) & 1][ai[1]] * tab.L[q >> 2][ai[2]] * colv[q];
                            acc += gj * s;
                        }
                    }
        }
        A[idx] = acc;
    }
}

// Inverse of the symmetric positive definite n x n matrix of the coarsest
// level by Gauss-Jordan elimination without pivoting, one kernel per pivot
// over the whole device: step k reads only the previous matrix Ain (its
// pivot row and column) and writes the next one Aout, so the n steps
// alternate between two buffers and no step races with itself.
//   Aout[k][j] = Ain[k][j] / p (j != k),  Aout[k][k] = 1 / p,
//   Aout[i][j] = Ain[i][j] - Ain[i][k] Ain[k][j] / p,  Aout[i][k] = -Ain[i][k] / p  (i != k).
__global__ void k_gj_step(const double* Ain, double* Aout, int n, int k) {
    const double pinv = 1.0 / Ain[(long long)k * n + k];
    const long long nn = (long long)n * n;
    GRID_STRIDE(idx, nn) {
        const int i = (int)(idx / n), jj = (int)(idx - (long long)i * n);
        const double rk = jj == k ? pinv : Ain[(long long)k * n + jj] * pinv;   // new row k
        if (i == k) Aout[idx] = rk;
        else Aout[idx] = (jj == k ? 0.0 : Ain[idx]) - Ain[(long long)i * n + k] * rk;
    }
}

// Pure-Neumann Poisson: A + mean(diag A) / n on every entry (one block
// sums the diagonal in a fixed order, then every entry is shifted).
__global__ void k_mean_diag_shift(double* A, int n, double* shift) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += A[(long long)i * n + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *shift = red[0] / n / n;
}

__global__ void k_add_shift(double* A, long long nn, const double* shift) {
    const double v = *shift;
    GRID_STRIDE(i, nn) A[i] += v;
}

// z = Ainv r (FP64 products and sums): one wavefront per row.
template <typename T>
__global__ void k_dense_mv(const double* Ainv, const T* r, T* z, int n, const int* skip) {
    if (skip != nullptr && *skip) return;
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= n) return;
    const double* a = Ainv + (long long)row * n;
    double acc = 0.0;
    for (int k = lane; k < n; k += 64) acc += a[k] * (double)r[k];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) z[row] = (T)acc;
}

}  // namespace

template <typename T>
hipError_t launch_cg_gather(const CgGeo& g, const CgL<T>& tab, const T* cg, T* dg, bool add, const int* skip,
                            hipStream_t s) {
    const int ncell = g.nx * g.ny * g.nz;
    const dim3 grid((unsigned)(ncell < 65535 ? ncell : 65535));
    if (add) launch_cell_n<T, true, true>(g, tab, cg, dg, skip, grid, s);
    else launch_cell_n<T, true, false>(g, tab, cg, dg, skip, grid, s);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_assemble(const CgGeo& g, const T* local, T* cg, const int* skip, hipStream_t s, int mode,
                              const T* r, const T* z, T* d, const T* dinv, const double* coef);

template <typename T>
hipError_t launch_cg_scatter(const CgGeo& g, const CgL<T>& tab, T* dg, T* cg, const int* skip, hipStream_t s,
                             int mode, const T* r, const T* z, T* d, const T* dinv, const double* coef) {
    const int ncell = g.nx * g.ny * g.nz;
    const dim3 grid((unsigned)(ncell < 65535 ? ncell : 65535));
    launch_cell_n<T, false, false>(g, tab, dg, dg, skip, grid, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_cg_assemble<T>(g, dg, cg, skip, s, mode, r, z, d, dinv, coef);
}

template <typename T>
hipError_t launch_cg_assemble(const CgGeo& g, const T* local, T* cg, const int* skip, hipStream_t s, int mode,
                              const T* r, const T* z, T* d, const T* dinv, const double* coef) {
    const long long total = (long long)g.Mx * g.My * g.Mz * g.C;
    AsmIO<T> io;
    io.r = r; io.z = z; io.d = d; io.dinv = dinv; io.coef = coef;
    const long long planes = (long long)g.Mz * g.C;
    if (g.j >= 1 && g.j <= 5 && planes <= 65535) {
        const dim3 grid((unsigned)(((long long)g.Mx * g.My + kThreads - 1) / kThreads), (unsigned)planes);
        auto go = [&](auto jc) {
            constexpr int J = decltype(jc)::value;
            if (mode == 1)
                hipLaunchKernelGGL((k_cg_assemble_j<T, ASM_RESID, J>), grid, dim3(kThreads), 0, s, g, local, cg, io, skip);
            else if (mode == 2)
                hipLaunchKernelGGL((k_cg_assemble_j<T, ASM_CHEB, J>), grid, dim3(kThreads), 0, s, g, local, cg, io, skip);
            else if (mode == 3)
                hipLaunchKernelGGL((k_cg_assemble_j<T, ASM_CHEB_ACC, J>), grid, dim3(kThreads), 0, s, g, local, cg, io,
                                   skip);
            else
                hipLaunchKernelGGL((k_cg_assemble_j<T, ASM_SUM, J>), grid, dim3(kThreads), 0, s, g, local, cg, io, skip);
        };
        switch (g.j) {
            case 1: go(std::integral_constant<int, 1>{}); break;
            case 2: go(std::integral_constant<int, 2>{}); break;
            case 3: go(std::integral_constant<int, 3>{}); break;
            case 4: go(std::integral_constant<int, 4>{}); break;
            default: go(std::integral_constant<int, 5>{}); break;
        }
        return hipGetLastError();
    }
    const dim3 ag(grid_for(total));
    if (mode == 1) hipLaunchKernelGGL((k_cg_assemble<T, ASM_RESID>), ag, dim3(kThreads), 0, s, g, local, cg, io, skip);
    else if (mode == 2) hipLaunchKernelGGL((k_cg_assemble<T, ASM_CHEB>), ag, dim3(kThreads), 0, s, g, local, cg, io, skip);
    else if (mode == 3)
        hipLaunchKernelGGL((k_cg_assemble<T, ASM_CHEB_ACC>), ag, dim3(kThreads), 0, s, g, local, cg, io, skip);
    else hipLaunchKernelGGL((k_cg_assemble<T, ASM_SUM>), ag, dim3(kThreads), 0, s, g, local, cg, io, skip);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_axis(const AxisMat<T>& M, int axis, int C, int n0, int n1, int n2, const T* in, T* out, bool add,
                       const int* skip, hipStream_t s) {
    long long total = (long long)C * (axis == 0 ? M.rows : n0) * (axis == 1 ? M.rows : n1) * (axis == 2 ? M.rows : n2);
    const int o0 = axis == 0 ? M.rows : n0, o1 = axis == 1 ? M.rows : n1, o2 = axis == 2 ? M.rows : n2;
    const long long plane = (long long)o0 * o1, planes = (long long)o2 * C;
    if (plane < (1ll << 31) && planes <= 65535) {
        const dim3 grid((unsigned)((plane + kThreads - 1) / kThreads), (unsigned)planes);
        if (add)
            hipLaunchKernelGGL((k_axis2<T, true>), grid, dim3(kThreads), 0, s, M, axis, n0, n1, n2, o0, o1, o2, in, out,
                               skip);
        else
            hipLaunchKernelGGL((k_axis2<T, false>), grid, dim3(kThreads), 0, s, M, axis, n0, n1, n2, o0, o1, o2, in, out,
                               skip);
        return hipGetLastError();
    }
    if (add)
        hipLaunchKernelGGL((k_axis<T, true>), dim3(grid_for(total)), dim3(kThreads), 0, s, M, axis, C, n0, n1, n2, in,
                           out, skip);
    else
        hipLaunchKernelGGL((k_axis<T, false>), dim3(grid_for(total)), dim3(kThreads), 0, s, M, axis, C, n0, n1, n2, in,
                           out, skip);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_cheb(const T* z, T* zn, T* d, const T* r, const T* t, const T* dinv, const double* coef,
                          long long n, const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_cheb<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, z, zn, d, r, t, dinv, coef, n, skip);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_sub(T* y, const T* r, const T* t, long long n, const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_sub<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, y, r, t, n, skip);
    return hipGetLastError();
}

template <int N>
void launch_cg_diag_n(int C, const OpData<double>& op, const CgDiagTab& tab, double* local, hipStream_t s) {
    constexpr int CPB = kDiagThreads / (N * N * N);
    const long long blocks = (op.ncell + CPB - 1) / CPB;
    const dim3 grid((unsigned)(blocks < 65535 ? blocks : 65535)), block(CPB * N * N * N);
    if (C == 3) hipLaunchKernelGGL((k_cg_diag_local<3, N>), grid, block, 0, s, op, tab, local);
    else hipLaunchKernelGGL((k_cg_diag_local<1, N>), grid, block, 0, s, op, tab, local);
}

hipError_t launch_cg_diagonal(const CgGeo& g, const OpData<double>& op, const CgDiagTab& tab, double* local,
                              double* diag, double* dinv64, float* dinv32, hipStream_t s) {
    switch (g.j + 1) {
        case 2: launch_cg_diag_n<2>(g.C, op, tab, local, s); break;
        case 3: launch_cg_diag_n<3>(g.C, op, tab, local, s); break;
        case 4: launch_cg_diag_n<4>(g.C, op, tab, local, s); break;
        case 5: launch_cg_diag_n<5>(g.C, op, tab, local, s); break;
        case 6: launch_cg_diag_n<6>(g.C, op, tab, local, s); break;
        default: return hipErrorInvalidValue;
    }
    const long long total = (long long)g.Mx * g.My * g.Mz * g.C;
    AsmIO<double> io;
    std::memset(&io, 0, sizeof(io));
    hipLaunchKernelGGL((k_cg_assemble<double, ASM_SUM>), dim3(grid_for(total)), dim3(kThreads), 0, s, g, local, diag,
                       io, nullptr);
    hipLaunchKernelGGL(k_cg_invert, dim3(grid_for(total)), dim3(kThreads), 0, s, diag, dinv64, dinv32, total);
    return hipGetLastError();
}

hipError_t launch_cg_probe(double* v, int C, long long ncell, int col, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_probe, dim3(grid_for(ncell * C * 8)), dim3(kThreads), 0, s, v, C, ncell, col);
    return hipGetLastError();
}

hipError_t launch_cg_coarse_inverse(const CgGeo& g, const double* probes, long long dgsize, const CgL<double>& tab,
                                    double* A, double* work, int mean_zero, hipStream_t s) {
    const long long nc = (long long)g.Mx * g.My * g.Mz * g.C, nn = nc * nc;
    // the steps alternate between A and work; start where the last step writes A
    double* buf[2] = {(nc % 2 == 0) ? A : work, (nc % 2 == 0) ? work : A};
    hipLaunchKernelGGL(k_cg_coarse_matrix, dim3(grid_for(nn)), dim3(kThreads), 0, s, g, probes, dgsize, tab, buf[0]);
    if (mean_zero) {
        hipLaunchKernelGGL(k_mean_diag_shift, dim3(1), dim3(256), 0, s, buf[0], (int)nc, work + nn);
        hipLaunchKernelGGL(k_add_shift, dim3(grid_for(nn)), dim3(kThreads), 0, s, buf[0], nn, work + nn);
    }
    for (int k = 0; k < (int)nc; ++k)
        hipLaunchKernelGGL(k_gj_step, dim3(grid_for(nn)), dim3(kThreads), 0, s, buf[k & 1], buf[(k + 1) & 1], (int)nc, k);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dense_mv(const double* Ainv, const T* r, T* z, int n, const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_mv<T>, dim3((n + 3) / 4), dim3(256), 0, s, Ainv, r, z, n, skip);
    return hipGetLastError();
}

#define INST(T)                                                                                                     \
    template hipError_t launch_cg_gather<T>(const CgGeo&, const CgL<T>&, const T*, T*, bool, const int*, hipStream_t); \
    template hipError_t launch_cg_scatter<T>(const CgGeo&, const CgL<T>&, T*, T*, const int*, hipStream_t, int,    \
                                             const T*, const T*, T*, const T*, const double*);                    \
    template hipError_t launch_cg_assemble<T>(const CgGeo&, const T*, T*, const int*, hipStream_t, int, const T*,   \
                                              const T*, T*, const T*, const double*);                              \
    template hipError_t launch_axis<T>(const AxisMat<T>&, int, int, int, int, int, const T*, T*, bool, const int*,  \
                                       hipStream_t);                                                                \
    template hipError_t launch_cg_cheb<T>(const T*, T*, T*, const T*, const T*, const T*, const double*, long long, \
                                          const int*, hipStream_t);                                                 \
    template hipError_t launch_cg_sub<T>(T*, const T*, const T*, long long, const int*, hipStream_t);               \
    template hipError_t launch_dense_mv<T>(const double*, const T*, T*, int, const int*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace sipg
