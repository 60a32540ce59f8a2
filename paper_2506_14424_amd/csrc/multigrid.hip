// Multigrid transfers and level vector kernels of the hp-multigrid
// preconditioner (Sec. 5.3): the polynomial degree is lowered from k to k-1
// on the same mesh (degree step), then the mesh is coarsened by two in every
// direction (mesh step).  Prolongation evaluates the coarse polynomial of a
// cell at the fine nodes: for a degree step through P[i][j] = l^c_j(x^f_i) in
// every direction of the same cell, for a mesh step through
// H[b][i][j] = l_j((b + x_i) / 2) from the parent cell to its child b in
// every direction.  Restriction is the transpose.  Degree steps run as
// three 1D sweeps per cell in LDS; mesh steps (small, coarse levels) use one
// thread per output value summing the few (n <= 6) tensor-product terms
// directly.  No output is written by more than one thread and no atomics
// are needed.

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

// rc = P^T tf: one thread per coarse value
template <typename T, bool MESH>
__global__ void k_restrict(int C, int nf, int nc, int fx, int fy, int fz, const MgTab<T> tab, const T* tf, T* rc,
                           long long total, const int* skip) {
    if (skip != nullptr && *skip) return;
    const int ncx = MESH ? fx / 2 : fx, ncy = MESH ? fy / 2 : fy;
    const int nc3 = nc * nc * nc, nf3 = nf * nf * nf;
    GRID_STRIDE(idx, total) {
        const int j = (int)(idx % nc3);
        const long long ec_c = idx / nc3;  // coarse cell * C + component
        const int c = (int)(ec_c % C);
        const int ecell = (int)(ec_c / C);
        const int j1 = j % nc, j2 = (j / nc) % nc, j3 = j / (nc * nc);
        T acc = 0;
        if constexpr (!MESH) {
            const T* src = tf + ((long long)ecell * C + c) * nf3;
            for (int i3 = 0; i3 < nf; ++i3) {
                const T w3 = tab.P[i3][j3];
                for (int i2 = 0; i2 < nf; ++i2) {
                    const T w23 = w3 * tab.P[i2][j2];
                    const T* row = src + (i3 * nf + i2) * nf;
                    T s = 0;
                    for (int i1 = 0; i1 < nf; ++i1) s += tab.P[i1][j1] * row[i1];
                    acc += w23 * s;
                }
            }
        } else {
            const int ex = ecell % ncx, ey = (ecell / ncx) % ncy, ez = ecell / (ncx * ncy);
            for (int bz = 0; bz < 2; ++bz)
                for (int by = 0; by < 2; ++by)
                    for (int bx = 0; bx < 2; ++bx) {
                        const int ef = ((2 * ez + bz) * fy + 2 * ey + by) * fx + 2 * ex + bx;
                        const T* src = tf + ((long long)ef * C + c) * nf3;
                        for (int i3 = 0; i3 < nf; ++i3) {
                            const T w3 = tab.H[bz][i3][j3];
                            for (int i2 = 0; i2 < nf; ++i2) {
                                const T w23 = w3 * tab.H[by][i2][j2];
                                const T* row = src + (i3 * nf + i2) * nf;
                                T s = 0;
                                for (int i1 = 0; i1 < nf; ++i1) s += tab.H[bx][i1][j1] * row[i1];
                                acc += w23 * s;
                            }
                        }
                    }
        }
        rc[idx] = acc;
    }
}

// zf += P zc: one thread per fine value
template <typename T, bool MESH>
__global__ void k_prolong_add(int C, int nf, int nc, int fx, int fy, int fz, const MgTab<T> tab, const T* zc, T* zf,
                              long long total, const int* skip) {
    if (skip != nullptr && *skip) return;
    const int nc3 = nc * nc * nc, nf3 = nf * nf * nf;
    GRID_STRIDE(idx, total) {
        const int i = (int)(idx % nf3);
        const long long ef_c = idx / nf3;
        const int c = (int)(ef_c % C);
        const int ef = (int)(ef_c / C);
        const int i1 = i % nf, i2 = (i / nf) % nf, i3 = i / (nf * nf);
        long long ecell;
        int b1 = 0, b2 = 0, b3 = 0;  // child position in the parent (mesh step)
        if constexpr (!MESH) {
            ecell = ef;
        } else {
            const int ex = ef % fx, ey = (ef / fx) % fy, ez = ef / (fx * fy);
            ecell = ((long long)(ez / 2) * (fy / 2) + ey / 2) * (fx / 2) + ex / 2;
            b1 = ex & 1; b2 = ey & 1; b3 = ez & 1;
        }
        auto w = [&](int b, int a, int j) -> T { return MESH ? tab.H[b][a][j] : tab.P[a][j]; };
        const T* src = zc + (ecell * C + c) * nc3;
        T acc = 0;
        for (int j3 = 0; j3 < nc; ++j3)
            for (int j2 = 0; j2 < nc; ++j2) {
                const T* row = src + (j3 * nc + j2) * nc;
                T s = 0;
                for (int j1 = 0; j1 < nc; ++j1) s += w(b1, i1, j1) * row[j1];
                acc += (w(b3, i3, j3) * w(b2, i2, j2)) * s;
            }
        zf[idx] += acc;
    }
}

// Degree steps (same cell) by sum factorisation: one block per cell, the
// cell's C n^3 input values in LDS, three 1D sweeps with the n_f x n_c table
// P (restriction: contraction over the fine index; prolongation: over the
// coarse index), the result written (restriction) or added (prolongation)
// with coalesced accesses.  O(n) operations per intermediate value instead
// of O(n^3) per output.
constexpr int kSfThreads = 128;
constexpr int kSfVals = 3 * kMaxN * kMaxN * kMaxN;

template <typename T, bool RESTRICT>
__global__ void __launch_bounds__(kSfThreads) k_pstep(int C, int nf, int nc, int ncell, const MgTab<T> tab,
                                                     const T* in, T* out, const int* skip) {
    if (skip != nullptr && *skip) return;
    __shared__ T A[kSfVals], B[kSfVals];
    // input extent (a) and output extent (b) along one direction
    const int na = RESTRICT ? nf : nc, nb = RESTRICT ? nc : nf;
    const int nin = C * na * na * na;
    for (int e = blockIdx.x; e < ncell; e += gridDim.x) {
        __syncthreads();
        for (int i = threadIdx.x; i < nin; i += kSfThreads) A[i] = in[(long long)e * nin + i];
        __syncthreads();
        // sweep 1 (first index): B[c][a3][a2][b1] = sum_a1 W(a1, b1) A[c][a3][a2][a1]
        const int n1 = C * na * na * nb;
        for (int k = threadIdx.x; k < n1; k += kSfThreads) {
            const int b1 = k % nb, rest = k / nb;  // rest = (c, a3, a2)
            const T* src = A + rest * na;
            T acc = 0;
            for (int a = 0; a < na; ++a) acc += (RESTRICT ? tab.P[a][b1] : tab.P[b1][a]) * src[a];
            B[k] = acc;
        }
        __syncthreads();
        // sweep 2 (second index): A[c][a3][b2][b1] = sum_a2 W(a2, b2) B[c][a3][a2][b1]
        const int n2 = C * na * nb * nb;
        for (int k = threadIdx.x; k < n2; k += kSfThreads) {
            const int b1 = k % nb, b2 = (k / nb) % nb, rest = k / (nb * nb);  // rest = (c, a3)
            const T* src = B + rest * na * nb + b1;
            T acc = 0;
            for (int a = 0; a < na; ++a) acc += (RESTRICT ? tab.P[a][b2] : tab.P[b2][a]) * src[a * nb];
            A[k] = acc;
        }
        __syncthreads();
        // sweep 3 (third index): out[c][b3][b2][b1] = sum_a3 W(a3, b3) A[c][a3][b2][b1]
        const int nbb = nb * nb, n3 = C * nb * nbb;
        for (int k = threadIdx.x; k < n3; k += kSfThreads) {
            const int b12 = k % nbb, b3 = (k / nbb) % nb, c = k / (nbb * nb);
            const T* src = A + c * na * nbb + b12;
            T acc = 0;
            for (int a = 0; a < na; ++a) acc += (RESTRICT ? tab.P[a][b3] : tab.P[b3][a]) * src[a * nbb];
            if (RESTRICT) out[(long long)e * n3 + k] = acc;
            else out[(long long)e * n3 + k] += acc;
        }
    }
}

template <typename T>
__global__ void k_cheb_start_t(const T* r, T* z, T* d, const T* dinv, long long n, const SolveState* st,
                               const int* skip) {
    if (*skip) return;
    const T ti = T(st->theta_inv);
    GRID_STRIDE(i, n) {
        const T zv = ti * dinv[i] * r[i];
        z[i] = zv;
        d[i] = zv;
    }
}

template <typename T>
__global__ void k_copy_t(T* y, const T* x, long long n, const int* skip) {
    if (*skip) return;
    GRID_STRIDE(i, n) y[i] = x[i];
}

template <typename T>
__global__ void k_add_t(T* y, const T* x, long long n, const int* skip) {
    if (*skip) return;
    GRID_STRIDE(i, n) y[i] += x[i];
}

template <typename T>
__global__ void k_to_f64(double* y, const T* x, long long n) {
    GRID_STRIDE(i, n) y[i] = (double)x[i];
}

}  // namespace

template <typename T>
hipError_t launch_restrict(bool mesh_step, int C, int nf, int nc, int fx, int fy, int fz, const MgTab<T>& tab,
                           const T* tf, T* rc, const int* skip, hipStream_t s) {
    const long long ncell = mesh_step ? (long long)(fx / 2) * (fy / 2) * (fz / 2) : (long long)fx * fy * fz;
    const long long total = ncell * C * nc * nc * nc;
    if (mesh_step)
        hipLaunchKernelGGL((k_restrict<T, true>), dim3(grid_for(total)), dim3(kThreads), 0, s, C, nf, nc, fx, fy, fz,
                           tab, tf, rc, total, skip);
    else
        hipLaunchKernelGGL((k_pstep<T, true>), dim3((unsigned)(ncell < 65535 ? ncell : 65535)), dim3(kSfThreads), 0, s,
                           C, nf, nc, (int)ncell, tab, tf, rc, skip);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(bool mesh_step, int C, int nf, int nc, int fx, int fy, int fz, const MgTab<T>& tab,
                              const T* zc, T* zf, const int* skip, hipStream_t s) {
    const long long total = (long long)fx * fy * fz * C * nf * nf * nf;
    const long long ncell = (long long)fx * fy * fz;
    if (mesh_step)
        hipLaunchKernelGGL((k_prolong_add<T, true>), dim3(grid_for(total)), dim3(kThreads), 0, s, C, nf, nc, fx, fy,
                           fz, tab, zc, zf, total, skip);
    else
        hipLaunchKernelGGL((k_pstep<T, false>), dim3((unsigned)(ncell < 65535 ? ncell : 65535)), dim3(kSfThreads), 0,
                           s, C, nf, nc, (int)ncell, tab, zc, zf, skip);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cheb_start_t(const T* r, T* z, T* d, const T* dinv, long long n, const SolveState* st,
                               const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(k_cheb_start_t<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, r, z, d, dinv, n, st, skip);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_copy_t(T* y, const T* x, long long n, const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_t<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, y, x, n, skip);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_add_t(T* y, const T* x, long long n, const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(k_add_t<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, y, x, n, skip);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_to_f64(double* y, const T* x, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_f64<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, y, x, n);
    return hipGetLastError();
}

#define INST(T)                                                                                                  \
    template hipError_t launch_restrict<T>(bool, int, int, int, int, int, int, const MgTab<T>&, const T*, T*,     \
                                           const int*, hipStream_t);                                             \
    template hipError_t launch_prolong_add<T>(bool, int, int, int, int, int, int, const MgTab<T>&, const T*, T*,  \
                                              const int*, hipStream_t);                                          \
    template hipError_t launch_cheb_start_t<T>(const T*, T*, T*, const T*, long long, const SolveState*,          \
                                               const int*, hipStream_t);                                         \
    template hipError_t launch_copy_t<T>(T*, const T*, long long, const int*, hipStream_t);                       \
    template hipError_t launch_add_t<T>(T*, const T*, long long, const int*, hipStream_t);                        \
    template hipError_t launch_to_f64<T>(double*, const T*, long long, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace sipg
