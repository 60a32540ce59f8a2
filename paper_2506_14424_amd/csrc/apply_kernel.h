// Matrix-free operator application (SIPG viscous and Poisson, penalty step) for gfx950:
// the kernel template, instantiated by apply.hip and apply_penalty.hip.
//
// One workgroup handles CPB cells; each cell gets n*n threads.  Everything a
// cell needs is computed by its own threads ("cell-centric"): the cell
// integral and all six face integrals for the cell's own test functions.  A
// face is therefore evaluated once from each side, but every output entry is
// written exactly once, with no atomics and no second pass over the output.
// The neighbour's trace on a shared face is interpolated from the
// neighbour's nodal values, which the XCD-aware block order keeps in the L2.
//
// Sum factorisation (Sec. 5.3): with nodes at the Gauss points, values at
// quadrature points are the nodal values, and reference derivatives are 1D
// contractions with D[q][j] = l_j'(g_q) along one axis.  For every 1D sweep a
// thread owns a whole line of n values (the n*n threads of a cell own the
// n*n lines of each direction), so all sweep coefficients are the same for
// the whole wavefront and stay in scalar registers; lines are exchanged
// through LDS between sweeps.  The thread (i1, i2) owns the xi_3 line
// (i1, i2, 0..n-1) of quadrature points and outputs.  FP64 n = 4 runs the
// sweeps across lanes (xi_1, xi_2 in the cell term, the tangential
// directions of a face) as FP64 matrix-core products of 4 x 4 tiles, one
// tile per cell of the wavefront (mf_r, mf_c); its lanes are ordered for
// that (lane 16 i1 + 4 cell + i2).
//
// Forms (Sec. 4.1), per quadrature point, for the test functions of the cell
// that owns the thread (outward unit normal n, [u] = u_own - u_nbr):
//   cell      viscous: sigma = 2 mu eps(u) JxW, mass alpha u JxW
//             poisson: sigma = grad u JxW,      mass alpha u JxW
//   face      viscous: a = -2 {{mu eps(u)}} n + tau([u] + n([u].n)),
//                      B = -mu sym([u] (x) n)
//             poisson: a = -{{grad u}}.n + tau [u],  B = -[u] n / 2
//   and the test integration y_i += sum ds (phi_i a + grad phi_i : B).
// Dirichlet faces use the mirror state u_nbr = -u_own, grad u_nbr = grad u_own;
// Neumann faces contribute nothing.

#pragma once

#include "device_common.h"

namespace sipg {

template <int N, int C, bool DBL>
struct Shape {
    // cells per workgroup: one wavefront for n <= 4 and for FP64 n = 5 (two
    // cells, 50 lanes: wavefront fences instead of workgroup barriers beat
    // the idle lanes there; FP32 n = 5 keeps five cells in two wavefronts),
    // LDS well under 64 KB
    static constexpr int CPB = N == 2 ? 16 : N == 3 ? 7 : N == 4 ? 4 : N == 5 ? (DBL ? 2 : 5) : (DBL && C == 3 ? 3 : 7);
    static constexpr int THREADS = CPB * N * N;
    static constexpr int NNN = N * N * N, NN = N * N;
    // LDS layout of a cell's volume arrays: node (i1, i2, i3) of component c at
    //   plain:  c*CS + i3*S3 + i2*N + i1,
    //   skewed: c*CS + ((i3 + x) % N)*S3 + ((i2 + i3) % N)*N + (i1 + x) % N, x = cell % 4.
    // The skew (FP64, n = 4, lanes 16 i1 + 4 cell + i2) makes the xi_1-line,
    // xi_2-line and xi_3-column patterns of the wavefront's 64 lanes hit
    // every bank pair equally often without padding (no conflicts with
    // either 32 or 64 banks of 4 bytes).  In FP32 the padded xi_3
    // stride S3 spreads the three patterns instead (n = 3, 4); there the
    // padding costs no occupancy.
    static constexpr bool SKEW = DBL && N == 4;
    static constexpr int S3 = DBL ? NN : (N == 3 ? 12 : N == 4 ? 19 : NN);
    static constexpr int CS = N * S3;
    // per-cell LDS: nodal values and a work space for the cell sweeps and the
    // face stages; +1 staggers consecutive cells over the LDS banks (plain layout)
    static constexpr int U = C * CS + (SKEW ? 0 : 1);
    // work-space stride +1 (staggers consecutive cells over the banks).
    // FP32 n = 4: the face stages' tangential sweeps exchange values across
    // lanes (DPP) instead of through LDS.
    // FP64 n = 4: the 1D sweeps across lanes run on the matrix cores instead
    // (v_mfma_f64_4x4x4: four 16-lane blocks, each a 4 x 4 product that
    // contracts over lane bits 5:4).  Lane 16 i1 + 4 cell + i2 owns the xi_3
    // column (i1, i2) of its cell, so a 4 x 4 tile of points (i1, i2) of the
    // four cells is one operand: sweeps along i1 are one product, sweeps
    // along i2 a product with the identity (which moves i2 to bits 5:4)
    // and then one more.  No DPP moves, and the cell pass needs no LDS.
    static constexpr bool MF = DBL && N == 4;
    static constexpr bool DPP = (N == 4 && !MF) || N == 2;
    // n = 2 (cell and face passes across lanes): only the projection's
    // coefficient array remains, so the work space shrinks to that
    // (FP64 n = 4: the projection's array only, stride 2 C n^2 + 4)
    static constexpr int W = N == 2 ? 2 * C * NN + 1
                           : MF     ? 2 * C * NN + 4
                                    : (2 * C * CS > 8 * C * NN ? 2 * C * CS : 8 * C * NN) + 1;
};

// Matrix-core sweeps of a 4 x 4 tile per cell (FP64 n = 4 layout, lane
// 16 r + 4 cell + c holds U[r][c] of its cell).  m is the lane's entry
// M[c][r] of the 1D matrix M; id is (r == c).
//   mf_r: V[i][c] = sum_k M[i][k] U[k][c]   (one product, in place)
//   mf_c: V[r][j] = sum_k M[j][k] U[r][k]   (the identity product gives the
//         transpose of U, whose rows then contract with M^T)
__device__ __forceinline__ double mf_r(double u, double m) {
    return __builtin_amdgcn_mfma_f64_4x4x4f64(m, u, 0.0, 0, 0, 0);
}
__device__ __forceinline__ double mf_c(double u, double m, double id) {
    const double ut = __builtin_amdgcn_mfma_f64_4x4x4f64(u, id, 0.0, 0, 0, 0);
    return __builtin_amdgcn_mfma_f64_4x4x4f64(ut, m, 0.0, 0, 0, 0);
}

// Barrier between LDS stages.  A workgroup of one wavefront only needs the
// wavefront's own (in-order) LDS accesses fenced against compiler reordering.
template <int THREADS>
__device__ __forceinline__ void stage_sync() {
    if constexpr (THREADS <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Reciprocal: hardware estimate refined by Newton steps to full precision.
template <typename T>
__device__ __forceinline__ T recip(T d) {
    if constexpr (sizeof(T) == 8) {
        double r = __builtin_amdgcn_rcp(d);
        double e = __builtin_fma(-d, r, 1.0);
        r = __builtin_fma(r, e, r);
        e = __builtin_fma(-d, r, 1.0);
        return __builtin_fma(r, e, r);
    } else {
        float r = __builtin_amdgcn_rcpf(d);
        const float e = __builtin_fmaf(-d, r, 1.0f);
        return __builtin_fmaf(r, e, r);
    }
}

// 1/sqrt(v): hardware estimate refined by Newton steps to full precision.
template <typename T>
__device__ __forceinline__ T rsqrt_nr(T v) {
    if constexpr (sizeof(T) == 8) {
        double r = __builtin_amdgcn_rsq(v);
        double h = 0.5 * v;
        r = r * __builtin_fma(-h * r, r, 1.5);
        r = r * __builtin_fma(-h * r, r, 1.5);
        return r;
    } else {
        float r = __builtin_amdgcn_rsqf(v);
        return r * __builtin_fmaf(-0.5f * v * r, r, 1.5f);
    }
}

// Columns a_d = d x / d xi_d of the Jacobian of a trilinear cell at xi.
template <typename T>
__device__ __forceinline__ void jac_columns(const T (*g)[3], const T xi[3], T a[3][3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        a[0][i] = g[1][i] + g[4][i] * xi[1] + g[5][i] * xi[2] + g[7][i] * (xi[1] * xi[2]);
        a[1][i] = g[2][i] + g[4][i] * xi[0] + g[6][i] * xi[2] + g[7][i] * (xi[0] * xi[2]);
        a[2][i] = g[3][i] + g[5][i] * xi[0] + g[6][i] * xi[1] + g[7][i] * (xi[0] * xi[1]);
    }
}

template <typename T>
__device__ __forceinline__ void cross3(const T u[3], const T v[3], T w[3]) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
}

// Rows of J^-1 from the columns: row d = (a_{d+1} x a_{d+2}) / det.
template <typename T>
__device__ __forceinline__ void inverse_from_columns(const T a[3][3], T Ji[3][3], T& det) {
    T c0[3], c1[3], c2[3];
    cross3(a[1], a[2], c0);
    cross3(a[2], a[0], c1);
    cross3(a[0], a[1], c2);
    det = a[0][0] * c0[0] + a[0][1] * c0[1] + a[0][2] * c0[2];
    const T inv = recip(det);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Ji[0][i] = c0[i] * inv;
        Ji[1][i] = c1[i] * inv;
        Ji[2][i] = c2[i] * inv;
    }
}

struct CellIdx {
    int lc, t, i1, i2, ec, ex, ey, ez;
    int ra[4], rb[4];  // n = 4: a / b index of the lane whose value line_a / line_b delivers in slot r
    double md, mt, mi; // matrix-core layout: D[i2][i1], D[i1][i2], (i1 == i2)
    bool active;
};

// Per-lane LDS offsets of the three line patterns of a cell's volume arrays
// (lane (la, lb) = (t % n, t / n)): oz[j] = node (la, lb, j), the lane's
// xi_3 column; ox[j] = node (j, la, lb), a xi_1 line; oy[j] = node (la, j, lb),
// a xi_2 line.
template <int N>
struct VolOff {
    int oz[N], ox[N], oy[N];
};

template <int N, int S3, bool SKEW>
__device__ __forceinline__ int vol_pos(int i1, int i2, int i3, int px) {
    if constexpr (!SKEW) {
        return i3 * S3 + i2 * N + i1;
    } else {
        int a = i2 + i3, b = i1 + px, c = i3 + px;
        a = a >= N ? a - N : a;
        b = b >= N ? b - N : b;
        c = c >= N ? c - N : c;
        return c * S3 + a * N + b;
    }
}

template <int N, int S3, bool SKEW>
__device__ __forceinline__ void vol_offsets(int la, int lb, int lc, VolOff<N>& o) {
    const int px = lc & 3;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        o.oz[j] = vol_pos<N, S3, SKEW>(la, lb, j, px);
        o.ox[j] = vol_pos<N, S3, SKEW>(j, la, lb, px);
        o.oy[j] = vol_pos<N, S3, SKEW>(la, j, lb, px);
    }
}

// Small per-lane tables kept in LDS: points, weights, face values/derivatives.
template <typename T, int N>
struct LaneTab {
    T x[N], w[N], S[2][N], G[2][N];
    T D[N][N];  // D[q][j] = l_j'(g_q), read per lane by the cross-lane face sweeps
};

// Cross-lane moves within rows of 16 lanes (DPP).  For n = 4 a cell's 16
// lanes are one row and lane 4 b + a holds face point (a, b), so the lines
// of a face are a quad (along a) or the lanes 4 apart (along b).
// (quad permutations and row rotations read a valid lane everywhere, so
// no "old" value has to be kept: bound_ctrl lets the move write directly)
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}

template <int CTRL, typename T>
__device__ __forceinline__ T dpp_mov(T v) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = (unsigned)dpp_i<CTRL>((int)(unsigned)(b & 0xffffffffull));
        const unsigned hi = (unsigned)dpp_i<CTRL>((int)(unsigned)(b >> 32));
        return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
    } else {
        return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, v)));
    }
}

// The n values of a lane's line along a (own value, then the quad
// permuted so that slot r holds a' = CellIdx::ra[r]) and along b (own value,
// then, for n = 4, rows rotated by 4, 8, 12 lanes; for n = 2 the other pair
// of the quad; slot r holds b' = CellIdx::rb[r]).  n = 4: a cell is a row of
// 16 lanes; n = 2: a cell is a quad, lane 2 b + a.
template <int N, typename T>
__device__ __forceinline__ void line_a(T v, T out[N]) {
    out[0] = v;
    if constexpr (N == 4) {
        out[1] = dpp_mov<0x39>(v);  // quad_perm [1, 2, 3, 0]
        out[2] = dpp_mov<0x4E>(v);  // quad_perm [2, 3, 0, 1]
        out[3] = dpp_mov<0x93>(v);  // quad_perm [3, 0, 1, 2]
    } else {
        out[1] = dpp_mov<0xB1>(v);  // quad_perm [1, 0, 3, 2]
    }
}
template <int N, typename T>
__device__ __forceinline__ void line_b(T v, T out[N]) {
    out[0] = v;
    if constexpr (N == 4) {
        out[1] = dpp_mov<0x124>(v);  // row_ror:4
        out[2] = dpp_mov<0x128>(v);  // row_ror:8
        out[3] = dpp_mov<0x12C>(v);  // row_ror:12
    } else {
        out[1] = dpp_mov<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    }
}

// The neighbour's line of nodal values through face point (i1, i2) of face
// (D, s), and the face viscosity and penalty factor at that point.
template <int N, int C, typename T, bool CURVED, int D>
__device__ __forceinline__ void face_prefetch(const OpData<T>& op, const ApplyIO<T>& io, const CellIdx& ci, int s,
                                              T (&nb)[C][N], T& mu, T& tf, T (&gn)[8]) {
    constexpr int NN = N * N, NNN = N * N * N;
    const int i1 = ci.i1, i2 = ci.i2;
    const int pos = D == 0 ? ci.ex : D == 1 ? ci.ey : ci.ez;
    const int lim = D == 0 ? op.nx : D == 1 ? op.ny : op.nz;
    const bool has_nb = s == 1 ? pos + 1 < lim : pos > 0;
    const int stride = D == 0 ? 1 : D == 1 ? op.nx : op.nx * op.ny;
    const int en = has_nb ? ci.ec + (s == 1 ? stride : -stride) : ci.ec;
    const bool dir = !has_nb && op.bc[2 * D + s] == 0;
    const bool live = ci.active && (has_nb ? (io.parts & SIPG_PART_INTERIOR) != 0
                                           : (dir && (io.parts & SIPG_PART_BOUNDARY) != 0));
    int fid;
    if (D == 0) fid = (ci.ez * op.ny + ci.ey) * (op.nx + 1) + ci.ex + s;
    else if (D == 1) fid = op.nfx + (ci.ez * (op.ny + 1) + ci.ey + s) * op.nx + ci.ex;
    else fid = op.nfx + op.nfy + ((ci.ez + s) * op.ny + ci.ey) * op.nx + ci.ex;
    if constexpr (CURVED) {
        const int dn = has_nb ? (s == 1 ? 1 : -1) : 0;  // the neighbour is one cell away along xi_D
        trilinear_coeffs(op.verts, op.nx, op.ny, ci.ex + (D == 0 ? dn : 0), ci.ey + (D == 1 ? dn : 0),
                         ci.ez + (D == 2 ? dn : 0), ci.t % 3, gn);
    }
    const T* xn = (io.xnb ? io.xnb : io.x) + (size_t)en * (C * NNN);
    const bool ld = live && has_nb;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            int off;
            if (D == 2) off = (c * N + j) * NN + i2 * N + i1;
            else if (D == 0) off = (c * N + i2) * NN + i1 * N + j;
            else off = (c * N + i2) * NN + j * N + i1;
            const T v = xn[off];  // en and fid are valid for every lane: load unconditionally
            nb[c][j] = ld ? v : T(0);
        }
    const T muf = C == 3 ? op.mu_face[(size_t)fid * NN + ci.t] : T(1);
    const T tff = op.tfac[fid];
    mu = live ? muf : T(1);
    tf = live ? tff : T(0);
}

// The neighbour's line of nodal values through this lane's face point of
// face f = 2 D + s (D known only at run time): the next face's data, loaded
// while the current face is computed.  Unmasked: the face that uses them
// zeroes the traces formed from them where there is no live neighbour, so
// that no instruction of the issuing face waits for the loads.
template <int N, int C, typename T>
struct FacePre {
    T nb[C][N];
};

template <int N, int C, typename T>
__device__ __forceinline__ void face_load_rt(const OpData<T>& op, const ApplyIO<T>& io, const CellIdx& ci, int f,
                                             FacePre<N, C, T>& p) {
    constexpr int NN = N * N, NNN = N * N * N;
    const int D = f >> 1, s = f & 1;
    // arithmetic selects: a select of struct fields by a run-time D becomes
    // a run-time address and sends the whole struct to scratch
    const int d0 = D == 0, d1 = D == 1, d2 = D == 2;
    const int pos = d0 * ci.ex + d1 * ci.ey + d2 * ci.ez;
    const int lim = d0 * op.nx + d1 * op.ny + d2 * op.nz;
    const bool has_nb = s == 1 ? pos + 1 < lim : pos > 0;
    const int stride = d0 + d1 * op.nx + d2 * op.nx * op.ny;
    const int en = has_nb ? ci.ec + (s == 1 ? stride : -stride) : ci.ec;
    // node j along D of the line through face point (i1, i2): base + j * step
    const int base = d2 * (ci.i2 * N + ci.i1) + d0 * (ci.i2 * NN + ci.i1 * N) + d1 * (ci.i2 * NN + ci.i1);
    const int step = d2 * NN + d0 + d1 * N;
    const T* xn = (io.xnb ? io.xnb : io.x) + (size_t)en * (C * NNN) + base;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int j = 0; j < N; ++j)
            p.nb[c][j] = xn[c * NNN + j * step];  // en is valid for every lane: load unconditionally
}

// ---------------------------------------------------------------- faces
//
// One face of the cell (direction D, side s), in stages separated by LDS
// barriers:
//   A  traces of both sides at face point (a, b) = (i1, i2): values into LDS,
//      d/dxi_D in registers;
//   B1 tangential derivatives of both traces, one line per task;
//   B2 geometry and flux at the face point;
//   C1 transposed tangential sweeps of the flux, one line per task;
//   C2 projection onto the cell's nodes (accumulated in y).
template <int N, int C, typename T, bool CURVED, int D, int THREADS, bool G7, bool LA>
__device__ __forceinline__ void face_pass(const OpData<T>& op, const ApplyIO<T>& io, const CellIdx& ci, int s,
                                          T (&y)[C][N], const T* su, T* sw, T (*geo)[8][3],
                                          const LaneTab<T, N>& lt, const VolOff<N>& vo, FacePre<N, C, T>& pre,
                                          int fnext) {
    // G7: the six neighbours' trilinear coefficients were staged in LDS at
    // the start (geo[1 + face]); LA: this face's neighbour line was loaded
    // during the previous face (pre; its traces are masked below) and the
    // face viscosity and penalty factor are loaded below; else all of them
    // are loaded here (and the neighbour's coefficients into geo[1])
    T nbl[C][N], mu_pre, tf_pre, gnb[8];
    if constexpr (!LA) face_prefetch<N, C, T, CURVED && !G7, D>(op, io, ci, s, nbl, mu_pre, tf_pre, gnb);
    constexpr int NN = N * N, NNN = N * N * N;
    constexpr int CS = Shape<N, C, sizeof(T) == 8>::CS;
    constexpr int t1 = D == 0 ? 1 : 0, t2 = D == 2 ? 1 : 2;
    const auto& tb = op.tab;
    const int i1 = ci.i1, i2 = ci.i2, t = ci.t;
    const int pos = D == 0 ? ci.ex : D == 1 ? ci.ey : ci.ez;
    const int lim = D == 0 ? op.nx : D == 1 ? op.ny : op.nz;
    const bool has_nb = s == 1 ? pos + 1 < lim : pos > 0;
    const int stride = D == 0 ? 1 : D == 1 ? op.nx : op.nx * op.ny;
    const int en = has_nb ? ci.ec + (s == 1 ? stride : -stride) : ci.ec;
    const bool dir = !has_nb && op.bc[2 * D + s] == 0;
    const bool live = ci.active && (has_nb ? (io.parts & SIPG_PART_INTERIOR) != 0
                                           : (dir && (io.parts & SIPG_PART_BOUNDARY) != 0));
    int fid;
    if (D == 0) fid = (ci.ez * op.ny + ci.ey) * (op.nx + 1) + ci.ex + s;
    else if (D == 1) fid = op.nfx + (ci.ez * (op.ny + 1) + ci.ey + s) * op.nx + ci.ex;
    else fid = op.nfx + op.nfy + ((ci.ez + s) * op.ny + ci.ey) * op.nx + ci.ex;
    if constexpr (LA) {
        // the look-ahead line is used as loaded (its traces are masked in
        // stage A); the face viscosity and penalty factor are loaded now,
        // used at the flux (masked by live there)
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int j = 0; j < N; ++j) nbl[c][j] = pre.nb[c][j];
        mu_pre = C == 3 ? op.mu_face[(size_t)fid * NN + ci.t] : T(1);
        tf_pre = op.tfac[fid];
    }
    constexpr bool DPP = Shape<N, C, sizeof(T) == 8>::DPP;
    constexpr bool MF = Shape<N, C, sizeof(T) == 8>::MF;
    // LDS regions of the work space, each [.][C][NN]
    T* FT = sw;               // [2] trace values (own, neighbour)          A  -> B1
    T* TD = sw + 2 * C * NN;  // [2][2] tangential derivatives (side, dir)  B1 -> B2
    T* BT = sw;               // [2] flux components along t1, t2           B2 -> C1
    T* VT = sw + 2 * C * NN;  // [2] transposed sweeps                      C1 -> C2
    T* VV = sw + (DPP || MF ? 0 : 6 * C * NN);  // [2] value / normal coefficients (D < 2)    C2

    // ---- A: traces
    T ju[C], uno[C], unn[C];  // jump u_own - u_nbr (mirror state on Dirichlet faces), normal derivatives
    T tv[C], tw[C];           // trace values of both sides (kept in registers for the cross-lane sweeps)
#pragma unroll
    for (int c = 0; c < C; ++c) {
        T v0 = 0, v1 = 0, w0 = 0, w1 = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            T own;
            if (D == 2) own = su[c * CS + vo.oz[j]];
            else if (D == 0) own = su[c * CS + vo.ox[j]];
            else own = su[c * CS + vo.oy[j]];
            v0 += tb.S[s][j] * own;
            v1 += tb.G[s][j] * own;
            w0 += tb.S[1 - s][j] * nbl[c][j];
            w1 += tb.G[1 - s][j] * nbl[c][j];
        }
        if constexpr (LA) {
            // the neighbour's traces, not its line, are masked (a select:
            // values of a cell without a live neighbour never enter)
            const bool ld = live && has_nb;
            w0 = ld ? w0 : T(0);
            w1 = ld ? w1 : T(0);
        }
        ju[c] = has_nb ? v0 - w0 : T(2) * v0;
        uno[c] = v1;
        unn[c] = w1;
        tv[c] = v0;
        tw[c] = w0;
        if constexpr (!DPP && !MF) {
            FT[c * NN + t] = v0;
            FT[(C + c) * NN + t] = w0;
        }
    }
    if constexpr (CURVED && !G7) {
        if (t < 3)
#pragma unroll
            for (int k = 0; k < 8; ++k) geo[1][k][t] = gnb[k];
    }
    if constexpr (LA) {
        // the traces are formed; after the last face a reload of it (unused),
        // so that the loads sit in no branch whose join would wait for them
        face_load_rt<N, C, T>(op, io, ci, fnext < 6 ? fnext : 5, pre);
    }
    if constexpr ((CURVED && !G7) || !(DPP || MF)) stage_sync<THREADS>();

    // ---- B1: tangential derivatives; task k = ((side*2 + dir)*C + c)*N + line
    // (n = 4: computed per lane from cross-lane moves or matrix-core products in B2)
    if constexpr (!DPP && !MF)
#pragma unroll
    for (int k0 = 0; k0 < 4 * C * N; k0 += NN) {
        const int k = k0 + t;
        if (k < 4 * C * N) {
            const int line = k % N, c = (k / N) % C, dirn = (k / (N * C)) % 2, side = k / (2 * N * C);
            const T* in = FT + (side * C + c) * NN;
            T* out = TD + ((side * 2 + dirn) * C + c) * NN;
            const int base = dirn == 0 ? line * N : line;
            const int step = dirn == 0 ? 1 : N;
            T v[N];
#pragma unroll
            for (int j = 0; j < N; ++j) v[j] = in[base + j * step];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                T a = 0;
#pragma unroll
                for (int j = 0; j < N; ++j) a += tb.D[q][j] * v[j];
                out[base + q * step] = a;
            }
        }
    }
    if constexpr (!DPP && !MF) stage_sync<THREADS>();

    // ---- B2: geometry and flux at the face point
    //
    // Own side: columns a_d = dx/dxi_d, adjugate rows c_d (c_0 = a_1 x a_2 and
    // cyclic), J^-1 = rows c_d / det.  The neighbour's Jacobian J' differs only
    // in column D, and its adjugate row D equals c_D, so with M = J'^-1 J
    // (identity except column D, v = J'^-1 a_D: v_D = det / det',
    // v_d = -(a'_D . c_d) / det' for d != D, det' = a'_D . c_D) the sum of the
    // two physical gradients is (gr + gr' M) J^-1: one transformation with the
    // own J^-1 for both sides.  The unit normal is sign * c_D / |c_D| and
    // ds = |c_D| w_a w_b.  On straight cells J^-1 = diag(1/h) and M = I.
    T xi[3];
    xi[t1] = lt.x[i1];
    xi[t2] = lt.x[i2];
    xi[D] = T(s);
    const T sgn = s == 1 ? T(1) : T(-1);
    T Cr[3][3], idet;  // rows c_d (curved: adjugate, 1/det; straight: J^-1, 1)
    T nrm[3], ds;
    T v[3];            // curved: column D of M
    if constexpr (CURVED) {
        T a[3][3];
        jac_columns(geo[0], xi, a);
        cross3(a[1], a[2], Cr[0]);
        cross3(a[2], a[0], Cr[1]);
        cross3(a[0], a[1], Cr[2]);
        const T det = a[0][0] * Cr[0][0] + a[0][1] * Cr[0][1] + a[0][2] * Cr[0][2];
        idet = recip(det);
        const T nv2 = Cr[D][0] * Cr[D][0] + Cr[D][1] * Cr[D][1] + Cr[D][2] * Cr[D][2];
        const T rinv = rsqrt_nr(nv2);
        const T sr = sgn * rinv;
        nrm[0] = Cr[D][0] * sr; nrm[1] = Cr[D][1] * sr; nrm[2] = Cr[D][2] * sr;
        ds = (nv2 * rinv) * (lt.w[i1] * lt.w[i2]);
        if (has_nb) {
            // the neighbour's xi_D column at the same face point
            T xin[3] = {xi[0], xi[1], xi[2]};
            xin[D] = T(1 - s);
            const T(*g)[3] = geo[G7 ? 1 + 2 * D + s : 1];
            T an[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if (D == 0) an[i] = g[1][i] + g[4][i] * xin[1] + g[5][i] * xin[2] + g[7][i] * (xin[1] * xin[2]);
                if (D == 1) an[i] = g[2][i] + g[4][i] * xin[0] + g[6][i] * xin[2] + g[7][i] * (xin[0] * xin[2]);
                if (D == 2) an[i] = g[3][i] + g[5][i] * xin[0] + g[6][i] * xin[1] + g[7][i] * (xin[0] * xin[1]);
            }
            const T rdn = recip(an[0] * Cr[D][0] + an[1] * Cr[D][1] + an[2] * Cr[D][2]);
#pragma unroll
            for (int d = 0; d < 3; ++d)
                v[d] = d == D ? det * rdn : -(an[0] * Cr[d][0] + an[1] * Cr[d][1] + an[2] * Cr[d][2]) * rdn;
        }
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) Cr[a][b] = a == b ? op.hinv[a] : T(0);
        idet = T(1);
        nrm[0] = nrm[1] = nrm[2] = T(0);
        nrm[D] = sgn;
        ds = op.h[t1] * op.h[t2] * (lt.w[i1] * lt.w[i2]);
    }
    // gs = gr + gr' M: reference gradient of both sides in the own frame
    // (Dirichlet mirror: grad u+ = grad u-, so gs = 2 gr)
    T gs[C][3];
    T da[DPP ? N : 1], db[DPP ? N : 1];  // this lane's rows of D along a and b (cross-lane sweeps)
    if constexpr (DPP) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            da[j] = lt.D[i1][ci.ra[j]];
            db[j] = lt.D[i2][ci.rb[j]];
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        // tangential derivatives of both traces (own: o1, o2; neighbour: n1, n2)
        T o1, o2, n1, n2;
        if constexpr (DPP) {
            T la[N], lb[N], ma[N], mb[N];
            line_a<N>(tv[c], la);
            line_b<N>(tv[c], lb);
            line_a<N>(tw[c], ma);
            line_b<N>(tw[c], mb);
            o1 = o2 = n1 = n2 = T(0);
#pragma unroll
            for (int j = 0; j < N; ++j) {
                o1 += da[j] * la[j];
                o2 += db[j] * lb[j];
                n1 += da[j] * ma[j];
                n2 += db[j] * mb[j];
            }
        } else if constexpr (MF) {
            // whole-wavefront products: outside any lane-dependent branch
            o1 = mf_r(tv[c], ci.md);
            n1 = mf_r(tw[c], ci.md);
            o2 = mf_c(tv[c], ci.md, ci.mi);
            n2 = mf_c(tw[c], ci.md, ci.mi);
        } else {
            o1 = TD[(0 * C + c) * NN + t];
            o2 = TD[(1 * C + c) * NN + t];
            n1 = TD[(2 * C + c) * NN + t];
            n2 = TD[(3 * C + c) * NN + t];
        }
        if constexpr (MF) {
            // selects, not branches, so that the products stay unconditional
            T gD = unn[c];
            if constexpr (CURVED) {
                T nr[3];
                nr[t1] = n1; nr[t2] = n2; nr[D] = unn[c];
                gD = nr[0] * v[0] + nr[1] * v[1] + nr[2] * v[2];
            }
            gs[c][t1] = o1 + (has_nb ? n1 : o1);
            gs[c][t2] = o2 + (has_nb ? n2 : o2);
            gs[c][D] = uno[c] + (has_nb ? gD : uno[c]);
        } else if (has_nb) {
            gs[c][t1] = o1 + n1;
            gs[c][t2] = o2 + n2;
            if constexpr (CURVED) {
                T nr[3];
                nr[t1] = n1; nr[t2] = n2; nr[D] = unn[c];
                gs[c][D] = uno[c] + (nr[0] * v[0] + nr[1] * v[1] + nr[2] * v[2]);
            } else {
                gs[c][D] = uno[c] + unn[c];
            }
        } else {
            gs[c][t1] = T(2) * o1;
            gs[c][t2] = T(2) * o2;
            gs[c][D] = T(2) * uno[c];
        }
    }
    // m' = adj n (J^-1 n = m' / det), p' = adj [u]
    T mo[3], p[3], en_[C];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        mo[d] = Cr[d][0] * nrm[0] + Cr[d][1] * nrm[1] + Cr[d][2] * nrm[2];
        if constexpr (C == 3) p[d] = Cr[d][0] * ju[0] + Cr[d][1] * ju[1] + Cr[d][2] * ju[2];
    }
    // viscous: (G + G^T) n of the summed gradient G = gs J^-1, with G n = gs m
    // and (G^T n)_c = sum_d J^-1[d][c] (n . gs[:, d]);  poisson: G . n
    if constexpr (C == 3) {
        T w[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) w[d] = nrm[0] * gs[0][d] + nrm[1] * gs[1][d] + nrm[2] * gs[2][d];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            en_[c] = (gs[c][0] * mo[0] + gs[c][1] * mo[1] + gs[c][2] * mo[2] +
                      Cr[0][c] * w[0] + Cr[1][c] * w[1] + Cr[2][c] * w[2]) * idet;
    } else {
        en_[0] = (gs[0][0] * mo[0] + gs[0][1] * mo[1] + gs[0][2] * mo[2]) * idet;
    }
    const T mu = (C == 3 && live) ? mu_pre : T(1);
    const T tau = live ? tf_pre * mu : T(0);
    const T lf = live ? T(1) : T(0);
    (void)fid;
    T av[C], Bh[C][3];
    if constexpr (C == 3) {
        // a = -2 {{mu eps(u)}} n + tau ([u] + n([u].n)),  B = -mu sym([u] (x) n),
        // B^ = J^-1 B:  B^[c][d] = -mu/2 (ju_c m_d + n_c p_d) / det
        const T jn = ju[0] * nrm[0] + ju[1] * nrm[1] + ju[2] * nrm[2];
        const T dl = ds * lf;
        const T hm = -T(0.5) * mu * dl * idet;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            av[c] = dl * (-T(0.5) * mu * en_[c] + tau * (ju[c] + nrm[c] * jn));
#pragma unroll
            for (int d = 0; d < 3; ++d) Bh[c][d] = hm * (ju[c] * mo[d] + nrm[c] * p[d]);
        }
    } else {
        // a = -{{grad u}}.n + tau [u],  B = -[u] n / 2,  B^ = -[u] m / 2
        const T dl = ds * lf;
        av[0] = dl * (-T(0.5) * en_[0] + tau * ju[0]);
        const T hb = -T(0.5) * dl * ju[0] * idet;
#pragma unroll
        for (int d = 0; d < 3; ++d) Bh[0][d] = hb * mo[d];
    }
    T vt[2][C];  // transposed tangential sweeps of the flux at this lane's point
    if constexpr (DPP) {
        T dat[N], dbt[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            dat[j] = lt.D[ci.ra[j]][i1];
            dbt[j] = lt.D[ci.rb[j]][i2];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            T la[N], lb[N];
            line_a<N>(Bh[c][t1], la);
            line_b<N>(Bh[c][t2], lb);
            T a1 = 0, a2 = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                a1 += dat[j] * la[j];
                a2 += dbt[j] * lb[j];
            }
            vt[0][c] = a1;
            vt[1][c] = a2;
        }
    } else if constexpr (MF) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            vt[0][c] = mf_r(Bh[c][t1], ci.mt);
            vt[1][c] = mf_c(Bh[c][t2], ci.mt, ci.mi);
        }
    } else {
    stage_sync<THREADS>();  // TD reads done before BT/VT overwrite the space
#pragma unroll
    for (int c = 0; c < C; ++c) {
        BT[c * NN + t] = Bh[c][t1];
        BT[(C + c) * NN + t] = Bh[c][t2];
    }
    stage_sync<THREADS>();

    // ---- C1: transposed tangential sweeps; task k = (dir*C + c)*N + line
#pragma unroll
    for (int k0 = 0; k0 < 2 * C * N; k0 += NN) {
        const int k = k0 + t;
        if (k < 2 * C * N) {
            const int line = k % N, c = (k / N) % C, dirn = k / (N * C);
            const T* in = BT + (dirn * C + c) * NN;
            T* out = VT + (dirn * C + c) * NN;
            const int base = dirn == 0 ? line * N : line;
            const int step = dirn == 0 ? 1 : N;
            T v[N];
#pragma unroll
            for (int q = 0; q < N; ++q) v[q] = in[base + q * step];
#pragma unroll
            for (int a = 0; a < N; ++a) {
                T acc = 0;
#pragma unroll
                for (int q = 0; q < N; ++q) acc += tb.D[q][a] * v[q];
                out[base + a * step] = acc;
            }
        }
    }
    stage_sync<THREADS>();
#pragma unroll
    for (int c = 0; c < C; ++c) {
        vt[0][c] = VT[c * NN + t];
        vt[1][c] = VT[(C + c) * NN + t];
    }
    }

    // ---- C2: projection onto the nodes
    T vv[C], vn[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        vv[c] = av[c] + vt[0][c] + vt[1][c];
        vn[c] = Bh[c][D];
    }
    if (D == 2) {
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int i3 = 0; i3 < N; ++i3) y[c][i3] += tb.S[s][i3] * vv[c] + tb.G[s][i3] * vn[c];
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            VV[c * NN + t] = vv[c];
            VV[(C + c) * NN + t] = vn[c];
        }
        stage_sync<THREADS>();
        // node (i1, i2, i3): D = 0 -> face point (i2, i3), normal index i1
        //                    D = 1 -> face point (i1, i3), normal index i2
        const int ni = D == 0 ? i1 : i2;
        const T sv = lt.S[s][ni], gv = lt.G[s][ni];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int i3 = 0; i3 < N; ++i3) {
                const int fp = D == 0 ? i3 * N + i2 : i3 * N + i1;
                y[c][i3] += sv * VV[c * NN + fp] + gv * VV[(C + c) * NN + fp];
            }
    }
    stage_sync<THREADS>();
}

// Face of the penalty-step operator (direction D, side s): only the jump of
// the normal component is penalised, tau_F ([v].n)([u].n), with [u] = u_own -
// u_nbr inside and u_own on a Dirichlet face (the oriented jump u - g; no
// mirror doubling).  Needs the traces of both sides, the unit normal and ds:
// no gradients, no tangential sweeps.
template <int N, typename T, bool CURVED, int D, int THREADS>
__device__ __forceinline__ void face_pass_pen(const OpData<T>& op, const ApplyIO<T>& io, const CellIdx& ci, int s,
                                              T (&y)[3][N], const T* su, T* sw, T (*geo)[8][3],
                                              const LaneTab<T, N>& lt, const VolOff<N>& vo) {
    constexpr int C = 3, NN = N * N, NNN = N * N * N;
    constexpr int CS = Shape<N, C, sizeof(T) == 8>::CS;
    constexpr int t1 = D == 0 ? 1 : 0, t2 = D == 2 ? 1 : 2;
    const auto& tb = op.tab;
    const int i1 = ci.i1, i2 = ci.i2, t = ci.t;
    const int pos = D == 0 ? ci.ex : D == 1 ? ci.ey : ci.ez;
    const int lim = D == 0 ? op.nx : D == 1 ? op.ny : op.nz;
    const bool has_nb = s == 1 ? pos + 1 < lim : pos > 0;
    const int stride = D == 0 ? 1 : D == 1 ? op.nx : op.nx * op.ny;
    const int en = has_nb ? ci.ec + (s == 1 ? stride : -stride) : ci.ec;
    const bool dir = !has_nb && op.bc[2 * D + s] == 0;
    const bool live = ci.active && (has_nb ? (io.parts & SIPG_PART_INTERIOR) != 0
                                           : (dir && (io.parts & SIPG_PART_BOUNDARY) != 0));
    int fid;
    if (D == 0) fid = (ci.ez * op.ny + ci.ey) * (op.nx + 1) + ci.ex + s;
    else if (D == 1) fid = op.nfx + (ci.ez * (op.ny + 1) + ci.ey + s) * op.nx + ci.ex;
    else fid = op.nfx + op.nfy + ((ci.ez + s) * op.ny + ci.ey) * op.nx + ci.ex;
    // neighbour line and face factor: every index is valid on every lane
    const T* xn = (io.xnb ? io.xnb : io.x) + (size_t)en * (C * NNN);
    T nbl[C][N];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            int off;
            if (D == 2) off = (c * N + j) * NN + i2 * N + i1;
            else if (D == 0) off = (c * N + i2) * NN + i1 * N + j;
            else off = (c * N + i2) * NN + j * N + i1;
            nbl[c][j] = xn[off];
        }
    const T tff = op.tfac[fid];
    // traces and the jump
    T ju[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        T v0 = 0, w0 = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            T own;
            if (D == 2) own = su[c * CS + vo.oz[j]];
            else if (D == 0) own = su[c * CS + vo.ox[j]];
            else own = su[c * CS + vo.oy[j]];
            v0 += tb.S[s][j] * own;
            w0 += tb.S[1 - s][j] * nbl[c][j];
        }
        ju[c] = has_nb ? v0 - w0 : v0;
    }
    // unit normal and surface measure: row D of the adjugate of J is normal to the face
    const T sgn = s == 1 ? T(1) : T(-1);
    T nrm[3], ds;
    if constexpr (CURVED) {
        T xi[3];
        xi[t1] = lt.x[i1];
        xi[t2] = lt.x[i2];
        xi[D] = T(s);
        T a[3][3], cD[3];
        jac_columns(geo[0], xi, a);
        cross3(a[(D + 1) % 3], a[(D + 2) % 3], cD);
        const T nv2 = cD[0] * cD[0] + cD[1] * cD[1] + cD[2] * cD[2];
        const T rinv = rsqrt_nr(nv2);
        nrm[0] = sgn * cD[0] * rinv; nrm[1] = sgn * cD[1] * rinv; nrm[2] = sgn * cD[2] * rinv;
        ds = (nv2 * rinv) * (lt.w[i1] * lt.w[i2]);
    } else {
        nrm[0] = nrm[1] = nrm[2] = T(0);
        nrm[D] = sgn;
        ds = op.h[t1] * op.h[t2] * (lt.w[i1] * lt.w[i2]);
    }
    const T jn = ju[0] * nrm[0] + ju[1] * nrm[1] + ju[2] * nrm[2];
    const T g = live ? ds * tff * jn : T(0);
    T av[C];
#pragma unroll
    for (int c = 0; c < C; ++c) av[c] = g * nrm[c];
    // projection onto the nodes: node (i1, i2, i3) gets S[s][i_D] av at its face point
    if constexpr (D == 2) {
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int i3 = 0; i3 < N; ++i3) y[c][i3] += tb.S[s][i3] * av[c];
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) sw[c * NN + t] = av[c];
        stage_sync<THREADS>();
        const int ni = D == 0 ? i1 : i2;
        const T sv = lt.S[s][ni];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int i3 = 0; i3 < N; ++i3) {
                const int fp = D == 0 ? i3 * N + i2 : i3 * N + i1;
                y[c][i3] += sv * sw[c * NN + fp];
            }
    }
    stage_sync<THREADS>();
}

// Cell term for n = 2 by slices xi_3 = const: the xi_1 and xi_2 derivatives
// of the own node come from cross-lane moves within the cell's quad, the
// stress is formed pointwise, and its xi_1 / xi_2 test-function sweeps go
// back across the lanes the same way; the xi_3 direction stays in the
// lane's registers (g3).  No LDS stores and no fences.  (For n = 4 the
// moves cost more than the LDS stages they replace.)
template <int N, int C, typename T, bool CURVED, bool PEN>
__device__ __forceinline__ void cell_pass_dpp(const OpData<T>& op, const CellIdx& ci, const T* su, T (*geo)[8][3],
                                              const LaneTab<T, N>& lt, const VolOff<N>& vo, T (&g3)[C][N],
                                              const T (&muq)[N], T (&y)[C][N]) {
    constexpr int CS = Shape<N, C, sizeof(T) == 8>::CS;
    const auto& tb = op.tab;
    const int i1 = ci.i1, i2 = ci.i2;
    T da[N], db[N], dat[N], dbt[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        da[j] = lt.D[i1][ci.ra[j]];
        db[j] = lt.D[i2][ci.rb[j]];
        dat[j] = lt.D[ci.ra[j]][i1];
        dbt[j] = lt.D[ci.rb[j]][i2];
    }
    // along the own xi_3 line the Jacobian columns of a trilinear cell are
    // a_0 = A0 + B0 xi_3, a_1 = A1 + B1 xi_3 and a_2 constant
    T A0[3], B0[3], A1[3], B1[3], a2c[3];
    if constexpr (CURVED) {
        const T(*g)[3] = geo[0];
        const T x1 = lt.x[i1], x2 = lt.x[i2];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            A0[i] = g[1][i] + g[4][i] * x2;
            B0[i] = g[5][i] + g[7][i] * x2;
            A1[i] = g[2][i] + g[4][i] * x1;
            B1[i] = g[6][i] + g[7][i] * x1;
            a2c[i] = g[3][i] + g[5][i] * x1 + g[6][i] * x2 + g[7][i] * (x1 * x2);
        }
    }
#pragma unroll
    for (int q3 = 0; q3 < N; ++q3) {
        T Ji[3][3], JxW;
        if constexpr (CURVED) {
            const T x3 = tb.x[q3];
            T a[3][3], det;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                a[0][i] = A0[i] + B0[i] * x3;
                a[1][i] = A1[i] + B1[i] * x3;
                a[2][i] = a2c[i];
            }
            inverse_from_columns(a, Ji, det);
            JxW = det * (lt.w[i1] * lt.w[i2] * tb.w[q3]);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) Ji[a][b] = a == b ? op.hinv[a] : T(0);
            JxW = op.h[0] * op.h[1] * op.h[2] * (lt.w[i1] * lt.w[i2] * tb.w[q3]);
        }
        T u[C], G[C][3];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            u[c] = su[c * CS + vo.oz[q3]];
            T la[N], lb[N];
            line_a<N>(u[c], la);
            line_b<N>(u[c], lb);
            T g1 = 0, g2 = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                g1 += da[j] * la[j];
                g2 += db[j] * lb[j];
            }
            const T gg3 = g3[c][q3];
#pragma unroll
            for (int i = 0; i < 3; ++i) G[c][i] = g1 * Ji[0][i] + g2 * Ji[1][i] + gg3 * Ji[2][i];
        }
        T S[C][3];
        if constexpr (PEN) {
            const T dv = muq[q3] * JxW * (G[0][0] + G[1][1] + G[2][2]);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) S[c][i] = c == i ? dv : T(0);
        } else if constexpr (C == 3) {
            const T f = muq[q3] * JxW;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) S[c][i] = f * (G[c][i] + G[i][c]);
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) S[0][i] = JxW * G[0][i];
        }
        const T mass = op.alpha * JxW;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const T b1 = Ji[0][0] * S[c][0] + Ji[0][1] * S[c][1] + Ji[0][2] * S[c][2];
            const T b2 = Ji[1][0] * S[c][0] + Ji[1][1] * S[c][1] + Ji[1][2] * S[c][2];
            g3[c][q3] = Ji[2][0] * S[c][0] + Ji[2][1] * S[c][1] + Ji[2][2] * S[c][2];
            T la[N], lb[N];
            line_a<N>(b1, la);
            line_b<N>(b2, lb);
            T acc = mass * u[c];
#pragma unroll
            for (int j = 0; j < N; ++j) acc += dat[j] * la[j] + dbt[j] * lb[j];
            y[c][q3] = acc;
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int i3 = 0; i3 < N; ++i3) {
            T acc = y[c][i3];
#pragma unroll
            for (int q = 0; q < N; ++q) acc += tb.D[q][i3] * g3[c][q];
            y[c][i3] = acc;
        }
}

// Cell term on the matrix cores (FP64 n = 4): the xi_1 and xi_2 derivatives
// of each xi_3 slice are tile products (mf_r, mf_c), the xi_3 derivative is
// the lane's own column (g3); the stress is formed pointwise and its xi_1 /
// xi_2 test-function sweeps are the transposed products.
template <int N, int C, typename T, bool CURVED, bool PEN>
__device__ __forceinline__ void cell_pass_mf(const OpData<T>& op, const CellIdx& ci, const T* su, T (*geo)[8][3],
                                             const LaneTab<T, N>& lt, const VolOff<N>& vo, T (&g3)[C][N],
                                             const T (&muq)[N], T (&y)[C][N]) {
    constexpr int CS = Shape<N, C, sizeof(T) == 8>::CS;
    const auto& tb = op.tab;
    const int i1 = ci.i1, i2 = ci.i2;
    T b1[C][N], b2[C][N];  // reference derivatives on the own column, then B^_1, B^_2
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const T u = su[c * CS + vo.oz[q]];
            b1[c][q] = mf_r(u, ci.md);
            b2[c][q] = mf_c(u, ci.md, ci.mi);
        }
    // pointwise, on the own xi_3 line: a_0 = A0 + B0 xi_3, a_1 = A1 + B1 xi_3, a_2 constant
    T A0[3], B0[3], A1[3], B1[3], a2c[3];
    if constexpr (CURVED) {
        const T(*g)[3] = geo[0];
        const T x1 = lt.x[i1], x2 = lt.x[i2];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            A0[i] = g[1][i] + g[4][i] * x2;
            B0[i] = g[5][i] + g[7][i] * x2;
            A1[i] = g[2][i] + g[4][i] * x1;
            B1[i] = g[6][i] + g[7][i] * x1;
            a2c[i] = g[3][i] + g[5][i] * x1 + g[6][i] * x2 + g[7][i] * (x1 * x2);
        }
    }
#pragma unroll
    for (int q3 = 0; q3 < N; ++q3) {
        T Ji[3][3], JxW;
        if constexpr (CURVED) {
            const T x3 = tb.x[q3];
            T a[3][3], det;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                a[0][i] = A0[i] + B0[i] * x3;
                a[1][i] = A1[i] + B1[i] * x3;
                a[2][i] = a2c[i];
            }
            inverse_from_columns(a, Ji, det);
            JxW = det * (lt.w[i1] * lt.w[i2] * tb.w[q3]);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) Ji[a][b] = a == b ? op.hinv[a] : T(0);
            JxW = op.h[0] * op.h[1] * op.h[2] * (lt.w[i1] * lt.w[i2] * tb.w[q3]);
        }
        T G[C][3];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const T g1 = b1[c][q3], g2 = b2[c][q3], gg3 = g3[c][q3];
#pragma unroll
            for (int i = 0; i < 3; ++i) G[c][i] = g1 * Ji[0][i] + g2 * Ji[1][i] + gg3 * Ji[2][i];
        }
        T S[C][3];
        if constexpr (PEN) {
            const T dv = muq[q3] * JxW * (G[0][0] + G[1][1] + G[2][2]);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) S[c][i] = c == i ? dv : T(0);
        } else if constexpr (C == 3) {
            const T f = muq[q3] * JxW;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) S[c][i] = f * (G[c][i] + G[i][c]);
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) S[0][i] = JxW * G[0][i];
        }
        const T mass = op.alpha * JxW;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            b1[c][q3] = Ji[0][0] * S[c][0] + Ji[0][1] * S[c][1] + Ji[0][2] * S[c][2];
            b2[c][q3] = Ji[1][0] * S[c][0] + Ji[1][1] * S[c][1] + Ji[1][2] * S[c][2];
            g3[c][q3] = Ji[2][0] * S[c][0] + Ji[2][1] * S[c][1] + Ji[2][2] * S[c][2];
            y[c][q3] = mass * su[c * CS + vo.oz[q3]];
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int i3 = 0; i3 < N; ++i3) {
            T acc = y[c][i3] + mf_r(b1[c][i3], ci.mt) + mf_c(b2[c][i3], ci.mt, ci.mi);
#pragma unroll
            for (int q = 0; q < N; ++q) acc += tb.D[q][i3] * g3[c][q];
            y[c][i3] = acc;
        }
}

// ---------------------------------------------------------------- kernel

template <int N, int C, typename T, bool CURVED, int MODE, bool PEN>
__global__ void __launch_bounds__((Shape<N, C, sizeof(T) == 8>::THREADS)) __attribute__((amdgpu_waves_per_eu(2)))
    k_apply(const OpData<T> op, const ApplyIO<T> io) {
    using Sh = Shape<N, C, sizeof(T) == 8>;
    constexpr int NN = N * N, NNN = N * N * N;
    constexpr int CPB = Sh::CPB, THREADS = Sh::THREADS;
    constexpr int S3 = Sh::S3, CS = Sh::CS;
    constexpr bool SKEW = Sh::SKEW;

    if (io.skip != nullptr && *io.skip) return;  // uniform over the grid

    __shared__ T s_u[CPB][Sh::U];      // the cell's nodal values
    __shared__ T s_w[CPB][Sh::W];      // work space of the cell and face passes
    // own / neighbour trilinear coefficients, [2][8][3] per cell; the odd cell
    // stride puts the four cells of a wavefront on different banks (their
    // reads are per-cell broadcasts)
    // G7 (curved cells, all six faces computed; FP64 n = 4 and FP32 n >= 5):
    // the cell's and its six face neighbours' trilinear coefficients,
    // [7][8][3] per cell plus 8 spare slots for lanes without a task, loaded
    // with the nodal values.  Measured per instance: c2 FP64 116 -> 111 us,
    // c3 FP32 82 -> 70 us; slower for FP64 n = 5 (133 -> 142 us, its
    // registers are full) and FP32 n = 4 (71 -> 73 us); for n <= 3 a cell has
    // too few lanes for the 21 tasks.  LA (where the registers fit: every
    // G7 instance, FP64 n = 4 and FP32 n = 5, 6): each face's neighbour line
    // loaded during the previous face (FP32 n = 5: 151 -> 165 VGPRs, still
    // 3 wavefronts per SIMD; c3 FP32 apply 69.4 -> 66.9 us)
    constexpr bool G7 = CURVED && !PEN && MODE != MODE_CONT && (Sh::MF || (sizeof(T) == 4 && N >= 5));
    constexpr bool LA = G7;
    constexpr int GS = G7 ? 7 * 8 * 3 + 9 : 2 * 8 * 3 + 1;
    __shared__ T s_geo_all[CPB * GS];
    __shared__ LaneTab<T, N> s_lt;

    CellIdx ci;
    if constexpr (Sh::MF) {
        // lane 16 i1 + 4 cell + i2 (the matrix-core tile layout)
        ci.lc = (threadIdx.x >> 2) & 3;
        ci.i1 = threadIdx.x >> 4;
        ci.i2 = threadIdx.x & 3;
        ci.t = ci.i2 * N + ci.i1;
    } else {
        ci.lc = threadIdx.x / NN;
        ci.t = threadIdx.x - ci.lc * NN;
        ci.i1 = ci.t % N;
        ci.i2 = ci.t / N;
    }
    const int e = xcd_block(blockIdx.x, gridDim.x) * CPB + ci.lc;
    ci.active = e < op.ncell;
    {
        // rank r -> cell: the mesh is cut into octants (halves along each
        // axis, floor / ceil for odd counts), taken in z, y, x order, each
        // lexicographic inside.  With the XCD-aware block order each XCD's
        // contiguous share of ranks is about one octant, so a cell's face
        // neighbours are mostly read by the same XCD within a few layers of
        // its octant (a hit in that XCD's L2) instead of one full mesh layer
        // apart.  Measured: c4v FP64 apply 130 -> 125 us, c2 and c3 unchanged
        // within the noise.
        const int r = ci.active ? e : 0;
        const int lx = op.nx >> 1, ly = op.ny >> 1, lz = op.nz >> 1;
        const int sZ = op.nx * op.ny * lz;
        const int oz = r >= sZ, sz = oz ? op.nz - lz : lz, r1 = r - (oz ? sZ : 0);
        const int sY = op.nx * ly * sz;
        const int oy = r1 >= sY, sy = oy ? op.ny - ly : ly, r2 = r1 - (oy ? sY : 0);
        const int sX = lx * sy * sz;
        const int ox = r2 >= sX, sx = ox ? op.nx - lx : lx, r3 = r2 - (ox ? sX : 0);
        const int q = r3 / sx;
        ci.ex = (ox ? lx : 0) + (r3 - q * sx);
        ci.ey = (oy ? ly : 0) + q % sy;
        ci.ez = (oz ? lz : 0) + q / sy;
        ci.ec = (ci.ez * op.ny + ci.ey) * op.nx + ci.ex;
    }
    const int lc = ci.lc, t = ci.t, i1 = ci.i1, i2 = ci.i2;
    T(*geo)[8][3] = reinterpret_cast<T(*)[8][3]>(s_geo_all + lc * GS);
    const auto& tb = op.tab;
    T* su = s_u[lc];
    T* sw = s_w[lc];
    // thread t as a line: (la, lb) = (i2, i3) for xi_1 sweeps, (i1, i3) for xi_2 sweeps
    const int la = t % N, lb = t / N;
    VolOff<N> vo;
    vol_offsets<N, S3, SKEW>(la, lb, lc, vo);

    if (threadIdx.x < N) {
        const int j = threadIdx.x;
        s_lt.x[j] = tb.x[j];
        s_lt.w[j] = tb.w[j];
        s_lt.S[0][j] = tb.S[0][j];
        s_lt.S[1][j] = tb.S[1][j];
        s_lt.G[0][j] = tb.G[0][j];
        s_lt.G[1][j] = tb.G[1][j];
#pragma unroll
        for (int q = 0; q < N; ++q) s_lt.D[q][j] = tb.D[q][j];
    }
    if constexpr (Sh::DPP) {
        // which a / b each slot of line_a / line_b delivers, read off the lane
        // index itself (no assumption on the direction of a rotation)
        ci.ra[0] = i1;
        ci.rb[0] = i2;
        if constexpr (N == 4) {
            ci.rb[1] = dpp_i<0x124>(t) / N;
            ci.rb[2] = dpp_i<0x128>(t) / N;
            ci.rb[3] = dpp_i<0x12C>(t) / N;
            ci.ra[1] = dpp_i<0x39>(t) % N;
            ci.ra[2] = dpp_i<0x4E>(t) % N;
            ci.ra[3] = dpp_i<0x93>(t) % N;
        } else {
            ci.ra[1] = dpp_i<0xB1>(t) % N;
            ci.rb[1] = dpp_i<0x4E>(t) / N;
        }
    }

    // ------------------------------------------------------------ load; xi_3 derivative of the own line
    constexpr int GR = G7 ? (21 + NN - 1) / NN : 1;   // rounds of the 21 staging tasks over a cell's n^2 lanes
    T gt[GR][8];
    int gslot[GR], gcrd[GR];
    if constexpr (G7) {
        // 21 tasks (7 cells x 3 coordinates): lane t takes tasks t, t + n^2, ...;
        // slot 0 = the cell, slot 1 + f = the neighbour across face f = 2 D + s (the cell itself on the boundary)
        auto cell_of = [&](int slot, int& cx, int& cy, int& cz) {
            cx = ci.ex; cy = ci.ey; cz = ci.ez;
            if (slot > 0) {
                const int f = slot - 1, D = f >> 1, sd = f & 1;
                if (D == 0) cx += sd ? (cx + 1 < op.nx ? 1 : 0) : (cx > 0 ? -1 : 0);
                else if (D == 1) cy += sd ? (cy + 1 < op.ny ? 1 : 0) : (cy > 0 ? -1 : 0);
                else cz += sd ? (cz + 1 < op.nz ? 1 : 0) : (cz > 0 ? -1 : 0);
            }
        };
#pragma unroll
        for (int r = 0; r < GR; ++r) {
            const int task = t + r * NN;
            const int tk = task < 21 ? task : 0;   // past the last task: a duplicate of task 0, stored into the spare slots
            int cx, cy, cz;
            cell_of(tk / 3, cx, cy, cz);
            trilinear_coeffs(op.verts, op.nx, op.ny, cx, cy, cz, tk % 3, gt[r]);
            gslot[r] = task < 21 ? tk / 3 : 7;
            gcrd[r] = tk % 3;
        }
    } else if constexpr (CURVED) {
        trilinear_coeffs(op.verts, op.nx, op.ny, ci.ex, ci.ey, ci.ez, t % 3, gt[0]);
    }
    T muq[N];  // viscosity on the own xi_3 line of quadrature points, loaded with the nodal values
    if constexpr (C == 3)
#pragma unroll
        for (int q3 = 0; q3 < N; ++q3) muq[q3] = op.mu_cell[(size_t)ci.ec * NNN + q3 * NN + t];
    T g3[C][N];
    if constexpr (MODE == MODE_CONT) {
        // the cell's Lobatto values (own xi_3 column (i1, i2, .) per thread),
        // then Lobatto -> Gauss along xi_1 and xi_2 (lines, in place in LDS)
        // and xi_3 (own column, in registers)
        const int jd = io.cj;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const T v = io.x[c * io.cnv + ((long long)(ci.ez * jd + j) * io.cMy + ci.ey * jd + i2) * io.cMx +
                                 ci.ex * jd + i1];  // ec = 0 on inactive lanes: in bounds
                su[c * CS + vo.oz[j]] = ci.active ? v : T(0);
            }
        stage_sync<THREADS>();
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                T v[N];
#pragma unroll
                for (int a = 0; a < N; ++a) v[a] = su[c * CS + (pass == 0 ? vo.ox[a] : vo.oy[a])];
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    T acc = 0;
#pragma unroll
                    for (int a = 0; a < N; ++a) acc += io.cL[q][a] * v[a];
                    su[c * CS + (pass == 0 ? vo.ox[q] : vo.oy[q])] = acc;
                }
            }
            stage_sync<THREADS>();
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            T v[N], col[N];
#pragma unroll
            for (int a = 0; a < N; ++a) v[a] = su[c * CS + vo.oz[a]];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                T acc = 0;
#pragma unroll
                for (int a = 0; a < N; ++a) acc += io.cL[q][a] * v[a];
                col[q] = acc;
            }
#pragma unroll
            for (int q = 0; q < N; ++q) {
                su[c * CS + vo.oz[q]] = col[q];
                T a = 0;
#pragma unroll
                for (int j = 0; j < N; ++j) a += tb.D[q][j] * col[j];
                g3[c][q] = a;
            }
        }
    } else {
        const T* xe = io.x + (size_t)ci.ec * (C * NNN);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            T col[N];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const T v = xe[(c * N + j) * NN + t];  // ec = 0 on inactive lanes: in bounds
                col[j] = ci.active ? v : T(0);
                su[c * CS + vo.oz[j]] = col[j];
            }
#pragma unroll
            for (int q = 0; q < N; ++q) {
                T a = 0;
#pragma unroll
                for (int j = 0; j < N; ++j) a += tb.D[q][j] * col[j];
                g3[c][q] = a;
            }
        }
    }
    if constexpr (G7) {
        T* gl = s_geo_all + lc * GS;
#pragma unroll
        for (int r = 0; r < GR; ++r)
#pragma unroll
            for (int k = 0; k < 8; ++k) gl[gslot[r] < 7 ? (gslot[r] * 8 + k) * 3 + gcrd[r] : 7 * 24 + k] = gt[r][k];
    } else if constexpr (CURVED) {
        // unconditional stores keep the loads at the top (lanes t >= 3 write into the
        // neighbour slot, which every face stage rewrites before reading it)
#pragma unroll
        for (int k = 0; k < 8; ++k) *(t < 3 ? &geo[0][k][t] : &geo[1][k][0]) = gt[0][k];
    }
    __syncthreads();
    const LaneTab<T, N>& lt = s_lt;
    if constexpr (Sh::MF) {
        ci.md = lt.D[i2][i1];
        ci.mt = lt.D[i1][i2];
        ci.mi = i1 == i2 ? 1.0 : 0.0;
    }

    T y[C][N];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int j = 0; j < N; ++j) y[c][j] = T(0);

    // ------------------------------------------------------------ cell
    if constexpr (N == 2) {
        if (io.parts & SIPG_PART_CELL) cell_pass_dpp<N, C, T, CURVED, PEN>(op, ci, su, geo, lt, vo, g3, muq, y);
    } else if constexpr (Sh::MF) {
        if (io.parts & SIPG_PART_CELL) cell_pass_mf<N, C, T, CURVED, PEN>(op, ci, su, geo, lt, vo, g3, muq, y);
    } else if (io.parts & SIPG_PART_CELL) {
        T* W1 = sw;            // [C][NNN] d/dxi_1, then B^_1
        T* W2 = sw + C * CS;  // [C][NNN] d/dxi_2, then B^_2
        // forward sweeps along xi_1 and xi_2
#pragma unroll
        for (int c = 0; c < C; ++c) {
            T v[N], w[N];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                v[j] = su[c * CS + vo.ox[j]];
                w[j] = su[c * CS + vo.oy[j]];
            }
#pragma unroll
            for (int q = 0; q < N; ++q) {
                T a = 0, b = 0;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    a += tb.D[q][j] * v[j];
                    b += tb.D[q][j] * w[j];
                }
                W1[c * CS + vo.ox[q]] = a;
                W2[c * CS + vo.oy[q]] = b;
            }
        }
        stage_sync<THREADS>();
        // pointwise, on the own xi_3 line of quadrature points.  Along that
        // line the Jacobian columns of a trilinear cell are a_0 = A0 + B0 xi_3,
        // a_1 = A1 + B1 xi_3 and a_2 constant.
        T A0[3], B0[3], A1[3], B1[3], a2c[3];
        if constexpr (CURVED) {
            const T(*g)[3] = geo[0];
            const T x1 = lt.x[i1], x2 = lt.x[i2];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                A0[i] = g[1][i] + g[4][i] * x2;
                B0[i] = g[5][i] + g[7][i] * x2;
                A1[i] = g[2][i] + g[4][i] * x1;
                B1[i] = g[6][i] + g[7][i] * x1;
                a2c[i] = g[3][i] + g[5][i] * x1 + g[6][i] * x2 + g[7][i] * (x1 * x2);
            }
        }
#pragma unroll
        for (int q3 = 0; q3 < N; ++q3) {
            T Ji[3][3], JxW;
            if constexpr (CURVED) {
                const T x3 = tb.x[q3];
                T a[3][3], det;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    a[0][i] = A0[i] + B0[i] * x3;
                    a[1][i] = A1[i] + B1[i] * x3;
                    a[2][i] = a2c[i];
                }
                inverse_from_columns(a, Ji, det);
                JxW = det * (lt.w[i1] * lt.w[i2] * tb.w[q3]);
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) Ji[a][b] = a == b ? op.hinv[a] : T(0);
                JxW = op.h[0] * op.h[1] * op.h[2] * (lt.w[i1] * lt.w[i2] * tb.w[q3]);
            }
            T G[C][3];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const T g1 = W1[c * CS + vo.oz[q3]], g2 = W2[c * CS + vo.oz[q3]], gg3 = g3[c][q3];
#pragma unroll
                for (int i = 0; i < 3; ++i) G[c][i] = g1 * Ji[0][i] + g2 * Ji[1][i] + gg3 * Ji[2][i];
            }
            T S[C][3];
            if constexpr (PEN) {
                // penalty step: tau_div div(u) I JxW (muq holds tau_div)
                const T dv = muq[q3] * JxW * (G[0][0] + G[1][1] + G[2][2]);
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int i = 0; i < 3; ++i) S[c][i] = c == i ? dv : T(0);
            } else if constexpr (C == 3) {
                const T f = muq[q3] * JxW;  // 2 mu eps = mu (G + G^T)
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int i = 0; i < 3; ++i) S[c][i] = f * (G[c][i] + G[i][c]);
            } else {
#pragma unroll
                for (int i = 0; i < 3; ++i) S[0][i] = JxW * G[0][i];
            }
            const T mass = op.alpha * JxW;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                W1[c * CS + vo.oz[q3]] = Ji[0][0] * S[c][0] + Ji[0][1] * S[c][1] + Ji[0][2] * S[c][2];
                W2[c * CS + vo.oz[q3]] = Ji[1][0] * S[c][0] + Ji[1][1] * S[c][1] + Ji[1][2] * S[c][2];
                g3[c][q3] = Ji[2][0] * S[c][0] + Ji[2][1] * S[c][1] + Ji[2][2] * S[c][2];
                y[c][q3] = mass * su[c * CS + vo.oz[q3]];
            }
        }
        stage_sync<THREADS>();
        // transposed sweeps, in place on the lines (each line is read and written by one thread)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            T v[N], w[N];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                v[q] = W1[c * CS + vo.ox[q]];
                w[q] = W2[c * CS + vo.oy[q]];
            }
#pragma unroll
            for (int j = 0; j < N; ++j) {
                T a = 0, b = 0;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    a += tb.D[q][j] * v[q];
                    b += tb.D[q][j] * w[q];
                }
                W1[c * CS + vo.ox[j]] = a;
                W2[c * CS + vo.oy[j]] = b;
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int i3 = 0; i3 < N; ++i3) {
                T acc = y[c][i3];
#pragma unroll
                for (int q = 0; q < N; ++q) acc += tb.D[q][i3] * g3[c][q];
                y[c][i3] = acc;
            }
        stage_sync<THREADS>();
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int i3 = 0; i3 < N; ++i3) y[c][i3] += W1[c * CS + vo.oz[i3]] + W2[c * CS + vo.oz[i3]];
        stage_sync<THREADS>();
    }

    // ------------------------------------------------------------ faces
    if (io.parts & (SIPG_PART_INTERIOR | SIPG_PART_BOUNDARY)) {
        // boundary terms only (the continuous levels of the multigrid
        // preconditioner): a face pass that no cell of the workgroup needs
        // is skipped as a whole (the vote is uniform over the workgroup)
        const bool only_boundary = (io.parts & SIPG_PART_INTERIOR) == 0;
        FacePre<N, C, T> pre;
        if constexpr (LA) face_load_rt<N, C, T>(op, io, ci, 0, pre);
        // the six faces unrolled: a loop whose body branches to the three
        // direction variants makes the compiler copy every loop-carried
        // register (the accumulators y, the look-ahead line) at the latch,
        // after waiting for the look-ahead loads; unrolled, the face
        // variants are inlined in sequence with no copies.  It also lowers
        // the register count by 10-45 per instance (n = 6 FP64 loses its
        // spills).  Measured: c2 FP64 109 -> 103.5 us, c4v FP64 125 -> 113
        // us, c3 FP64 130 -> 128 us; FP32 n = 4 (the cross-lane version)
        // was 3 % slower unrolled and keeps the loop
        constexpr int FU = (sizeof(T) == 4 && N == 4) ? 1 : 6;
#pragma unroll FU
        for (int f = 0; f < 6; ++f) {
            const int s = f & 1;
            if (only_boundary) {
                const int D = f >> 1;
                const int pos = D == 0 ? ci.ex : D == 1 ? ci.ey : ci.ez;
                const int lim = D == 0 ? op.nx : D == 1 ? op.ny : op.nz;
                const bool wall = s == 1 ? pos + 1 >= lim : pos == 0;
                const bool need = ci.active && wall && op.bc[2 * D + s] == 0;
                bool any;
                if constexpr (THREADS <= 64) any = __ballot(need) != 0;
                else any = __syncthreads_or(need) != 0;
                if (!any) {
                    if constexpr (LA) {
                        if (f + 1 < 6) face_load_rt<N, C, T>(op, io, ci, f + 1, pre);
                    }
                    continue;
                }
            }
            if constexpr (PEN) {
                if (f < 2) face_pass_pen<N, T, CURVED, 0, THREADS>(op, io, ci, s, y, su, sw, geo, lt, vo);
                else if (f < 4) face_pass_pen<N, T, CURVED, 1, THREADS>(op, io, ci, s, y, su, sw, geo, lt, vo);
                else face_pass_pen<N, T, CURVED, 2, THREADS>(op, io, ci, s, y, su, sw, geo, lt, vo);
            } else {
                if (f < 2) face_pass<N, C, T, CURVED, 0, THREADS, G7, LA>(op, io, ci, s, y, su, sw, geo, lt, vo, pre, f + 1);
                else if (f < 4) face_pass<N, C, T, CURVED, 1, THREADS, G7, LA>(op, io, ci, s, y, su, sw, geo, lt, vo, pre, f + 1);
                else face_pass<N, C, T, CURVED, 2, THREADS, G7, LA>(op, io, ci, s, y, su, sw, geo, lt, vo, pre, f + 1);
            }
        }
    }

    // ------------------------------------------------------------ store
    if constexpr (MODE == MODE_CONT) {
        // local contributions G_e^T y: Gauss -> Lobatto transposed along xi_3
        // (own column), then xi_2 and xi_1 (lines in LDS; every lane takes
        // part, inactive cells write nothing)
        stage_sync<THREADS>();   // the face passes' last reads of su
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int a = 0; a < N; ++a) {
                T acc = 0;
#pragma unroll
                for (int q = 0; q < N; ++q) acc += io.cL[q][a] * y[c][q];
                su[c * CS + vo.oz[a]] = acc;
            }
        stage_sync<THREADS>();
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                T v[N];
#pragma unroll
                for (int q = 0; q < N; ++q) v[q] = su[c * CS + (pass == 0 ? vo.oy[q] : vo.ox[q])];
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    T acc = 0;
#pragma unroll
                    for (int q = 0; q < N; ++q) acc += io.cL[q][a] * v[q];
                    su[c * CS + (pass == 0 ? vo.oy[a] : vo.ox[a])] = acc;
                }
            }
            stage_sync<THREADS>();
        }
        if (!ci.active) return;
        const size_t base = (size_t)ci.ec * (C * NNN);
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int j = 0; j < N; ++j) io.y[base + (c * N + j) * NN + t] = su[c * CS + vo.oz[j]];
        return;
    }
    if (!ci.active) return;
    const size_t base = (size_t)ci.ec * (C * NNN);
    if constexpr (MODE == MODE_APPLY) {
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int j = 0; j < N; ++j) io.y[base + (c * N + j) * NN + t] = y[c][j];
    } else if constexpr (MODE == MODE_RESID) {
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const size_t idx = base + (c * N + j) * NN + t;
                io.y[idx] = io.r[idx] - y[c][j];
            }
    } else {
        const T c1 = T(io.coef[0]), c2 = T(io.coef[1]);
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const size_t idx = base + (c * N + j) * NN + t;
                const T dn = c1 * io.d[idx] + c2 * io.dinv[idx] * (io.r[idx] - y[c][j]);
                io.d[idx] = dn;
                io.y[idx] = su[c * CS + vo.oz[j]] + dn;
            }
    }
}

}  // namespace sipg
