// Device helpers: trilinear cell geometry, viscosity laws, block mapping.
#pragma once

#include "sipg_internal.h"

namespace sipg {

// Monomial form of the trilinear map of one cell, for one coordinate i:
//   x_i(xi) = g0 + g1 xi1 + g2 xi2 + g3 xi3 + g4 xi1 xi2 + g5 xi1 xi3
//           + g6 xi2 xi3 + g7 xi1 xi2 xi3,
// from the 8 vertex coordinates X_abc (a along xi1, b along xi2, c along xi3).
// 32-bit offsets: the plan rejects meshes with 2^31 or more vertex coordinates.
template <typename T>
__device__ __forceinline__ void trilinear_coeffs(const T* verts, int nx, int ny, int ex, int ey,
                                                 int ez, int i, T g[8]) {
    const int sy = 3 * (nx + 1), sz = sy * (ny + 1);
    const int base = ez * sz + ey * sy + ex * 3 + i;
    auto X = [&](int a, int b, int c) { return verts[base + c * sz + b * sy + a * 3]; };
    const T x000 = X(0, 0, 0), x100 = X(1, 0, 0), x010 = X(0, 1, 0), x001 = X(0, 0, 1);
    const T x110 = X(1, 1, 0), x101 = X(1, 0, 1), x011 = X(0, 1, 1), x111 = X(1, 1, 1);
    g[0] = x000;
    g[1] = x100 - x000;
    g[2] = x010 - x000;
    g[3] = x001 - x000;
    g[4] = (x110 - x100) - (x010 - x000);
    g[5] = (x101 - x100) - (x001 - x000);
    g[6] = (x011 - x010) - (x001 - x000);
    g[7] = ((x111 - x110) - (x101 - x100)) - ((x011 - x010) - (x001 - x000));
}

// Inverse Jacobian Ji[d][i] = d xi_d / d x_i and det J at reference point
// (x1, x2, x3), from monomial coefficients geo[k][i] (k = 0..7, i = 0..2).
// Rows of J^-1 are cross products of the columns a_d = d x / d xi_d.
template <typename T>
__device__ __forceinline__ void jacobian_inverse(const T (*geo)[3], T x1, T x2, T x3,
                                                 T Ji[3][3], T& det) {
    T a0[3], a1[3], a2[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        a0[i] = geo[1][i] + geo[4][i] * x2 + geo[5][i] * x3 + geo[7][i] * (x2 * x3);
        a1[i] = geo[2][i] + geo[4][i] * x1 + geo[6][i] * x3 + geo[7][i] * (x1 * x3);
        a2[i] = geo[3][i] + geo[5][i] * x1 + geo[6][i] * x2 + geo[7][i] * (x1 * x2);
    }
    T c12[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2],
                a1[0] * a2[1] - a1[1] * a2[0]};
    T c20[3] = {a2[1] * a0[2] - a2[2] * a0[1], a2[2] * a0[0] - a2[0] * a0[2],
                a2[0] * a0[1] - a2[1] * a0[0]};
    T c01[3] = {a0[1] * a1[2] - a0[2] * a1[1], a0[2] * a1[0] - a0[0] * a1[2],
                a0[0] * a1[1] - a0[1] * a1[0]};
    det = a0[0] * c12[0] + a0[1] * c12[1] + a0[2] * c12[2];
    const T inv = T(1) / det;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Ji[0][i] = c12[i] * inv;
        Ji[1][i] = c20[i] * inv;
        Ji[2][i] = c01[i] * inv;
    }
}

template <typename T>
__device__ __forceinline__ void map_point(const T (*geo)[3], T x1, T x2, T x3, T X[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
        X[i] = geo[0][i] + geo[1][i] * x1 + geo[2][i] * x2 + geo[3][i] * x3 + geo[4][i] * (x1 * x2) +
               geo[5][i] * (x1 * x3) + geo[6][i] * (x2 * x3) + geo[7][i] * (x1 * x2 * x3);
}

// Monomial coefficients geo[k][i] of cell e: from the vertices, or for the
// straight unit box x_i = (pos_i + xi_i) h_i.
__device__ inline void cell_geo_full(const OpData<double>& op, int e, double geo[8][3]) {
    const int ex = e % op.nx, ey = (e / op.nx) % op.ny, ez = e / (op.nx * op.ny);
    for (int i = 0; i < 3; ++i) {
        double g[8];
        if (op.verts) {
            trilinear_coeffs(op.verts, op.nx, op.ny, ex, ey, ez, i, g);
        } else {
            for (int k = 0; k < 8; ++k) g[k] = 0.0;
            const int pos = i == 0 ? ex : i == 1 ? ey : ez;
            g[0] = pos * op.h[i];
            g[1 + i] = op.h[i];
        }
        for (int k = 0; k < 8; ++k) geo[k][i] = g[k];
    }
}

// Viscosity laws (Sec. 2 and smooth prescribed fields), FP64.
__device__ inline double law_value(const LawDev& L, const double X[3]) {
    const double twopi = 6.283185307179586476925286766559;
    switch (L.kind) {
        case SIPG_LAW_CONST:
            return L.mu;
        case SIPG_LAW_SINE:
            return L.mu * (1.0 + L.amp * sin(twopi * X[0]) * sin(twopi * X[1]) * sin(twopi * X[2]));
        case SIPG_LAW_LOGFIELD: {
            double r = 0.0;
            for (int m = 0; m < L.n_modes; ++m) {
                const double kx = L.k[m][0] * X[0] + L.k[m][1] * X[1] + L.k[m][2] * X[2];
                r += L.a[m] * cos(twopi * kx + L.phi[m]);
            }
            double s = (r - L.rmin) / (L.rmax - L.rmin);
            s = fmin(fmax(s, 0.0), 1.0);
            return pow(L.contrast, s);
        }
        case SIPG_LAW_CARREAU: {
            double gw[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // d w_i / d x_j
            for (int m = 0; m < L.n_modes; ++m) {
                const double kx = L.k[m][0] * X[0] + L.k[m][1] * X[1] + L.k[m][2] * X[2];
                const double sn = -twopi * sin(twopi * kx + L.phi[m]);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) gw[i][j] += sn * L.v[m][i] * L.k[m][j];
            }
            double ee = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    const double e = 0.5 * (gw[i][j] + gw[j][i]);
                    ee += e * e;
                }
            const double gdot = sqrt(2.0 * ee);
            return L.mu_inf + (L.mu0 - L.mu_inf) *
                                  pow(L.kappa + pow(L.lam * gdot, L.a_exp), (L.n_exp - 1.0) / L.a_exp);
        }
    }
    return 0.0;
}

// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X, each
// with its own L2.  Remap so that XCD x handles one contiguous range of cell
// blocks: neighbouring cells, whose traces every face term re-reads, then
// share an L2.  Bijective on [0, nblocks).
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
    constexpr int kXcd = 8;
    const int per = nblocks / kXcd, rem = nblocks % kXcd;
    const int x = b % kXcd, slot = b / kXcd;
    return x * per + (x < rem ? x : rem) + slot;
}

}  // namespace sipg
