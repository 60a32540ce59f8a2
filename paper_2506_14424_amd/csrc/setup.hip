// Plan setup on the device: cell sizes, penalty factors, viscosity at the
// quadrature points (Sec. 4.1 stores the viscosity pointwise) and the matrix
// diagonal with its inverse (Sec. 5.3, for the Jacobi-type smoother).

#include "device_common.h"

namespace sipg {

// ---------------------------------------------------------------- geometry

// Per cell: h_e = |e|^(1/3) into hcell[e], and the penalty's surface-to-volume
// ratio sigma_e = (sum_f w_f |f|) / |e| into hcell[ncell + e], w_f = 1/2 for a
// face shared with another cell and 1 on the boundary of the box.  Volume and
// face areas by the n-point Gauss rules (exact for the volume of a trilinear
// cell); the area element of face xi_d = s is |a_t1 x a_t2|, the length of
// the adjugate row d.
__global__ void k_cell_size(const OpData<double> op, int n, double* hcell) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= op.ncell) return;
    const int ex = e % op.nx, ey = (e / op.nx) % op.ny, ez = e / (op.nx * op.ny);
    double vol = 0.0, area[3][2];
    if (op.verts) {
        double geo[8][3];
        cell_geo_full(op, e, geo);
        for (int q3 = 0; q3 < n; ++q3)
            for (int q2 = 0; q2 < n; ++q2)
                for (int q1 = 0; q1 < n; ++q1) {
                    double Ji[3][3], det;
                    jacobian_inverse<double>(geo, op.tab.x[q1], op.tab.x[q2], op.tab.x[q3], Ji, det);
                    vol += det * op.tab.w[q1] * op.tab.w[q2] * op.tab.w[q3];
                }
        for (int d = 0; d < 3; ++d) {
            const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            for (int s = 0; s < 2; ++s) {
                double A = 0.0;
                for (int qb = 0; qb < n; ++qb)
                    for (int qa = 0; qa < n; ++qa) {
                        double xi[3];
                        xi[t1] = op.tab.x[qa];
                        xi[t2] = op.tab.x[qb];
                        xi[d] = (double)s;
                        double Ji[3][3], det;
                        jacobian_inverse<double>(geo, xi[0], xi[1], xi[2], Ji, det);
                        // adjugate row d = det * (row d of J^-1)
                        const double r = det * sqrt(Ji[d][0] * Ji[d][0] + Ji[d][1] * Ji[d][1] + Ji[d][2] * Ji[d][2]);
                        A += r * op.tab.w[qa] * op.tab.w[qb];
                    }
                area[d][s] = A;
            }
        }
    } else {
        vol = op.h[0] * op.h[1] * op.h[2];
        for (int d = 0; d < 3; ++d) area[d][0] = area[d][1] = vol / op.h[d];
    }
    double surf = 0.0;
    const int pos[3] = {ex, ey, ez}, lim[3] = {op.nx, op.ny, op.nz};
    for (int d = 0; d < 3; ++d) {
        surf += (pos[d] == 0 ? 1.0 : 0.5) * area[d][0];
        surf += (pos[d] == lim[d] - 1 ? 1.0 : 0.5) * area[d][1];
    }
    hcell[e] = cbrt(vol);
    hcell[op.ncell + e] = surf / vol;
}

// Decode a face id into its direction, the lower ("-") and upper ("+")
// cells (-1 where absent) and the boundary side when one is absent.
struct FaceInfo {
    int d, em, ep;
};

__device__ inline FaceInfo decode_face(const OpData<double>& op, int fid) {
    FaceInfo f;
    const int nx = op.nx, ny = op.ny, nz = op.nz;
    if (fid < op.nfx) {
        const int fx = fid % (nx + 1), r = fid / (nx + 1), ey = r % ny, ez = r / ny;
        f.d = 0;
        f.em = fx > 0 ? (ez * ny + ey) * nx + fx - 1 : -1;
        f.ep = fx < nx ? (ez * ny + ey) * nx + fx : -1;
    } else if (fid < op.nfx + op.nfy) {
        const int r0 = fid - op.nfx;
        const int ex = r0 % nx, r = r0 / nx, fy = r % (ny + 1), ez = r / (ny + 1);
        f.d = 1;
        f.em = fy > 0 ? (ez * ny + fy - 1) * nx + ex : -1;
        f.ep = fy < ny ? (ez * ny + fy) * nx + ex : -1;
    } else {
        const int r0 = fid - op.nfx - op.nfy;
        const int ex = r0 % nx, r = r0 / nx, ey = r % ny, fz = r / ny;
        f.d = 2;
        f.em = fz > 0 ? ((fz - 1) * ny + ey) * nx + ex : -1;
        f.ep = fz < nz ? (fz * ny + ey) * nx + ex : -1;
    }
    return f;
}

// Penalty factor of a face, P (k+1)^2 sigma_F (the kernels multiply by the
// viscosity at the face point): sigma_F = max(sigma^-, sigma^+) inside, the
// cell's own sigma on the boundary.
__global__ void k_face_penalty(const OpData<double> op, int nface, double pk2, const double* hcell,
                               double* tfac64, float* tfac32) {
    const int fid = blockIdx.x * blockDim.x + threadIdx.x;
    if (fid >= nface) return;
    const FaceInfo f = decode_face(op, fid);
    const double* sig = hcell + op.ncell;
    double sF;
    if (f.em >= 0 && f.ep >= 0) sF = fmax(sig[f.em], sig[f.ep]);
    else sF = sig[f.em >= 0 ? f.em : f.ep];
    const double t = pk2 * sF;
    tfac64[fid] = t;
    tfac32[fid] = (float)t;
}

__global__ void k_visc_cell(const OpData<double> op, int n, const LawDev law, double* mu64, float* mu32) {
    const int nnn = n * n * n;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)op.ncell * nnn) return;
    const int e = (int)(id / nnn), q = (int)(id % nnn);
    const int q1 = q % n, q2 = (q / n) % n, q3 = q / (n * n);
    double geo[8][3], X[3];
    cell_geo_full(op, e, geo);
    map_point<double>(geo, op.tab.x[q1], op.tab.x[q2], op.tab.x[q3], X);
    const double mu = law_value(law, X);
    mu64[id] = mu;
    mu32[id] = (float)mu;
}

// face points are evaluated from the lower cell (xi_d = 1) where it exists
__global__ void k_visc_face(const OpData<double> op, int n, int nface, const LawDev law, double* mu64,
                            float* mu32) {
    const int nn = n * n;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)nface * nn) return;
    const int fid = (int)(id / nn), fp = (int)(id % nn);
    const FaceInfo f = decode_face(op, fid);
    const int a = fp % n, b = fp / n;
    const int t1 = f.d == 0 ? 1 : 0, t2 = f.d == 2 ? 1 : 2;
    double xi[3];
    xi[t1] = op.tab.x[a];
    xi[t2] = op.tab.x[b];
    xi[f.d] = f.em >= 0 ? 1.0 : 0.0;
    double geo[8][3], X[3];
    cell_geo_full(op, f.em >= 0 ? f.em : f.ep, geo);
    map_point<double>(geo, xi[0], xi[1], xi[2], X);
    const double mu = law_value(law, X);
    mu64[id] = mu;
    mu32[id] = (float)mu;
}

// penalty step: tau_div of the cell at each of its quadrature points
__global__ void k_pen_cell(const OpData<double> op, int n, const double* tau_div, double* mu64, float* mu32) {
    const int nnn = n * n * n;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)op.ncell * nnn) return;
    const double t = tau_div[id / nnn];
    mu64[id] = t;
    mu32[id] = (float)t;
}

// penalty step: face factor = mean of the two cells' tau_cont, the cell's own on the boundary
__global__ void k_pen_face(const OpData<double> op, int nface, const double* tau_cont, double* tfac64,
                           float* tfac32) {
    const int fid = blockIdx.x * blockDim.x + threadIdx.x;
    if (fid >= nface) return;
    const FaceInfo f = decode_face(op, fid);
    const double t = (f.em >= 0 && f.ep >= 0) ? 0.5 * (tau_cont[f.em] + tau_cont[f.ep])
                                              : tau_cont[f.em >= 0 ? f.em : f.ep];
    tfac64[fid] = t;
    tfac32[fid] = (float)t;
}

// ---------------------------------------------------------------- diagonal
//
// d_{(c,i)} = a(phi_i e_c, phi_i e_c).  With nodes at the Gauss points the
// reference gradient of phi_i vanishes at every quadrature point off the three
// lines through node i, so the cell part needs 3n-2 points per node:
//   viscous  alpha JxW_i + sum_q mu JxW (|grad phi_i|^2 + (d_c phi_i)^2)
//   poisson  alpha JxW_i + sum_q JxW |grad phi_i|^2
//   penalty  alpha JxW_i + sum_q tau_div JxW (d_c phi_i)^2
// and each face contributes at the single face point below node i:
//   viscous  ds [ -mu phi (grad phi.n + n_c d_c phi) + tau phi^2 (1 + n_c^2) ]
//   poisson  ds [ -phi grad phi.n + tau phi^2 ]
// (twice that on a Dirichlet face, nothing on a Neumann face);
//   penalty  ds tau_F phi^2 n_c^2 on interior and Dirichlet faces alike.

template <int C>
__global__ void k_diagonal(const OpData<double> op, int n, double* diag, double* dinv, float* dinv32) {
    const int nn = n * n, nnn = nn * n;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)op.ncell * nnn) return;
    const int e = (int)(id / nnn), node = (int)(id % nnn);
    const int i[3] = {node % n, (node / n) % n, node / nn};
    const int ex = e % op.nx, ey = (e / op.nx) % op.ny, ez = e / (op.nx * op.ny);
    const auto& tb = op.tab;
    double geo[8][3];
    cell_geo_full(op, e, geo);
    double acc[C];
    for (int c = 0; c < C; ++c) acc[c] = 0.0;

    auto geom = [&](double x1, double x2, double x3, double Ji[3][3], double& det) {
        jacobian_inverse<double>(geo, x1, x2, x3, Ji, det);
    };

    // cell: points q on the lines through i
    for (int dir = -1; dir < 3; ++dir) {
        for (int m = 0; m < n; ++m) {
            int q[3] = {i[0], i[1], i[2]};
            double gr[3] = {0, 0, 0};
            if (dir < 0) {
                if (m > 0) break;
                for (int k = 0; k < 3; ++k) gr[k] = tb.D[i[k]][i[k]];
            } else {
                if (m == i[dir]) continue;
                q[dir] = m;
                gr[dir] = tb.D[m][i[dir]];
            }
            double Ji[3][3], det;
            geom(tb.x[q[0]], tb.x[q[1]], tb.x[q[2]], Ji, det);
            const double JxW = det * tb.w[q[0]] * tb.w[q[1]] * tb.w[q[2]];
            double g[3];
            for (int k = 0; k < 3; ++k) g[k] = gr[0] * Ji[0][k] + gr[1] * Ji[1][k] + gr[2] * Ji[2][k];
            const double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
            const int qi = (q[2] * n + q[1]) * n + q[0];
            if (C == 3 && op.pen) {
                const double td = op.mu_cell[(size_t)e * nnn + qi];
                for (int c = 0; c < 3; ++c) acc[c] += td * JxW * g[c] * g[c];
            } else if (C == 3) {
                const double mu = op.mu_cell[(size_t)e * nnn + qi];
                for (int c = 0; c < 3; ++c) acc[c] += mu * JxW * (g2 + g[c] * g[c]);
            } else {
                acc[0] += JxW * g2;
            }
            if (dir < 0)
                for (int c = 0; c < C; ++c) acc[c] += op.alpha * JxW;
        }
    }

    // faces
    for (int d = 0; d < 3; ++d) {
        for (int s = 0; s < 2; ++s) {
            const int pos = d == 0 ? ex : d == 1 ? ey : ez;
            const int lim = d == 0 ? op.nx : d == 1 ? op.ny : op.nz;
            const bool has_nb = s == 1 ? pos + 1 < lim : pos > 0;
            if (!has_nb && op.bc[2 * d + s] != 0) continue;
            const double factor = has_nb ? 1.0 : 2.0;
            const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            int fid;
            if (d == 0) fid = (ez * op.ny + ey) * (op.nx + 1) + ex + s;
            else if (d == 1) fid = op.nfx + (ez * (op.ny + 1) + ey + s) * op.nx + ex;
            else fid = op.nfx + op.nfy + ((ez + s) * op.ny + ey) * op.nx + ex;
            const int fp = i[t2] * n + i[t1];
            double xi[3];
            xi[t1] = tb.x[i[t1]];
            xi[t2] = tb.x[i[t2]];
            xi[d] = (double)s;
            double Ji[3][3], det;
            geom(xi[0], xi[1], xi[2], Ji, det);
            const double v0 = Ji[d][0], v1 = Ji[d][1], v2 = Ji[d][2];
            const double nv = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
            const double sg = s == 1 ? 1.0 : -1.0;
            const double nrm[3] = {sg * v0 / nv, sg * v1 / nv, sg * v2 / nv};
            const double ds = det * nv * tb.w[i[t1]] * tb.w[i[t2]];
            const double phi = tb.S[s][i[d]];
            double gr[3];
            gr[t1] = phi * tb.D[i[t1]][i[t1]];
            gr[t2] = phi * tb.D[i[t2]][i[t2]];
            gr[d] = tb.G[s][i[d]];
            double g[3];
            for (int k = 0; k < 3; ++k) g[k] = gr[0] * Ji[0][k] + gr[1] * Ji[1][k] + gr[2] * Ji[2][k];
            const double gn = g[0] * nrm[0] + g[1] * nrm[1] + g[2] * nrm[2];
            if (C == 3 && op.pen) {
                const double tau = op.tfac[fid];
                for (int c = 0; c < 3; ++c) acc[c] += ds * tau * phi * phi * nrm[c] * nrm[c];
            } else if (C == 3) {
                const double mu = op.mu_face[(size_t)fid * nn + fp];
                const double tau = op.tfac[fid] * mu;
                for (int c = 0; c < 3; ++c)
                    acc[c] += factor * ds *
                              (-mu * phi * (gn + nrm[c] * g[c]) + tau * phi * phi * (1.0 + nrm[c] * nrm[c]));
            } else {
                const double tau = op.tfac[fid];
                acc[0] += factor * ds * (-phi * gn + tau * phi * phi);
            }
        }
    }
    for (int c = 0; c < C; ++c) {
        const size_t idx = ((size_t)e * C + c) * nnn + node;
        diag[idx] = acc[c];
        dinv[idx] = 1.0 / acc[c];
        dinv32[idx] = (float)(1.0 / acc[c]);
    }
}

hipError_t launch_setup(int n, int C, bool curved, const OpData<double>& op, const LawDev& law, double penalty,
                        double* hcell, double* tfac64, float* tfac32, double* mu_cell64, float* mu_cell32,
                        double* mu_face64, float* mu_face32, int nface, const double* tau_div,
                        const double* tau_cont, hipStream_t s) {
    (void)curved;
    const int bt = 256;
    hipLaunchKernelGGL(k_cell_size, dim3((op.ncell + bt - 1) / bt), dim3(bt), 0, s, op, n, hcell);
    if (op.pen) {
        const long long nc = (long long)op.ncell * n * n * n;
        hipLaunchKernelGGL(k_pen_cell, dim3((unsigned)((nc + bt - 1) / bt)), dim3(bt), 0, s, op, n, tau_div,
                           mu_cell64, mu_cell32);
        hipLaunchKernelGGL(k_pen_face, dim3((nface + bt - 1) / bt), dim3(bt), 0, s, op, nface, tau_cont, tfac64,
                           tfac32);
        return hipGetLastError();
    }
    const double pk2 = penalty * (double)n * (double)n;
    hipLaunchKernelGGL(k_face_penalty, dim3((nface + bt - 1) / bt), dim3(bt), 0, s, op, nface, pk2, hcell, tfac64,
                       tfac32);
    if (C == 3 && law.kind != SIPG_LAW_ARRAYS) {  // ARRAYS: the values are copied in by the plan
        const long long nc = (long long)op.ncell * n * n * n;
        hipLaunchKernelGGL(k_visc_cell, dim3((unsigned)((nc + bt - 1) / bt)), dim3(bt), 0, s, op, n, law, mu_cell64,
                           mu_cell32);
        const long long nf = (long long)nface * n * n;
        hipLaunchKernelGGL(k_visc_face, dim3((unsigned)((nf + bt - 1) / bt)), dim3(bt), 0, s, op, n, nface, law,
                           mu_face64, mu_face32);
    }
    return hipGetLastError();
}

hipError_t launch_diagonal(int n, int C, bool curved, const OpData<double>& op, double* diag, double* dinv,
                           float* dinv32, hipStream_t s) {
    (void)curved;
    const int bt = 256;
    const long long nn = (long long)op.ncell * n * n * n;
    const dim3 grid((unsigned)((nn + bt - 1) / bt));
    if (C == 3) hipLaunchKernelGGL(k_diagonal<3>, grid, dim3(bt), 0, s, op, n, diag, dinv, dinv32);
    else hipLaunchKernelGGL(k_diagonal<1>, grid, dim3(bt), 0, s, op, n, diag, dinv, dinv32);
    return hipGetLastError();
}

}  // namespace sipg
