// Internal declarations shared by the host code and the HIP kernels of libsipg.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/sipg.h"

namespace sipg {

constexpr int kMaxN = 6;  // n = k + 1 <= 6

// One-dimensional tables on the n Gauss-Legendre points g_q of [0, 1] with
// the Lagrange basis l_j through the same points.
template <typename T>
struct Tables {
    T D[kMaxN][kMaxN];  // D[q][j] = l_j'(g_q)
    T S[2][kMaxN];      // S[s][j] = l_j(s), s = 0, 1 (face values)
    T G[2][kMaxN];      // G[s][j] = l_j'(s)     (face normal derivatives)
    T w[kMaxN];         // quadrature weights, sum 1
    T x[kMaxN];         // quadrature points
};

// Geometry, viscosity and penalty data of one operator in precision T.
template <typename T>
struct OpData {
    int nx, ny, nz, ncell;
    int nfx, nfy;            // number of x-faces, y-faces (face id offsets)
    int bc[6];               // 0 = Dirichlet, 1 = Neumann, sides -x,+x,-y,+y,-z,+z
    int pen;                 // penalty-step operator (mu_cell holds tau_div, tfac the face tau_cont)
    T alpha;                 // mass factor gamma_0/dt
    T h[3];                  // straight cells: edge lengths
    T hinv[3];               // and their inverses
    const T* verts;          // curved cells: vertex coordinates, else nullptr
    const T* mu_cell;        // [ncell][n^3]
    const T* mu_face;        // [nface][n^2]
    const T* tfac;           // [nface] P (k+1)^2 sigma_F (penalty per unit viscosity)
    Tables<T> tab;
};

// Device law parameters (copied by value into kernels).
struct LawDev {
    int kind;
    int n_modes;
    double mu, amp, contrast, rmin, rmax;
    double mu0, mu_inf, lam, n_exp, kappa, a_exp;
    int k[SIPG_MAX_MODES][3];
    double a[SIPG_MAX_MODES];
    double v[SIPG_MAX_MODES][3];
    double phi[SIPG_MAX_MODES];
};

// MODE_APPLY: y = A x;  MODE_CHEB: Chebyshev step (below);  MODE_RESID: y = r - A x;
// MODE_CONT: a continuous level of the multigrid hierarchy (below)
enum ApplyMode { MODE_APPLY = 0, MODE_CHEB = 1, MODE_RESID = 2, MODE_CONT = 3 };

// Vector arguments of one operator application.
template <typename T>
struct ApplyIO {
    const T* x;      // input (MODE_CHEB: current iterate z_j)
    T* y;            // output (MODE_CHEB: next iterate z_{j+1})
    int parts;       // SIPG_PART_* mask
    // MODE_CHEB: d <- c1 d + c2 Dinv (r - A z); z_{j+1} = z_j + d;  MODE_RESID: y = r - A x
    const T* r;
    const T* dinv;
    T* d;
    const double* coef;  // device {c1, c2}
    const int* skip;     // device flag: nonzero => kernel returns at once (may be null)
    // MODE_CONT: x holds the values of a continuous level at its Gauss-Lobatto
    // nodes (degree cj, cMx * cMy * (cj nz + 1) nodes per component,
    // component-major); the kernel interpolates every cell's values to its
    // Gauss nodes (cL[q][a] = l^Lobatto_a(x^Gauss_q)), applies the operator
    // and writes the cell's local contributions G_e^T (A G x) to y (DG
    // layout).  xnb: a DG-sized array the face passes may read their
    // (unused) neighbour values from; null: x.
    const T* xnb;
    int cj, cMx, cMy;
    long long cnv;
    T cL[kMaxN][kMaxN];
};

// Device-side state of one CG solve (lives in the workspace).
struct SolveState {
    double bnorm2, rz, alpha, beta;
    double tol2;             // rel_tol^2
    double rr;               // last recursive residual norm^2
    double rr_true;          // last true residual norm^2
    double mean;             // scratch for mean-zero projections
    double scale;            // scratch
    double lam_max;
    double theta_inv;
    double cheb[64][2];      // per Chebyshev step (c1, c2), step 1..degree-1
    double lz_alpha[64], lz_beta[65];
    int lz_m;                // Lanczos steps taken
    int done;                // 0 running, 1 converged (recursive), 2 breakdown, 3 max_iter
    int iter;
    int max_iter;
    int skip;                // nonzero while done != 0 (read by apply kernels)
    unsigned arrive;         // blocks of the running fused reduction that have finished (0 between kernels)
    int pad[2];
};

constexpr int kRedBlocks = 512;   // blocks of the deterministic reductions
constexpr int kRedThreads = 256;
constexpr int kRedSlots = 4;      // partial sums per block

// 1D multigrid transfer tables: P[i][j] = l^coarse_j(x^fine_i) between
// degrees (nf x nc); H[c][i][j] = l_j((c + x_i) / 2) from an interval to its
// half c (n x n).
template <typename T>
struct MgTab {
    T P[kMaxN][kMaxN];
    T H[2][kMaxN][kMaxN];
};

// Continuous level of the cph-multigrid hierarchy: degree j on nx*ny*nz
// cells, (Mx, My, Mz) = (j nx + 1, j ny + 1, j nz + 1) Lobatto nodes per
// direction, C components (component-major).
struct CgGeo {
    int j, C, nx, ny, nz, Mx, My, Mz;
};
// L[b][a] = l^Lobatto_a(x^Gauss_b): a cell's Lobatto interpolant at its Gauss nodes.
template <typename T>
struct CgL {
    T L[kMaxN][kMaxN];
};
// Diagonal of a continuous level: Lobatto basis values and derivatives at
// the Gauss points, LV[q][a], LD[q][a], and derivatives at the end points LGs[s][a].
struct CgDiagTab {
    double LV[kMaxN][kMaxN], LD[kMaxN][kMaxN], LGs[2][kMaxN];
};
// 1D sparse transfer matrix (CSR) along one axis.
template <typename T>
struct AxisMat {
    int rows;
    const int* rp;
    const int* ci;
    const T* v;
};

// Picard viscosity update: the finest level's velocity (3 components) and
// the points of the level whose viscosity is evaluated.
struct FineVelocity {
    const double* u;          // [ncell][3][n^3]
    const double* verts;      // curved cells: vertex coordinates, else nullptr (unit box)
    int nx, ny, nz, n;
    double g[kMaxN];          // Gauss points of [0, 1]
    double inv_den[kMaxN];    // 1 / prod_{m != j} (g_j - g_m)
};

struct LevelPoints {
    int nx, ny, nz, n;
    int r;                    // fine cells per level cell and direction (2^mesh steps)
    double g[kMaxN];          // the level's Gauss points
};

constexpr int kPicardBlocks = 512;  // blocks of the residual sums (partials: 3 * kPicardBlocks)

// Dual-splitting step: the velocity mesh and 1D tables, and the pressure
// basis (n - 1 Gauss points) evaluated at the velocity's n Gauss points.
struct SplitGeo {
    int nx, ny, nz;
    const double* verts;         // curved cells, else nullptr (straight cells of edge h)
    double h[3], hinv[3];
    Tables<double> tab;          // velocity: n Gauss points
    double PV[kMaxN][kMaxN];     // PV[q][j] = l^p_j(g_q)
    double PD[kMaxN][kMaxN];     // PD[q][j] = l^p_j'(g_q)
    double PS[2][kMaxN];         // PS[s][j] = l^p_j(s)
    const double* gw;            // velocity data on the walls (wall rows x n^2 points x 3), or nullptr (0)
    int order;                   // BDF order m (1, 2) of the step
    double gamma0, alpha[2], beta[2];   // BDF coefficients and extrapolation weights
    double beta_bar;             // extrapolation weight of the pressure wall data (m_p = 1), 0 for m = 1
    double eta[6];               // mu0, mu_inf, lam, n_exp, kappa, a_exp of the Carreau law (m = 2)
};

// ---------------------------------------------------------------- launchers
// (defined in the .hip files; return hipError_t of the launch)

template <typename T>
hipError_t launch_apply(int n, int C, bool curved, const OpData<T>& op, const ApplyIO<T>& io,
                        int mode, hipStream_t s);
// the penalty-step operator (op.pen), dispatched to by launch_apply
template <typename T>
hipError_t launch_apply_pen(int n, bool curved, const OpData<T>& op, const ApplyIO<T>& io, int mode, hipStream_t s);

hipError_t launch_setup(int n, int C, bool curved, const OpData<double>& op, const LawDev& law,
                        double penalty, double* hcell, double* tfac64, float* tfac32,
                        double* mu_cell64, float* mu_cell32, double* mu_face64, float* mu_face32,
                        int nface, const double* tau_div, const double* tau_cont, hipStream_t s);

hipError_t launch_diagonal(int n, int C, bool curved, const OpData<double>& op, double* diag,
                           double* dinv, float* dinv32, hipStream_t s);

// viscosity eta(gdot(u)) at all cell and face points of one level (FP64 + FP32)
hipError_t launch_picard_viscosity(const FineVelocity& F, const LevelPoints& Lv, const LawDev& law, long long nface,
                                   double* mu_cell64, float* mu_cell32, double* mu_face64, float* mu_face32,
                                   hipStream_t s);
// out[0..2] = |R|^2, Rp.(R - Rp), |R - Rp|^2 (Rp may be null: zeros); deterministic
hipError_t launch_picard_sums(const double* R, const double* Rp, long long n, double* partials, double* out,
                              hipStream_t s);
hipError_t launch_axpy(double* x, const double* d, double omega, long long n, hipStream_t s);

// Dual-splitting step operators (n = 3..6; one workgroup per cell)
hipError_t launch_split_convective(int n, const SplitGeo& S, const double* u, const double* u_prev, const double* b,
                                   double dt, double* uhat, hipStream_t s);
hipError_t launch_split_ppe_rhs(int n, const SplitGeo& S, const double* uhat, const double* u_old,
                                const double* u_prev, const double* b, double dt, double* f, hipStream_t s);
// penalty factors of a mesh-step level: the mean of each coarse cell's 8 children
hipError_t launch_pen_coarsen(int fx, int fy, int fz, const double* td, const double* tc, double* ctd, double* ctc,
                              hipStream_t s);
// y = a x + c z (n values)
hipError_t launch_lincomb(long long n, double a, const double* x, double c, const double* z, double* y, hipStream_t s);
hipError_t launch_split_projection(int n, const SplitGeo& S, const double* uhat, const double* p, double dt,
                                   double* uhh, double* rhs, hipStream_t s);
hipError_t launch_split_mass(int n, const SplitGeo& S, const double* x, double scale, double* y, hipStream_t s);
hipError_t launch_pen_factors(int n, const SplitGeo& S, const double* u, double dt, double zeta, const double* hcell,
                              double* tau_div, double* tau_cont, hipStream_t s);
// y += load of the wall data S.gw: viscous (pen = 0; mu_face, tfac = P(k+1)^2 sigma_F
// per face) or penalty step (pen = 1; tfac = the face's continuity factor)
hipError_t launch_wall_load(int n, const SplitGeo& S, const double* mu_face, const double* tfac, int pen, double* y,
                            hipStream_t s);

// Multigrid transfers between a fine level (nf nodes per direction, fine
// mesh fx*fy*fz cells) and the next coarser one (nc; same mesh for a degree
// step, half the cells per direction for a mesh step).  restrict: rc = P^T tf;
// prolong: zf += P zc.  Every kernel returns at once when *skip != 0.
template <typename T>
hipError_t launch_restrict(bool mesh_step, int C, int nf, int nc, int fx, int fy, int fz, const MgTab<T>& tab,
                           const T* tf, T* rc, const int* skip, hipStream_t s);
template <typename T>
hipError_t launch_prolong_add(bool mesh_step, int C, int nf, int nc, int fx, int fy, int fz, const MgTab<T>& tab,
                              const T* zc, T* zf, const int* skip, hipStream_t s);
// Level vector kernels in the preconditioner precision T (all skip-aware):
// Chebyshev start z = theta^-1 dinv r, d = z (theta from the level's state);
// y = x; y += x; z64 = (double) zT.
template <typename T>
hipError_t launch_cheb_start_t(const T* r, T* z, T* d, const T* dinv, long long n, const SolveState* st,
                               const int* skip, hipStream_t s);
template <typename T>
hipError_t launch_copy_t(T* y, const T* x, long long n, const int* skip, hipStream_t s);
template <typename T>
hipError_t launch_add_t(T* y, const T* x, long long n, const int* skip, hipStream_t s);
template <typename T>
hipError_t launch_to_f64(double* y, const T* x, long long n, hipStream_t s);

// Continuous levels (cph-multigrid): dg = G cg (add: +=); cg = G^T dg
// (dg is overwritten by the cells' local contributions); out = M in along
// one axis of a (C, n2, n1, n0) array; Chebyshev step d <- c1 d + c2 dinv
// (r - t), zn = z + d; y = r - t; diagonal of G^T A G (local: a DG-sized
// work array) with its inverses; probe vectors and the coarsest level's
// dense inverse (in A); z = Ainv r.  Kernels used in a solve are skip-aware.
template <typename T>
hipError_t launch_cg_gather(const CgGeo& g, const CgL<T>& tab, const T* cg, T* dg, bool add, const int* skip,
                            hipStream_t s);
// scatter modes: 0 cg = G^T dg; 1 cg = r - G^T dg; 2 Chebyshev step with
// t = G^T dg: d <- c1 d + c2 dinv (r - t), cg = z + d (coef = {c1, c2})
template <typename T>
hipError_t launch_cg_scatter(const CgGeo& g, const CgL<T>& tab, T* dg, T* cg, const int* skip, hipStream_t s,
                             int mode = 0, const T* r = nullptr, const T* z = nullptr, T* d = nullptr,
                             const T* dinv = nullptr, const double* coef = nullptr);
// the node sums alone (modes as launch_cg_scatter), from the cells' local contributions
template <typename T>
hipError_t launch_cg_assemble(const CgGeo& g, const T* local, T* cg, const int* skip, hipStream_t s, int mode,
                              const T* r, const T* z, T* d, const T* dinv, const double* coef);
template <typename T>
hipError_t launch_axis(const AxisMat<T>& M, int axis, int C, int n0, int n1, int n2, const T* in, T* out, bool add,
                       const int* skip, hipStream_t s);
template <typename T>
hipError_t launch_cg_cheb(const T* z, T* zn, T* d, const T* r, const T* t, const T* dinv, const double* coef,
                          long long n, const int* skip, hipStream_t s);
template <typename T>
hipError_t launch_cg_sub(T* y, const T* r, const T* t, long long n, const int* skip, hipStream_t s);
hipError_t launch_cg_diagonal(const CgGeo& g, const OpData<double>& op, const CgDiagTab& tab, double* local,
                              double* diag, double* dinv64, float* dinv32, hipStream_t s);
hipError_t launch_cg_probe(double* v, int C, long long ncell, int col, hipStream_t s);
// A (n x n) = the inverse of the coarsest level's matrix; work: n * n + 1 doubles
hipError_t launch_cg_coarse_inverse(const CgGeo& g, const double* probes, long long dgsize, const CgL<double>& tab,
                                    double* A, double* work, int mean_zero, hipStream_t s);
template <typename T>
hipError_t launch_dense_mv(const double* Ainv, const T* r, T* z, int n, const int* skip, hipStream_t s);

}  // namespace sipg
