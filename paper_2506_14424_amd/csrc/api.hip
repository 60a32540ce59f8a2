// Host side of libsipg: plans, workspace layout, the C ABI of include/sipg.h.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sipg_internal.h"
#include "solver_kernels.h"

using namespace sipg;

namespace {

thread_local std::string g_err;

sipg_status fail(sipg_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return fail(SIPG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------ 1D tables
// Gauss-Legendre points of [-1, 1] by Newton's method on P_n (three-term
// recurrence), mapped to [0, 1]; derivative matrix from barycentric weights.
void gauss_legendre01(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) p0 = 1.0;
        dp = n == 1 ? 1.0 : n * (z * p1 - p0) / (z * z - 1.0);
        // z_i descending in i; store ascending on [0, 1]
        x[n - 1 - i] = 0.5 * (1.0 + z);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2)P'^2) halved for [0,1]
    }
}

template <typename T>
void fill_tables(int n, Tables<T>& tb) {
    double x[kMaxN], w[kMaxN], lam[kMaxN];
    gauss_legendre01(n, x, w);
    std::memset(&tb, 0, sizeof(tb));
    for (int j = 0; j < n; ++j) {
        double p = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != j) p *= x[j] - x[m];
        lam[j] = 1.0 / p;
    }
    for (int q = 0; q < n; ++q) {
        double diag = 0.0;
        for (int j = 0; j < n; ++j)
            if (j != q) {
                const double v = lam[j] / lam[q] / (x[q] - x[j]);
                tb.D[q][j] = T(v);
                diag -= v;
            }
        tb.D[q][q] = T(diag);
        tb.w[q] = T(w[q]);
        tb.x[q] = T(x[q]);
    }
    for (int s = 0; s < 2; ++s) {
        const double t = s;
        for (int j = 0; j < n; ++j) {
            double val = 1.0, der = 0.0;
            for (int m = 0; m < n; ++m) {
                if (m == j) continue;
                // product rule: d/dt prod (t - x_m)/(x_j - x_m)
                der = der * (t - x[m]) / (x[j] - x[m]) + val / (x[j] - x[m]);
                val *= (t - x[m]) / (x[j] - x[m]);
            }
            tb.S[s][j] = T(val);
            tb.G[s][j] = T(der);
        }
    }
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

enum Phase { PH_IDLE = 0, PH_RUNNING, PH_CHECKING, PH_DONE };

// Gauss-Lobatto points of degree j on [0, 1] (j + 1 points, ascending): the
// end points and the roots of P_j', by Newton's method from the
// Chebyshev-Lobatto points (P_j and P_j' from the three-term recurrence,
// P_j'' = (2 z P_j' - j (j + 1) P_j) / (1 - z^2)).
void gll01(int j, double* x) {
    x[0] = 0.0;
    x[j] = 1.0;
    for (int i = 1; i < j; ++i) {
        double z = -std::cos(M_PI * i / j);
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= j; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double d1 = j * (z * p1 - p0) / (z * z - 1.0);           // P_j'
            const double d2 = (2.0 * z * d1 - j * (j + 1.0) * p1) / (1.0 - z * z);
            const double dz = d1 / d2;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        x[i] = 0.5 * (1.0 + z);
    }
}

// Lagrange basis through nodes[0..m-1] at t: values and derivatives.
void lagrange_vd(const double* nodes, int m, double t, double* val, double* der) {
    for (int a = 0; a < m; ++a) {
        double v = 1.0, d = 0.0;
        for (int k = 0; k < m; ++k) {
            if (k == a) continue;
            double term = 1.0 / (nodes[a] - nodes[k]);
            for (int l = 0; l < m; ++l)
                if (l != a && l != k) term *= (t - nodes[l]) / (nodes[a] - nodes[l]);
            d += term;
            v *= (t - nodes[k]) / (nodes[a] - nodes[k]);
        }
        val[a] = v;
        if (der) der[a] = d;
    }
}

// A 1D transfer matrix in CSR form (host).
struct Csr {
    int rows = 0;
    std::vector<int> rp, ci;
    std::vector<double> v;
};

Csr csr_of(const std::vector<std::vector<double>>& M, int cols) {
    Csr c;
    c.rows = (int)M.size();
    c.rp.push_back(0);
    for (const auto& row : M) {
        for (int k = 0; k < cols; ++k)
            if (row[k] != 0.0) { c.ci.push_back(k); c.v.push_back(row[k]); }
        c.rp.push_back((int)c.ci.size());
    }
    return c;
}

Csr csr_transpose(const std::vector<std::vector<double>>& M, int cols) {
    std::vector<std::vector<double>> T(cols, std::vector<double>(M.size(), 0.0));
    for (size_t i = 0; i < M.size(); ++i)
        for (int k = 0; k < cols; ++k) T[k][i] = M[i][k];
    return csr_of(T, (int)M.size());
}

// One continuous level of the cph hierarchy (see sipg_mg_opts): host tables
// built with the hierarchy, device pointers set at binding (all in the
// finest plan's workspace, 8 bytes per vector entry in either precision).
struct CgLevel {
    sipg_plan* carrier = nullptr;    // the DG plan of the same degree and mesh
    CgGeo geo;
    long long n = 0;                 // unknowns
    long long dgsize = 0;            // the carrier's unknowns
    CgL<double> L64;
    CgL<float> L32;
    CgDiagTab dtab;
    // transfer to the next coarser level: prolongation (rows: this level's
    // nodes along an axis) and its transpose, per axis
    Csr P[3], R[3];
    bool direct = false;             // coarsest, degree 1, n <= direct_max: dense FP64 inverse
    void *r = nullptr, *za = nullptr, *zb = nullptr, *d = nullptr, *t = nullptr, *zk = nullptr;
    void *ta = nullptr, *tb = nullptr;
    double *diag64 = nullptr, *dinv64 = nullptr;
    float* dinv32 = nullptr;
    void *dgx = nullptr, *dgy = nullptr;
    SolveState* st = nullptr;
    double* partials = nullptr;
    int *prp[3] = {}, *pci[3] = {}, *rrp[3] = {}, *rci[3] = {};
    double *pv64[3] = {}, *rv64[3] = {};
    float *pv32[3] = {}, *rv32[3] = {};
    double* cinv = nullptr;          // coarsest: dense inverse
    double* cwork = nullptr;         // coarsest: the inversion's second buffer
    double* probes = nullptr;        // coarsest: the carrier applied to C*8 probe vectors
    bool lz_valid = false, lz_stale = false;
    int lz_steps = 0;
};

}  // namespace

struct sipg_plan {
    int nx, ny, nz, bc[6];
    int op, degree, n, C;
    double alpha, penalty;
    bool curved;
    std::vector<double> verts;
    std::vector<float> verts32;
    bool pen = false;                    // penalty-step operator
    std::vector<double> tau_div, tau_cont;   // its per-cell factors (host)
    double *tau_div_d = nullptr, *tau_cont_d = nullptr;
    LawDev law;
    std::vector<double> mu_cell_h, mu_face_h;   // ARRAYS law: the caller's values (host)
    std::vector<float> mu_cell_h32, mu_face_h32;
    long long ncell, ndof, nface, nvert;
    Tables<double> tab64;
    Tables<float> tab32;

    // device workspace
    bool bound = false, with_solver = false;
    char* ws = nullptr;
    double *verts64_d = nullptr, *hcell = nullptr, *tfac64 = nullptr, *mu_cell64 = nullptr, *mu_face64 = nullptr;
    float *verts32_d = nullptr, *tfac32 = nullptr, *mu_cell32 = nullptr, *mu_face32 = nullptr;
    double *diag64 = nullptr, *dinv64 = nullptr;
    float* dinv32 = nullptr;
    double *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr, *zo = nullptr;
    void *cr = nullptr, *cd = nullptr, *cz0 = nullptr, *cz1 = nullptr;
    double* partials = nullptr;
    SolveState* st = nullptr;

    // solve session
    SolveState* mirror = nullptr;  // pinned host copy of *st
    hipEvent_t ev = nullptr;
    hipStream_t sstream = nullptr;
    const double* b = nullptr;
    double* x = nullptr;
    sipg_solve_opts opts;
    int phase = PH_IDLE;
    int restarts = 0;
    bool mean_zero = false;
    bool lz_valid = false;               // eigenvalue estimates exist (lz_steps Lanczos steps)
    bool lz_stale = false;               // ... but the operator changed since (viscosity, penalty factors)
    int lz_steps = 0;
    sipg_solve_info info;

    // captured CG chunks (sipg_solve_opts::use_graph): key and executable
    struct GraphEntry {
        hipGraphExec_t exec = nullptr;
        int iters = 0, prec = -1, kind = -1, deg = -1, mz = -1;
        const void* x = nullptr;
        const void* z = nullptr;
    };
    hipStream_t cap_stream = nullptr;
    GraphEntry graphs[2];
    int graph_next = 0;
    // per-level work side by side (Lanczos estimates, viscosity updates;
    // created at first use, default priority): fork and join events
    static constexpr int kAuxStreams = 3;
    hipStream_t aux_streams[kAuxStreams] = {};
    hipEvent_t aux_fork = nullptr, aux_join[kAuxStreams] = {};
    bool aux_failed = false;
    bool no_alloc = false;           // inside the no-allocation entry point: everything on the caller's stream

    // multigrid hierarchy: this plan is the finest level, mg[i] is level i+1
    bool mg_on = false;
    sipg_mg_opts mg_opts;
    std::vector<sipg_plan*> mg;
    bool mesh_step = false;          // (coarse level) transfer from the finer level is a mesh step
    MgTab<double> tr64;              // (coarse level) 1D tables of that transfer
    MgTab<float> tr32;
    void *mgz = nullptr, *mgt = nullptr;  // (finest level) V-cycle correction and residual
    std::vector<CgLevel> cg;              // (finest level, continuous hierarchy) the continuous levels

    template <typename T>
    OpData<T> opdata() const;
};

template <typename T>
OpData<T> sipg_plan::opdata() const {
    OpData<T> o;
    std::memset(&o, 0, sizeof(o));
    o.nx = nx; o.ny = ny; o.nz = nz;
    o.ncell = (int)ncell;
    o.nfx = (nx + 1) * ny * nz;
    o.nfy = nx * (ny + 1) * nz;
    for (int i = 0; i < 6; ++i) o.bc[i] = bc[i];
    o.pen = pen ? 1 : 0;
    o.alpha = T(alpha);
    o.h[0] = T(1.0 / nx); o.h[1] = T(1.0 / ny); o.h[2] = T(1.0 / nz);
    o.hinv[0] = T(nx); o.hinv[1] = T(ny); o.hinv[2] = T(nz);
    if constexpr (sizeof(T) == 8) {
        o.verts = curved ? verts64_d : nullptr;
        o.mu_cell = mu_cell64; o.mu_face = mu_face64; o.tfac = tfac64;
        o.tab = tab64;
    } else {
        o.verts = curved ? verts32_d : nullptr;
        o.mu_cell = mu_cell32; o.mu_face = mu_face32; o.tfac = tfac32;
        o.tab = tab32;
    }
    return o;
}

namespace {

struct Layout;
Layout layout(const sipg_plan* P);

struct Layout {
    size_t verts64, verts32, hcell, tfac64, tfac32, mu_cell64, mu_cell32, mu_face64, mu_face32, diag64, dinv64,
        dinv32;
    size_t r, p, q, z, zo, cr, cd, cz0, cz1, partials, st;
    size_t tdiv = 0, tcont = 0;       // penalty step: per-cell factors
    size_t mgz = 0, mgt = 0;          // multigrid: finest-level vectors
    std::vector<size_t> level, level_bytes;   // multigrid: workspaces of the coarser levels
    struct Cg {
        size_t vec[8], diag64, dinv64, dinv32, dgx, dgy, st, partials, cinv, cwork, probes;
        size_t prp[3], pci[3], pv64[3], pv32[3], rrp[3], rci[3], rv64[3], rv32[3];
    };
    std::vector<Cg> cg;               // continuous levels
    size_t op_end, total;
};

Layout layout(const sipg_plan* P) {
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    const size_t nv = P->curved ? (size_t)P->nvert * 3 : 0;
    const size_t nqc = P->C == 3 ? (size_t)P->ncell * P->n * P->n * P->n : 0;
    const size_t nqf = (P->C == 3 && !P->pen) ? (size_t)P->nface * P->n * P->n : 0;
    const size_t ntau = P->pen ? (size_t)P->ncell : 0;
    const size_t nd = (size_t)P->ndof;
    L.verts64 = take(nv * 8); L.verts32 = take(nv * 4);
    L.hcell = take((size_t)P->ncell * 16);   // h_e, then the penalty's sigma_e
    L.tfac64 = take((size_t)P->nface * 8); L.tfac32 = take((size_t)P->nface * 4);
    L.mu_cell64 = take(nqc * 8); L.mu_cell32 = take(nqc * 4);
    L.mu_face64 = take(nqf * 8); L.mu_face32 = take(nqf * 4);
    L.diag64 = take(nd * 8); L.dinv64 = take(nd * 8); L.dinv32 = take(nd * 4);
    L.tdiv = take(ntau * 8); L.tcont = take(ntau * 8);
    L.op_end = off;
    L.r = take(nd * 8); L.p = take(nd * 8); L.q = take(nd * 8); L.z = take(nd * 8); L.zo = take(nd * 8);
    L.cr = take(nd * 8); L.cd = take(nd * 8); L.cz0 = take(nd * 8); L.cz1 = take(nd * 8);
    L.partials = take(kRedSlots * kRedBlocks * 8);
    L.st = take(sizeof(SolveState));
    if (P->mg_on) {
        L.mgz = take(nd * 8);
        L.mgt = take(nd * 8);
        for (const sipg_plan* c : P->mg) {
            const size_t b = layout(c).total;
            L.level.push_back(take(b));
            L.level_bytes.push_back(b);
        }
    }
    for (const CgLevel& c : P->cg) {
        Layout::Cg g;
        std::memset(&g, 0, sizeof(g));
        for (int k = 0; k < 8; ++k) g.vec[k] = take((size_t)c.n * 8);
        g.diag64 = take((size_t)c.n * 8); g.dinv64 = take((size_t)c.n * 8); g.dinv32 = take((size_t)c.n * 4);
        g.dgx = take((size_t)c.dgsize * 8); g.dgy = take((size_t)c.dgsize * 8);
        g.st = take(sizeof(SolveState));
        g.partials = take(kRedSlots * kRedBlocks * 8);
        for (int a = 0; a < 3; ++a) {
            g.prp[a] = take(c.P[a].rp.size() * 4); g.pci[a] = take(c.P[a].ci.size() * 4);
            g.pv64[a] = take(c.P[a].v.size() * 8); g.pv32[a] = take(c.P[a].v.size() * 4);
            g.rrp[a] = take(c.R[a].rp.size() * 4); g.rci[a] = take(c.R[a].ci.size() * 4);
            g.rv64[a] = take(c.R[a].v.size() * 8); g.rv32[a] = take(c.R[a].v.size() * 4);
        }
        g.cinv = c.direct ? take((size_t)c.n * c.n * 8) : 0;
        g.cwork = c.direct ? take(((size_t)c.n * c.n + 1) * 8) : 0;
        g.probes = c.direct ? take((size_t)c.geo.C * 8 * c.dgsize * 8) : 0;
        L.cg.push_back(g);
    }
    L.total = off;
    return L;
}

bool valid_plan(const sipg_plan* P) { return P != nullptr; }

int mg_levels(const sipg_plan* P) { return P->mg_on ? 1 + (int)P->mg.size() : 1; }
sipg_plan* mg_level(sipg_plan* P, int l) { return l == 0 ? P : P->mg[l - 1]; }

// The continuous levels of the cph hierarchy: one per DG level of the
// hierarchy (same degree and mesh; the finest DG level itself is the first
// carrier), with the tables of G (Lobatto -> Gauss per cell), the diagonal's
// Lobatto basis tables, and the 1D prolongations to each level from the next
// coarser one (degree step: the coarse Lobatto interpolant at the fine
// Lobatto nodes of a cell; mesh step at degree 1: fine vertex 2i <- i,
// 2i + 1 <- the mean of i and i + 1).
void build_continuous_levels(sipg_plan* P) {
    P->cg.clear();
    const int nl = mg_levels(P);
    for (int l = 0; l < nl; ++l) {
        sipg_plan* Cr = mg_level(P, l);
        CgLevel c;
        c.carrier = Cr;
        const int j = Cr->degree, n = Cr->n;
        c.geo.j = j; c.geo.C = Cr->C; c.geo.nx = Cr->nx; c.geo.ny = Cr->ny; c.geo.nz = Cr->nz;
        c.geo.Mx = j * Cr->nx + 1; c.geo.My = j * Cr->ny + 1; c.geo.Mz = j * Cr->nz + 1;
        c.n = (long long)Cr->C * c.geo.Mx * c.geo.My * c.geo.Mz;
        c.dgsize = Cr->ndof;
        double lob[kMaxN], gx[kMaxN], gw[kMaxN];
        gll01(j, lob);
        gauss_legendre01(n, gx, gw);
        std::memset(&c.L64, 0, sizeof(c.L64));
        std::memset(&c.L32, 0, sizeof(c.L32));
        std::memset(&c.dtab, 0, sizeof(c.dtab));
        for (int q = 0; q < n; ++q) {
            double v[kMaxN], d[kMaxN];
            lagrange_vd(lob, n, gx[q], v, d);
            for (int a = 0; a < n; ++a) {
                c.L64.L[q][a] = v[a];
                c.L32.L[q][a] = (float)v[a];
                c.dtab.LV[q][a] = v[a];
                c.dtab.LD[q][a] = d[a];
            }
        }
        for (int side = 0; side < 2; ++side) {
            double v[kMaxN], d[kMaxN];
            lagrange_vd(lob, n, (double)side, v, d);
            for (int a = 0; a < n; ++a) c.dtab.LGs[side][a] = d[a];
        }
        P->cg.push_back(c);
    }
    for (int l = 0; l + 1 < nl; ++l) {
        CgLevel& f = P->cg[l];
        const CgLevel& c = P->cg[l + 1];
        const bool mesh_step = c.geo.nx != f.geo.nx || c.geo.ny != f.geo.ny || c.geo.nz != f.geo.nz;
        const int cells_c[3] = {c.geo.nx, c.geo.ny, c.geo.nz};
        for (int a = 0; a < 3; ++a) {
            const int nc = cells_c[a];
            std::vector<std::vector<double>> M;
            int cols;
            if (mesh_step) {                       // degree 1 on both levels
                cols = nc + 1;
                M.assign(2 * nc + 1, std::vector<double>(cols, 0.0));
                for (int i = 0; i <= 2 * nc; ++i) {
                    if (i % 2 == 0) M[i][i / 2] = 1.0;
                    else M[i][i / 2] = M[i][i / 2 + 1] = 0.5;
                }
            } else {
                const int jf = f.geo.j, jc = c.geo.j;
                double lf[kMaxN], lc[kMaxN];
                gll01(jf, lf);
                gll01(jc, lc);
                cols = jc * nc + 1;
                M.assign(jf * nc + 1, std::vector<double>(cols, 0.0));
                for (int i = 0; i <= jf * nc; ++i) {
                    const int e = std::min(i / jf, nc - 1), loc = i - e * jf;
                    double v[kMaxN];
                    lagrange_vd(lc, jc + 1, lf[loc], v, nullptr);
                    for (int b = 0; b <= jc; ++b) M[i][e * jc + b] = v[b];
                }
            }
            f.P[a] = csr_of(M, cols);
            f.R[a] = csr_transpose(M, cols);
        }
    }
    CgLevel& last = P->cg.back();
    last.direct = last.geo.j == 1 && last.n <= P->mg_opts.direct_max;
}

double cell_corner_det_min(const sipg_plan* P) {
    // det J of a trilinear cell at its 8 corners; positive everywhere iff the cell is valid enough
    double mn = 1e300;
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    auto V = [&](int ix, int iy, int iz, int i) { return P->verts[(((size_t)iz * (ny + 1) + iy) * (nx + 1) + ix) * 3 + i]; };
    for (int ez = 0; ez < nz; ++ez)
        for (int ey = 0; ey < ny; ++ey)
            for (int ex = 0; ex < nx; ++ex)
                for (int c = 0; c < 8; ++c) {
                    const int a = c & 1, b = (c >> 1) & 1, d = (c >> 2) & 1;
                    double J[3][3];
                    for (int i = 0; i < 3; ++i) {
                        // edges leaving corner (a,b,d) along each axis, pointing in +xi
                        J[i][0] = V(ex + 1, ey + b, ez + d, i) - V(ex, ey + b, ez + d, i);
                        J[i][1] = V(ex + a, ey + 1, ez + d, i) - V(ex + a, ey, ez + d, i);
                        J[i][2] = V(ex + a, ey + b, ez + 1, i) - V(ex + a, ey + b, ez, i);
                    }
                    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                    mn = std::min(mn, det);
                }
    return mn;
}

template <typename T>
sipg_status do_apply(sipg_plan* P, int parts, const void* x, void* y, hipStream_t s) {
    ApplyIO<T> io;
    std::memset(&io, 0, sizeof(io));
    io.x = static_cast<const T*>(x);
    io.y = static_cast<T*>(y);
    io.parts = parts;
    HIP_TRY(launch_apply<T>(P->n, P->C, P->curved, P->opdata<T>(), io, MODE_APPLY, s));
    return SIPG_OK;
}

template <typename T>
const T* dinv_of(const sipg_plan* P) {
    if constexpr (sizeof(T) == 8) return P->dinv64; else return P->dinv32;
}

template <typename T>
const MgTab<T>& tab_of(const sipg_plan* P) {
    if constexpr (sizeof(T) == 8) return P->tr64; else return P->tr32;
}

// Chebyshev-Jacobi steps 1..degree-1 (Sec. 5.3) of level L in precision T for
// the right-hand side rhs, from the start z_1 = theta^-1 D^-1 rhs already in
// L's cz0 (d = z_1 in cd); *zlast receives the buffer holding the last iterate
// (dst, when given and degree >= 2: the last step writes there).
template <typename T>
sipg_status cheb_steps(sipg_plan* L, int degree, const T* rhs, const int* skip, const T** zlast, hipStream_t s,
                       T* dst = nullptr) {
    T* d = static_cast<T*>(L->cd);
    T* za = static_cast<T*>(L->cz0);
    T* zb = static_cast<T*>(L->cz1);
    const OpData<T> od = L->opdata<T>();
    for (int j = 1; j < degree; ++j) {
        const bool into = dst != nullptr && j + 1 == degree;
        ApplyIO<T> io;
        std::memset(&io, 0, sizeof(io));
        io.x = za; io.y = into ? dst : zb; io.parts = SIPG_PART_ALL;
        io.r = rhs; io.dinv = dinv_of<T>(L); io.d = d;
        io.coef = &L->st->cheb[j][0];
        io.skip = skip;
        HIP_TRY(launch_apply<T>(L->n, L->C, L->curved, od, io, MODE_CHEB, s));
        if (into) {
            *zlast = dst;
            return SIPG_OK;
        }
        std::swap(za, zb);
    }
    *zlast = za;
    return SIPG_OK;
}

// ------------------------------------------------------------ continuous levels

bool pure_neumann_poisson(const sipg_plan* P) {
    if (P->C != 1 || P->alpha != 0.0) return false;
    for (int i = 0; i < 6; ++i)
        if (P->bc[i] != SIPG_BC_NEUMANN) return false;
    return true;
}

// Diagonals of the continuous levels and the coarsest level's dense inverse,
// from the carriers' current data (after binding and after every viscosity
// or penalty-factor update); the eigenvalue estimates become stale.
sipg_status refresh_cg_level(sipg_plan* P, CgLevel& c, hipStream_t s) {
    {
        const sipg_plan* Cr = c.carrier;
        HIP_TRY(launch_cg_diagonal(c.geo, Cr->opdata<double>(), c.dtab, static_cast<double*>(c.dgx), c.diag64,
                                   c.dinv64, c.dinv32, s));
        c.lz_stale = true;
        if (c.direct) {
            const int ncol = c.geo.C * 8;
            for (int col = 0; col < ncol; ++col) {
                HIP_TRY(launch_cg_probe(static_cast<double*>(c.dgx), c.geo.C, Cr->ncell, col, s));
                ApplyIO<double> io;
                std::memset(&io, 0, sizeof(io));
                io.x = static_cast<const double*>(c.dgx);
                io.y = c.probes + (size_t)col * c.dgsize;
                io.parts = SIPG_PART_CELL | SIPG_PART_BOUNDARY;
                HIP_TRY(launch_apply<double>(Cr->n, Cr->C, Cr->curved, Cr->opdata<double>(), io, MODE_APPLY, s));
            }
            HIP_TRY(launch_cg_coarse_inverse(c.geo, c.probes, c.dgsize, c.L64, c.cinv, c.cwork,
                                             pure_neumann_poisson(P) ? 1 : 0, s));
        }
    }
    return SIPG_OK;
}

sipg_status refresh_continuous(sipg_plan* P, hipStream_t s) {
    for (CgLevel& c : P->cg) {
        const sipg_status rc = refresh_cg_level(P, c, s);
        if (rc != SIPG_OK) return rc;
    }
    return SIPG_OK;
}


template <typename T>
const CgL<T>& cg_tab(const CgLevel& c) {
    if constexpr (sizeof(T) == 8) return c.L64; else return c.L32;
}
template <typename T>
const T* cg_dinv(const CgLevel& c) {
    if constexpr (sizeof(T) == 8) return c.dinv64; else return c.dinv32;
}
template <typename T>
AxisMat<T> cg_axis(const CgLevel& c, int a, bool restrict_) {
    AxisMat<T> M;
    M.rows = restrict_ ? c.R[a].rows : c.P[a].rows;
    M.rp = restrict_ ? c.rrp[a] : c.prp[a];
    M.ci = restrict_ ? c.rci[a] : c.pci[a];
    if constexpr (sizeof(T) == 8) M.v = restrict_ ? c.rv64[a] : c.pv64[a];
    else M.v = restrict_ ? c.rv32[a] : c.pv32[a];
    return M;
}

// y = G^T A_(cell+boundary) G x on a continuous level, in precision T; with
// mode 1 y = r - (that), with mode 2 the Chebyshev step of cg_cheb fused in
// (d, z, dinv, coef as there)
template <typename T>
sipg_status cg_apply(CgLevel& c, const T* x, T* y, const int* skip, hipStream_t s, int mode = 0,
                     const T* r = nullptr, const T* z = nullptr, T* d = nullptr, const T* dinv = nullptr,
                     const double* coef = nullptr) {
    // the carrier's kernel in its continuous mode: Lobatto -> Gauss per cell,
    // cell and boundary terms, local G_e^T; then the node sums
    const sipg_plan* Cr = c.carrier;
    T* dy = static_cast<T*>(c.dgy);
    ApplyIO<T> io;
    std::memset(&io, 0, sizeof(io));
    io.x = x; io.y = dy; io.parts = SIPG_PART_CELL | SIPG_PART_BOUNDARY; io.skip = skip;
    io.xnb = static_cast<const T*>(c.dgx);
    io.cj = c.geo.j; io.cMx = c.geo.Mx; io.cMy = c.geo.My;
    io.cnv = (long long)c.geo.Mx * c.geo.My * c.geo.Mz;
    const CgL<T>& L = cg_tab<T>(c);
    for (int q = 0; q < kMaxN; ++q)
        for (int a = 0; a < kMaxN; ++a) io.cL[q][a] = L.L[q][a];
    HIP_TRY(launch_apply<T>(Cr->n, Cr->C, Cr->curved, Cr->opdata<T>(), io, MODE_CONT, s));
    HIP_TRY(launch_cg_assemble<T>(c.geo, dy, y, skip, s, mode, r, z, d, dinv, coef));
    return SIPG_OK;
}

// Lanczos estimate of lambda_max(D^-1 A) of a continuous level (FP64, the
// same start vector and steps as the DG levels).
sipg_status run_lanczos_cg(CgLevel& c, int steps, hipStream_t s) {
    const long long n = c.n;
    double *v = static_cast<double*>(c.za), *vprev = static_cast<double*>(c.zb);
    double *w = static_cast<double*>(c.t), *tt = static_cast<double*>(c.d);
    sk_lz_start(v, n, 12345ull, c.partials, s);
    sk_scalar(c.st, c.partials, 1, SC_LZ_NORM, n, s);
    sk_lz_normalize(v, vprev, n, c.st, s);
    sk_lz_pre(tt, v, c.dinv64, n, s);
    for (int k = 0; k < steps; ++k) {
        const sipg_status rc = cg_apply<double>(c, tt, w, nullptr, s);
        if (rc != SIPG_OK) return rc;
        sk_lz_post_alpha(w, v, c.dinv64, n, c.st, c.partials, s);
        sk_lz_orth_beta(w, v, vprev, n, c.st, c.partials, s);
        sk_lz_next_pre(vprev, tt, w, c.dinv64, n, c.st, s);
        std::swap(v, vprev);
    }
    sk_lz_eig(c.st, s);
    HIP_TRY(hipGetLastError());
    c.lz_valid = true;
    c.lz_stale = false;
    c.lz_steps = steps;
    return SIPG_OK;
}

// Chebyshev-Jacobi polynomial of `degree` of a continuous level applied to
// rhs from zero (za, zb, d; ta receives A z); *out: the buffer of the result.
// With dst (and degree >= 2) the last step writes its result into dst, or
// with acc adds it to dst, and *out = dst; the caller copies or adds
// otherwise (*out != dst).
template <typename T>
sipg_status cg_cheb(CgLevel& c, int degree, const T* rhs, const int* skip, const T** out, hipStream_t s,
                    T* dst = nullptr, bool acc = false) {
    T* za = static_cast<T*>(c.za);
    T* zb = static_cast<T*>(c.zb);
    T* d = static_cast<T*>(c.d);
    HIP_TRY(launch_cheb_start_t<T>(rhs, za, d, cg_dinv<T>(c), c.n, c.st, skip, s));
    for (int k = 1; k < degree; ++k) {
        // zb = za + d with d <- c1 d + c2 dinv (rhs - A za), fused into the node sums
        const bool into = dst != nullptr && k + 1 == degree;
        const sipg_status rc = cg_apply<T>(c, za, into ? dst : zb, skip, s, into && acc ? 3 : 2, rhs, za, d,
                                           cg_dinv<T>(c), &c.st->cheb[k][0]);
        if (rc != SIPG_OK) return rc;
        if (into) {
            *out = dst;
            return SIPG_OK;
        }
        std::swap(za, zb);
    }
    *out = za;
    return SIPG_OK;
}

// One V-cycle from zero on continuous level i of the finest plan P (right-hand
// side in the level's r), result in *out.
template <typename T>
sipg_status cg_vcycle(sipg_plan* P, int i, const T** out, hipStream_t s) {
    CgLevel& c = P->cg[i];
    const int* skip = &P->st->skip;
    const T* R = static_cast<const T*>(c.r);
    const bool last = i + 1 == (int)P->cg.size();
    if (last) {
        if (c.direct) {
            HIP_TRY(launch_dense_mv<T>(c.cinv, R, static_cast<T*>(c.za), (int)c.n, skip, s));
            *out = static_cast<const T*>(c.za);
            return SIPG_OK;
        }
        return cg_cheb<T>(c, P->mg_opts.coarse_degree, R, skip, out, s);
    }
    const int deg = P->opts.cheb_degree;
    T* Z = static_cast<T*>(c.zk);
    T* Tt = static_cast<T*>(c.t);
    T* ta = static_cast<T*>(c.ta);
    T* tb = static_cast<T*>(c.tb);
    const T* zs = nullptr;
    sipg_status rc = cg_cheb<T>(c, deg, R, skip, &zs, s, Z);                        // pre-smoothing, into Z
    if (rc != SIPG_OK) return rc;
    if (zs != Z) HIP_TRY(launch_copy_t<T>(Z, zs, c.n, skip, s));
    auto residual = [&]() -> sipg_status {                                          // Tt = R - A Z
        return cg_apply<T>(c, Z, Tt, skip, s, 1, R);
    };
    if ((rc = residual()) != SIPG_OK) return rc;
    CgLevel& cc = P->cg[i + 1];
    const int C = c.geo.C;
    // restriction: along x, y, z with the transposed 1D prolongations
    HIP_TRY(launch_axis<T>(cg_axis<T>(c, 0, true), 0, C, c.geo.Mx, c.geo.My, c.geo.Mz, Tt, ta, false, skip, s));
    HIP_TRY(launch_axis<T>(cg_axis<T>(c, 1, true), 1, C, cc.geo.Mx, c.geo.My, c.geo.Mz, ta, tb, false, skip, s));
    HIP_TRY(launch_axis<T>(cg_axis<T>(c, 2, true), 2, C, cc.geo.Mx, cc.geo.My, c.geo.Mz, tb, static_cast<T*>(cc.r),
                           false, skip, s));
    const T* zc = nullptr;
    if ((rc = cg_vcycle<T>(P, i + 1, &zc, s)) != SIPG_OK) return rc;             // coarse correction
    HIP_TRY(launch_axis<T>(cg_axis<T>(c, 0, false), 0, C, cc.geo.Mx, cc.geo.My, cc.geo.Mz, zc, ta, false, skip, s));
    HIP_TRY(launch_axis<T>(cg_axis<T>(c, 1, false), 1, C, c.geo.Mx, cc.geo.My, cc.geo.Mz, ta, tb, false, skip, s));
    HIP_TRY(launch_axis<T>(cg_axis<T>(c, 2, false), 2, C, c.geo.Mx, c.geo.My, cc.geo.Mz, tb, Z, true, skip, s));
    if ((rc = residual()) != SIPG_OK) return rc;
    if ((rc = cg_cheb<T>(c, deg, Tt, skip, &zs, s, Z, true)) != SIPG_OK) return rc;  // post-smoothing, added to Z
    if (zs != Z) HIP_TRY(launch_add_t<T>(Z, zs, c.n, skip, s));
    *out = Z;
    return SIPG_OK;
}

// One V-cycle from zero on level l of the finest plan `top` (Sec. 5.3):
// right-hand side in the level's cr (precision T), result in *out.  Level 0's
// first Chebyshev step has been written by the CG kernels; every kernel
// follows the finest plan's skip flag.
template <typename T>
sipg_status vcycle(sipg_plan* top, int l, const T** out, hipStream_t s) {
    sipg_plan* L = mg_level(top, l);
    const int* skip = &top->st->skip;
    const long long n = L->ndof;
    const T* R = static_cast<const T*>(L->cr);
    const bool last = top->cg.empty() && l == mg_levels(top) - 1;   // cph: the DG level is never the last
    const int deg = last ? top->mg_opts.coarse_degree : top->opts.cheb_degree;
    if (l > 0) HIP_TRY(launch_cheb_start_t<T>(R, static_cast<T*>(L->cz0), static_cast<T*>(L->cd), dinv_of<T>(L), n,
                                              L->st, skip, s));
    const T* zs = nullptr;
    T* Z = static_cast<T*>(l == 0 ? top->mgz : static_cast<void*>(L->p));
    sipg_status rc = cheb_steps<T>(L, deg, R, skip, &zs, s, last ? nullptr : Z);  // pre-smoothing (into Z)
    if (rc != SIPG_OK || last) {
        *out = zs;
        return rc;
    }
    T* Tm = static_cast<T*>(l == 0 ? top->mgt : static_cast<void*>(L->q));
    const OpData<T> od = L->opdata<T>();
    auto residual = [&]() -> sipg_status {                                       // Tm = R - A Z
        ApplyIO<T> io;
        std::memset(&io, 0, sizeof(io));
        io.x = Z; io.y = Tm; io.parts = SIPG_PART_ALL; io.r = R; io.skip = skip;
        HIP_TRY(launch_apply<T>(L->n, L->C, L->curved, od, io, MODE_RESID, s));
        return SIPG_OK;
    };
    if (zs != Z) HIP_TRY(launch_copy_t<T>(Z, zs, n, skip, s));
    if ((rc = residual()) != SIPG_OK) return rc;
    if (l == 0 && !top->cg.empty()) {
        // cph: the continuous levels below the DG level (restriction G^T,
        // which overwrites Tm with the cells' local contributions, and
        // prolongation Z += G zc)
        CgLevel& c0 = top->cg[0];
        HIP_TRY(launch_cg_scatter<T>(c0.geo, cg_tab<T>(c0), Tm, static_cast<T*>(c0.r), skip, s));
        const T* zc = nullptr;
        if ((rc = cg_vcycle<T>(top, 0, &zc, s)) != SIPG_OK) return rc;
        HIP_TRY(launch_cg_gather<T>(c0.geo, cg_tab<T>(c0), zc, Z, true, skip, s));
    } else {
        sipg_plan* Cc = top->mg[l];
        HIP_TRY(launch_restrict<T>(Cc->mesh_step, L->C, L->n, Cc->n, L->nx, L->ny, L->nz, tab_of<T>(Cc), Tm,
                                   static_cast<T*>(Cc->cr), skip, s));
        const T* zc = nullptr;
        if ((rc = vcycle<T>(top, l + 1, &zc, s)) != SIPG_OK) return rc;           // coarse correction
        HIP_TRY(launch_prolong_add<T>(Cc->mesh_step, L->C, L->n, Cc->n, L->nx, L->ny, L->nz, tab_of<T>(Cc), zc, Z,
                                      skip, s));
    }
    if ((rc = residual()) != SIPG_OK) return rc;
    HIP_TRY(launch_cheb_start_t<T>(Tm, static_cast<T*>(L->cz0), static_cast<T*>(L->cd), dinv_of<T>(L), n, L->st,
                                   skip, s));
    if ((rc = cheb_steps<T>(L, deg, Tm, skip, &zs, s)) != SIPG_OK) return rc;    // post-smoothing
    HIP_TRY(launch_add_t<T>(Z, zs, n, skip, s));
    *out = Z;
    return SIPG_OK;
}

// The preconditioner after its first Chebyshev step (written by the CG
// kernels into the finest level's cr, cz0, cd): the rest of the one-level
// Chebyshev-Jacobi polynomial, or a V-cycle.
template <typename T>
sipg_status precond_body(sipg_plan* P, const T** zl, hipStream_t s) {
    if (P->opts.precond_kind == SIPG_PRECOND_MULTIGRID) return vcycle<T>(P, 0, zl, s);
    return cheb_steps<T>(P, P->opts.cheb_degree, static_cast<const T*>(P->cr), &P->st->skip, zl, s);
}

// (Re)start of the flexible CG from r = b - A x: z = M r, rz = r.z, p = z.
template <typename T>
sipg_status cg_start(sipg_plan* P) {
    hipStream_t s = P->sstream;
    const long long n = P->ndof;
    const int mz = P->mean_zero ? 1 : 0;
    sk_cheb_start<T>(P->r, static_cast<T*>(P->cr), static_cast<T*>(P->cz0), static_cast<T*>(P->cd), dinv_of<T>(P),
                     n, P->st, s);
    const T* zl = nullptr;
    sipg_status rc = precond_body<T>(P, &zl, s);
    if (rc != SIPG_OK) return rc;
    sk_cg_beta<T>(zl, P->z, P->r, nullptr, n, mz, 1, P->st, P->partials, s);
    sk_cg_direction(P->p, P->z, n, mz, 1, P->st, s);
    HIP_TRY(hipGetLastError());
    return SIPG_OK;
}

// `iters` flexible-CG iterations (Sec. 5.3: FP64 CG, preconditioner in T):
// q = A p; alpha; x, r update with the convergence test and the first
// Chebyshev step; the remaining Chebyshev steps; beta; p = z + beta p.
template <typename T>
sipg_status cg_iterations(sipg_plan* P, int iters) {
    hipStream_t s = P->sstream;
    const long long n = P->ndof;
    const int mz = P->mean_zero ? 1 : 0;
    const OpData<double> od = P->opdata<double>();
    for (int it = 0; it < iters; ++it) {
        ApplyIO<double> io;
        std::memset(&io, 0, sizeof(io));
        io.x = P->p; io.y = P->q; io.parts = SIPG_PART_ALL; io.skip = &P->st->skip;
        HIP_TRY(launch_apply<double>(P->n, P->C, P->curved, od, io, MODE_APPLY, s));
        sk_cg_alpha(P->p, P->q, n, P->st, P->partials, s);
        sk_cg_update<T>(P->x, P->r, P->p, P->q, static_cast<T*>(P->cr), static_cast<T*>(P->cz0),
                        static_cast<T*>(P->cd), dinv_of<T>(P), n, P->st, P->partials, s);
        const T* zl = nullptr;
        sipg_status rc = precond_body<T>(P, &zl, s);
        if (rc != SIPG_OK) return rc;
        sk_cg_beta<T>(zl, P->zo, P->r, P->z, n, mz, 0, P->st, P->partials, s);
        sk_cg_direction(P->p, P->zo, n, mz, 0, P->st, s);
        std::swap(P->z, P->zo);
    }
    HIP_TRY(hipGetLastError());
    return SIPG_OK;
}

// `iters` CG iterations, eagerly or (opts.use_graph) by replaying a captured
// HIP graph of them.  A capture runs the eager enqueue on a private stream
// (the solve stream may be the null stream, which cannot be captured); its
// host-side pointer swaps are undone and re-applied on every replay, so the
// key includes the parity of z at the chunk's start.  Any failure to
// capture or instantiate falls back to the eager path.
sipg_status cg_chunk(sipg_plan* P, int iters) {
    auto eager = [&]() {
        return P->opts.precond_precision == SIPG_F32 ? cg_iterations<float>(P, iters) : cg_iterations<double>(P, iters);
    };
    if (!P->opts.use_graph) return eager();
    const int prec = P->opts.precond_precision, kind = P->opts.precond_kind, deg = P->opts.cheb_degree;
    const int mz = P->mean_zero ? 1 : 0;
    auto swaps = [&]() {
        for (int i = 0; i < iters; ++i) std::swap(P->z, P->zo);
    };
    for (auto& g : P->graphs)
        if (g.exec && g.iters == iters && g.x == P->x && g.z == P->z && g.prec == prec && g.kind == kind &&
            g.deg == deg && g.mz == mz) {
            HIP_TRY(hipGraphLaunch(g.exec, P->sstream));
            swaps();
            return SIPG_OK;
        }
    if (!P->cap_stream && hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        P->cap_stream = nullptr;
        return eager();
    }
    double *z0 = P->z, *zo0 = P->zo;
    hipStream_t real = P->sstream;
    P->sstream = P->cap_stream;
    hipGraph_t graph = nullptr;
    bool ok = hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        const sipg_status rc = eager();
        ok = hipStreamEndCapture(P->cap_stream, &graph) == hipSuccess && rc == SIPG_OK && graph != nullptr;
    }
    P->sstream = real;
    P->z = z0;
    P->zo = zo0;
    hipGraphExec_t exec = nullptr;
    if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    if (!ok) {
        if (exec) (void)hipGraphExecDestroy(exec);
        return eager();
    }
    auto& g = P->graphs[P->graph_next];
    P->graph_next ^= 1;
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = exec;
    g.iters = iters; g.prec = prec; g.kind = kind; g.deg = deg; g.mz = mz;
    g.x = P->x;
    g.z = z0;
    HIP_TRY(hipGraphLaunch(g.exec, P->sstream));
    swaps();
    return SIPG_OK;
}

sipg_status run_lanczos(sipg_plan* P, hipStream_t s) {
    const long long n = P->ndof;
    double *v = P->z, *vprev = P->zo, *w = P->q, *t = P->p;
    sk_lz_start(v, n, 12345ull, P->partials, s);
    sk_scalar(P->st, P->partials, 1, SC_LZ_NORM, n, s);
    sk_lz_normalize(v, vprev, n, P->st, s);
    sk_lz_pre(t, v, P->dinv64, n, s);
    for (int j = 0; j < P->opts.lanczos_steps; ++j) {
        sipg_status rc = do_apply<double>(P, SIPG_PART_ALL, t, w, s);
        if (rc != SIPG_OK) return rc;
        sk_lz_post_alpha(w, v, P->dinv64, n, P->st, P->partials, s);
        sk_lz_orth_beta(w, v, vprev, n, P->st, P->partials, s);
        sk_lz_next_pre(vprev, t, w, P->dinv64, n, P->st, s);  // vprev <- w / beta, t <- its pre-scaling
        std::swap(v, vprev);                                  // (vprev, v) <- (v, w/beta)
    }
    sk_lz_eig(P->st, s);
    HIP_TRY(hipGetLastError());
    P->lz_valid = true;
    P->lz_stale = false;
    P->lz_steps = P->opts.lanczos_steps;
    return SIPG_OK;
}

sipg_status enqueue_readback(sipg_plan* P) {
    HIP_TRY(hipMemcpyAsync(P->mirror, P->st, sizeof(SolveState), hipMemcpyDeviceToHost, P->sstream));
    HIP_TRY(hipEventRecord(P->ev, P->sstream));
    return SIPG_OK;
}

// restart CG from the current x with r already holding b - A x
sipg_status cg_start_from_residual(sipg_plan* P) {
    return P->opts.precond_precision == SIPG_F32 ? cg_start<float>(P) : cg_start<double>(P);
}

sipg_status enqueue_true_residual(sipg_plan* P) {
    hipStream_t s = P->sstream;
    const long long n = P->ndof;
    if (P->mean_zero) {
        sk_sum(P->x, n, P->partials, nullptr, s);
        sk_scalar(P->st, P->partials, 1, SC_MEAN, n, s);
        sk_sub_mean(P->x, n, P->st, nullptr, s);
    }
    sipg_status rc = do_apply<double>(P, SIPG_PART_ALL, P->x, P->q, s);
    if (rc != SIPG_OK) return rc;
    if (P->mean_zero) {
        sk_sum(P->b, n, P->partials, nullptr, s);
        sk_scalar(P->st, P->partials, 1, SC_MEAN, n, s);
    }
    sk_residual(P->b, P->q, P->r, n, P->mean_zero ? 1 : 0, P->st, P->partials, s);
    HIP_TRY(hipGetLastError());
    return enqueue_readback(P);
}

sipg_status check_opts(const sipg_plan* P, const sipg_solve_opts& o) {
    if (!(o.rel_tol > 0.0) || o.max_iter < 1 || o.cheb_degree < 1 || o.cheb_degree > 63 || !(o.cheb_ratio > 1.0) ||
        !(o.cheb_safety > 0.0) || o.lanczos_steps < 1 || o.lanczos_steps > 64 || o.check_every < 1 ||
        o.max_restarts < 0 || (o.precond_precision != SIPG_F32 && o.precond_precision != SIPG_F64) ||
        (o.precond_kind != SIPG_PRECOND_CHEBYSHEV && o.precond_kind != SIPG_PRECOND_MULTIGRID))
        return fail(SIPG_ERR_INVALID, "bad solve options");
    if (o.precond_kind == SIPG_PRECOND_MULTIGRID && !P->mg_on)
        return fail(SIPG_ERR_STATE, "multigrid preconditioner requested but no hierarchy was set before binding");
    return SIPG_OK;
}

// Picard work layout: vectors padded to 32 doubles (256 bytes)
long long picard_stride(long long n) { return (n + 31) / 32 * 32; }

// Viscosity from the finest level's velocity u on every level, then each
// level's diagonal; cached eigenvalue estimates are dropped.
sipg_status update_viscosity(sipg_plan* P, const double* u, hipStream_t s) {
    FineVelocity F;
    std::memset(&F, 0, sizeof(F));
    F.u = u;
    F.verts = P->curved ? P->verts64_d : nullptr;
    F.nx = P->nx; F.ny = P->ny; F.nz = P->nz; F.n = P->n;
    for (int j = 0; j < P->n; ++j) {
        F.g[j] = P->tab64.x[j];
        double den = 1.0;
        for (int m = 0; m < P->n; ++m)
            if (m != j) den *= P->tab64.x[j] - P->tab64.x[m];
        F.inv_den[j] = 1.0 / den;
    }
    const int nl = mg_levels(P);
    for (int l = 0; l < nl; ++l) {
        sipg_plan* L = mg_level(P, l);
        if (!L->bound) break;                  // coarse levels are bound only with solver workspace
        LevelPoints Lv;
        std::memset(&Lv, 0, sizeof(Lv));
        Lv.nx = L->nx; Lv.ny = L->ny; Lv.nz = L->nz; Lv.n = L->n;
        Lv.r = P->nx / L->nx;
        if (Lv.r * L->nx != P->nx || Lv.r * L->ny != P->ny || Lv.r * L->nz != P->nz || (Lv.r & (Lv.r - 1)) != 0)
            return fail(SIPG_ERR_INVALID, "multigrid level is not a power-of-two coarsening of the plan's mesh");
        for (int j = 0; j < L->n; ++j) Lv.g[j] = L->tab64.x[j];
        HIP_TRY(launch_picard_viscosity(F, Lv, L->law, L->nface, L->mu_cell64, L->mu_cell32, L->mu_face64,
                                        L->mu_face32, s));
        HIP_TRY(launch_diagonal(L->n, L->C, L->curved, L->opdata<double>(), L->diag64, L->dinv64, L->dinv32, s));
        L->lz_stale = true;
    }
    // (in order: the levels' kernels each fill the device, so side-by-side
    // streams gained nothing here, unlike the latency-bound Lanczos chains)
    if (!P->cg.empty() && P->with_solver) return refresh_continuous(P, s);
    return SIPG_OK;
}

// Streams and events for side-by-side per-level work, created once per plan;
// false (and nothing kept) if the runtime refuses any of them.
bool aux_ready(sipg_plan* P) {
    if (P->aux_fork) return true;
    if (P->aux_failed) return false;
    bool ok = hipEventCreateWithFlags(&P->aux_fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; ok && k < sipg_plan::kAuxStreams; ++k)
        ok = hipStreamCreateWithFlags(&P->aux_streams[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&P->aux_join[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        for (int k = 0; k < sipg_plan::kAuxStreams; ++k) {
            if (P->aux_streams[k]) (void)hipStreamDestroy(P->aux_streams[k]);
            if (P->aux_join[k]) (void)hipEventDestroy(P->aux_join[k]);
            P->aux_streams[k] = nullptr;
            P->aux_join[k] = nullptr;
        }
        if (P->aux_fork) (void)hipEventDestroy(P->aux_fork);
        P->aux_fork = nullptr;
        P->aux_failed = true;
        (void)hipGetLastError();
    }
    return ok;
}

// Runs per-level jobs: in order on s, or, when there are several and the
// plan may use its own streams (not while s is being captured, not in the
// no-allocation entry point), side by side on the plan's auxiliary streams
// between a fork and a join on s.  Every job works on its own level's
// buffers, state and partial sums, so the results do not depend on the
// schedule.
sipg_status run_jobs(sipg_plan* P, std::vector<std::function<sipg_status(hipStream_t)>>& jobs, hipStream_t s) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool side = jobs.size() > 1 && !P->no_alloc && hipStreamIsCapturing(s, &cap) == hipSuccess &&
                      cap == hipStreamCaptureStatusNone && aux_ready(P);
    if (!side) {
        for (auto& j : jobs) {
            const sipg_status rc = j(s);
            if (rc != SIPG_OK) return rc;
        }
        return SIPG_OK;
    }
    const int K = sipg_plan::kAuxStreams;
    HIP_TRY(hipEventRecord(P->aux_fork, s));
    for (int k = 0; k < K; ++k) HIP_TRY(hipStreamWaitEvent(P->aux_streams[k], P->aux_fork, 0));
    sipg_status first = SIPG_OK;
    for (size_t i = 0; i < jobs.size(); ++i) {
        const sipg_status rc = jobs[i](P->aux_streams[i % K]);
        if (rc != SIPG_OK && first == SIPG_OK) first = rc;
        if (rc != SIPG_OK) break;
    }
    // join every stream, also after a failure, so that s orders after all of them
    for (int k = 0; k < K; ++k) {
        HIP_TRY(hipEventRecord(P->aux_join[k], P->aux_streams[k]));
        HIP_TRY(hipStreamWaitEvent(s, P->aux_join[k], 0));
    }
    return first;
}

// Eigenvalue estimates (cached per level) and Chebyshev coefficients of the
// preconditioner in P->opts: the finest level's polynomial, and with
// multigrid every coarser level's (coarse_degree on the coarsest).
sipg_status prepare_precond(sipg_plan* P, hipStream_t s) {
    const sipg_solve_opts& o = P->opts;
    const bool mg = o.precond_kind == SIPG_PRECOND_MULTIGRID;
    const bool cph = mg && !P->cg.empty();
    // cph: the DG level and the continuous levels (the coarser DG plans only
    // carry the continuous levels' operators)
    const int nl = mg ? (cph ? 1 : mg_levels(P)) : 1;
    // the levels whose estimates are missing or stale, largest first
    std::vector<std::function<sipg_status(hipStream_t)>> jobs;
    for (int l = 0; l < nl; ++l) {
        sipg_plan* L = mg_level(P, l);
        if (l > 0) L->opts = o;
        if (!L->lz_valid || L->lz_steps != o.lanczos_steps || (L->lz_stale && !o.reuse_eigs))
            jobs.push_back([L](hipStream_t t) { return run_lanczos(L, t); });
    }
    if (cph) {
        for (size_t i = 0; i < P->cg.size(); ++i) {
            CgLevel& c = P->cg[i];
            if (!c.lz_valid || c.lz_steps != o.lanczos_steps || (c.lz_stale && !o.reuse_eigs)) {
                const int steps = o.lanczos_steps;
                jobs.push_back([&c, steps](hipStream_t t) { return run_lanczos_cg(c, steps, t); });
            }
        }
    }
    const sipg_status rc = run_jobs(P, jobs, s);
    if (rc != SIPG_OK) return rc;
    if (cph) {
        for (size_t i = 0; i < P->cg.size(); ++i) {
            CgLevel& c = P->cg[i];
            const bool coarse_poly = i + 1 == P->cg.size() && !c.direct;
            sk_lz_coef(c.st, o.cheb_safety, o.cheb_ratio, coarse_poly ? P->mg_opts.coarse_degree : o.cheb_degree, s);
        }
    }
    for (int l = 0; l < nl; ++l) {
        sipg_plan* L = mg_level(P, l);
        const int deg = (mg && !cph && l == nl - 1) ? P->mg_opts.coarse_degree : o.cheb_degree;
        sk_lz_coef(L->st, o.cheb_safety, o.cheb_ratio, deg, s);
    }
    HIP_TRY(hipGetLastError());
    return SIPG_OK;
}

// Lagrange basis of the n Gauss points of [0, 1] at x.
void lagrange_at(int n, double x, double* out) {
    double g[kMaxN], w[kMaxN];
    gauss_legendre01(n, g, w);
    for (int j = 0; j < n; ++j) {
        double v = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != j) v *= (x - g[m]) / (g[j] - g[m]);
        out[j] = v;
    }
}

// Transfer tables from a level with nf nodes per direction to one with nc.
void fill_transfer(sipg_plan* Cc, int nf, int nc) {
    double xf[kMaxN], wf[kMaxN], row[kMaxN];
    gauss_legendre01(nf, xf, wf);
    std::memset(&Cc->tr64, 0, sizeof(Cc->tr64));
    std::memset(&Cc->tr32, 0, sizeof(Cc->tr32));
    for (int i = 0; i < nf; ++i) {
        lagrange_at(nc, xf[i], row);                       // degree step: coarse basis at fine nodes
        for (int j = 0; j < nc; ++j) { Cc->tr64.P[i][j] = row[j]; Cc->tr32.P[i][j] = float(row[j]); }
        for (int b = 0; b < 2; ++b) {                      // mesh step: parent basis at child b's nodes
            lagrange_at(nc, 0.5 * (b + xf[i]), row);
            for (int j = 0; j < nc; ++j) { Cc->tr64.H[b][i][j] = row[j]; Cc->tr32.H[b][i][j] = float(row[j]); }
        }
    }
}

}  // namespace

extern "C" {

int32_t sipg_abi_version(void) { return 2; }

const char* sipg_last_error(void) { return g_err.c_str(); }

sipg_status sipg_plan_create(const sipg_mesh* mesh, const sipg_viscosity* law, const sipg_params* params,
                             sipg_plan** out) {
    if (out) *out = nullptr;
    if (!mesh || !params || !out) return fail(SIPG_ERR_INVALID, "null argument");
    if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1) return fail(SIPG_ERR_INVALID, "mesh needs >= 1 cell per direction");
    if (params->degree < 1 || params->degree > 5) return fail(SIPG_ERR_INVALID, "degree must be 1..5");
    if (params->op != SIPG_VISCOUS && params->op != SIPG_POISSON && params->op != SIPG_PENALTY)
        return fail(SIPG_ERR_INVALID, "unknown operator");
    if (params->op == SIPG_PENALTY && (!params->tau_div || !params->tau_cont))
        return fail(SIPG_ERR_INVALID, "penalty operator needs tau_div and tau_cont per cell");
    if (!(params->alpha >= 0.0) || !std::isfinite(params->alpha)) return fail(SIPG_ERR_INVALID, "alpha must be >= 0");
    if (!(params->penalty > 0.0) || !std::isfinite(params->penalty)) return fail(SIPG_ERR_INVALID, "penalty must be > 0");
    for (int i = 0; i < 6; ++i)
        if (mesh->bc[i] != SIPG_BC_DIRICHLET && mesh->bc[i] != SIPG_BC_NEUMANN) return fail(SIPG_ERR_INVALID, "bad bc value");
    if ((long long)(mesh->nx + 1) * (mesh->ny + 1) * (mesh->nz + 1) * 3 >= (1ll << 31))
        return fail(SIPG_ERR_INVALID, "mesh too large: 2^31 or more vertex coordinates");
    const long long ncell = (long long)mesh->nx * mesh->ny * mesh->nz;
    const int n = params->degree + 1, C = params->op == SIPG_POISSON ? 1 : 3;
    const long long ndof = ncell * C * n * n * n;
    if (ndof > (1ll << 31) - 1 || ncell * n * n * n > (1ll << 31) - 1)
        return fail(SIPG_ERR_UNSUPPORTED, "problem too large for 32-bit cell indexing");

    sipg_plan* P = new (std::nothrow) sipg_plan();
    if (!P) return fail(SIPG_ERR_OOM, "host allocation failed");
    P->nx = mesh->nx; P->ny = mesh->ny; P->nz = mesh->nz;
    for (int i = 0; i < 6; ++i) P->bc[i] = mesh->bc[i];
    P->op = params->op; P->degree = params->degree; P->n = n; P->C = C;
    P->alpha = params->alpha; P->penalty = params->penalty;
    P->ncell = ncell; P->ndof = ndof;
    P->nface = (long long)(mesh->nx + 1) * mesh->ny * mesh->nz + (long long)mesh->nx * (mesh->ny + 1) * mesh->nz +
               (long long)mesh->nx * mesh->ny * (mesh->nz + 1);
    P->nvert = (long long)(mesh->nx + 1) * (mesh->ny + 1) * (mesh->nz + 1);
    P->curved = mesh->vertices != nullptr;
    if (P->curved) {
        P->verts.assign(mesh->vertices, mesh->vertices + P->nvert * 3);
        for (double v : P->verts)
            if (!std::isfinite(v)) { delete P; return fail(SIPG_ERR_INVALID, "non-finite vertex"); }
        if (cell_corner_det_min(P) <= 0.0) { delete P; return fail(SIPG_ERR_INVALID, "a cell has det J <= 0 at a corner"); }
        P->verts32.assign(P->verts.begin(), P->verts.end());
    }
    std::memset(&P->law, 0, sizeof(P->law));
    if (params->op == SIPG_PENALTY) {
        P->pen = true;
        P->tau_div.assign(params->tau_div, params->tau_div + ncell);
        P->tau_cont.assign(params->tau_cont, params->tau_cont + ncell);
        for (long long e = 0; e < ncell; ++e)
            if (!(P->tau_div[e] >= 0.0) || !(P->tau_cont[e] >= 0.0) || !std::isfinite(P->tau_div[e]) ||
                !std::isfinite(P->tau_cont[e])) {
                delete P;
                return fail(SIPG_ERR_INVALID, "penalty factors must be finite and >= 0");
            }
    } else if (C == 3) {
        if (!law) { delete P; return fail(SIPG_ERR_INVALID, "viscous operator needs a viscosity law"); }
        LawDev& L = P->law;
        L.kind = law->kind;
        L.mu = law->mu; L.amp = law->amp; L.contrast = law->contrast; L.rmin = law->rmin; L.rmax = law->rmax;
        L.mu0 = law->mu0; L.mu_inf = law->mu_inf; L.lam = law->lam; L.n_exp = law->n_exp; L.kappa = law->kappa;
        L.a_exp = law->a_exp;
        switch (law->kind) {
            case SIPG_LAW_CONST:
                if (!(law->mu >= 0.0)) { delete P; return fail(SIPG_ERR_INVALID, "CONST law needs mu >= 0"); }
                break;
            case SIPG_LAW_SINE:
                if (!(law->mu > 0.0) || !(std::fabs(law->amp) < 1.0)) {
                    delete P; return fail(SIPG_ERR_INVALID, "SINE law needs mu > 0 and |amp| < 1");
                }
                break;
            case SIPG_LAW_LOGFIELD:
            case SIPG_LAW_CARREAU: {
                if (law->n_modes < 0 || law->n_modes > SIPG_MAX_MODES || (law->n_modes > 0 && (!law->k || !law->phi))) {
                    delete P; return fail(SIPG_ERR_INVALID, "law modes missing or more than SIPG_MAX_MODES");
                }
                L.n_modes = law->n_modes;
                for (int m = 0; m < law->n_modes; ++m) {
                    for (int i = 0; i < 3; ++i) L.k[m][i] = law->k[3 * m + i];
                    L.phi[m] = law->phi[m];
                }
                if (law->kind == SIPG_LAW_LOGFIELD) {
                    if (law->n_modes > 0 && !law->a) { delete P; return fail(SIPG_ERR_INVALID, "LOGFIELD needs amplitudes"); }
                    if (!(law->contrast > 0.0) || !(law->rmax > law->rmin)) {
                        delete P; return fail(SIPG_ERR_INVALID, "LOGFIELD needs contrast > 0 and rmax > rmin");
                    }
                    for (int m = 0; m < law->n_modes; ++m) L.a[m] = law->a[m];
                } else {
                    if (law->n_modes > 0 && !law->v) { delete P; return fail(SIPG_ERR_INVALID, "CARREAU needs velocity modes"); }
                    if (!(law->mu_inf >= 0.0) || !(law->mu0 > 0.0) || !(law->a_exp > 0.0)) {
                        delete P; return fail(SIPG_ERR_INVALID, "CARREAU needs mu0 > 0, mu_inf >= 0, a > 0");
                    }
                    for (int m = 0; m < law->n_modes; ++m)
                        for (int i = 0; i < 3; ++i) L.v[m][i] = law->v[3 * m + i];
                }
                break;
            }
            case SIPG_LAW_ARRAYS: {
                if (!law->mu_cell || !law->mu_face) {
                    delete P; return fail(SIPG_ERR_INVALID, "ARRAYS law needs mu_cell and mu_face");
                }
                const size_t nc = (size_t)ncell * n * n * n, nf = (size_t)P->nface * n * n;
                P->mu_cell_h.assign(law->mu_cell, law->mu_cell + nc);
                P->mu_face_h.assign(law->mu_face, law->mu_face + nf);
                for (double v : P->mu_cell_h)
                    if (!(v >= 0.0) || !std::isfinite(v)) { delete P; return fail(SIPG_ERR_INVALID, "ARRAYS values must be finite and >= 0"); }
                for (double v : P->mu_face_h)
                    if (!(v >= 0.0) || !std::isfinite(v)) { delete P; return fail(SIPG_ERR_INVALID, "ARRAYS values must be finite and >= 0"); }
                P->mu_cell_h32.assign(P->mu_cell_h.begin(), P->mu_cell_h.end());
                P->mu_face_h32.assign(P->mu_face_h.begin(), P->mu_face_h.end());
                break;
            }
            default:
                delete P;
                return fail(SIPG_ERR_INVALID, "unknown viscosity law");
        }
    }
    fill_tables<double>(n, P->tab64);
    fill_tables<float>(n, P->tab32);
    std::memset(&P->info, 0, sizeof(P->info));
    sipg_solve_opts_default(&P->opts);
    *out = P;
    g_err.clear();
    return SIPG_OK;
}

void drop_graphs(sipg_plan* P) {
    for (auto& g : P->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = sipg_plan::GraphEntry();
    }
}

void sipg_plan_destroy(sipg_plan* P) {
    if (!P) return;
    drop_graphs(P);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    for (int k = 0; k < sipg_plan::kAuxStreams; ++k) {
        if (P->aux_streams[k]) (void)hipStreamDestroy(P->aux_streams[k]);
        if (P->aux_join[k]) (void)hipEventDestroy(P->aux_join[k]);
    }
    if (P->aux_fork) (void)hipEventDestroy(P->aux_fork);
    for (sipg_plan* c : P->mg) sipg_plan_destroy(c);
    if (P->mirror) (void)hipHostFree(P->mirror);
    if (P->ev) (void)hipEventDestroy(P->ev);
    delete P;
}

int64_t sipg_dof_count(const sipg_plan* P) { return P ? P->ndof : -1; }
int64_t sipg_face_count(const sipg_plan* P) { return P ? P->nface : -1; }

sipg_status sipg_plan_workspace_bytes(const sipg_plan* P, int32_t with_solver, size_t* bytes) {
    if (!valid_plan(P) || !bytes) return fail(SIPG_ERR_INVALID, "null argument");
    const Layout L = layout(P);
    *bytes = with_solver ? L.total : L.op_end;
    return SIPG_OK;
}

sipg_status sipg_plan_bind(sipg_plan* P, void* workspace, size_t bytes, int32_t with_solver, void* stream) {
    if (!valid_plan(P)) return fail(SIPG_ERR_INVALID, "null plan");
    if (!workspace) return fail(SIPG_ERR_INVALID, "null workspace");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(SIPG_ERR_INVALID, "workspace must be 256-byte aligned");
    const Layout L = layout(P);
    const size_t need = with_solver ? L.total : L.op_end;
    if (bytes < need) return fail(SIPG_ERR_OOM, "workspace too small: need " + std::to_string(need) + " bytes");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(workspace);
    P->ws = w;
    P->verts64_d = P->curved ? reinterpret_cast<double*>(w + L.verts64) : nullptr;
    P->verts32_d = P->curved ? reinterpret_cast<float*>(w + L.verts32) : nullptr;
    P->hcell = reinterpret_cast<double*>(w + L.hcell);
    P->tfac64 = reinterpret_cast<double*>(w + L.tfac64);
    P->tfac32 = reinterpret_cast<float*>(w + L.tfac32);
    if (P->C == 3) {
        P->mu_cell64 = reinterpret_cast<double*>(w + L.mu_cell64);
        P->mu_cell32 = reinterpret_cast<float*>(w + L.mu_cell32);
        if (!P->pen) {
            P->mu_face64 = reinterpret_cast<double*>(w + L.mu_face64);
            P->mu_face32 = reinterpret_cast<float*>(w + L.mu_face32);
        }
    }
    if (P->pen) {
        P->tau_div_d = reinterpret_cast<double*>(w + L.tdiv);
        P->tau_cont_d = reinterpret_cast<double*>(w + L.tcont);
    }
    P->diag64 = reinterpret_cast<double*>(w + L.diag64);
    P->dinv64 = reinterpret_cast<double*>(w + L.dinv64);
    P->dinv32 = reinterpret_cast<float*>(w + L.dinv32);
    P->with_solver = with_solver != 0;
    if (P->with_solver) {
        P->r = reinterpret_cast<double*>(w + L.r);
        P->p = reinterpret_cast<double*>(w + L.p);
        P->q = reinterpret_cast<double*>(w + L.q);
        P->z = reinterpret_cast<double*>(w + L.z);
        P->zo = reinterpret_cast<double*>(w + L.zo);
        P->cr = w + L.cr; P->cd = w + L.cd; P->cz0 = w + L.cz0; P->cz1 = w + L.cz1;
        P->partials = reinterpret_cast<double*>(w + L.partials);
        P->st = reinterpret_cast<SolveState*>(w + L.st);
        if (!P->mirror) HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&P->mirror), sizeof(SolveState), hipHostMallocDefault));
        if (!P->ev) HIP_TRY(hipEventCreateWithFlags(&P->ev, hipEventDisableTiming));
        HIP_TRY(hipMemsetAsync(P->st, 0, sizeof(SolveState), s));
    }
    P->lz_valid = false;
    P->phase = PH_IDLE;
    drop_graphs(P);  // captured chunks refer to the old workspace
    if (P->curved) {
        HIP_TRY(hipMemcpyAsync(P->verts64_d, P->verts.data(), P->verts.size() * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(P->verts32_d, P->verts32.data(), P->verts32.size() * 4, hipMemcpyHostToDevice, s));
    }
    if (P->pen) {
        HIP_TRY(hipMemcpyAsync(P->tau_div_d, P->tau_div.data(), P->ncell * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(P->tau_cont_d, P->tau_cont.data(), P->ncell * 8, hipMemcpyHostToDevice, s));
    }
    const OpData<double> od = P->opdata<double>();
    HIP_TRY(launch_setup(P->n, P->C, P->curved, od, P->law, P->penalty, P->hcell, P->tfac64, P->tfac32, P->mu_cell64,
                         P->mu_cell32, P->mu_face64, P->mu_face32, (int)P->nface, P->tau_div_d, P->tau_cont_d, s));
    if (P->law.kind == SIPG_LAW_ARRAYS && P->C == 3 && !P->pen) {
        HIP_TRY(hipMemcpyAsync(P->mu_cell64, P->mu_cell_h.data(), P->mu_cell_h.size() * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(P->mu_face64, P->mu_face_h.data(), P->mu_face_h.size() * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(P->mu_cell32, P->mu_cell_h32.data(), P->mu_cell_h32.size() * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(P->mu_face32, P->mu_face_h32.data(), P->mu_face_h32.size() * 4, hipMemcpyHostToDevice, s));
    }
    const OpData<double> od2 = P->opdata<double>();
    HIP_TRY(launch_diagonal(P->n, P->C, P->curved, od2, P->diag64, P->dinv64, P->dinv32, s));
    if (P->mg_on && P->with_solver) {
        P->mgz = w + L.mgz;
        P->mgt = w + L.mgt;
        for (size_t i = 0; i < P->mg.size(); ++i) {
            const sipg_status rc = sipg_plan_bind(P->mg[i], w + L.level[i], L.level_bytes[i], 1, stream);
            if (rc != SIPG_OK) return rc;
        }
        for (size_t i = 0; i < P->cg.size(); ++i) {
            CgLevel& c = P->cg[i];
            const Layout::Cg& g = L.cg[i];
            void** vecs[8] = {&c.r, &c.za, &c.zb, &c.d, &c.t, &c.zk, &c.ta, &c.tb};
            for (int k = 0; k < 8; ++k) *vecs[k] = w + g.vec[k];
            c.diag64 = reinterpret_cast<double*>(w + g.diag64);
            c.dinv64 = reinterpret_cast<double*>(w + g.dinv64);
            c.dinv32 = reinterpret_cast<float*>(w + g.dinv32);
            c.dgx = w + g.dgx;
            c.dgy = w + g.dgy;
            c.st = reinterpret_cast<SolveState*>(w + g.st);
            c.partials = reinterpret_cast<double*>(w + g.partials);
            HIP_TRY(hipMemsetAsync(c.st, 0, sizeof(SolveState), s));
            for (int a = 0; a < 3; ++a) {
                c.prp[a] = reinterpret_cast<int*>(w + g.prp[a]);
                c.pci[a] = reinterpret_cast<int*>(w + g.pci[a]);
                c.pv64[a] = reinterpret_cast<double*>(w + g.pv64[a]);
                c.pv32[a] = reinterpret_cast<float*>(w + g.pv32[a]);
                c.rrp[a] = reinterpret_cast<int*>(w + g.rrp[a]);
                c.rci[a] = reinterpret_cast<int*>(w + g.rci[a]);
                c.rv64[a] = reinterpret_cast<double*>(w + g.rv64[a]);
                c.rv32[a] = reinterpret_cast<float*>(w + g.rv32[a]);
                auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
                    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
                };
                HIP_TRY(up(c.prp[a], c.P[a].rp.data(), c.P[a].rp.size() * 4));
                HIP_TRY(up(c.pci[a], c.P[a].ci.data(), c.P[a].ci.size() * 4));
                HIP_TRY(up(c.pv64[a], c.P[a].v.data(), c.P[a].v.size() * 8));
                HIP_TRY(up(c.rrp[a], c.R[a].rp.data(), c.R[a].rp.size() * 4));
                HIP_TRY(up(c.rci[a], c.R[a].ci.data(), c.R[a].ci.size() * 4));
                HIP_TRY(up(c.rv64[a], c.R[a].v.data(), c.R[a].v.size() * 8));
                if (!c.P[a].v.empty()) sk_cast(c.pv32[a], c.pv64[a], (long long)c.P[a].v.size(), s);
                if (!c.R[a].v.empty()) sk_cast(c.rv32[a], c.rv64[a], (long long)c.R[a].v.size(), s);
            }
            c.cinv = c.direct ? reinterpret_cast<double*>(w + g.cinv) : nullptr;
            c.cwork = c.direct ? reinterpret_cast<double*>(w + g.cwork) : nullptr;
            c.probes = c.direct ? reinterpret_cast<double*>(w + g.probes) : nullptr;
            c.lz_valid = false;
        }
        const sipg_status rc = refresh_continuous(P, s);
        if (rc != SIPG_OK) return rc;
    }
    P->bound = true;
    g_err.clear();
    return SIPG_OK;
}

sipg_status sipg_apply_parts(sipg_plan* P, int32_t precision, int32_t parts, const void* x, void* y, void* stream) {
    if (!valid_plan(P) || !x || !y) return fail(SIPG_ERR_INVALID, "null argument");
    if (!P->bound) return fail(SIPG_ERR_STATE, "plan not bound");
    if (x == y) return fail(SIPG_ERR_INVALID, "x and y must not alias");
    if (parts & ~SIPG_PART_ALL) return fail(SIPG_ERR_INVALID, "bad parts mask");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == SIPG_F64) return do_apply<double>(P, parts, x, y, s);
    if (precision == SIPG_F32) return do_apply<float>(P, parts, x, y, s);
    return fail(SIPG_ERR_INVALID, "bad precision");
}

sipg_status sipg_apply(sipg_plan* P, int32_t precision, const void* x, void* y, void* stream) {
    return sipg_apply_parts(P, precision, SIPG_PART_ALL, x, y, stream);
}

sipg_status sipg_diagonal(sipg_plan* P, int32_t precision, int32_t inverse, void* out, void* stream) {
    if (!valid_plan(P) || !out) return fail(SIPG_ERR_INVALID, "null argument");
    if (!P->bound) return fail(SIPG_ERR_STATE, "plan not bound");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long long n = P->ndof;
    if (precision == SIPG_F64) {
        HIP_TRY(hipMemcpyAsync(out, inverse ? P->dinv64 : P->diag64, n * 8, hipMemcpyDeviceToDevice, s));
    } else if (precision == SIPG_F32) {
        if (inverse) HIP_TRY(hipMemcpyAsync(out, P->dinv32, n * 4, hipMemcpyDeviceToDevice, s));
        else sk_cast(static_cast<float*>(out), P->diag64, n, s);
    } else {
        return fail(SIPG_ERR_INVALID, "bad precision");
    }
    HIP_TRY(hipGetLastError());
    return SIPG_OK;
}

sipg_status sipg_viscosity_values(sipg_plan* P, double* mu_cell, double* mu_face, void* stream) {
    if (!valid_plan(P)) return fail(SIPG_ERR_INVALID, "null plan");
    if (!P->bound) return fail(SIPG_ERR_STATE, "plan not bound");
    if (P->op != SIPG_VISCOUS) return fail(SIPG_ERR_INVALID, "only the viscous operator has a viscosity");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nn = (size_t)P->n * P->n;
    if (mu_cell) HIP_TRY(hipMemcpyAsync(mu_cell, P->mu_cell64, P->ncell * nn * P->n * 8, hipMemcpyDeviceToDevice, s));
    if (mu_face) HIP_TRY(hipMemcpyAsync(mu_face, P->mu_face64, P->nface * nn * 8, hipMemcpyDeviceToDevice, s));
    return SIPG_OK;
}

void sipg_solve_opts_default(sipg_solve_opts* o) {
    if (!o) return;
    o->rel_tol = 1e-8;
    o->max_iter = 5000;
    o->precond_precision = SIPG_F32;
    o->cheb_degree = 5;
    o->cheb_ratio = 20.0;
    o->cheb_safety = 1.2;
    o->lanczos_steps = 20;
    o->check_every = 10;
    o->max_restarts = 3;
    o->precond_kind = SIPG_PRECOND_CHEBYSHEV;
    o->use_graph = 0;
    o->reuse_eigs = 0;
}

void sipg_mg_opts_default(sipg_mg_opts* o) {
    if (!o) return;
    o->coarse_degree = 12;
    o->min_cells = 2;
    o->max_levels = 16;
    o->h_coarsen = 1;
    o->continuous = 1;
    o->direct_max = 1024;
}

sipg_status sipg_plan_set_multigrid(sipg_plan* P, const sipg_mg_opts* opts) {
    if (!valid_plan(P)) return fail(SIPG_ERR_INVALID, "null plan");
    if (P->bound) return fail(SIPG_ERR_STATE, "set the multigrid hierarchy before binding the plan");
    sipg_mg_opts o;
    if (opts) o = *opts; else sipg_mg_opts_default(&o);
    if (o.coarse_degree < 1 || o.coarse_degree > 63 || o.min_cells < 1 || o.max_levels < 1 ||
        (o.continuous != 0 && o.continuous != 1) || o.direct_max < 0 || o.direct_max > 2048)
        return fail(SIPG_ERR_INVALID, "bad multigrid options");
    P->cg.clear();
    if (P->C == 3 && !P->pen && P->law.kind == SIPG_LAW_ARRAYS)
        return fail(SIPG_ERR_UNSUPPORTED, "tabulated viscosity (ARRAYS law) has no values on coarse levels");
    for (sipg_plan* c : P->mg) sipg_plan_destroy(c);
    P->mg.clear();
    // levels: degree k-1 .. 1 on the plan's mesh, then the mesh halved while possible
    int deg = P->degree, nx = P->nx, ny = P->ny, nz = P->nz;
    std::vector<double> verts = P->verts;
    std::vector<double> td = P->tau_div, tc = P->tau_cont;   // penalty step: factors of the level's cells
    int nlev = 1, n_prev = P->n;
    auto add_level = [&](bool mesh_step) -> sipg_status {
        sipg_mesh m;
        std::memset(&m, 0, sizeof(m));
        m.nx = nx; m.ny = ny; m.nz = nz;
        m.vertices = P->curved ? verts.data() : nullptr;
        for (int i = 0; i < 6; ++i) m.bc[i] = P->bc[i];
        sipg_viscosity law;
        std::memset(&law, 0, sizeof(law));
        law.kind = SIPG_LAW_CONST;
        law.mu = 1.0;                                   // replaced by the plan's law below
        sipg_params par;
        std::memset(&par, 0, sizeof(par));
        par.op = P->op; par.degree = deg; par.alpha = P->alpha; par.penalty = P->penalty;
        par.tau_div = td.empty() ? nullptr : td.data();
        par.tau_cont = tc.empty() ? nullptr : tc.data();
        sipg_plan* c = nullptr;
        const sipg_status rc = sipg_plan_create(&m, &law, &par, &c);
        if (rc != SIPG_OK) return rc;
        c->law = P->law;
        c->mesh_step = mesh_step;
        fill_transfer(c, n_prev, c->n);
        n_prev = c->n;
        P->mg.push_back(c);
        ++nlev;
        return SIPG_OK;
    };
    sipg_status rc = SIPG_OK;
    while (rc == SIPG_OK && deg > 1 && nlev < o.max_levels) {
        --deg;
        rc = add_level(false);
    }
    auto halvable = [&](int c) { return c % 2 == 0 && c / 2 >= o.min_cells; };
    while (rc == SIPG_OK && o.h_coarsen && nlev < o.max_levels && halvable(nx) && halvable(ny) && halvable(nz)) {
        if (P->curved) {                                 // every other vertex of the finer mesh
            std::vector<double> cv;
            cv.reserve((size_t)(nx / 2 + 1) * (ny / 2 + 1) * (nz / 2 + 1) * 3);
            for (int k = 0; k <= nz; k += 2)
                for (int j = 0; j <= ny; j += 2)
                    for (int i = 0; i <= nx; i += 2)
                        for (int d = 0; d < 3; ++d)
                            cv.push_back(verts[(((size_t)k * (ny + 1) + j) * (nx + 1) + i) * 3 + d]);
            verts.swap(cv);
        }
        if (P->pen) {                                    // a coarse cell takes the mean of its 8 children
            std::vector<double> ctd((size_t)(nx / 2) * (ny / 2) * (nz / 2)), ctc(ctd.size());
            for (int k = 0; k < nz / 2; ++k)
                for (int j = 0; j < ny / 2; ++j)
                    for (int i = 0; i < nx / 2; ++i) {
                        double a = 0.0, b = 0.0;
                        for (int c = 0; c < 8; ++c) {
                            const size_t f = ((size_t)(2 * k + (c >> 2)) * ny + 2 * j + ((c >> 1) & 1)) * nx +
                                             2 * i + (c & 1);
                            a += td[f];
                            b += tc[f];
                        }
                        const size_t e = ((size_t)k * (ny / 2) + j) * (nx / 2) + i;
                        ctd[e] = a / 8.0;
                        ctc[e] = b / 8.0;
                    }
            td.swap(ctd);
            tc.swap(ctc);
        }
        nx /= 2; ny /= 2; nz /= 2;
        rc = add_level(true);
    }
    if (rc != SIPG_OK) {
        for (sipg_plan* c : P->mg) sipg_plan_destroy(c);
        P->mg.clear();
        P->mg_on = false;
        return rc;
    }
    P->mg_opts = o;
    P->mg_on = true;
    if (o.continuous) build_continuous_levels(P);
    g_err.clear();
    return SIPG_OK;
}

int32_t sipg_multigrid_levels(const sipg_plan* P, int32_t* degrees, int32_t* cells, int32_t cap) {
    if (!P) return 0;
    const int nl = P->mg_on ? 1 + (int)P->mg.size() : 1;
    for (int l = 0; l < nl && l < cap; ++l) {
        const sipg_plan* L = l == 0 ? P : P->mg[l - 1];
        if (degrees) degrees[l] = L->degree;
        if (cells) { cells[3 * l] = L->nx; cells[3 * l + 1] = L->ny; cells[3 * l + 2] = L->nz; }
    }
    return nl;
}

sipg_status sipg_multigrid_transfer(sipg_plan* P, int32_t level, int32_t restrict_, int32_t precision,
                                    const void* in, void* out, void* stream) {
    if (!valid_plan(P) || !in || !out) return fail(SIPG_ERR_INVALID, "null argument");
    if (!P->bound) return fail(SIPG_ERR_STATE, "plan not bound");
    if (!P->mg_on || level < 0 || level + 1 >= mg_levels(P)) return fail(SIPG_ERR_INVALID, "no such level pair");
    if (precision != SIPG_F64 && precision != SIPG_F32) return fail(SIPG_ERR_INVALID, "bad precision");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const sipg_plan* F = mg_level(P, level);
    const sipg_plan* Cc = P->mg[level];
    if (precision == SIPG_F64) {
        if (restrict_)
            HIP_TRY(launch_restrict<double>(Cc->mesh_step, F->C, F->n, Cc->n, F->nx, F->ny, F->nz, Cc->tr64,
                                            static_cast<const double*>(in), static_cast<double*>(out), nullptr, s));
        else
            HIP_TRY(launch_prolong_add<double>(Cc->mesh_step, F->C, F->n, Cc->n, F->nx, F->ny, F->nz, Cc->tr64,
                                               static_cast<const double*>(in), static_cast<double*>(out), nullptr, s));
    } else {
        if (restrict_)
            HIP_TRY(launch_restrict<float>(Cc->mesh_step, F->C, F->n, Cc->n, F->nx, F->ny, F->nz, Cc->tr32,
                                           static_cast<const float*>(in), static_cast<float*>(out), nullptr, s));
        else
            HIP_TRY(launch_prolong_add<float>(Cc->mesh_step, F->C, F->n, Cc->n, F->nx, F->ny, F->nz, Cc->tr32,
                                              static_cast<const float*>(in), static_cast<float*>(out), nullptr, s));
    }
    return SIPG_OK;
}

sipg_status sipg_precondition(sipg_plan* P, const double* r, double* z, const sipg_solve_opts* opts, void* stream) {
    if (!valid_plan(P) || !r || !z) return fail(SIPG_ERR_INVALID, "null argument");
    if (!P->bound || !P->with_solver) return fail(SIPG_ERR_STATE, "plan not bound with solver workspace");
    if (P->phase == PH_RUNNING || P->phase == PH_CHECKING) return fail(SIPG_ERR_STATE, "a solve is in progress on this plan");
    sipg_solve_opts o;
    if (opts) o = *opts; else sipg_solve_opts_default(&o);
    sipg_status rc = check_opts(P, o);
    if (rc != SIPG_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    P->opts = o;
    const long long n = P->ndof;
    sk_state_init(P->st, 0.0, 1, s);                    // clears the skip flag
    if ((rc = prepare_precond(P, s)) != SIPG_OK) return rc;
    sk_copy(P->r, r, n, s);
    if (o.precond_precision == SIPG_F32) {
        sk_cheb_start<float>(P->r, static_cast<float*>(P->cr), static_cast<float*>(P->cz0), static_cast<float*>(P->cd),
                             P->dinv32, n, P->st, s);
        const float* zl = nullptr;
        if ((rc = precond_body<float>(P, &zl, s)) != SIPG_OK) return rc;
        HIP_TRY(launch_to_f64<float>(z, zl, n, s));
    } else {
        sk_cheb_start<double>(P->r, static_cast<double*>(P->cr), static_cast<double*>(P->cz0),
                              static_cast<double*>(P->cd), P->dinv64, n, P->st, s);
        const double* zl = nullptr;
        if ((rc = precond_body<double>(P, &zl, s)) != SIPG_OK) return rc;
        HIP_TRY(launch_to_f64<double>(z, zl, n, s));
    }
    P->phase = PH_IDLE;
    return SIPG_OK;
}

sipg_status sipg_solve_begin(sipg_plan* P, const double* b, double* x, const sipg_solve_opts* opts, void* stream) {
    if (!valid_plan(P) || !b || !x) return fail(SIPG_ERR_INVALID, "null argument");
    if (!P->bound || !P->with_solver) return fail(SIPG_ERR_STATE, "plan not bound with solver workspace");
    if (P->phase == PH_RUNNING || P->phase == PH_CHECKING) return fail(SIPG_ERR_STATE, "a solve is in progress on this plan");
    sipg_solve_opts o;
    if (opts) o = *opts; else sipg_solve_opts_default(&o);
    sipg_status vrc = check_opts(P, o);
    if (vrc != SIPG_OK) return vrc;
    const bool all_neumann = std::all_of(P->bc, P->bc + 6, [](int v) { return v == SIPG_BC_NEUMANN; });
    if (P->pen && P->alpha == 0.0)
        return fail(SIPG_ERR_UNSUPPORTED, "penalty operator with alpha = 0 is singular (continuous divergence-free fields)");
    if (P->C == 3 && all_neumann && P->alpha == 0.0)
        return fail(SIPG_ERR_UNSUPPORTED, "pure-Neumann viscous operator with alpha = 0 is singular (rigid motions)");
    P->mean_zero = P->C == 1 && all_neumann && P->alpha == 0.0;
    P->sstream = static_cast<hipStream_t>(stream);
    P->b = b;
    P->x = x;
    P->opts = o;
    P->restarts = 0;
    std::memset(&P->info, 0, sizeof(P->info));
    hipStream_t s = P->sstream;
    const long long n = P->ndof;
    sk_state_init(P->st, o.rel_tol * o.rel_tol, o.max_iter, s);
    vrc = prepare_precond(P, s);
    if (vrc != SIPG_OK) return vrc;
    if (P->mean_zero) {
        sk_sum(b, n, P->partials, nullptr, s);
        sk_scalar(P->st, P->partials, 1, SC_MEAN, n, s);
    }
    sk_pcg_start(b, P->r, x, n, P->mean_zero ? 1 : 0, P->st, P->partials, s);
    sipg_status rc = cg_start_from_residual(P);
    if (rc != SIPG_OK) return rc;
    P->phase = PH_RUNNING;
    return enqueue_readback(P);
}

sipg_status sipg_solve_advance(sipg_plan* P, int32_t iters) {
    if (!valid_plan(P)) return fail(SIPG_ERR_INVALID, "null plan");
    if (P->phase == PH_IDLE) return fail(SIPG_ERR_STATE, "no solve in progress");
    if (P->phase != PH_RUNNING || iters <= 0) return SIPG_OK;  // checking, done: nothing to enqueue
    const sipg_status rc = cg_chunk(P, iters);
    if (rc != SIPG_OK) return rc;
    return enqueue_readback(P);
}

sipg_status sipg_solve_poll(sipg_plan* P, int32_t* done, sipg_solve_info* info) {
    if (!valid_plan(P) || !done) return fail(SIPG_ERR_INVALID, "null argument");
    *done = 0;
    if (P->phase == PH_IDLE) return fail(SIPG_ERR_STATE, "no solve in progress");
    if (P->phase == PH_DONE) {
        *done = 1;
        if (info) *info = P->info;
        return SIPG_OK;
    }
    const hipError_t q = hipEventQuery(P->ev);
    if (q == hipErrorNotReady) return SIPG_OK;
    if (q != hipSuccess) return fail(SIPG_ERR_HIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
    const SolveState& m = *P->mirror;
    if (P->phase == PH_RUNNING) {
        if (m.done == 0) return SIPG_OK;  // caller should advance further
        P->phase = PH_CHECKING;
        return enqueue_true_residual(P);
    }
    // PH_CHECKING: the true residual has arrived
    const double rel = m.bnorm2 == 0.0 ? 0.0 : std::sqrt(m.rr_true / m.bnorm2);  // NaN if b is not finite
    const bool ok = rel <= P->opts.rel_tol;
    if (ok || m.done == 2 || m.iter >= P->opts.max_iter || P->restarts >= P->opts.max_restarts) {
        P->phase = PH_DONE;
        P->info.iterations = m.iter;
        P->info.restarts = P->restarts;
        P->info.rel_residual = rel;
        P->info.lambda_max = m.lam_max;
        P->info.status = ok ? SIPG_OK : (m.done == 2 ? SIPG_ERR_BREAKDOWN : SIPG_ERR_NOT_CONVERGED);
        *done = 1;
        if (info) *info = P->info;
        return SIPG_OK;
    }
    // restart from x: r = b - A x is already in place
    P->restarts += 1;
    sk_state_resume(P->st, P->opts.max_iter, P->sstream);
    sipg_status rc = cg_start_from_residual(P);
    if (rc != SIPG_OK) return rc;
    P->phase = PH_RUNNING;
    return enqueue_readback(P);
}

sipg_status sipg_solve(sipg_plan* P, const double* b, double* x, const sipg_solve_opts* opts, sipg_solve_info* info,
                       void* stream) {
    sipg_status rc = sipg_solve_begin(P, b, x, opts, stream);
    if (rc != SIPG_OK) return rc;
    for (;;) {
        int32_t done = 0;
        if (P->phase == PH_RUNNING) {
            rc = sipg_solve_advance(P, P->opts.check_every);
            if (rc != SIPG_OK) return rc;
        }
        HIP_TRY(hipEventSynchronize(P->ev));
        rc = sipg_solve_poll(P, &done, info);
        if (rc != SIPG_OK) return rc;
        if (done) break;
    }
    return P->info.status == SIPG_OK ? SIPG_OK
                                     : fail((sipg_status)P->info.status, "solve did not reach the tolerance");
}


// ------------------------------------------------------------ Picard update

void sipg_picard_opts_default(sipg_picard_opts* o) {
    if (!o) return;
    o->rel_tol = 1e-8;
    o->abs_tol = 0.0;
    o->max_iter = 50;
    o->aitken = 1;
}

size_t sipg_picard_work_bytes(const sipg_plan* P) {
    if (!valid_plan(P)) return 0;
    return (size_t)(3 * picard_stride(P->ndof) + 3 * kPicardBlocks + 8) * sizeof(double);
}

sipg_status sipg_update_viscosity(sipg_plan* P, const double* u, void* stream) {
    if (!valid_plan(P) || !u) return fail(SIPG_ERR_INVALID, "null argument");
    if (!P->bound) return fail(SIPG_ERR_STATE, "plan not bound");
    if (P->op != SIPG_VISCOUS || P->law.kind != SIPG_LAW_CARREAU)
        return fail(SIPG_ERR_INVALID, "the viscosity update needs a viscous plan with the CARREAU law");
    if (P->phase == PH_RUNNING || P->phase == PH_CHECKING) return fail(SIPG_ERR_STATE, "a solve is in progress on this plan");
    return update_viscosity(P, u, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

// The Picard iteration on a work area of sipg_picard_work_bytes(P) bytes
// (three vectors and the reduction partials; nothing in it has to start at
// zero: every value is written before it is read).
sipg_status picard_run(sipg_plan* P, const double* b, double* x, void* work, const sipg_solve_opts* lin_opts,
                       const sipg_picard_opts* opts, sipg_picard_info* info, void* stream) {
    if (!valid_plan(P) || !b || !x || !work) return fail(SIPG_ERR_INVALID, "null argument");
    if (!P->bound || !P->with_solver) return fail(SIPG_ERR_STATE, "plan not bound with solver workspace");
    if (P->op != SIPG_VISCOUS || P->law.kind != SIPG_LAW_CARREAU)
        return fail(SIPG_ERR_INVALID, "the Picard iteration needs a viscous plan with the CARREAU law");
    if (P->phase == PH_RUNNING || P->phase == PH_CHECKING) return fail(SIPG_ERR_STATE, "a solve is in progress on this plan");
    if (reinterpret_cast<uintptr_t>(work) % 256 != 0) return fail(SIPG_ERR_INVALID, "work must be 256-byte aligned");
    if (static_cast<const void*>(b) == static_cast<void*>(x)) return fail(SIPG_ERR_INVALID, "b and x must not alias");
    sipg_picard_opts o;
    if (opts) o = *opts; else sipg_picard_opts_default(&o);
    if (!(o.rel_tol >= 0.0) || !(o.abs_tol >= 0.0) || !std::isfinite(o.rel_tol) || !std::isfinite(o.abs_tol) ||
        o.max_iter < 0)
        return fail(SIPG_ERR_INVALID, "Picard options: tolerances must be finite and >= 0, max_iter >= 0");
    sipg_solve_opts lo;
    if (lin_opts) lo = *lin_opts; else sipg_solve_opts_default(&lo);
    const sipg_status vrc = check_opts(P, lo);
    if (vrc != SIPG_OK) return vrc;

    hipStream_t s = static_cast<hipStream_t>(stream);
    const long long n = P->ndof, stride = picard_stride(n);
    double* R = static_cast<double*>(work);
    double* Rp = R + stride;
    double* dl = Rp + stride;
    double* partials = dl + stride;
    double* sums = partials + 3 * kPicardBlocks;
    const char* wb = static_cast<const char*>(work);
    const char* we = wb + sipg_picard_work_bytes(P);
    auto overlaps = [&](const void* v) {
        const char* a = static_cast<const char*>(v);
        return a + n * sizeof(double) > wb && a < we;
    };
    if (overlaps(b) || overlaps(x)) return fail(SIPG_ERR_INVALID, "work must not alias b or x");

    sipg_picard_info inf;
    std::memset(&inf, 0, sizeof(inf));
    double h[3] = {0.0, 0.0, 0.0};
    // R <- b - A(nu(x)) x with the viscosity updated from x; h <- sums with Rp
    auto residual = [&](const double* prev) -> sipg_status {
        sipg_status rc = update_viscosity(P, x, s);
        if (rc != SIPG_OK) return rc;
        ApplyIO<double> io;
        std::memset(&io, 0, sizeof(io));
        io.x = x; io.y = R; io.parts = SIPG_PART_ALL; io.r = b;
        HIP_TRY(launch_apply<double>(P->n, P->C, P->curved, P->opdata<double>(), io, MODE_RESID, s));
        HIP_TRY(launch_picard_sums(R, prev, n, partials, sums, s));
        HIP_TRY(hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return SIPG_OK;
    };
    sipg_status rc = residual(nullptr);
    if (rc != SIPG_OK) return rc;
    const double r0 = std::sqrt(h[0]);
    double rn = r0, omega = 1.0;
    inf.residual_initial = r0;
    inf.residual_norms[0] = r0;
    inf.recorded = 1;
    inf.status = SIPG_ERR_NOT_CONVERGED;
    for (int k = 0;; ++k) {
        if (!std::isfinite(rn)) { inf.status = SIPG_ERR_BREAKDOWN; break; }
        if (rn <= o.rel_tol * r0 || rn <= o.abs_tol) { inf.status = SIPG_OK; break; }
        if (k >= o.max_iter) break;
        if (o.aitken && k > 0 && h[2] > 0.0) omega = -omega * h[1] / h[2];
        sipg_solve_info li;
        rc = sipg_solve(P, R, dl, &lo, &li, stream);
        inf.linear_iterations += li.iterations;
        if (rc != SIPG_OK) { inf.status = rc; break; }
        HIP_TRY(launch_axpy(x, dl, omega, n, s));
        std::swap(R, Rp);
        rc = residual(Rp);
        if (rc != SIPG_OK) return rc;
        rn = std::sqrt(h[0]);
        inf.iterations = k + 1;
        if (k < SIPG_PICARD_HISTORY) inf.omegas[k] = omega;
        if (k + 1 < SIPG_PICARD_HISTORY) {
            inf.residual_norms[k + 1] = rn;
            inf.recorded = k + 2;
        }
    }
    inf.residual_final = rn;
    if (info) *info = inf;
    if (inf.status == SIPG_OK) {
        g_err.clear();
        return SIPG_OK;
    }
    return fail((sipg_status)inf.status, inf.status == SIPG_ERR_NOT_CONVERGED
                                             ? "Picard iteration did not reach the tolerance"
                                             : "Picard iteration stopped: linear solve failed or residual not finite");
}

}  // namespace

// Work area of sipg_picard_solve_noalloc: a static device array, one copy per
// GPU, held until the process ends.  Host code must not use its name as an
// address (that is a host-side stand-in); the device address comes from
// hipGetSymbolAddress, once per device, and is kept in g_scratch_ptr.
constexpr size_t kScratchBytes = (3 * (size_t)SIPG_PICARD_NOALLOC_MAX_DOF + 3 * kPicardBlocks + 8) * sizeof(double);
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
sipg_status scratch_address(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SIPG_ERR_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SIPG_ERR_HIP, "hipGetSymbolAddress returned a null address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SIPG_OK;
}

}  // namespace

extern "C" {

sipg_status sipg_picard_solve(sipg_plan* P, const double* b, double* x, void* work, const sipg_solve_opts* lin_opts,
                              const sipg_picard_opts* opts, sipg_picard_info* info, void* stream) {
    return picard_run(P, b, x, work, lin_opts, opts, info, stream);
}

sipg_status sipg_picard_solve_noalloc(sipg_plan* P, const double* b, double* x, const sipg_solve_opts* lin_opts,
                                      const sipg_picard_opts* opts, sipg_picard_info* info, void* stream) {
    if (!valid_plan(P) || !b || !x) return fail(SIPG_ERR_INVALID, "null argument");
    if (P->ndof > SIPG_PICARD_NOALLOC_MAX_DOF || sipg_picard_work_bytes(P) > kScratchBytes)
        return fail(SIPG_ERR_INVALID, "sipg_picard_solve_noalloc: the plan has " + std::to_string(P->ndof) +
                                          " unknowns, more than the static work area holds (" +
                                          std::to_string((long long)SIPG_PICARD_NOALLOC_MAX_DOF) + ")");
    if (lin_opts && lin_opts->use_graph)
        return fail(SIPG_ERR_INVALID, "sipg_picard_solve_noalloc: use_graph would instantiate graphs (allocation)");
    void* work = nullptr;
    const sipg_status rc = scratch_address(&work);
    if (rc != SIPG_OK) return rc;
    P->no_alloc = true;   // no stream or event creation on this path
    const sipg_status r = picard_run(P, b, x, work, lin_opts, opts, info, stream);
    P->no_alloc = false;
    return r;
}

// ------------------------------------------------------------ dual splitting step

}  // extern "C"

namespace {

bool same_mesh(const sipg_plan* A, const sipg_plan* B) {
    return A->nx == B->nx && A->ny == B->ny && A->nz == B->nz && A->curved == B->curved && A->verts == B->verts;
}

bool all_bc(const sipg_plan* P, int v) {
    return std::all_of(P->bc, P->bc + 6, [v](int b) { return b == v; });
}

bool busy(const sipg_plan* P) { return P->phase == PH_RUNNING || P->phase == PH_CHECKING; }

// velocity plan: viscous or penalty, degree 2..5, no-slip walls, bound
sipg_status check_velocity(const sipg_plan* V) {
    if (!valid_plan(V)) return fail(SIPG_ERR_INVALID, "null plan");
    if (V->C != 3) return fail(SIPG_ERR_INVALID, "the velocity plan needs 3 components");
    if (V->degree < 2 || V->degree > 5) return fail(SIPG_ERR_INVALID, "the splitting step needs velocity degree 2..5");
    if (!all_bc(V, SIPG_BC_DIRICHLET)) return fail(SIPG_ERR_INVALID, "the splitting step needs no-slip walls (all Dirichlet)");
    if (!V->bound) return fail(SIPG_ERR_STATE, "plan not bound");
    return SIPG_OK;
}

sipg_status check_pressure(const sipg_plan* V, const sipg_plan* Pp) {
    if (!valid_plan(Pp)) return fail(SIPG_ERR_INVALID, "null plan");
    if (Pp->op != SIPG_POISSON || Pp->degree != V->degree - 1 || !all_bc(Pp, SIPG_BC_NEUMANN) || Pp->alpha != 0.0)
        return fail(SIPG_ERR_INVALID, "the pressure plan must be Poisson of degree k-1, all Neumann, alpha = 0");
    if (!same_mesh(V, Pp)) return fail(SIPG_ERR_INVALID, "velocity and pressure plans are on different meshes");
    if (!Pp->bound) return fail(SIPG_ERR_STATE, "plan not bound");
    return SIPG_OK;
}

void fill_split_geo(const sipg_plan* V, SplitGeo& S, int order = 1) {
    std::memset(&S, 0, sizeof(S));
    S.order = order;
    if (order == 2) {
        S.gamma0 = 1.5; S.alpha[0] = 2.0; S.alpha[1] = -0.5; S.beta[0] = 2.0; S.beta[1] = -1.0; S.beta_bar = 1.0;
    } else {
        S.gamma0 = 1.0; S.alpha[0] = 1.0; S.beta[0] = 1.0; S.beta_bar = 0.0;
    }
    S.eta[0] = V->law.mu0; S.eta[1] = V->law.mu_inf; S.eta[2] = V->law.lam;
    S.eta[3] = V->law.n_exp; S.eta[4] = V->law.kappa; S.eta[5] = V->law.a_exp;
    S.nx = V->nx; S.ny = V->ny; S.nz = V->nz;
    S.verts = V->curved ? V->verts64_d : nullptr;
    S.h[0] = 1.0 / V->nx; S.h[1] = 1.0 / V->ny; S.h[2] = 1.0 / V->nz;
    S.hinv[0] = V->nx; S.hinv[1] = V->ny; S.hinv[2] = V->nz;
    S.tab = V->tab64;
    const int n = V->n, np = n - 1;
    double xp[kMaxN], wp[kMaxN];
    gauss_legendre01(np, xp, wp);
    // Lagrange basis on the np pressure points and its derivative (product rule) at t
    auto basis = [&](double t, int j, double& val, double& der) {
        val = 1.0;
        der = 0.0;
        for (int m = 0; m < np; ++m) {
            if (m == j) continue;
            der = der * (t - xp[m]) / (xp[j] - xp[m]) + val / (xp[j] - xp[m]);
            val *= (t - xp[m]) / (xp[j] - xp[m]);
        }
    };
    for (int q = 0; q < n; ++q)
        for (int j = 0; j < np; ++j) basis(V->tab64.x[q], j, S.PV[q][j], S.PD[q][j]);
    for (int s = 0; s < 2; ++s)
        for (int j = 0; j < np; ++j) {
            double d;
            basis((double)s, j, S.PS[s][j], d);
        }
}

size_t split_vec_bytes(long long n) { return align256((size_t)n * sizeof(double)); }

long long wall_faces(const sipg_plan* V) {
    return 2LL * ((long long)V->ny * V->nz + (long long)V->nx * V->nz + (long long)V->nx * V->ny);
}

}  // namespace

extern "C" {

sipg_status sipg_convective_step(sipg_plan* V, const double* u, const double* u_prev, const double* b,
                                 const double* g_wall, double dt, double* uhat, void* stream) {
    sipg_status rc = check_velocity(V);
    if (rc != SIPG_OK) return rc;
    if (!u || !uhat) return fail(SIPG_ERR_INVALID, "null argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SIPG_ERR_INVALID, "dt must be finite and > 0");
    if (static_cast<const void*>(u) == static_cast<void*>(uhat) || static_cast<const void*>(b) == static_cast<void*>(uhat) ||
        static_cast<const void*>(u_prev) == static_cast<void*>(uhat))
        return fail(SIPG_ERR_INVALID, "uhat must not alias u, u_prev or b (neighbours' values are read)");
    SplitGeo S;
    fill_split_geo(V, S, u_prev ? 2 : 1);
    S.gw = g_wall;
    HIP_TRY(launch_split_convective(V->n, S, u, u_prev, b, dt, uhat, static_cast<hipStream_t>(stream)));
    return SIPG_OK;
}

sipg_status sipg_pressure_rhs(sipg_plan* V, sipg_plan* Pp, const double* uhat, const double* u_old,
                              const double* u_prev, const double* b, const double* g_wall, double dt, double* f,
                              void* stream) {
    sipg_status rc = check_velocity(V);
    if (rc == SIPG_OK) rc = check_pressure(V, Pp);
    if (rc != SIPG_OK) return rc;
    if (!uhat || !u_old || !f) return fail(SIPG_ERR_INVALID, "null argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SIPG_ERR_INVALID, "dt must be finite and > 0");
    if (u_prev && (V->law.kind != SIPG_LAW_CARREAU || V->op != SIPG_VISCOUS))
        return fail(SIPG_ERR_INVALID, "the BDF2 pressure wall data need the velocity plan's CARREAU law");
    SplitGeo S;
    fill_split_geo(V, S, u_prev ? 2 : 1);
    S.gw = g_wall;
    HIP_TRY(launch_split_ppe_rhs(V->n, S, uhat, u_old, u_prev, b, dt, f, static_cast<hipStream_t>(stream)));
    return SIPG_OK;
}

sipg_status sipg_projection(sipg_plan* V, sipg_plan* Pp, const double* uhat, const double* p, int32_t order, double dt,
                            double* uhh, double* rhs_visc, void* stream) {
    sipg_status rc = check_velocity(V);
    if (rc == SIPG_OK) rc = check_pressure(V, Pp);
    if (rc != SIPG_OK) return rc;
    if (!uhat || !p || !uhh) return fail(SIPG_ERR_INVALID, "null argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SIPG_ERR_INVALID, "dt must be finite and > 0");
    if (static_cast<const void*>(p) == static_cast<void*>(uhh) || (rhs_visc && static_cast<const void*>(p) == rhs_visc) ||
        (rhs_visc && static_cast<const void*>(uhat) == rhs_visc) || rhs_visc == uhh)
        return fail(SIPG_ERR_INVALID, "outputs must not alias p, each other, or (rhs_visc) uhat");
    if (order != 1 && order != 2) return fail(SIPG_ERR_INVALID, "BDF order 1 or 2");
    SplitGeo S;
    fill_split_geo(V, S, order);
    HIP_TRY(launch_split_projection(V->n, S, uhat, p, dt, uhh, rhs_visc, static_cast<hipStream_t>(stream)));
    return SIPG_OK;
}

sipg_status sipg_update_penalty_factors(sipg_plan* P, const double* u, double dt, double zeta, void* stream) {
    sipg_status rc = check_velocity(P);
    if (rc != SIPG_OK) return rc;
    if (!P->pen) return fail(SIPG_ERR_INVALID, "not a penalty-step plan");
    if (!u) return fail(SIPG_ERR_INVALID, "null argument");
    if (busy(P)) return fail(SIPG_ERR_STATE, "a solve is in progress on this plan");
    if (!(dt > 0.0) || !std::isfinite(dt) || !(zeta >= 0.0) || !std::isfinite(zeta))
        return fail(SIPG_ERR_INVALID, "dt must be finite and > 0, zeta finite and >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    SplitGeo S;
    fill_split_geo(P, S);
    HIP_TRY(launch_pen_factors(P->n, S, u, dt, zeta, P->hcell, P->tau_div_d, P->tau_cont_d, s));
    const OpData<double> od = P->opdata<double>();
    HIP_TRY(launch_setup(P->n, P->C, P->curved, od, P->law, P->penalty, P->hcell, P->tfac64, P->tfac32, P->mu_cell64,
                         P->mu_cell32, P->mu_face64, P->mu_face32, (int)P->nface, P->tau_div_d, P->tau_cont_d, s));
    HIP_TRY(launch_diagonal(P->n, P->C, P->curved, P->opdata<double>(), P->diag64, P->dinv64, P->dinv32, s));
    P->lz_stale = true;
    // multigrid levels: a degree step keeps the finer level's factors, a mesh
    // step averages each coarse cell's 8 children (as the hierarchy is built)
    const double* td = P->tau_div_d;
    const double* tc = P->tau_cont_d;
    int fx = P->nx, fy = P->ny, fz = P->nz;
    for (sipg_plan* L : P->mg) {
        if (!L->bound) break;                  // levels are bound only with solver workspace
        if (L->mesh_step) {
            HIP_TRY(launch_pen_coarsen(fx, fy, fz, td, tc, L->tau_div_d, L->tau_cont_d, s));
        } else {
            HIP_TRY(hipMemcpyAsync(L->tau_div_d, td, L->ncell * 8, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(L->tau_cont_d, tc, L->ncell * 8, hipMemcpyDeviceToDevice, s));
        }
        HIP_TRY(launch_setup(L->n, L->C, L->curved, L->opdata<double>(), L->law, L->penalty, L->hcell, L->tfac64,
                             L->tfac32, L->mu_cell64, L->mu_cell32, L->mu_face64, L->mu_face32, (int)L->nface,
                             L->tau_div_d, L->tau_cont_d, s));
        HIP_TRY(launch_diagonal(L->n, L->C, L->curved, L->opdata<double>(), L->diag64, L->dinv64, L->dinv32, s));
        L->lz_stale = true;
        td = L->tau_div_d;
        tc = L->tau_cont_d;
        fx = L->nx; fy = L->ny; fz = L->nz;
    }
    if (!P->cg.empty() && P->with_solver) return refresh_continuous(P, s);
    return SIPG_OK;
}

sipg_status sipg_wall_load(sipg_plan* P, const double* g_wall, double* y, void* stream) {
    sipg_status rc = check_velocity(P);
    if (rc != SIPG_OK) return rc;
    if (!g_wall || !y) return fail(SIPG_ERR_INVALID, "null argument");
    if (P->op != SIPG_VISCOUS && !P->pen) return fail(SIPG_ERR_INVALID, "wall load: viscous or penalty-step plan");
    SplitGeo S;
    fill_split_geo(P, S);
    S.gw = g_wall;
    HIP_TRY(launch_wall_load(P->n, S, P->mu_face64, P->tfac64, P->pen ? 1 : 0, y, static_cast<hipStream_t>(stream)));
    return SIPG_OK;
}

}  // extern "C"

namespace {

// Solve A x = b starting from x0: R = b - A x0 (operator kernel, residual
// mode), then A d = R to the relative tolerance that makes |b - A x| <=
// rel_tol |b|, and x = x0 + d (x must not alias x0; R: a scratch vector;
// sums: 3 kPicardBlocks + 8 doubles).  info->rel_residual is relative to |b|.
sipg_status warm_solve(sipg_plan* P, const double* b, const double* x0, double* x, double* R, double* sums,
                       const sipg_solve_opts& o, sipg_solve_info* info, hipStream_t s) {
    const long long n = P->ndof;
    double* partials = sums;
    double* out = sums + 3 * kPicardBlocks;
    ApplyIO<double> io;
    std::memset(&io, 0, sizeof(io));
    io.x = x0; io.y = R; io.parts = SIPG_PART_ALL; io.r = b;
    HIP_TRY(launch_apply<double>(P->n, P->C, P->curved, P->opdata<double>(), io, MODE_RESID, s));
    double h[2];
    HIP_TRY(launch_picard_sums(b, nullptr, n, partials, out, s));
    HIP_TRY(hipMemcpyAsync(&h[0], out, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(launch_picard_sums(R, nullptr, n, partials, out, s));
    HIP_TRY(hipMemcpyAsync(&h[1], out, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double bn = std::sqrt(h[0]), rn = std::sqrt(h[1]);
    sipg_solve_opts od = o;
    if (rn > 0.0) od.rel_tol = std::min(1.0, o.rel_tol * bn / rn);
    sipg_solve_info inf;
    std::memset(&inf, 0, sizeof(inf));
    sipg_status rc = SIPG_OK;
    if (!(rn > o.rel_tol * bn)) {             // x0 already solves to the tolerance
        HIP_TRY(hipMemcpyAsync(x, x0, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        inf.status = SIPG_OK;
        inf.rel_residual = bn > 0.0 ? rn / bn : 0.0;
    } else {
        rc = sipg_solve(P, R, x, &od, &inf, s);
        HIP_TRY(launch_axpy(x, x0, 1.0, n, s));
        inf.rel_residual = bn > 0.0 ? inf.rel_residual * rn / bn : 0.0;
    }
    if (info) *info = inf;
    return rc;
}

}  // namespace

extern "C" {

void sipg_split_opts_default(sipg_split_opts* o) {
    if (!o) return;
    sipg_solve_opts_default(&o->pressure);
    sipg_solve_opts_default(&o->viscous);
    sipg_solve_opts_default(&o->penalty);
    // the step's smoothers take 10-step Lanczos estimates (the same solver
    // iteration counts as 20 steps on the lid-driven box, half the cost)
    o->pressure.lanczos_steps = o->viscous.lanczos_steps = o->penalty.lanczos_steps = 10;
    o->zeta = 1.0;
    o->warm_start = 0;
}

size_t sipg_split_work_bytes(const sipg_plan* V, const sipg_plan* Pp) {
    if (!valid_plan(V) || !valid_plan(Pp)) return 0;
    return 5 * split_vec_bytes(V->ndof) + split_vec_bytes(Pp->ndof) +
           align256((3 * kPicardBlocks + 8) * sizeof(double));
}

sipg_status sipg_split_step(sipg_plan* V, sipg_plan* Pp, sipg_plan* Pen, const double* u_old, const double* u_prev,
                            const double* b, const double* g_wall, double dt, double* u_new, double* p, void* work,
                            const sipg_split_opts* opts, sipg_split_info* info, void* stream) {
    sipg_status rc = check_velocity(V);
    if (rc == SIPG_OK) rc = check_pressure(V, Pp);
    if (rc == SIPG_OK) rc = check_velocity(Pen);
    if (rc != SIPG_OK) return rc;
    if (V->op != SIPG_VISCOUS || V->law.kind != SIPG_LAW_CARREAU)
        return fail(SIPG_ERR_INVALID, "the velocity plan must be viscous with the CARREAU law");
    if (!Pen->pen || Pen->degree != V->degree || Pen->alpha != 1.0 || !same_mesh(V, Pen))
        return fail(SIPG_ERR_INVALID, "the penalty plan must be a penalty step of the same degree and mesh, alpha = 1");
    if (!V->with_solver || !Pp->with_solver || !Pen->with_solver)
        return fail(SIPG_ERR_STATE, "plans must be bound with solver workspace");
    if (busy(V) || busy(Pp) || busy(Pen)) return fail(SIPG_ERR_STATE, "a solve is in progress on one of the plans");
    if (!u_old || !u_new || !p || !work) return fail(SIPG_ERR_INVALID, "null argument");
    if (reinterpret_cast<uintptr_t>(work) % 256 != 0) return fail(SIPG_ERR_INVALID, "work must be 256-byte aligned");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SIPG_ERR_INVALID, "dt must be finite and > 0");
    const int order = u_prev ? 2 : 1;
    const double gamma0 = order == 2 ? 1.5 : 1.0;
    if (std::fabs(V->alpha * dt - gamma0) > 1e-12 * gamma0)
        return fail(SIPG_ERR_INVALID, "the velocity plan's alpha must be gamma_0/dt (BDF1: 1/dt, BDF2: 1.5/dt)");
    if (static_cast<const void*>(u_old) == static_cast<void*>(u_new) ||
        static_cast<const void*>(u_prev) == static_cast<void*>(u_new))
        return fail(SIPG_ERR_INVALID, "u_new must not alias u_old or u_prev");
    sipg_split_opts o;
    if (opts) o = *opts; else sipg_split_opts_default(&o);
    if (!(o.zeta >= 0.0) || !std::isfinite(o.zeta)) return fail(SIPG_ERR_INVALID, "zeta must be finite and >= 0");
    const long long nu = V->ndof;
    char* w = static_cast<char*>(work);
    const size_t vb = split_vec_bytes(nu);
    double* uhat = reinterpret_cast<double*>(w);
    double* uhh = reinterpret_cast<double*>(w + vb);
    double* rhs = reinterpret_cast<double*>(w + 2 * vb);
    double* uvisc = reinterpret_cast<double*>(w + 3 * vb);
    double* uex = reinterpret_cast<double*>(w + 4 * vb);
    double* f = reinterpret_cast<double*>(w + 5 * vb);
    double* sums = reinterpret_cast<double*>(w + 5 * vb + split_vec_bytes(Pp->ndof));
    const char* we = w + sipg_split_work_bytes(V, Pp);
    auto overlaps = [&](const void* v, size_t bytes) {
        const char* a = static_cast<const char*>(v);
        return v && a + bytes > w && a < we;
    };
    const size_t gw_bytes = (size_t)wall_faces(V) * V->n * V->n * 3 * 8;
    if (overlaps(u_old, nu * 8) || overlaps(u_prev, nu * 8) || overlaps(b, nu * 8) || overlaps(u_new, nu * 8) ||
        overlaps(p, Pp->ndof * 8) || overlaps(g_wall, gw_bytes))
        return fail(SIPG_ERR_INVALID, "work must not alias the step's vectors");

    sipg_split_info inf;
    std::memset(&inf, 0, sizeof(inf));
    auto finish = [&](sipg_status r) {
        if (info) *info = inf;
        return r;
    };
    // u^# = sum_i beta_i u^{n-i}: the viscosity and the penalty factors of the step
    const double* ux = u_old;
    if (order == 2) {
        HIP_TRY(launch_lincomb(nu, 2.0, u_old, -1.0, u_prev, uex, static_cast<hipStream_t>(stream)));
        ux = uex;
    }
    rc = sipg_convective_step(V, u_old, u_prev, b, g_wall, dt, uhat, stream);
    if (rc == SIPG_OK) rc = sipg_pressure_rhs(V, Pp, uhat, u_old, u_prev, b, g_wall, dt, f, stream);
    if (rc == SIPG_OK) rc = sipg_solve(Pp, f, p, &o.pressure, &inf.pressure, stream);
    if (rc == SIPG_OK) rc = sipg_projection(V, Pp, uhat, p, order, dt, uhh, rhs, stream);
    if (rc == SIPG_OK) rc = update_viscosity(V, ux, static_cast<hipStream_t>(stream));
    if (rc == SIPG_OK && g_wall) rc = sipg_wall_load(V, g_wall, rhs, stream);
    if (rc == SIPG_OK) {
        rc = o.warm_start ? warm_solve(V, rhs, uhh, uvisc, uhat, sums, o.viscous, &inf.viscous,
                                       static_cast<hipStream_t>(stream))
                          : sipg_solve(V, rhs, uvisc, &o.viscous, &inf.viscous, stream);
    }
    if (rc == SIPG_OK) rc = sipg_update_penalty_factors(Pen, ux, dt, o.zeta, stream);
    if (rc == SIPG_OK) {
        SplitGeo S;
        fill_split_geo(V, S);
        const hipError_t e = launch_split_mass(V->n, S, uvisc, 1.0, rhs, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) rc = fail(SIPG_ERR_HIP, std::string("split mass: ") + hipGetErrorString(e));
    }
    if (rc == SIPG_OK && g_wall) rc = sipg_wall_load(Pen, g_wall, rhs, stream);
    if (rc == SIPG_OK) {
        rc = o.warm_start ? warm_solve(Pen, rhs, uvisc, u_new, uhat, sums, o.penalty, &inf.penalty,
                                       static_cast<hipStream_t>(stream))
                          : sipg_solve(Pen, rhs, u_new, &o.penalty, &inf.penalty, stream);
    }
    if (rc == SIPG_OK) g_err.clear();
    return finish(rc);
}

}  // extern "C"
