// Krylov solve of A u = b (Sec. 2.3, eq. matrix_eqn).
//
// Restarted flexible GMRES in FP64 (the paper's GMRES; flexible so that the
// preconditioner may vary, e.g. run in FP32), or flexible CG.  The true
// residual b - A u is recomputed at restarts, every 50 CG iterations and at
// convergence, in FP64 or, on request, in double-double arithmetic
// (residual.hip): iterative refinement in two or three precisions.
//
// Preconditioner: a multigrid V-cycle (Sec. 2.3) on a hierarchy that first
// lowers the polynomial degree (p -> p/2 -> ... -> 1) on the same mesh, then
// merges 2 x 2 columns; every level re-discretises the DG operator of
// Sec. 2.2 on its own mesh.  On each level the smoother is additive Schwarz
// with one subdomain per element (no overlap), damped; the subdomain solve is
// the fast-diagonalisation inverse of a separable approximation of the
// element-diagonal block: for displacement component c and reference
// direction d the 1D element operator of the same DG scheme (volume term,
// lift and interior-penalty faces, neighbours set to zero) with modulus
// kappa_cd = c11 n_c^2 + c44 (1 - n_c^2) along the direction n of that axis.
// The coarsest level is solved with an explicit dense inverse.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <exception>
#include <cmath>
#include <limits>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "context.h"
#include "mg.h"

namespace dgtn {

constexpr int kMaxDenseCoarse = 16384;

struct Transfer {
    int type = 0;  // 0: degree, 1: columns (2 x 2 children), 2: z-element pairs
    std::vector<double> I;
    std::vector<int> parent, child, children;
    std::vector<int> zpar, zch;  // type 2: coarse z of each fine z; fine z pair of each coarse z
    size_t off_I[2] = {0, 0}, off_parent = 0, off_child = 0, off_children = 0, off_zpar = 0, off_zch = 0;
};

struct MgLevel {
    std::vector<double> fdm;  // [E][3 comps][3 dirs][N*N (S, row = node) + N (kappa * lambda)]
    size_t off_fdm[2] = {0, 0};
    size_t off_b[2] = {0, 0}, off_x[2] = {0, 0}, off_t[2] = {0, 0};
    // column smoother: S [n_cols][2][P2], lam [n_cols][2][P], rat [n_cols][6], V [3][n][n], lz [3][n];
    // P = N, or N + 2k for overlapping patches with gather / sum tables pg, ps
    int P = 0;
    std::vector<double> cS, clam, crat, cV, clz;
    std::vector<int> pg, ps;
    std::vector<double> cw;   // [n_cols][N2] count^(-1/2) of the patches holding each node
    size_t off_cS[2] = {0, 0}, off_clam[2] = {0, 0}, off_crat[2] = {0, 0}, off_cV[2] = {0, 0}, off_clz[2] = {0, 0};
    size_t off_cT[2] = {0, 0}, off_cY[2] = {0, 0}, off_pg = 0, off_ps = 0, off_cw[2] = {0, 0};
};

struct SolverState {
    int key_levels = -1;
    std::vector<MgLevel> mg;
    std::vector<Transfer> tr;
    bool dense = false;
    int n_coarse = 0;
    size_t off_Ainv[2] = {0, 0}, off_col = 0;
    int m = 0, nblk = 0;
    size_t off_V = 0, off_Z = 0, off_w = 0, off_r = 0, off_partial = 0, off_dots = 0, off_coef = 0, off_sc = 0;
    bool planned = false;
    // pinned host slots and events for reading solver monitors without stalling the stream
    double* host_mon = nullptr;
    hipEvent_t mon_event[2] = {nullptr, nullptr};
    dgtn_status host_monitor();
    // V-cycles recorded once as HIP graphs (per precision and smoother setting) on a
    // private stream and replayed on the caller's stream: one launch instead of one
    // per kernel.  They hold workspace addresses, so binding drops them.
    struct VGraph {
        int prec, nu, smoother;
        double omega;
        hipGraphExec_t exec;
    };
    std::vector<VGraph> vgraphs;
    hipStream_t cap_stream = nullptr;
    bool graphs_off = std::getenv("DGTN_NO_GRAPHS") != nullptr;  // eager V-cycles (for comparison)
    void drop_graphs();
    ~SolverState();
};

namespace {

size_t ndof(const Level& L) { return (size_t)3 * L.E * L.N * L.N * L.N; }

// ---- fast-diagonalisation data ---------------------------------------------

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix A (destroyed):
// A = Q diag(lam) Q^T, Q[i*n + a] = component i of eigenvector a.
void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& Q, std::vector<double>& lam) {
    Q.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0, tot = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) {  // A <- A J
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = cs * akp - sn * akq;
                    A[k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = cs * apk - sn * aqk;
                    A[q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double qkp = Q[k * n + p], qkq = Q[k * n + q];
                    Q[k * n + p] = cs * qkp - sn * qkq;
                    Q[k * n + q] = sn * qkp + cs * qkq;
                }
            }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
}

enum EndType { END_NONE = 0, END_INTERIOR = 1, END_DIRICHLET = 2 };

// 1D element operator of the DG scheme for a unit modulus on an element of
// width h: K = D^T W (D u + lift) - face fluxes, neighbours zero.
std::vector<double> element_1d(const Lgl& g, double h, int lo, double sig_lo, int hi, double sig_hi) {
    const int N = g.N;
    std::vector<double> K(N * N, 0.0), u(N), gr(N), S(N), r(N);
    for (int col = 0; col < N; ++col) {
        std::fill(u.begin(), u.end(), 0.0);
        u[col] = 1.0;
        for (int i = 0; i < N; ++i) {
            double acc = 0;
            for (int a = 0; a < N; ++a) acc += g.D[i * N + a] * u[a];
            gr[i] = 2.0 / h * acc;
            S[i] = gr[i];
        }
        const double jlo = lo == END_INTERIOR ? u[0] : lo == END_DIRICHLET ? 2.0 * u[0] : 0.0;
        const double jhi = hi == END_INTERIOR ? u[N - 1] : hi == END_DIRICHLET ? 2.0 * u[N - 1] : 0.0;
        S[0] += jlo / (g.w[0] * h);
        S[N - 1] -= jhi / (g.w[N - 1] * h);
        for (int a = 0; a < N; ++a) {
            double acc = 0;
            for (int i = 0; i < N; ++i) acc += g.D[i * N + a] * g.w[i] * S[i];
            r[a] = acc;
        }
        if (lo == END_INTERIOR) r[0] += 0.5 * gr[0] + sig_lo * jlo;
        if (lo == END_DIRICHLET) r[0] += gr[0] + sig_lo * jlo;
        if (hi == END_INTERIOR) r[N - 1] -= 0.5 * gr[N - 1] - sig_hi * jhi;
        if (hi == END_DIRICHLET) r[N - 1] -= gr[N - 1] - sig_hi * jhi;
        for (int i = 0; i < N; ++i) K[i * N + col] = r[i];
    }
    for (int i = 0; i < N; ++i)
        for (int j = i + 1; j < N; ++j) {
            const double s = 0.5 * (K[i * N + j] + K[j * N + i]);
            K[i * N + j] = K[j * N + i] = s;
        }
    return K;
}

// S (row = node, column = eigenvector, S^T M S = I) and lambda of K S = M S diag(lambda).
void fdm_1d(const Lgl& g, double h, const std::vector<double>& K, double* S_out, double* lam_out, double kappa) {
    const int N = g.N;
    std::vector<double> A(N * N), Q, lam;
    std::vector<double> ms(N);
    for (int i = 0; i < N; ++i) ms[i] = 1.0 / std::sqrt(g.w[i] * 0.5 * h);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) A[i * N + j] = ms[i] * K[i * N + j] * ms[j];
    jacobi_eigen(N, A, Q, lam);
    double lmax = 0;
    for (double l : lam) lmax = std::max(lmax, l);
    for (int a = 0; a < N; ++a) {
        lam_out[a] = kappa * std::max(lam[a], 1e-14 * lmax);
        for (int i = 0; i < N; ++i) S_out[i * N + a] = ms[i] * Q[i * N + a];
    }
}

int end_type(int bc) { return bc == DGTN_BC_DIRICHLET ? END_DIRICHLET : END_NONE; }

void build_fdm(const dgtn_ctx* c, const Level& L, std::vector<double>& out) {
    const int N = L.N, N2 = N * N, PER = N2 + N;
    out.assign((size_t)L.E * 9 * PER, 0.0);
    const double yr = c->y_ref;
    const double cn2 = L.pen_z;
    const std::vector<double>& mc = level_mat(c, L);
    auto consts = [&](int m, double& c11, double& c12, double& c44) {
        c11 = mc[3 * m] / yr;
        c12 = mc[3 * m + 1] / yr;
        c44 = mc[3 * m + 2] / yr;
    };
    std::map<std::array<double, 6>, std::vector<double>> solved;
    for (int col = 0; col < L.n_cols; ++col) {
        const double* gg = &L.geo2[(size_t)col * 5 * N2];
        // mean widths and axis directions of the column in the xy-plane
        double hd[2], dir[2][2];
        for (int d = 0; d < 2; ++d) {
            double sw = 0, sx = 0, sy = 0;
            for (int q = 0; q < N2; ++q) {
                const double ax = gg[(2 * d) * N2 + q], ay = gg[(2 * d + 1) * N2 + q];
                const double am = std::hypot(ax, ay);
                sw += 2.0 / am;
                sx += ax / am;
                sy += ay / am;
            }
            hd[d] = sw / N2;
            const double nm = std::hypot(sx, sy);
            dir[d][0] = sx / nm;
            dir[d][1] = sy / nm;
        }
        double sig_side[4];
        int end_side[4];
        for (int f = 0; f < 4; ++f) {
            double s = 0;
            for (int t = 0; t < N; ++t) s += L.sig_side[((size_t)col * 4 + f) * N + t];
            sig_side[f] = s / N;
            end_side[f] = L.cnbr[col * 4 + f] >= 0 ? END_INTERIOR : end_type(L.cnf[col * 4 + f]);
        }
        for (int iz = 0; iz < L.n_z; ++iz) {
            const int e = iz * L.n_cols + col;
            const int m = L.zmat[iz];
            double c11, c12, c44;
            consts(m, c11, c12, c44);
            (void)c12;
            double* fe = &out[(size_t)e * 9 * PER];
            for (int d = 0; d < 3; ++d) {
                double h, nvec[3] = {0, 0, 0};
                int lo, hi;
                double slo, shi;
                int mlo = -1, mhi = -1;
                if (d < 2) {
                    h = hd[d];
                    nvec[0] = dir[d][0];
                    nvec[1] = dir[d][1];
                    lo = end_side[2 * d];
                    hi = end_side[2 * d + 1];
                    slo = sig_side[2 * d];
                    shi = sig_side[2 * d + 1];
                } else {
                    h = L.hz[iz];
                    nvec[2] = 1.0;
                    if (iz == 0) { lo = end_type(c->prob.bc_top); slo = cn2 / h; }
                    else { lo = END_INTERIOR; slo = cn2 / std::min(h, L.hz[iz - 1]); mlo = L.zmat[iz - 1]; }
                    if (iz == L.n_z - 1) { hi = end_type(c->prob.bc_bottom); shi = cn2 / h; }
                    else { hi = END_INTERIOR; shi = cn2 / std::min(h, L.hz[iz + 1]); mhi = L.zmat[iz + 1]; }
                }
                for (int cc = 0; cc < 3; ++cc) {
                    auto kap = [&](int mm) {
                        double a11, a12, a44;
                        consts(mm, a11, a12, a44);
                        return a11 * nvec[cc] * nvec[cc] + a44 * (1.0 - nvec[cc] * nvec[cc]);
                    };
                    const double kappa = kap(m);
                    const double rlo = mlo >= 0 ? 0.5 * (kappa + kap(mlo)) / kappa : 1.0;
                    const double rhi = mhi >= 0 ? 0.5 * (kappa + kap(mhi)) / kappa : 1.0;
                    double* blk = fe + (cc * 3 + d) * PER;
                    // many elements share the same 1D problem (a column's widths, a layer's
                    // thickness and material): solve each distinct one once
                    const std::array<double, 6> key{h, (double)lo, slo * rlo, (double)hi, shi * rhi, kappa};
                    auto it = solved.find(key);
                    if (it == solved.end()) {
                        auto K = element_1d(L.lgl, h, lo, slo * rlo, hi, shi * rhi);
                        std::vector<double> res(PER);
                        fdm_1d(L.lgl, h, K, res.data(), res.data() + N2, kappa);
                        it = solved.emplace(key, std::move(res)).first;
                    }
                    std::copy(it->second.begin(), it->second.end(), blk);
                }
            }
        }
    }
}

// ---- column smoother -----------------------------------------------------------
//
// Subdomain = one whole z-column of elements (all layers under one 2D column),
// which holds the stiff z-coupling of thin layers exactly.  The column block of
// displacement component c is approximated by the separable operator
//   sum_e [kx(e) Kx (x) My (x) Mz(e) + ky(e) Mx (x) Ky (x) Mz(e)] + Mx (x) My (x) Kz_c,
// with Kx, Ky the unit-modulus 1D element operators of the column in xi and eta,
// Kz_c the 1D DG operator along the whole column (per-element modulus, averaged
// moduli and penalties on the interfaces, boundary conditions at both ends), and
// kx(e) = rx * c44(e), ky(e) = ry * c44(e).  Kx, Ky are diagonalised per
// column; Kz_c with respect to the c44-weighted z-mass once per component
// (every column has the same z-structure), so the inverse is
//   (Sx (x) Sy (x) V) diag(1 / (rx lx_a + ry ly_b + lz_i)) (Sx (x) Sy (x) V)^T.

// Symmetric eigen-decomposition A = Q diag(d) Q^T of a row-major n x n matrix:
// Householder reduction to tridiagonal form, then implicit-shift QL sweeps.
// Q[i * n + a] is component i of eigenvector a.
void sym_eigen(int n, std::vector<double> A, std::vector<double>& Q, std::vector<double>& d) {
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    std::vector<double> v(n), p(n), q(n);
    for (int k = 0; k + 2 < n; ++k) {
        double nrm = 0;
        for (int i = k + 1; i < n; ++i) nrm += A[(size_t)i * n + k] * A[(size_t)i * n + k];
        nrm = std::sqrt(nrm);
        if (nrm == 0) continue;
        const double x0 = A[(size_t)(k + 1) * n + k];
        const double alpha = x0 > 0 ? -nrm : nrm;
        std::fill(v.begin(), v.end(), 0.0);
        for (int i = k + 1; i < n; ++i) v[i] = A[(size_t)i * n + k];
        v[k + 1] -= alpha;
        double vv = 0;
        for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
        if (vv == 0) continue;
        const double beta = 2.0 / vv;
        // A <- H A H, H = I - beta v v^T: p = beta A v, w = p - (beta/2)(v.p) v, A -= v w^T + w v^T
        for (int i = k; i < n; ++i) {
            double acc = 0;
            for (int j = k + 1; j < n; ++j) acc += A[(size_t)i * n + j] * v[j];
            p[i] = beta * acc;
        }
        double vp = 0;
        for (int i = k + 1; i < n; ++i) vp += v[i] * p[i];
        for (int i = k; i < n; ++i) q[i] = p[i] - 0.5 * beta * vp * v[i];
        for (int i = k; i < n; ++i)
            for (int j = k; j < n; ++j) A[(size_t)i * n + j] -= v[i] * q[j] + q[i] * v[j];
        // Q <- Q H
        for (int i = 0; i < n; ++i) {
            double acc = 0;
            for (int j = k + 1; j < n; ++j) acc += Q[(size_t)i * n + j] * v[j];
            acc *= beta;
            for (int j = k + 1; j < n; ++j) Q[(size_t)i * n + j] -= acc * v[j];
        }
    }
    d.assign(n, 0.0);
    std::vector<double> e(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];
    // implicit QL on the tridiagonal (d, e), rotations accumulated into Q held
    // transposed (each rotation then updates two contiguous rows)
    std::vector<double> QT((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) QT[(size_t)k * n + i] = Q[(size_t)i * n + k];
    for (int l = 0; l < n; ++l) {
        for (int iter = 0; iter < 200; ++iter) {
            int m = l;
            for (; m + 1 < n; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-16 * dd) break;
            }
            if (m == l) break;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double s = 1.0, cth = 1.0, pp = 0.0;
            int i = m - 1;
            for (; i >= l; --i) {
                double f = s * e[i], b = cth * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= pp;
                    e[m] = 0.0;
                    break;
                }
                s = f / r;
                cth = g / r;
                g = d[i + 1] - pp;
                r = (d[i] - g) * s + 2.0 * cth * b;
                pp = s * r;
                d[i + 1] = g + pp;
                g = cth * r - b;
                double* qi = &QT[(size_t)i * n];
                double* qj = &QT[(size_t)(i + 1) * n];
                for (int k = 0; k < n; ++k) {
                    const double qa = qj[k];
                    qj[k] = s * qi[k] + cth * qa;
                    qi[k] = cth * qi[k] - s * qa;
                }
            }
            if (r == 0.0 && i >= l) continue;
            d[l] -= pp;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) Q[(size_t)i * n + k] = QT[(size_t)k * n + i];
}

// The 1D DG operator of the scheme along a whole z-column for one component:
// per element modulus kap[e], width hz[e]; lift, averaged traction and
// penalty C (p0+1)^2 / min(h) with the averaged modulus on interfaces; the
// boundary conditions of the top and bottom faces.  n = n_z N unknowns.
std::vector<double> column_1d(const Lgl& g, const std::vector<double>& hz, const std::vector<double>& kap,
                              double cn2, int bc_top, int bc_bot) {
    const int N = g.N, nz = (int)hz.size(), n = nz * N;
    std::vector<double> K((size_t)n * n, 0.0), u(n), gr(n), S(n), r(n), jl(nz), jh(nz);
    const bool dtop = bc_top == DGTN_BC_DIRICHLET, dbot = bc_bot == DGTN_BC_DIRICHLET;
    for (int col = 0; col < n; ++col) {
        std::fill(u.begin(), u.end(), 0.0);
        u[col] = 1.0;
        // only elements within one of the unit node see a change; evaluate all for clarity
        const int e0 = std::max(0, col / N - 1), e1 = std::min(nz - 1, col / N + 1);
        std::fill(r.begin(), r.end(), 0.0);
        for (int e = std::max(0, e0 - 1); e <= std::min(nz - 1, e1 + 1); ++e) {
            for (int i = 0; i < N; ++i) {
                double acc = 0;
                for (int a = 0; a < N; ++a) acc += g.D[i * N + a] * u[e * N + a];
                gr[e * N + i] = 2.0 / hz[e] * acc;
                S[e * N + i] = gr[e * N + i];
            }
        }
        for (int e = e0; e <= e1; ++e) {
            jl[e] = e > 0 ? u[e * N] - u[(e - 1) * N + N - 1] : (dtop ? 2.0 * u[e * N] : 0.0);
            jh[e] = e < nz - 1 ? u[e * N + N - 1] - u[(e + 1) * N] : (dbot ? 2.0 * u[e * N + N - 1] : 0.0);
            S[e * N] += jl[e] / (g.w[0] * hz[e]);
            S[e * N + N - 1] -= jh[e] / (g.w[N - 1] * hz[e]);
        }
        for (int e = e0; e <= e1; ++e) {
            for (int a = 0; a < N; ++a) {
                double acc = 0;
                for (int i = 0; i < N; ++i) acc += g.D[i * N + a] * g.w[i] * kap[e] * S[e * N + i];
                r[e * N + a] = acc;
            }
            if (e > 0) {
                const double ks = 0.5 * (kap[e] + kap[e - 1]), sig = cn2 / std::min(hz[e], hz[e - 1]);
                const double fl = -0.5 * (kap[e] * gr[e * N] + kap[e - 1] * gr[(e - 1) * N + N - 1]) - sig * ks * jl[e];
                r[e * N] -= fl;
            } else if (dtop) {
                const double sig = cn2 / hz[e];
                r[e * N] -= -kap[e] * gr[e * N] - sig * kap[e] * jl[e];
            }
            if (e < nz - 1) {
                const double ks = 0.5 * (kap[e] + kap[e + 1]), sig = cn2 / std::min(hz[e], hz[e + 1]);
                const double fl = 0.5 * (kap[e] * gr[e * N + N - 1] + kap[e + 1] * gr[(e + 1) * N]) - sig * ks * jh[e];
                r[e * N + N - 1] -= fl;
            } else if (dbot) {
                const double sig = cn2 / hz[e];
                r[e * N + N - 1] -= kap[e] * gr[e * N + N - 1] - sig * kap[e] * jh[e];
            }
        }
        for (int i = 0; i < n; ++i) K[(size_t)i * n + col] = r[i];
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double s = 0.5 * (K[(size_t)i * n + j] + K[(size_t)j * n + i]);
            K[(size_t)i * n + j] = K[(size_t)j * n + i] = s;
        }
    return K;
}

// 1D DG operator for a unit modulus along a line of elements of widths h[e],
// interface penalties sig_if[e] between elements e and e + 1, and end
// conditions lo / hi (END_NONE or END_DIRICHLET with penalties sig_lo / sig_hi).
std::vector<double> line_1d(const Lgl& g, const std::vector<double>& h, const std::vector<double>& sig_if, int lo,
                            double sig_lo, int hi, double sig_hi) {
    const int N = g.N, ne = (int)h.size(), n = ne * N;
    std::vector<double> K((size_t)n * n, 0.0), u(n), gr(n), S(n), r(n), jl(ne), jh(ne);
    for (int col = 0; col < n; ++col) {
        std::fill(u.begin(), u.end(), 0.0);
        u[col] = 1.0;
        for (int e = 0; e < ne; ++e)
            for (int i = 0; i < N; ++i) {
                double acc = 0;
                for (int a = 0; a < N; ++a) acc += g.D[i * N + a] * u[e * N + a];
                gr[e * N + i] = S[e * N + i] = 2.0 / h[e] * acc;
            }
        for (int e = 0; e < ne; ++e) {
            jl[e] = e > 0 ? u[e * N] - u[(e - 1) * N + N - 1] : (lo == END_DIRICHLET ? 2.0 * u[e * N] : 0.0);
            jh[e] = e < ne - 1 ? u[e * N + N - 1] - u[(e + 1) * N] : (hi == END_DIRICHLET ? 2.0 * u[e * N + N - 1] : 0.0);
            S[e * N] += jl[e] / (g.w[0] * h[e]);
            S[e * N + N - 1] -= jh[e] / (g.w[N - 1] * h[e]);
        }
        for (int e = 0; e < ne; ++e) {
            for (int a = 0; a < N; ++a) {
                double acc = 0;
                for (int i = 0; i < N; ++i) acc += g.D[i * N + a] * g.w[i] * S[e * N + i];
                r[e * N + a] = acc;
            }
            if (e > 0) r[e * N] += 0.5 * (gr[e * N] + gr[(e - 1) * N + N - 1]) + sig_if[e - 1] * jl[e];
            else if (lo == END_DIRICHLET) r[e * N] += gr[e * N] + sig_lo * jl[e];
            if (e < ne - 1) r[e * N + N - 1] -= 0.5 * (gr[e * N + N - 1] + gr[(e + 1) * N]) - sig_if[e] * jh[e];
            else if (hi == END_DIRICHLET) r[e * N + N - 1] -= gr[e * N + N - 1] - sig_hi * jh[e];
        }
        for (int i = 0; i < n; ++i) K[(size_t)i * n + col] = r[i];
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double v = 0.5 * (K[(size_t)i * n + j] + K[(size_t)j * n + i]);
            K[(size_t)i * n + j] = K[(size_t)j * n + i] = v;
        }
    return K;
}

// Node of the 2D column grid at extended coordinates (x, y) of column col (own
// nodes 0..N-1), reached by crossing faces: col' * N^2 + y' * N + x', or -1.
// A corner point is accepted only if crossing the xi face first and the eta
// face first reach the same node (a vertex shared by four columns).
int locate_node(const Level& L, int col, int x, int y) {
    const int N = L.N;
    auto inside = [&](int v) { return v >= 0 && v < N; };
    auto walk = [&](int c, int px, int py, int first) {
        for (int step = 0; step < 3; ++step) {
            if (inside(px) && inside(py)) return c * N * N + py * N + px;
            const int axis = (!inside(px) && !inside(py)) ? first : (!inside(px) ? 0 : 1);
            int f, d, t;
            if (axis == 0) { f = px < 0 ? 0 : 1; d = px < 0 ? -1 - px : px - N; t = py; }
            else { f = py < 0 ? 2 : 3; d = py < 0 ? -1 - py : py - N; t = px; }
            const int nb = L.cnbr[c * 4 + f];
            if (nb < 0) return -1;
            const int code = L.cnf[c * 4 + f], f2 = code & 3;
            const int t2 = (code >> 2) ? N - 1 - t : t;
            switch (f2) {
                case 0: px = d; py = t2; break;
                case 1: px = N - 1 - d; py = t2; break;
                case 2: px = t2; py = d; break;
                default: px = t2; py = N - 1 - d; break;
            }
            c = nb;
        }
        return -1;
    };
    const int a = walk(col, x, y, 0);
    if (inside(x) || inside(y)) return a;
    const int b = walk(col, x, y, 1);
    return a == b ? a : -1;
}

// Generalised eigen-decomposition of the restriction of the line operator K
// (line nodes `idx`, -1 for positions without a node) with the lumped mass
// `mass`: S (row = patch node, column = mode, S^T M S = I) and lambda; modes
// of the absent positions are unit vectors with lambda = 1 (they never see data).
void patch_fdm(const std::vector<double>& K, int nline, const std::vector<double>& mass, const std::vector<int>& idx,
               double* S_out, double* lam_out) {
    const int P = (int)idx.size();
    std::vector<int> real;
    for (int a = 0; a < P; ++a)
        if (idx[a] >= 0) real.push_back(a);
    const int m = (int)real.size();
    std::vector<double> A((size_t)m * m), Q, lam, ms(m);
    for (int i = 0; i < m; ++i) ms[i] = 1.0 / std::sqrt(mass[idx[real[i]]]);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
            A[(size_t)i * m + j] = ms[i] * K[(size_t)idx[real[i]] * nline + idx[real[j]]] * ms[j];
    jacobi_eigen(m, A, Q, lam);
    double lmax = 0;
    for (double l : lam) lmax = std::max(lmax, l);
    for (int q = 0; q < P * P; ++q) S_out[q] = 0.0;
    for (int a = 0; a < m; ++a) {
        lam_out[a] = std::max(lam[a], 1e-14 * lmax);
        for (int i = 0; i < m; ++i) S_out[real[i] * P + a] = ms[i] * Q[(size_t)i * m + a];
    }
    int mode = m;
    for (int a = 0; a < P; ++a)
        if (idx[a] < 0) {
            S_out[a * P + mode] = 1.0;
            lam_out[mode++] = 1.0;
        }
}

struct ColumnData {
    int P = 0;                // patch width N + 2k (N without overlap)
    std::vector<double> S;    // [n_cols][2][P*P]  S_xi, S_eta (row = node, column = mode)
    std::vector<double> lam;  // [n_cols][2][P]    unit-modulus eigenvalues
    std::vector<int> pg;      // [n_cols][P*P]     patch gather table (overlap only)
    std::vector<int> ps;      // [n_cols][N*N][4]  patch sum table (overlap only)
    std::vector<double> rat;  // [n_cols][3][2]    horizontal modulus / c44 per component
    std::vector<double> V;    // [2][3][n][n]      z-eigenvectors (row = z node, column = mode), then transposed
    std::vector<double> Lz;   // [3][n]
};

void build_column(const dgtn_ctx* c, const Level& L, int overlap, ColumnData& out) {
    const int N = L.N, N2 = N * N, nz = L.n_z, n = nz * N;
    const double yr = c->y_ref;
    const int ko = std::max(0, std::min(overlap, N / 2));
    out.P = N + 2 * ko;
    out.S.assign((size_t)L.n_cols * 2 * N2, 0.0);
    out.lam.assign((size_t)L.n_cols * 2 * N, 0.0);
    std::vector<double> width((size_t)L.n_cols * 2, 0.0), sigf((size_t)L.n_cols * 4, 0.0);
    out.rat.assign((size_t)L.n_cols * 6, 1.0);
    // reference c11 / c44 for the horizontal moduli: the thickest layer's material
    int thick = 0;
    for (size_t li = 1; li < c->prob.layers.size(); ++li)
        if (c->prob.layers[li].thickness > c->prob.layers[thick].thickness) thick = (int)li;
    const int mref = c->prob.layers[thick].material;
    const double r11 = c->matc[3 * mref] / c->matc[3 * mref + 2];
    for (int col = 0; col < L.n_cols; ++col) {
        const double* gg = &L.geo2[(size_t)col * 5 * N2];
        for (int d = 0; d < 2; ++d) {
            double sw = 0, sx = 0, sy = 0;
            for (int q = 0; q < N2; ++q) {
                const double ax = gg[(2 * d) * N2 + q], ay = gg[(2 * d + 1) * N2 + q];
                const double am = std::hypot(ax, ay);
                sw += 2.0 / am;
                sx += ax / am;
                sy += ay / am;
            }
            const double h = sw / N2, nm = std::hypot(sx, sy);
            const double dir[2] = {sx / nm, sy / nm};
            int ends[2];
            double sig[2];
            for (int k = 0; k < 2; ++k) {
                const int f = 2 * d + k;
                double s = 0;
                for (int t = 0; t < N; ++t) s += L.sig_side[((size_t)col * 4 + f) * N + t];
                sig[k] = s / N;
                sigf[(size_t)col * 4 + f] = sig[k];
                ends[k] = L.cnbr[col * 4 + f] >= 0 ? END_INTERIOR : end_type(L.cnf[col * 4 + f]);
            }
            width[(size_t)col * 2 + d] = h;
            auto K = element_1d(L.lgl, h, ends[0], sig[0], ends[1], sig[1]);
            fdm_1d(L.lgl, h, K, &out.S[((size_t)col * 2 + d) * N2], &out.lam[((size_t)col * 2 + d) * N], 1.0);
            for (int cc = 0; cc < 2; ++cc)
                out.rat[(size_t)col * 6 + cc * 2 + d] = r11 * dir[cc] * dir[cc] + (1.0 - dir[cc] * dir[cc]);
        }
    }
    if (ko > 0) {
        // overlapping patches: 1D operators along (left neighbour, column, right
        // neighbour) restricted to the k node lines next to each shared face
        const int P = out.P, P2 = P * P;
        out.S.assign((size_t)L.n_cols * 2 * P2, 0.0);
        out.lam.assign((size_t)L.n_cols * 2 * P, 1.0);
        for (int col = 0; col < L.n_cols; ++col)
            for (int d = 0; d < 2; ++d) {
                const int flo = 2 * d, fhi = 2 * d + 1;
                const int nlo = L.cnbr[col * 4 + flo], nhi = L.cnbr[col * 4 + fhi];
                std::vector<double> hs, sig_if;
                if (nlo >= 0) {
                    hs.push_back(width[(size_t)nlo * 2 + ((L.cnf[col * 4 + flo] & 3) >> 1)]);
                    sig_if.push_back(sigf[(size_t)col * 4 + flo]);
                }
                const int own = (int)hs.size() * N;
                hs.push_back(width[(size_t)col * 2 + d]);
                if (nhi >= 0) {
                    hs.push_back(width[(size_t)nhi * 2 + ((L.cnf[col * 4 + fhi] & 3) >> 1)]);
                    sig_if.push_back(sigf[(size_t)col * 4 + fhi]);
                }
                const int lo = nlo >= 0 ? END_NONE : end_type(L.cnf[col * 4 + flo]);
                const int hi = nhi >= 0 ? END_NONE : end_type(L.cnf[col * 4 + fhi]);
                const auto K = line_1d(L.lgl, hs, sig_if, lo, sigf[(size_t)col * 4 + flo], hi,
                                       sigf[(size_t)col * 4 + fhi]);
                const int nline = (int)hs.size() * N;
                std::vector<double> mass(nline);
                for (int e = 0; e < (int)hs.size(); ++e)
                    for (int i = 0; i < N; ++i) mass[e * N + i] = L.lgl.w[i] * 0.5 * hs[e];
                std::vector<int> idx(P, -1);
                for (int a = 0; a < P; ++a) {
                    const int x = a - ko;
                    if (x >= 0 && x < N) idx[a] = own + x;
                    else if (x < 0 && nlo >= 0) idx[a] = own + x;
                    else if (x >= N && nhi >= 0) idx[a] = own + x;
                }
                patch_fdm(K, nline, mass, idx, &out.S[((size_t)col * 2 + d) * P2], &out.lam[((size_t)col * 2 + d) * P]);
            }
        out.pg.assign((size_t)L.n_cols * P2, -1);
        out.ps.assign((size_t)L.n_cols * N2 * 4, -1);
        for (int col = 0; col < L.n_cols; ++col)
            for (int b = 0; b < P; ++b)
                for (int a = 0; a < P; ++a) {
                    const int src = locate_node(L, col, a - ko, b - ko);
                    out.pg[(size_t)col * P2 + b * P + a] = src;
                    if (src < 0) continue;
                    int* slot = &out.ps[(size_t)src * 4];
                    int q = 0;
                    while (q < 4 && slot[q] >= 0) ++q;
                    if (q == 4) throw std::runtime_error("a node lies in more than four column patches");
                    slot[q] = col * P2 + b * P + a;
                }
    }
    // z: one generalized eigenproblem per component, K_z V = M V diag(lz), M = diag(c44 w h / 2)
    out.V.assign((size_t)6 * n * n, 0.0);
    out.Lz.assign((size_t)3 * n, 0.0);
    std::vector<double> ms(n);
    for (int e = 0; e < nz; ++e)
        for (int k = 0; k < N; ++k)
            ms[e * N + k] = 1.0 / std::sqrt(level_mat(c, L)[3 * L.zmat[e] + 2] / yr * L.lgl.w[k] * 0.5 * L.hz[e]);
    // components 0 (= 1, the same modulus along z) and 2 are independent: solved concurrently
    auto solve_component = [&](int cc) {
        std::vector<double> kap(nz);
        for (int e = 0; e < nz; ++e) kap[e] = level_mat(c, L)[3 * L.zmat[e] + (cc == 2 ? 0 : 2)] / yr;
        auto K = column_1d(L.lgl, L.hz, kap, L.pen_z, c->prob.bc_top, c->prob.bc_bottom);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) K[(size_t)i * n + j] *= ms[i] * ms[j];
        std::vector<double> Q, d;
        sym_eigen(n, K, Q, d);
        double dmax = 0;
        for (double x : d) dmax = std::max(dmax, x);
        for (int a = 0; a < n; ++a) {
            out.Lz[(size_t)cc * n + a] = std::max(d[a], 1e-14 * dmax);
            for (int i = 0; i < n; ++i) out.V[((size_t)cc * n + i) * n + a] = ms[i] * Q[(size_t)i * n + a];
        }
    };
    std::thread other(solve_component, 2);
    solve_component(0);
    other.join();
    std::copy(out.V.begin(), out.V.begin() + (size_t)n * n, out.V.begin() + (size_t)n * n);
    std::copy(out.Lz.begin(), out.Lz.begin() + n, out.Lz.begin() + n);
    // the transposes, so that both z-products read their left factor with the row index contiguous
    double* Vt = out.V.data() + (size_t)3 * n * n;
    for (int cc = 0; cc < 3; ++cc)
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < n; ++a) Vt[((size_t)cc * n + a) * n + i] = out.V[((size_t)cc * n + i) * n + a];
}

// ---- level hierarchy -----------------------------------------------------------

// The level with each column's z-elements merged in pairs (an unpaired last one
// kept): fiducial layers whose material, where the pair mixes two, is the
// thickness-weighted average of the two stiffness constants.  Columns, degree and
// side geometry are those of F.
// z-coarsening stops once the coarsest level has at most this many unknowns
constexpr size_t kCoarseTarget = 4096;

Level zcoarsen(const dgtn_ctx* c, const Level& F) {
    Level C = F;
    C.mat = level_mat(c, F);
    C.hz.clear();
    C.ztop.clear();
    C.zmat.clear();
    C.zlayer.clear();
    for (int a = 0; a < F.n_z; a += 2) {
        const int b = a + 1;
        if (b >= F.n_z) {
            C.hz.push_back(F.hz[a]);
            C.ztop.push_back(F.ztop[a]);
            C.zmat.push_back(F.zmat[a]);
            C.zlayer.push_back(F.zlayer[a]);
            continue;
        }
        const double H = F.hz[a] + F.hz[b];
        C.hz.push_back(H);
        C.ztop.push_back(F.ztop[a]);
        C.zlayer.push_back(F.zlayer[a]);
        if (F.zmat[a] == F.zmat[b]) {
            C.zmat.push_back(F.zmat[a]);
            continue;
        }
        const std::vector<double>& fm = level_mat(c, F);
        for (int q = 0; q < 3; ++q)
            C.mat.push_back((F.hz[a] * fm[3 * F.zmat[a] + q] + F.hz[b] * fm[3 * F.zmat[b] + q]) / H);
        C.zmat.push_back((int)C.mat.size() / 3 - 1);
    }
    C.n_z = (int)C.hz.size();
    C.E = C.n_z * C.n_cols;
    return C;
}

void build_transfer(const dgtn_ctx* c, const Level& F, const Level& C, Transfer& T) {
    if (F.N == C.N && F.n_cols == C.n_cols && F.n_z != C.n_z) {
        // z-element pairs: fine element a (upper) and b of coarse element m; the
        // fine nodes sit at coarse coordinates split in proportion to the widths
        T.type = 2;
        const int N = F.N, N2 = N * N;
        T.I.assign((size_t)F.n_z * N2, 0.0);
        T.zpar.assign(F.n_z, -1);
        T.zch.assign((size_t)C.n_z * 2, -1);
        for (int m = 0; m < C.n_z; ++m) {
            const int a = 2 * m, b = 2 * m + 1;
            const bool pair = b < F.n_z;
            const double ha = F.hz[a], hb = pair ? F.hz[b] : 0.0, H = ha + hb;
            for (int half = 0; half < (pair ? 2 : 1); ++half) {
                const int f = a + half;
                std::vector<double> y(N);
                for (int k = 0; k < N; ++k) {
                    const double t = 0.5 * (F.lgl.x[k] + 1.0);  // position within the fine element
                    y[k] = half == 0 ? -1.0 + 2.0 * ha * t / H : -1.0 + 2.0 * (ha + hb * t) / H;
                }
                auto M = lagrange_matrix(C.lgl, y);
                std::copy(M.begin(), M.end(), T.I.begin() + (size_t)f * N2);
                T.zpar[f] = m;
                T.zch[(size_t)m * 2 + half] = f;
            }
        }
        return;
    }
    if (F.N != C.N) {
        T.type = 0;
        T.I = lagrange_matrix(C.lgl, F.lgl.x);  // [Nf][Nc]
        return;
    }
    T.type = 1;
    const int N = F.N;
    T.I.assign(2 * N * N, 0.0);
    for (int s = 0; s < 2; ++s) {
        std::vector<double> y(N);
        for (int a = 0; a < N; ++a) y[a] = -1.0 + s + 0.5 * (F.lgl.x[a] + 1.0);
        auto M = lagrange_matrix(C.lgl, y);
        std::copy(M.begin(), M.end(), T.I.begin() + s * N * N);
    }
    T.parent.assign(F.n_cols, 0);
    T.child.assign(F.n_cols, 0);
    T.children.assign(C.n_cols * 4, -1);
    const auto& P = c->prob;
    for (int cf = 0; cf < F.n_cols; ++cf) {
        int pc, ch;
        if (P.domain == DGTN_DOMAIN_CYLINDER) {
            const int mf = 1 << F.refine, mc = 1 << C.refine;
            const int b = cf / (mf * mf), rem = cf % (mf * mf), t = rem / mf, s = rem % mf;
            pc = b * mc * mc + (t / 2) * mc + s / 2;
            ch = (s % 2) + 2 * (t % 2);
        } else {
            const int nxf = P.nx << F.refine, nxc = P.nx << C.refine;
            const int t = cf / nxf, s = cf % nxf;
            pc = (t / 2) * nxc + s / 2;
            ch = (s % 2) + 2 * (t % 2);
        }
        T.parent[cf] = pc;
        T.child[cf] = ch;
        T.children[pc * 4 + ch] = cf;
    }
    for (int v : T.children)
        if (v < 0) throw std::runtime_error("column hierarchy is not a 2 x 2 refinement");
}

}  // namespace

int solver_key(const dgtn_solve_opts* opts) {
    if (!opts) return 2;
    return 2 * std::max(1, opts->mg_levels) + 1 + 1000 * std::max(0, opts->overlap);
}

dgtn_status prepare_levels(dgtn_ctx* c, const dgtn_solve_opts* opts) {
    const int want = opts ? std::max(1, opts->mg_levels) : 1;
    if (!c->solver) c->solver = new SolverState();
    SolverState& S = *c->solver;
    if (opts && (opts->overlap < 0 || opts->overlap > 3)) {
        set_error("overlap must be 0..3");
        return DGTN_EINVAL;
    }
    if (opts && opts->overlap > 0) {
        // the patch kernels stage 2 x 3 N P^2 + 2 P^2 doubles in LDS
        const int N = c->levels[0].N, P = N + 2 * std::min(opts->overlap, N / 2);
        if (8 * (6 * N * P * P + 2 * P * P) > 65536) {
            set_error("overlap too wide for this polynomial degree");
            return DGTN_EINVAL;
        }
    }
    const int key = solver_key(opts);
    if (S.key_levels == key && (int)S.mg.size() == (int)c->levels.size()) return DGTN_OK;
    c->levels.resize(1);
    int p = c->levels[0].N - 1, r = c->levels[0].refine;
    while ((int)c->levels.size() < want) {
        if (p > 1) p = std::max(1, p / 2);
        else if (r > 0) --r;
        else if (c->levels.back().n_z > 2 && ndof(c->levels.back()) > kCoarseTarget) {
            // then merge layers into fiducial ones until the coarsest solve is small
            c->levels.push_back(zcoarsen(c, c->levels.back()));
            continue;
        } else break;
        c->levels.push_back(build_level(c->prob, p, r, c->levels[0].N - 1, c->levels[0].refine));
    }
    S.mg.assign(c->levels.size(), MgLevel{});
    S.tr.assign(c->levels.size() - 1, Transfer{});
    if (opts) {
        // the levels' smoother data are independent: built concurrently, one thread per level
        std::vector<ColumnData> cols(c->levels.size());
        std::vector<std::exception_ptr> fail(c->levels.size());
        std::vector<std::thread> workers;
        for (size_t l = 0; l < c->levels.size(); ++l)
            workers.emplace_back([&, l]() {
                try {
                    build_fdm(c, c->levels[l], S.mg[l].fdm);
                    build_column(c, c->levels[l], opts->overlap, cols[l]);
                } catch (...) {
                    fail[l] = std::current_exception();
                }
            });
        for (auto& t : workers) t.join();
        for (auto& f : fail)
            if (f) std::rethrow_exception(f);
        for (size_t l = 0; l < c->levels.size(); ++l) {
            ColumnData& cd = cols[l];
            MgLevel& M = S.mg[l];
            M.P = cd.P;
            M.pg = std::move(cd.pg);
            M.ps = std::move(cd.ps);
            M.cw.assign(M.ps.size() / 4, 1.0);
            for (size_t q = 0; q < M.cw.size(); ++q) {
                int cnt = 0;
                for (int t = 0; t < 4; ++t) cnt += M.ps[q * 4 + t] >= 0;
                M.cw[q] = 1.0 / std::sqrt((double)std::max(cnt, 1));
            }
            M.cS = std::move(cd.S);
            M.clam = std::move(cd.lam);
            M.crat = std::move(cd.rat);
            M.cV = std::move(cd.V);
            M.clz = std::move(cd.Lz);
        }
        for (size_t l = 0; l + 1 < c->levels.size(); ++l) build_transfer(c, c->levels[l], c->levels[l + 1], S.tr[l]);
    }
    const Level& Lc = c->levels.back();
    S.n_coarse = (int)ndof(Lc);
    S.dense = opts && c->levels.size() > 1 && S.n_coarse <= kMaxDenseCoarse;
    S.key_levels = key;
    S.planned = false;
    return DGTN_OK;
}

void plan_solver(dgtn_ctx* c, const dgtn_solve_opts* opts, Layout& lay) {
    SolverState& S = *c->solver;
    if (!opts) { S.planned = false; return; }
    for (size_t l = 0; l < c->levels.size(); ++l) {
        const Level& L = c->levels[l];
        MgLevel& M = S.mg[l];
        const size_t n = ndof(L);
        for (int pi = 0; pi < 2; ++pi) {
            const size_t rs = pi == 0 ? 8 : 4;
            M.off_fdm[pi] = lay.take(rs * M.fdm.size());
            M.off_cS[pi] = lay.take(rs * M.cS.size());
            M.off_clam[pi] = lay.take(rs * M.clam.size());
            M.off_crat[pi] = lay.take(rs * M.crat.size());
            M.off_cV[pi] = lay.take(rs * M.cV.size());
            M.off_clz[pi] = lay.take(rs * M.clz.size());
            const size_t np = M.P > 0 ? n / ((size_t)L.N * L.N) * M.P * M.P : n;
            M.off_cT[pi] = lay.take(rs * np);
            M.off_cY[pi] = lay.take(rs * np);
            M.off_b[pi] = lay.take(rs * n);
            if (pi == 0) {
                M.off_pg = lay.take(4 * M.pg.size());
                M.off_ps = lay.take(4 * M.ps.size());
            }
            M.off_cw[pi] = lay.take(rs * M.cw.size());
            M.off_x[pi] = lay.take(rs * n);
            M.off_t[pi] = lay.take(rs * n);
        }
    }
    for (auto& T : S.tr) {
        for (int pi = 0; pi < 2; ++pi) T.off_I[pi] = lay.take((pi == 0 ? 8 : 4) * T.I.size());
        if (T.type == 1) {
            T.off_parent = lay.take(4 * T.parent.size());
            T.off_child = lay.take(4 * T.child.size());
            T.off_children = lay.take(4 * T.children.size());
        } else if (T.type == 2) {
            T.off_zpar = lay.take(4 * T.zpar.size());
            T.off_zch = lay.take(4 * T.zch.size());
        }
    }
    if (S.dense) {
        const size_t nc = S.n_coarse;
        S.off_Ainv[0] = lay.take(8 * nc * nc);
        S.off_Ainv[1] = lay.take(4 * nc * nc);
        S.off_col = lay.take(8 * dense_invert_scratch((int)nc));
    }
    const size_t n = ndof(c->levels[0]);
    S.m = std::max(4, std::min(200, opts->restart));
    S.nblk = (int)std::min<size_t>(1024, std::max<size_t>(1, n / 4096));
    S.off_V = lay.take(8 * n * (S.m + 1));
    S.off_Z = lay.take(8 * n * S.m);
    S.off_w = lay.take(8 * n);
    S.off_r = lay.take(8 * n);
    S.off_partial = lay.take(8 * (size_t)(S.m + 2) * S.nblk);
    S.off_dots = lay.take(8 * (size_t)(S.m + 2));
    S.off_coef = lay.take(8 * (size_t)(S.m + 2));
    S.off_sc = lay.take(8 * 16);
    S.planned = true;
}

#define SHIP(...)                                                                    \
    do {                                                                             \
        hipError_t e_ = (__VA_ARGS__);                                               \
        if (e_ != hipSuccess) {                                                      \
            set_error(std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_));     \
            return DGTN_EHIP;                                                        \
        }                                                                            \
    } while (0)

namespace {

template <typename R>
R* at(const dgtn_ctx* c, size_t off) {
    return reinterpret_cast<R*>(c->ws + off);
}

template <typename R>
dgtn_status level_apply(dgtn_ctx* c, int l, const R* u, R* out, R scale, hipStream_t s) {
    const Level& L = c->levels[l];
    auto v = view_of<R>(c, L);
    SHIP(launch_traction<R>(v, u, tau_of<R>(c, L), s));
    SHIP(launch_apply<R>(v, u, tau_of<R>(c, L), out, scale, s));
    return DGTN_OK;
}

dgtn_status upload(dgtn_ctx* c, size_t off, const void* src, size_t bytes, hipStream_t s) {
    SHIP(hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, s));
    return DGTN_OK;
}

}  // namespace

dgtn_status bind_solver(dgtn_ctx* c, hipStream_t s) {
    SolverState& S = *c->solver;
    S.drop_graphs();
    if (!S.planned) return DGTN_OK;
    std::vector<std::vector<float>> keep;
    auto up2 = [&](const size_t off[2], const std::vector<double>& v) -> dgtn_status {
        dgtn_status st = upload(c, off[0], v.data(), 8 * v.size(), s);
        if (st != DGTN_OK) return st;
        keep.emplace_back(v.begin(), v.end());
        return upload(c, off[1], keep.back().data(), 4 * v.size(), s);
    };
    for (auto& M : S.mg) {
        dgtn_status st;
        if ((st = up2(M.off_fdm, M.fdm)) != DGTN_OK) return st;
        if ((st = up2(M.off_cS, M.cS)) != DGTN_OK) return st;
        if ((st = up2(M.off_clam, M.clam)) != DGTN_OK) return st;
        if ((st = up2(M.off_crat, M.crat)) != DGTN_OK) return st;
        if ((st = up2(M.off_cV, M.cV)) != DGTN_OK) return st;
        if ((st = up2(M.off_clz, M.clz)) != DGTN_OK) return st;
        if (!M.pg.empty()) {
            if ((st = upload(c, M.off_pg, M.pg.data(), 4 * M.pg.size(), s)) != DGTN_OK) return st;
            if ((st = upload(c, M.off_ps, M.ps.data(), 4 * M.ps.size(), s)) != DGTN_OK) return st;
            if ((st = up2(M.off_cw, M.cw)) != DGTN_OK) return st;
        }
    }
    for (auto& T : S.tr) {
        dgtn_status st = up2(T.off_I, T.I);
        if (st != DGTN_OK) return st;
        if (T.type == 1) {
            if ((st = upload(c, T.off_parent, T.parent.data(), 4 * T.parent.size(), s)) != DGTN_OK) return st;
            if ((st = upload(c, T.off_child, T.child.data(), 4 * T.child.size(), s)) != DGTN_OK) return st;
            if ((st = upload(c, T.off_children, T.children.data(), 4 * T.children.size(), s)) != DGTN_OK) return st;
        } else if (T.type == 2) {
            if ((st = upload(c, T.off_zpar, T.zpar.data(), 4 * T.zpar.size(), s)) != DGTN_OK) return st;
            if ((st = upload(c, T.off_zch, T.zch.data(), 4 * T.zch.size(), s)) != DGTN_OK) return st;
        }
    }
    SHIP(hipStreamSynchronize(s));
    if (S.dense) {
        // assemble the coarsest operator column by column (A is symmetric, so
        // column j is stored as row j), then invert it in place
        const int lc = (int)c->levels.size() - 1;
        const int nc = S.n_coarse;
        double* e = at<double>(c, S.mg[lc].off_b[0]);
        double* A = at<double>(c, S.off_Ainv[0]);
        SHIP(vec_zero<double>(e, nc, s));
        for (int j = 0; j < nc; ++j) {
            SHIP(dense_set_unit(e, j, s));
            dgtn_status st = level_apply<double>(c, lc, e, A + (size_t)j * nc, 1.0, s);
            if (st != DGTN_OK) return st;
        }
        SHIP(dense_invert(A, at<double>(c, S.off_col), nc, s));
        SHIP(vec_cast<double, float>(A, at<float>(c, S.off_Ainv[1]), (size_t)nc * nc, 1.0, s));
        SHIP(hipStreamSynchronize(s));
    }
    return DGTN_OK;
}

namespace {

struct VOpts {
    int nu;
    double omega;
    bool identity;
    int smoother;
};

// One damped additive-Schwarz sweep on level l: x = (x or 0) + omega M^{-1} (b - Ax).
template <typename R>
dgtn_status smooth(dgtn_ctx* c, int l, const VOpts& o, const R* b, const R* Ax, R* x, hipStream_t s) {
    SolverState& S = *c->solver;
    const int pi = sizeof(R) == 8 ? 0 : 1;
    const Level& L = c->levels[l];
    MgLevel& M = S.mg[l];
    if (o.smoother == DGTN_SMOOTH_COLUMN && M.P > L.N) {
        SHIP(mg_ovl_smooth<R>(L.N, L.n_cols, L.n_z, M.P, at<int>(c, M.off_pg), at<int>(c, M.off_ps),
                              at<R>(c, M.off_cw[pi]),
                              at<R>(c, M.off_cS[pi]), at<R>(c, M.off_clam[pi]), at<R>(c, M.off_crat[pi]),
                              at<R>(c, M.off_cV[pi]), at<R>(c, M.off_clz[pi]), b, Ax, x, (R)o.omega,
                              at<R>(c, M.off_cT[pi]), at<R>(c, M.off_cY[pi]), s));
    } else if (o.smoother == DGTN_SMOOTH_COLUMN) {
        SHIP(mg_col_smooth<R>(L.N, L.n_cols, L.n_z, at<R>(c, M.off_cS[pi]), at<R>(c, M.off_clam[pi]),
                              at<R>(c, M.off_crat[pi]), at<R>(c, M.off_cV[pi]), at<R>(c, M.off_clz[pi]), b, Ax, x,
                              (R)o.omega, at<R>(c, M.off_cT[pi]), at<R>(c, M.off_cY[pi]), s));
    } else {
        SHIP(mg_smooth<R>(L.N, L.E, at<R>(c, M.off_fdm[pi]), b, Ax, x, (R)o.omega, s));
    }
    return DGTN_OK;
}

// x_l = V-cycle(b_l), zero initial guess, on level l.
template <typename R>
dgtn_status vcycle(dgtn_ctx* c, int l, const VOpts& o, hipStream_t s) {
    SolverState& S = *c->solver;
    const int pi = sizeof(R) == 8 ? 0 : 1;
    const Level& L = c->levels[l];
    MgLevel& M = S.mg[l];
    R* b = at<R>(c, M.off_b[pi]);
    R* x = at<R>(c, M.off_x[pi]);
    R* t = at<R>(c, M.off_t[pi]);
    const R* fdm = at<R>(c, M.off_fdm[pi]);
    const size_t n = ndof(L);
    const bool last = l == (int)c->levels.size() - 1;
    if (last && S.dense) {
        SHIP(dense_gemv<R>(at<R>(c, S.off_Ainv[pi]), b, x, (int)n, s));
        return DGTN_OK;
    }
    const int nu = o.nu;
    (void)fdm;
    dgtn_status st0 = smooth<R>(c, l, o, b, nullptr, x, s);
    if (st0 != DGTN_OK) return st0;
    for (int k = 1; k < nu; ++k) {
        dgtn_status st = level_apply<R>(c, l, x, t, R(1), s);
        if (st != DGTN_OK) return st;
        if ((st = smooth<R>(c, l, o, b, t, x, s)) != DGTN_OK) return st;
    }
    if (last) return DGTN_OK;
    dgtn_status st = level_apply<R>(c, l, x, t, R(1), s);
    if (st != DGTN_OK) return st;
    SHIP(vec_resid<R>(b, t, n, s));
    const Level& C = c->levels[l + 1];
    MgLevel& MC = S.mg[l + 1];
    const Transfer& T = S.tr[l];
    R* bc = at<R>(c, MC.off_b[pi]);
    R* xc = at<R>(c, MC.off_x[pi]);
    const R* I = at<R>(c, T.off_I[pi]);
    if (T.type == 0) SHIP(mg_restrict_p<R>(L.E, L.N, C.N, I, t, bc, s));
    else if (T.type == 2) SHIP(mg_restrict_z<R>(L.N, C.E, L.n_cols, at<int>(c, T.off_zch), I, t, bc, s));
    else SHIP(mg_restrict_h<R>(L.N, C.E, L.n_cols, C.n_cols, at<int>(c, T.off_children), I, t, bc, s));
    st = vcycle<R>(c, l + 1, o, s);
    if (st != DGTN_OK) return st;
    if (T.type == 0) SHIP(mg_prolong_p<R>(L.E, L.N, C.N, I, xc, x, s));
    else if (T.type == 2) SHIP(mg_prolong_z<R>(L.N, L.E, L.n_cols, at<int>(c, T.off_zpar), I, xc, x, s));
    else
        SHIP(mg_prolong_h<R>(L.N, L.E, L.n_cols, C.n_cols, at<int>(c, T.off_parent), at<int>(c, T.off_child), I, xc,
                             x, s));
    for (int k = 0; k < o.nu; ++k) {
        st = level_apply<R>(c, l, x, t, R(1), s);
        if (st != DGTN_OK) return st;
        if ((st = smooth<R>(c, l, o, b, t, x, s)) != DGTN_OK) return st;
    }
    return DGTN_OK;
}

// The level-0 V-cycle (b -> x in the level-0 workspace buffers) on stream s: the
// recorded graph for this precision and smoother setting, recorded on first use.
// If recording fails, V-cycles run eagerly from then on.
dgtn_status vcycle_launch(dgtn_ctx* c, int prec, const VOpts& o, hipStream_t s) {
    SolverState& S = *c->solver;
    auto eager = [&]() { return prec == 32 ? vcycle<float>(c, 0, o, s) : vcycle<double>(c, 0, o, s); };
    if (S.graphs_off) return eager();
    for (const auto& g : S.vgraphs)
        if (g.prec == prec && g.nu == o.nu && g.smoother == o.smoother && g.omega == o.omega) {
            SHIP(hipGraphLaunch(g.exec, s));
            return DGTN_OK;
        }
    if (!S.cap_stream && hipStreamCreateWithFlags(&S.cap_stream, hipStreamNonBlocking) != hipSuccess) {
        S.graphs_off = true;
        return eager();
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamBeginCapture(S.cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        S.graphs_off = true;
        return eager();
    }
    const dgtn_status st = prec == 32 ? vcycle<float>(c, 0, o, S.cap_stream) : vcycle<double>(c, 0, o, S.cap_stream);
    const hipError_t ec = hipStreamEndCapture(S.cap_stream, &graph);
    if (st != DGTN_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    const bool ok = ec == hipSuccess && graph && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    if (!ok) {
        S.graphs_off = true;
        return eager();
    }
    S.vgraphs.push_back({prec, o.nu, o.smoother, o.omega, exec});
    SHIP(hipGraphLaunch(exec, s));
    return DGTN_OK;
}

// The FP32 preconditioner's input is the FP64 vector times scale32, a power of
// two, and its output is divided by it: exact in FP64, and for a vector of RMS
// entry about 1 it keeps the FP32 values in the normal range.  (An adjoint load
// of S_x, 4 kB T phi / (pi f F0^2) ~ 1e-27 times the layer energy operators,
// otherwise puts the small residual entries below FP32's 1.2e-38, where they
// lose their digits: the FP32-preconditioned solve of the forty-layer mirror's
// adjoint stalled near 2e-6.)  Where all values stay normal, the roundings are
// those of the unscaled vector: the solve is unchanged bit for bit.
double fp32_scale(double norm, size_t n) {
    if (!(norm > 0) || !std::isfinite(norm) || n == 0) return 1.0;
    int e = 0;
    std::frexp(norm / std::sqrt((double)n), &e);
    return std::ldexp(1.0, std::max(-900, std::min(900, -e)));
}

// z = M^{-1} v in the preconditioner's precision (v, z FP64); scale32 as above.
dgtn_status precondition(dgtn_ctx* c, int prec, const VOpts& o, const double* v, double* z, hipStream_t s,
                         double scale32 = 1.0) {
    SolverState& S = *c->solver;
    const size_t n = ndof(c->levels[0]);
    if (o.identity) {
        SHIP(vec_cast<double, double>(v, z, n, 1.0, s));
        return DGTN_OK;
    }
    if (prec == 32) {
        SHIP(vec_cast<double, float>(v, at<float>(c, S.mg[0].off_b[1]), n, scale32, s));
        dgtn_status st = vcycle_launch(c, 32, o, s);
        if (st != DGTN_OK) return st;
        SHIP(vec_cast<float, double>(at<float>(c, S.mg[0].off_x[1]), z, n, 1.0 / scale32, s));
    } else {
        SHIP(vec_cast<double, double>(v, at<double>(c, S.mg[0].off_b[0]), n, 1.0, s));
        dgtn_status st = vcycle_launch(c, 64, o, s);
        if (st != DGTN_OK) return st;
        SHIP(vec_cast<double, double>(at<double>(c, S.mg[0].off_x[0]), z, n, 1.0, s));
    }
    return DGTN_OK;
}

dgtn_status dots(dgtn_ctx* c, const double* V, int nv, const double* w, size_t n, std::vector<double>& out,
                 hipStream_t s) {
    SolverState& S = *c->solver;
    double* dd = at<double>(c, S.off_dots);
    SHIP(vec_multidot(V, n, nv, w, n, at<double>(c, S.off_partial), S.nblk, dd, s));
    out.resize(nv + 1);
    SHIP(hipMemcpyAsync(out.data(), dd, 8 * (nv + 1), hipMemcpyDeviceToHost, s));
    SHIP(hipStreamSynchronize(s));
    return DGTN_OK;
}

dgtn_status axpys(dgtn_ctx* c, double* w, const double* V, int nv, const std::vector<double>& coef, size_t n,
                  hipStream_t s) {
    SolverState& S = *c->solver;
    double* cd = at<double>(c, S.off_coef);
    SHIP(hipMemcpyAsync(cd, coef.data(), 8 * nv, hipMemcpyHostToDevice, s));
    SHIP(vec_multiaxpy(w, V, n, nv, cd, n, s));
    return DGTN_OK;
}

}  // namespace

}  // namespace dgtn

dgtn_status dgtn::SolverState::host_monitor() {
    if (host_mon) return DGTN_OK;
    void* h = nullptr;
    if (hipHostMalloc(&h, 32 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        set_error("pinned host allocation for the solver monitors failed");
        return DGTN_ENOMEM;
    }
    host_mon = static_cast<double*>(h);
    for (auto& e : mon_event)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            set_error("hipEventCreate failed");
            return DGTN_EHIP;
        }
    return DGTN_OK;
}

void dgtn::SolverState::drop_graphs() {
    for (auto& g : vgraphs) (void)hipGraphExecDestroy(g.exec);
    vgraphs.clear();
}

dgtn::SolverState::~SolverState() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto& e : mon_event)
        if (e) (void)hipEventDestroy(e);
    if (host_mon) (void)hipHostFree(host_mon);
}

dgtn_ctx::~dgtn_ctx() { delete solver; }

using namespace dgtn;

extern "C" dgtn_status dgtn_level_info(dgtn_ctx* c, const dgtn_solve_opts* opts, int level, int* N, int* n_elem,
                                       int* n_cols) {
    if (!c || !N || !n_elem || !n_cols) { set_error("null argument"); return DGTN_EINVAL; }
    try {
        dgtn_status st = prepare_levels(c, opts);
        if (st != DGTN_OK) return st;
    } catch (const std::exception& ex) {
        set_error(ex.what());
        return DGTN_EINVAL;
    }
    if (level < 0 || level >= (int)c->levels.size()) { set_error("no such level"); return DGTN_EINVAL; }
    const Level& L = c->levels[level];
    *N = L.N;
    *n_elem = L.E;
    *n_cols = L.n_cols;
    return DGTN_OK;
}

extern "C" dgtn_status dgtn_smoother_block(dgtn_ctx* c, const dgtn_solve_opts* opts, int level, int elem,
                                           double* out) {
    if (!c || !opts || !out) { set_error("null argument"); return DGTN_EINVAL; }
    try {
        dgtn_status st = prepare_levels(c, opts);
        if (st != DGTN_OK) return st;
    } catch (const std::exception& ex) {
        set_error(ex.what());
        return DGTN_EINVAL;
    }
    if (level < 0 || level >= (int)c->levels.size()) { set_error("no such level"); return DGTN_EINVAL; }
    const Level& L = c->levels[level];
    if (elem < 0 || elem >= L.E) { set_error("no such element"); return DGTN_EINVAL; }
    const size_t per = 9 * (size_t)(L.N * L.N + L.N);
    const auto& f = c->solver->mg[level].fdm;
    std::copy(f.begin() + elem * per, f.begin() + (elem + 1) * per, out);
    return DGTN_OK;
}

extern "C" dgtn_status dgtn_patch_table(dgtn_ctx* c, const dgtn_solve_opts* opts, int level, int* P, int* table) {
    if (!c || !opts || !P) { set_error("null argument"); return DGTN_EINVAL; }
    try {
        dgtn_status st = prepare_levels(c, opts);
        if (st != DGTN_OK) return st;
    } catch (const std::exception& ex) {
        set_error(ex.what());
        return DGTN_EINVAL;
    }
    if (level < 0 || level >= (int)c->levels.size()) { set_error("no such level"); return DGTN_EINVAL; }
    const MgLevel& M = c->solver->mg[level];
    const Level& L = c->levels[level];
    *P = M.P;
    if (table) {
        if (M.pg.empty()) {  // no overlap: every column's patch is its own grid
            for (int col = 0; col < L.n_cols; ++col)
                for (int q = 0; q < L.N * L.N; ++q) table[(size_t)col * L.N * L.N + q] = col * L.N * L.N + q;
        } else {
            std::copy(M.pg.begin(), M.pg.end(), table);
        }
    }
    return DGTN_OK;
}

extern "C" dgtn_status dgtn_precondition(dgtn_ctx* c, const dgtn_solve_opts* opts, const double* v, double* z,
                                         hipStream_t s) {
    if (!c || !opts || !v || !z) { set_error("null argument"); return DGTN_EINVAL; }
    if (!c->bound || !c->has_opts || !c->solver || !c->solver->planned ||
        solver_key(opts) != c->solver->key_levels) {
        set_error("bind a workspace with these solve options first");
        return DGTN_EINVAL;
    }
    if (opts->precond_precision != 64 && opts->precond_precision != 32) {
        set_error("precond_precision must be 64 or 32"); return DGTN_EINVAL;
    }
    const VOpts vo{opts->smooth_steps, opts->smooth_damping, opts->mg_levels == 0, opts->smoother};
    double scale32 = 1.0;
    if (opts->precond_precision == 32 && !vo.identity) {
        std::vector<double> d;
        const size_t n = ndof(c->levels[0]);
        const dgtn_status st = dots(c, nullptr, 0, v, n, d, s);
        if (st != DGTN_OK) return st;
        scale32 = fp32_scale(std::sqrt(d[0]), n);
    }
    return precondition(c, opts->precond_precision, vo, v, z, s, scale32);
}

extern "C" dgtn_status dgtn_solve(dgtn_ctx* c, const dgtn_solve_opts* opts, const double* b, double* u,
                                  dgtn_solve_stats* stats, hipStream_t s) {
    if (!c || !opts || !b || !u) { set_error("null argument"); return DGTN_EINVAL; }
    if (!c->bound || !c->has_opts || !c->solver || !c->solver->planned) {
        set_error("bind a workspace with solve options first");
        return DGTN_EINVAL;
    }
    if (opts->precond_precision != 64 && opts->precond_precision != 32) {
        set_error("precond_precision must be 64 or 32"); return DGTN_EINVAL;
    }
    if (opts->mg_levels < 0 || solver_key(opts) != c->solver->key_levels ||
        std::max(4, opts->restart) > c->solver->m || opts->restart < 1) {
        set_error("solve options differ from the bound ones (mg_levels/overlap/restart)");
        return DGTN_EINVAL;
    }
    if (!(opts->rtol > 0) || opts->max_iter < 1 || opts->smooth_steps < 1 || !(opts->smooth_damping > 0)) {
        set_error("invalid solve options"); return DGTN_EINVAL;
    }
    if (opts->residual_precision != 0 && opts->residual_precision != 64 && opts->residual_precision != 128) {
        set_error("residual_precision must be 64 or 128"); return DGTN_EINVAL;
    }
    if (opts->residual_precision == 128 && !c->res.ok) {
        set_error("the double-double residual covers p <= 7"); return DGTN_EINVAL;
    }
    const auto t0 = std::chrono::steady_clock::now();
    const bool verbose = std::getenv("DGTN_VERBOSE") != nullptr;
    SolverState& S = *c->solver;
    const size_t n = ndof(c->levels[0]);
    const int m = opts->restart;
    const VOpts vo{opts->smooth_steps, opts->smooth_damping, opts->mg_levels == 0, opts->smoother};
    double* V = at<double>(c, S.off_V);
    double* Z = at<double>(c, S.off_Z);
    double* w = at<double>(c, S.off_w);
    double* r = at<double>(c, S.off_r);
    const double yr = c->y_ref;
    std::vector<double> d;
    dgtn_status st;

    // ||b||
    if ((st = dots(c, nullptr, 0, b, n, d, s)) != DGTN_OK) return st;
    const double bnorm = std::sqrt(d[0]);
    if (!std::isfinite(bnorm)) { set_error("non-finite right-hand side"); return DGTN_ENAN; }
    const double s32 = fp32_scale(bnorm, n);  // FP32 preconditioner input scaling
    // b - A u into `out`, in FP64 or (residual_precision 128) double-double
    const bool dd_resid = opts->residual_precision == 128;
    auto residual_into = [&](double* out) -> dgtn_status {
        if (dd_resid) {
            SHIP(residual_dd(c, b, u, out, s));
            return DGTN_OK;
        }
        dgtn_status e = level_apply<double>(c, 0, u, out, yr, s);
        if (e != DGTN_OK) return e;
        SHIP(vec_resid<double>(b, out, n, s));
        return DGTN_OK;
    };
    auto true_residual = [&](double& beta) -> dgtn_status {
        dgtn_status e = residual_into(r);
        if (e != DGTN_OK) return e;
        e = dots(c, nullptr, 0, r, n, d, s);
        if (e != DGTN_OK) return e;
        beta = std::sqrt(d[0]);
        return DGTN_OK;
    };
    double beta;
    if ((st = true_residual(beta)) != DGTN_OK) return st;
    int iters = 0, restarts = 0;
    const double target = opts->rtol * (bnorm > 0 ? bnorm : 1.0);
    dgtn_status result = DGTN_OK;
    std::string why = "iteration limit reached";
    if (opts->krylov == DGTN_KRYLOV_FCG && beta > target) {
        // Flexible preconditioned conjugate gradients (Polak-Ribiere beta).  The
        // scalars stay on the device; the host reads the residual norm and the
        // breakdown flag of iteration k while iteration k+1 is already queued, so
        // the GPU never waits for the host.  The FP64 true residual replaces the
        // recurrence every `refresh` iterations and confirms convergence.
        double* pr = r;                    // residual
        double* zn = V;                    // z_{k+1}
        double* zo = V + n;                // z_k
        double* pp = V + 2 * n;            // search direction
        double* q = w;                     // A p
        double* sc = at<double>(c, S.off_sc);  // [0] p.Ap, [1] breakdown flag, [4 + 4s ..] r.z slots
        const int refresh = 50;
        // FP32 preconditioner input (level 0), written by the CG update; null otherwise
        float* const b32 = opts->precond_precision == 32 && !vo.identity ? at<float>(c, S.mg[0].off_b[1]) : nullptr;
        if ((st = S.host_monitor()) != DGTN_OK) return st;
        auto slot = [&](int k) { return sc + 4 + 4 * (k & 1); };
        int par = 0;
        const double* dx[4];
        const double* dy[4];
        // (re)start from the residual in pr: z = M r, p = z, slot(par)[0] = r.z
        auto start = [&]() -> dgtn_status {
            dgtn_status e = precondition(c, opts->precond_precision, vo, pr, zn, s, s32);
            if (e != DGTN_OK) return e;
            SHIP(vec_cast<double, double>(zn, pp, n, 1.0, s));
            dx[0] = pr; dy[0] = zn;
            SHIP(vec_dotpairs(1, dx, dy, n, at<double>(c, S.off_partial), S.nblk, slot(par), s));
            SHIP(hipMemsetAsync(sc + 1, 0, sizeof(double), s));
            std::swap(zn, zo);
            return DGTN_OK;
        };
        if ((st = start()) != DGTN_OK) return st;
        double breakdown_beta = std::numeric_limits<double>::infinity();
        double best_beta = std::numeric_limits<double>::infinity();
        int best_it = 0;
        const int patience = 200;
        bool have_prev = false;
        int mon_slot[2] = {0, 0};
        while (true) {
            if (iters >= opts->max_iter) { result = DGTN_ENOCONV; break; }
            double* cur = slot(par);
            double* nxt = slot(par + 1);
            if ((st = level_apply<double>(c, 0, pp, q, yr, s)) != DGTN_OK) return st;
            dx[0] = pp; dy[0] = q;
            SHIP(vec_dotpairs(1, dx, dy, n, at<double>(c, S.off_partial), S.nblk, sc, s));
            // FP32 V-cycle: the update writes its input and the dot products widen its
            // output (the same roundings as precondition's two casts, without their passes)
            SHIP(fcg_update(u, pr, pp, q, cur, sc, b32, s32, n, s));
            const int it = iters++;
            const bool replace = iters % refresh == 0;
            if (replace) {  // residual replacement
                if ((st = residual_into(pr)) != DGTN_OK) return st;
                ++restarts;
            }
            if (b32) {
                if (replace) SHIP(vec_cast<double, float>(pr, b32, n, s32, s));
                if ((st = vcycle_launch(c, 32, vo, s)) != DGTN_OK) return st;
                SHIP(vec_dot3_widen(pr, at<float>(c, S.mg[0].off_x[1]), zn, zo, 1.0 / s32, n, at<double>(c, S.off_partial),
                                    S.nblk, nxt, s));
            } else {
                if ((st = precondition(c, opts->precond_precision, vo, pr, zn, s, s32)) != DGTN_OK) return st;
                dx[0] = pr; dy[0] = zn;
                dx[1] = pr; dy[1] = zo;
                dx[2] = pr; dy[2] = pr;
                SHIP(vec_dotpairs(3, dx, dy, n, at<double>(c, S.off_partial), S.nblk, nxt, s));
            }
            SHIP(fcg_direction(pp, zn, cur, nxt, n, s));
            std::swap(zn, zo);
            par ^= 1;
            // post this iteration's monitors, then read the previous iteration's
            double* hm = S.host_mon + 16 * (it & 1);
            mon_slot[it & 1] = par;  // slot(par) now holds this iteration's r.z, r.z_old, r.r
            SHIP(hipMemcpyAsync(hm, sc, 16 * sizeof(double), hipMemcpyDeviceToHost, s));
            SHIP(hipEventRecord(S.mon_event[it & 1], s));
            if (!have_prev) { have_prev = true; continue; }
            const int pj = (it - 1) & 1;
            SHIP(hipEventSynchronize(S.mon_event[pj]));
            const double* pm = S.host_mon + 16 * pj;
            const double rr = pm[4 + 4 * (mon_slot[pj] & 1) + 2];
            const bool broke = pm[1] != 0.0;
            if (!std::isfinite(rr)) { set_error("NaN/Inf in the solver"); return DGTN_ENAN; }
            beta = std::sqrt(std::max(rr, 0.0));
            if (verbose && it % 10 == 0) std::fprintf(stderr, "dgtn fcg it %d rel %.3e\n", it, beta / bnorm);
            // stagnation: no 1 % progress of the residual in `patience` iterations
            if (beta < 0.99 * best_beta) {
                best_beta = beta;
                best_it = it;
            } else if (it - best_it > patience && beta > target) {
                SHIP(hipStreamSynchronize(s));
                if ((st = true_residual(beta)) != DGTN_OK) return st;
                if (beta <= target) break;
                char msg[128];
                std::snprintf(msg, sizeof msg, "stagnated at relative residual %.3e (the attainable accuracy of "
                              "the operator's arithmetic)", beta / bnorm);
                why = msg;
                result = DGTN_ENOCONV;
                break;
            }
            if (!broke && beta > target) continue;
            // converged by the recurrence, or lost positive curvature: decide on the
            // FP64 true residual of the current iterate
            SHIP(hipStreamSynchronize(s));
            if ((st = true_residual(beta)) != DGTN_OK) return st;
            if (beta <= target) break;
            if (broke) {
                // rounding at the attainable accuracy, or a stale direction: restart
                // once per improvement of the true residual, else report stagnation
                if (!(beta < breakdown_beta)) {
                    char msg[96];
                    std::snprintf(msg, sizeof msg, "stagnated (p.Ap <= 0) at relative residual %.3e", beta / bnorm);
                    why = msg;
                    result = DGTN_ENOCONV;
                    break;
                }
                breakdown_beta = beta;
            }
            ++restarts;
            if ((st = start()) != DGTN_OK) return st;
            have_prev = false;
        }
    }
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    while (opts->krylov != DGTN_KRYLOV_FCG && beta > target) {
        if (!std::isfinite(beta)) { set_error("NaN/Inf in the solver"); return DGTN_ENAN; }
        if (iters >= opts->max_iter) { result = DGTN_ENOCONV; break; }
        SHIP(vec_scale_copy(r, V, 1.0 / beta, n, s));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0;
        bool done = false;
        for (; j < m && iters < opts->max_iter; ++j) {
            double* Vj = V + (size_t)j * n;
            double* Zj = Z + (size_t)j * n;
            if ((st = precondition(c, opts->precond_precision, vo, Vj, Zj, s, s32)) != DGTN_OK) return st;
            if ((st = level_apply<double>(c, 0, Zj, w, yr, s)) != DGTN_OK) return st;
            // classical Gram-Schmidt, repeated when the first pass cancels strongly
            if ((st = dots(c, V, j + 1, w, n, d, s)) != DGTN_OK) return st;
            const double ww0 = d[j + 1];
            std::vector<double> h(d.begin(), d.begin() + j + 1), neg(j + 1);
            for (int i = 0; i <= j; ++i) neg[i] = -h[i];
            if ((st = axpys(c, w, V, j + 1, neg, n, s)) != DGTN_OK) return st;
            if ((st = dots(c, V, j + 1, w, n, d, s)) != DGTN_OK) return st;
            double ww = d[j + 1];
            if (ww < 0.5 * ww0) {
                for (int i = 0; i <= j; ++i) { h[i] += d[i]; neg[i] = -d[i]; }
                if ((st = axpys(c, w, V, j + 1, neg, n, s)) != DGTN_OK) return st;
                double sq = 0;
                for (int i = 0; i <= j; ++i) sq += d[i] * d[i];
                ww = std::max(0.0, ww - sq);
            }
            const double hn = std::sqrt(ww);
            ++iters;
            if (!std::isfinite(hn)) { set_error("NaN/Inf in the solver"); return DGTN_ENAN; }
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i];
            H[(size_t)(j + 1) * m + j] = hn;
            if (hn > 0) SHIP(vec_scale_copy(w, V + (size_t)(j + 1) * n, 1.0 / hn, n, s));
            for (int i = 0; i < j; ++i) {  // previous Givens rotations
                const double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
            const double rho = std::hypot(a, bb);
            cs[j] = rho > 0 ? a / rho : 1.0;
            sn[j] = rho > 0 ? bb / rho : 0.0;
            H[(size_t)j * m + j] = rho;
            H[(size_t)(j + 1) * m + j] = 0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            if (verbose) std::fprintf(stderr, "dgtn fgmres it %d est %.3e\n", iters, std::fabs(g[j + 1]) / bnorm);
            if (std::fabs(g[j + 1]) <= target || hn == 0) { ++j; done = true; break; }
        }
        // u += Z y, H y = g
        for (int i = j - 1; i >= 0; --i) {
            double acc = g[i];
            for (int k = i + 1; k < j; ++k) acc -= H[(size_t)i * m + k] * y[k];
            y[i] = acc / H[(size_t)i * m + i];
        }
        std::vector<double> yy(y.begin(), y.begin() + j);
        if (j > 0 && (st = axpys(c, u, Z, j, yy, n, s)) != DGTN_OK) return st;
        ++restarts;
        if ((st = true_residual(beta)) != DGTN_OK) return st;
        if (verbose) std::fprintf(stderr, "dgtn fgmres restart %d true %.3e\n", restarts, beta / bnorm);
        (void)done;
    }
    SHIP(hipStreamSynchronize(s));
    if (stats) {
        stats->iters = iters;
        stats->restarts = restarts;
        stats->rel_res = bnorm > 0 ? beta / bnorm : beta;
        stats->t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (result == DGTN_ENOCONV) set_error(why);
    return result;
}
