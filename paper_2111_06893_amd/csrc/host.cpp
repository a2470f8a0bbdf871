// Host-side mesh and geometry of the layered mirror (Sec. 2.2.1).
//
// Every mesh here is a two-dimensional quadrilateral disk (or rectangle) mesh
// extruded through the z-layers with an affine z-map per element.  The element
// Jacobian then factorises: dx/dxi and dx/deta lie in the xy-plane and depend
// on (xi, eta) only, dz/dzeta = h_z / 2 is one number per element.  The
// geometry is stored per column (2D inverse metric and determinant at the
// N x N nodes) and per z-element (thickness), which is the same metric as the
// per-node 3D Jacobian written out, in O(N^2) numbers per column.
#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>

#include "internal.h"

namespace dgtn {

namespace {

// Legendre polynomial P_n and its derivative at x (three-term recurrence).
void legendre(int n, double x, double& P, double& dP) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { P = 1.0; dP = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    P = p1;
    dP = (std::fabs(x) < 1.0) ? n * (p0 - x * p1) / (1.0 - x * x)
                              : 0.5 * n * (n + 1.0) * std::pow(x, n + 1);
}

}  // namespace

Lgl make_lgl(int N) {
    Lgl r;
    r.N = N;
    r.x.assign(N, 0.0);
    r.w.assign(N, 0.0);
    r.D.assign(N * N, 0.0);
    const int n = N - 1;
    for (int i = 0; i < N; ++i) {
        // interior nodes: roots of P_n', by Newton from the Chebyshev-Lobatto guess,
        // using (1 - x^2) P_n'' = 2 x P_n' - n (n + 1) P_n
        double x = -std::cos(M_PI * i / n);
        if (i > 0 && i < n) {
            for (int it = 0; it < 100; ++it) {
                double P, dP;
                legendre(n, x, P, dP);
                double d2P = (2.0 * x * dP - n * (n + 1.0) * P) / (1.0 - x * x);
                double dx = dP / d2P;
                x -= dx;
                if (std::fabs(dx) < 1e-16) break;
            }
        }
        r.x[i] = x;
    }
    std::vector<double> Pn(N);
    for (int i = 0; i < N; ++i) {
        double P, dP;
        legendre(n, r.x[i], P, dP);
        Pn[i] = P;
        r.w[i] = 2.0 / (n * (n + 1.0) * P * P);
    }
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double v = 0.0;
            if (i != j) v = Pn[i] / (Pn[j] * (r.x[i] - r.x[j]));
            else if (i == 0) v = -0.25 * n * (n + 1.0);
            else if (i == n) v = 0.25 * n * (n + 1.0);
            r.D[i * N + j] = v;
        }
    return r;
}

std::vector<double> lagrange_matrix(const Lgl& from, const std::vector<double>& y) {
    const int N = from.N;
    std::vector<double> I(y.size() * N, 1.0);
    for (size_t a = 0; a < y.size(); ++a)
        for (int j = 0; j < N; ++j)
            for (int m = 0; m < N; ++m)
                if (m != j) I[a * N + j] *= (y[a] - from.x[m]) / (from.x[j] - from.x[m]);
    return I;
}

namespace {

void cylinder_block(int block, double R, double xi, double eta, double& x, double& y) {
    const double a = R / (2.0 * std::sqrt(2.0));
    if (block == 0) {
        x = a * xi;
        y = a * eta;
        return;
    }
    const double th = M_PI * eta / 4.0;
    double px = 0.5 * (1.0 - xi) * a + 0.5 * (1.0 + xi) * R * std::cos(th);
    double py = 0.5 * (1.0 - xi) * a * eta + 0.5 * (1.0 + xi) * R * std::sin(th);
    for (int q = 1; q < block; ++q) {  // quarter turns
        double t = px;
        px = -py;
        py = t;
    }
    x = px;
    y = py;
}

// (xi, eta) of column col -> (x, y)
void column_point(const Problem& P, int refine, int col, double xi, double eta,
                  double& x, double& y) {
    if (P.domain == DGTN_DOMAIN_CYLINDER) {
        const int m = 1 << refine;
        const int block = col / (m * m);
        const int rem = col % (m * m);
        const int t = rem / m, s = rem % m;
        const double XB = -1.0 + (s + 0.5 * (xi + 1.0)) * (2.0 / m);
        const double EB = -1.0 + (t + 0.5 * (eta + 1.0)) * (2.0 / m);
        cylinder_block(block, P.R, XB, EB, x, y);
    } else if (P.domain == DGTN_DOMAIN_COLUMNS) {
        // the given map of degree q at (xi, eta) by Lagrange interpolation over its LGL points
        const int q1 = P.map_order + 1;
        static thread_local Lgl map;
        if (map.N != q1) map = make_lgl(q1);
        const auto lx = lagrange_matrix(map, {xi});
        const auto ly = lagrange_matrix(map, {eta});
        const double* m = &P.col_xy[(size_t)col * 2 * q1 * q1];
        x = y = 0.0;
        for (int b = 0; b < q1; ++b)
            for (int a = 0; a < q1; ++a) {
                const double wgt = ly[b] * lx[a];
                x += wgt * m[b * q1 + a];
                y += wgt * m[q1 * q1 + b * q1 + a];
            }
    } else {
        // refine multiplies the box resolution by 2^refine in each direction
        const int nx = P.nx << refine, ny = P.ny << refine;
        const int t = col / nx, s = col % nx;
        x = -0.5 * P.Lx + (s + 0.5 * (xi + 1.0)) * (P.Lx / nx);
        y = -0.5 * P.Ly + (t + 0.5 * (eta + 1.0)) * (P.Ly / ny);
    }
}

int columns_of(const Problem& P, int refine) {
    if (P.domain == DGTN_DOMAIN_CYLINDER) return 5 * (1 << (2 * refine));
    if (P.domain == DGTN_DOMAIN_COLUMNS) return P.n_cols_user;
    return (P.nx << refine) * (P.ny << refine);
}

// node (i, j) of side face f at the 1D index t
inline void side_node(int f, int t, int N, int& i, int& j) {
    switch (f) {
        case 0: i = 0; j = t; break;
        case 1: i = N - 1; j = t; break;
        case 2: i = t; j = 0; break;
        default: i = t; j = N - 1; break;
    }
}

}  // namespace

std::vector<double> material_constants(const Problem& P) {
    std::vector<double> c;
    for (const auto& m : P.materials) {
        double c11, c12, c44;
        if (m.kind == DGTN_MAT_ISO) {
            const double Y = m.youngs, nu = m.poisson;
            const double lam = Y * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
            const double mu = Y / (2.0 * (1.0 + nu));
            c11 = lam + 2.0 * mu;
            c12 = lam;
            c44 = mu;
        } else {
            c11 = m.c11;
            c12 = m.c12;
            c44 = m.c44;
        }
        c.push_back(c11);
        c.push_back(c12);
        c.push_back(c44);
    }
    return c;
}

Level build_level(const Problem& P, int p, int refine, int p0, int r0) {
    Level L;
    L.N = p + 1;
    L.pen_z = P.penalty * (p0 + 1.0) * (p0 + 1.0);
    L.refine = refine;
    const int N = L.N, N2 = N * N;
    L.lgl = make_lgl(N);
    L.n_cols = columns_of(P, refine);
    // z-elements from z = 0 downward
    double z = 0.0;
    for (size_t li = 0; li < P.layers.size(); ++li) {
        const auto& lay = P.layers[li];
        std::vector<double> h(lay.n_elem);
        double tot = 0.0;
        for (int i = 0; i < lay.n_elem; ++i) {
            h[i] = std::pow(lay.ratio, i);
            tot += h[i];
        }
        double zz = z;
        for (int i = 0; i < lay.n_elem; ++i) {
            double hz = lay.thickness * h[i] / tot;
            if (i == lay.n_elem - 1) hz = (z + lay.thickness) - zz;
            L.ztop.push_back(zz);
            L.hz.push_back(hz);
            L.zmat.push_back(lay.material);
            L.zlayer.push_back((int)li);
            zz += hz;
        }
        z += lay.thickness;
    }
    L.n_z = (int)L.hz.size();
    L.E = L.n_z * L.n_cols;
    for (double h : L.hz)
        if (!(h > 0.0)) throw std::runtime_error("non-positive element thickness");

    // column node coordinates and the 2D isoparametric metric
    const auto& x = L.lgl.x;
    const auto& D = L.lgl.D;
    L.xy.assign((size_t)L.n_cols * 2 * N2, 0.0);
    L.geo2.assign((size_t)L.n_cols * 5 * N2, 0.0);
    for (int c = 0; c < L.n_cols; ++c) {
        double* X = &L.xy[(size_t)c * 2 * N2];
        double* Y = X + N2;
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) column_point(P, refine, c, x[i], x[j], X[j * N + i], Y[j * N + i]);
        double* g = &L.geo2[(size_t)c * 5 * N2];
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                double Xxi = 0, Xeta = 0, Yxi = 0, Yeta = 0;
                for (int a = 0; a < N; ++a) {
                    Xxi += D[i * N + a] * X[j * N + a];
                    Yxi += D[i * N + a] * Y[j * N + a];
                    Xeta += D[j * N + a] * X[a * N + i];
                    Yeta += D[j * N + a] * Y[a * N + i];
                }
                const double det = Xxi * Yeta - Xeta * Yxi;
                if (!(det > 0.0)) throw std::runtime_error("element map with det J <= 0");
                const int q = j * N + i;
                g[0 * N2 + q] = Yeta / det;   // dxi/dx
                g[1 * N2 + q] = -Xeta / det;  // dxi/dy
                g[2 * N2 + q] = -Yxi / det;   // deta/dx
                g[3 * N2 + q] = Xxi / det;    // deta/dy
                g[4 * N2 + q] = det;
            }
    }

    // side-face connectivity by matching edge node coordinates
    L.cnbr.assign(L.n_cols * 4, -1);
    L.cnf.assign(L.n_cols * 4, 0);
    double scale = 0.0;
    for (double v : L.xy) scale = std::max(scale, std::fabs(v));
    const double tol = 1e-10 * std::max(scale, 1e-300);
    auto edge_pt = [&](int c, int f, int t, double& ex, double& ey) {
        int i, j;
        side_node(f, t, N, i, j);
        ex = L.xy[(size_t)c * 2 * N2 + j * N + i];
        ey = L.xy[(size_t)c * 2 * N2 + N2 + j * N + i];
    };
    struct Edge { double mx, my; int c, f; };
    std::vector<Edge> edges;
    for (int c = 0; c < L.n_cols; ++c)
        for (int f = 0; f < 4; ++f) {
            double mx = 0, my = 0;
            for (int t = 0; t < N; ++t) {
                double ex, ey;
                edge_pt(c, f, t, ex, ey);
                mx += ex;
                my += ey;
            }
            edges.push_back({mx / N, my / N, c, f});
        }
    std::sort(edges.begin(), edges.end(), [](const Edge& a, const Edge& b) { return a.mx < b.mx; });
    for (size_t a = 0; a < edges.size(); ++a) {
        for (size_t b = a + 1; b < edges.size() && edges[b].mx - edges[a].mx <= tol; ++b) {
            if (std::fabs(edges[b].my - edges[a].my) > tol) continue;
            const Edge &A = edges[a], &B = edges[b];
            if (A.c == B.c) continue;
            // orientation: compare the first node of A with the ends of B
            double ax, ay, bx, by, cx, cy;
            edge_pt(A.c, A.f, 0, ax, ay);
            edge_pt(B.c, B.f, 0, bx, by);
            edge_pt(B.c, B.f, N - 1, cx, cy);
            int flip;
            if (std::hypot(ax - bx, ay - by) <= tol) flip = 0;
            else if (std::hypot(ax - cx, ay - cy) <= tol) flip = 1;
            else throw std::runtime_error("non-conforming side faces");
            for (int t = 0; t < N; ++t) {  // every node must match
                double px, py, qx, qy;
                edge_pt(A.c, A.f, t, px, py);
                edge_pt(B.c, B.f, flip ? N - 1 - t : t, qx, qy);
                if (std::hypot(px - qx, py - qy) > tol) throw std::runtime_error("non-conforming side faces");
            }
            if (L.cnbr[A.c * 4 + A.f] >= 0 || L.cnbr[B.c * 4 + B.f] >= 0)
                throw std::runtime_error("face matched twice");
            L.cnbr[A.c * 4 + A.f] = B.c;
            L.cnf[A.c * 4 + A.f] = B.f | (flip << 2);
            L.cnbr[B.c * 4 + B.f] = A.c;
            L.cnf[B.c * 4 + B.f] = A.f | (flip << 2);
        }
    }
    // An unmatched edge is a boundary edge.  Two unmatched edges with the same two
    // end points (a shared edge whose nodes differ), or an unmatched edge whose
    // end point lies inside another (a hanging node), would be a crack between
    // columns: reject those meshes instead of treating them as free boundaries.
    {
        std::vector<int> open;
        for (int k = 0; k < L.n_cols * 4; ++k)
            if (L.cnbr[k] < 0) open.push_back(k);
        auto end_pts = [&](int k, double p[2][2]) {
            edge_pt(k / 4, k % 4, 0, p[0][0], p[0][1]);
            edge_pt(k / 4, k % 4, N - 1, p[1][0], p[1][1]);
        };
        auto near = [&](const double* a, const double* b) { return std::hypot(a[0] - b[0], a[1] - b[1]) <= tol; };
        for (size_t a = 0; a < open.size(); ++a) {
            double pa[2][2];
            end_pts(open[a], pa);
            for (size_t b = 0; b < open.size(); ++b) {
                if (a == b) continue;
                double pb[2][2];
                end_pts(open[b], pb);
                if ((near(pa[0], pb[0]) && near(pa[1], pb[1])) || (near(pa[0], pb[1]) && near(pa[1], pb[0])))
                    throw std::runtime_error("non-conforming side faces (a shared edge whose nodes differ)");
                // end points of a strictly inside the polyline of b's edge nodes
                for (int s = 0; s < 2; ++s) {
                    if (near(pa[s], pb[0]) || near(pa[s], pb[1])) continue;
                    for (int t = 0; t + 1 < N; ++t) {
                        double x0, y0, x1, y1;
                        edge_pt(open[b] / 4, open[b] % 4, t, x0, y0);
                        edge_pt(open[b] / 4, open[b] % 4, t + 1, x1, y1);
                        const double dx = x1 - x0, dy = y1 - y0, l2 = dx * dx + dy * dy;
                        if (!(l2 > 0)) continue;
                        const double u = ((pa[s][0] - x0) * dx + (pa[s][1] - y0) * dy) / l2;
                        if (u < 0 || u > 1) continue;
                        // the polyline is a chord of a curved edge: allow its sagitta
                        const double d = std::hypot(x0 + u * dx - pa[s][0], y0 + u * dy - pa[s][1]);
                        if (d <= tol + 0.05 * std::sqrt(l2))
                            throw std::runtime_error("non-conforming side faces (a hanging node)");
                    }
                }
            }
        }
    }
    for (int k = 0; k < L.n_cols * 4; ++k)
        if (L.cnbr[k] < 0) L.cnf[k] = P.bc_side;

    // side-face penalty, eq. penalty: C (p + 1)^2 / min(h_int, h_ext), h = 2 / |grad xi^m|
    auto width = [&](int c, int f, int t) {
        int i, j;
        side_node(f, t, N, i, j);
        const double* g = &L.geo2[(size_t)c * 5 * N2];
        const int q = j * N + i;
        const int m = (f < 2) ? 0 : 2;
        return 2.0 / std::hypot(g[m * N2 + q], g[(m + 1) * N2 + q]);
    };
    // outward unit normals of the side faces and |grad xi^m| there (z-independent)
    L.fnrm.assign((size_t)L.n_cols * 4 * 3 * N, 0.0);
    for (int c = 0; c < L.n_cols; ++c)
        for (int f = 0; f < 4; ++f)
            for (int t = 0; t < N; ++t) {
                int i, j;
                side_node(f, t, N, i, j);
                const double* g = &L.geo2[(size_t)c * 5 * N2];
                const int q = j * N + i, m = (f < 2) ? 0 : 2;
                const double ax = g[m * N2 + q], ay = g[(m + 1) * N2 + q], a = std::hypot(ax, ay);
                const double s = (f & 1) ? 1.0 : -1.0;
                double* o = &L.fnrm[((size_t)c * 4 + f) * 3 * N];
                o[t] = s * ax / a;
                o[N + t] = s * ay / a;
                o[2 * N + t] = a;
            }
    L.sig_side.assign((size_t)L.n_cols * 4 * N, 0.0);
    const double cn2 = L.pen_z * double(1 << (r0 - refine));
    for (int c = 0; c < L.n_cols; ++c)
        for (int f = 0; f < 4; ++f)
            for (int t = 0; t < N; ++t) {
                double h = width(c, f, t);
                const int nb = L.cnbr[c * 4 + f];
                if (nb >= 0) {
                    const int code = L.cnf[c * 4 + f];
                    const int tt = (code >> 2) ? N - 1 - t : t;
                    h = std::min(h, width(nb, code & 3, tt));
                }
                L.sig_side[((size_t)c * 4 + f) * N + t] = cn2 / h;
            }
    return L;
}

}  // namespace dgtn
