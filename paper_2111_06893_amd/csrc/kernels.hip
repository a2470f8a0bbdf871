// gfx950 kernels of the DG elasticity operator (Sec. 2.2.2 - 2.2.4).
//
// One workgroup per element, one lane per LGL node (N^3 lanes rounded up to
// whole 64-wide waves).  The element's displacement is staged in LDS, the
// reference derivatives are LGL contractions along the three tensor
// directions, and everything pointwise (metric, lift, constitutive relation,
// fluxes) stays in registers.  FP64 and FP32 are the same template.
//
// The operator is applied in two passes:
//   k_traction  t = n . Y . D u on the 6 N^2 face nodes of every element (the
//               unlifted derivative entering the flux of eq. numflux);
//   k_apply     lifted strain, stress, weak divergence and face fluxes, which
//               read the neighbours' displacement traces and tractions.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace dgtn {

namespace {

template <int N>
constexpr int threads_for() {
    return ((N * N * N + 63) / 64) * 64;
}

// Symmetric tensors are held as (xx, yy, zz, xy, xz, yz).
template <typename R>
__device__ __forceinline__ void cubic_stress(R c11, R c12, R c44, const R S[6], R T[6]) {
    T[0] = c11 * S[0] + c12 * (S[1] + S[2]);
    T[1] = c11 * S[1] + c12 * (S[0] + S[2]);
    T[2] = c11 * S[2] + c12 * (S[0] + S[1]);
    T[3] = R(2) * c44 * S[3];
    T[4] = R(2) * c44 * S[4];
    T[5] = R(2) * c44 * S[5];
}

template <typename R>
__device__ __forceinline__ void traction(const R n[3], const R T[6], R t[3]) {
    t[0] = n[0] * T[0] + n[1] * T[3] + n[2] * T[4];
    t[1] = n[0] * T[3] + n[1] * T[1] + n[2] * T[5];
    t[2] = n[0] * T[4] + n[1] * T[5] + n[2] * T[2];
}

// sym(n (x) v)
template <typename R>
__device__ __forceinline__ void sym_outer(const R n[3], const R v[3], R S[6]) {
    S[0] = n[0] * v[0];
    S[1] = n[1] * v[1];
    S[2] = n[2] * v[2];
    S[3] = R(0.5) * (n[0] * v[1] + n[1] * v[0]);
    S[4] = R(0.5) * (n[0] * v[2] + n[2] * v[0]);
    S[5] = R(0.5) * (n[1] * v[2] + n[2] * v[1]);
}

// Per-node geometry of an extruded element.
template <typename R>
struct NodeGeo {
    R axx, axy, aex, aey;  // dxi/dx, dxi/dy, deta/dx, deta/dy
    R det2, hz;
};

// Gradient G[d][l] = D_d u_l at node (i, j, k) from the LDS copy of u.
template <int N, typename R>
__device__ __forceinline__ void gradient(const R* su, const R* sD, int i, int j, int k,
                                         const NodeGeo<R>& g, R G[3][3]) {
    constexpr int N2 = N * N, N3 = N2 * N;
    const R dz = R(2) / g.hz;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        R dxi = 0, deta = 0, dzeta = 0;
        const R* ul = su + l * N3;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            dxi += sD[i * N + a] * ul[k * N2 + j * N + a];
            deta += sD[j * N + a] * ul[k * N2 + a * N + i];
            dzeta += sD[k * N + a] * ul[a * N2 + j * N + i];
        }
        G[0][l] = g.axx * dxi + g.aex * deta;
        G[1][l] = g.axy * dxi + g.aey * deta;
        G[2][l] = dz * dzeta;
    }
}

template <typename R>
__device__ __forceinline__ void sym_of(const R G[3][3], R S[6]) {
    S[0] = G[0][0];
    S[1] = G[1][1];
    S[2] = G[2][2];
    S[3] = R(0.5) * (G[0][1] + G[1][0]);
    S[4] = R(0.5) * (G[0][2] + G[2][0]);
    S[5] = R(0.5) * (G[1][2] + G[2][1]);
}

// Outward unit normal of face f at a node, and |grad xi^m| for side faces.
template <typename R>
__device__ __forceinline__ void face_normal(int f, const NodeGeo<R>& g, R n[3], R& amag) {
    if (f < 4) {
        const R ax = (f < 2) ? g.axx : g.aex;
        const R ay = (f < 2) ? g.axy : g.aey;
        amag = sqrt(ax * ax + ay * ay);
        const R s = (f & 1) ? R(1) : R(-1);
        n[0] = s * ax / amag;
        n[1] = s * ay / amag;
        n[2] = 0;
    } else {
        amag = 0;
        n[0] = 0;
        n[1] = 0;
        n[2] = (f == 5) ? R(1) : R(-1);
    }
}

// Flattened index of node (i, j, k) within face f (the face-buffer order).
template <int N>
__device__ __forceinline__ int face_index(int f, int i, int j, int k) {
    return (f < 2) ? k * N + j : (f < 4) ? k * N + i : j * N + i;
}

struct Nbr {
    int e, f, flip, bc;  // bc != 0 on boundary faces
};

template <typename R>
__device__ __forceinline__ Nbr neighbour(const LevelView<R>& L, int col, int iz, int f) {
    Nbr r{-1, -1, 0, 0};
    if (f < 4) {
        const int nc = L.cnbr[col * 4 + f];
        const int code = L.cnf[col * 4 + f];
        if (nc < 0) {
            r.bc = code;
        } else {
            r.e = iz * L.n_cols + nc;
            r.f = code & 3;
            r.flip = code >> 2;
        }
    } else if (f == 4) {
        if (iz == 0) r.bc = L.bc_top;
        else { r.e = (iz - 1) * L.n_cols + col; r.f = 5; }
    } else {
        if (iz == L.n_z - 1) r.bc = L.bc_bottom;
        else { r.e = (iz + 1) * L.n_cols + col; r.f = 4; }
    }
    return r;
}

// Node of the neighbour matching node (i, j, k) across face f.
template <int N>
__device__ __forceinline__ void matching_node(int f, const Nbr& nb, int i, int j, int k,
                                              int& i2, int& j2, int& k2) {
    if (f >= 4) {
        i2 = i;
        j2 = j;
        k2 = (f == 4) ? N - 1 : 0;
        return;
    }
    int t = (f < 2) ? j : i;
    if (nb.flip) t = N - 1 - t;
    k2 = k;
    switch (nb.f) {
        case 0: i2 = 0; j2 = t; break;
        case 1: i2 = N - 1; j2 = t; break;
        case 2: i2 = t; j2 = 0; break;
        default: i2 = t; j2 = N - 1; break;
    }
}

template <int N, typename R>
__device__ __forceinline__ NodeGeo<R> node_geo(const LevelView<R>& L, int col, int iz, int i, int j) {
    constexpr int N2 = N * N;
    const R* g = L.geo2 + (size_t)col * 5 * N2 + j * N + i;
    NodeGeo<R> r;
    r.axx = g[0];
    r.axy = g[N2];
    r.aex = g[2 * N2];
    r.aey = g[3 * N2];
    r.det2 = g[4 * N2];
    r.hz = L.hz[iz];
    return r;
}

template <int N, typename R>
__global__ __launch_bounds__(threads_for<N>()) void k_traction(LevelView<R> L, const R* __restrict__ u,
                                                              R* __restrict__ tau) {
    constexpr int N2 = N * N, N3 = N2 * N;
    __shared__ R su[3 * N3];
    __shared__ R sD[N2];
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    const R* ue = u + (size_t)e * 3 * N3;
    for (int q = tid; q < 3 * N3; q += blockDim.x) su[q] = ue[q];
    for (int q = tid; q < N2; q += blockDim.x) sD[q] = L.D[q];
    __syncthreads();
    if (tid >= N3) return;
    const int i = tid % N, j = (tid / N) % N, k = tid / N2;
    const bool fi = (i == 0) | (i == N - 1), fj = (j == 0) | (j == N - 1), fk = (k == 0) | (k == N - 1);
    if (!(fi | fj | fk)) return;
    const int col = e % L.n_cols, iz = e / L.n_cols;
    const NodeGeo<R> g = node_geo<N>(L, col, iz, i, j);
    R G[3][3], S[6], T[6];
    gradient<N>(su, sD, i, j, k, g, G);
    sym_of(G, S);
    const int m = L.zmat[iz];
    cubic_stress(L.mat[3 * m], L.mat[3 * m + 1], L.mat[3 * m + 2], S, T);
    const int faces[3] = {fi ? (i == 0 ? 0 : 1) : -1, fj ? (j == 0 ? 2 : 3) : -1, fk ? (k == 0 ? 4 : 5) : -1};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int f = faces[q];
        if (f < 0) continue;
        R n[3], amag, t[3];
        face_normal(f, g, n, amag);
        traction(n, T, t);
        R* dst = tau + ((size_t)e * 6 + f) * 3 * N2 + face_index<N>(f, i, j, k);
        dst[0] = t[0];
        dst[N2] = t[1];
        dst[2 * N2] = t[2];
    }
}

template <int N, typename R>
__global__ __launch_bounds__(threads_for<N>()) void k_apply(LevelView<R> L, const R* __restrict__ u,
                                                           const R* __restrict__ tau, R* __restrict__ out,
                                                           R scale) {
    constexpr int N2 = N * N, N3 = N2 * N;
    __shared__ R su[3 * N3];
    __shared__ R sF[9 * N3];
    __shared__ R sD[N2];
    __shared__ R sw[N];
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    const R* ue = u + (size_t)e * 3 * N3;
    for (int q = tid; q < 3 * N3; q += blockDim.x) su[q] = ue[q];
    for (int q = tid; q < N2; q += blockDim.x) sD[q] = L.D[q];
    for (int q = tid; q < N; q += blockDim.x) sw[q] = L.w[q];
    __syncthreads();
    const bool active = tid < N3;
    const int i = tid % N, j = (tid / N) % N, k = tid / N2;
    R facc[3] = {0, 0, 0};
    if (active) {
        const int col = e % L.n_cols, iz = e / L.n_cols;
        const NodeGeo<R> g = node_geo<N>(L, col, iz, i, j);
        R G[3][3], S[6], T[6];
        gradient<N>(su, sD, i, j, k, g, G);
        sym_of(G, S);
        const int m = L.zmat[iz];
        const R c11 = L.mat[3 * m], c12 = L.mat[3 * m + 1], c44 = L.mat[3 * m + 2];
        R Tint[6];
        cubic_stress(c11, c12, c44, S, Tint);
        const bool fi = (i == 0) | (i == N - 1), fj = (j == 0) | (j == N - 1), fk = (k == 0) | (k == N - 1);
        const int faces[3] = {fi ? (i == 0 ? 0 : 1) : -1, fj ? (j == 0 ? 2 : 3) : -1, fk ? (k == 0 ? 4 : 5) : -1};
        R lift[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int f = faces[q];
            if (f < 0) continue;
            R n[3], amag;
            face_normal(f, g, n, amag);
            // w_face J^Sigma and the lift factor w_face J^Sigma / (w J)
            R wsig, lr;
            if (f >= 4) {
                wsig = sw[i] * sw[j] * g.det2;
                lr = R(2) / (sw[k] * g.hz);
            } else if (f < 2) {
                wsig = sw[j] * sw[k] * R(0.5) * g.hz * g.det2 * amag;
                lr = amag / sw[i];
            } else {
                wsig = sw[i] * sw[k] * R(0.5) * g.hz * g.det2 * amag;
                lr = amag / sw[j];
            }
            R tint[3];
            traction(n, Tint, tint);
            const Nbr nb = neighbour(L, col, iz, f);
            R jump[3] = {0, 0, 0}, flux[3] = {0, 0, 0};
            const R* uo = su;  // own values at this node
            const int qn = k * N2 + j * N + i;
            if (nb.bc == 0) {
                int i2, j2, k2;
                matching_node<N>(f, nb, i, j, k, i2, j2, k2);
                const R* un = u + (size_t)nb.e * 3 * N3 + k2 * N2 + j2 * N + i2;
                const R* tn = tau + ((size_t)nb.e * 6 + nb.f) * 3 * N2 + face_index<N>(nb.f, i2, j2, k2);
                const int izn = nb.e / L.n_cols;
                const int mn = L.zmat[izn];
                R sigma;
                if (f < 4) {
                    const int t = (f < 2) ? j : i;
                    sigma = L.sig_side[((size_t)col * 4 + f) * N + t];
                } else {
                    sigma = L.penalty_n2 / min(g.hz, L.hz[izn]);
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) jump[c] = uo[c * N3 + qn] - un[c * N3];
                R Sj[6], Tj[6], pen[3];
                sym_outer(n, jump, Sj);
                cubic_stress(R(0.5) * (c11 + L.mat[3 * mn]), R(0.5) * (c12 + L.mat[3 * mn + 1]),
                             R(0.5) * (c44 + L.mat[3 * mn + 2]), Sj, Tj);
                traction(n, Tj, pen);
#pragma unroll
                for (int c = 0; c < 3; ++c) flux[c] = R(0.5) * (tint[c] - tn[c * N2]) - sigma * pen[c];
            } else if (nb.bc == DGTN_BC_DIRICHLET) {
                R sigma;
                if (f < 4) {
                    const int t = (f < 2) ? j : i;
                    sigma = L.sig_side[((size_t)col * 4 + f) * N + t];
                } else {
                    sigma = L.penalty_n2 / g.hz;
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) jump[c] = R(2) * uo[c * N3 + qn];
                R Sj[6], Tj[6], pen[3];
                sym_outer(n, jump, Sj);
                cubic_stress(c11, c12, c44, Sj, Tj);
                traction(n, Tj, pen);
#pragma unroll
                for (int c = 0; c < 3; ++c) flux[c] = tint[c] - sigma * pen[c];
            }
            // Neumann faces: no jump and, for homogeneous data, no flux
            R Sj[6];
            sym_outer(n, jump, Sj);
#pragma unroll
            for (int s = 0; s < 6; ++s) lift[s] -= R(0.5) * lr * Sj[s];
#pragma unroll
            for (int c = 0; c < 3; ++c) facc[c] -= wsig * flux[c];
        }
#pragma unroll
        for (int s = 0; s < 6; ++s) S[s] += lift[s];
        cubic_stress(c11, c12, c44, S, T);
        const R wJ = sw[i] * sw[j] * sw[k] * g.det2 * R(0.5) * g.hz;
        const R dz = R(2) / g.hz;
        // F^m_c = w J (J^-1)^m_d T^{dc}
        const R Tx[3] = {T[0], T[3], T[4]};
        const R Ty[3] = {T[3], T[1], T[5]};
        const R Tz[3] = {T[4], T[5], T[2]};
        const int qn = k * N2 + j * N + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sF[(0 + c) * N3 + qn] = wJ * (g.axx * Tx[c] + g.axy * Ty[c]);
            sF[(3 + c) * N3 + qn] = wJ * (g.aex * Tx[c] + g.aey * Ty[c]);
            sF[(6 + c) * N3 + qn] = wJ * dz * Tz[c];
        }
    }
    __syncthreads();
    if (!active) return;
    R* oe = out + (size_t)e * 3 * N3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        R r = 0;
        const R* Fx = sF + (0 + c) * N3;
        const R* Fy = sF + (3 + c) * N3;
        const R* Fz = sF + (6 + c) * N3;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            r += sD[a * N + i] * Fx[k * N2 + j * N + a];
            r += sD[a * N + j] * Fy[k * N2 + a * N + i];
            r += sD[a * N + k] * Fz[a * N2 + j * N + i];
        }
        oe[c * N3 + tid] = scale * (r + facc[c]);
    }
}

// Load vector of the Gaussian pressure on DGTN_BC_PRESSURE faces:
// b = -w_face J^Sigma n p(r), which is +z on the loaded face z = 0.
template <int N>
__global__ __launch_bounds__(threads_for<N>()) void k_rhs(LevelView<double> L, const double* __restrict__ xy,
                                                         double F0, double r0, double xc, double yc,
                                                         double* __restrict__ b) {
    constexpr int N2 = N * N, N3 = N2 * N;
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid >= N3) return;
    const int i = tid % N, j = (tid / N) % N, k = tid / N2;
    const int col = e % L.n_cols, iz = e / L.n_cols;
    const NodeGeo<double> g = node_geo<N>(L, col, iz, i, j);
    double acc[3] = {0, 0, 0};
    const bool fi = (i == 0) | (i == N - 1), fj = (j == 0) | (j == N - 1), fk = (k == 0) | (k == N - 1);
    const int faces[3] = {fi ? (i == 0 ? 0 : 1) : -1, fj ? (j == 0 ? 2 : 3) : -1, fk ? (k == 0 ? 4 : 5) : -1};
    const double x = xy[(size_t)col * 2 * N2 + j * N + i] - xc;
    const double y = xy[(size_t)col * 2 * N2 + N2 + j * N + i] - yc;
    const double p = F0 * exp(-(x * x + y * y) / (r0 * r0)) / (M_PI * r0 * r0);
    for (int q = 0; q < 3; ++q) {
        const int f = faces[q];
        if (f < 0) continue;
        const Nbr nb = neighbour(L, col, iz, f);
        if (nb.bc != DGTN_BC_PRESSURE) continue;
        double n[3], amag, wsig;
        face_normal(f, g, n, amag);
        if (f >= 4) wsig = L.w[i] * L.w[j] * g.det2;
        else if (f < 2) wsig = L.w[j] * L.w[k] * 0.5 * g.hz * g.det2 * amag;
        else wsig = L.w[i] * L.w[k] * 0.5 * g.hz * g.det2 * amag;
        for (int c = 0; c < 3; ++c) acc[c] -= wsig * n[c] * p;
    }
    double* be = b + (size_t)e * 3 * N3;
    for (int c = 0; c < 3; ++c) be[c * N3 + tid] = acc[c];
}

// Per-element energy 1/2 sum_nodes w J D_(i u_j) Y D_(k u_l), in units of y_ref.
template <int N>
__global__ __launch_bounds__(threads_for<N>()) void k_energy(LevelView<double> L, const double* __restrict__ u,
                                                            double* __restrict__ Ue) {
    constexpr int N2 = N * N, N3 = N2 * N, NT = threads_for<N>();
    __shared__ double su[3 * N3];
    __shared__ double sD[N2];
    __shared__ double red[NT];
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    const double* ue = u + (size_t)e * 3 * N3;
    for (int q = tid; q < 3 * N3; q += blockDim.x) su[q] = ue[q];
    for (int q = tid; q < N2; q += blockDim.x) sD[q] = L.D[q];
    __syncthreads();
    double dens = 0;
    if (tid < N3) {
        const int i = tid % N, j = (tid / N) % N, k = tid / N2;
        const int col = e % L.n_cols, iz = e / L.n_cols;
        const NodeGeo<double> g = node_geo<N>(L, col, iz, i, j);
        double G[3][3], S[6], T[6];
        gradient<N>(su, sD, i, j, k, g, G);
        sym_of(G, S);
        const int m = L.zmat[iz];
        cubic_stress(L.mat[3 * m], L.mat[3 * m + 1], L.mat[3 * m + 2], S, T);
        const double sdt = S[0] * T[0] + S[1] * T[1] + S[2] * T[2] +
                           2.0 * (S[3] * T[3] + S[4] * T[4] + S[5] * T[5]);
        dens = 0.5 * L.w[i] * L.w[j] * L.w[k] * g.det2 * 0.5 * g.hz * sdt;
    }
    red[tid] = dens;
    __syncthreads();
    // fixed-order reduction (deterministic): strided sums into 64 slots, then a tree
    if (tid < 64) {
        double acc = 0;
        for (int q = tid; q < NT; q += 64) acc += red[q];
        red[tid] = acc;
    }
    __syncthreads();
    for (int s = 32; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) Ue[e] = red[0];
}

}  // namespace

template <typename F>
hipError_t dispatch_n(int N, F&& f) {
    switch (N) {
        case 2: return f(std::integral_constant<int, 2>{});
        case 3: return f(std::integral_constant<int, 3>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 5: return f(std::integral_constant<int, 5>{});
        case 6: return f(std::integral_constant<int, 6>{});
        case 7: return f(std::integral_constant<int, 7>{});
        case 8: return f(std::integral_constant<int, 8>{});
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_traction(const LevelView<R>& L, const R* u, R* tau, hipStream_t s) {
    return dispatch_n(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_traction<NN, R>), dim3(L.E), dim3(threads_for<NN>()), 0, s, L, u, tau);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t launch_apply(const LevelView<R>& L, const R* u, const R* tau, R* out, R scale, hipStream_t s) {
    return dispatch_n(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_apply<NN, R>), dim3(L.E), dim3(threads_for<NN>()), 0, s, L, u, tau, out, scale);
        return hipGetLastError();
    });
}

hipError_t launch_rhs(const LevelView<double>& L, const double* xy, double F0, double r0, double xc, double yc,
                      double* b, hipStream_t s) {
    return dispatch_n(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_rhs<NN>), dim3(L.E), dim3(threads_for<NN>()), 0, s, L, xy, F0, r0, xc, yc, b);
        return hipGetLastError();
    });
}

hipError_t launch_energy(const LevelView<double>& L, const double* u, double* Ue, hipStream_t s) {
    return dispatch_n(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_energy<NN>), dim3(L.E), dim3(threads_for<NN>()), 0, s, L, u, Ue);
        return hipGetLastError();
    });
}

template hipError_t launch_traction<double>(const LevelView<double>&, const double*, double*, hipStream_t);
template hipError_t launch_traction<float>(const LevelView<float>&, const float*, float*, hipStream_t);
template hipError_t launch_apply<double>(const LevelView<double>&, const double*, const double*, double*, double,
                                         hipStream_t);
template hipError_t launch_apply<float>(const LevelView<float>&, const float*, const float*, float*, float,
                                        hipStream_t);

}  // namespace dgtn
