// gfx950 kernels of the DG elasticity operator (Sec. 2.2.2 - 2.2.4).
//
// One workgroup per element.  The element's displacement is staged in LDS and
// the work alternates between three lane roles separated by barriers: line
// lanes (one per line of N nodes along xi, eta or zeta and per component) do
// the sum-factorised LGL contractions, reading each input once from LDS with
// the 1D matrix D in scalar registers; node lanes (one per LGL node) do the
// pointwise metric, lift and constitutive work; face lanes (one per face node)
// do the jumps and numerical fluxes.  FP64, FP32 and the dual numbers of the
// adjoint are the same template.
//
// The operator is applied in two passes:
//   k_traction  t = n . Y . D u on the 6 N^2 face nodes of every element (the
//               unlifted derivative entering the flux of eq. numflux);
//   k_apply     lifted strain, stress, weak divergence and face fluxes, which
//               read the neighbours' displacement traces and tractions.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dual.h"
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
#pragma unroll 1
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

// Workgroups are dispatched round-robin over the eight XCDs; map them so that
// each XCD processes one contiguous range of elements, whose face neighbours
// (the next column and the next z-layer) then mostly sit in the same L2.
__device__ __forceinline__ int xcd_element(int bid, int E) {
    const int q = E / 8, rem = E % 8;
    const int x = bid % 8, r = bid / 8;
    return x * q + min(x, rem) + r;
}

// Per-face data of one element, resolved once per workgroup into LDS.
template <typename R>
struct FaceInfo {
    int e, f, flip, bc;   // neighbour element, its face, orientation; bc != 0 on boundaries
    R c11, c12, c44;      // averaged moduli on the face (own on boundaries)
    R hz;                 // neighbour thickness (own on boundaries)
};

template <int N, typename R>
__device__ __forceinline__ void load_faces(const LevelView<R>& L, int col, int iz, int tid, FaceInfo<R>* sf,
                                           R* sown) {
    if (tid < 6) {
        const Nbr nb = neighbour(L, col, iz, tid);
        FaceInfo<R> fi;
        fi.e = nb.e;
        fi.f = nb.f;
        fi.flip = nb.flip;
        fi.bc = nb.bc;
        const int m = L.zmat[iz];
        const int mn = nb.bc == 0 ? L.zmat[nb.e / L.n_cols] : m;
        fi.c11 = R(0.5) * (L.mat[3 * m] + L.mat[3 * mn]);
        fi.c12 = R(0.5) * (L.mat[3 * m + 1] + L.mat[3 * mn + 1]);
        fi.c44 = R(0.5) * (L.mat[3 * m + 2] + L.mat[3 * mn + 2]);
        fi.hz = nb.bc == 0 ? L.hz[nb.e / L.n_cols] : L.hz[iz];
        sf[tid] = fi;
    } else if (tid == 6) {
        const int m = L.zmat[iz];
        sown[0] = L.mat[3 * m];
        sown[1] = L.mat[3 * m + 1];
        sown[2] = L.mat[3 * m + 2];
        sown[3] = L.hz[iz];
    }
}

// Node (i, j, k) of face node fi on face f (the face-buffer order).
template <int N>
__device__ __forceinline__ void face_node(int f, int fi, int& i, int& j, int& k) {
    const int a = fi % N, b = fi / N;
    const int s = (f & 1) ? N - 1 : 0;
    if (f < 2) { i = s; j = a; k = b; }
    else if (f < 4) { i = a; j = s; k = b; }
    else { i = a; j = b; k = s; }
}

// Lanes of the operator kernels: 9 N^2 line tasks (3 directions x 3 components
// x N^2 lines), N^3 nodes, 6 N^2 face nodes, rounded up to whole waves.
template <int N>
constexpr int line_threads() {
    constexpr int a = 9 * N * N, b = N * N * N, c = 6 * N * N;
    constexpr int m = a > b ? (a > c ? a : c) : (b > c ? b : c);
    return ((m + 63) / 64) * 64;
}

// Line task t < 9 N^2: direction d (xi, eta, zeta), component c, and the offset
// and stride of the line's N nodes within one component's N^3 block.
template <int N>
__device__ __forceinline__ void line_of(int t, int& d, int& c, int& base, int& stride) {
    constexpr int N2 = N * N;
    d = t / (3 * N2);
    const int rem = t % (3 * N2);
    c = rem / N2;
    const int q = rem % N2, q1 = q % N, q2 = q / N;
    base = d == 0 ? q2 * N2 + q1 * N : d == 1 ? q2 * N2 + q1 : q2 * N + q1;
    stride = d == 0 ? 1 : d == 1 ? N : N2;
}

// Sum-factorised 1D contraction along one line, one lane per line: the N
// inputs are read from LDS once, D comes from the kernel arguments (uniform
// across the wave, so it sits in scalar registers).
//   transpose = false: dst[x] = sum_a D[x][a] src[a]   (derivative)
//   transpose = true:  dst[x] = sum_a D[a][x] src[a]   (weak divergence)
// emit(x, value) consumes output x.
template <int N, bool transpose, typename R, typename Emit>
__device__ __forceinline__ void line_contract(const LevelView<R>& L, const R* src, int base, int stride, Emit&& emit) {
    R v[N];
#pragma unroll
    for (int a = 0; a < N; ++a) v[a] = src[base + a * stride];
    // one row of D (or D^T) per output, loaded as the loop reaches it: the
    // whole matrix would not fit the scalar register file
#pragma unroll 1
    for (int x = 0; x < N; ++x) {
        const R* row = (transpose ? L.Dt : L.Dk) + x * N;
        R acc = 0;
#pragma unroll
        for (int a = 0; a < N; ++a) acc += row[a] * v[a];
        emit(x, acc);
    }
}

// Reference derivatives of the three components along the three directions,
// sG[(d * 3 + c) * N^3 + node], from the LDS copy of u.
template <int N, typename R>
__device__ __forceinline__ void ref_derivatives(const LevelView<R>& L, const R* su, R* sG, int tid) {
    constexpr int N3 = N * N * N;
    if (tid < 9 * N * N) {
        int d, c, base, stride;
        line_of<N>(tid, d, c, base, stride);
        R* dst = sG + (d * 3 + c) * N3 + base;
        line_contract<N, false>(L, su + c * N3, base, stride, [&](int x, R v) { dst[x * stride] = v; });
    }
}

// Physical gradient G[d][l] = D_d u_l at node q from the reference derivatives.
template <int N, typename R>
__device__ __forceinline__ void node_gradient(const R* sG, int q, const NodeGeo<R>& g, R G[3][3]) {
    constexpr int N3 = N * N * N;
    const R dz = R(2) / g.hz;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const R dxi = sG[l * N3 + q], deta = sG[(3 + l) * N3 + q], dzeta = sG[(6 + l) * N3 + q];
        G[0][l] = g.axx * dxi + g.aex * deta;
        G[1][l] = g.axy * dxi + g.aey * deta;
        G[2][l] = dz * dzeta;
    }
}

template <int N, typename R>
__global__ __launch_bounds__(line_threads<N>()) void k_traction(LevelView<R> L, const R* __restrict__ u,
                                                               R* __restrict__ tau) {
    constexpr int N2 = N * N, N3 = N2 * N;
    __shared__ R su[3 * N3];
    __shared__ R sG[9 * N3];
    __shared__ R sown[4];
    const int e = xcd_element(blockIdx.x, L.E);
    const int tid = threadIdx.x;
    const int col = e % L.n_cols, iz = e / L.n_cols;
    const R* ue = u + (size_t)e * 3 * N3;
    for (int q = tid; q < 3 * N3; q += blockDim.x) su[q] = ue[q];
    if (tid == 0) {
        const int m = L.zmat[iz];
        sown[0] = L.mat[3 * m];
        sown[1] = L.mat[3 * m + 1];
        sown[2] = L.mat[3 * m + 2];
        sown[3] = L.hz[iz];
    }
    const bool act = tid < 6 * N2;
    const int f = tid / N2, fi = tid % N2;
    int i = 0, j = 0, k = 0;
    if (act) face_node<N>(f, fi, i, j, k);
    NodeGeo<R> g = act ? node_geo<N>(L, col, iz, i, j) : NodeGeo<R>{1, 0, 0, 1, 1, 1};
    __syncthreads();
    ref_derivatives<N>(L, su, sG, tid);
    __syncthreads();
    if (!act) return;
    g.hz = sown[3];
    R G[3][3], S[6], T[6], n[3], amag, t[3];
    node_gradient<N>(sG, k * N2 + j * N + i, g, G);
    sym_of(G, S);
    cubic_stress(sown[0], sown[1], sown[2], S, T);
    face_normal(f, g, n, amag);
    traction(n, T, t);
    R* dst = tau + ((size_t)e * 6 + f) * 3 * N2 + fi;
    dst[0] = t[0];
    dst[N2] = t[1];
    dst[2 * N2] = t[2];
}

// Six waves per SIMD: with the LDS below that fits three workgroups per CU (FP64,
// N = 7) at the cost of a few spilled registers; measured faster than two.
template <int N, typename R>
__global__ __launch_bounds__(line_threads<N>(), 6) void k_apply(LevelView<R> L, const R* __restrict__ u,
                                                            const R* __restrict__ tau, R* __restrict__ out,
                                                            R scale) {
    constexpr int N2 = N * N, N3 = N2 * N;
    __shared__ R su[3 * N3];          // u
    __shared__ R sG[9 * N3];          // reference derivatives; later the volume fluxes F, then D^T F
    __shared__ R sFT[6 * 3 * N2];     // per face node: interior traction, then -w J^Sigma (n Y S)*
    __shared__ R sLF[6 * 3 * N2];     // per face node: lifting factor times the jump
    __shared__ R sw[N];
    __shared__ FaceInfo<R> sface[6];
    __shared__ R sown[4];
    const int e = xcd_element(blockIdx.x, L.E);
    const int tid = threadIdx.x;
    const int col = e % L.n_cols, iz = e / L.n_cols;
    const R* ue = u + (size_t)e * 3 * N3;
    for (int q = tid; q < 3 * N3; q += blockDim.x) su[q] = ue[q];
    for (int q = tid; q < N; q += blockDim.x) sw[q] = L.w[q];
    load_faces<N>(L, col, iz, tid, sface, sown);
    // node role
    const bool nact = tid < N3;
    const int i = tid % N, j = (tid / N) % N, k = tid / N2;
    NodeGeo<R> g = nact ? node_geo<N>(L, col, iz, i, j) : NodeGeo<R>{1, 0, 0, 1, 1, 1};
    // face role
    const bool fact = tid < 6 * N2;
    const int f = tid / N2, fi = tid % N2;
    int fi_i = 0, fi_j = 0, fi_k = 0;
    if (fact) face_node<N>(f, fi, fi_i, fi_j, fi_k);
    __syncthreads();
    g.hz = sown[3];
    // neighbour trace and traction of this face node: in flight during the derivatives
    R un[3] = {0, 0, 0}, tn[3] = {0, 0, 0};
    if (fact && sface[f].bc == 0) {
        const FaceInfo<R>& fo = sface[f];
        int i2, j2, k2;
        const Nbr nb{fo.e, fo.f, fo.flip, 0};
        matching_node<N>(f, nb, fi_i, fi_j, fi_k, i2, j2, k2);
        const R* up = u + (size_t)fo.e * 3 * N3 + k2 * N2 + j2 * N + i2;
        const R* tp = tau + ((size_t)fo.e * 6 + fo.f) * 3 * N2 + face_index<N>(fo.f, i2, j2, k2);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            un[c] = up[c * N3];
            tn[c] = tp[c * N2];
        }
    }
    const R c11 = sown[0], c12 = sown[1], c44 = sown[2];
    // 1. line lanes: reference derivatives of u
    ref_derivatives<N>(L, su, sG, tid);
    __syncthreads();
    // 2. node lanes: unlifted gradient and stress; interior traction on each face slot.
    // Only this lane reads its node's derivatives, so S is parked in those slots.
    const bool fxi = (i == 0) | (i == N - 1), feta = (j == 0) | (j == N - 1), fzeta = (k == 0) | (k == N - 1);
    if (nact) {
        R G[3][3], T[6], S[6];
        node_gradient<N>(sG, tid, g, G);
        sym_of(G, S);
#pragma unroll
        for (int q = 0; q < 6; ++q) sG[q * N3 + tid] = S[q];
        if (fxi | feta | fzeta) {
            cubic_stress(c11, c12, c44, S, T);
            const int faces[3] = {fxi ? (i == 0 ? 0 : 1) : -1, feta ? (j == 0 ? 2 : 3) : -1,
                                  fzeta ? (k == 0 ? 4 : 5) : -1};
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (faces[q] < 0) continue;
                R n[3], amag, t[3];
                face_normal(faces[q], g, n, amag);
                traction(n, T, t);
                const int slot = faces[q] * 3 * N2 + face_index<N>(faces[q], i, j, k);
                sFT[slot] = t[0];
                sFT[slot + N2] = t[1];
                sFT[slot + 2 * N2] = t[2];
            }
        }
    }
    __syncthreads();
    // 3. face lanes: jump, lift and numerical flux (eqs. numflux, penalty, bc)
    if (fact) {
        // face geometry loaded here rather than held through the earlier phases (register pressure)
        NodeGeo<R> gf = node_geo<N>(L, col, iz, fi_i, fi_j);
        gf.hz = sown[3];
        const R sig_side = f < 4 ? L.sig_side[((size_t)col * 4 + f) * N + (f < 2 ? fi_j : fi_i)] : R(0);
        const FaceInfo<R> fo = sface[f];
        R n[3], amag;
        face_normal(f, gf, n, amag);
        R wsig, lr;
        if (f >= 4) {
            wsig = sw[fi_i] * sw[fi_j] * gf.det2;
            lr = R(2) / (sw[fi_k] * gf.hz);
        } else if (f < 2) {
            wsig = sw[fi_j] * sw[fi_k] * R(0.5) * gf.hz * gf.det2 * amag;
            lr = amag / sw[fi_i];
        } else {
            wsig = sw[fi_i] * sw[fi_k] * R(0.5) * gf.hz * gf.det2 * amag;
            lr = amag / sw[fi_j];
        }
        const int qn = fi_k * N2 + fi_j * N + fi_i;
        const int slot = f * 3 * N2 + fi;
        R jump[3] = {0, 0, 0}, flux[3] = {0, 0, 0};
        if (fo.bc == 0 || fo.bc == DGTN_BC_DIRICHLET) {
            const bool interior = fo.bc == 0;
            const R sigma = (f < 4) ? sig_side : L.penalty_n2 / (interior ? min(gf.hz, fo.hz) : gf.hz);
#pragma unroll
            for (int c = 0; c < 3; ++c) jump[c] = interior ? su[c * N3 + qn] - un[c] : R(2) * su[c * N3 + qn];
            R Sj[6], Tj[6], pen[3];
            sym_outer(n, jump, Sj);
            cubic_stress(fo.c11, fo.c12, fo.c44, Sj, Tj);
            traction(n, Tj, pen);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const R tint = sFT[slot + c * N2];
                flux[c] = (interior ? R(0.5) * (tint - tn[c]) : tint) - sigma * pen[c];
            }
        }
        // Neumann faces: no jump and, for homogeneous data, no flux
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sLF[slot + c * N2] = R(-0.5) * lr * jump[c];
            sFT[slot + c * N2] = -wsig * flux[c];
        }
    }
    __syncthreads();
    // 4. node lanes: lifted strain, stress and the volume fluxes F^m_c = w J (J^-1)^m_d T^{dc}
    if (nact) {
        R S[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) S[q] = sG[q * N3 + tid];
        const int faces[3] = {fxi ? (i == 0 ? 0 : 1) : -1, feta ? (j == 0 ? 2 : 3) : -1,
                              fzeta ? (k == 0 ? 4 : 5) : -1};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (faces[q] < 0) continue;
            const int slot = faces[q] * 3 * N2 + face_index<N>(faces[q], i, j, k);
            R n[3], amag, lj[3], Sl[6];
            face_normal(faces[q], g, n, amag);
#pragma unroll
            for (int c = 0; c < 3; ++c) lj[c] = sLF[slot + c * N2];
            sym_outer(n, lj, Sl);
#pragma unroll
            for (int s = 0; s < 6; ++s) S[s] += Sl[s];
        }
        R T[6];
        cubic_stress(c11, c12, c44, S, T);
        const R wJ = sw[i] * sw[j] * sw[k] * g.det2 * R(0.5) * g.hz;
        const R dz = R(2) / g.hz;
        const R Tx[3] = {T[0], T[3], T[4]};
        const R Ty[3] = {T[3], T[1], T[5]};
        const R Tz[3] = {T[4], T[5], T[2]};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sG[c * N3 + tid] = wJ * (g.axx * Tx[c] + g.axy * Ty[c]);
            sG[(3 + c) * N3 + tid] = wJ * (g.aex * Tx[c] + g.aey * Ty[c]);
            sG[(6 + c) * N3 + tid] = wJ * dz * Tz[c];
        }
    }
    __syncthreads();
    // 5. weak divergence sum_m D_m^T F^m, one lane per line: F^m_c along a line is
    // read by that line's lane only, so each lane overwrites its line in place
    if (tid < 9 * N2) {
        int d, c, base, stride;
        line_of<N>(tid, d, c, base, stride);
        R* line = sG + (d * 3 + c) * N3 + base;
        R v[N];
#pragma unroll
        for (int a = 0; a < N; ++a) v[a] = line[a * stride];
#pragma unroll 1
        for (int x = 0; x < N; ++x) {
            const R* row = L.Dt + x * N;
            R acc = 0;
#pragma unroll
            for (int a = 0; a < N; ++a) acc += row[a] * v[a];
            line[x * stride] = acc;
        }
    }
    __syncthreads();
    // 6. node lanes: sum of the three directions and the face fluxes, written as A u
    if (nact) {
        const int faces[3] = {fxi ? (i == 0 ? 0 : 1) : -1, feta ? (j == 0 ? 2 : 3) : -1,
                              fzeta ? (k == 0 ? 4 : 5) : -1};
        R* oe = out + (size_t)e * 3 * N3 + tid;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            R r = sG[c * N3 + tid] + sG[(3 + c) * N3 + tid] + sG[(6 + c) * N3 + tid];
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (faces[q] >= 0) r += sFT[faces[q] * 3 * N2 + c * N2 + face_index<N>(faces[q], i, j, k)];
            oe[c * N3] = scale * r;
        }
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
// Arithmetic type R (double, or Dual for its derivative along a parameter).
template <int N, typename R>
__global__ __launch_bounds__(threads_for<N>()) void k_energy(LevelView<R> L, const double* __restrict__ u,
                                                            R* __restrict__ Ue) {
    constexpr int N2 = N * N, N3 = N2 * N, NT = threads_for<N>();
    __shared__ R su[3 * N3];
    __shared__ R sD[N2];
    __shared__ R red[NT];
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    const double* ue = u + (size_t)e * 3 * N3;
    for (int q = tid; q < 3 * N3; q += blockDim.x) su[q] = R(ue[q]);
    for (int q = tid; q < N2; q += blockDim.x) sD[q] = L.D[q];
    __syncthreads();
    R dens = 0;
    if (tid < N3) {
        const int i = tid % N, j = (tid / N) % N, k = tid / N2;
        const int col = e % L.n_cols, iz = e / L.n_cols;
        const NodeGeo<R> g = node_geo<N>(L, col, iz, i, j);
        R G[3][3], S[6], T[6];
        gradient<N>(su, sD, i, j, k, g, G);
        sym_of(G, S);
        const int m = L.zmat[iz];
        cubic_stress(L.mat[3 * m], L.mat[3 * m + 1], L.mat[3 * m + 2], S, T);
        const R sdt = S[0] * T[0] + S[1] * T[1] + S[2] * T[2] + R(2) * (S[3] * T[3] + S[4] * T[4] + S[5] * T[5]);
        dens = R(0.25) * L.w[i] * L.w[j] * L.w[k] * g.det2 * g.hz * sdt;
    }
    red[tid] = dens;
    __syncthreads();
    // fixed-order reduction (deterministic): strided sums into 64 slots, then a tree
    if (tid < 64) {
        R acc = 0;
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

// Per element, the three quadrature sums from which every per-modulus part of the
// energy follows (the moduli are applied on the host):
//   A = 1/2 int sum_i S_ii^2,   B = int sum_{i<j} S_ii S_jj,   C = 2 int sum_{i<j} S_ij^2,
// so that U = c11 A + c12 B + c44 C and the bulk part is K (A + B).
template <int N>
__global__ __launch_bounds__(threads_for<N>()) void k_energy_invariants(LevelView<double> L,
                                                                      const double* __restrict__ u,
                                                                      double* __restrict__ abc) {
    constexpr int N2 = N * N, N3 = N2 * N, NT = threads_for<N>();
    __shared__ double su[3 * N3];
    __shared__ double sD[N2];
    __shared__ double red[3][NT];
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    const double* ue = u + (size_t)e * 3 * N3;
    for (int q = tid; q < 3 * N3; q += blockDim.x) su[q] = ue[q];
    for (int q = tid; q < N2; q += blockDim.x) sD[q] = L.D[q];
    __syncthreads();
    double a = 0, b = 0, c = 0;
    if (tid < N3) {
        const int i = tid % N, j = (tid / N) % N, k = tid / N2;
        const int col = e % L.n_cols, iz = e / L.n_cols;
        const NodeGeo<double> g = node_geo<N>(L, col, iz, i, j);
        double G[3][3], S[6];
        gradient<N>(su, sD, i, j, k, g, G);
        sym_of(G, S);
        const double wJ = L.w[i] * L.w[j] * L.w[k] * g.det2 * 0.5 * g.hz;
        a = wJ * 0.5 * (S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
        b = wJ * (S[0] * S[1] + S[1] * S[2] + S[0] * S[2]);
        c = wJ * 2.0 * (S[3] * S[3] + S[4] * S[4] + S[5] * S[5]);
    }
    red[0][tid] = a;
    red[1][tid] = b;
    red[2][tid] = c;
    __syncthreads();
    if (tid < 64) {  // fixed-order reduction
        double s0 = 0, s1 = 0, s2 = 0;
        for (int q = tid; q < NT; q += 64) {
            s0 += red[0][q];
            s1 += red[1][q];
            s2 += red[2][q];
        }
        red[0][tid] = s0;
        red[1][tid] = s1;
        red[2][tid] = s2;
    }
    __syncthreads();
    for (int st = 32; st > 0; st >>= 1) {
        if (tid < st) {
            red[0][tid] += red[0][tid + st];
            red[1][tid] += red[1][tid + st];
            red[2][tid] += red[2][tid + st];
        }
        __syncthreads();
    }
    if (tid < 3) abc[(size_t)e * 3 + tid] = red[tid][0];
}

// g = scale * w(layer) * sum_m Dhat_m^T [w J (J^-1)^m_i Y^{ijkl} D_(k u_l)]: the
// derivative with respect to u of the layer-weighted energy sum_k w_k U_k.
template <int N>
__global__ __launch_bounds__(threads_for<N>()) void k_energy_grad(LevelView<double> L, const double* __restrict__ u,
                                                                 const double* __restrict__ wz,
                                                                 double* __restrict__ gout, double scale) {
    constexpr int N2 = N * N, N3 = N2 * N;
    __shared__ double sbuf[9 * N3];
    __shared__ double sD[N2];
    double* su = sbuf;
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    const double* ue = u + (size_t)e * 3 * N3;
    for (int q = tid; q < 3 * N3; q += blockDim.x) su[q] = ue[q];
    for (int q = tid; q < N2; q += blockDim.x) sD[q] = L.D[q];
    __syncthreads();
    const bool act = tid < N3;
    const int i = tid % N, j = (tid / N) % N, k = tid / N2;
    const int col = e % L.n_cols, iz = e / L.n_cols;
    double Fr[9];
    if (act) {
        const NodeGeo<double> g = node_geo<N>(L, col, iz, i, j);
        double G[3][3], S[6], T[6];
        gradient<N>(su, sD, i, j, k, g, G);
        sym_of(G, S);
        const int m = L.zmat[iz];
        cubic_stress(L.mat[3 * m], L.mat[3 * m + 1], L.mat[3 * m + 2], S, T);
        const double wJ = L.w[i] * L.w[j] * L.w[k] * g.det2 * 0.5 * g.hz;
        const double dz = 2.0 / g.hz;
        const double Tx[3] = {T[0], T[3], T[4]}, Ty[3] = {T[3], T[1], T[5]}, Tz[3] = {T[4], T[5], T[2]};
        for (int c = 0; c < 3; ++c) {
            Fr[c] = wJ * (g.axx * Tx[c] + g.axy * Ty[c]);
            Fr[3 + c] = wJ * (g.aex * Tx[c] + g.aey * Ty[c]);
            Fr[6 + c] = wJ * dz * Tz[c];
        }
    }
    __syncthreads();
    if (act)
        for (int s = 0; s < 9; ++s) sbuf[s * N3 + tid] = Fr[s];
    __syncthreads();
    if (!act) return;
    const double wl = wz[iz] * scale;
    for (int c = 0; c < 3; ++c) {
        double r = 0;
        for (int a = 0; a < N; ++a) {
            r += sD[a * N + i] * sbuf[(0 + c) * N3 + k * N2 + j * N + a];
            r += sD[a * N + j] * sbuf[(3 + c) * N3 + k * N2 + a * N + i];
            r += sD[a * N + k] * sbuf[(6 + c) * N3 + a * N2 + j * N + i];
        }
        gout[(size_t)e * 3 * N3 + c * N3 + tid] = wl * r;
    }
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
        hipLaunchKernelGGL((k_traction<NN, R>), dim3(L.E), dim3(line_threads<NN>()), 0, s, L, u, tau);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t launch_apply(const LevelView<R>& L, const R* u, const R* tau, R* out, R scale, hipStream_t s) {
    return dispatch_n(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_apply<NN, R>), dim3(L.E), dim3(line_threads<NN>()), 0, s, L, u, tau, out, scale);
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

template <typename R>
hipError_t launch_energy(const LevelView<R>& L, const double* u, R* Ue, hipStream_t s) {
    return dispatch_n(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_energy<NN, R>), dim3(L.E), dim3(threads_for<NN>()), 0, s, L, u, Ue);
        return hipGetLastError();
    });
}

hipError_t launch_energy_invariants(const LevelView<double>& L, const double* u, double* abc, hipStream_t s) {
    return dispatch_n(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_energy_invariants<NN>), dim3(L.E), dim3(threads_for<NN>()), 0, s, L, u, abc);
        return hipGetLastError();
    });
}

hipError_t launch_energy_grad(const LevelView<double>& L, const double* u, const double* wz, double* g, double scale,
                              hipStream_t s) {
    return dispatch_n(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_energy_grad<NN>), dim3(L.E), dim3(threads_for<NN>()), 0, s, L, u, wz, g, scale);
        return hipGetLastError();
    });
}

// The dual-number operator is used for parameter derivatives at p <= 5 (its
// LDS footprint doubles); larger N return hipErrorInvalidValue.
template <typename F>
hipError_t dispatch_dual(int N, F&& f) {
    switch (N) {
        case 2: return f(std::integral_constant<int, 2>{});
        case 3: return f(std::integral_constant<int, 3>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 5: return f(std::integral_constant<int, 5>{});
        case 6: return f(std::integral_constant<int, 6>{});
        case 7: return f(std::integral_constant<int, 7>{});
        default: return hipErrorInvalidValue;
    }
}

template <>
hipError_t launch_traction<Dual>(const LevelView<Dual>& L, const Dual* u, Dual* tau, hipStream_t s) {
    return dispatch_dual(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_traction<NN, Dual>), dim3(L.E), dim3(line_threads<NN>()), 0, s, L, u, tau);
        return hipGetLastError();
    });
}

template <>
hipError_t launch_apply<Dual>(const LevelView<Dual>& L, const Dual* u, const Dual* tau, Dual* out, Dual scale,
                              hipStream_t s) {
    return dispatch_dual(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_apply<NN, Dual>), dim3(L.E), dim3(line_threads<NN>()), 0, s, L, u, tau, out, scale);
        return hipGetLastError();
    });
}

template <>
hipError_t launch_energy<Dual>(const LevelView<Dual>& L, const double* u, Dual* Ue, hipStream_t s) {
    return dispatch_dual(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_energy<NN, Dual>), dim3(L.E), dim3(threads_for<NN>()), 0, s, L, u, Ue);
        return hipGetLastError();
    });
}

template hipError_t launch_energy<double>(const LevelView<double>&, const double*, double*, hipStream_t);
template hipError_t launch_traction<double>(const LevelView<double>&, const double*, double*, hipStream_t);
template hipError_t launch_traction<float>(const LevelView<float>&, const float*, float*, hipStream_t);
template hipError_t launch_apply<double>(const LevelView<double>&, const double*, const double*, double*, double,
                                         hipStream_t);
template hipError_t launch_apply<float>(const LevelView<float>&, const float*, const float*, float*, float,
                                        hipStream_t);

}  // namespace dgtn
