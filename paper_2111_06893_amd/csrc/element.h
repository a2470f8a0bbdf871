// Device building blocks shared by the operator kernels and the load and
// energy kernels: constitutive relation, metric, face normals and neighbours,
// the lane decomposition of the element kernels, and the N dispatch.
#pragma once

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

// The same products with the zero components of a face normal left out: a
// side face's normal has no z-component, a z-face's is (0, 0, s), s = +-1.
// IEEE arithmetic does not let the compiler drop x * 0 or x + 0 by itself (x
// could be infinite, or -0), and those terms were about a tenth of the FP64
// work of the face and node phases.  For finite values the results are the
// same as the general forms.
template <typename R>
__device__ __forceinline__ void traction_xy(R nx, R ny, const R T[6], R t[3]) {
    t[0] = nx * T[0] + ny * T[3];
    t[1] = nx * T[3] + ny * T[1];
    t[2] = nx * T[4] + ny * T[5];
}

template <typename R>
__device__ __forceinline__ void traction_z(R s, const R T[6], R t[3]) {
    t[0] = s * T[4];
    t[1] = s * T[5];
    t[2] = s * T[2];
}

// S += sym(n (x) v), side face and z-face
template <typename R>
__device__ __forceinline__ void add_sym_outer_xy(R nx, R ny, const R v[3], R S[6]) {
    S[0] += nx * v[0];
    S[1] += ny * v[1];
    S[3] += R(0.5) * (nx * v[1] + ny * v[0]);
    S[4] += R(0.5) * (nx * v[2]);
    S[5] += R(0.5) * (ny * v[2]);
}

template <typename R>
__device__ __forceinline__ void add_sym_outer_z(R s, const R v[3], R S[6]) {
    S[2] += s * v[2];
    S[4] += R(0.5) * (s * v[0]);
    S[5] += R(0.5) * (s * v[1]);
}

// n . Y : sym(n (x) v) for a side-face normal (n_z = 0) and cubic moduli: the
// penalty traction of a jump v (eq. penalty).  On a z-face it reduces to
// (c44 v_x, c44 v_y, c11 v_z) whatever the sign of the normal.
template <typename R>
__device__ __forceinline__ void penalty_traction_xy(R c11, R c12, R c44, R nx, R ny, const R v[3], R t[3]) {
    const R S0 = nx * v[0], S1 = ny * v[1];
    const R S3 = R(0.5) * (nx * v[1] + ny * v[0]);
    const R S4 = R(0.5) * (nx * v[2]), S5 = R(0.5) * (ny * v[2]);
    const R T[6] = {c11 * S0 + c12 * S1, c11 * S1 + c12 * S0, R(0), R(2) * c44 * S3, R(2) * c44 * S4,
                    R(2) * c44 * S5};
    traction_xy(nx, ny, T, t);
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

// The same from the per-column table of side-face normals (no square root or
// division in the kernel); (i, j) is the node's position in the column.
template <int N, typename R>
__device__ __forceinline__ void face_frame(const LevelView<R>& L, int col, int f, int i, int j, R n[3], R& amag) {
    if (f < 4) {
        const R* t = L.fnrm + ((size_t)col * 4 + f) * 3 * N + (f < 2 ? j : i);
        n[0] = t[0];
        n[1] = t[N];
        n[2] = 0;
        amag = t[2 * N];
    } else {
        amag = 0;
        n[0] = 0;
        n[1] = 0;
        n[2] = (f == 5) ? R(1) : R(-1);
    }
}

// Outward unit normal (nx, ny, 0) and |grad xi^m| of side face f < 4 at a node.
template <int N, typename R>
__device__ __forceinline__ void side_normal(const LevelView<R>& L, int col, int f, int i, int j, R& nx, R& ny,
                                            R& amag) {
    const R* t = L.fnrm + ((size_t)col * 4 + f) * 3 * N + (f < 2 ? j : i);
    nx = t[0];
    ny = t[N];
    amag = t[2 * N];
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

// Copies CNT consecutive values into LDS with a workgroup of NT threads: every
// load of a thread is issued before its first store, so that they are in flight
// together.  Items past CNT re-read the last value and store it again in its own
// slot (the same value from every such thread): no branch, so the compiler cannot
// sink a load into one behind the stores.
template <int CNT, int NT, typename R>
__device__ __forceinline__ void stage_to_lds(R* dst, const R* __restrict__ src, int tid) {
    constexpr int IT = (CNT + NT - 1) / NT;
    R v[IT];
#pragma unroll
    for (int t = 0; t < IT; ++t) v[t] = src[min(tid + t * NT, CNT - 1)];
#pragma unroll
    for (int t = 0; t < IT; ++t) dst[min(tid + t * NT, CNT - 1)] = v[t];
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
    R sig;                // z faces: penalty sigma, C N^2 / min(h, h_neighbour) (own h on boundaries)
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
        // the neighbour's z-element index does not wait for the column tables: a side
        // neighbour lies in the same z-layer, a z-neighbour one layer up or down
        const int izn = tid < 4 ? iz : (tid == 4 ? max(iz - 1, 0) : min(iz + 1, L.n_z - 1));
        const int m = L.zmat[iz];
        const int mn = L.zmat[izn];
        const bool in = nb.bc == 0;
        fi.c11 = R(0.5) * (L.mat[3 * m] + L.mat[3 * (in ? mn : m)]);
        fi.c12 = R(0.5) * (L.mat[3 * m + 1] + L.mat[3 * (in ? mn : m) + 1]);
        fi.c44 = R(0.5) * (L.mat[3 * m + 2] + L.mat[3 * (in ? mn : m) + 2]);
        fi.hz = in ? L.hz[izn] : L.hz[iz];
        fi.sig = L.penalty_n2 / min(fi.hz, L.hz[iz]);
        sf[tid] = fi;
    } else if (tid == 6) {
        const int m = L.zmat[iz];
        sown[0] = L.mat[3 * m];
        sown[1] = L.mat[3 * m + 1];
        sown[2] = L.mat[3 * m + 2];
        sown[3] = L.hz[iz];
        sown[4] = R(2) / L.hz[iz];
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
// x N^2 lines), N^3 nodes, 6 N^2 face nodes, rounded up to an even number of
// waves: a CU holds three workgroups of seven waves but four of eight (measured).
template <int N>
constexpr int line_threads() {
    constexpr int a = 9 * N * N, b = N * N * N, c = 6 * N * N;
    constexpr int m = a > b ? (a > c ? a : c) : (b > c ? b : c);
    return ((m + 127) / 128) * 128;
}

// Lanes of the two operator kernels (k_traction, k_apply).  At N = 6 the node
// and face phases have 216 tasks and the line phases 324: 256 lanes, whose
// line phases take a second pass over the 68 remaining lines, let six
// workgroups share a CU (their LDS allows it) where 384 lanes allowed four
// within the same number of waves, so more elements hide each other's
// latencies.  Elsewhere one lane per task of the largest phase.
template <int N>
constexpr int op_threads() {
    return N == 6 ? 256 : line_threads<N>();
}

// Line task t < 9 N^2: direction d (xi, eta, zeta), component c, and the offset
// and stride of the line's N nodes within one component's N^3 block, packed
// into one word per task (base | c << 10 | d << 12 | stride << 14) at compile
// time.  A lane reads its word with one load instead of decoding t by divisions
// by constants, about twenty instructions per pass.
template <int N>
struct LineCodes {
    int v[9 * N * N];
    constexpr LineCodes() : v() {
        constexpr int N2 = N * N;
        for (int t = 0; t < 9 * N2; ++t) {
            const int d = t / (3 * N2), rem = t % (3 * N2), c = rem / N2;
            const int q = rem % N2, q1 = q % N, q2 = q / N;
            const int base = d == 0 ? q2 * N2 + q1 * N : d == 1 ? q2 * N2 + q1 : q2 * N + q1;
            const int stride = d == 0 ? 1 : d == 1 ? N : N2;
            v[t] = base | c << 10 | d << 12 | stride << 14;
        }
    }
};

template <int N>
__device__ constexpr LineCodes<N> kLineCodes{};

// The same tasks for kernels that need the derivatives at face nodes only
// (the tractions): a line whose two transverse indices are both interior
// crosses the element's faces at its two ends alone, so only its end outputs
// are computed (bit 21 of the word).  The lines are ordered with the full
// ones first, so that most waves take one branch: 20 full and 16 end-only
// lines of 36 per direction at N = 6, 28 % fewer products.
template <int N>
struct FaceLineCodes {
    int v[9 * N * N];
    constexpr FaceLineCodes() : v() {
        constexpr int N2 = N * N;
        const LineCodes<N> all{};
        int m = 0;
        for (int pass = 0; pass < 2; ++pass)
            for (int t = 0; t < 9 * N2; ++t) {
                const int q = (t % (3 * N2)) % N2, q1 = q % N, q2 = q / N;
                const bool ends = q1 > 0 && q1 < N - 1 && q2 > 0 && q2 < N - 1;
                if (ends != (pass == 1)) continue;
                v[m++] = all.v[t] | (ends ? 1 << 21 : 0);
            }
    }
};

template <int N>
__device__ constexpr FaceLineCodes<N> kFaceLineCodes{};

template <int N>
__device__ __forceinline__ void line_of(int w, int& d, int& c, int& base, int& stride) {
    static_assert(N * N * N <= 1024, "base takes ten bits");
    base = w & 1023;
    c = (w >> 10) & 3;
    d = (w >> 12) & 3;
    stride = (w >> 14) & 127;
}

// A lane's line tasks t = tid + p NT, p < passes: their code words, loaded at the
// start of a kernel so that the load is in flight while u is staged.
template <int N, int NT>
struct LineTasks {
    static constexpr int passes = (9 * N * N + NT - 1) / NT;
    int w[passes];
};

template <int N, int NT, bool FACES = false>
__device__ __forceinline__ LineTasks<N, NT> line_tasks(int tid) {
    LineTasks<N, NT> r;
#pragma unroll
    for (int p = 0; p < LineTasks<N, NT>::passes; ++p) {
        const int t = min(tid + p * NT, 9 * N * N - 1);
        r.w[p] = FACES ? kFaceLineCodes<N>.v[t] : kLineCodes<N>.v[t];
    }
    return r;
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
    // unrolled: the scalar loads of the rows of D are issued ahead of their use
    // instead of one exposed load latency per output
#pragma unroll
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
// NT lanes take the 9 N^2 lines in passes of NT.
template <int N, typename R, int NT = line_threads<N>(), bool FACES = false>
__device__ __forceinline__ void ref_derivatives(const LevelView<R>& L, const R* su, R* sG, int tid,
                                                const LineTasks<N, NT>& tasks) {
    constexpr int N3 = N * N * N;
#pragma unroll
    for (int p = 0; p < LineTasks<N, NT>::passes; ++p) {
        if (tid + p * NT >= 9 * N * N) break;
        int d, c, base, stride;
        line_of<N>(tasks.w[p], d, c, base, stride);
        R* dst = sG + (d * 3 + c) * N3 + base;
        if (FACES && (tasks.w[p] >> 21)) {  // the line's two end outputs only (face-node kernels)
            const R* src = su + c * N3;
            R v[N];
#pragma unroll
            for (int a = 0; a < N; ++a) v[a] = src[base + a * stride];
#pragma unroll
            for (int e2 = 0; e2 < 2; ++e2) {
                const int x = e2 ? N - 1 : 0;
                R acc = 0;
#pragma unroll
                for (int a = 0; a < N; ++a) acc += L.Dk[x * N + a] * v[a];
                dst[x * stride] = acc;
            }
        } else {
            line_contract<N, false>(L, su + c * N3, base, stride, [&](int x, R v) { dst[x * stride] = v; });
        }
    }
}

// Physical gradient G[d][l] = D_d u_l at node q from the reference derivatives.
template <int N, typename R>
__device__ __forceinline__ void node_gradient(const R* sG, int q, const NodeGeo<R>& g, R dz, R G[3][3]) {
    constexpr int N3 = N * N * N;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const R dxi = sG[l * N3 + q], deta = sG[(3 + l) * N3 + q], dzeta = sG[(6 + l) * N3 + q];
        G[0][l] = g.axx * dxi + g.aex * deta;
        G[1][l] = g.axy * dxi + g.aey * deta;
        G[2][l] = dz * dzeta;
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

// The 16-byte kernels (dual numbers of the parameter derivatives, double-double
// numbers of the extended-precision residual) for every degree p = 1..7: their
// LDS footprint doubles, 135 KB at N = 8, within gfx950's 160 KB.
template <typename F>
hipError_t dispatch_dual(int N, F&& f) {
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

}  // namespace dgtn
