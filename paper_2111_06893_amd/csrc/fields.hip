// gfx950 kernels of the load vector and the elastic energy (Sec. 2.1 and eq.
// laserbeam): one workgroup per element, one lane per LGL node, the element's
// displacement staged in LDS.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "element.h"

namespace dgtn {

namespace {

// Load vector of the Gaussian pressure on DGTN_BC_PRESSURE faces at node
// (i, j, k) of element e: b = -w_face J^Sigma n p(r), which is +z on the loaded
// face z = 0, summed over the element faces the node lies on.
// mode 0: p itself; 1, 2, 3: its derivative with respect to the beam width r0
// and the beam centre xc, yc (the load vector's parameter derivatives).
template <int N>
__device__ inline void load_at_node(const LevelView<double>& L, const double* __restrict__ xy, double F0, double r0,
                                    double xc, double yc, int mode, int e, int i, int j, int k, double acc[3]) {
    constexpr int N2 = N * N;
    acc[0] = acc[1] = acc[2] = 0;
    const bool fi = (i == 0) | (i == N - 1), fj = (j == 0) | (j == N - 1), fk = (k == 0) | (k == N - 1);
    if (!(fi | fj | fk)) return;
    const int col = e % L.n_cols, iz = e / L.n_cols;
    const NodeGeo<double> g = node_geo<N>(L, col, iz, i, j);
    const int faces[3] = {fi ? (i == 0 ? 0 : 1) : -1, fj ? (j == 0 ? 2 : 3) : -1, fk ? (k == 0 ? 4 : 5) : -1};
    const double x = xy[(size_t)col * 2 * N2 + j * N + i] - xc;
    const double y = xy[(size_t)col * 2 * N2 + N2 + j * N + i] - yc;
    const double rho2 = x * x + y * y, ir2 = 1.0 / (r0 * r0);
    double p = F0 * exp(-rho2 * ir2) / (M_PI * r0 * r0);
    if (mode == 1) p *= 2.0 * (rho2 * ir2 - 1.0) / r0;
    else if (mode == 2) p *= 2.0 * x * ir2;
    else if (mode == 3) p *= 2.0 * y * ir2;
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
}

template <int N>
__global__ __launch_bounds__(threads_for<N>()) void k_rhs(LevelView<double> L, const double* __restrict__ xy,
                                                         double F0, double r0, double xc, double yc, int mode,
                                                         double* __restrict__ b) {
    constexpr int N2 = N * N, N3 = N2 * N;
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid >= N3) return;
    double acc[3];
    load_at_node<N>(L, xy, F0, r0, xc, yc, mode, e, tid % N, (tid / N) % N, tid / N2, acc);
    double* be = b + (size_t)e * 3 * N3;
    for (int c = 0; c < 3; ++c) be[c * N3 + tid] = acc[c];
}

// Per element, sum over its nodes of b . u with b the load vector (mode 0 of
// load_at_node): the element's share of the compliance u . b, without storing b.
template <int N>
__global__ __launch_bounds__(threads_for<N>()) void k_load_dot(LevelView<double> L, const double* __restrict__ xy,
                                                              double F0, double r0, double xc, double yc,
                                                              const double* __restrict__ u, double* __restrict__ out) {
    constexpr int N2 = N * N, N3 = N2 * N, NT = threads_for<N>();
    __shared__ double red[NT / 64];
    const int e = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double d = 0;
    if (tid < N3) {
        double acc[3];
        load_at_node<N>(L, xy, F0, r0, xc, yc, 0, e, tid % N, (tid / N) % N, tid / N2, acc);
        const double* ue = u + (size_t)e * 3 * N3 + tid;
        if (acc[0] != 0 || acc[1] != 0 || acc[2] != 0) d = acc[0] * ue[0] + acc[1] * ue[N3] + acc[2] * ue[2 * N3];
    }
    for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off);   // fixed order: deterministic
    if (lane == 0) red[wave] = d;
    __syncthreads();
    if (tid == 0) {
        double t = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) t += red[w];
        out[e] = t;
    }
}

// Per-layer sums of per-element values in a fixed order (deterministic):
// block k < n_layers sums v[lay_e0[k] .. lay_e0[k+1]) times `scale` into
// sums[k]; block n_layers, when dot is given, sums dot[0 .. lay_e0[n_layers])
// times `dot_scale` into sums[n_layers].
constexpr int kSumThreads = 256;
__global__ __launch_bounds__(kSumThreads) void k_layer_sums(const double* __restrict__ v, const double* __restrict__ dot,
                                                           const int* __restrict__ lay_e0, int n_layers, double scale,
                                                           double dot_scale, double* __restrict__ sums) {
    __shared__ double red[kSumThreads];
    const int k = blockIdx.x, tid = threadIdx.x;
    const bool is_dot = k == n_layers;
    const double* src = is_dot ? dot : v;
    const int a = is_dot ? 0 : lay_e0[k], b = is_dot ? lay_e0[n_layers] : lay_e0[k + 1];
    double t = 0;
    for (int q = a + tid; q < b; q += kSumThreads) t += src[q];
    red[tid] = t;
    __syncthreads();
    for (int w = kSumThreads / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) sums[k] = red[0] * (is_dot ? dot_scale : scale);
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
    const int e = L.e0 + blockIdx.x;
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

// Face-jump indicator of adaptive refinement: eta_e^2 = sum over the element's
// faces of 1/2 int |u_e - u_nb|^2 dS on interior faces and int |u_e|^2 dS on
// Dirichlet faces (homogeneous data), none on Neumann faces, with the face
// quadrature of the operator (w_face J^Sigma).  The jump is what the interior
// penalty of eq. penalty acts on; Sec. 4 names adaptive refinement as the next
// step.  The sum may be restricted to the side faces or to the z-faces, where
// refinement across the layers acts, and each term may be weighted by the
// penalty sigma at its node (the jump part of the DG energy norm).  One
// workgroup per element: wave 0 resolves the face records, one lane per face
// node, a fixed-order sum.
template <int N>
__global__ __launch_bounds__(line_threads<N>()) void k_jump_indicator(LevelView<double> L,
                                                                     const double* __restrict__ u, int which,
                                                                     double* __restrict__ eta) {
    constexpr int N2 = N * N, N3 = N2 * N, NT = line_threads<N>();
    __shared__ FaceInfo<double> sface[6];
    __shared__ double sown[5];
    __shared__ double red[NT / 64];
    const int e = L.e0 + blockIdx.x;
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int col = e % L.n_cols, iz = e / L.n_cols;
    if (tid < 64) load_faces<N>(L, col, iz, tid, sface, sown);
    __syncthreads();
    double dens = 0;
    // which: 1 the side faces (logical xi, eta), 2 the z-faces (zeta), 3 both;
    // bit 4: weighted by the penalty sigma
    if (tid < 6 * N2 && (which & (tid / N2 < 4 ? 1 : 2))) {
        const int f = tid / N2, fi = tid % N2;
        int i, j, k;
        face_node<N>(f, fi, i, j, k);
        const FaceInfo<double>& fo = sface[f];
        const double det2 = L.geo2[(size_t)col * 5 * N2 + 4 * N2 + j * N + i];
        double n[3], amag;
        face_frame<N>(L, col, f, i, j, n, amag);
        const double hz = sown[3];
        const double ws = f >= 4 ? L.w[i] * L.w[j] * det2
                        : f < 2  ? L.w[j] * L.w[k] * 0.5 * hz * det2 * amag
                                 : L.w[i] * L.w[k] * 0.5 * hz * det2 * amag;
        const double* ue = u + (size_t)e * 3 * N3 + k * N2 + j * N + i;
        if (fo.bc == 0) {
            int i2, j2, k2;
            const Nbr nb{fo.e, fo.f, fo.flip, 0};
            matching_node<N>(f, nb, i, j, k, i2, j2, k2);
            const double* un = u + (size_t)fo.e * 3 * N3 + k2 * N2 + j2 * N + i2;
            double s2 = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double d = ue[c * N3] - un[c * N3];
                s2 += d * d;
            }
            dens = 0.5 * ws * s2;
        } else if (fo.bc == DGTN_BC_DIRICHLET) {
            double s2 = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) s2 += ue[c * N3] * ue[c * N3];
            dens = ws * s2;
        }
        if (which & 4) dens *= f < 4 ? L.sig_side[((size_t)col * 4 + f) * N + (f < 2 ? j : i)] : fo.sig;
    }
    for (int off = 32; off > 0; off >>= 1) dens += __shfl_xor(dens, off);
    if (lane == 0) red[wave] = dens;
    __syncthreads();
    if (tid == 0) {
        double t = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) t += red[w];
        eta[blockIdx.x] = t;
    }
}

}  // namespace

hipError_t launch_rhs(const LevelView<double>& L, const double* xy, double F0, double r0, double xc, double yc,
                      int mode, double* b, hipStream_t s) {
    return dispatch_n(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_rhs<NN>), dim3(L.E), dim3(threads_for<NN>()), 0, s, L, xy, F0, r0, xc, yc, mode, b);
        return hipGetLastError();
    });
}

hipError_t launch_load_dot(const LevelView<double>& L, const double* xy, double F0, double r0, double xc, double yc,
                           const double* u, double* out, hipStream_t s) {
    return dispatch_n(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_load_dot<NN>), dim3(L.E), dim3(threads_for<NN>()), 0, s, L, xy, F0, r0, xc, yc, u, out);
        return hipGetLastError();
    });
}

hipError_t launch_layer_sums(const double* v, const double* dot, const int* lay_e0, int n_layers, double scale,
                             double dot_scale, double* sums, hipStream_t s) {
    hipLaunchKernelGGL(k_layer_sums, dim3(n_layers + (dot ? 1 : 0)), dim3(kSumThreads), 0, s, v, dot, lay_e0, n_layers,
                       scale, dot_scale, sums);
    return hipGetLastError();
}

hipError_t launch_jump_indicator(const LevelView<double>& L, const double* u, int which, double* eta,
                                 hipStream_t s) {
    return dispatch_n(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_jump_indicator<NN>), dim3(L.E), dim3(line_threads<NN>()), 0, s, L, u, which, eta);
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

template <>
hipError_t launch_energy<Dual>(const LevelView<Dual>& L, const double* u, Dual* Ue, hipStream_t s) {
    return dispatch_dual(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_energy<NN, Dual>), dim3(L.E), dim3(threads_for<NN>()), 0, s, L, u, Ue);
        return hipGetLastError();
    });
}

template hipError_t launch_energy<double>(const LevelView<double>&, const double*, double*, hipStream_t);

}  // namespace dgtn
