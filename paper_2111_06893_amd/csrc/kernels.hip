// gfx950 kernels of the DG elasticity operator (Sec. 2.2.2 - 2.2.4).
//
// One workgroup per element.  The element's displacement is staged in LDS and
// the work alternates between three lane roles separated by barriers: line
// lanes (one per line of N nodes along xi, eta or zeta and per component) do
// the sum-factorised LGL contractions, reading each input once from LDS with
// the 1D matrix D in scalar registers; node lanes (one per LGL node) do the
// pointwise metric, lift and constitutive work; face lanes (one per face node)
// do the jumps and numerical fluxes.  FP64, FP32, the dual numbers of the
// adjoint and the double-double numbers of the extended-precision residual are
// the same template.
//
// The operator is applied in two passes:
//   k_traction  t = n . Y . D u on the 6 N^2 face nodes of every element (the
//               unlifted derivative entering the flux of eq. numflux);
//   k_apply     lifted strain, stress, weak divergence and face fluxes, which
//               read the neighbours' displacement traces and tractions.
#include "ddouble.h"
#include "element.h"

namespace dgtn {

namespace {

template <int N, typename R>
__global__ __launch_bounds__(op_threads<N>()) void k_traction(LevelView<R> L, const R* __restrict__ u,
                                                             R* __restrict__ tau) {
    constexpr int N2 = N * N, N3 = N2 * N, NT = op_threads<N>();
    __shared__ R su[3 * N3];
    __shared__ R sG[9 * N3];
    __shared__ R sown[5];
    const int e = L.e0 + xcd_element(blockIdx.x, L.E);
    const int tid = threadIdx.x;
    const int col = e % L.n_cols, iz = e / L.n_cols;
    const R* ue = u + (size_t)e * 3 * N3;
    const LineTasks<N, NT> tasks = line_tasks<N, NT, true>(tid);  // face nodes only
    // waves 1.. stage u while wave 0 reads the element's material (two dependent
    // table reads), so that the two latencies overlap instead of adding up
    if (tid >= 64) {
        stage_to_lds<3 * N3, NT - 64>(su, ue, tid - 64);
    } else if (tid == 0) {
        const int m = L.zmat[iz];
        sown[0] = L.mat[3 * m];
        sown[1] = L.mat[3 * m + 1];
        sown[2] = L.mat[3 * m + 2];
        sown[3] = L.hz[iz];
        sown[4] = R(2) / L.hz[iz];
    }
    const bool act = tid < 6 * N2;
    const int f = tid / N2, fi = tid % N2;
    int i = 0, j = 0, k = 0;
    if (act) face_node<N>(f, fi, i, j, k);
    NodeGeo<R> g = act ? node_geo<N>(L, col, iz, i, j) : NodeGeo<R>{1, 0, 0, 1, 1, 1};
    __syncthreads();
    ref_derivatives<N, R, NT, true>(L, su, sG, tid, tasks);
    __syncthreads();
    if (!act) return;
    R G[3][3], S[6], T[6], t[3];
    node_gradient<N>(sG, k * N2 + j * N + i, g, sown[4], G);
    sym_of(G, S);
    cubic_stress(sown[0], sown[1], sown[2], S, T);
    if (f < 4) {
        R nx, ny, amag;
        side_normal<N>(L, col, f, i, j, nx, ny, amag);
        traction_xy(nx, ny, T, t);
    } else {
        traction_z(f == 5 ? R(1) : R(-1), T, t);
    }
    R* dst = tau + ((size_t)e * 6 + f) * 3 * N2 + fi;
    dst[0] = t[0];
    dst[N2] = t[1];
    dst[2 * N2] = t[2];
}

// Waves per SIMD asked of the compiler: eight (four workgroups of eight waves
// per CU at N = 7), except for the FP64 instantiations that need more than the
// 64 registers this allows and would spill (N = 2, 5, 6: seven).  FP64 at N = 7
// fits because the face data are read from LDS where used rather than copied
// into registers, and its lift factors are stored over u (below), which keeps
// the LDS at 40.5 KB.
template <int N, typename R>
constexpr int apply_waves() {
    if constexpr (sizeof(R) == 16) return 4;  // dual and double-double numbers: 128 registers
    if constexpr (sizeof(R) == 8 && N == 6) return 6;  // six workgroups of four waves per CU
    return (sizeof(R) == 8 && (N == 2 || N == 5)) ? 7 : 8;
}

template <int N, typename R>
__global__ __launch_bounds__(op_threads<N>(), (apply_waves<N, R>())) void k_apply(LevelView<R> L, const R* __restrict__ u,
                                                            const R* __restrict__ tau, R* __restrict__ out,
                                                            R scale) {
    constexpr int N2 = N * N, N3 = N2 * N, NT = op_threads<N>();
    static_assert(NT >= N3 && NT >= 6 * N2, "node and face phases take one pass");
    __shared__ R su[3 * N3];          // u
    __shared__ R sG[9 * N3];          // reference derivatives; later the volume fluxes F, then D^T F
    __shared__ R sFT[6 * 3 * N2];     // per face node: interior traction, then -w J^Sigma (n Y S)*
    // per face node: lifting factor times the jump.  In FP64 (N >= 6) it is written
    // over u, which is dead once the face lanes have taken their jumps.
    constexpr bool kLiftOverU = sizeof(R) == 8 && 6 * N2 <= N3;
    __shared__ R sLFown[kLiftOverU ? 1 : 6 * 3 * N2];
    R* const sLF = kLiftOverU ? su : sLFown;
    __shared__ R sw[N];
    __shared__ R swi[N];
    __shared__ FaceInfo<R> sface[6];
    __shared__ R sown[5];
    const int e = L.e0 + xcd_element(blockIdx.x, L.E);
    const int tid = threadIdx.x;
    const int col = e % L.n_cols, iz = e / L.n_cols;
    const R* ue = u + (size_t)e * 3 * N3;
    const LineTasks<N, NT> tasks = line_tasks<N, NT>(tid);
    // waves 1.. stage u and the weights while wave 0 resolves the face records,
    // whose table reads depend on one another: the two latencies overlap instead
    // of adding up
    if (tid >= 64) {
        const int t = tid - 64;
        const R wq = L.w[min(t, N - 1)];
        stage_to_lds<3 * N3, NT - 64>(su, ue, t);
        if (t < N) {  // one wave divides
            sw[t] = wq;
            swi[t] = R(1) / wq;
        }
    } else {
        load_faces<N>(L, col, iz, tid, sface, sown);
    }
    // node role
    const bool nact = tid < N3;
    const int i = tid % N, j = (tid / N) % N, k = tid / N2;
    // node metric: held in registers in FP32; in FP64 and the 16-byte types, where
    // registers bound the occupancy, loaded again (from cache) by the two phases
    // that use it
    constexpr bool kReloadGeo = sizeof(R) >= 8;
    NodeGeo<R> g_held{1, 0, 0, 1, 1, 1};
    if constexpr (!kReloadGeo) {
        if (nact) g_held = node_geo<N>(L, col, iz, i, j);
    }
    auto node_metric = [&]() {
        if constexpr (kReloadGeo) return node_geo<N>(L, col, iz, i, j);
        else return g_held;
    };
    // face role
    const bool fact = tid < 6 * N2;
    const int f = tid / N2, fi = tid % N2;
    int fi_i = 0, fi_j = 0, fi_k = 0;
    if (fact) face_node<N>(f, fi, fi_i, fi_j, fi_k);
    __syncthreads();
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
    ref_derivatives<N, R, NT>(L, su, sG, tid, tasks);
    __syncthreads();
    // 2. node lanes: unlifted gradient and stress; interior traction on each face slot.
    // Only this lane reads its node's derivatives, so S is parked in those slots.
    const bool fxi = (i == 0) | (i == N - 1), feta = (j == 0) | (j == N - 1), fzeta = (k == 0) | (k == N - 1);
    if (nact) {
        const NodeGeo<R> g = node_metric();
        R G[3][3], T[6], S[6];
        node_gradient<N>(sG, tid, g, sown[4], G);
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
                R t[3];
                if (q < 2) {
                    R nx, ny, amag;
                    side_normal<N>(L, col, faces[q], i, j, nx, ny, amag);
                    traction_xy(nx, ny, T, t);
                } else {
                    traction_z(faces[q] == 5 ? R(1) : R(-1), T, t);
                }
                const int slot = faces[q] * 3 * N2 + face_index<N>(faces[q], i, j, k);
                sFT[slot] = t[0];
                sFT[slot + N2] = t[1];
                sFT[slot + 2 * N2] = t[2];
            }
        }
    }
    __syncthreads();
    // 3. face lanes: jump, lift and numerical flux (eqs. numflux, penalty, bc)
    R lfj[3] = {0, 0, 0};
    if (fact) {
        // face geometry loaded here rather than held through the earlier phases (register pressure)
        const R det2 = L.geo2[(size_t)col * 5 * N2 + 4 * N2 + fi_j * N + fi_i];
        const R hz = sown[3];
        const FaceInfo<R>& fo = sface[f];  // read from LDS where used
        const int qn = fi_k * N2 + fi_j * N + fi_i;
        const int slot = f * 3 * N2 + fi;
        const bool interior = fo.bc == 0, penalised = interior || fo.bc == DGTN_BC_DIRICHLET;
        R jump[3] = {0, 0, 0}, flux[3] = {0, 0, 0}, pen[3] = {0, 0, 0};
        if (penalised) {
#pragma unroll
            for (int c = 0; c < 3; ++c) jump[c] = interior ? su[c * N3 + qn] - un[c] : R(2) * su[c * N3 + qn];
        }
        // sigma n . Y* : sym(n (x) [u]) by face family (the z-faces' normal has one component)
        R wsig, lr, sigma;
        if (f < 4) {
            R nx, ny, amag;
            side_normal<N>(L, col, f, fi_i, fi_j, nx, ny, amag);
            sigma = L.sig_side[((size_t)col * 4 + f) * N + (f < 2 ? fi_j : fi_i)];
            wsig = sw[f < 2 ? fi_j : fi_i] * sw[fi_k] * R(0.5) * hz * det2 * amag;
            lr = amag * swi[f < 2 ? fi_i : fi_j];
            if (penalised) penalty_traction_xy(fo.c11, fo.c12, fo.c44, nx, ny, jump, pen);
        } else {
            sigma = fo.sig;
            wsig = sw[fi_i] * sw[fi_j] * det2;
            lr = swi[fi_k] * sown[4];
            pen[0] = fo.c44 * jump[0];
            pen[1] = fo.c44 * jump[1];
            pen[2] = fo.c11 * jump[2];
        }
        if (penalised) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const R tint = sFT[slot + c * N2];
                flux[c] = (interior ? R(0.5) * (tint - tn[c]) : tint) - sigma * pen[c];
            }
        }
        // Neumann faces: no jump and, for homogeneous data, no flux
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lfj[c] = R(-0.5) * lr * jump[c];
            sFT[slot + c * N2] = -wsig * flux[c];
        }
    }
    if constexpr (kLiftOverU) __syncthreads();  // every face lane has read u
    if (fact) {
#pragma unroll
        for (int c = 0; c < 3; ++c) sLF[f * 3 * N2 + fi + c * N2] = lfj[c];
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
            R lj[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) lj[c] = sLF[slot + c * N2];
            if (q < 2) {
                R nx, ny, amag;
                side_normal<N>(L, col, faces[q], i, j, nx, ny, amag);
                add_sym_outer_xy(nx, ny, lj, S);
            } else {
                add_sym_outer_z(faces[q] == 5 ? R(1) : R(-1), lj, S);
            }
        }
        R T[6];
        cubic_stress(c11, c12, c44, S, T);
        const NodeGeo<R> g = node_metric();
        const R wJ = sw[i] * sw[j] * sw[k] * g.det2 * R(0.5) * sown[3];
        const R dz = sown[4];
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
#pragma unroll
    for (int p = 0; p < LineTasks<N, NT>::passes; ++p) {
        if (tid + p * NT >= 9 * N2) break;
        int d, c, base, stride;
        line_of<N>(tasks.w[p], d, c, base, stride);
        R* line = sG + (d * 3 + c) * N3 + base;
        R v[N];
#pragma unroll
        for (int a = 0; a < N; ++a) v[a] = line[a * stride];
#pragma unroll
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

}  // namespace

template <typename R>
hipError_t launch_traction(const LevelView<R>& L, const R* u, R* tau, hipStream_t s) {
    return dispatch_n(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_traction<NN, R>), dim3(L.E), dim3(op_threads<NN>()), 0, s, L, u, tau);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t launch_apply(const LevelView<R>& L, const R* u, const R* tau, R* out, R scale, hipStream_t s) {
    return dispatch_n(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_apply<NN, R>), dim3(L.E), dim3(op_threads<NN>()), 0, s, L, u, tau, out, scale);
        return hipGetLastError();
    });
}

template <>
hipError_t launch_traction<Dual>(const LevelView<Dual>& L, const Dual* u, Dual* tau, hipStream_t s) {
    return dispatch_dual(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_traction<NN, Dual>), dim3(L.E), dim3(op_threads<NN>()), 0, s, L, u, tau);
        return hipGetLastError();
    });
}

template <>
hipError_t launch_apply<Dual>(const LevelView<Dual>& L, const Dual* u, const Dual* tau, Dual* out, Dual scale,
                              hipStream_t s) {
    return dispatch_dual(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_apply<NN, Dual>), dim3(L.E), dim3(op_threads<NN>()), 0, s, L, u, tau, out, scale);
        return hipGetLastError();
    });
}

template <>
hipError_t launch_traction<DD>(const LevelView<DD>& L, const DD* u, DD* tau, hipStream_t s) {
    return dispatch_dual(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_traction<NN, DD>), dim3(L.E), dim3(op_threads<NN>()), 0, s, L, u, tau);
        return hipGetLastError();
    });
}

template <>
hipError_t launch_apply<DD>(const LevelView<DD>& L, const DD* u, const DD* tau, DD* out, DD scale, hipStream_t s) {
    return dispatch_dual(L.N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_apply<NN, DD>), dim3(L.E), dim3(op_threads<NN>()), 0, s, L, u, tau, out, scale);
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
