// gfx950 kernels of the preconditioner and of the Krylov vector algebra.
//
//  * k_fdm_smooth   one damped additive-Schwarz sweep with one subdomain per
//                   element; the subdomain solve is the fast-diagonalisation
//                   inverse of a separable approximation of the element block
//                   (per component c: sum_d kappa_cd K_d (x) M (x) M), applied
//                   as six 1D contractions with the per-element eigenvectors.
//  * k_prolong_p / k_restrict_p   polynomial-degree transfers (tensor-product
//                   Lagrange interpolation between LGL grids, and its transpose).
//  * k_prolong_h / k_restrict_h   transfers between a column and its 2 x 2
//                   children (z unchanged).
//  * k_prolong_z / k_restrict_z   transfers between pairs of z-elements and
//                   their merged (fiducial-layer) element.
//  * k_ovl_fwd / k_col_gemm_mfma / k_ovl_bwd / k_ovl_sum   the overlapping
//                   column-Schwarz smoother: patch gather and x/y transforms, the
//                   shared z-eigenbasis products on the matrix cores with the
//                   eigenvalue division, back transforms and the weighted sum.
//  * dense coarse solve: blocked Gauss-Jordan inversion (k_gjb_*) and a
//                   matrix-vector product.
//  * vector algebra for flexible CG and FGMRES: fused dots, CG updates,
//                   multi-dot, multi-axpy, casts.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "mg.h"

namespace dgtn {

namespace {

template <int N>
constexpr int nthreads() {
    return ((N * N * N + 63) / 64) * 64;
}

// z = x + omega * FDM^{-1} (b - Ax), per element.  Ax == nullptr means x = 0
// (first sweep from a zero guess): z = omega FDM^{-1} b.
template <int N, typename R>
__global__ __launch_bounds__(nthreads<N>()) void k_fdm_smooth(int E, const R* __restrict__ fdm,
                                                              const R* __restrict__ b, const R* __restrict__ Ax,
                                                              R* __restrict__ x, R omega) {
    constexpr int N2 = N * N, N3 = N2 * N, PER = N2 + N;  // per (c, d): S then lambda
    __shared__ R sr[3 * N3];
    __shared__ R st[3 * N3];
    __shared__ R sS[9 * PER];
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    const size_t base = (size_t)e * 3 * N3;
    for (int q = tid; q < 3 * N3; q += blockDim.x) sr[q] = Ax ? b[base + q] - Ax[base + q] : b[base + q];
    const R* fe = fdm + (size_t)e * 9 * PER;
    for (int q = tid; q < 9 * PER; q += blockDim.x) sS[q] = fe[q];
    __syncthreads();
    const bool act = tid < N3;
    const int i = tid % N, j = (tid / N) % N, k = tid / N2;
    // t = (S_x^T (x) S_y^T (x) S_z^T) r, one direction at a time
    // direction x: t[c][k][j][a] = sum_i S_x[i][a] r[c][k][j][i]
    if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R* S = sS + (c * 3 + 0) * PER;
            R acc = 0;
#pragma unroll
            for (int a = 0; a < N; ++a) acc += S[a * N + i] * sr[c * N3 + k * N2 + j * N + a];
            st[c * N3 + tid] = acc;
        }
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R* S = sS + (c * 3 + 1) * PER;
            R acc = 0;
#pragma unroll
            for (int a = 0; a < N; ++a) acc += S[a * N + j] * st[c * N3 + k * N2 + a * N + i];
            sr[c * N3 + tid] = acc;
        }
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R* S = sS + (c * 3 + 2) * PER;
            R acc = 0;
#pragma unroll
            for (int a = 0; a < N; ++a) acc += S[a * N + k] * sr[c * N3 + a * N2 + j * N + i];
            const R lam = sS[(c * 3 + 0) * PER + N2 + i] + sS[(c * 3 + 1) * PER + N2 + j] +
                          sS[(c * 3 + 2) * PER + N2 + k];
            st[c * N3 + tid] = acc / lam;
        }
    }
    __syncthreads();
    // back: z = (S_x (x) S_y (x) S_z) t
    if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R* S = sS + (c * 3 + 2) * PER;
            R acc = 0;
#pragma unroll
            for (int a = 0; a < N; ++a) acc += S[k * N + a] * st[c * N3 + a * N2 + j * N + i];
            sr[c * N3 + tid] = acc;
        }
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R* S = sS + (c * 3 + 1) * PER;
            R acc = 0;
#pragma unroll
            for (int a = 0; a < N; ++a) acc += S[j * N + a] * sr[c * N3 + k * N2 + a * N + i];
            st[c * N3 + tid] = acc;
        }
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R* S = sS + (c * 3 + 0) * PER;
            R acc = 0;
#pragma unroll
            for (int a = 0; a < N; ++a) acc += S[i * N + a] * st[c * N3 + k * N2 + j * N + a];
            const size_t o = base + c * N3 + tid;
            x[o] = (Ax ? x[o] : R(0)) + omega * acc;
        }
    }
}

// ---- column smoother ------------------------------------------------------------
// Forward x/y transform of r = b - Ax (or b) per element:
// T[c][iz*N + k][col*N2 + b*N + a] = sum_{i,j} Sx[i][a] Sy[j][b] r[c][k][j][i].
template <int N, typename R>
__global__ __launch_bounds__(nthreads<N>()) void k_col_fwd(int n_cols, int nzN, const R* __restrict__ S,
                                                           const R* __restrict__ b, const R* __restrict__ Ax,
                                                           R* __restrict__ T) {
    constexpr int N2 = N * N, N3 = N2 * N;
    __shared__ R sr[3 * N3];
    __shared__ R st[3 * N3];
    __shared__ R sS[2 * N2];
    const int e = blockIdx.x, tid = threadIdx.x;
    const int col = e % n_cols, iz = e / n_cols;
    const size_t base = (size_t)e * 3 * N3;
    for (int q = tid; q < 3 * N3; q += blockDim.x) sr[q] = Ax ? b[base + q] - Ax[base + q] : b[base + q];
    for (int q = tid; q < 2 * N2; q += blockDim.x) sS[q] = S[(size_t)col * 2 * N2 + q];
    __syncthreads();
    const bool act = tid < N3;
    const int i = tid % N, j = (tid / N) % N, k = tid / N2;
    if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            R acc = 0;
#pragma unroll
            for (int a = 0; a < N; ++a) acc += sS[a * N + i] * sr[c * N3 + k * N2 + j * N + a];
            st[c * N3 + tid] = acc;
        }
    }
    __syncthreads();
    if (act) {
        const size_t ld = (size_t)n_cols * N2;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            R acc = 0;
#pragma unroll
            for (int a = 0; a < N; ++a) acc += sS[N2 + a * N + j] * st[c * N3 + k * N2 + a * N + i];
            T[((size_t)c * nzN + iz * N + k) * ld + (size_t)col * N2 + j * N + i] = acc;
        }
    }
}

// Backward x/y transform and update: x = (x or 0) + omega (Sx (x) Sy) X.
template <int N, typename R>
__global__ __launch_bounds__(nthreads<N>()) void k_col_bwd(int n_cols, int nzN, const R* __restrict__ S,
                                                           const R* __restrict__ X, R* __restrict__ x, R omega,
                                                           int accumulate) {
    constexpr int N2 = N * N, N3 = N2 * N;
    __shared__ R sr[3 * N3];
    __shared__ R st[3 * N3];
    __shared__ R sS[2 * N2];
    const int e = blockIdx.x, tid = threadIdx.x;
    const int col = e % n_cols, iz = e / n_cols;
    const size_t ld = (size_t)n_cols * N2;
    for (int q = tid; q < 3 * N3; q += blockDim.x) {
        const int c = q / N3, r = q % N3, kk = r / N2, ab = r % N2;
        sr[q] = X[((size_t)c * nzN + iz * N + kk) * ld + (size_t)col * N2 + ab];
    }
    for (int q = tid; q < 2 * N2; q += blockDim.x) sS[q] = S[(size_t)col * 2 * N2 + q];
    __syncthreads();
    const bool act = tid < N3;
    const int i = tid % N, j = (tid / N) % N, k = tid / N2;
    if (act) {  // y: st[c][k][j][a] = sum_b Sy[j][b] sr[c][k][b][a]
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            R acc = 0;
#pragma unroll
            for (int bb = 0; bb < N; ++bb) acc += sS[N2 + j * N + bb] * sr[c * N3 + k * N2 + bb * N + i];
            st[c * N3 + tid] = acc;
        }
    }
    __syncthreads();
    if (act) {
        const size_t base = (size_t)e * 3 * N3;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            R acc = 0;
#pragma unroll
            for (int a = 0; a < N; ++a) acc += sS[i * N + a] * st[c * N3 + k * N2 + j * N + a];
            const size_t o = base + c * N3 + tid;
            x[o] = (accumulate ? x[o] : R(0)) + omega * acc;
        }
    }
}

// ---- overlapping column patches ---------------------------------------------------
// A column's subdomain is its own N x N node grid extended by k node lines into
// every horizontal neighbour (and k x k corners of the diagonal neighbours):
// a P x P patch, P = N + 2k, in the column's own (xi, eta) orientation.
// pg[col][b * P + a] names the node feeding patch position (a, b) as
// src_col * N^2 + j * N + i, or -1 where the patch has no node (outside the
// domain, or a corner at a vertex that is not shared by four columns).

// Threads of a patch workgroup: a compile-time stride, so that the loops over a
// patch's values unroll and their loads are issued together.
constexpr int kOvlThreads = 256;

// Gather of r = b - Ax (or b) onto the patches and forward x/y transform:
// T[c][iz*N + k][col*P2 + b'*P + a'] = sum_{a,b} Sx[a][a'] Sy[b][b'] r_patch[c][k][b][a].
// P = N + 2 overlap is a template parameter: every index split below is by a
// compile-time constant and the transform loops unroll.
template <int N, int P, typename R>
__global__ __launch_bounds__(kOvlThreads) void k_ovl_fwd(int n_cols, int nzN, const int* __restrict__ pg,
                                                 const R* __restrict__ wsq, const R* __restrict__ S,
                                                 const R* __restrict__ b, const R* __restrict__ Ax,
                                                 R* __restrict__ T) {
    constexpr int N2 = N * N, N3 = N2 * N;
    extern __shared__ char smem[];
    constexpr int P2 = P * P, NP = 3 * N * P2;
    R* sr = reinterpret_cast<R*>(smem);
    R* st = sr + NP;
    R* sS = st + NP;
    const int e = blockIdx.x, tid = threadIdx.x;
    const int col = e % n_cols, iz = e / n_cols;
#pragma unroll
    for (int q = tid; q < 2 * P2; q += kOvlThreads) sS[q] = S[(size_t)col * 2 * P2 + q];
    // the gather in three phases (table entries, then every value load, then the
    // selects), so that a thread's loads are in flight together; items past NP
    // take the last item's indices and holes (src < 0) node 0's, and neither is stored
    auto gather = [&](auto has_ax) {
        constexpr bool HA = decltype(has_ax)::value;
        constexpr int IT = (NP + kOvlThreads - 1) / kOvlThreads;
        int src[IT];
#pragma unroll
        for (int t = 0; t < IT; ++t) {
            const int q = min(tid + t * kOvlThreads, NP - 1);
            src[t] = pg[(size_t)col * P2 + (q % (N * P2)) % P2];
        }
        R vb[IT], va[IT], vw[IT];
#pragma unroll
        for (int t = 0; t < IT; ++t) {
            const int q = min(tid + t * kOvlThreads, NP - 1);
            const int c = q / (N * P2), k = (q % (N * P2)) / P2, sc = max(src[t], 0);
            const size_t o = ((size_t)(iz * n_cols + sc / N2) * 3 + c) * N3 + k * N2 + sc % N2;
            vb[t] = b[o];
            if constexpr (HA) va[t] = Ax[o];
            vw[t] = wsq[sc];
        }
#pragma unroll
        for (int t = 0; t < IT; ++t) {
            const int q = tid + t * kOvlThreads;
            if (q < NP) sr[q] = src[t] >= 0 ? (HA ? vb[t] - va[t] : vb[t]) * vw[t] : R(0);
        }
    };
    if (Ax) gather(std::true_type{});
    else gather(std::false_type{});
    __syncthreads();
#pragma unroll
    for (int q = tid; q < NP; q += kOvlThreads) {  // x: st[c][k][b][a'] = sum_a Sx[a][a'] sr[c][k][b][a]
        const int row = q / P, a2 = q % P;
        R acc = 0;
#pragma unroll
        for (int a = 0; a < P; ++a) acc += sS[a * P + a2] * sr[row * P + a];
        st[q] = acc;
    }
    __syncthreads();
    const size_t ld = (size_t)n_cols * P2;
#pragma unroll
    for (int q = tid; q < NP; q += kOvlThreads) {  // y
        const int c = q / (N * P2), rem = q % (N * P2), k = rem / P2, ab = rem % P2, b2 = ab / P, a2 = ab % P;
        const R* sy = sS + P2;
        const R* src = st + (size_t)(c * N + k) * P2;
        R acc = 0;
#pragma unroll
        for (int bb = 0; bb < P; ++bb) acc += sy[bb * P + b2] * src[bb * P + a2];
        T[((size_t)c * nzN + iz * N + k) * ld + (size_t)col * P2 + ab] = acc;
    }
}

// Backward x/y transform in place: T[..][col*P2 + b*P + a] = sum Sx[a][a'] Sy[b][b'] T[..][b'*P + a'].
template <int N, int P, typename R>
__global__ __launch_bounds__(kOvlThreads) void k_ovl_bwd(int n_cols, int nzN, const R* __restrict__ S,
                                                 R* __restrict__ T) {
    extern __shared__ char smem[];
    constexpr int P2 = P * P, NP = 3 * N * P2;
    R* sr = reinterpret_cast<R*>(smem);
    R* st = sr + NP;
    R* sS = st + NP;
    const int e = blockIdx.x, tid = threadIdx.x;
    const int col = e % n_cols, iz = e / n_cols;
    const size_t ld = (size_t)n_cols * P2;
#pragma unroll
    for (int q = tid; q < 2 * P2; q += kOvlThreads) sS[q] = S[(size_t)col * 2 * P2 + q];
    {  // every load of the thread first (items past NP re-read the last one), then the stores
        constexpr int IT = (NP + kOvlThreads - 1) / kOvlThreads;
        R v[IT];
#pragma unroll
        for (int t = 0; t < IT; ++t) {
            const int q = min(tid + t * kOvlThreads, NP - 1);
            const int c = q / (N * P2), rem = q % (N * P2), k = rem / P2, ab = rem % P2;
            v[t] = T[((size_t)c * nzN + iz * N + k) * ld + (size_t)col * P2 + ab];
        }
#pragma unroll
        for (int t = 0; t < IT; ++t) {
            const int q = tid + t * kOvlThreads;
            if (q < NP) sr[q] = v[t];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = tid; q < NP; q += kOvlThreads) {  // y: st[c][k][b][a'] = sum_b' Sy[b][b'] sr[c][k][b'][a']
        const int row = q / P2, ab = q % P2, bb = ab / P, a2 = ab % P;
        const R* sy = sS + P2;
        const R* src = sr + (size_t)row * P2;
        R acc = 0;
#pragma unroll
        for (int b2 = 0; b2 < P; ++b2) acc += sy[bb * P + b2] * src[b2 * P + a2];
        st[q] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int q = tid; q < NP; q += kOvlThreads) {  // x
        const int c = q / (N * P2), rem = q % (N * P2), k = rem / P2, ab = rem % P2, aa = ab % P;
        const R* src = st + (size_t)q - aa;
        R acc = 0;
#pragma unroll
        for (int a2 = 0; a2 < P; ++a2) acc += sS[aa * P + a2] * src[a2];
        T[((size_t)c * nzN + iz * N + k) * ld + (size_t)col * P2 + ab] = acc;
    }
}

// Additive combination: every node sums the patch values of the (up to four)
// patches that hold it; ps[col][node][4] = patch_col * P2 + position, or -1.
// wsq = count^(-1/2) of the patches holding each node scales the gather and the
// sum alike, so the smoother stays symmetric while a node shared by four
// patches is not over-corrected four times.
template <int N, typename R>
__global__ __launch_bounds__(256) void k_ovl_sum(int n_cols, int n_z, int P, const int* __restrict__ ps,
                                                 const R* __restrict__ wsq, const R* __restrict__ T,
                                                 R* __restrict__ x, R omega, int accumulate) {
    constexpr int N2 = N * N, N3 = N2 * N;
    const size_t tot = (size_t)n_cols * n_z * 3 * N3;
    const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= tot) return;
    const int node = (int)(o % N2), k = (int)((o / N2) % N), c = (int)((o / N3) % 3);
    const size_t e = o / (3 * N3);
    const int col = (int)(e % n_cols), iz = (int)(e / n_cols);
    const int P2 = P * P, nzN = n_z * N;
    const R* row = T + ((size_t)c * nzN + iz * N + k) * (size_t)n_cols * P2;
    // the node's four slots in one 16-byte load (the workspace and every block in
    // it are 256-byte aligned), then the four values loaded together (an empty
    // slot re-reads position 0 and is not added)
    const int4 tab = *reinterpret_cast<const int4*>(ps + ((size_t)col * N2 + node) * 4);
    const int ts[4] = {tab.x, tab.y, tab.z, tab.w};
    R v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = row[max(ts[q], 0)];
    const R w = wsq[(size_t)col * N2 + node];
    const R x0 = accumulate ? x[o] : R(0);
    R acc = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (ts[q] >= 0) acc += v[q];
    x[o] = x0 + omega * w * acc;
}

// Batched (over the 3 components, blockIdx.z) product along z:
//   div = 1:  Y[i][m] = (sum_z V[z][i] T[z][m]) / (lz[i] + rx lx_a + ry ly_b)
//   div = 0:  T[z][m] =  sum_i V[z][i] Y[i][m]
// The left factor A [3][n][n] is read as A[k][row] in both: V itself for div = 1,
// its stored transpose for div = 0.  in/out [3][n][ncol], m = col*N2 + b*N + a,
// computed on the matrix cores: 16 x 16 x 4 MFMA blocks (FP64 or FP32
// inputs and accumulation).  A workgroup of four waves owns a 64 x 64 output
// tile, each wave a 32 x 32 quarter as 2 x 2 blocks; K is staged through LDS in
// chunks of 32, the next chunk fetched into registers during the products, and
// the eigenvalue denominators of the lane's outputs are fetched before the first
// chunk so that the division does not wait on memory after the last one.
// Lane l of a block holds A[l % 16][l / 16] and B[l / 16][l % 16];
// its four results are C[row(l, q)][l % 16], q = 0..3, with row = 4 (l / 16) + q
// for the FP32 instruction and row = 4 q + l / 16 for the FP64 one (measured).
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
template <typename R> struct MfmaAcc;
template <> struct MfmaAcc<double> {
    using type = d4_t;
    __device__ static type step(double a, double b, type c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int q) { return 4 * q + lane / 16; }
};
template <> struct MfmaAcc<float> {
    using type = f4_t;
    __device__ static type step(float a, float b, type c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int q) { return 4 * (lane / 16) + q; }
};

constexpr int kGK = 32, kGPad = 4;
// W: patch width (the eigenvalue division splits the column index by W and W^2,
// compile-time constants here); div = 0 takes W = 0.
// waves per SIMD asked of the compiler: five in FP32 (96 registers; four would
// leave 2400 workgroups of the forty-layer level in three rounds of 1024), three in FP64
template <typename R>
constexpr int gemm_waves() {
    return sizeof(R) == 4 ? 5 : 3;
}

// T: the workgroup's output tile, T x T (64, or 32 on the small coarse levels,
// whose 64 x 64 grids would leave most compute units idle: measured at M = K =
// 200 and 1280 / 320 columns, 11.7 -> 10.7 and 11.1 -> 5.7 us); each of the four
// waves takes a (T/2) x (T/2) quarter in 16 x 16 MFMA blocks.
template <typename R, int W, int div, int T>
__global__ __launch_bounds__(256, gemm_waves<R>()) void k_col_gemm_mfma(int n, int ncol, const R* __restrict__ A,
                                                       const R* __restrict__ in, R* __restrict__ out,
                                                       const R* __restrict__ lz, const R* __restrict__ lam,
                                                       const R* __restrict__ rat) {
    using Acc = MfmaAcc<R>;
    constexpr int kGM = T, kGN = T, BL = T / 32;  // BL x BL blocks per wave
    constexpr int LA = kGK * kGM / 256, LB = kGK * kGN / 256;  // staged values per thread
    __shared__ R As[kGK][kGM + kGPad];  // As[k][row]
    __shared__ R Bs[kGK][kGN + kGPad];  // Bs[k][col]
    const int c = blockIdx.z;
    const int row0 = blockIdx.y * kGM, col0 = blockIdx.x * kGN;
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wr = (wave / 2) * (T / 2), wc = (wave % 2) * (T / 2);
    const R* Ac = A + (size_t)c * n * n;
    const R* Bc = in + (size_t)c * n * ncol;
    // the next K chunk is fetched into registers while the current one is
    // multiplied: every load reads a clamped (valid) index, and the values
    // outside the matrices are zeroed only when stored to LDS, after the
    // products, so that no select waits on a load in flight (zeroing at the
    // load made the kernel 1.8x slower; per-load branches cost 8 %)
    R ra[LA], rb[LB];
    bool va[LA], vb[LB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < LA; ++t) {
            const int q = tid + 256 * t;
            const int kg = k0 + q / kGM, rg = row0 + q % kGM;
            ra[t] = Ac[(size_t)min(kg, n - 1) * n + min(rg, n - 1)];
            va[t] = kg < n && rg < n;
        }
#pragma unroll
        for (int t = 0; t < LB; ++t) {
            const int q = tid + 256 * t;
            const int kg = k0 + q / kGN, cg = col0 + q % kGN;
            rb[t] = Bc[(size_t)min(kg, n - 1) * ncol + min(cg, ncol - 1)];
            vb[t] = kg < n && cg < ncol;
        }
    };
    typename Acc::type acc[BL][BL];
#pragma unroll
    for (int a = 0; a < BL; ++a)
#pragma unroll
        for (int b = 0; b < BL; ++b) acc[a][b] = typename Acc::type{0, 0, 0, 0};
    fetch(0);
    // in-plane part of the denominators of this lane's outputs, whose table reads
    // depend on one another, fetched before the K loop (indices clamped: outputs
    // past n or ncol are computed but not stored); the z-eigenvalues, single
    // loads, are read after it, which keeps the registers at five waves per SIMD
    R lxy[BL];
    if constexpr (div) {
        constexpr int W2 = W * W;
#pragma unroll
        for (int b = 0; b < BL; ++b) {
            const int cg = min(col0 + wc + 16 * b + lane % 16, ncol - 1);
            const int colm = cg / W2, ab = cg % W2, bb = ab / W, aa = ab % W;
            lxy[b] = rat[(size_t)colm * 6 + c * 2 + 0] * lam[((size_t)colm * 2 + 0) * W + aa] +
                     rat[(size_t)colm * 6 + c * 2 + 1] * lam[((size_t)colm * 2 + 1) * W + bb];
        }
    }
    for (int k0 = 0; k0 < n; k0 += kGK) {
#pragma unroll
        for (int t = 0; t < LA; ++t) {
            const int q = tid + 256 * t;
            As[q / kGM][q % kGM] = va[t] ? ra[t] : R(0);
        }
#pragma unroll
        for (int t = 0; t < LB; ++t) {
            const int q = tid + 256 * t;
            Bs[q / kGN][q % kGN] = vb[t] ? rb[t] : R(0);
        }
        __syncthreads();
        if (k0 + kGK < n) fetch(k0 + kGK);
        // fragments of the next K step read from LDS while this step's products run
        R af[2][BL], bf[2][BL];
#pragma unroll
        for (int a = 0; a < BL; ++a) af[0][a] = As[lane / 16][wr + 16 * a + lane % 16];
#pragma unroll
        for (int b = 0; b < BL; ++b) bf[0][b] = Bs[lane / 16][wc + 16 * b + lane % 16];
#pragma unroll
        for (int ks = 0; ks < kGK; ks += 4) {
            const int cur = (ks / 4) & 1, nx = cur ^ 1;
            if (ks + 4 < kGK) {
#pragma unroll
                for (int a = 0; a < BL; ++a) af[nx][a] = As[ks + 4 + lane / 16][wr + 16 * a + lane % 16];
#pragma unroll
                for (int b = 0; b < BL; ++b) bf[nx][b] = Bs[ks + 4 + lane / 16][wc + 16 * b + lane % 16];
            }
#pragma unroll
            for (int a = 0; a < BL; ++a)
#pragma unroll
                for (int b = 0; b < BL; ++b) acc[a][b] = Acc::step(af[cur][a], bf[cur][b], acc[a][b]);
        }
        __syncthreads();
    }
    R* Oc = out + (size_t)c * n * ncol;
#pragma unroll
    for (int a = 0; a < BL; ++a)
#pragma unroll
        for (int b = 0; b < BL; ++b) {
            const int cg = col0 + wc + 16 * b + lane % 16;
            if (cg >= ncol) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rg = row0 + wr + 16 * a + Acc::row(lane, q);
                if (rg >= n) continue;
                R v = acc[a][b][q];
                if constexpr (div) v /= lz[(size_t)c * n + rg] + lxy[b];
                Oc[(size_t)rg * ncol + cg] = v;
            }
        }
}

// The FP32 z-products on split bf16: each operand x is held as hi + lo, two
// bf16 numbers (hi = bf16(x), lo = bf16(x - hi), about 16 significant bits
// together, and bf16 has FP32's exponent range), and a block product is
// lo*hi + hi*lo + hi*hi on 16 x 16 x 16 bf16 MFMA with FP32 accumulation (the
// lo*lo term, 2^-16 smaller, is left out).  Three bf16 instructions take about a
// fifth of the matrix-core time of the FP32 instructions for the same K, and
// the smoother is a preconditioner: solves with operands rounded to this
// precision took the same iterations and gave the same energies as FP32 (forty
// layers and thin coating, every tolerance).  64 x 64 output tiles, K chunks of
// 32 split once when staged; in LDS each row keeps its 32 k (72-byte stride), so
// a lane's four k of a fragment are one 8-byte read.  The eigenvalue division
// and the clamped, deferred-zeroing fetch are those of k_col_gemm_mfma.
constexpr int kBfRow = 36;  // bf16 per staged row: 32 k and 4 of padding

__device__ __forceinline__ void split_bf16(float x, unsigned short& hi, unsigned short& lo) {
    const __bf16 h = (__bf16)x;
    const __bf16 l = (__bf16)(x - (float)h);
    hi = __builtin_bit_cast(unsigned short, h);
    lo = __builtin_bit_cast(unsigned short, l);
}

template <int W, int div>
__global__ __launch_bounds__(256) void k_col_gemm_bf3(int n, int ncol, const float* __restrict__ A,
                                                      const float* __restrict__ in, float* __restrict__ out,
                                                      const float* __restrict__ lz, const float* __restrict__ lam,
                                                      const float* __restrict__ rat) {
    typedef short s4_t __attribute__((ext_vector_type(4)));
    constexpr int TM = 64, TN = 64, PA = kGK * TM / 512, PB = kGK * TN / 512;
    __shared__ __attribute__((aligned(16))) unsigned short Ah[TM * kBfRow], Al[TM * kBfRow], Bh[TN * kBfRow],
        Bl[TN * kBfRow];
    const int c = blockIdx.z, row0 = blockIdx.y * TM, col0 = blockIdx.x * TN;
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wr = (wave / 2) * 32, wc = (wave % 2) * 32;
    const int g4 = 4 * (lane / 16), l16 = lane % 16;
    const float* Ac = A + (size_t)c * n * n;
    const float* Bc = in + (size_t)c * n * ncol;
    float ra[PA][2], rb[PB][2];
    bool va[PA][2], vb[PB][2];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < PA; ++t) {
            const int q = tid + 256 * t, rg = row0 + q % TM, kp = k0 + 2 * (q / TM);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                ra[t][h] = Ac[(size_t)min(kp + h, n - 1) * n + min(rg, n - 1)];
                va[t][h] = kp + h < n && rg < n;
            }
        }
#pragma unroll
        for (int t = 0; t < PB; ++t) {
            const int q = tid + 256 * t, cg = col0 + q % TN, kp = k0 + 2 * (q / TN);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                rb[t][h] = Bc[(size_t)min(kp + h, n - 1) * ncol + min(cg, ncol - 1)];
                vb[t][h] = kp + h < n && cg < ncol;
            }
        }
    };
    auto stage = [](float x0, float x1, unsigned short* hi, unsigned short* lo, int o) {
        unsigned short h0, l0, h1, l1;
        split_bf16(x0, h0, l0);
        split_bf16(x1, h1, l1);
        *reinterpret_cast<unsigned*>(&hi[o]) = h0 | ((unsigned)h1 << 16);
        *reinterpret_cast<unsigned*>(&lo[o]) = l0 | ((unsigned)l1 << 16);
    };
    f4_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f4_t{0, 0, 0, 0};
    fetch(0);
    float lxy[2];
    if constexpr (div) {
        constexpr int W2 = W * W;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int cg = min(col0 + wc + 16 * b + l16, ncol - 1);
            const int colm = cg / W2, ab = cg % W2, bb = ab / W, aa = ab % W;
            lxy[b] = rat[(size_t)colm * 6 + c * 2 + 0] * lam[((size_t)colm * 2 + 0) * W + aa] +
                     rat[(size_t)colm * 6 + c * 2 + 1] * lam[((size_t)colm * 2 + 1) * W + bb];
        }
    }
    for (int k0 = 0; k0 < n; k0 += kGK) {
#pragma unroll
        for (int t = 0; t < PA; ++t) {
            const int q = tid + 256 * t;
            stage(va[t][0] ? ra[t][0] : 0.f, va[t][1] ? ra[t][1] : 0.f, Ah, Al, (q % TM) * kBfRow + 2 * (q / TM));
        }
#pragma unroll
        for (int t = 0; t < PB; ++t) {
            const int q = tid + 256 * t;
            stage(vb[t][0] ? rb[t][0] : 0.f, vb[t][1] ? rb[t][1] : 0.f, Bh, Bl, (q % TN) * kBfRow + 2 * (q / TN));
        }
        __syncthreads();
        if (k0 + kGK < n) fetch(k0 + kGK);
#pragma unroll
        for (int ks = 0; ks < kGK; ks += 16) {
            s4_t ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int o = (wr + 16 * a + l16) * kBfRow + ks + g4;
                ah[a] = *reinterpret_cast<const s4_t*>(&Ah[o]);
                al[a] = *reinterpret_cast<const s4_t*>(&Al[o]);
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int o = (wc + 16 * b + l16) * kBfRow + ks + g4;
                bh[b] = *reinterpret_cast<const s4_t*>(&Bh[o]);
                bl[b] = *reinterpret_cast<const s4_t*>(&Bl[o]);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[a], bh[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[a], bl[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[a], bh[b], acc[a][b], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    float* Oc = out + (size_t)c * n * ncol;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int cg = col0 + wc + 16 * b + l16;
            if (cg >= ncol) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rg = row0 + wr + 16 * a + g4 + q;  // the 16 x 16 output layout of the FP32 instruction
                if (rg >= n) continue;
                float v = acc[a][b][q];
                if constexpr (div) v /= lz[(size_t)c * n + rg] + lxy[b];
                Oc[(size_t)rg * ncol + cg] = v;
            }
        }
}

// Fine += P coarse over the same elements, P = I (x) I (x) I with I [Nf][Nc].
// NF, NC: the sizes as compile-time constants (the pairs p -> max(1, p / 2)
// produces), or 0 to take them from the arguments.
template <typename R, int NF, int NC>
__global__ void k_prolong_p(int E, int Nf_, int Nc_, const R* __restrict__ I, const R* __restrict__ uc,
                            R* __restrict__ uf) {
    __shared__ R s[3 * kMaxN * kMaxN * kMaxN];
    __shared__ R t[3 * kMaxN * kMaxN * kMaxN];
    __shared__ R sI[kMaxN * kMaxN];
    const int Nf = NF ? NF : Nf_, Nc = NC ? NC : Nc_;
    const int e = blockIdx.x, tid = threadIdx.x;
    const int Nc3 = Nc * Nc * Nc, Nf3 = Nf * Nf * Nf;
    for (int q = tid; q < 3 * Nc3; q += blockDim.x) s[q] = uc[(size_t)e * 3 * Nc3 + q];
    for (int q = tid; q < Nf * Nc; q += blockDim.x) sI[q] = I[q];
    __syncthreads();
    // x: [c][kc][jc][if]
    for (int q = tid; q < 3 * Nc * Nc * Nf; q += blockDim.x) {
        const int a = q % Nf, jc = (q / Nf) % Nc, kc = (q / (Nf * Nc)) % Nc, c = q / (Nf * Nc * Nc);
        R acc = 0;
        for (int b = 0; b < Nc; ++b) acc += sI[a * Nc + b] * s[c * Nc3 + kc * Nc * Nc + jc * Nc + b];
        t[q] = acc;
    }
    __syncthreads();
    // y: [c][kc][jf][if]
    for (int q = tid; q < 3 * Nc * Nf * Nf; q += blockDim.x) {
        const int a = q % Nf, jf = (q / Nf) % Nf, kc = (q / (Nf * Nf)) % Nc, c = q / (Nf * Nf * Nc);
        R acc = 0;
        for (int b = 0; b < Nc; ++b) acc += sI[jf * Nc + b] * t[((c * Nc + kc) * Nc + b) * Nf + a];
        s[q] = acc;
    }
    __syncthreads();
    for (int q = tid; q < 3 * Nf3; q += blockDim.x) {
        const int a = q % Nf, jf = (q / Nf) % Nf, kf = (q / (Nf * Nf)) % Nf, c = q / Nf3;
        R acc = 0;
        for (int b = 0; b < Nc; ++b) acc += sI[kf * Nc + b] * s[((c * Nc + b) * Nf + jf) * Nf + a];
        uf[(size_t)e * 3 * Nf3 + q] += acc;
    }
}

// Coarse = P^T fine.
template <typename R, int NF, int NC>
__global__ void k_restrict_p(int E, int Nf_, int Nc_, const R* __restrict__ I, const R* __restrict__ rf,
                             R* __restrict__ rc) {
    __shared__ R s[3 * kMaxN * kMaxN * kMaxN];
    __shared__ R t[3 * kMaxN * kMaxN * kMaxN];
    __shared__ R sI[kMaxN * kMaxN];
    const int Nf = NF ? NF : Nf_, Nc = NC ? NC : Nc_;
    const int e = blockIdx.x, tid = threadIdx.x;
    const int Nc3 = Nc * Nc * Nc, Nf3 = Nf * Nf * Nf;
    for (int q = tid; q < 3 * Nf3; q += blockDim.x) s[q] = rf[(size_t)e * 3 * Nf3 + q];
    for (int q = tid; q < Nf * Nc; q += blockDim.x) sI[q] = I[q];
    __syncthreads();
    // x: [c][kf][jf][ic]
    for (int q = tid; q < 3 * Nf * Nf * Nc; q += blockDim.x) {
        const int a = q % Nc, jf = (q / Nc) % Nf, kf = (q / (Nc * Nf)) % Nf, c = q / (Nc * Nf * Nf);
        R acc = 0;
        for (int b = 0; b < Nf; ++b) acc += sI[b * Nc + a] * s[c * Nf3 + kf * Nf * Nf + jf * Nf + b];
        t[q] = acc;
    }
    __syncthreads();
    // y: [c][kf][jc][ic]
    for (int q = tid; q < 3 * Nf * Nc * Nc; q += blockDim.x) {
        const int a = q % Nc, jc = (q / Nc) % Nc, kf = (q / (Nc * Nc)) % Nf, c = q / (Nc * Nc * Nf);
        R acc = 0;
        for (int b = 0; b < Nf; ++b) acc += sI[b * Nc + jc] * t[((c * Nf + kf) * Nf + b) * Nc + a];
        s[q] = acc;
    }
    __syncthreads();
    for (int q = tid; q < 3 * Nc3; q += blockDim.x) {
        const int a = q % Nc, jc = (q / Nc) % Nc, kc = (q / (Nc * Nc)) % Nc, c = q / Nc3;
        R acc = 0;
        for (int b = 0; b < Nf; ++b) acc += sI[b * Nc + kc] * s[((c * Nf + b) * Nc + jc) * Nc + a];
        rc[(size_t)e * 3 * Nc3 + q] = acc;
    }
}

// h-transfers.  Ih [2][N][N]: Ih[s][a][b] = l_b(child-s node a in parent coordinates).
// Fine element e_f = iz * ncf + colf; parent[colf] = coarse column, child[colf] = sx + 2 sy.
template <typename R, int NT>
__global__ void k_prolong_h(int N_, int ncf, int ncc, const int* __restrict__ parent,
                            const int* __restrict__ child, const R* __restrict__ Ih, const R* __restrict__ uc,
                            R* __restrict__ uf) {
    const int N = NT ? NT : N_;  // NT: N as a compile-time constant, or 0
    const int ef = blockIdx.x, tid = threadIdx.x;
    const int colf = ef % ncf, iz = ef / ncf;
    const int ec = iz * ncc + parent[colf];
    const int sx = child[colf] & 1, sy = child[colf] >> 1;
    const int N2 = N * N, N3 = N2 * N;
    const R* Ix = Ih + sx * N2;
    const R* Iy = Ih + sy * N2;
    for (int q = tid; q < 3 * N3; q += blockDim.x) {
        const int i = q % N, j = (q / N) % N, k = (q / N2) % N, c = q / N3;
        const R* src = uc + (size_t)ec * 3 * N3 + c * N3 + k * N2;
        R acc = 0;
        for (int b = 0; b < N; ++b) {
            R row = 0;
            for (int a = 0; a < N; ++a) row += Ix[i * N + a] * src[b * N + a];
            acc += Iy[j * N + b] * row;
        }
        uf[(size_t)ef * 3 * N3 + q] += acc;
    }
}

// Transfers between a level and its z-coarsened level (each column's z-elements
// merged in pairs; an unpaired last element is carried over).  Iz[izf][k][kk] is
// coarse basis function kk at node k of fine z-element izf, zpar[izf] its coarse
// element, zch[izc][2] the fine elements of coarse element izc (-1 if none).
template <typename R, int NT>
__global__ void k_prolong_z(int N_, int n_cols, const int* __restrict__ zpar, const R* __restrict__ Iz,
                            const R* __restrict__ uc, R* __restrict__ uf) {
    const int N = NT ? NT : N_;  // NT: N as a compile-time constant, or 0
    const int ef = blockIdx.x, tid = threadIdx.x;
    const int col = ef % n_cols, izf = ef / n_cols;
    const size_t ec = (size_t)zpar[izf] * n_cols + col;
    const int N2 = N * N, N3 = N2 * N;
    const R* I = Iz + (size_t)izf * N2;
    for (int q = tid; q < 3 * N3; q += blockDim.x) {
        const int ij = q % N2, k = (q / N2) % N, c = q / N3;
        const R* src = uc + ec * 3 * N3 + c * N3 + ij;
        R acc = 0;
        for (int kk = 0; kk < N; ++kk) acc += I[k * N + kk] * src[kk * N2];
        uf[(size_t)ef * 3 * N3 + q] += acc;
    }
}

template <typename R, int NT>
__global__ void k_restrict_z(int N_, int n_cols, const int* __restrict__ zch, const R* __restrict__ Iz,
                             const R* __restrict__ rf, R* __restrict__ rc) {
    const int N = NT ? NT : N_;  // NT: N as a compile-time constant, or 0
    const int ec = blockIdx.x, tid = threadIdx.x;
    const int col = ec % n_cols, izc = ec / n_cols;
    const int N2 = N * N, N3 = N2 * N;
    for (int q = tid; q < 3 * N3; q += blockDim.x) {
        const int ij = q % N2, kk = (q / N2) % N, c = q / N3;
        R acc = 0;
        for (int s = 0; s < 2; ++s) {
            const int izf = zch[izc * 2 + s];
            if (izf < 0) continue;
            const R* I = Iz + (size_t)izf * N2;
            const R* src = rf + ((size_t)izf * n_cols + col) * 3 * N3 + c * N3 + ij;
            for (int k = 0; k < N; ++k) acc += I[k * N + kk] * src[k * N2];
        }
        rc[(size_t)ec * 3 * N3 + q] = acc;
    }
}

template <typename R, int NT>
__global__ void k_restrict_h(int N_, int ncf, int ncc, const int* __restrict__ children,
                             const R* __restrict__ Ih, const R* __restrict__ rf, R* __restrict__ rc) {
    const int N = NT ? NT : N_;  // NT: N as a compile-time constant, or 0
    const int ec = blockIdx.x, tid = threadIdx.x;
    const int colc = ec % ncc, iz = ec / ncc;
    const int N2 = N * N, N3 = N2 * N;
    for (int q = tid; q < 3 * N3; q += blockDim.x) {
        const int ic = q % N, jc = (q / N) % N, k = (q / N2) % N, c = q / N3;
        R acc = 0;
        for (int s = 0; s < 4; ++s) {
            const int ef = iz * ncf + children[colc * 4 + s];
            const R* Ix = Ih + (s & 1) * N2;
            const R* Iy = Ih + (s >> 1) * N2;
            const R* src = rf + (size_t)ef * 3 * N3 + c * N3 + k * N2;
            for (int j = 0; j < N; ++j) {
                R row = 0;
                for (int i = 0; i < N; ++i) row += Ix[i * N + ic] * src[j * N + i];
                acc += Iy[j * N + jc] * row;
            }
        }
        rc[(size_t)ec * 3 * N3 + q] = acc;
    }
}

// ---- dense coarse solve ------------------------------------------------------

__global__ void k_set_unit(double* e, int j) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (j > 0) e[j - 1] = 0.0;
        e[j] = 1.0;
    }
}

// Blocked Gauss-Jordan inversion in place of the n x n SPD matrix A, without
// pivoting (the Schur complements of an SPD matrix stay SPD), in column blocks
// K = [k0, k0 + b) of width b <= kGJB:
//   P = A_KK^-1,  R = P A_K*,  A_ij -= A_iK R_j (i, j not in K),
//   A_iK = -A_iK P (i not in K),  A_K* = R (A_KK = P).
constexpr int kGJB = 32;

// P = inverse of the diagonal block, by unpivoted Gauss-Jordan in LDS (one workgroup).
__global__ __launch_bounds__(256) void k_gjb_diag(const double* __restrict__ A, int n, int k0, int b,
                                                  double* __restrict__ P) {
    __shared__ double M[kGJB][kGJB + 1];
    __shared__ double pivrow[kGJB];
    __shared__ double pivcol[kGJB];
    const int tid = threadIdx.x;
    for (int q = tid; q < b * b; q += blockDim.x) M[q / b][q % b] = A[(size_t)(k0 + q / b) * n + k0 + q % b];
    __syncthreads();
    for (int p = 0; p < b; ++p) {
        const double inv = 1.0 / M[p][p];
        if (tid < b) {
            pivrow[tid] = tid == p ? inv : M[p][tid] * inv;
            pivcol[tid] = M[tid][p];
        }
        __syncthreads();
        for (int q = tid; q < b * b; q += blockDim.x) {
            const int i = q / b, j = q % b;
            if (i == p) M[i][j] = pivrow[j];
            else if (j == p) M[i][j] = -pivcol[i] * inv;
            else M[i][j] -= pivcol[i] * pivrow[j];
        }
        __syncthreads();
    }
    for (int q = tid; q < b * b; q += blockDim.x) P[q] = M[q / b][q % b];
}

// R[t][j] = sum_s P[t][s] A[k0 + s][j], all columns j (R is b x n); one lane per (t, j).
__global__ __launch_bounds__(256) void k_gjb_row(const double* __restrict__ A, int n, int k0, int b,
                                                 const double* __restrict__ P, double* __restrict__ R) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (size_t)b * n) return;
    const int t = (int)(q / n), jj = (int)(q % n);
    double acc = 0;
    for (int s2 = 0; s2 < b; ++s2) acc += P[t * b + s2] * A[(size_t)(k0 + s2) * n + jj];
    R[q] = acc;
}

// A_ij -= sum_t A[i][k0 + t] R[t][j] for i, j outside K: 64 x 64 tiles, 4 x 4 per lane.
__global__ __launch_bounds__(256) void k_gjb_update(double* __restrict__ A, int n, int k0, int b,
                                                    const double* __restrict__ R) {
    __shared__ double Ls[kGJB][64 + 1];  // Ls[t][row]
    __shared__ double Rs[kGJB][64 + 1];  // Rs[t][col]
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64, tid = threadIdx.x;
    for (int q = tid; q < 64 * b; q += blockDim.x) {
        const int r = q / b, t = q % b, i = i0 + r;
        Ls[t][r] = i < n ? A[(size_t)i * n + k0 + t] : 0.0;
    }
    for (int q = tid; q < 64 * b; q += blockDim.x) {
        const int t = q / 64, cidx = q % 64, j = j0 + cidx;
        Rs[t][cidx] = j < n ? R[(size_t)t * n + j] : 0.0;
    }
    __syncthreads();
    const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
    double acc[4][4] = {};
    for (int t = 0; t < b; ++t) {
        double l[4], r[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            l[a] = Ls[t][tr + a];
            r[a] = Rs[t][tc + a];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][c] += l[a] * r[c];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = i0 + tr + a;
        if (i >= n || (i >= k0 && i < k0 + b)) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = j0 + tc + c;
            if (j >= n || (j >= k0 && j < k0 + b)) continue;
            A[(size_t)i * n + j] -= acc[a][c];
        }
    }
}

// C[i][t] = -sum_s A[i][k0 + s] P[s][t] (the new column block, rows outside K);
// one lane per (i, t), written to C so that A's column block stays intact until stored.
__global__ __launch_bounds__(256) void k_gjb_col(const double* __restrict__ A, int n, int k0, int b,
                                                 const double* __restrict__ P, double* __restrict__ C) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (size_t)n * b) return;
    const int i = (int)(q / b), t = (int)(q % b);
    if (i >= k0 && i < k0 + b) return;
    double acc = 0;
    for (int s2 = 0; s2 < b; ++s2) acc += A[(size_t)i * n + k0 + s2] * P[s2 * b + t];
    C[q] = -acc;
}

// Column block K of the other rows = C; row block K = R, with A_KK = P.
__global__ __launch_bounds__(256) void k_gjb_store(double* __restrict__ A, int n, int k0, int b,
                                                   const double* __restrict__ R, const double* __restrict__ P,
                                                   const double* __restrict__ C) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < (size_t)n * b) {  // column block, one lane per (i, t)
        const int i = (int)(q / b), t = (int)(q % b);
        if (i < k0 || i >= k0 + b) A[(size_t)i * n + k0 + t] = C[q];
    } else if (q < (size_t)2 * n * b) {  // row block, one lane per (t, j)
        const size_t r = q - (size_t)n * b;
        const int t = (int)(r / n), jj = (int)(r % n);
        const bool inK = jj >= k0 && jj < k0 + b;
        A[(size_t)(k0 + t) * n + jj] = inK ? P[t * b + (jj - k0)] : R[r];
    }
}

// y = A x, one 64-lane wave per row, fixed-order reduction.  VEC: 16-byte loads
// (the host takes this form only when n is a multiple of 16 / sizeof(R) and A
// and x are 16-byte aligned, so that every row starts on a 16-byte boundary),
// four loads per lane in flight on four accumulators.
template <typename R, bool VEC>
__global__ __launch_bounds__(256) void k_gemv(const R* __restrict__ A, const R* __restrict__ x, R* __restrict__ y,
                                              int n) {
    const int row = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (row >= n) return;
    const R* a = A + (size_t)row * n;
    R acc[4] = {0, 0, 0, 0};
    if constexpr (VEC) {
        constexpr int V = 16 / sizeof(R);
        typedef R vec_t __attribute__((ext_vector_type(V)));
        const vec_t* av = reinterpret_cast<const vec_t*>(a);
        const vec_t* xv = reinterpret_cast<const vec_t*>(x);
        const int nv = n / V;
        int j = lane;
        for (; j + 192 < nv; j += 256) {
            vec_t p[4], q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                p[u] = av[j + 64 * u];
                q[u] = xv[j + 64 * u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int t = 0; t < V; ++t) acc[u] += p[u][t] * q[u][t];
        }
        for (; j < nv; j += 64) {
            const vec_t p = av[j], q = xv[j];
#pragma unroll
            for (int t = 0; t < V; ++t) acc[0] += p[t] * q[t];
        }
    } else {
        for (int j = lane; j < n; j += 64) acc[0] += a[j] * x[j];
    }
    R r = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    for (int off = 32; off > 0; off >>= 1) r += __shfl_xor(r, off);
    if (lane == 0) y[row] = r;
}

template <typename R>
__global__ void k_zero(R* x, size_t n) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) x[q] = R(0);
}

template <typename A, typename B>
__global__ void k_cast(const A* __restrict__ x, B* __restrict__ y, size_t n, double scale) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) y[q] = (B)((double)x[q] * scale);
}

// y = b - y
template <typename R>
__global__ void k_resid(const R* __restrict__ b, R* __restrict__ y, size_t n) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) y[q] = b[q] - y[q];
}

// partial[v][blk] = sum over the block's slice of V_v . w, for v < nv; the
// last slot (v == nv) holds w . w.  Fixed order: deterministic.
constexpr int kDotThreads = 256;
__global__ __launch_bounds__(kDotThreads) void k_multidot(const double* __restrict__ V, size_t ldv, int nv,
                                                          const double* __restrict__ w, size_t n,
                                                          double* __restrict__ partial, int nblk) {
    __shared__ double red[kDotThreads];
    const int tid = threadIdx.x;
    const size_t chunk = (n + nblk - 1) / nblk;
    const size_t lo = (size_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
    for (int v = 0; v <= nv; ++v) {
        const double* a = (v < nv) ? V + (size_t)v * ldv : w;
        double acc = 0;
        for (size_t q = lo + tid; q < hi; q += kDotThreads) acc += a[q] * w[q];
        red[tid] = acc;
        __syncthreads();
        for (int s = kDotThreads / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        if (tid == 0) partial[(size_t)v * nblk + blockIdx.x] = red[0];
        __syncthreads();
    }
}

// out[v] = sum_b partial[v][b]: one workgroup per vector, strided loads then a
// tree in LDS (fixed order, so the result is deterministic).
__global__ __launch_bounds__(kDotThreads) void k_reduce_partials(const double* __restrict__ partial, int nblk,
                                                                 double* __restrict__ out) {
    __shared__ double red[kDotThreads];
    const int v = blockIdx.x, tid = threadIdx.x;
    double acc = 0;
    for (int b = tid; b < nblk; b += kDotThreads) acc += partial[(size_t)v * nblk + b];
    red[tid] = acc;
    __syncthreads();
    for (int st = kDotThreads / 2; st > 0; st >>= 1) {
        if (tid < st) red[tid] += red[tid + st];
        __syncthreads();
    }
    if (tid == 0) out[v] = red[0];
}

// Flexible-CG steps with the scalars kept on the device (no host round trip):
// sc[0] = p.Ap, sc[1] = breakdown flag; cur[0] = r.z of this iteration.
// u += alpha p, r -= alpha Ap with alpha = cur[0] / sc[0]; a non-positive p.Ap
// skips the update and raises the flag for the host to act on.  r32, if not
// null, receives the new residual rounded to FP32 (the FP32 preconditioner's
// input, written here instead of by a separate pass).
__global__ void k_fcg_update(double* __restrict__ u, double* __restrict__ r, const double* __restrict__ p,
                             const double* __restrict__ q, const double* __restrict__ cur,
                             double* __restrict__ sc, float* __restrict__ r32, double scale32, size_t n) {
    const double pq = sc[0];
    const bool ok = pq > 0;
    const double alpha = ok ? cur[0] / pq : 0.0;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!ok && t == 0) sc[1] = 1.0;
    if (t >= n) return;
    u[t] += alpha * p[t];
    const double rn = r[t] - alpha * q[t];
    r[t] = rn;
    if (r32) r32[t] = (float)(scale32 * rn);  // a power of two: keeps the FP32 input in range
}

// p = z + beta p, beta = (nxt[0] - nxt[1]) / cur[0]  (Polak-Ribiere)
__global__ void k_fcg_direction(double* __restrict__ p, const double* __restrict__ z,
                                const double* __restrict__ cur, const double* __restrict__ nxt, size_t n) {
    const double beta = (nxt[0] - nxt[1]) / cur[0];
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = z[t] + beta * p[t];
}

// w += sum_v coef[v] V_v   (coef on the device)
__global__ void k_multiaxpy(double* __restrict__ w, const double* __restrict__ V, size_t ldv, int nv,
                            const double* __restrict__ coef, size_t n) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double acc = w[q];
    for (int v = 0; v < nv; ++v) acc += coef[v] * V[(size_t)v * ldv + q];
    w[q] = acc;
}

__global__ void k_scale_copy(const double* __restrict__ x, double* __restrict__ y, double s, size_t n) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) y[q] = s * x[q];
}

// y += a x
__global__ void k_axpy(double* __restrict__ y, double a, const double* __restrict__ x, size_t n) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) y[q] += a * x[q];
}

// p = z + beta p
__global__ void k_xpby(double* __restrict__ p, const double* __restrict__ z, double beta, size_t n) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) p[q] = z[q] + beta * p[q];
}

struct DotPairs {
    const double* x[4];
    const double* y[4];
    int np;
};

// partial[v][blk] = x_v . y_v over the block's slice (fixed order): the NP
// pairs are read in one pass, then reduced across each wave by shuffles and
// across the block's waves in wave order.
template <int NP>
__global__ __launch_bounds__(kDotThreads) void k_dotpairs(DotPairs d, size_t n, double* __restrict__ partial,
                                                          int nblk) {
    constexpr int NW = kDotThreads / 64;
    __shared__ double red[NP][NW];
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const size_t chunk = (n + nblk - 1) / nblk;
    const size_t lo = (size_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
    double acc[NP];
#pragma unroll
    for (int v = 0; v < NP; ++v) acc[v] = 0;
#pragma unroll 4
    for (size_t q = lo + tid; q < hi; q += kDotThreads)
#pragma unroll
        for (int v = 0; v < NP; ++v) acc[v] += d.x[v][q] * d.y[v][q];
#pragma unroll
    for (int v = 0; v < NP; ++v) {
        double r = acc[v];
        for (int off = 32; off > 0; off >>= 1) r += __shfl_xor(r, off);
        if (lane == 0) red[v][wave] = r;
    }
    __syncthreads();
    if (tid < NP) {
        double r = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) r += red[tid][w];
        partial[(size_t)tid * nblk + blockIdx.x] = r;
    }
}

// The three dot products of a flexible-CG step with an FP32 preconditioner:
// zn = unscale * (double) z32 is written here (the widening pass folded in), and
// partial[0..2][blk] = r.zn, r.zo, r.r over the block's slice, in the order
// and with the reductions of k_dotpairs<3>.
__global__ __launch_bounds__(kDotThreads) void k_dot3_widen(const double* __restrict__ r,
                                                            const float* __restrict__ z32, double* __restrict__ zn,
                                                            const double* __restrict__ zo, double unscale,
                                                            size_t n, double* __restrict__ partial, int nblk) {
    constexpr int NW = kDotThreads / 64;
    __shared__ double red[3][NW];
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const size_t chunk = (n + nblk - 1) / nblk;
    const size_t lo = (size_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
    double acc[3] = {0, 0, 0};
#pragma unroll 4
    for (size_t q = lo + tid; q < hi; q += kDotThreads) {
        const double rq = r[q], z = unscale * (double)z32[q];
        zn[q] = z;
        acc[0] += rq * z;
        acc[1] += rq * zo[q];
        acc[2] += rq * rq;
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        double x = acc[v];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (lane == 0) red[v][wave] = x;
    }
    __syncthreads();
    if (tid < 3) {
        double x = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) x += red[tid][w];
        partial[(size_t)tid * nblk + blockIdx.x] = x;
    }
}

inline unsigned blocks_for(size_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <typename F>
hipError_t dispatch(int N, F&& f) {
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

// Both z-products of one smoother application: Y = (V^T T) / (lz + lxy), then T = V Y.
// V [2][3][n][n] holds the eigenvectors and, after them, their transposes.
// 64 x 64 output tiles unless their grid would have fewer workgroups than
// gfx950 has compute units (256); then 32 x 32.
template <typename R, int TT>
hipError_t col_gemm_pair_t(int W, int n, int ncol, const R* V, R* T, R* Y, const R* lz, const R* lam, const R* rat,
                           hipStream_t s) {
    const dim3 grid((ncol + TT - 1) / TT, (n + TT - 1) / TT, 3);
    hipError_t err = hipErrorInvalidValue;
    auto fwd = [&](auto w) {
        constexpr int WW = decltype(w)::value;
        hipLaunchKernelGGL((k_col_gemm_mfma<R, WW, 1, TT>), grid, dim3(256), 0, s, n, ncol, V, T, Y, lz, lam, rat);
        return hipGetLastError();
    };
    switch (W) {
        case 2: err = fwd(std::integral_constant<int, 2>{}); break;
        case 3: err = fwd(std::integral_constant<int, 3>{}); break;
        case 4: err = fwd(std::integral_constant<int, 4>{}); break;
        case 5: err = fwd(std::integral_constant<int, 5>{}); break;
        case 6: err = fwd(std::integral_constant<int, 6>{}); break;
        case 7: err = fwd(std::integral_constant<int, 7>{}); break;
        case 8: err = fwd(std::integral_constant<int, 8>{}); break;
        case 9: err = fwd(std::integral_constant<int, 9>{}); break;
        case 10: err = fwd(std::integral_constant<int, 10>{}); break;
        case 11: err = fwd(std::integral_constant<int, 11>{}); break;
        case 12: err = fwd(std::integral_constant<int, 12>{}); break;
        case 13: err = fwd(std::integral_constant<int, 13>{}); break;
        case 14: err = fwd(std::integral_constant<int, 14>{}); break;
        default: break;
    }
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((k_col_gemm_mfma<R, 0, 0, TT>), grid, dim3(256), 0, s, n, ncol, V + (size_t)3 * n * n, Y, T,
                       lz, lam, rat);
    return hipGetLastError();
}

// FP32 on split bf16 (k_col_gemm_bf3), 64 x 64 tiles
inline hipError_t col_gemm_pair_bf3(int W, int n, int ncol, const float* V, float* T, float* Y, const float* lz,
                                    const float* lam, const float* rat, hipStream_t s) {
    const dim3 grid((ncol + 63) / 64, (n + 63) / 64, 3);
    hipError_t err = hipErrorInvalidValue;
    auto fwd = [&](auto w) {
        constexpr int WW = decltype(w)::value;
        hipLaunchKernelGGL((k_col_gemm_bf3<WW, 1>), grid, dim3(256), 0, s, n, ncol, V, T, Y, lz, lam, rat);
        return hipGetLastError();
    };
    switch (W) {
        case 2: err = fwd(std::integral_constant<int, 2>{}); break;
        case 3: err = fwd(std::integral_constant<int, 3>{}); break;
        case 4: err = fwd(std::integral_constant<int, 4>{}); break;
        case 5: err = fwd(std::integral_constant<int, 5>{}); break;
        case 6: err = fwd(std::integral_constant<int, 6>{}); break;
        case 7: err = fwd(std::integral_constant<int, 7>{}); break;
        case 8: err = fwd(std::integral_constant<int, 8>{}); break;
        case 9: err = fwd(std::integral_constant<int, 9>{}); break;
        case 10: err = fwd(std::integral_constant<int, 10>{}); break;
        case 11: err = fwd(std::integral_constant<int, 11>{}); break;
        case 12: err = fwd(std::integral_constant<int, 12>{}); break;
        case 13: err = fwd(std::integral_constant<int, 13>{}); break;
        case 14: err = fwd(std::integral_constant<int, 14>{}); break;
        default: break;
    }
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((k_col_gemm_bf3<0, 0>), grid, dim3(256), 0, s, n, ncol, V + (size_t)3 * n * n, Y, T, lz, lam,
                       rat);
    return hipGetLastError();
}

// Small grids (fewer 64 x 64 tiles than compute units): 32 x 32 tiles in the
// working precision.  Otherwise FP32 runs on split bf16 (forty-layer finest
// level 163 -> 120 us per product in a probe) and FP64 on 64 x 64 FP64 tiles.
template <typename R>
hipError_t col_gemm_pair(int W, int n, int ncol, const R* V, R* T, R* Y, const R* lz, const R* lam, const R* rat,
                         hipStream_t s) {
    constexpr long kComputeUnits = 256;
    const long tiles64 = 3L * ((ncol + 63) / 64) * ((n + 63) / 64);
    if (tiles64 < kComputeUnits) return col_gemm_pair_t<R, 32>(W, n, ncol, V, T, Y, lz, lam, rat, s);
    if constexpr (sizeof(R) == 4) return col_gemm_pair_bf3(W, n, ncol, V, T, Y, lz, lam, rat, s);
    return col_gemm_pair_t<R, 64>(W, n, ncol, V, T, Y, lz, lam, rat, s);
}

// (Nf, Nc) pairs of the p-coarsening as compile-time constants; other pairs run
// the kernels with runtime sizes.
template <typename F>
hipError_t dispatch_pair(int Nf, int Nc, F&& f) {
    using std::integral_constant;
    if (Nf == 8 && Nc == 4) return f(integral_constant<int, 8>{}, integral_constant<int, 4>{});
    if (Nf == 7 && Nc == 4) return f(integral_constant<int, 7>{}, integral_constant<int, 4>{});
    if (Nf == 6 && Nc == 3) return f(integral_constant<int, 6>{}, integral_constant<int, 3>{});
    if (Nf == 5 && Nc == 3) return f(integral_constant<int, 5>{}, integral_constant<int, 3>{});
    if (Nf == 4 && Nc == 2) return f(integral_constant<int, 4>{}, integral_constant<int, 2>{});
    if (Nf == 3 && Nc == 2) return f(integral_constant<int, 3>{}, integral_constant<int, 2>{});
    return f(integral_constant<int, 0>{}, integral_constant<int, 0>{});
}

// Patch width P = N + 2 overlap, overlap 0..3, as a compile-time constant.
template <int N, typename F>
hipError_t dispatch_patch(int P, F&& f) {
    switch (P - N) {
        case 0: return f(std::integral_constant<int, N>{});
        case 2: return f(std::integral_constant<int, N + 2>{});
        case 4: return f(std::integral_constant<int, N + 4>{});
        case 6: return f(std::integral_constant<int, N + 6>{});
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <typename R>
hipError_t mg_smooth(int N, int E, const R* fdm, const R* b, const R* Ax, R* x, R omega, hipStream_t s) {
    return dispatch(N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_fdm_smooth<NN, R>), dim3(E), dim3(nthreads<NN>()), 0, s, E, fdm, b, Ax, x, omega);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t mg_col_smooth(int N, int n_cols, int n_z, const R* S, const R* lam, const R* rat, const R* V,
                         const R* lz, const R* b, const R* Ax, R* x, R omega, R* T, R* Y, hipStream_t s) {
    const int E = n_cols * n_z, n = n_z * N, ncol = n_cols * N * N;
    hipError_t err = dispatch(N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_col_fwd<NN, R>), dim3(E), dim3(nthreads<NN>()), 0, s, n_cols, n, S, b, Ax, T);
        return hipGetLastError();
    });
    if (err != hipSuccess) return err;
    if ((err = col_gemm_pair<R>(N, n, ncol, V, T, Y, lz, lam, rat, s)) != hipSuccess) return err;
    return dispatch(N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        hipLaunchKernelGGL((k_col_bwd<NN, R>), dim3(E), dim3(nthreads<NN>()), 0, s, n_cols, n, S, T, x, omega,
                           Ax ? 1 : 0);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t mg_ovl_smooth(int N, int n_cols, int n_z, int P, const int* pg, const int* ps, const R* wsq,
                         const R* S, const R* lam, const R* rat, const R* V, const R* lz, const R* b, const R* Ax,
                         R* x, R omega, R* T, R* Y, hipStream_t s) {
    const int E = n_cols * n_z, n = n_z * N, ncol = n_cols * P * P;
    const size_t shm = sizeof(R) * (size_t)(2 * 3 * N * P * P + 2 * P * P);
    hipError_t err = dispatch(N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        return dispatch_patch<NN>(P, [&](auto pp) {
            constexpr int PP = decltype(pp)::value;
            hipLaunchKernelGGL((k_ovl_fwd<NN, PP, R>), dim3(E), dim3(kOvlThreads), shm, s, n_cols, n, pg, wsq, S, b, Ax, T);
            return hipGetLastError();
        });
    });
    if (err != hipSuccess) return err;
    if ((err = col_gemm_pair<R>(P, n, ncol, V, T, Y, lz, lam, rat, s)) != hipSuccess) return err;
    return dispatch(N, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        const hipError_t e = dispatch_patch<NN>(P, [&](auto pp) {
            constexpr int PP = decltype(pp)::value;
            hipLaunchKernelGGL((k_ovl_bwd<NN, PP, R>), dim3(E), dim3(kOvlThreads), shm, s, n_cols, n, S, T);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
        const size_t tot = (size_t)E * 3 * NN * NN * NN;
        hipLaunchKernelGGL((k_ovl_sum<NN, R>), dim3(blocks_for(tot, 256)), dim3(256), 0, s, n_cols, n_z, P, ps, wsq,
                           T, x, omega, Ax ? 1 : 0);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t mg_prolong_z(int N, int Ef, int n_cols, const int* zpar, const R* Iz, const R* uc, R* uf, hipStream_t s) {
    return dispatch(N, [&](auto nn) {
        hipLaunchKernelGGL((k_prolong_z<R, decltype(nn)::value>), dim3(Ef), dim3(256), 0, s, N, n_cols, zpar, Iz, uc,
                           uf);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t mg_restrict_z(int N, int Ec, int n_cols, const int* zch, const R* Iz, const R* rf, R* rc, hipStream_t s) {
    return dispatch(N, [&](auto nn) {
        hipLaunchKernelGGL((k_restrict_z<R, decltype(nn)::value>), dim3(Ec), dim3(256), 0, s, N, n_cols, zch, Iz, rf,
                           rc);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t mg_prolong_p(int E, int Nf, int Nc, const R* I, const R* uc, R* uf, hipStream_t s) {
    return dispatch_pair(Nf, Nc, [&](auto f, auto c) {
        hipLaunchKernelGGL((k_prolong_p<R, decltype(f)::value, decltype(c)::value>), dim3(E), dim3(256), 0, s, E, Nf,
                           Nc, I, uc, uf);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t mg_restrict_p(int E, int Nf, int Nc, const R* I, const R* rf, R* rc, hipStream_t s) {
    return dispatch_pair(Nf, Nc, [&](auto f, auto c) {
        hipLaunchKernelGGL((k_restrict_p<R, decltype(f)::value, decltype(c)::value>), dim3(E), dim3(256), 0, s, E, Nf,
                           Nc, I, rf, rc);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t mg_prolong_h(int N, int Ef, int ncf, int ncc, const int* parent, const int* child, const R* Ih,
                        const R* uc, R* uf, hipStream_t s) {
    return dispatch(N, [&](auto nn) {
        hipLaunchKernelGGL((k_prolong_h<R, decltype(nn)::value>), dim3(Ef), dim3(256), 0, s, N, ncf, ncc, parent,
                           child, Ih, uc, uf);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t mg_restrict_h(int N, int Ec, int ncf, int ncc, const int* children, const R* Ih, const R* rf, R* rc,
                         hipStream_t s) {
    return dispatch(N, [&](auto nn) {
        hipLaunchKernelGGL((k_restrict_h<R, decltype(nn)::value>), dim3(Ec), dim3(256), 0, s, N, ncf, ncc, children,
                           Ih, rf, rc);
        return hipGetLastError();
    });
}

hipError_t dense_set_unit(double* e, int j, hipStream_t s) {
    hipLaunchKernelGGL(k_set_unit, dim3(1), dim3(64), 0, s, e, j);
    return hipGetLastError();
}

size_t dense_invert_scratch(int n) { return 2 * (size_t)kGJB * n + (size_t)kGJB * kGJB; }

hipError_t dense_invert(double* A, double* scratch, int n, hipStream_t s) {
    double* R = scratch;                           // [kGJB][n]
    double* C = scratch + (size_t)kGJB * n;        // [n][kGJB]
    double* P = scratch + 2 * (size_t)kGJB * n;    // [kGJB][kGJB]
    const unsigned tiles = (unsigned)((n + 63) / 64);
    for (int k0 = 0; k0 < n; k0 += kGJB) {
        const int b = std::min(kGJB, n - k0);
        const size_t nb = (size_t)n * b;
        hipLaunchKernelGGL(k_gjb_diag, dim3(1), dim3(256), 0, s, A, n, k0, b, P);
        hipLaunchKernelGGL(k_gjb_row, dim3(blocks_for(nb, 256)), dim3(256), 0, s, A, n, k0, b, P, R);
        hipLaunchKernelGGL(k_gjb_update, dim3(tiles, tiles), dim3(256), 0, s, A, n, k0, b, R);
        hipLaunchKernelGGL(k_gjb_col, dim3(blocks_for(nb, 256)), dim3(256), 0, s, A, n, k0, b, P, C);
        hipLaunchKernelGGL(k_gjb_store, dim3(blocks_for(2 * nb, 256)), dim3(256), 0, s, A, n, k0, b, R, P, C);
    }
    return hipGetLastError();
}

template <typename R>
hipError_t dense_gemv(const R* A, const R* x, R* y, int n, hipStream_t s) {
    const bool vec = n % (16 / (int)sizeof(R)) == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(x) % 16 == 0;
    if (vec)
        hipLaunchKernelGGL((k_gemv<R, true>), dim3(blocks_for((size_t)n * 64, 256)), dim3(256), 0, s, A, x, y, n);
    else
        hipLaunchKernelGGL((k_gemv<R, false>), dim3(blocks_for((size_t)n * 64, 256)), dim3(256), 0, s, A, x, y, n);
    return hipGetLastError();
}

template <typename R>
hipError_t vec_zero(R* x, size_t n, hipStream_t s) {
    hipLaunchKernelGGL((k_zero<R>), dim3(blocks_for(n, 256)), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

template <typename A, typename B>
hipError_t vec_cast(const A* x, B* y, size_t n, double scale, hipStream_t s) {
    hipLaunchKernelGGL((k_cast<A, B>), dim3(blocks_for(n, 256)), dim3(256), 0, s, x, y, n, scale);
    return hipGetLastError();
}

template <typename R>
hipError_t vec_resid(const R* b, R* y, size_t n, hipStream_t s) {
    hipLaunchKernelGGL((k_resid<R>), dim3(blocks_for(n, 256)), dim3(256), 0, s, b, y, n);
    return hipGetLastError();
}

hipError_t vec_multidot(const double* V, size_t ldv, int nv, const double* w, size_t n, double* partial, int nblk,
                        double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_multidot, dim3(nblk), dim3(kDotThreads), 0, s, V, ldv, nv, w, n, partial, nblk);
    hipLaunchKernelGGL(k_reduce_partials, dim3(nv + 1), dim3(kDotThreads), 0, s, partial, nblk, out);
    return hipGetLastError();
}

hipError_t fcg_update(double* u, double* r, const double* p, const double* q, const double* cur, double* sc,
                      float* r32, double scale32, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fcg_update, dim3(blocks_for(n, 256)), dim3(256), 0, s, u, r, p, q, cur, sc, r32, scale32,
                       n);
    return hipGetLastError();
}

hipError_t vec_dot3_widen(const double* r, const float* z32, double* zn, const double* zo, double unscale, size_t n,
                          double* partial, int nblk, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_dot3_widen, dim3(nblk), dim3(kDotThreads), 0, s, r, z32, zn, zo, unscale, n, partial, nblk);
    hipLaunchKernelGGL(k_reduce_partials, dim3(3), dim3(kDotThreads), 0, s, partial, nblk, out);
    return hipGetLastError();
}

hipError_t fcg_direction(double* p, const double* z, const double* cur, const double* nxt, size_t n,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_fcg_direction, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, z, cur, nxt, n);
    return hipGetLastError();
}

hipError_t vec_multiaxpy(double* w, const double* V, size_t ldv, int nv, const double* coef, size_t n,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_multiaxpy, dim3(blocks_for(n, 256)), dim3(256), 0, s, w, V, ldv, nv, coef, n);
    return hipGetLastError();
}

hipError_t vec_axpy(double* y, double a, const double* x, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n, 256)), dim3(256), 0, s, y, a, x, n);
    return hipGetLastError();
}

hipError_t vec_xpby(double* p, const double* z, double beta, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_xpby, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, z, beta, n);
    return hipGetLastError();
}

hipError_t vec_dotpairs(int np, const double* const* x, const double* const* y, size_t n, double* partial, int nblk,
                        double* out, hipStream_t s) {
    DotPairs d{};
    d.np = np;
    for (int v = 0; v < np; ++v) {
        d.x[v] = x[v];
        d.y[v] = y[v];
    }
    switch (np) {
        case 1: hipLaunchKernelGGL(k_dotpairs<1>, dim3(nblk), dim3(kDotThreads), 0, s, d, n, partial, nblk); break;
        case 2: hipLaunchKernelGGL(k_dotpairs<2>, dim3(nblk), dim3(kDotThreads), 0, s, d, n, partial, nblk); break;
        case 3: hipLaunchKernelGGL(k_dotpairs<3>, dim3(nblk), dim3(kDotThreads), 0, s, d, n, partial, nblk); break;
        case 4: hipLaunchKernelGGL(k_dotpairs<4>, dim3(nblk), dim3(kDotThreads), 0, s, d, n, partial, nblk); break;
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_reduce_partials, dim3(np), dim3(kDotThreads), 0, s, partial, nblk, out);
    return hipGetLastError();
}

hipError_t vec_scale_copy(const double* x, double* y, double a, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_copy, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, y, a, n);
    return hipGetLastError();
}

#define INST(R)                                                                                        \
    template hipError_t mg_smooth<R>(int, int, const R*, const R*, const R*, R*, R, hipStream_t);      \
    template hipError_t mg_col_smooth<R>(int, int, int, const R*, const R*, const R*, const R*,         \
                                         const R*, const R*, const R*, R*, R, R*, R*, hipStream_t);    \
    template hipError_t mg_ovl_smooth<R>(int, int, int, int, const int*, const int*, const R*, const R*, \
                                         const R*, \
                                         const R*, const R*, const R*, const R*, const R*, R*, R, R*, R*, \
                                         hipStream_t);                                                  \
    template hipError_t mg_prolong_z<R>(int, int, int, const int*, const R*, const R*, R*, hipStream_t); \
    template hipError_t mg_restrict_z<R>(int, int, int, const int*, const R*, const R*, R*, hipStream_t); \
    template hipError_t mg_prolong_p<R>(int, int, int, const R*, const R*, R*, hipStream_t);           \
    template hipError_t mg_restrict_p<R>(int, int, int, const R*, const R*, R*, hipStream_t);          \
    template hipError_t mg_prolong_h<R>(int, int, int, int, const int*, const int*, const R*, const R*, \
                                        R*, hipStream_t);                                              \
    template hipError_t mg_restrict_h<R>(int, int, int, int, const int*, const R*, const R*, R*,       \
                                         hipStream_t);                                                 \
    template hipError_t dense_gemv<R>(const R*, const R*, R*, int, hipStream_t);                       \
    template hipError_t vec_zero<R>(R*, size_t, hipStream_t);                                          \
    template hipError_t vec_resid<R>(const R*, R*, size_t, hipStream_t);
INST(double)
INST(float)
template hipError_t vec_cast<double, float>(const double*, float*, size_t, double, hipStream_t);
template hipError_t vec_cast<float, double>(const float*, double*, size_t, double, hipStream_t);
template hipError_t vec_cast<double, double>(const double*, double*, size_t, double, hipStream_t);

}  // namespace dgtn
