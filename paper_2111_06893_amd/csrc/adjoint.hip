// Adjoint gradient of the layer-weighted elastic energy J = sum_k w_k U_k.
//
// With A u = b,
//   dJ/dtheta = 1/2 u^T K_w,theta u - lambda^T A_theta u + lambda^T b_theta,
//   A lambda = K_w u,
// K_w the layer-weighted energy form (A is symmetric, so the adjoint system is
// the forward one).  Material and thickness parameters leave the load on
// z = 0 unchanged: A_theta u and K_w,theta are evaluated by the forward
// operator and energy kernels instantiated on dual numbers, with the
// derivative of the seeded material constants or element thicknesses.  The
// beam parameters (width r0, centre xc, yc of the pressure of eq. laserbeam)
// leave A and K unchanged: only lambda^T b_theta remains, b_theta being the
// load kernel with the derivative of the pressure profile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "context.h"

namespace dgtn {

namespace {

constexpr int kDotThreads = 256;

__global__ void k_to_dual(const double* __restrict__ x, Dual* __restrict__ y, size_t n) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) y[q] = Dual(x[q], 0.0);
}

// partial[blk] = sum over the block's slice of lam[q] * Au[q].d (fixed order)
__global__ __launch_bounds__(kDotThreads) void k_dot_deriv(const double* __restrict__ lam, const Dual* __restrict__ Au,
                                                           size_t n, double* __restrict__ partial, int nblk) {
    __shared__ double red[kDotThreads];
    const int tid = threadIdx.x;
    const size_t chunk = (n + nblk - 1) / nblk;
    const size_t lo = (size_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
    double acc = 0;
    for (size_t q = lo + tid; q < hi; q += kDotThreads) acc += lam[q] * Au[q].d;
    red[tid] = acc;
    __syncthreads();
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) partial[blockIdx.x] = red[0];
}

// partial[blk] = sum over the block's slice of lam[q] * b[q] (fixed order)
__global__ __launch_bounds__(kDotThreads) void k_dot_plain(const double* __restrict__ lam,
                                                           const double* __restrict__ b, size_t n,
                                                           double* __restrict__ partial, int nblk) {
    __shared__ double red[kDotThreads];
    const int tid = threadIdx.x;
    const size_t chunk = (n + nblk - 1) / nblk;
    const size_t lo = (size_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
    double acc = 0;
    for (size_t q = lo + tid; q < hi; q += kDotThreads) acc += lam[q] * b[q];
    red[tid] = acc;
    __syncthreads();
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) partial[blockIdx.x] = red[0];
}

size_t ndof(const Level& L) { return (size_t)3 * L.E * L.N * L.N * L.N; }

template <typename T>
T* at(const dgtn_ctx* c, size_t off) {
    return reinterpret_cast<T*>(c->ws + off);
}

std::vector<Dual> to_dual(const std::vector<double>& v) {
    std::vector<Dual> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = Dual(v[i], 0.0);
    return o;
}

LevelView<Dual> dual_view(const dgtn_ctx* c) {
    const Level& L = c->levels[0];
    const AdjointLayout& A = c->adj;
    LevelView<Dual> v;
    v.N = L.N;
    v.n_cols = L.n_cols;
    v.n_z = L.n_z;
    v.E = L.E;
    v.e0 = 0;
    v.geo2 = at<const Dual>(c, A.geo2);
    v.sig_side = at<const Dual>(c, A.sig);
    v.fnrm = at<const Dual>(c, A.fnrm);
    v.cnbr = at<const int>(c, L.off_cnbr);
    v.cnf = at<const int>(c, L.off_cnf);
    v.hz = at<const Dual>(c, A.hz);
    v.zmat = at<const int>(c, L.off_zmat);
    v.mat = at<const Dual>(c, A.mat);
    v.D = at<const Dual>(c, A.D);
    v.w = at<const Dual>(c, A.w);
    v.bc_top = c->prob.bc_top;
    v.bc_bottom = c->prob.bc_bottom;
    v.penalty_n2 = Dual(L.pen_z, 0.0);
    for (int q = 0; q < 64; ++q) {
        const bool in = q < L.N * L.N;
        v.Dk[q] = Dual(in ? L.lgl.D[q] : 0.0, 0.0);
        v.Dt[q] = Dual(in ? L.lgl.D[(q % L.N) * L.N + q / L.N] : 0.0, 0.0);
    }
    return v;
}

#define AHIP(...)                                                                    \
    do {                                                                             \
        hipError_t e_ = (__VA_ARGS__);                                               \
        if (e_ != hipSuccess) {                                                      \
            set_error(std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_));     \
            return DGTN_EHIP;                                                        \
        }                                                                            \
    } while (0)

}  // namespace

void plan_adjoint(dgtn_ctx* c, Layout& lay) {
    const Level& L = c->levels[0];
    AdjointLayout& A = c->adj;
    const size_t N = L.N, N2 = N * N, n = ndof(L), ds = sizeof(Dual);
    A.wz = lay.take(8 * (size_t)L.n_z);
    A.ok = L.N <= 8;
    if (!A.ok) return;
    A.u = lay.take(ds * n);
    A.Au = lay.take(ds * n);
    A.tau = lay.take(ds * (size_t)L.E * 6 * 3 * N2);
    A.geo2 = lay.take(ds * (size_t)L.n_cols * 5 * N2);
    A.sig = lay.take(ds * (size_t)L.n_cols * 4 * N);
    A.fnrm = lay.take(ds * (size_t)L.n_cols * 4 * 3 * N);
    A.hz = lay.take(ds * (size_t)L.n_z);
    A.mat = lay.take(ds * c->matc.size());
    A.D = lay.take(ds * N2);
    A.w = lay.take(ds * N);
    A.Ue = lay.take(ds * (size_t)L.E);
    A.nblk = (int)std::min<size_t>(1024, std::max<size_t>(1, n / 4096));
    A.partial = lay.take(8 * (size_t)A.nblk);
    A.dots = lay.take(8);
}

dgtn_status bind_adjoint(dgtn_ctx* c, hipStream_t s) {
    const AdjointLayout& A = c->adj;
    if (!A.ok) return DGTN_OK;
    const Level& L = c->levels[0];
    auto up = [&](size_t off, const std::vector<Dual>& v) {
        return hipMemcpyAsync(c->ws + off, v.data(), sizeof(Dual) * v.size(), hipMemcpyHostToDevice, s);
    };
    std::vector<double> matn(c->matc.size());
    for (size_t i = 0; i < matn.size(); ++i) matn[i] = c->matc[i] / c->y_ref;
    const auto g = to_dual(L.geo2), sg = to_dual(L.sig_side), fn = to_dual(L.fnrm), hz = to_dual(L.hz), mt = to_dual(matn),
               D = to_dual(L.lgl.D), w = to_dual(L.lgl.w);
    AHIP(up(A.geo2, g));
    AHIP(up(A.sig, sg));
    AHIP(up(A.fnrm, fn));
    AHIP(up(A.hz, hz));
    AHIP(up(A.mat, mt));
    AHIP(up(A.D, D));
    AHIP(up(A.w, w));
    AHIP(hipStreamSynchronize(s));
    return DGTN_OK;
}

}  // namespace dgtn

using namespace dgtn;

namespace {

dgtn_status upload_weights(dgtn_ctx* c, const double* w_layers, hipStream_t s) {
    const Level& L = c->levels[0];
    std::vector<double> wz(L.n_z);
    for (int iz = 0; iz < L.n_z; ++iz) wz[iz] = w_layers ? w_layers[L.zlayer[iz]] : 1.0;
    AHIP(hipMemcpyAsync(c->ws + c->adj.wz, wz.data(), 8 * wz.size(), hipMemcpyHostToDevice, s));
    AHIP(hipStreamSynchronize(s));
    return DGTN_OK;
}

}  // namespace

extern "C" dgtn_status dgtn_energy_grad(dgtn_ctx* c, const double* u, const double* w_layers, double* g,
                                        hipStream_t s) {
    if (!c || !u || !g) { set_error("null argument"); return DGTN_EINVAL; }
    if (!c->bound) { set_error("no workspace bound"); return DGTN_EINVAL; }
    if (u == g) { set_error("u and g must not alias"); return DGTN_EINVAL; }
    dgtn_status st = upload_weights(c, w_layers, s);
    if (st != DGTN_OK) return st;
    const Level& L = c->levels[0];
    AHIP(launch_energy_grad(view_of<double>(c, L), u, at<const double>(c, c->adj.wz), g, c->y_ref, s));
    return DGTN_OK;
}

extern "C" dgtn_status dgtn_grad(dgtn_ctx* c, const double* u, const double* lam, const double* w_layers,
                                 int n_params, const dgtn_param* params, double* dJ, hipStream_t s) {
    if (!c || !u || !lam || !dJ || (n_params > 0 && !params) || n_params < 0) {
        set_error("invalid argument");
        return DGTN_EINVAL;
    }
    if (!c->bound) { set_error("no workspace bound"); return DGTN_EINVAL; }
    const AdjointLayout& A = c->adj;
    if (!A.ok) { set_error("parameter derivatives are available for p <= 7"); return DGTN_EINVAL; }
    const Level& L = c->levels[0];
    const int nmat = (int)c->prob.materials.size(), nlay = (int)c->prob.layers.size();
    for (int i = 0; i < n_params; ++i) {
        const dgtn_param& p = params[i];
        const bool mod = p.kind == DGTN_PARAM_C11 || p.kind == DGTN_PARAM_C12 || p.kind == DGTN_PARAM_C44;
        const bool iso = p.kind == DGTN_PARAM_YOUNGS || p.kind == DGTN_PARAM_POISSON;
        if ((mod || iso) && (p.index < 0 || p.index >= nmat)) { set_error("no such material"); return DGTN_EINVAL; }
        if (iso && c->prob.materials[p.index].kind != DGTN_MAT_ISO) {
            set_error("Young's modulus / Poisson ratio of a cubic material");
            return DGTN_EINVAL;
        }
        if (p.kind == DGTN_PARAM_THICKNESS && (p.index < 0 || p.index >= nlay)) {
            set_error("no such layer");
            return DGTN_EINVAL;
        }
        const bool beam = p.kind == DGTN_PARAM_BEAM_WIDTH || p.kind == DGTN_PARAM_BEAM_X || p.kind == DGTN_PARAM_BEAM_Y;
        if (!mod && !iso && !beam && p.kind != DGTN_PARAM_THICKNESS) {
            set_error("unknown parameter kind");
            return DGTN_EINVAL;
        }
    }
    dgtn_status st = upload_weights(c, w_layers, s);
    if (st != DGTN_OK) return st;
    const size_t n = ndof(L);
    Dual* ud = at<Dual>(c, A.u);
    Dual* Aud = at<Dual>(c, A.Au);
    hipLaunchKernelGGL(k_to_dual, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, u, ud, n);
    AHIP(hipGetLastError());
    const LevelView<Dual> v = dual_view(c);
    const double yr = c->y_ref;
    std::vector<double> wz(L.n_z);
    for (int iz = 0; iz < L.n_z; ++iz) wz[iz] = w_layers ? w_layers[L.zlayer[iz]] : 1.0;
    std::vector<Dual> hz(L.n_z), mat(c->matc.size());
    std::vector<Dual> Ue(L.E);
    std::vector<double> part(A.nblk);
    for (int ip = 0; ip < n_params; ++ip) {
        const dgtn_param& p = params[ip];
        if (p.kind >= DGTN_PARAM_BEAM_WIDTH) {
            // lambda^T b_theta, b_theta written over the dual scratch vector
            const Problem& P = c->prob;
            double* db = at<double>(c, A.Au);
            AHIP(launch_rhs(view_of<double>(c, L), reinterpret_cast<const double*>(c->ws + L.off_xy), P.F0, P.r0,
                            P.xc, P.yc, p.kind - DGTN_PARAM_BEAM_WIDTH + 1, db, s));
            hipLaunchKernelGGL(k_dot_plain, dim3(A.nblk), dim3(kDotThreads), 0, s, lam, db, n,
                               at<double>(c, A.partial), A.nblk);
            AHIP(hipGetLastError());
            AHIP(hipMemcpyAsync(part.data(), at<double>(c, A.partial), 8 * part.size(), hipMemcpyDeviceToHost, s));
            AHIP(hipStreamSynchronize(s));
            double lb = 0;
            for (double x : part) lb += x;
            dJ[ip] = lb;
            if (!std::isfinite(dJ[ip])) { set_error("non-finite gradient"); return DGTN_ENAN; }
            continue;
        }
        for (int iz = 0; iz < L.n_z; ++iz) hz[iz] = Dual(L.hz[iz], 0.0);
        for (size_t q = 0; q < mat.size(); ++q) mat[q] = Dual(c->matc[q] / yr, 0.0);
        if (p.kind == DGTN_PARAM_THICKNESS) {
            // every element thickness of the layer scales with it; layers below translate
            const double t = c->prob.layers[p.index].thickness;
            for (int iz = 0; iz < L.n_z; ++iz)
                if (L.zlayer[iz] == p.index) hz[iz].d = L.hz[iz] / t;
        } else if (p.kind == DGTN_PARAM_C11 || p.kind == DGTN_PARAM_C12 || p.kind == DGTN_PARAM_C44) {
            mat[3 * p.index + (p.kind - DGTN_PARAM_C11)].d = 1.0 / yr;
        } else {
            // isotropic: c11 = lambda + 2 mu, c12 = lambda, c44 = mu
            const double Y = c->prob.materials[p.index].youngs, nu = c->prob.materials[p.index].poisson;
            double dlam, dmu;
            if (p.kind == DGTN_PARAM_YOUNGS) {
                dlam = nu / ((1 + nu) * (1 - 2 * nu));
                dmu = 1.0 / (2 * (1 + nu));
            } else {
                const double den = (1 + nu) * (1 - 2 * nu);
                dlam = Y * (1 + 2 * nu * nu) / (den * den);
                dmu = -Y / (2 * (1 + nu) * (1 + nu));
            }
            mat[3 * p.index].d = (dlam + 2 * dmu) / yr;
            mat[3 * p.index + 1].d = dlam / yr;
            mat[3 * p.index + 2].d = dmu / yr;
        }
        AHIP(hipMemcpyAsync(c->ws + A.hz, hz.data(), sizeof(Dual) * hz.size(), hipMemcpyHostToDevice, s));
        AHIP(hipMemcpyAsync(c->ws + A.mat, mat.data(), sizeof(Dual) * mat.size(), hipMemcpyHostToDevice, s));
        // Element ranges (in z-layers) that see the parameter: the z-elements of the
        // layer (thickness) or of every layer made of the material, from the first to
        // the last.  K_w,theta lives on them; rows of A_theta u are nonzero on them
        // and their z-neighbours (penalty, lift, averaged moduli and the neighbours'
        // tractions), which read the tractions of one layer further.
        int rz0 = 0, rz1 = L.n_z, tz0 = 0, tz1 = L.n_z, ez0 = 0, ez1 = L.n_z;
        {
            int z0 = L.n_z, z1 = 0;
            for (int iz = 0; iz < L.n_z; ++iz)
                if (p.kind == DGTN_PARAM_THICKNESS ? L.zlayer[iz] == p.index : L.zmat[iz] == p.index) {
                    z0 = std::min(z0, iz);
                    z1 = std::max(z1, iz + 1);
                }
            if (z1 <= z0) {  // a material no layer uses: no derivative
                dJ[ip] = 0.0;
                continue;
            }
            ez0 = z0;
            ez1 = z1;
            rz0 = std::max(0, z0 - 1);
            rz1 = std::min(L.n_z, z1 + 1);
            tz0 = std::max(0, z0 - 2);
            tz1 = std::min(L.n_z, z1 + 2);
        }
        auto range = [&](int a, int b) {
            LevelView<Dual> r = v;
            r.e0 = a * L.n_cols;
            r.E = (b - a) * L.n_cols;
            return r;
        };
        // lambda^T A_theta u
        AHIP(launch_traction<Dual>(range(tz0, tz1), ud, at<Dual>(c, A.tau), s));
        AHIP(launch_apply<Dual>(range(rz0, rz1), ud, at<const Dual>(c, A.tau), Aud, Dual(yr, 0.0), s));
        const size_t per_layer = n / L.n_z, r_off = (size_t)rz0 * per_layer;
        hipLaunchKernelGGL(k_dot_deriv, dim3(A.nblk), dim3(kDotThreads), 0, s, lam + r_off, Aud + r_off,
                           (size_t)(rz1 - rz0) * per_layer, at<double>(c, A.partial), A.nblk);
        AHIP(hipGetLastError());
        // 1/2 u^T K_w,theta u, per element
        AHIP(launch_energy<Dual>(range(ez0, ez1), u, at<Dual>(c, A.Ue), s));
        const int eb = ez0 * L.n_cols, ne = (ez1 - ez0) * L.n_cols;
        AHIP(hipMemcpyAsync(part.data(), at<double>(c, A.partial), 8 * part.size(), hipMemcpyDeviceToHost, s));
        AHIP(hipMemcpyAsync(Ue.data() + eb, at<Dual>(c, A.Ue) + eb, sizeof(Dual) * ne, hipMemcpyDeviceToHost, s));
        AHIP(hipStreamSynchronize(s));
        double lAu = 0, dU = 0;
        for (double x : part) lAu += x;
        for (int e = eb; e < eb + ne; ++e) dU += wz[e / L.n_cols] * Ue[e].d;
        dJ[ip] = dU * yr - lAu;
        if (!std::isfinite(dJ[ip])) { set_error("non-finite gradient"); return DGTN_ENAN; }
    }
    // restore the undifferentiated tables
    for (int iz = 0; iz < L.n_z; ++iz) hz[iz] = Dual(L.hz[iz], 0.0);
    for (size_t q = 0; q < mat.size(); ++q) mat[q] = Dual(c->matc[q] / yr, 0.0);
    AHIP(hipMemcpyAsync(c->ws + A.hz, hz.data(), sizeof(Dual) * hz.size(), hipMemcpyHostToDevice, s));
    AHIP(hipMemcpyAsync(c->ws + A.mat, mat.data(), sizeof(Dual) * mat.size(), hipMemcpyHostToDevice, s));
    AHIP(hipStreamSynchronize(s));
    return DGTN_OK;
}
