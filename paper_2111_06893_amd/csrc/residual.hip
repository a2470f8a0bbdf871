// Residual b - A u of a double u in double-double arithmetic (Sec. 2.3, eq.
// matrix_eqn; iterative refinement with an extended-precision residual).
//
// In FP64 the residual of an accurate solution is computed with cancellation:
// the interior-penalty terms sigma Y [u] with sigma = C N^2 / h are large on
// thin layers and cancel against each other and against the load, so b - A u
// carries a rounding error of about eps |A| |u|.  Here the operator kernels run
// on double-double numbers over the same double coefficient tables as the FP64
// operator (geometry, materials, LGL matrix and weights, each with a zero low
// part), u enters exactly, and b - A u is rounded to double once at the end.
// Comparing the two residuals of one u tells the rounding of the arithmetic
// apart from that of u itself, which alone bounds the attainable residual of a
// double u to the same eps |A| |u| (measured: at a stagnated solve the two
// residuals agree to 1e-4 of their size).
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "context.h"

namespace dgtn {

namespace {

template <typename T>
T* at(const dgtn_ctx* c, size_t off) {
    return reinterpret_cast<T*>(c->ws + off);
}

size_t ndof0(const Level& L) { return (size_t)3 * L.E * L.N * L.N * L.N; }

__global__ void k_to_dd(const double* __restrict__ x, DD* __restrict__ y, size_t n) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) y[q] = DD(x[q], 0.0);
}

// r = b - Au rounded once: (b - hi) exactly by two-sum, then - lo
__global__ void k_resid_dd(const double* __restrict__ b, const DD* __restrict__ Au, double* __restrict__ r, size_t n) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) {
        const DD a = Au[q];
        DD t = two_sum(b[q], -a.hi);
        t.lo -= a.lo;
        r[q] = t.hi + t.lo;
    }
}

std::vector<DD> to_dd(const std::vector<double>& v) {
    std::vector<DD> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = DD(v[i], 0.0);
    return o;
}

LevelView<DD> dd_view(const dgtn_ctx* c) {
    const Level& L = c->levels[0];
    const ResidualLayout& Q = c->res;
    LevelView<DD> v;
    v.N = L.N;
    v.n_cols = L.n_cols;
    v.n_z = L.n_z;
    v.E = L.E;
    v.e0 = 0;
    v.geo2 = at<const DD>(c, Q.geo2);
    v.sig_side = at<const DD>(c, Q.sig);
    v.fnrm = at<const DD>(c, Q.fnrm);
    v.cnbr = at<const int>(c, L.off_cnbr);
    v.cnf = at<const int>(c, L.off_cnf);
    v.hz = at<const DD>(c, Q.hz);
    v.zmat = at<const int>(c, L.off_zmat);
    v.mat = at<const DD>(c, Q.mat);
    v.D = at<const DD>(c, Q.D);
    v.w = at<const DD>(c, Q.w);
    v.bc_top = c->prob.bc_top;
    v.bc_bottom = c->prob.bc_bottom;
    v.penalty_n2 = DD(L.pen_z);
    for (int q = 0; q < 64; ++q) {
        const bool in = q < L.N * L.N;
        v.Dk[q] = DD(in ? L.lgl.D[q] : 0.0);
        v.Dt[q] = DD(in ? L.lgl.D[(q % L.N) * L.N + q / L.N] : 0.0);
    }
    return v;
}

}  // namespace

void plan_residual(dgtn_ctx* c, Layout& lay) {
    const Level& L = c->levels[0];
    ResidualLayout& Q = c->res;
    // the field buffers are the adjoint's dual-number ones (same size), idle during a solve
    Q.ok = c->adj.ok;
    if (!Q.ok) return;
    const size_t N = L.N, N2 = N * N, ds = sizeof(DD);
    Q.geo2 = lay.take(ds * (size_t)L.n_cols * 5 * N2);
    Q.sig = lay.take(ds * (size_t)L.n_cols * 4 * N);
    Q.fnrm = lay.take(ds * (size_t)L.n_cols * 4 * 3 * N);
    Q.hz = lay.take(ds * (size_t)L.n_z);
    Q.mat = lay.take(ds * c->matc.size());
    Q.D = lay.take(ds * N2);
    Q.w = lay.take(ds * N);
}

dgtn_status bind_residual(dgtn_ctx* c, hipStream_t s) {
    const ResidualLayout& Q = c->res;
    if (!Q.ok) return DGTN_OK;
    const Level& L = c->levels[0];
    std::vector<double> matn(c->matc.size());
    for (size_t i = 0; i < matn.size(); ++i) matn[i] = c->matc[i] / c->y_ref;  // as the FP64 tables
    const std::vector<DD> tabs[7] = {to_dd(L.geo2), to_dd(L.sig_side), to_dd(L.fnrm), to_dd(L.hz),
                                     to_dd(matn),   to_dd(L.lgl.D),    to_dd(L.lgl.w)};
    const size_t offs[7] = {Q.geo2, Q.sig, Q.fnrm, Q.hz, Q.mat, Q.D, Q.w};
    for (int t = 0; t < 7; ++t) {
        const hipError_t e = hipMemcpyAsync(c->ws + offs[t], tabs[t].data(), sizeof(DD) * tabs[t].size(),
                                            hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            set_error(std::string("residual tables: ") + hipGetErrorString(e));
            return DGTN_EHIP;
        }
    }
    const hipError_t e = hipStreamSynchronize(s);  // the host vectors die here
    if (e != hipSuccess) {
        set_error(std::string("residual tables: ") + hipGetErrorString(e));
        return DGTN_EHIP;
    }
    return DGTN_OK;
}

hipError_t residual_dd(dgtn_ctx* c, const double* b, const double* u, double* r, hipStream_t s) {
    const Level& L = c->levels[0];
    const AdjointLayout& A = c->adj;
    const size_t n = ndof0(L);
    const unsigned nb = (unsigned)((n + 255) / 256);
    DD* ud = at<DD>(c, A.u);
    DD* Aud = at<DD>(c, A.Au);
    DD* taud = at<DD>(c, A.tau);
    const LevelView<DD> v = dd_view(c);
    hipLaunchKernelGGL(k_to_dd, dim3(nb), dim3(256), 0, s, u, ud, n);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_traction<DD>(v, ud, taud, s);
    if (e == hipSuccess) e = launch_apply<DD>(v, ud, taud, Aud, DD(c->y_ref), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_resid_dd, dim3(nb), dim3(256), 0, s, b, Aud, r, n);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace dgtn

using namespace dgtn;

extern "C" dgtn_status dgtn_residual(dgtn_ctx* c, const double* b, const double* u, double* r, hipStream_t s) {
    if (!c || !b || !u || !r) { set_error("null argument"); return DGTN_EINVAL; }
    if (!c->bound) { set_error("no workspace bound"); return DGTN_EINVAL; }
    if (r == u) { set_error("r and u must not alias"); return DGTN_EINVAL; }
    if (!c->res.ok) { set_error("the extended-precision residual covers p <= 7"); return DGTN_EINVAL; }
    const hipError_t e = residual_dd(c, b, u, r, s);
    if (e != hipSuccess) {
        set_error(std::string("dgtn_residual: ") + hipGetErrorString(e));
        return DGTN_EHIP;
    }
    return DGTN_OK;
}
