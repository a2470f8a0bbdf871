// C ABI of the library: context, workspace binding and the operator calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "context.h"

namespace dgtn {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

size_t Layout::take(size_t bytes) {
    size_t off = (cursor + 255) & ~size_t(255);
    cursor = off + bytes;
    return off;
}

template <typename R>
LevelView<R> view_of(const dgtn_ctx* c, const Level& L) {
    const int pi = sizeof(R) == 8 ? 0 : 1;
    LevelView<R> v;
    v.N = L.N;
    v.n_cols = L.n_cols;
    v.n_z = L.n_z;
    v.E = L.E;
    v.e0 = 0;
    char* b = c->ws;
    v.geo2 = reinterpret_cast<const R*>(b + L.off_geo2[pi]);
    v.sig_side = reinterpret_cast<const R*>(b + L.off_sig[pi]);
    v.fnrm = reinterpret_cast<const R*>(b + L.off_fnrm[pi]);
    v.cnbr = reinterpret_cast<const int*>(b + L.off_cnbr);
    v.cnf = reinterpret_cast<const int*>(b + L.off_cnf);
    v.hz = reinterpret_cast<const R*>(b + L.off_hz[pi]);
    v.zmat = reinterpret_cast<const int*>(b + L.off_zmat);
    v.mat = reinterpret_cast<const R*>(b + L.off_mat[pi]);
    v.D = reinterpret_cast<const R*>(b + L.off_D[pi]);
    v.w = reinterpret_cast<const R*>(b + L.off_w[pi]);
    v.bc_top = c->prob.bc_top;
    v.bc_bottom = c->prob.bc_bottom;
    v.penalty_n2 = R(L.pen_z);
    for (int q = 0; q < 64; ++q) {
        const bool in = q < L.N * L.N;
        v.Dk[q] = in ? R(L.lgl.D[q]) : R(0);
        v.Dt[q] = in ? R(L.lgl.D[(q % L.N) * L.N + q / L.N]) : R(0);
    }
    return v;
}
template LevelView<double> view_of<double>(const dgtn_ctx*, const Level&);
template LevelView<float> view_of<float>(const dgtn_ctx*, const Level&);

template <typename R>
R* tau_of(const dgtn_ctx* c, const Level& L) {
    return reinterpret_cast<R*>(c->ws + L.off_tau[sizeof(R) == 8 ? 0 : 1]);
}
template double* tau_of<double>(const dgtn_ctx*, const Level&);
template float* tau_of<float>(const dgtn_ctx*, const Level&);

// First element of every layer on the finest level (layers occupy consecutive
// z-elements, elements are numbered iz * n_cols + col), and the element count.
std::vector<int> layer_first_elements(const dgtn_ctx* c) {
    const Level& L = c->levels[0];
    const int nl = (int)c->prob.layers.size();
    std::vector<int> e0(nl + 1, L.E);
    for (int iz = L.n_z - 1; iz >= 0; --iz) e0[L.zlayer[iz]] = iz * L.n_cols;
    return e0;
}

// Layer energies and, if U_compl is given, the compliance 1/2 u . b, with the
// per-element partial sums in ue / dot (E doubles each) and the per-layer sums
// in sums (n_layers + 1 doubles): device buffers of the caller's choosing.
// The results are copied to the host and the stream synchronised.
dgtn_status energy_into(dgtn_ctx* c, const double* u, double* ue, double* dot, double* sums, double* U_layers,
                        double* U_compl, hipStream_t s) {
    const Level& L = c->levels[0];
    const auto v = view_of<double>(c, L);
    const auto& P = c->prob;
    const int nl = (int)P.layers.size();
    const int* lay_e0 = reinterpret_cast<const int*>(c->ws + c->off_lay);
    hipError_t e = launch_energy(v, u, ue, s);
    if (e == hipSuccess && U_compl)
        e = launch_load_dot(v, reinterpret_cast<const double*>(c->ws + L.off_xy), P.F0, P.r0, P.xc, P.yc, u, dot, s);
    if (e == hipSuccess) e = launch_layer_sums(ue, U_compl ? dot : nullptr, lay_e0, nl, c->y_ref, 0.5, sums, s);
    if (e == hipSuccess) e = hipMemcpyAsync(U_layers, sums, 8 * (size_t)nl, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && U_compl) e = hipMemcpyAsync(U_compl, sums + nl, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error(std::string("energy: ") + hipGetErrorString(e));
        return DGTN_EHIP;
    }
    for (int k = 0; k < nl; ++k)
        if (!std::isfinite(U_layers[k])) { set_error("non-finite energy"); return DGTN_ENAN; }
    if (U_compl && !std::isfinite(*U_compl)) { set_error("non-finite compliance"); return DGTN_ENAN; }
    return DGTN_OK;
}

// Workspace plan: geometry of every level (FP64 and FP32 mirrors), face
// buffers, energy scratch, and the solver's vectors for `opts`.
static void plan_layout(dgtn_ctx* c, const dgtn_solve_opts* opts, Layout& lay) {
    lay.cursor = 0;
    for (auto& L : c->levels) {
        const size_t N = L.N, N2 = N * N;
        for (int pi = 0; pi < 2; ++pi) {
            const size_t rs = pi == 0 ? 8 : 4;
            L.off_geo2[pi] = lay.take(rs * L.n_cols * 5 * N2);
            L.off_sig[pi] = lay.take(rs * L.n_cols * 4 * N);
            L.off_fnrm[pi] = lay.take(rs * L.n_cols * 4 * 3 * N);
            L.off_hz[pi] = lay.take(rs * L.n_z);
            L.off_mat[pi] = lay.take(rs * level_mat(c, L).size());
            L.off_D[pi] = lay.take(rs * N2);
            L.off_w[pi] = lay.take(rs * N);
            L.off_tau[pi] = lay.take(rs * (size_t)L.E * 6 * 3 * N2);
        }
        L.off_cnbr = lay.take(sizeof(int) * L.n_cols * 4);
        L.off_cnf = lay.take(sizeof(int) * L.n_cols * 4);
        L.off_zmat = lay.take(sizeof(int) * L.n_z);
        L.off_xy = lay.take(8 * (size_t)L.n_cols * 2 * N2);
    }
    c->off_Ue = lay.take(8 * (size_t)c->levels[0].E);
    c->off_abc = lay.take(8 * 3 * (size_t)c->levels[0].E);
    c->off_lay = lay.take(sizeof(int) * (c->prob.layers.size() + 1));
    c->off_lsum = lay.take(8 * (c->prob.layers.size() + 1));
    plan_adjoint(c, lay);
    plan_residual(c, lay);
    plan_solver(c, opts, lay);
}

}  // namespace dgtn

using namespace dgtn;

#define DGTN_TRY(body)                                    \
    try {                                                 \
        body                                              \
    } catch (const std::exception& ex) {                  \
        set_error(ex.what());                             \
        return DGTN_EINVAL;                               \
    } catch (...) {                                       \
        set_error("unknown error");                       \
        return DGTN_EINVAL;                               \
    }

#define HIP_CHECK(call)                                                          \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            set_error(std::string(#call) + ": " + hipGetErrorString(e_));        \
            return DGTN_EHIP;                                                    \
        }                                                                        \
    } while (0)

// Positive definiteness of a material's stiffness (isotropic: Y > 0,
// -1 < nu < 1/2; cubic: c44 > 0, c11 > |c12|, c11 + 2 c12 > 0).
static bool material_ok(const dgtn_material& m) {
    if (m.kind == DGTN_MAT_ISO) return m.youngs > 0 && m.poisson > -1.0 && m.poisson < 0.5;
    if (m.kind == DGTN_MAT_CUBIC) return m.c44 > 0 && m.c11 > std::fabs(m.c12) && m.c11 + 2 * m.c12 > 0;
    return false;
}

static dgtn_status validate(const dgtn_problem* p) {
    if (!p) { set_error("null problem"); return DGTN_EINVAL; }
    if (p->p < 1 || p->p > 7) { set_error("p must be in 1..7"); return DGTN_EINVAL; }
    if (p->domain != DGTN_DOMAIN_CYLINDER && p->domain != DGTN_DOMAIN_BOX && p->domain != DGTN_DOMAIN_COLUMNS) {
        set_error("unknown domain"); return DGTN_EINVAL;
    }
    if (p->domain == DGTN_DOMAIN_COLUMNS) {
        if (p->n_columns < 1 || p->map_order < 1 || p->map_order > 8 || !p->columns_xy) {
            set_error("columns domain: need n_columns >= 1, map_order in 1..8 and the column maps");
            return DGTN_EINVAL;
        }
        if (p->refine != 0) { set_error("columns domain: refine must be 0"); return DGTN_EINVAL; }
        const size_t n = (size_t)p->n_columns * 2 * (p->map_order + 1) * (p->map_order + 1);
        for (size_t q = 0; q < n; ++q)
            if (!std::isfinite(p->columns_xy[q])) { set_error("columns domain: non-finite node"); return DGTN_EINVAL; }
    }
    if (p->domain == DGTN_DOMAIN_CYLINDER && !(p->R > 0)) { set_error("R must be > 0"); return DGTN_EINVAL; }
    if (p->domain == DGTN_DOMAIN_BOX && (!(p->Lx > 0) || !(p->Ly > 0) || p->nx < 1 || p->ny < 1)) {
        set_error("invalid box"); return DGTN_EINVAL;
    }
    if (p->refine < 0 || p->refine > 6) { set_error("refine must be in 0..6"); return DGTN_EINVAL; }
    if (p->n_layers < 1 || !p->layers) { set_error("need at least one layer"); return DGTN_EINVAL; }
    if (p->n_materials < 1 || p->n_materials > kMaxMaterials || !p->materials) {
        set_error("need 1..64 materials"); return DGTN_EINVAL;
    }
    for (int i = 0; i < p->n_layers; ++i) {
        const auto& l = p->layers[i];
        if (!(l.thickness > 0) || l.n_elem < 1 || !(l.ratio > 0) || l.material < 0 || l.material >= p->n_materials) {
            set_error("invalid layer " + std::to_string(i)); return DGTN_EINVAL;
        }
    }
    for (int i = 0; i < p->n_materials; ++i)
        if (!material_ok(p->materials[i])) {
            set_error("material " + std::to_string(i) + " is not positive definite");
            return DGTN_EINVAL;
        }
    const int bcs[3] = {p->bc_top, p->bc_bottom, p->bc_side};
    for (int b : bcs)
        if (b < DGTN_BC_DIRICHLET || b > DGTN_BC_FREE) { set_error("invalid boundary condition"); return DGTN_EINVAL; }
    if (!(p->penalty > 0)) { set_error("penalty must be > 0"); return DGTN_EINVAL; }
    if (!(p->r0 > 0)) { set_error("r0 must be > 0"); return DGTN_EINVAL; }
    return DGTN_OK;
}

// Device scratch of dgtn_energy_noalloc, for callers that cannot allocate device
// memory: per-element energies [kNoallocElems], per-element load products
// [kNoallocElems] and per-layer sums [kNoallocLayers + 1] (2.03 MiB per device,
// held until the process ends).  Host code never uses the array's name as an
// address: the device address is resolved once per device with
// hipGetSymbolAddress and kept in g_scratch_ptr.
static constexpr int kNoallocElems = 1 << 17;
static constexpr int kNoallocLayers = 4096;
static constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[2 * (size_t)kNoallocElems + kNoallocLayers + 1];
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device, resolved on the first call there.
static dgtn_status scratch_for_current_device(double** out) {
    int dev = -1;
    HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) { set_error("device index out of range"); return DGTN_EINVAL; }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) { set_error("no device address for the scratch array"); return DGTN_EHIP; }
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return DGTN_OK;
}

extern "C" {

dgtn_status dgtn_create(const dgtn_problem* p, dgtn_ctx** out) {
    if (!out) { set_error("null output"); return DGTN_EINVAL; }
    *out = nullptr;
    dgtn_status st = validate(p);
    if (st != DGTN_OK) return st;
    auto* c = new dgtn_ctx();
    try {
        Problem& P = c->prob;
        P.domain = p->domain;
        P.R = p->R;
        P.Lx = p->Lx;
        P.Ly = p->Ly;
        P.nx = p->nx;
        P.ny = p->ny;
        P.refine = p->refine;
        P.p = p->p;
        P.layers.assign(p->layers, p->layers + p->n_layers);
        P.materials.assign(p->materials, p->materials + p->n_materials);
        P.F0 = p->F0;
        P.r0 = p->r0;
        P.xc = p->xc;
        P.yc = p->yc;
        P.bc_top = p->bc_top;
        P.bc_bottom = p->bc_bottom;
        P.bc_side = p->bc_side;
        P.penalty = p->penalty;
        if (P.domain == DGTN_DOMAIN_COLUMNS) {
            P.n_cols_user = p->n_columns;
            P.map_order = p->map_order;
            const size_t n = (size_t)p->n_columns * 2 * (p->map_order + 1) * (p->map_order + 1);
            P.col_xy.assign(p->columns_xy, p->columns_xy + n);
        }
        c->matc = material_constants(P);
        c->y_ref = 0;
        for (size_t m = 0; m < c->matc.size(); m += 3) c->y_ref = std::max(c->y_ref, c->matc[m]);
        c->levels.push_back(build_level(P, P.p, P.refine, P.p, P.refine));
    } catch (const std::exception& ex) {
        set_error(std::string("mesh: ") + ex.what());
        delete c;
        return DGTN_EMESH;
    }
    *out = c;
    return DGTN_OK;
}

dgtn_status dgtn_get_info(const dgtn_ctx* c, dgtn_info* info) {
    if (!c || !info) { set_error("null argument"); return DGTN_EINVAL; }
    const Level& L = c->levels[0];
    info->n_elem = L.E;
    info->N = L.N;
    info->n_cols = L.n_cols;
    info->n_zelem = L.n_z;
    info->n_layers = (int)c->prob.layers.size();
    info->n_dof = 3LL * L.E * L.N * L.N * L.N;
    info->y_ref = c->y_ref;
    return DGTN_OK;
}

dgtn_status dgtn_workspace_bytes(const dgtn_ctx* cc, const dgtn_solve_opts* opts, size_t* bytes) {
    if (!cc || !bytes) { set_error("null argument"); return DGTN_EINVAL; }
    auto* c = const_cast<dgtn_ctx*>(cc);
    DGTN_TRY({
        dgtn_status st = prepare_levels(c, opts);
        if (st != DGTN_OK) return st;
        Layout lay;
        plan_layout(c, opts, lay);
        *bytes = lay.cursor + 256;
    })
    return DGTN_OK;
}

dgtn_status dgtn_bind(dgtn_ctx* c, void* ws, size_t bytes, const dgtn_solve_opts* opts, hipStream_t s) {
    if (!c || !ws) { set_error("null argument"); return DGTN_EINVAL; }
    if (reinterpret_cast<uintptr_t>(ws) % 256) { set_error("workspace must be 256-byte aligned"); return DGTN_EINVAL; }
    DGTN_TRY({
        dgtn_status st = prepare_levels(c, opts);
        if (st != DGTN_OK) return st;
        Layout lay;
        plan_layout(c, opts, lay);
        if (lay.cursor > bytes) {
            set_error("workspace too small: need " + std::to_string(lay.cursor) + " bytes");
            return DGTN_ENOMEM;
        }
        c->ws = static_cast<char*>(ws);
        c->ws_bytes = bytes;
        c->bound_opts = opts ? *opts : dgtn_solve_opts{};
        c->has_opts = opts != nullptr;
        // upload geometry, FP64 and FP32 mirrors
        const double yr = c->y_ref;
        c->staging.clear();
        auto put64 = [&](size_t off, const std::vector<double>& v) -> hipError_t {
            return hipMemcpyAsync(c->ws + off, v.data(), v.size() * 8, hipMemcpyHostToDevice, s);
        };
        auto put32 = [&](size_t off, const std::vector<double>& v) -> hipError_t {
            c->staging.emplace_back(v.size() * 4);
            auto& buf = c->staging.back();
            float* f = reinterpret_cast<float*>(buf.data());
            for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
            return hipMemcpyAsync(c->ws + off, f, v.size() * 4, hipMemcpyHostToDevice, s);
        };
        auto puti = [&](size_t off, const std::vector<int>& v) -> hipError_t {
            return hipMemcpyAsync(c->ws + off, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, s);
        };
        for (auto& L : c->levels) {
            HIP_CHECK(put64(L.off_geo2[0], L.geo2));
            HIP_CHECK(put32(L.off_geo2[1], L.geo2));
            HIP_CHECK(put64(L.off_sig[0], L.sig_side));
            HIP_CHECK(put32(L.off_sig[1], L.sig_side));
            HIP_CHECK(put64(L.off_fnrm[0], L.fnrm));
            HIP_CHECK(put32(L.off_fnrm[1], L.fnrm));
            HIP_CHECK(put64(L.off_hz[0], L.hz));
            HIP_CHECK(put32(L.off_hz[1], L.hz));
            std::vector<double> matn(level_mat(c, L));
            for (auto& v : matn) v /= yr;
            HIP_CHECK(put64(L.off_mat[0], matn));
            HIP_CHECK(put32(L.off_mat[1], matn));
            HIP_CHECK(put64(L.off_D[0], L.lgl.D));
            HIP_CHECK(put32(L.off_D[1], L.lgl.D));
            HIP_CHECK(put64(L.off_w[0], L.lgl.w));
            HIP_CHECK(put32(L.off_w[1], L.lgl.w));
            HIP_CHECK(puti(L.off_cnbr, L.cnbr));
            HIP_CHECK(puti(L.off_cnf, L.cnf));
            HIP_CHECK(puti(L.off_zmat, L.zmat));
            HIP_CHECK(put64(L.off_xy, L.xy));
        }
        HIP_CHECK(puti(c->off_lay, layer_first_elements(c)));
        st = bind_adjoint(c, s);
        if (st != DGTN_OK) return st;
        st = bind_residual(c, s);
        if (st != DGTN_OK) return st;
        st = bind_solver(c, s);
        if (st != DGTN_OK) return st;
        HIP_CHECK(hipStreamSynchronize(s));
        c->staging.clear();
        c->bound = true;
    })
    return DGTN_OK;
}

dgtn_status dgtn_apply_stage(dgtn_ctx* c, int precision, int stage, const void* u, void* Au, hipStream_t s) {
    if (!c || !u || !Au) { set_error("null argument"); return DGTN_EINVAL; }
    if (!c->bound) { set_error("no workspace bound"); return DGTN_EINVAL; }
    if (u == Au) { set_error("u and Au must not alias"); return DGTN_EINVAL; }
    if (stage < 1 || stage > 3) { set_error("stage must be 1, 2 or 3"); return DGTN_EINVAL; }
    const Level& L = c->levels[0];
    if (precision == 64) {
        auto v = view_of<double>(c, L);
        if (stage & 1) HIP_CHECK(launch_traction<double>(v, (const double*)u, tau_of<double>(c, L), s));
        if (stage & 2)
            HIP_CHECK(launch_apply<double>(v, (const double*)u, tau_of<double>(c, L), (double*)Au, c->y_ref, s));
    } else if (precision == 32) {
        auto v = view_of<float>(c, L);
        if (stage & 1) HIP_CHECK(launch_traction<float>(v, (const float*)u, tau_of<float>(c, L), s));
        if (stage & 2)
            HIP_CHECK(launch_apply<float>(v, (const float*)u, tau_of<float>(c, L), (float*)Au, (float)c->y_ref, s));
    } else {
        set_error("precision must be 64 or 32");
        return DGTN_EINVAL;
    }
    return DGTN_OK;
}

dgtn_status dgtn_apply(dgtn_ctx* c, int precision, const void* u, void* Au, hipStream_t s) {
    return dgtn_apply_stage(c, precision, 3, u, Au, s);
}

dgtn_status dgtn_rhs(dgtn_ctx* c, double* b, hipStream_t s) {
    if (!c || !b) { set_error("null argument"); return DGTN_EINVAL; }
    if (!c->bound) { set_error("no workspace bound"); return DGTN_EINVAL; }
    const Level& L = c->levels[0];
    auto v = view_of<double>(c, L);
    const auto& P = c->prob;
    HIP_CHECK(launch_rhs(v, reinterpret_cast<const double*>(c->ws + L.off_xy), P.F0, P.r0, P.xc, P.yc, 0, b, s));
    return DGTN_OK;
}

dgtn_status dgtn_energy(dgtn_ctx* c, const double* u, double* U_layers, double* U_compl, hipStream_t s) {
    if (!c || !u || !U_layers) { set_error("null argument"); return DGTN_EINVAL; }
    if (!c->bound) { set_error("no workspace bound"); return DGTN_EINVAL; }
    return energy_into(c, u, reinterpret_cast<double*>(c->ws + c->off_Ue), reinterpret_cast<double*>(c->ws + c->off_abc),
                       reinterpret_cast<double*>(c->ws + c->off_lsum), U_layers, U_compl, s);
}

dgtn_status dgtn_energy_noalloc(dgtn_ctx* c, const double* u, double* U_layers, double* U_compl, hipStream_t s) {
    if (!c || !u || !U_layers) { set_error("null argument"); return DGTN_EINVAL; }
    const Level& L = c->levels[0];
    if (L.E > kNoallocElems) {
        set_error("dgtn_energy_noalloc: " + std::to_string(L.E) + " elements exceed its maximum of " +
                  std::to_string(kNoallocElems));
        return DGTN_EINVAL;
    }
    if ((int)c->prob.layers.size() > kNoallocLayers) {
        set_error("dgtn_energy_noalloc: more than " + std::to_string(kNoallocLayers) + " layers");
        return DGTN_EINVAL;
    }
    if (!c->bound) { set_error("no workspace bound"); return DGTN_EINVAL; }
    double* sp = nullptr;
    const dgtn_status st = scratch_for_current_device(&sp);
    if (st != DGTN_OK) return st;
    return energy_into(c, u, sp, sp + kNoallocElems, sp + 2 * (size_t)kNoallocElems, U_layers, U_compl, s);
}

dgtn_status dgtn_material_constants(const dgtn_material* m, double* out) {
    if (!m || !out) { set_error("null argument"); return DGTN_EINVAL; }
    if (!material_ok(*m)) { set_error("material is not positive definite"); return DGTN_EINVAL; }
    Problem P;
    P.materials.assign(1, *m);
    const std::vector<double> c = material_constants(P);
    std::copy(c.begin(), c.end(), out);
    return DGTN_OK;
}

dgtn_status dgtn_jump_indicator(dgtn_ctx* c, const double* u, int faces, double* eta_elem, double* eta_layers,
                                hipStream_t s) {
    if (!c || !u || (!eta_elem && !eta_layers)) { set_error("null argument"); return DGTN_EINVAL; }
    if ((faces & DGTN_FACES_ALL) == 0 || (faces & ~(DGTN_FACES_ALL | DGTN_FACES_PENALTY)) != 0) {
        set_error("faces must be 1, 2 or 3, optionally or-ed with DGTN_FACES_PENALTY (4)");
        return DGTN_EINVAL;
    }
    if (!c->bound) { set_error("no workspace bound"); return DGTN_EINVAL; }
    const Level& L = c->levels[0];
    auto v = view_of<double>(c, L);
    double* d = reinterpret_cast<double*>(c->ws + c->off_Ue);  // per-element scratch of the energies
    HIP_CHECK(launch_jump_indicator(v, u, faces, d, s));
    std::vector<double> h(L.E);
    HIP_CHECK(hipMemcpyAsync(h.data(), d, 8 * (size_t)L.E, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    for (int e = 0; e < L.E; ++e)
        if (!std::isfinite(h[e])) { set_error("non-finite indicator"); return DGTN_ENAN; }
    if (eta_elem) std::copy(h.begin(), h.end(), eta_elem);
    if (eta_layers) {
        const int nl = (int)c->prob.layers.size();
        for (int k = 0; k < nl; ++k) eta_layers[k] = 0;
        for (int e = 0; e < L.E; ++e) eta_layers[L.zlayer[e / L.n_cols]] += h[e];  // fixed order
    }
    return DGTN_OK;
}

dgtn_status dgtn_energy_parts(dgtn_ctx* c, const double* u, double* parts, hipStream_t s) {
    if (!c || !u || !parts) { set_error("null argument"); return DGTN_EINVAL; }
    if (!c->bound) { set_error("no workspace bound"); return DGTN_EINVAL; }
    const Level& L = c->levels[0];
    auto v = view_of<double>(c, L);
    double* abc = reinterpret_cast<double*>(c->ws + c->off_abc);
    HIP_CHECK(launch_energy_invariants(v, u, abc, s));
    std::vector<double> h((size_t)3 * L.E);
    HIP_CHECK(hipMemcpyAsync(h.data(), abc, 8 * h.size(), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    const int nl = (int)c->prob.layers.size();
    std::vector<double> inv((size_t)3 * nl, 0.0);
    for (int e = 0; e < L.E; ++e) {  // fixed order: deterministic
        const int k = L.zlayer[e / L.n_cols];
        for (int q = 0; q < 3; ++q) inv[(size_t)3 * k + q] += h[(size_t)3 * e + q];
    }
    for (int k = 0; k < nl; ++k) {
        const int m = c->prob.layers[k].material;
        const double c11 = c->matc[3 * m], c12 = c->matc[3 * m + 1], c44 = c->matc[3 * m + 2];
        const double A = inv[3 * k], B = inv[3 * k + 1], C = inv[3 * k + 2];
        double* out = parts + 3 * k;
        if (c->prob.materials[m].kind == DGTN_MAT_ISO) {
            const double K = (c11 + 2.0 * c12) / 3.0;  // lambda + 2 mu / 3
            out[0] = K * (A + B);
            out[1] = c11 * A + c12 * B + c44 * C - out[0];
            out[2] = 0.0;
        } else {
            out[0] = c11 * A;
            out[1] = c12 * B;
            out[2] = c44 * C;
        }
        for (int q = 0; q < 3; ++q)
            if (!std::isfinite(out[q])) { set_error("non-finite energy"); return DGTN_ENAN; }
    }
    return DGTN_OK;
}

dgtn_status dgtn_noise_psd_parts(const double* parts, const double* phi, int n_layers, double T, double f, double F0,
                                 double* S) {
    if (!parts || !phi || !S || n_layers < 1) { set_error("invalid argument"); return DGTN_EINVAL; }
    if (!(T > 0) || !(f > 0) || !(F0 != 0)) { set_error("T, f must be > 0 and F0 != 0"); return DGTN_EINVAL; }
    const double kB = 1.380649e-23;
    double W = 0;
    for (int q = 0; q < 3 * n_layers; ++q) W += phi[q] * parts[q];
    *S = 4.0 * kB * T * W / (M_PI * f * F0 * F0);
    return DGTN_OK;
}

dgtn_status dgtn_noise_psd(const double* U, const double* phi, int n, double T, double f, double F0, double* S) {
    if (!U || !phi || !S || n < 1) { set_error("invalid argument"); return DGTN_EINVAL; }
    if (!(T > 0) || !(f > 0) || !(F0 != 0)) { set_error("T, f must be > 0 and F0 != 0"); return DGTN_EINVAL; }
    const double kB = 1.380649e-23;
    double W = 0;
    for (int k = 0; k < n; ++k) W += phi[k] * U[k];
    *S = 4.0 * kB * T * W / (M_PI * f * F0 * F0);
    return DGTN_OK;
}

dgtn_status dgtn_node_coords(const dgtn_ctx* c, double* xyz) {
    if (!c || !xyz) { set_error("null argument"); return DGTN_EINVAL; }
    const Level& L = c->levels[0];
    const int N = L.N, N2 = N * N, N3 = N2 * N;
    const auto& x = L.lgl.x;
    for (int e = 0; e < L.E; ++e) {
        const int col = e % L.n_cols, iz = e / L.n_cols;
        double* o = xyz + (size_t)e * 3 * N3;
        for (int k = 0; k < N; ++k)
            for (int q = 0; q < N2; ++q) {
                o[k * N2 + q] = L.xy[(size_t)col * 2 * N2 + q];
                o[N3 + k * N2 + q] = L.xy[(size_t)col * 2 * N2 + N2 + q];
                o[2 * N3 + k * N2 + q] = L.ztop[iz] + 0.5 * (x[k] + 1.0) * L.hz[iz];
            }
    }
    return DGTN_OK;
}

void dgtn_destroy(dgtn_ctx* c) { delete c; }

const char* dgtn_last_error(void) { return g_err.c_str(); }

}  // extern "C"
