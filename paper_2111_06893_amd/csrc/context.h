// The library context and the interfaces between its translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "ddouble.h"
#include "dual.h"
#include "internal.h"

namespace dgtn {

// Workspace offsets of the adjoint's dual-number copies of the finest level.
struct AdjointLayout {
    bool ok = false;  // allocated (the dual kernels cover N <= 8)
    size_t wz = 0, u = 0, Au = 0, tau = 0, geo2 = 0, sig = 0, fnrm = 0, hz = 0, mat = 0, D = 0, w = 0, Ue = 0;
    size_t partial = 0, dots = 0;
    int nblk = 0;
};

// Workspace offsets of the double-double copies of the finest level's
// coefficient tables (the extended-precision residual).
struct ResidualLayout {
    bool ok = false;  // available (the 16-byte kernels cover N <= 8)
    size_t geo2 = 0, sig = 0, fnrm = 0, hz = 0, mat = 0, D = 0, w = 0;
};

struct Layout {
    size_t cursor = 0;
    size_t take(size_t bytes);  // 256-byte aligned bump allocation
};

struct SolverState;  // defined in solver.hip

}  // namespace dgtn

struct dgtn_ctx {
    dgtn::Problem prob;
    std::vector<dgtn::Level> levels;  // levels[0] is the problem's own resolution
    std::vector<double> matc;         // c11, c12, c44 per material (Pa)
    double y_ref = 1;                 // modulus scale of the device arithmetic
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    dgtn_solve_opts bound_opts{};
    bool has_opts = false;
    size_t off_Ue = 0, off_abc = 0;
    size_t off_lay = 0, off_lsum = 0;  // per-layer first elements [n_layers + 1]; per-layer sums [n_layers + 1]
    dgtn::AdjointLayout adj;
    dgtn::ResidualLayout res;
    std::vector<std::vector<char>> staging;  // host staging of FP32 uploads
    dgtn::SolverState* solver = nullptr;
    ~dgtn_ctx();
};

namespace dgtn {

// materials of a level (the problem's own unless the level merged layers)
inline const std::vector<double>& level_mat(const dgtn_ctx* c, const Level& L) {
    return L.mat.empty() ? c->matc : L.mat;
}

template <typename R>
LevelView<R> view_of(const dgtn_ctx* c, const Level& L);
template <typename R>
R* tau_of(const dgtn_ctx* c, const Level& L);

template <typename R>
hipError_t launch_traction(const LevelView<R>& L, const R* u, R* tau, hipStream_t s);
template <typename R>
hipError_t launch_apply(const LevelView<R>& L, const R* u, const R* tau, R* out, R scale, hipStream_t s);
hipError_t launch_rhs(const LevelView<double>& L, const double* xy, double F0, double r0, double xc, double yc,
                      int mode, double* b, hipStream_t s);
hipError_t launch_load_dot(const LevelView<double>& L, const double* xy, double F0, double r0, double xc, double yc,
                           const double* u, double* out, hipStream_t s);
hipError_t launch_layer_sums(const double* v, const double* dot, const int* lay_e0, int n_layers, double scale,
                             double dot_scale, double* sums, hipStream_t s);
template <typename R>
hipError_t launch_energy(const LevelView<R>& L, const double* u, R* Ue, hipStream_t s);
hipError_t launch_energy_invariants(const LevelView<double>& L, const double* u, double* abc, hipStream_t s);
hipError_t launch_jump_indicator(const LevelView<double>& L, const double* u, int which, double* eta,
                                 hipStream_t s);
hipError_t launch_energy_grad(const LevelView<double>& L, const double* u, const double* wz, double* g, double scale,
                              hipStream_t s);
template <>
hipError_t launch_traction<Dual>(const LevelView<Dual>& L, const Dual* u, Dual* tau, hipStream_t s);
template <>
hipError_t launch_apply<Dual>(const LevelView<Dual>& L, const Dual* u, const Dual* tau, Dual* out, Dual scale,
                              hipStream_t s);
template <>
hipError_t launch_energy<Dual>(const LevelView<Dual>& L, const double* u, Dual* Ue, hipStream_t s);
template <>
hipError_t launch_traction<DD>(const LevelView<DD>& L, const DD* u, DD* tau, hipStream_t s);
template <>
hipError_t launch_apply<DD>(const LevelView<DD>& L, const DD* u, const DD* tau, DD* out, DD scale, hipStream_t s);

// residual.hip
void plan_residual(dgtn_ctx* c, Layout& lay);
dgtn_status bind_residual(dgtn_ctx* c, hipStream_t s);
hipError_t residual_dd(dgtn_ctx* c, const double* b, const double* u, double* r, hipStream_t s);

// adjoint.hip
void plan_adjoint(dgtn_ctx* c, Layout& lay);
dgtn_status bind_adjoint(dgtn_ctx* c, hipStream_t s);

// solver.hip
dgtn_status prepare_levels(dgtn_ctx* c, const dgtn_solve_opts* opts);
void plan_solver(dgtn_ctx* c, const dgtn_solve_opts* opts, Layout& lay);
dgtn_status bind_solver(dgtn_ctx* c, hipStream_t s);

}  // namespace dgtn
