// Launchers of the preconditioner and vector-algebra kernels (mg.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace dgtn {

template <typename R>
hipError_t mg_smooth(int N, int E, const R* fdm, const R* b, const R* Ax, R* x, R omega, hipStream_t s);
// V [2][3][n][n]: the z-eigenvectors of each component (row = z node), then their transposes
template <typename R>
hipError_t mg_col_smooth(int N, int n_cols, int n_z, const R* S, const R* lam, const R* rat, const R* V,
                         const R* lz, const R* b, const R* Ax, R* x, R omega, R* T, R* Y, hipStream_t s);
// overlapping column patches of width P = N + 2k (gather table pg, sum table ps)
template <typename R>
hipError_t mg_ovl_smooth(int N, int n_cols, int n_z, int P, const int* pg, const int* ps, const R* wsq,
                         const R* S, const R* lam, const R* rat, const R* V, const R* lz, const R* b, const R* Ax,
                         R* x, R omega, R* T, R* Y, hipStream_t s);
template <typename R>
hipError_t mg_prolong_z(int N, int Ef, int n_cols, const int* zpar, const R* Iz, const R* uc, R* uf, hipStream_t s);
template <typename R>
hipError_t mg_restrict_z(int N, int Ec, int n_cols, const int* zch, const R* Iz, const R* rf, R* rc, hipStream_t s);
template <typename R>
hipError_t mg_prolong_p(int E, int Nf, int Nc, const R* I, const R* uc, R* uf, hipStream_t s);
template <typename R>
hipError_t mg_restrict_p(int E, int Nf, int Nc, const R* I, const R* rf, R* rc, hipStream_t s);
template <typename R>
hipError_t mg_prolong_h(int N, int Ef, int ncf, int ncc, const int* parent, const int* child, const R* Ih,
                        const R* uc, R* uf, hipStream_t s);
template <typename R>
hipError_t mg_restrict_h(int N, int Ec, int ncf, int ncc, const int* children, const R* Ih, const R* rf, R* rc,
                         hipStream_t s);

hipError_t dense_set_unit(double* e, int j, hipStream_t s);
// In-place inverse of the n x n SPD matrix A (blocked Gauss-Jordan, no pivoting);
// scratch: dense_invert_scratch(n) doubles of device memory.
size_t dense_invert_scratch(int n);
hipError_t dense_invert(double* A, double* scratch, int n, hipStream_t s);
template <typename R>
hipError_t dense_gemv(const R* A, const R* x, R* y, int n, hipStream_t s);

template <typename R>
hipError_t vec_zero(R* x, size_t n, hipStream_t s);
template <typename A, typename B>
hipError_t vec_cast(const A* x, B* y, size_t n, double scale, hipStream_t s);
template <typename R>
hipError_t vec_resid(const R* b, R* y, size_t n, hipStream_t s);
hipError_t vec_multidot(const double* V, size_t ldv, int nv, const double* w, size_t n, double* partial, int nblk,
                        double* out, hipStream_t s);
hipError_t vec_multiaxpy(double* w, const double* V, size_t ldv, int nv, const double* coef, size_t n,
                         hipStream_t s);
hipError_t vec_scale_copy(const double* x, double* y, double a, size_t n, hipStream_t s);
hipError_t vec_axpy(double* y, double a, const double* x, size_t n, hipStream_t s);
hipError_t vec_xpby(double* p, const double* z, double beta, size_t n, hipStream_t s);
// flexible-CG vector steps reading their scalars from device memory; r32, if
// not null, receives the new residual times scale32 (a power of two) in FP32
hipError_t fcg_update(double* u, double* r, const double* p, const double* q, const double* cur, double* sc,
                      float* r32, double scale32, size_t n, hipStream_t s);
hipError_t fcg_direction(double* p, const double* z, const double* cur, const double* nxt, size_t n,
                         hipStream_t s);
// out[v] = x[v] . y[v] for v < np <= 4 (deterministic order)
hipError_t vec_dotpairs(int np, const double* const* x, const double* const* y, size_t n, double* partial, int nblk,
                        double* out, hipStream_t s);
// zn = unscale * (double) z32, then out[0..2] = r . zn, r . zo, r . r (as vec_dotpairs with those pairs)
hipError_t vec_dot3_widen(const double* r, const float* z32, double* zn, const double* zo, double unscale, size_t n,
                          double* partial, int nblk, double* out, hipStream_t s);

}  // namespace dgtn
