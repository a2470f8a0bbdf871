// Internal declarations of the dgtn library (host side and kernel launchers).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dgtn.h"

namespace dgtn {

constexpr int kMaxN = 8;
constexpr int kMaxMaterials = 64;

// One-dimensional LGL rule: nodes x, weights w, D[i*N + j] = l_j'(x_i).
struct Lgl {
    int N = 0;
    std::vector<double> x, w, D;
};
Lgl make_lgl(int N);
// Lagrange interpolation matrix I[a*N + j] = l_j(y_a) through the nodes of `from`.
std::vector<double> lagrange_matrix(const Lgl& from, const std::vector<double>& y);

// Device-side view of one discretisation level, in precision R.  All arrays
// live in the bound workspace.
template <typename R>
struct LevelView {
    int N, n_cols, n_z, E;
    // The operator and energy kernels process the E elements e0, e0 + 1, ... (the
    // whole level with e0 = 0; a range of z-layers for parameter derivatives).
    int e0;
    const R* geo2;       // [n_cols][5][N*N]: a^xi_x, a^xi_y, a^eta_x, a^eta_y, det2
    const R* sig_side;   // [n_cols][4][N]   penalty sigma on the side faces
    const R* fnrm;       // [n_cols][4][3][N] side faces: outward unit normal n_x, n_y and |grad xi^m|
    const int* cnbr;     // [n_cols][4]      neighbour column or -1
    const int* cnf;      // [n_cols][4]      neighbour face | flip << 2, or the bc code if boundary
    const R* hz;         // [n_z]            element thickness
    const int* zmat;     // [n_z]            material index
    const R* mat;        // [n_mat][3]       c11, c12, c44 divided by y_ref
    const R* D;          // [N*N]
    const R* w;          // [N]
    int bc_top, bc_bottom;
    R penalty_n2;        // C * N^2
    // D by value: the kernels read it from the kernel-argument segment with
    // wave-uniform indices, i.e. through scalar loads instead of LDS.
    R Dk[64];            // D[x * N + a], N <= 8
    R Dt[64];            // D^T
};

// Host description of one level (mesh + geometry), built from the problem.
struct Level {
    int N = 0, refine = 0, n_cols = 0, n_z = 0, E = 0;
    double pen_z = 0;    // C (p0 + 1)^2 of the finest level, used on every level
    Lgl lgl;
    std::vector<double> geo2, xy, sig_side;
    std::vector<double> fnrm;  // [n_cols][4][3][N]: n_x, n_y, |grad xi^m| at the side-face nodes
    std::vector<int> cnbr, cnf;
    std::vector<double> hz, ztop;
    std::vector<int> zmat, zlayer;
    // c11, c12, c44 (Pa) of the materials zmat indexes on this level; empty on levels
    // that use the problem's own materials (z-coarsened levels add effective ones)
    std::vector<double> mat;
    // workspace offsets (bytes) of the uploaded arrays, FP64 and FP32 mirrors
    size_t off_geo2[2], off_sig[2], off_fnrm[2], off_hz[2], off_mat[2], off_D[2], off_w[2];
    size_t off_cnbr, off_cnf, off_zmat, off_xy;
    size_t off_tau[2];   // face traction buffer [E][6][3][N*N]
};

struct Problem {
    int domain = 0;
    double R = 1, Lx = 1, Ly = 1;
    int nx = 1, ny = 1;
    int refine = 0, p = 1;
    std::vector<dgtn_layer> layers;
    std::vector<dgtn_material> materials;
    double F0 = 1, r0 = 0.1, xc = 0, yc = 0;
    int bc_top = DGTN_BC_PRESSURE, bc_bottom = DGTN_BC_DIRICHLET, bc_side = DGTN_BC_FREE;
    double penalty = 100;
    // explicit 2D mesh (DGTN_DOMAIN_COLUMNS): column maps of degree map_order at
    // the LGL points, [n_cols][2][(map_order + 1)^2]
    int n_cols_user = 0, map_order = 0;
    std::vector<double> col_xy;
};

// Builds the level of polynomial degree p with `refine` horizontal splits.
// The penalty of eq. penalty is that of the finest level (degree p0,
// refinement r0) on every level: C (p0 + 1)^2 / h on z-faces, and on side
// faces with the width of the finest columns (h / 2^(r0 - refine)), so that a
// coarse level's penalty matches the fine operator restricted to coarse
// functions.  Throws std::runtime_error with a message on invalid meshes.
Level build_level(const Problem& prob, int p, int refine, int p0, int r0);

// Cubic constants (c11, c12, c44) of each material in Pa.
std::vector<double> material_constants(const Problem& prob);

void set_error(const std::string& msg);

}  // namespace dgtn
