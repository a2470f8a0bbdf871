/*
 * dgtn.h -- C ABI of the MI355X (gfx950) discontinuous-Galerkin elasticity
 * library for Brownian thermal noise in layered mirrors.
 *
 * Method: Vu et al., "High-accuracy numerical models of Brownian thermal noise
 * in thin mirror coatings" (arXiv:2111.06893).  The library solves the
 * auxiliary elastostatic problem of Sec. 2.1 (eqs. Newton, Hooke,
 * elasticity_eqns) with the DG discretisation of Sec. 2.2 (eqs. dg_residuals,
 * numflux, penalty, bc) and the Krylov solve of Sec. 2.3 (eq. matrix_eqn), and
 * returns the elastic energy U (per layer) and the noise S_x of eqs.
 * thermalnoise / wdiss.
 *
 * Conventions
 *  - Every call returns a dgtn_status; 0 is success, negative is failure, and
 *    dgtn_last_error() then returns a thread-local message.  No C++ exception
 *    crosses this interface.
 *  - Units are SI.  Device pointers are HIP device memory owned by the caller;
 *    the library never frees caller memory.  Host pointers are plain host
 *    memory.  Streams are the caller's; calls that return host values
 *    synchronise the stream they were given.
 *  - Field layout: u[e][c][k][j][i] (i fastest), c the Cartesian component,
 *    (i, j, k) the LGL node indices along (xi, eta, zeta); zeta = -1 is the
 *    element side nearer the loaded face z = 0.  Elements are numbered
 *    e = iz * n_cols + col, iz counted from z = 0 downward; cylinder columns are
 *    numbered block-major (centre square, wedges +x, +y, -x, -y), then by the
 *    sub-square (s, t) of the block's 2^refine x 2^refine split, s fastest.
 *  - The library allocates no device memory: the caller binds one device
 *    workspace (dgtn_workspace_bytes / dgtn_bind) that holds the geometry,
 *    face buffers, solver vectors and preconditioner data.
 *  - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef DGTN_H
#define DGTN_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque library context: problem, mesh and host-side geometry. */
typedef struct dgtn_ctx dgtn_ctx;

typedef enum {
    DGTN_OK = 0,
    DGTN_EINVAL = -1,   /* invalid argument or problem description         */
    DGTN_EMESH = -2,    /* mesh construction failed (non-conforming, det<=0)*/
    DGTN_EHIP = -3,     /* a HIP runtime call failed                       */
    DGTN_ENOCONV = -4,  /* solver hit its iteration limit or stagnated     */
    DGTN_ENOMEM = -5,   /* bound workspace too small                       */
    DGTN_ENAN = -6      /* NaN/Inf met in the solver                       */
} dgtn_status;

enum { DGTN_DOMAIN_CYLINDER = 0, DGTN_DOMAIN_BOX = 1, DGTN_DOMAIN_COLUMNS = 2 };
enum { DGTN_MAT_ISO = 0, DGTN_MAT_CUBIC = 1 };
/* Boundary conditions (Sec. 2.2.4, eqs. bc, BCfixed, BCfree). */
enum { DGTN_BC_DIRICHLET = 1, DGTN_BC_PRESSURE = 2, DGTN_BC_FREE = 3 };

/* Constitutive relation of one material: isotropic (eq. constrel_iso, given
 * by Young's modulus and Poisson ratio) or cubic with crystal axes along
 * x, y, z (eq. constrel_cryst). */
typedef struct {
    int kind;                 /* DGTN_MAT_ISO or DGTN_MAT_CUBIC */
    double youngs, poisson;   /* used when kind == DGTN_MAT_ISO */
    double c11, c12, c44;     /* used when kind == DGTN_MAT_CUBIC */
} dgtn_material;

/* One z-layer (Sec. 2.2.1): thickness, number of elements across it, the
 * geometric growth factor of consecutive element thicknesses (1 = uniform)
 * and its material index. */
typedef struct {
    double thickness;
    int n_elem;
    double ratio;
    int material;
} dgtn_layer;

/* Problem description (Sec. 2.1 and 2.2.1).  Cylinder: radius R, five blocks
 * (centre square of half-width R/(2 sqrt 2) and four wedges blending its edges
 * into the arc), each split 2^refine x 2^refine.  Box:
 * [-Lx/2, Lx/2] x [-Ly/2, Ly/2] with nx x ny columns.  Columns: an explicit
 * 2D mesh of n_columns quadrilateral columns, each given by its isoparametric
 * map of degree map_order (1..8): columns_xy[c][d][j][i] (d = 0 x, 1 y; i
 * along xi fastest, j along eta) is the map at the LGL points (x_i, x_j) of
 * degree map_order, with det > 0 (counter-clockwise); the library takes the
 * map at its own nodes by Lagrange interpolation, matches neighbouring
 * columns by their edge nodes (conforming edges only) and tags the unmatched
 * edges as the side boundary; refine must be 0 (the multigrid then coarsens in
 * degree and across layers only).  columns_xy is copied by dgtn_create.  In z
 * the layers are stacked from the loaded face z = 0 downward.  Load: Gaussian
 * pressure of eq. laserbeam with total force F0, width r0, centred at (xc, yc),
 * on faces tagged DGTN_BC_PRESSURE.  penalty is C of eq. penalty (100 in the
 * paper). */
typedef struct {
    int domain;
    double R;
    int refine;
    double Lx, Ly;
    int nx, ny;
    int p;                    /* polynomial degree, N = p + 1 LGL points, 1..7 */
    int n_layers;
    const dgtn_layer* layers;
    int n_materials;
    const dgtn_material* materials;
    double F0, r0, xc, yc;
    int bc_top, bc_bottom, bc_side;
    double penalty;
    int n_columns;            /* DGTN_DOMAIN_COLUMNS only                      */
    int map_order;
    const double* columns_xy; /* [n_columns][2][map_order + 1][map_order + 1]  */
} dgtn_problem;

typedef struct {
    int n_elem, N, n_cols, n_zelem, n_layers;
    long long n_dof;          /* 3 * n_elem * N^3 */
    double y_ref;             /* modulus scale of the internal arithmetic (Pa) */
} dgtn_info;

/* Krylov solve (Sec. 2.3): flexible CG or restarted flexible GMRES in FP64
 * on A u = b, preconditioned by a multigrid V-cycle whose levels run in
 * precond_precision (64 or 32 bit); the FP64 true residual is recomputed
 * periodically and at convergence (iterative refinement when the
 * preconditioner is FP32).  mg_levels = 1 uses the additive-Schwarz smoother
 * alone, 0 no preconditioner.  The paper's Schwarz subdomains overlap; with
 * column subdomains, overlap = k > 0 extends every column by k node lines into
 * each horizontal neighbour (and the k x k corner blocks of the diagonal
 * neighbours), k < N on every level (clamped). */
typedef struct {
    int precond_precision;    /* 64 or 32                                      */
    int restart;              /* FGMRES restart length m (1..200)              */
    int max_iter;             /* total iteration cap                           */
    double rtol;              /* stop at ||b - A u|| <= rtol ||b||             */
    int mg_levels;            /* at most this many V-cycle levels (1 = smoother
                                 only): degree halved to 1, then 2 x 2 columns
                                 merged, then z-element pairs merged into
                                 fiducial layers while the coarsest level has
                                 more than 4096 unknowns                       */
    int smooth_steps;         /* pre- and post-smoothing sweeps per level       */
    double smooth_damping;    /* damping of the additive Schwarz smoother      */
    int smoother;             /* Schwarz subdomains: DGTN_SMOOTH_ELEMENT or DGTN_SMOOTH_COLUMN */
    int krylov;               /* DGTN_KRYLOV_FGMRES or DGTN_KRYLOV_FCG          */
    int overlap;              /* column-subdomain overlap in node lines (0..3)  */
    int residual_precision;   /* true residual b - A u: 64 (or 0) FP64, 128
                                 double-double (dgtn_residual)                  */
} dgtn_solve_opts;

/* Additive-Schwarz subdomains: one element, or one whole z-column of elements
 * (all layers under one 2D column), each solved by fast diagonalisation of a
 * separable approximation of its block. */
enum { DGTN_SMOOTH_ELEMENT = 0, DGTN_SMOOTH_COLUMN = 1 };
/* Outer Krylov method in FP64: restarted flexible GMRES (the paper's GMRES,
 * flexible so that the preconditioner may vary), or flexible conjugate
 * gradients (A is symmetric positive definite with a Dirichlet face). */
enum { DGTN_KRYLOV_FGMRES = 0, DGTN_KRYLOV_FCG = 1 };

typedef struct {
    int iters;
    int restarts;
    double rel_res;           /* final true relative residual (FP64)          */
    double t_solve_s;         /* wall time of the solve                         */
} dgtn_solve_stats;

/* Builds the mesh and the host-side geometry of the problem (Sec. 2.2.1:
 * isoparametric element maps, Jacobians, normals, surface Jacobians, widths h
 * and penalties of eq. penalty).  Validates: p in 1..7, positive thicknesses,
 * positive-definite materials (isotropic: Y > 0, -1 < nu < 1/2; cubic:
 * c44 > 0, c11 > |c12|, c11 + 2 c12 > 0), conforming faces, det J > 0.
 * On success *ctx owns host memory only. */
dgtn_status dgtn_create(const dgtn_problem* prob, dgtn_ctx** ctx);

dgtn_status dgtn_get_info(const dgtn_ctx* ctx, dgtn_info* info);

/* Bytes of device workspace needed for the apply/rhs/energy calls and, if
 * opts is non-NULL, for dgtn_solve with those options. */
dgtn_status dgtn_workspace_bytes(const dgtn_ctx* ctx, const dgtn_solve_opts* opts,
                                 size_t* bytes);

/* Binds a device workspace of `bytes` bytes (256-byte aligned) and uploads
 * the geometry into it on `stream`.  opts as in dgtn_workspace_bytes.  The
 * workspace must stay allocated until dgtn_destroy or the next dgtn_bind.
 * Binding discards the V-cycles recorded as HIP graphs (dgtn_solve), which
 * refer to the previous workspace.  Synchronises the stream. */
dgtn_status dgtn_bind(dgtn_ctx* ctx, void* workspace, size_t bytes,
                      const dgtn_solve_opts* opts, hipStream_t stream);

/* Au = A u, the matrix-free DG operator of eq. dg_residuals (weak form, flux
 * of eq. numflux with averaged moduli, penalty of eq. penalty, homogeneous
 * boundary data of eq. bc), in SI units.  precision 64: u, Au are double;
 * precision 32: float.  u and Au are device arrays of n_dof values in the
 * field layout and must not alias. */
dgtn_status dgtn_apply(dgtn_ctx* ctx, int precision, const void* u, void* Au,
                       hipStream_t stream);

/* One pass of dgtn_apply, for timing each kernel on its own: stage 1 runs
 * the face-traction pass (n . Y . D u on every element face node, into the
 * workspace face buffer), stage 2 the volume-and-flux pass that reads that
 * buffer and writes Au, stage 3 both (= dgtn_apply).  Stage 2 alone is only
 * meaningful after a stage 1 on the same u. */
dgtn_status dgtn_apply_stage(dgtn_ctx* ctx, int precision, int stage, const void* u, void* Au,
                             hipStream_t stream);

/* b = load vector of the Gaussian pressure (eq. laserbeam, scaled by F0) on
 * the DGTN_BC_PRESSURE faces, entering through the Neumann flux of eq. bc
 * (device, double, n_dof). */
dgtn_status dgtn_rhs(dgtn_ctx* ctx, double* b, hipStream_t stream);

/* Solves A u = b; u holds the initial guess on entry and the solution on
 * exit (device, double).  Returns DGTN_ENOCONV if max_iter is reached or
 * the residual stagnates above rtol (flexible CG: no 1 % progress in 200
 * iterations, or positive curvature lost twice without progress of the true
 * residual -- rtol below the attainable accuracy); u then holds the last
 * iterate.  DGTN_ENAN on a NaN/Inf. */
dgtn_status dgtn_solve(dgtn_ctx* ctx, const dgtn_solve_opts* opts, const double* b,
                       double* u, dgtn_solve_stats* stats, hipStream_t stream);

/* r = b - A u with A u evaluated in double-double arithmetic (about 106
 * significant bits) over the same double coefficient tables as dgtn_apply, and
 * r rounded to double once: the extended-precision residual of iterative
 * refinement in three precisions (Sec. 2.3, eq. matrix_eqn).  It tells rounding
 * in the evaluation of A u apart from the rounding of u itself: where the two
 * residuals agree, a solve that stagnates has reached the attainable accuracy
 * of a double u (eps |A| |u|, large on thin layers through the interior-penalty
 * terms of eq. penalty).  dgtn_solve uses it for its true residual when
 * opts->residual_precision is 128.  b, u, r: device double, n_dof values; r
 * must not alias u. */
dgtn_status dgtn_residual(dgtn_ctx* ctx, const double* b, const double* u, double* r, hipStream_t stream);

/* z = M^{-1} v: one application of the solver's preconditioner (the V-cycle
 * of dgtn_solve with the same options, in opts->precond_precision), for the
 * operator scaled by 1 / y_ref.  v, z: device double arrays of n_dof values,
 * not aliased.  The workspace must have been bound with the same options.
 * Here and in dgtn_solve the V-cycle is recorded once (per precision and
 * smoother setting) as a HIP graph on a stream the library owns and replayed
 * on `stream`; with the environment variable DGTN_NO_GRAPHS set when the
 * solver state is created, or if recording fails, it is launched kernel by
 * kernel instead (same kernels, same results).  In FP32 the V-cycle's input is
 * v times a power of two chosen from ||v|| (here; from ||b|| in dgtn_solve) and
 * its output is divided by it, so that small vectors keep FP32's normal range;
 * computing ||v|| synchronises the stream. */
dgtn_status dgtn_precondition(dgtn_ctx* ctx, const dgtn_solve_opts* opts, const double* v, double* z,
                              hipStream_t stream);

/* Elastic energy per layer, U_k = 1/2 sum over the elements of layer k of
 * int S_ij Y^ijkl S_kl dV with the unlifted strain S = D_(i u_j) and LGL
 * quadrature (Sec. 2.1: U = -1/2 int S_ij T^ij dV, split into the substrate
 * and coating parts), and optionally the compliance form of the same energy,
 * U_compl = 1/2 u . b with b the load vector of dgtn_rhs (the work of the
 * applied pressure; for the solution of A u = b the two agree up to the
 * discretisation error).  u: device double, n_dof values in the field layout;
 * U_layers: host, n_layers values (J); U_compl: host, one value (J), or NULL
 * to skip it.  Per-layer sums are taken on the device in a fixed order
 * (deterministic).  Synchronises the stream; DGTN_ENAN if a result is not
 * finite. */
dgtn_status dgtn_energy(dgtn_ctx* ctx, const double* u, double* U_layers, double* U_compl,
                        hipStream_t stream);

/* dgtn_energy for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels, the same results bit for bit, but the per-element and
 * per-layer partial sums live in a fixed device array of the library
 * (2.03 MiB per device, held until the process ends) instead of the bound
 * workspace.  Calls no hipMalloc / hipFree and no allocating library routine.
 * Maximum: 131072 elements and 4096 layers (DGTN_EINVAL beyond, before any
 * device work).  The workspace must still be bound (it holds the geometry) and
 * the device it was bound on must be current.  Every call on one device
 * shares that array, so calls that overlap on one device (other streams,
 * other threads, other contexts) race and must be serialised by the caller.
 * Arguments, outputs and errors as in dgtn_energy; synchronises the stream. */
dgtn_status dgtn_energy_noalloc(dgtn_ctx* ctx, const double* u, double* U_layers, double* U_compl,
                                hipStream_t stream);

/* Cubic constants of a material in Pa, out[0..2] = (c11, c12, c44): a cubic
 * material's own (eq. constrel_cryst), or those of an isotropic one from its
 * Young's modulus Y and Poisson ratio nu (eq. constrel_iso):
 * lambda = Y nu / ((1 + nu)(1 - 2 nu)), mu = Y / (2 (1 + nu)),
 * c11 = lambda + 2 mu, c12 = lambda, c44 = mu.  Pure host function;
 * DGTN_EINVAL for a material that dgtn_create would reject. */
dgtn_status dgtn_material_constants(const dgtn_material* material, double* out);

/* Parameters of the energy gradient (the derivative of the layer energies of
 * Sec. 2.1 with respect to the materials of eqs. constrel_iso / constrel_cryst
 * and the layer thicknesses: the quantity the design exploration proposed in
 * Sec. 4 needs).  DGTN_PARAM_C11/C12/C44: a cubic
 * constant of material `index` (any material: an isotropic one has
 * c11 = lambda + 2 mu, c12 = lambda, c44 = mu); DGTN_PARAM_YOUNGS / POISSON:
 * Young's modulus / Poisson ratio of isotropic material `index`;
 * DGTN_PARAM_THICKNESS: thickness of layer `index` (all its element
 * thicknesses scale with it, the layers below translate);
 * DGTN_PARAM_BEAM_WIDTH / BEAM_X / BEAM_Y: the width r0 and the centre xc, yc
 * of the Gaussian pressure of eq. laserbeam, the beam shape and position a
 * search over mirror configurations (Sec. 4) varies (`index` unused). */
enum { DGTN_PARAM_C11 = 0, DGTN_PARAM_C12 = 1, DGTN_PARAM_C44 = 2, DGTN_PARAM_YOUNGS = 3,
       DGTN_PARAM_POISSON = 4, DGTN_PARAM_THICKNESS = 5, DGTN_PARAM_BEAM_WIDTH = 6,
       DGTN_PARAM_BEAM_X = 7, DGTN_PARAM_BEAM_Y = 8 };
typedef struct {
    int kind;
    int index;
} dgtn_param;

/* g = dJ/du for J = sum_k w_k U_k (U_k the layer energies of dgtn_energy):
 * the layer-weighted energy form applied to u, which is the right-hand side of
 * the adjoint system A lambda = g.  w_layers: host, n_layers weights, or NULL
 * for all ones.  u, g: device double, n_dof values, not aliased. */
dgtn_status dgtn_energy_grad(dgtn_ctx* ctx, const double* u, const double* w_layers, double* g,
                             hipStream_t stream);

/* Adjoint gradient of J = sum_k w_k U_k with respect to n_params parameters:
 *   dJ/dtheta = 1/2 u^T K_w,theta u - lambda^T A_theta u + lambda^T b_theta,
 * u the solution of A u = b and lambda that of A lambda = dJ/du (A is
 * symmetric).  Material and thickness parameters leave b unchanged and beam
 * parameters leave A and K unchanged.  A_theta u and K_w,theta are evaluated
 * exactly by the operator and energy kernels on dual numbers, b_theta by the
 * load kernel with the derivative of the pressure profile.  u, lam: device
 * double; dJ: host, n_params values.  DGTN_EINVAL for an unknown kind or
 * index.  Synchronises the stream. */
dgtn_status dgtn_grad(dgtn_ctx* ctx, const double* u, const double* lam, const double* w_layers,
                      int n_params, const dgtn_param* params, double* dJ, hipStream_t stream);

/* The layer energies split by elastic modulus, the decomposition Sec. 2.1
 * notes for materials whose independent moduli carry their own loss angles:
 * parts[3 k + q] for layer k is, for an isotropic layer (eq. constrel_iso),
 * q = 0 the bulk part 1/2 int K (tr S)^2 with K = lambda + 2 mu / 3, q = 1 the
 * shear part (the rest), q = 2 zero; for a cubic layer (eq. constrel_cryst)
 * the parts carried by c11, c12 and c44.  The parts of a layer sum to its
 * energy of dgtn_energy.  u: device double, n_dof; parts: host, 3 n_layers (J).
 * Synchronises the stream. */
dgtn_status dgtn_energy_parts(dgtn_ctx* ctx, const double* u, double* parts, hipStream_t stream);

/* Face-jump indicator for adaptive refinement (the jump [u] is what the interior
 * penalty of Sec. 2.2.4, eq. penalty, acts on; Sec. 4 names adaptive mesh
 * refinement as the next step).  Per element e, with the face quadrature of the
 * operator (LGL weights times the surface Jacobian):
 *   eta_e^2 = sum over interior faces  1/2 int |u_e - u_neighbour|^2 dS
 *           + sum over Dirichlet faces     int |u_e|^2 dS   (homogeneous data),
 * nothing on Neumann faces, so the element values sum to the jump integral
 * over all faces.  faces selects the face families summed: DGTN_FACES_SIDE (the
 * four faces across the disk, logical xi and eta), DGTN_FACES_Z (the two faces
 * across the layers, logical zeta: the jumps that refinement in z reduces) or
 * DGTN_FACES_ALL, optionally or-ed with DGTN_FACES_PENALTY, which weights each
 * face node's term by the penalty of eq. penalty at that node,
 * sigma = C (p + 1)^2 / min(h_int, h_ext) (own h on Dirichlet faces): the jump
 * part of the DG energy norm, in which a thin layer's jumps count in proportion
 * to the penalty that acts on them.  Other values give DGTN_EINVAL.  u: device double, n_dof.
 * eta_elem: host, n_elem, element
 * order of u (may be null); eta_layers: host, n_layers, the per-layer sums in
 * fixed order (may be null; not both).  Lengths in the problem's units.
 * Synchronises the stream; DGTN_ENAN if a value is not finite. */
enum { DGTN_FACES_SIDE = 1, DGTN_FACES_Z = 2, DGTN_FACES_ALL = 3, DGTN_FACES_PENALTY = 4 };
dgtn_status dgtn_jump_indicator(dgtn_ctx* ctx, const double* u, int faces, double* eta_elem, double* eta_layers,
                                hipStream_t stream);

/* S_x = 4 kB T sum_{k,q} phi[3 k + q] parts[3 k + q] / (pi f F0^2): the noise
 * with one loss angle per energy part of dgtn_energy_parts.  Pure host
 * function; DGTN_EINVAL for n_layers < 1, T <= 0, f <= 0 or F0 = 0. */
dgtn_status dgtn_noise_psd_parts(const double* parts, const double* phi, int n_layers, double T, double f,
                                 double F0, double* S_x);

/* Thermal-noise power spectral density from the layer energies:
 * S_x = 4 kB T sum_k phi_k U_k / (pi f F0^2), the reading of eqs.
 * thermalnoise / wdiss in which the dissipated power is 2 pi f U phi.  Pure
 * host function. */
dgtn_status dgtn_noise_psd(const double* U_layers, const double* phi, int n_layers,
                           double T, double f, double F0, double* S_x);

/* Introspection of the multigrid hierarchy built for `opts` (host only, no
 * workspace needed).  dgtn_level_info returns, for level l (0 = finest), its
 * LGL point count N, element count and column count, or DGTN_EINVAL past the
 * coarsest level.  dgtn_smoother_block copies the additive-Schwarz subdomain
 * data of element e on level l: for component c and reference direction d
 * (index 3c + d), N*N entries S[node][mode] (the M-orthonormal eigenvectors of
 * the 1D element operator) followed by N eigenvalues scaled by the modulus,
 * 9 (N*N + N) doubles in all. */
dgtn_status dgtn_level_info(dgtn_ctx* ctx, const dgtn_solve_opts* opts, int level, int* N,
                            int* n_elem, int* n_cols);
dgtn_status dgtn_smoother_block(dgtn_ctx* ctx, const dgtn_solve_opts* opts, int level, int elem,
                                double* out);

/* Overlapping column patches of level l (host only): *P = N + 2k (N without
 * overlap) and, if table is non-NULL, n_cols * P * P ints: for column c and
 * patch position (a, b) (a along the column's xi, b along eta, own nodes at
 * k..k+N-1), the node c' * N^2 + j' * N + i' of the 2D column grid it reads,
 * or -1 (outside the domain, or the corner at a vertex not shared by four
 * columns). */
dgtn_status dgtn_patch_table(dgtn_ctx* ctx, const dgtn_solve_opts* opts, int level, int* P, int* table);

/* Node coordinates (host, double, [E][3][N^3]) of the library's mesh. */
dgtn_status dgtn_node_coords(const dgtn_ctx* ctx, double* xyz);

void dgtn_destroy(dgtn_ctx* ctx);

const char* dgtn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DGTN_H */
