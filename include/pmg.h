/*
 * pmg.h -- C ABI of the MI355X p-multigrid solver for the statically
 * condensed spectral-element Helmholtz problem
 *
 *        lambda u - Laplace(u) = f   on a box,  u = 0 on the boundary,
 *
 * (inhomogeneous boundary values u = g by lifting: pmg_pcg_solve_dirichlet;
 * homogeneous Neumann and periodic sides: pmg_create_mesh_bc),
 *
 * after Huismann, Stiller & Froehlich, "Scaling to the stars -- a linearly
 * scaling elliptic solver for p-multigrid" (arXiv 1808.03595).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Return value: 0 on success; negative on error (PMG_EINVAL -1 invalid
 *    argument, PMG_EHIP -2 HIP runtime error, PMG_ENOMEM -3 device memory,
 *    PMG_EUNSUP -4 unsupported size); positive values are solver states
 *    (PMG_NOT_CONVERGED 1, PMG_BREAKDOWN 2).  pmg_last_error() returns a
 *    thread-local message for the last failing call.
 *  - Pointers named d_* are DEVICE pointers owned by the caller and only
 *    borrowed for the call.  Pointers named h_* are host pointers.
 *  - "stream" is a hipStream_t passed as void*; NULL is the default stream.
 *    All calls are stream-ordered and asynchronous unless stated otherwise.
 *  - A mesh handle is not thread-safe; use it from one stream at a time.
 *  - Node grids ("grid" arrays) are the global GLL node grids of the finest
 *    level, shape (N3, N2, N1) with N_d = n_d p + 1, x1 fastest, FP64.
 *  - Condensed vectors ("skeleton" arrays) hold the element-boundary
 *    unknowns of one multigrid level in the library's plane layout: for each
 *    direction d the planes normal to x_d at the element boundaries, each a
 *    2D row-major array over the two other global node indices.  Every
 *    unknown is stored exactly once (edges and vertices in the first plane
 *    family that contains them); all other slots, and Dirichlet nodes, hold
 *    0.  Hence plain sums over a skeleton array are sums over the unknowns.
 *    On a mesh with a periodic direction d (pmg_create_mesh_bc) the node
 *    layer i_d = N_d - 1 repeats the layer i_d = 0: its skeleton slots carry
 *    no unknown and are 0 between calls (calls that read element data fill
 *    them for their duration and clear them again, also in inputs), and in
 *    grid arrays that layer is written as a copy of the first and ignored on
 *    input.
 *    Its length is pmg_skeleton_len(); the element type is FP64 (dtype
 *    PMG_F64) or FP32 (PMG_F32) as the call states.
 */
#ifndef PMG_H
#define PMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pmg_mesh pmg_mesh;

enum { PMG_F64 = 0, PMG_F32 = 1 };
enum { PMG_OK = 0, PMG_EINVAL = -1, PMG_EHIP = -2, PMG_ENOMEM = -3,
       PMG_EUNSUP = -4, PMG_NOT_CONVERGED = 1, PMG_BREAKDOWN = 2 };
enum { PMG_MAX_DEGREE = 48, PMG_MAX_HIST = 512, PMG_MAX_COARSE_IT = 1000000 };
enum { PMG_BC_DIRICHLET = 0, PMG_BC_NEUMANN = 1, PMG_BC_PERIODIC = 2 };

typedef struct {
    int iters;                    /* outer iterations performed            */
    int status;                   /* 0, PMG_NOT_CONVERGED or PMG_BREAKDOWN */
    double res0;                  /* |r_0|_2 over the condensed unknowns   */
    double rel_res;               /* |r_k|_2 / |r_0|_2 (recursive residual) */
    double res_hist[PMG_MAX_HIST];/* |r_k|_2, k = 0..iters                 */
    int coarse_iters;             /* coarse CG iterations, summed          */
    double t_pre_ms, t_iter_ms, t_post_ms; /* stream-event timings         */
} pmg_stats;

/* Mesh of n1 x n2 x n3 cuboid elements on the unit cube, degree p, Helmholtz
 * parameter lambda >= 0.  stretch = alpha >= 1 grades the element widths
 * geometrically in every direction, h_{k+1} = alpha h_k (the stretched
 * meshes of Sec. 5.4); alpha = 1 is uniform.  Builds the p-multigrid levels
 * p_l = 2^(l+1) (l < L), p_L = p (Sec. 4.1) and all device tables.
 * 1 <= p <= PMG_MAX_DEGREE, n_d >= 1.  *out receives the handle. */
int pmg_create_mesh(int n1, int n2, int n3, int p, double lambda,
                    double stretch, pmg_mesh **out);

/* As pmg_create_mesh with explicit element widths (host arrays of n1, n2,
 * n3 positive values), e.g. the anisotropic brick meshes of Sec. 5.3. */
int pmg_create_mesh_widths(int n1, int n2, int n3, int p, double lambda,
                           const double *h_hx, const double *h_hy,
                           const double *h_hz, pmg_mesh **out);

/* As pmg_create_mesh_widths with a boundary kind per side (Sec. 3.3):
 * h_bc[6] = (x1 low, x1 high, x2 low, x2 high, x3 low, x3 high), each
 * PMG_BC_DIRICHLET (homogeneous, u = 0), PMG_BC_NEUMANN (homogeneous, zero
 * normal derivative: the boundary nodes are unknowns, a flux enters through
 * the right-hand side) or PMG_BC_PERIODIC (on both sides of a direction,
 * which then needs n_d >= 3 elements).  The star of a boundary vertex keeps
 * its size: the 1D star matrices are padded with identity where the ghost
 * element lies outside the domain and at a Dirichlet vertex; in a periodic
 * direction the ghost element is the last element.  Without a Dirichlet
 * side lambda must be > 0 (else the operator is singular): PMG_EINVAL.
 * Such a mesh always uses the exact coarse solve; pmg_set_coarse_solver(0),
 * pmg_set_coarse_mg with levels > 0 and the lifting calls
 * (pmg_lift_dirichlet, pmg_set_boundary, pmg_pcg_solve_dirichlet) return
 * PMG_EUNSUP on it unless every side is Dirichlet.  The element-centred
 * blocks (pmg_set_smoother(1)) take the same boundary treatment. */
int pmg_create_mesh_bc(int n1, int n2, int n3, int p, double lambda,
                       const double *h_hx, const double *h_hy,
                       const double *h_hz, const int *h_bc, pmg_mesh **out);

void pmg_destroy_mesh(pmg_mesh *m);

/* Number of coarsenings L (levels 0..L) and the degree of a level. */
int pmg_num_levels(const pmg_mesh *m, int *L);
int pmg_level_degree(const pmg_mesh *m, int level, int *p);

/* Length (elements) of a skeleton array of a level; grid length N1 N2 N3. */
int pmg_skeleton_len(const pmg_mesh *m, int level, int64_t *len);
int pmg_grid_len(const pmg_mesh *m, int64_t *len);

/* Global 1D node coordinates of the finest level (host arrays of N_d). */
int pmg_grid_coords(const pmg_mesh *m, double *h_x1, double *h_x2,
                    double *h_x3);

/* Layout conversion at a level whose degree divides the finest grid is not
 * needed: these act on the finest level only.  grid_to_skeleton copies the
 * free element-boundary nodes of d_grid (FP64) into d_skel (dtype);
 * skeleton_to_grid writes them back and sets all other grid nodes to 0. */
int pmg_grid_to_skeleton(pmg_mesh *m, int dtype, const double *d_grid,
                         void *d_skel, void *stream);
int pmg_skeleton_to_grid(pmg_mesh *m, int dtype, const void *d_skel,
                         double *d_grid, void *stream);

/* y = Hhat_l u: the statically condensed Helmholtz operator of level l,
 * H_BB - H_BI H_II^-1 H_IB assembled over elements (Sec. 2.2), applied
 * matrix-free with O(p^3) work per element.  d_u, d_y: skeleton arrays of
 * the level (dtype); they must not alias. */
int pmg_apply_condensed_op(pmg_mesh *m, int level, int dtype, const void *d_u,
                           void *d_y, void *stream);

/* du = omega * Smoother_l(r): the additive Schwarz star smoother of Alg. 2
 * with the star inverse of Alg. 1 and the degree-7 weight functions of
 * Sec. 3.2; omega = 1 is the paper's method.  d_r, d_du: skeleton arrays of
 * the level (dtype), not aliasing.  d_du is overwritten. */
int pmg_schwarz_smooth(pmg_mesh *m, int level, int dtype, const void *d_r,
                       void *d_du, double omega, void *stream);

/* d_u += omega * Smoother_l(r): the smoothing update of Alg. 3 as the
 * V-cycle applies it (same smoother as pmg_schwarz_smooth, added into d_u
 * instead of overwriting it).  d_r, d_u: skeleton arrays of the level
 * (dtype), not aliasing; d_u must be zero at the slots that hold no unknown
 * (as every array written by this library is). */
int pmg_schwarz_smooth_add(pmg_mesh *m, int level, int dtype, const void *d_r,
                           void *d_u, double omega, void *stream);

/* Grid transfers between level l-1 and l (Sec. 4.1): prolongation
 * d_fine += J_l d_coarse (embedded tensor interpolation restricted to the
 * condensed unknowns) and restriction d_coarse = J_l^T d_fine. */
int pmg_prolong_add(pmg_mesh *m, int level, int dtype, const void *d_coarse,
                    void *d_fine, void *stream);
int pmg_restrict(pmg_mesh *m, int level, int dtype, const void *d_fine,
                 void *d_coarse, void *stream);

/* Cycle parameters: nu_mode 0 = one pre- and one post-smoothing step per
 * level ("kMG"), 1 = 2^(L-l) steps on level l ("kvMG") (Sec. 4.1).  The
 * coarse problem (p_0 = 2) is solved by Jacobi-preconditioned CG to the
 * relative tolerance coarse_rtol (D^-1-weighted residual norm) or
 * coarse_maxit iterations; coarse_rtol = 0 runs exactly coarse_maxit.
 * 0 <= coarse_maxit <= PMG_MAX_COARSE_IT, else PMG_EINVAL. */
int pmg_set_cycle(pmg_mesh *m, int nu_mode, double coarse_rtol,
                  int coarse_maxit);

/* Optional low-order multigrid for the coarse problem (not the paper's
 * coarse solver; the remedy its complexity discussion in Sec. 4.2 names for
 * the O(n_e^(4/3)) coarse cost).  levels = 0 restores the paper's CG at
 * p_0 = 2.  levels >= 1 inserts degree-1 levels below p_0: first on the same
 * mesh, then on meshes with pairs of elements merged in every direction
 * (while all element counts are even and >= 4), at most `levels` of them;
 * each is smoothed `nu` times before and after the coarse correction by
 * the degree-1 star smoother (a point-Jacobi step) damped by `omega`; the
 * Jacobi CG then runs on the smallest mesh.  Synchronizes the device. */
int pmg_set_coarse_mg(pmg_mesh *m, int levels, double omega, int nu);

/* Solver of the coarsest level of the active cycle: kind 0 = the
 * Jacobi-preconditioned CG of pmg_set_cycle (Sec. 4.1; default); kind 1 =
 * an exact solve by fast diagonalization of the whole coarse mesh: on a
 * Cartesian mesh the assembled operator is the tensor sum of eq.
 * helmholtzop, so its inverse is (S3 x S2 x S1) diag(1 / (lambda + mu1 +
 * mu2 + mu3)) (S3 x S2 x S1)^T with the generalized eigenpairs of the
 * assembled 1D matrices (eq. fast_diagonalization on the whole mesh), and
 * the condensed solution is the skeleton part of the full solution with
 * zero interior right-hand side.  Six 1D passes of m_d = n_d p - 1 per
 * direction; no iteration, no tolerance, no host synchronisation (the
 * solvers capture it in their graphs); coarse iteration counts report 0.
 * Tables of 3 m_d^2 values and two work grids of m1 m2 m3 values on the
 * bottom level.  Synchronizes the device. */
int pmg_set_coarse_solver(pmg_mesh *m, int kind);

/* The p-level whose condensed system the exact coarse solve inverts at the
 * bottom of the V-cycle (Alg. 3): 0 (p_0 = 2, the default) up to the finest
 * level; the levels below it are not used.  A higher coarse level trades the
 * V-cycle work of the levels below it for a larger fast-diagonalization solve
 * (6 m^4 operations for m = n p_l per direction, Sec. 4.2's O(n_e^{4/3})
 * term with a larger constant).  Needs the exact coarse solve
 * (pmg_set_coarse_solver(m, 1)) and no degree-1 levels, else PMG_EUNSUP.
 * pmg_coarse_solve then solves that level's system. */
int pmg_set_coarse_level(pmg_mesh *m, int level);

/* Smoother of every level of degree >= 2 (pmg_schwarz_smooth(_add) and the
 * V-cycle): kind 0 = the vertex-centred star smoother of Alg. 2 (default);
 * kind 1 = the element-centred block smoother of Sec. 3.4: one subdomain
 * per element, the 3 x 3 x 3 element block around it (full overlap),
 * condensed to the six faces of the centre element extended over the block
 * (n_S = 3p - 1 nodes per direction), inverted by the six-face form of the
 * star algorithm (2D transforms into the block's 1D eigenbases, expansion,
 * inverse eigenvalue sums, contraction, back transforms; 73 n_S^3
 * operations), with the boundary treatment of Sec. 3.3 (identity padding of
 * ghost elements and Dirichlet vertices).  Block weights: the distance
 * functions q(t)/2, 1/2, q(1-t)/2 on the block's left, centre and right
 * element (q the degree-7 weight polynomial), normalised over the blocks
 * covering a node so that they sum to one.  Degree-1 levels keep their
 * point smoother.  The first switch to kind 1 builds the block tables and
 * two workspaces of n_e * 6 * np^2 FP64 values per level (np =
 * 16 ceil((3p - 1) / 16)); PMG_ENOMEM if they do not fit.  Synchronizes the
 * device. */
int pmg_set_smoother(pmg_mesh *m, int kind);

/* Per-level damping of the smoother correction, u_l += omega_l S_l(r_l).
 * h_omega[j] applies to level L - j (j = 0 is the finest); n <= L values;
 * NULL or n = 0 restores omega = 1 (the paper's method). */
int pmg_set_damping(pmg_mesh *m, const float *h_omega, int n);

/* z = MultigridCycle(0, r) of Alg. 3 on the finest level.  dtype PMG_F64
 * runs the cycle in FP64.  dtype PMG_F32 expects FP32 skeleton arrays and
 * runs the smoother, operator and transfers in FP32 while the coarse solve
 * stays FP64. */
int pmg_vcycle(pmg_mesh *m, int dtype, const void *d_r, void *d_z,
               void *stream);

/* Coarse-level solve Hhat_0 u_0 = F_0 (FP64 skeleton arrays of level 0)
 * with the configured Jacobi-CG; *h_iters (may be NULL) receives the
 * iteration count.  Synchronizes the stream. */
int pmg_coarse_solve(pmg_mesh *m, const double *d_F0, double *d_u0,
                     int *h_iters, void *stream);

/* Static condensation of the right-hand side (Alg. 4, first step):
 * Fhat = F_B - H_BI H_II^-1 F_I with F = M f (GLL-lumped mass).  d_f: grid
 * (FP64); d_Fhat: finest skeleton (FP64). */
int pmg_condense_rhs(pmg_mesh *m, const double *d_f, double *d_Fhat,
                     void *stream);

/* Interior recovery (Alg. 4, last step): u = (uhat, H_II^-1 (F_I - H_IB
 * uhat)) written to the full grid d_u (Dirichlet nodes 0). */
int pmg_recover_interior(pmg_mesh *m, const double *d_f, const double *d_uhat,
                         double *d_u, void *stream);

/* Whole solve of Alg. 5 (Krylov-accelerated MG, inexact preconditioned
 * CG): condense, iterate until |r| <= rtol |r_0| or maxit, recover.
 * precond_dtype PMG_F32 uses the mixed-precision cycle (FP32 V-cycle on
 * r/|r| inside FP64 CG; FP64 residuals, dots and coarse solve); with no
 * smoothed level (p <= 2 and no degree-1 levels) the cycle is the FP64
 * coarse solve alone and runs in FP64 for either value.  d_f, d_u:
 * grids (FP64).  Synchronizes the stream before filling *h_stats (may be
 * NULL).  Returns 0, PMG_NOT_CONVERGED or PMG_BREAKDOWN, or an error. */
int pmg_pcg_solve(pmg_mesh *m, const double *d_f, double *d_u, double rtol,
                  int maxit, int precond_dtype, pmg_stats *h_stats,
                  void *stream);

/* Alg. 4: fixed-point iteration of V-cycles (FP64), same contract as
 * pmg_pcg_solve; used to measure convergence rates. */
int pmg_mg_solve(pmg_mesh *m, const double *d_f, double *d_u, double rtol,
                 int maxit, pmg_stats *h_stats, void *stream);

/* ---- inhomogeneous Dirichlet data (Sec. 3.3, Sec. 5.2) ------------------
 * The paper's boundary treatment keeps Dirichlet values fixed while every
 * correction vanishes there, and its runtime test problem prescribes them
 * on the whole boundary.  They enter by lifting: with G = g on the boundary
 * nodes and 0 inside, u = u0 + G, where u0 vanishes on the boundary and
 * solves the homogeneous problem with f' = f - M^-1 H G (M the diagonal
 * GLL-lumped mass, H the assembled Helmholtz operator of Sec. 2.1).  Only
 * the boundary entries of d_g are read.  All arrays are FP64 grids. */

/* d_out = f - M^-1 H G on the inner grid nodes, 0 on the boundary nodes.
 * d_out may alias d_f but not d_g.  Stream-ordered. */
int pmg_lift_dirichlet(pmg_mesh *m, const double *d_f, const double *d_g,
                       double *d_out, void *stream);

/* d_u = d_g on the boundary nodes; inner nodes untouched.  Stream-ordered. */
int pmg_set_boundary(pmg_mesh *m, const double *d_g, double *d_u, void *stream);

/* pmg_pcg_solve with u = g on the boundary: lifts f into a grid-sized
 * workspace the mesh allocates on the first call (and keeps), solves, and
 * writes the boundary values of g into d_u.  d_u must not alias d_g.  Same
 * return values and synchronization as pmg_pcg_solve. */
int pmg_pcg_solve_dirichlet(pmg_mesh *m, const double *d_f, const double *d_g,
                            double *d_u, double rtol, int maxit,
                            int precond_dtype, pmg_stats *h_stats,
                            void *stream);

/* ---- learned damping: FP32 MLP 3 -> 64 -> 64 -> nout ------------------
 * Parameter vector (nparams = 64*3+64 + 64*64+64 + nout*64+nout floats):
 * W1[64][3], b1[64], W2[64][64], b2[64], W3[nout][64], b3[nout].
 * Forward: h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2),
 * y = 2 sigmoid(W3 h2 + b3).  d_x: [batch][3], d_y: [batch][nout],
 * d_cache: [batch][128 + nout] activations kept for the backward pass. */
int pmg_mlp_nparams(int nout);
int pmg_mlp_forward(const float *d_params, const float *d_x, float *d_y,
                    float *d_cache, int batch, int nout, void *stream);
/* Masked mean-squared error: loss = sum mask (y - t)^2 / sum mask, written
 * to d_loss[0]; d_dy = d loss / d y.  d_mask holds 0/1 per output. */
int pmg_mlp_loss(const float *d_y, const float *d_t, const float *d_mask,
                 float *d_dy, float *d_loss, int batch, int nout,
                 void *stream);
/* Gradient of sum_b dy . y(x_b) with respect to the parameters. */
int pmg_mlp_backward(const float *d_params, const float *d_x,
                     const float *d_cache, const float *d_dy,
                     float *d_grad, int batch, int nout, void *stream);
/* The same gradient as pmg_mlp_backward, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid allocation): no allocation of any kind.  The per-sample
 * deltas live in a fixed array of 2^21 floats (8 MiB) that the library
 * holds on each GPU it runs on until the process ends; batch * (128 + nout)
 * above 2^21 returns PMG_EUNSUP.  Every call on one GPU shares that GPU's
 * array, so calls that overlap on one GPU (other streams, other threads)
 * race and must be serialised by the caller.  The stream must belong to
 * the current device. */
int pmg_mlp_backward_noalloc(const float *d_params, const float *d_x,
                             const float *d_cache, const float *d_dy,
                             float *d_grad, int batch, int nout,
                             void *stream);
/* One Adam step (Kingma & Ba) at step t >= 1 on n parameters. */
int pmg_mlp_adam(float *d_params, const float *d_grad, float *d_m,
                 float *d_v, int n, float lr, float beta1, float beta2,
                 float eps, int t, void *stream);

const char *pmg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PMG_H */
