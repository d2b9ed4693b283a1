// Internal declarations shared by the host set-up, the kernels and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

namespace pmg {

// ---------------------------------------------------------------------------
// Plane layout of a condensed (skeleton) vector on one level.
//
// Family d holds the planes normal to x_d at the element boundaries
// i_d = j p, j = 0..n_d.  A family-0 plane is a row-major array [i3][i2], a
// family-1 plane [i3][i1], a family-2 plane [i2][i1], rows padded to `pitch`.
// Every condensed unknown is stored once: nodes with i1 % p == 0 live in
// family 0, else nodes with i2 % p == 0 in family 1, else family 2.  All
// other slots and the Dirichlet nodes are kept at zero.
//
// Boundary kinds (Sec. 3.3), per direction and side: homogeneous Dirichlet,
// homogeneous Neumann (the boundary nodes are unknowns) or periodic.  In a
// periodic direction the node layer i_d = N_d - 1 is the layer i_d = 0
// again; its slots (the mirror slots) carry no unknown and are zero between
// operations, so that sums over a vector count every unknown once.  The
// element kernels see the mesh unfolded: before them the mirror slots of
// their input receive a copy of the slots they repeat, after them the
// mirror slots of an accumulated output are added onto those slots.
// ---------------------------------------------------------------------------
constexpr int BC_ALL_DIRICHLET = 0x3f;

struct Layout {
    int p;
    int n[3];
    int N[3];            // n_d p + 1
    int pitch[3];        // row pitch of family-d planes
    int rows[3];         // rows per family-d plane
    int64_t pstride[3];  // elements per family-d plane
    int64_t off[3];      // start of family d
    int64_t len;         // total length
    // bit d: Dirichlet at the low end of direction d; bit 3 + d: Dirichlet at
    // its high end; bit 6 + d: direction d periodic (Neumann where no bit)
    int bc;

    __host__ __device__ inline bool dlo(int d) const { return (bc >> d) & 1; }
    __host__ __device__ inline bool dhi(int d) const { return (bc >> (3 + d)) & 1; }
    __host__ __device__ inline bool per(int d) const { return (bc >> (6 + d)) & 1; }
    __host__ __device__ inline bool any_per() const { return (bc >> 6) & 7; }

    // Storage slot of the skeleton node (i1, i2, i3); the caller guarantees
    // that it is a skeleton node and states which of i_d are multiples of p.
    __host__ __device__ inline int64_t slot(int i1, int i2, int i3, bool on1,
                                            bool on2) const {
        if (on1) return off[0] + (int64_t)(i1 / p) * pstride[0] + (int64_t)i3 * pitch[0] + i2;
        if (on2) return off[1] + (int64_t)(i2 / p) * pstride[1] + (int64_t)i3 * pitch[1] + i1;
        return off[2] + (int64_t)(i3 / p) * pstride[2] + (int64_t)i2 * pitch[2] + i1;
    }
    __host__ __device__ inline int64_t plane0(int j) const { return off[0] + (int64_t)j * pstride[0]; }
    __host__ __device__ inline int64_t plane1(int j) const { return off[1] + (int64_t)j * pstride[1]; }
    __host__ __device__ inline int64_t plane2(int j) const { return off[2] + (int64_t)j * pstride[2]; }
};

Layout make_layout(int n1, int n2, int n3, int p, int bc = BC_ALL_DIRICHLET);

// Device tables of one level, element type T.  Per-direction tables are
// indexed by element index (el_*) or vertex index (st_*).
template <typename T>
struct LevelTabs {
    Layout lay;
    T lam;
    // element tables, direction d, element e: offsets e * size
    const T* el_m[3];     // (p+1)        diagonal mass
    const T* el_L[3];     // (p+1)^2      stiffness, row-major
    const T* el_Sinv[3];  // (p-1)^2      S^-1 = S^T M_I,  [k][i]
    const T* el_MS[3];    // (p-1)^2      M_I S,           [i][k]
    const T* el_lam[3];   // (p-1)        interior eigenvalues
    const T* el_c0[3];    // (p-1)        S^T L[I,0]
    const T* el_cp[3];    // (p-1)        S^T L[I,p]
    // the seven tables above packed per element, in that order (m, L, Sinv,
    // MS, lam, c0, cp): one contiguous block of elem_table_size(p) / 3
    // entries per direction and element
    const T* el_pack[3];
    // per direction and element the interior eigenvector matrices in the
    // orientations the condensation and recovery apply: S^T = Sinv M_I^-1
    // ([k][i] = Sinv[k][i] / m_{i+1}), then S = (M_I S) M_I^-1 ([i][k] =
    // MS[i][k] / m_{i+1}); 2 (p-1)^2 entries per element
    const T* el_st[3];
    // star tables, direction d, vertex v: offsets v * size
    const T* st_S[3];     // nS^2         [i][k], identity padded
    const T* st_lam[3];   // nS           padded eigenvalues = 1
    const T* st_w;        // nS           1D weights
    // the same star tables padded to np x np, np = 16 ceil(nS / 16) (zeros;
    // eigenvalue 1; weight 0) for the matrix-core smoothers
    const T* st_SP[3];   // np^2 per vertex
    const T* st_lamP[3]; // np per vertex
    const T* st_wP;      // np
    int np;
    // interpolation from the next coarser level: (p+1) x (pc+1), row-major
    const T* J;
    int pc;
    // p <= 2: assembled 1D matrices per direction, one record of AXW entries
    // per global node index i: [M~(i,i), L~(i,i-p) .. L~(i,i+p), 0...]
    const T* ax[3];
    // p = 2: per element, (H_IB u)_e / (H_II)_e of the condensed operator
    T* tc;
    // workspace of the condensed operator: per element, the six face tiles
    // of its contribution, [e][6][(p+1)^2] (only canonical entries used)
    T* opE;
    // per-workgroup scratch in device memory for the general kernels when
    // their working set exceeds the LDS of a CU (large p); null otherwise
    T* gws;
    // two [star][3][np][np] workspaces of the batched star smoother (nS > 16)
    T* sbX[2];
    // batched condensation / recovery (finest level, p >= 9): two
    // [element][qp^3] arrays, qp = 16 ceil((p-1) / 16)
    double* ixX[2];
    int qp;
    // element-centred block smoother (Sec. 3.4), set up on request: per
    // direction d and element index e, the block's 1D eigenvectors [i][k]
    // (bnp x bnp, identity padded), eigenvalues (bnp, padding 1) and weights
    // (bnp, padding 0), bnp = 16 ceil((3p - 1) / 16); two
    // [element][6][bnp][bnp] workspaces
    const T* bl_S[3];
    const T* bl_lam[3];
    const T* bl_w[3];
    int bnp;
    T* bwX[2];
};

// Working-set sizes (elements of T) of the general per-element / per-star
// kernels: held in LDS when they fit, else in the level's device scratch.
__host__ __device__ inline int elem_table_size(int p) {
    const int n1 = p + 1, q = p - 1;
    return 3 * (n1 + n1 * n1 + 2 * q * q + 3 * q);
}
__host__ __device__ inline size_t ws_condensed_op(int p) {
    const size_t n1 = p + 1, q = p - 1;
    return 6 * n1 * n1 + 18 * q * q + (size_t)elem_table_size(p);
}
// in device scratch the q^3 eigenspace array V is formed once as well
__host__ __device__ inline size_t ws_condensed_op_v(int p) {
    const size_t q = p - 1;
    return ws_condensed_op(p) + q * q * q;
}
__host__ __device__ inline size_t ws_smoother(int p) {
    const size_t nS = 2 * p - 1;
    return 9 * nS * nS;
}
__host__ __device__ inline size_t ws_condense(int p) {
    const size_t q = p - 1;
    return 2 * q * q * q + 18 * q * q;
}
__host__ __device__ inline size_t ws_recover(int p) {
    const size_t n1 = p + 1, q = p - 1;
    return 6 * n1 * n1 + 2 * q * q * q + 12 * q * q;
}
constexpr size_t kLdsBytes = 160 * 1024;  // LDS per CU on gfx950

// Exact solve of a level's condensed system by fast diagonalization of the
// whole mesh (the full system with zero interior right-hand side): per
// direction m_d unknown node indices starting at o_d (n_d p - 1 from 1
// between two Dirichlet ends; a Neumann end adds its node, a periodic
// direction has n_d p from 0), the forward (S^T) and backward (S) transform
// matrices, row-major, and the eigenvalues; two [m3][m2][m1] work arrays.
struct FdTabs {
    int m[3];
    int o[3];
    const double* Af[3];
    const double* Ab[3];
    const double* mu[3];
    double* X;
    double* Y;
};

struct HostTables {
    // per direction: concatenated element / star tables (FP64)
    std::vector<double> el_m[3], el_L[3], el_Sinv[3], el_MS[3], el_lam[3],
        el_c0[3], el_cp[3], st_S[3], st_lam[3];
    std::vector<double> st_w, J;
    std::vector<double> st_SP[3], st_lamP[3], st_wP;
    std::vector<double> ax[3];  // p <= 2 only
    int np = 16;
};
constexpr int AXW = 8;  // entries per record of the assembled 1D tables

// Host set-up (pmg_setup.cpp)
void gll_nodes_weights(int p, std::vector<double>& x, std::vector<double>& w);
void stiffness_std(int p, const std::vector<double>& x, const std::vector<double>& w,
                   std::vector<double>& L);
void sym_eig_jacobi(int n, std::vector<double>& A, std::vector<double>& Q,
                    std::vector<double>& lam);
void gen_eig_diag(int n, const double* L, const double* m, std::vector<double>& S,
                  std::vector<double>& lam);
void lagrange_interp(const std::vector<double>& xf, const std::vector<double>& xt,
                     std::vector<double>& J);
double smoothstep(int pw, double t);
void build_level_tables(int p, int pc, const std::vector<double> h[3], HostTables& t,
                        int bc = BC_ALL_DIRICHLET);
// bc_d: bit 0 Dirichlet low end, bit 1 Dirichlet high end, bit 2 periodic
void build_fd_tables(int p, const std::vector<double>& h, int bc_d, std::vector<double>& Af,
                     std::vector<double>& Ab, std::vector<double>& mu, int& first);
void build_block_tables(int p, const std::vector<double>& h, int np, int bc_d, std::vector<double>& S,
                        std::vector<double>& lam, std::vector<double>& w);
void coarse_diagonal(const Layout& lay, double lam, const std::vector<double> h[3],
                     std::vector<double>& diag);

}  // namespace pmg

namespace pmg {

// Coarse-level (p_0 <= 2) problem for the Jacobi-CG iteration kernels; the
// vectors live in the level's plane layout, so an element finds its nodes'
// slots by arithmetic.
//
// Scalars of the coarse CG carried from one iteration launch to the next
// (written by block 0 of each launch into the other ring slot).
struct CoarseState {
    double gamma, alpha, gamma0, rtol2;
    int64_t id;      // coarse solve number (reported to the host when done)
    int it;          // completed updates; -1 before the first launch
    int done;
    int maxit;
    int pad;
};

// Mapped, coherent host memory the device writes completion notices to, so
// the host can wait by polling instead of a stream synchronisation.
struct HostMail {
    volatile int64_t seq;    // number of scalar publications so far
    volatile int64_t cseq;   // id of the last coarse solve that finished
    volatile int64_t rseq;   // (id << 20) | updates: a coarse solve whose queued launches ran out
    volatile int cit;        // update count of that coarse solve
    int pad;
    double sc[16];           // the published scalars
};

struct CoarseArgs {
    Layout lay;           // level-0 plane layout: all vectors below have lay.len entries
    int N0;               // unknowns
    int ne;               // elements
    int n[3];
    int p0;               // 1 or 2
    double lam;
    const double* diag;   // diagonal of the operator at unknowns, 0 at every other slot
    const double* el_m[3];  // level-0 element tables
    const double* el_L[3];
    double* X;            // level-0 skeleton array that receives the solution x
    // per slot one 64-byte record, so that a node's CG state is one cache
    // line: [diag, -, r0, q0, r1, q1, p, x] (r and q = A p ping-pong)
    double* rec;
    double *W[3];         // rotating accumulators of w = A z
    double *P[2];         // [2 * blocks] per-block partial sums (r.z, w.z)
    CoarseState* S;       // [2] scalar state, ping-pong
    int* stat;            // [2]: done flag and update count of the last solve
    int* iters;           // accumulated iteration count
    int blocks;           // workgroups of one iteration launch
    HostMail* mail;       // device address of the host notice block (or null)
    int64_t* seq;         // number of coarse solves started (device counter)
};

}  // namespace pmg
