// Kernel launchers (pmg_kernels.hip) used by the C ABI layer.
#pragma once

#include "pmg_internal.h"

namespace pmg {

constexpr int REDUCE_BLOCKS = 512;   // workgroups of the reduction kernels (two per CU)
constexpr int REDUCE_THREADS = 1024;

hipError_t init_kernel_attributes();
// Coarse CG (launch-per-iteration form): the init kernel, then iteration
// launches with ring index j = 0, 1, ..., COARSE_RING - 1, 0, ...
constexpr int COARSE_RING = 6;
// length of the restriction work buffer (coarse partial sums + row pass)
int64_t restrict_work_len(const Layout& Lf, const Layout& Lc);
constexpr int COARSE_GRAPH_MAXN = 256;  // longest captured chain of coarse iteration launches
hipError_t launch_coarse_init(const CoarseArgs& a, const double* b, int maxit, double rtol, hipStream_t st);
// exact solve of the level's condensed system by fast diagonalization: x = Hhat^-1 b
void launch_fd_solve(const Layout& L, const FdTabs& fd, double lam, const double* b, double* x, hipStream_t st);
// copy of a node grid with each periodic direction's last layer set to its first
void launch_grid_seam_copy(const Layout& L, const double* f, double* out, hipStream_t st);
void launch_publish(const double* sc, int n, int64_t* cnt, HostMail* mail, hipStream_t st);
void launch_pcg_start(const double* F, double* r, double* s, double* u, double* p, double* delta, int64_t n,
                      hipStream_t st);
hipError_t launch_coarse_iter(const CoarseArgs& a, int j, bool last, hipStream_t st);
// x of the finished coarse CG into the plane-layout array x
hipError_t launch_coarse_extract(const CoarseArgs& a, double* x, hipStream_t st);
int coarse_blocks(int ne, int p0);

template <typename T> void launch_grid_to_skel(const Layout&, const double*, T*, hipStream_t);
template <typename T> void launch_skel_to_grid(const Layout&, const T*, double*, hipStream_t);
// y = H_hat u, or y = F - H_hat u (the residual) when F is given
template <typename T> void launch_condensed_op(const LevelTabs<T>&, const T*, T*, hipStream_t, const T* F = nullptr);
template <typename T> void launch_smoother_add(const LevelTabs<T>&, const T*, T*, T, hipStream_t);
// element-centred block smoother (Sec. 3.4), p >= 2, tables set up
template <typename T> void launch_block_smoother_add(const LevelTabs<T>&, const T*, T*, T, hipStream_t);
// The coarse-side array (uc, rc) may be of a wider type TC than the level's T.
template <typename T, typename TC>
void launch_prolong_add(const Layout& Lc, const Layout& Lf, const T* J, const TC* uc, T* uf, hipStream_t);
template <typename T, typename TC>
void launch_restrict(const Layout& Lf, const Layout& Lc, const T* J, const T* rf, TC* rc, T* tbuf, hipStream_t);
template <typename T>
void launch_dot2(const T* x, const T* y, const T* z, int64_t n, double* partials, unsigned* counter,
                 double* out, hipStream_t);
template <typename T> void launch_sub_from(const T* x, T* y, int64_t n, hipStream_t);
template <typename T> void launch_axpy(T a, const T* x, T* y, int64_t n, hipStream_t);
template <typename T, typename U>
void launch_cast_scale(const T* x, U* y, const double* sc, int invert, int64_t n, hipStream_t);
template <typename T, typename TC>
void launch_hprolong_add(const Layout& Lc, const Layout& Lf, const T* const* t, const TC* uc, T* uf, hipStream_t);
template <typename T, typename TC>
void launch_hrestrict(const Layout& Lf, const Layout& Lc, const T* const* t, const T* rf, TC* rc, hipStream_t);
template <typename T>
void launch_point_smooth(const Layout& L, const T* dg, const T* r, T* u, T omega, hipStream_t);
template <typename T> size_t smem_condensed_op(int p);
template <typename T> size_t smem_smoother(int p);

void launch_condense(const LevelTabs<double>& tb, const double* m1, const double* m2, const double* m3,
                     const double* f, double* Fh, hipStream_t);
void launch_recover(const LevelTabs<double>& tb, const double* f, const double* uh, double* ug, hipStream_t);
// out = f - M^-1 H G on inner grid nodes, 0 on the boundary (G = g on the
// boundary, 0 inside); tab: [3][2][p + 1] 1D end couplings over the mass
void launch_lift_dirichlet(const int N[3], int p, const double* tab, const double* f, const double* g,
                           double* out, hipStream_t);
void launch_set_boundary(const int N[3], const double* g, double* u, hipStream_t);
void launch_pcg_dir(double* p, const double* z, const double* sc, int64_t n, hipStream_t);
void launch_pcg_update(double* u, double* r, double* s, const double* p, const double* q, const double* gam,
                       const double* qp, int64_t n, double* partials, unsigned* counter, double* out,
                       double* delta_out, hipStream_t st, float* r32 = nullptr, double* sc_zs = nullptr,
                       float* z32 = nullptr);
// FP32 preconditioner: r32 = r / sqrt(r.r) and the scale; gamma, gamma0 and
// the direction update from the FP32 result scaled back on the fly.  With
// z32 the update and the cast also clear the FP32 cycle's correction, which
// the next cycle then accumulates into without a fill of its own.
void launch_cast_down(const double* r, float* r32, const double* sc_rr, double* sc_zs, int64_t n, hipStream_t st,
                      float* z32 = nullptr);
void launch_dot_zmix(const float* z32, const double* sc_zs, const double* r, const double* s, int64_t n,
                     double* partials, unsigned* counter, double* out, hipStream_t st);
void launch_pcg_dir_mixed(double* p, const float* z32, const double* sc_zs, const double* sc, int64_t n,
                          hipStream_t st);
template <typename T> void launch_fill_zero(T* x, int64_t n, hipStream_t st);
void launch_jacobi(const double* r, const double* dg, double* z, int64_t n, double* partials,
                   unsigned* counter, double* out, hipStream_t);
void launch_cg_xr(double* x, double* r, const double* p, const double* q, const double* sc, int64_t n,
                  hipStream_t);
void launch_cg_p(double* p, const double* z, const double* rz_new, const double* rz_old, int64_t n,
                 hipStream_t);
void launch_mlp_forward(const float* prm, const float* x, float* y, float* cache, int batch, int nout,
                        hipStream_t);
void launch_mlp_loss(const float* y, const float* t, const float* m, float* dy, float* loss, int n,
                     hipStream_t);
void launch_mlp_backward(const float* prm, const float* x, const float* cache, const float* dy, float* work,
                         float* g, int batch, int nout, hipStream_t);
void launch_mlp_adam(float* prm, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                     float eps, int t, hipStream_t);

}  // namespace pmg
