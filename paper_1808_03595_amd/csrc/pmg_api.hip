// C ABI of the condensed p-multigrid solver: mesh handle, level
// hierarchy, V-cycle (Alg. 3), MG (Alg. 4) and ipCG (Alg. 5) orchestration.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <immintrin.h>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/pmg.h"
#include "pmg_kernels.h"

using namespace pmg;

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                      \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) return fail(PMG_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace {

// scalar slots in device memory
enum { SC_GAMMA = 0, SC_GAMMA0 = 1, SC_DELTA = 2, SC_QP = 3, SC_RR = 4, SC_RZ = 5, SC_PQ = 6, SC_RZN = 7, SC_ZS = 8,
       SC_N = 16 };

struct Level {
    int p = 0, pc = 0;
    Layout lay{};
    std::vector<double> h[3];   // element widths of this level's mesh
    LevelTabs<double> t64{};
    LevelTabs<float> t32{};
    // work vectors of this level
    double *u64 = nullptr, *F64 = nullptr, *y64 = nullptr, *tb64 = nullptr;
    float *u32 = nullptr, *F32 = nullptr, *y32 = nullptr, *tb32 = nullptr;
    // place in the active cycle (set by rebuild_active)
    char kind = 'p';            // transfer from the next coarser active level
    int nu = 1;
    double omega = 1.0;
    const double* Jd64 = nullptr;  // p-transfer matrix from the next coarser level
    const float* Jd32 = nullptr;
    // degree-1 levels: linear h-transfer weights of this (finer) mesh, and the
    // diagonal of the operator for the point smoother
    const double* ht64[3] = {nullptr, nullptr, nullptr};
    const float* ht32[3] = {nullptr, nullptr, nullptr};
    const double* jd64 = nullptr;
    const float* jd32 = nullptr;
    // p_0 = 2 level when degree-1 levels are active: J from degree 1
    const double* Jlow64 = nullptr;
    const float* Jlow32 = nullptr;
    // coarse CG structures when this level is the bottom of the cycle
    CoarseArgs ca{};
    bool has_ca = false;
    // smoothed by the element-centred block smoother (Sec. 3.4) instead of stars
    bool blocks = false;
    // exact coarse solve by fast diagonalization when this level is the bottom
    FdTabs fd{};
    bool has_fd = false;
    // graphs of n iteration launches with ring indices j0 .. j0 + n - 1,
    // [(n - 1) * COARSE_RING + j0 % COARSE_RING], captured on first use
    std::vector<hipGraphExec_t> coarse_exec;
};

template <typename T> struct Sel;
template <> struct Sel<double> {
    static LevelTabs<double>& tabs(Level& l) { return l.t64; }
    static double*& u(Level& l) { return l.u64; }
    static double*& F(Level& l) { return l.F64; }
    static double*& y(Level& l) { return l.y64; }
    static double*& tb(Level& l) { return l.tb64; }
};
template <> struct Sel<float> {
    static LevelTabs<float>& tabs(Level& l) { return l.t32; }
    static float*& u(Level& l) { return l.u32; }
    static float*& F(Level& l) { return l.F32; }
    static float*& y(Level& l) { return l.y32; }
    static float*& tb(Level& l) { return l.tb32; }
};

}  // namespace

struct pmg_mesh {
    int n[3] = {0, 0, 0};
    int p = 0;
    double lam = 0.0;
    std::vector<double> h[3];
    int L = 0;
    std::vector<Level> lv;
    int nu_mode = 0;
    double coarse_rtol = 1e-8;
    int coarse_maxit = 2000;
    std::vector<double> omega;  // per level index l
    // degree-1 levels below p_0 (optional low-order multigrid for the coarse
    // problem) and the active cycle, coarsest first
    std::vector<Level> hlv;
    std::vector<Level*> act;
    int hmg_levels = 0;
    double hmg_omega = 0.6;
    int hmg_nu = 1;
    int smoother_kind = 0;      // 0: star smoother (Alg. 2), 1: element-centred blocks (Sec. 3.4)
    int bc = BC_ALL_DIRICHLET;  // boundary kinds, as Layout::bc
    double* w_fgrid = nullptr;  // periodic meshes: right-hand side grid with its seam layers equal
    int coarse_kind = 0;        // 0: Jacobi CG (Sec. 4.1), 1: exact solve by fast diagonalization
    int coarse_level = 0;       // p-level solved exactly at the bottom of the cycle (levels below unused)
    // coarse CG counters shared by all bottom levels
    int* d_coarse_iters = nullptr;
    // number of coarse solves started, counted on the device by every coarse
    // level's initialisation (one counter per mesh, like coarse_id)
    int64_t* d_coarse_seq = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream for graph capture
    // Alg. 5 iteration graphs per preconditioner precision: [2 pdt + 0] up to
    // the coarse solve, [2 pdt + 1] after it; rebuilt after any change of
    // the cycle
    hipGraphExec_t solver_graphs[4] = {nullptr, nullptr, nullptr, nullptr};
    int coarse_last = 0;
    int coarse_recent[4] = {0, 0, 0, 0};  // update counts of the last coarse solves
    int coarse_nrec = 0;
    long coarse_total = 0;
    // finest-level solver vectors (FP64) and mixed-precision buffers
    double *w_u = nullptr, *w_r = nullptr, *w_s = nullptr, *w_p = nullptr, *w_q = nullptr, *w_z = nullptr,
           *w_F = nullptr;
    float *w_r32 = nullptr, *w_z32 = nullptr;
    double* m1d[3] = {nullptr, nullptr, nullptr};
    double* lift_tab = nullptr;   // [3][2][p + 1] Dirichlet lifting couplings (finest level)
    double* w_lift = nullptr;     // lifted right-hand side on the grid, allocated on first use
    double* partials = nullptr;
    unsigned* counter = nullptr;
    double* scal = nullptr;
    double* hscal = nullptr;  // pinned host copy of the scalars
    // notice block in mapped host memory (host and device addresses), the
    // device-side publication counter and the host-side expectations
    HostMail* hmail = nullptr;
    HostMail* dmail = nullptr;
    int64_t* d_pubcnt = nullptr;
    int64_t pub_expected = 0;
    int64_t coarse_id = 0;    // coarse solves queued (the device numbers them alike)
    int* hcit = nullptr;      // pinned host copy of the coarse iteration counter
    std::vector<void*> allocs;

    template <typename T>
    int alloc(T** ptr, size_t count) {
        void* q = nullptr;
        size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) return fail(PMG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        allocs.push_back(q);
        *ptr = static_cast<T*>(q);
        return 0;
    }
    template <typename T>
    int upload(const T** dst, const std::vector<double>& src) {
        T* d = nullptr;
        int rc = alloc(&d, src.size());
        if (rc) return rc;
        std::vector<T> tmp(src.begin(), src.end());
        if (!tmp.empty()) {
            hipError_t e = hipMemcpy(d, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(PMG_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
        }
        *dst = d;
        return 0;
    }
};

namespace {

std::vector<int> level_degrees(int p) {
    std::vector<int> d;
    if (p <= 2) {
        d.push_back(p);
        return d;
    }
    d.push_back(2);
    while (d.back() * 2 < p) d.push_back(d.back() * 2);
    d.push_back(p);
    return d;
}

template <typename T>
int fill_tabs(pmg_mesh* m, LevelTabs<T>& tb, const HostTables& t, const Layout& lay, int pc) {
    tb.lay = lay;
    tb.lam = (T)m->lam;
    tb.pc = pc;
    tb.np = t.np;
    int rc = 0;
    for (int d = 0; d < 3 && !rc; ++d) {
        if ((rc = m->upload(&tb.el_m[d], t.el_m[d]))) break;
        if ((rc = m->upload(&tb.el_L[d], t.el_L[d]))) break;
        if ((rc = m->upload(&tb.el_Sinv[d], t.el_Sinv[d]))) break;
        if ((rc = m->upload(&tb.el_MS[d], t.el_MS[d]))) break;
        if ((rc = m->upload(&tb.el_lam[d], t.el_lam[d]))) break;
        if ((rc = m->upload(&tb.el_c0[d], t.el_c0[d]))) break;
        if ((rc = m->upload(&tb.el_cp[d], t.el_cp[d]))) break;
        if ((rc = m->upload(&tb.st_S[d], t.st_S[d]))) break;
        if ((rc = m->upload(&tb.st_lam[d], t.st_lam[d]))) break;
        if ((rc = m->upload(&tb.st_SP[d], t.st_SP[d]))) break;
        if ((rc = m->upload(&tb.st_lamP[d], t.st_lamP[d]))) break;
        if (!t.ax[d].empty() && (rc = m->upload(&tb.ax[d], t.ax[d]))) break;
        // per element: m, L, Sinv, MS, lam, c0, cp contiguous
        const int p = lay.p, n1 = p + 1, q = p - 1, ne = lay.n[d];
        const std::vector<double>* src[7] = {&t.el_m[d], &t.el_L[d], &t.el_Sinv[d], &t.el_MS[d],
                                             &t.el_lam[d], &t.el_c0[d], &t.el_cp[d]};
        const size_t sz[7] = {(size_t)n1, (size_t)n1 * n1, (size_t)q * q, (size_t)q * q, (size_t)q, (size_t)q, (size_t)q};
        std::vector<double> pack;
        for (int e = 0; e < ne; ++e)
            for (int k = 0; k < 7; ++k)
                if (sz[k] && src[k]->size() >= (e + 1) * sz[k])
                    pack.insert(pack.end(), src[k]->begin() + e * sz[k], src[k]->begin() + (e + 1) * sz[k]);
        if ((rc = m->upload(&tb.el_pack[d], pack))) break;
        // per element S^T then S (each the division the condensation and
        // recovery would otherwise do per element on the device)
        std::vector<double> st;
        if (q > 0 && t.el_Sinv[d].size() >= (size_t)ne * q * q && t.el_MS[d].size() >= (size_t)ne * q * q &&
            t.el_m[d].size() >= (size_t)ne * n1) {
            st.resize((size_t)ne * 2 * q * q);
            for (int e = 0; e < ne; ++e) {
                const double* mm = t.el_m[d].data() + (size_t)e * n1;
                const double* si = t.el_Sinv[d].data() + (size_t)e * q * q;
                const double* ms = t.el_MS[d].data() + (size_t)e * q * q;
                double* o = st.data() + (size_t)e * 2 * q * q;
                for (int r = 0; r < q; ++r)
                    for (int c = 0; c < q; ++c) {
                        o[r * q + c] = si[r * q + c] / mm[c + 1];
                        o[q * q + r * q + c] = ms[r * q + c] / mm[r + 1];
                    }
            }
        }
        if ((rc = m->upload(&tb.el_st[d], st))) break;
    }
    if (!rc) rc = m->upload(&tb.st_wP, t.st_wP);
    if (!rc) rc = m->upload(&tb.st_w, t.st_w);
    if (!rc) rc = m->upload(&tb.J, t.J);
    return rc;
}


int check_lds(int p) {
    // working sets beyond the LDS of a CU run from device scratch (see
    // build_level); only the fixed-size kernels bound the degree
    (void)p;
    return 0;
}

// Free canonical node of a plane-layout slot (host mirror of the kernels'
// storage rule); returns false for holes, padding and Dirichlet nodes.
bool decode_slot(const Layout& L, int64_t s, int& i1, int& i2, int& i3) {
    int d = (s >= L.off[2]) ? 2 : (s >= L.off[1] ? 1 : 0);
    int64_t loc = s - L.off[d];
    int j = (int)(loc / L.pstride[d]);
    int64_t rem = loc - (int64_t)j * L.pstride[d];
    int r = (int)(rem / L.pitch[d]), c = (int)(rem - (int64_t)r * L.pitch[d]);
    const int p = L.p;
    if (r >= L.rows[d]) return false;
    bool canon;
    if (d == 0) { i1 = j * p; i3 = r; i2 = c; canon = c < L.N[1]; }
    else if (d == 1) { i2 = j * p; i3 = r; i1 = c; canon = c < L.N[0] && (c % p) != 0; }
    else { i3 = j * p; i2 = r; i1 = c; canon = c < L.N[0] && (c % p) != 0 && (r % p) != 0; }
    if (!canon) return false;
    return !(i1 == 0 || i2 == 0 || i3 == 0 || i1 == L.N[0] - 1 || i2 == L.N[1] - 1 || i3 == L.N[2] - 1);
}

int build_coarse(pmg_mesh* m, Level& lev) {
    if (lev.has_ca) return 0;
    const Layout& L0 = lev.lay;
    const int p0 = L0.p;
    if (p0 > 2) return fail(PMG_EUNSUP, "coarse level degree must be 1 or 2");
    // diagonal at the unknowns, zero at every other slot of the plane layout
    std::vector<double> dg;
    coarse_diagonal(L0, m->lam, lev.h, dg);
    int N0 = 0;
    for (int64_t s = 0; s < L0.len; ++s) {
        int i1, i2, i3;
        if (decode_slot(L0, s, i1, i2, i3)) ++N0;
        else dg[s] = 0.0;
    }
    const int* nl = L0.n;
    const int ne = nl[0] * nl[1] * nl[2];
    CoarseArgs& a = lev.ca;
    a.lay = L0;
    a.N0 = N0;
    a.ne = ne;
    for (int d = 0; d < 3; ++d) {
        a.n[d] = nl[d];
        a.el_m[d] = lev.t64.el_m[d];
        a.el_L[d] = lev.t64.el_L[d];
    }
    a.p0 = p0;
    a.lam = m->lam;
    int rc;
    if ((rc = m->upload(&a.diag, dg))) return rc;
    const size_t nv = (size_t)L0.len;
    a.X = lev.u64;  // the V-cycle reads the coarse solution from there
    if ((rc = m->alloc(&a.rec, 8 * nv))) return rc;
    for (int k = 0; k < 3; ++k)
        if ((rc = m->alloc(&a.W[k], nv))) return rc;
    a.blocks = coarse_blocks(ne, p0);
    for (int k = 0; k < 2; ++k)
        if ((rc = m->alloc(&a.P[k], 2 * (size_t)a.blocks))) return rc;
    if ((rc = m->alloc(&a.S, 2)) || (rc = m->alloc(&a.stat, 2))) return rc;
    HIPCHK(hipMemset(a.S, 0, 2 * sizeof(CoarseState)));
    HIPCHK(hipMemset(a.stat, 0, 2 * sizeof(int)));
    a.iters = m->d_coarse_iters;
    a.mail = m->dmail;
    a.seq = m->d_coarse_seq;
    lev.has_ca = true;
    return 0;
}

// Allocate the tables and work vectors of one level of degree p on the mesh
// with element widths h (pc: degree of the next coarser p-level, 0 = none).
int build_level(pmg_mesh* m, Level& L, int p, int pc, const std::vector<double> h[3]) {
    L.p = p;
    L.pc = pc;
    for (int d = 0; d < 3; ++d) L.h[d] = h[d];
    L.lay = make_layout((int)h[0].size(), (int)h[1].size(), (int)h[2].size(), p, m->bc);
    HostTables t;
    build_level_tables(p, pc, h, t, m->bc);
    int rc;
    if ((rc = fill_tabs(m, L.t64, t, L.lay, pc))) return rc;
    if ((rc = fill_tabs(m, L.t32, t, L.lay, pc))) return rc;
    int64_t n = L.lay.len;
    if ((rc = m->alloc(&L.u64, n)) || (rc = m->alloc(&L.F64, n)) || (rc = m->alloc(&L.y64, n)) ||
        (rc = m->alloc(&L.u32, n)) || (rc = m->alloc(&L.F32, n)) || (rc = m->alloc(&L.y32, n)))
        return rc;
    // condensed-operator workspace, shared by the FP64 and FP32 tables
    // (degrees 1 and 2 form the operator per node, without one)
    const size_t ne = (size_t)L.lay.n[0] * L.lay.n[1] * L.lay.n[2];
    if (p > 2) {
        double* ew = nullptr;
        if ((rc = m->alloc(&ew, ne * 6 * (size_t)(p + 1) * (p + 1)))) return rc;
        L.t64.opE = ew;
        L.t32.opE = reinterpret_cast<float*>(ew);
    } else if (p == 2) {  // one value per element (its interior node)
        double* tw = nullptr;
        if ((rc = m->alloc(&tw, ne))) return rc;
        L.t64.tc = tw;
        L.t32.tc = reinterpret_cast<float*>(tw);
    }
    // workspaces of the batched star smoother (n_S > 16)
    if (2 * p - 1 > 16) {
        const int np = L.t64.np;
        const size_t ns = (size_t)(L.lay.n[0] + 1) * (L.lay.n[1] + 1) * (L.lay.n[2] + 1);
        for (int k = 0; k < 2; ++k) {
            double* x = nullptr;
            if ((rc = m->alloc(&x, ns * 3 * (size_t)np * np))) return rc;
            L.t64.sbX[k] = x;
            L.t32.sbX[k] = reinterpret_cast<float*>(x);
        }
    }
    // device scratch of the general kernels whose working set exceeds the LDS
    {
        const int* n = L.lay.n;
        const size_t nv = (size_t)(n[0] + 1) * (n[1] + 1) * (n[2] + 1);
        const size_t col_e = (size_t)((n[0] + 1) / 2) * ((n[1] + 1) / 2) * ((n[2] + 1) / 2);
        const size_t col_v = (size_t)((n[0] + 2) / 2) * ((n[1] + 2) / 2) * ((n[2] + 2) / 2);
        auto over = [](size_t elems) { return elems * sizeof(double) > kLdsBytes; };
        size_t need = 0;
        if (over(ws_condensed_op(p))) need = std::max(need, ne * ws_condensed_op_v(p));
        if (over(ws_smoother(p)) && 2 * p - 1 <= 16) need = std::max(need, std::min(nv, col_v) * ws_smoother(p));
        if (over(ws_condense(p))) need = std::max(need, std::min(ne, col_e) * ws_condense(p));
        if (over(ws_recover(p))) need = std::max(need, ne * ws_recover(p));
        if (need) {
            double* g = nullptr;
            if ((rc = m->alloc(&g, need))) return rc;
            L.t64.gws = g;
            L.t32.gws = reinterpret_cast<float*>(g);
        }
    }
    return 0;
}

// Degree-1 levels below p_0: hlv[0] on the mesh of p_0, hlv[k] on the mesh
// with pairs of elements of hlv[k-1] merged (while every count is even and
// at least 4).  Built on demand; hlv[k-1] keeps the linear h-transfer
// weights of its mesh and the restriction buffer for hlv[k].
int build_h_levels(pmg_mesh* m, int want) {
    int rc;
    while ((int)m->hlv.size() < want) {
        const int k = (int)m->hlv.size();
        std::vector<double> h[3];
        if (k == 0) {
            for (int d = 0; d < 3; ++d) h[d] = m->h[d];
        } else {
            const Level& f = m->hlv[k - 1];
            bool ok = true;
            for (int d = 0; d < 3; ++d) ok = ok && f.h[d].size() % 2 == 0 && f.h[d].size() >= 4;
            if (!ok) break;
            for (int d = 0; d < 3; ++d)
                for (size_t e = 0; e + 1 < f.h[d].size(); e += 2) h[d].push_back(f.h[d][e] + f.h[d][e + 1]);
        }
        m->hlv.emplace_back();
        Level& L = m->hlv.back();
        if ((rc = build_level(m, L, 1, 0, h))) return rc;
        std::vector<double> dg;
        coarse_diagonal(L.lay, m->lam, L.h, dg);
        if ((rc = m->upload(&L.jd64, dg)) || (rc = m->upload(&L.jd32, dg))) return rc;
        if (k > 0) {
            // the finer level hlv[k-1] gets the weights t_i = h_{i-1} / (h_{i-1} + h_i)
            // of its odd vertices and the restriction buffer
            Level& f = m->hlv[k - 1];
            for (int d = 0; d < 3; ++d) {
                std::vector<double> t(f.h[d].size() + 1, 0.0);
                for (size_t i = 1; i < f.h[d].size(); i += 2) t[i] = f.h[d][i - 1] / (f.h[d][i - 1] + f.h[d][i]);
                if ((rc = m->upload(&f.ht64[d], t)) || (rc = m->upload(&f.ht32[d], t))) return rc;
            }
        }
    }
    // p_0 level: transfer matrix from degree 1 and restriction buffer
    Level& p0 = m->lv[0];
    if (!m->hlv.empty() && !p0.Jlow64) {
        std::vector<double> xc, wc, xf, wf, J;
        gll_nodes_weights(1, xc, wc);
        gll_nodes_weights(p0.p, xf, wf);
        lagrange_interp(xc, xf, J);
        if ((rc = m->upload(&p0.Jlow64, J)) || (rc = m->upload(&p0.Jlow32, J))) return rc;
        const int64_t wl = restrict_work_len(p0.lay, m->hlv[0].lay);
        if ((rc = m->alloc(&p0.tb64, wl)) || (rc = m->alloc(&p0.tb32, wl))) return rc;
    }
    for (size_t k = 1; k < m->hlv.size(); ++k) {
        Level& f = m->hlv[k - 1];
        if (!f.tb64) {
            if ((rc = m->alloc(&f.tb64, m->hlv[k].lay.len)) || (rc = m->alloc(&f.tb32, m->hlv[k].lay.len))) return rc;
        }
    }
    return 0;
}

// Active cycle, coarsest level first: hlv[k-1..0] then the p-levels.
// Tables and work arrays of the exact coarse solve on one level.
int setup_fd(pmg_mesh* m, Level& L) {
    if (L.has_fd) return 0;
    int rc;
    for (int d = 0; d < 3; ++d) {
        std::vector<double> Af, Ab, mu;
        const int bcd = (L.lay.dlo(d) ? 1 : 0) | (L.lay.dhi(d) ? 2 : 0) | (L.lay.per(d) ? 4 : 0);
        build_fd_tables(L.p, L.h[d], bcd, Af, Ab, mu, L.fd.o[d]);
        L.fd.m[d] = (int)mu.size();
        if ((rc = m->upload(&L.fd.Af[d], Af)) || (rc = m->upload(&L.fd.Ab[d], Ab)) || (rc = m->upload(&L.fd.mu[d], mu)))
            return rc;
    }
    const size_t M = (size_t)L.fd.m[0] * L.fd.m[1] * L.fd.m[2];
    if ((rc = m->alloc(&L.fd.X, M)) || (rc = m->alloc(&L.fd.Y, M))) return rc;
    L.has_fd = true;
    return 0;
}

int rebuild_active(pmg_mesh* m) {
    m->coarse_nrec = 0;  // the coarse update counts of another cycle do not carry over
    for (auto& g : m->solver_graphs)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    int nh = std::min(m->hmg_levels, (int)m->hlv.size());
    m->act.clear();
    for (int k = nh - 1; k >= 0; --k) m->act.push_back(&m->hlv[k]);
    for (size_t k = (size_t)m->coarse_level; k < m->lv.size(); ++k) m->act.push_back(&m->lv[k]);
    const int L = (int)m->act.size() - 1;
    for (int l = 0; l <= L; ++l) {
        Level& v = *m->act[l];
        if (l < nh) {
            v.nu = m->hmg_nu;
            v.omega = m->hmg_omega;
        } else {
            v.nu = m->nu_mode == 0 ? 1 : (1 << std::min(20, L - l));
            v.omega = m->omega[l - nh + m->coarse_level];
        }
        if (l > 0) {
            const Level& c = *m->act[l - 1];
            bool same = c.lay.n[0] == v.lay.n[0] && c.lay.n[1] == v.lay.n[1] && c.lay.n[2] == v.lay.n[2];
            v.kind = same ? 'p' : 'h';
            if (same) {
                v.Jd64 = (l == nh) ? v.Jlow64 : v.t64.J;
                v.Jd32 = (l == nh) ? v.Jlow32 : v.t32.J;
            }
        }
    }
    if (m->coarse_kind == 1) return setup_fd(m, *m->act[0]);
    return build_coarse(m, *m->act[0]);
}

int build_mesh(pmg_mesh* m) {
    auto degs = level_degrees(m->p);
    m->L = (int)degs.size() - 1;
    m->lv.resize(degs.size());
    m->hlv.reserve(32);
    m->omega.assign(degs.size(), 1.0);
    int rc = check_lds(m->p);
    if (rc) return rc;
    if ((rc = m->alloc(&m->d_coarse_iters, 1)) || (rc = m->alloc(&m->d_coarse_seq, 1))) return rc;
    HIPCHK(hipMemset(m->d_coarse_iters, 0, sizeof(int)));
    HIPCHK(hipMemset(m->d_coarse_seq, 0, sizeof(int64_t)));
    HIPCHK(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
    for (size_t l = 0; l < degs.size(); ++l) {
        Level& L = m->lv[l];
        if ((rc = build_level(m, L, degs[l], l ? degs[l - 1] : 0, m->h))) return rc;
        if (l > 0) {
            int64_t nc = restrict_work_len(L.lay, m->lv[l - 1].lay);
            if ((rc = m->alloc(&L.tb64, nc)) || (rc = m->alloc(&L.tb32, nc))) return rc;
        }
    }
    if ((rc = rebuild_active(m))) return rc;
    // batched condensation / recovery workspaces on the finest level
    if (m->p >= 9) {
        Level& F = m->lv.back();
        const int q = m->p - 1, qp = 16 * ((q + 15) / 16);
        const size_t ne = (size_t)m->n[0] * m->n[1] * m->n[2];
        F.t64.qp = qp;
        for (int k = 0; k < 2; ++k)
            if ((rc = m->alloc(&F.t64.ixX[k], ne * qp * qp * qp))) return rc;
    }
    const Layout& Lf = m->lv.back().lay;
    int64_t nf = Lf.len;
    if (Lf.any_per() && (rc = m->alloc(&m->w_fgrid, (size_t)Lf.N[0] * Lf.N[1] * Lf.N[2]))) return rc;
    if ((rc = m->alloc(&m->w_u, nf)) || (rc = m->alloc(&m->w_r, nf)) || (rc = m->alloc(&m->w_s, nf)) ||
        (rc = m->alloc(&m->w_p, nf)) || (rc = m->alloc(&m->w_q, nf)) || (rc = m->alloc(&m->w_z, nf)) ||
        (rc = m->alloc(&m->w_F, nf)) || (rc = m->alloc(&m->w_r32, nf)) || (rc = m->alloc(&m->w_z32, nf)))
        return rc;
    // assembled 1D GLL mass of the finest level
    {
        std::vector<double> x, w;
        gll_nodes_weights(m->p, x, w);
        for (int d = 0; d < 3; ++d) {
            std::vector<double> ma(Lf.N[d], 0.0);
            for (int e = 0; e < m->n[d]; ++e)
                for (int i = 0; i <= m->p; ++i) ma[e * m->p + i] += 0.5 * m->h[d][e] * w[i];
            const double* dd = nullptr;
            if ((rc = m->upload(&dd, ma))) return rc;
            m->m1d[d] = const_cast<double*>(dd);
        }
        // lifting of Dirichlet data: coupling of node k of the first (last)
        // element with the line's end node 0 (N - 1), over the assembled mass
        std::vector<double> Ls, tab(6 * (m->p + 1), 0.0);
        stiffness_std(m->p, x, w, Ls);
        const int n1 = m->p + 1;
        for (int d = 0; d < 3; ++d) {
            std::vector<double> ma(Lf.N[d], 0.0);
            for (int e = 0; e < m->n[d]; ++e)
                for (int i = 0; i <= m->p; ++i) ma[e * m->p + i] += 0.5 * m->h[d][e] * w[i];
            const double h0 = m->h[d][0], hl = m->h[d][m->n[d] - 1];
            const int off = Lf.N[d] - 1 - m->p;
            for (int k = 0; k <= m->p; ++k) {
                tab[(2 * d) * n1 + k] = (2.0 / h0) * Ls[k * n1 + 0] / ma[k];
                tab[(2 * d + 1) * n1 + k] = (2.0 / hl) * Ls[k * n1 + m->p] / ma[off + k];
            }
        }
        const double* dt = nullptr;
        if ((rc = m->upload(&dt, tab))) return rc;
        m->lift_tab = const_cast<double*>(dt);
    }
    if ((rc = m->alloc(&m->partials, 2 * REDUCE_BLOCKS)) || (rc = m->alloc(&m->counter, 4)) ||
        (rc = m->alloc(&m->scal, SC_N)))
        return rc;
    HIPCHK(hipMemset(m->counter, 0, 4 * sizeof(unsigned)));
    HIPCHK(hipMemset(m->scal, 0, SC_N * sizeof(double)));
    HIPCHK(hipHostMalloc((void**)&m->hscal, SC_N * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&m->hcit, sizeof(int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&m->hmail, sizeof(HostMail), hipHostMallocMapped | hipHostMallocCoherent));
    std::memset((void*)m->hmail, 0, sizeof(HostMail));
    HIPCHK(hipHostGetDevicePointer((void**)&m->dmail, m->hmail, 0));
    if ((rc = m->alloc(&m->d_pubcnt, 1))) return rc;
    HIPCHK(hipMemset(m->d_pubcnt, 0, sizeof(int64_t)));
    for (auto* v : {&m->lv, &m->hlv})
        for (Level& l : *v) l.ca.mail = m->dmail;
    // large dynamic LDS for the element / star kernels
    HIPCHK(init_kernel_attributes());
    HIPCHK(hipDeviceSynchronize());
    return 0;
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Wait until `ready()` holds, polling the mapped notice block; the stream
// is queried now and then so that a device error or a stream that drained
// without the notice ends the wait with an error instead of spinning.
template <typename P>
int host_wait(hipStream_t st, P ready) {
    const auto t0 = std::chrono::steady_clock::now();
    unsigned k = 0;
    while (!ready()) {
        _mm_pause();
        if ((++k & 255) == 0) {
            const hipError_t e = hipStreamQuery(st);
            if (e != hipSuccess && e != hipErrorNotReady)
                return fail(PMG_EHIP, std::string("device error while waiting: ") + hipGetErrorString(e));
            if (e == hipSuccess) {
                std::atomic_thread_fence(std::memory_order_acquire);
                if (ready()) break;
                return fail(PMG_EHIP, "stream finished without the expected device notice");
            }
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(120))
                return fail(PMG_EHIP, "timed out waiting for the device");
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return 0;
}

// Scalars of the outer solver on the host: the device publishes them to
// the notice block (k_publish, queued here unless `queued`), the host polls.
int read_scalars(pmg_mesh* m, hipStream_t st, bool queued = false) {
    if (!queued) launch_publish(m->scal, SC_N, m->d_pubcnt, m->dmail, st);
    const int64_t want = ++m->pub_expected;
    int rc = host_wait(st, [&] { return m->hmail->seq >= want; });
    if (rc) return rc;
    for (int k = 0; k < SC_N; ++k) m->hscal[k] = m->hmail->sc[k];
    return 0;
}

template <typename T>
void residual(Level& L, const T* F, const T* u, T* y, hipStream_t st) {
    launch_condensed_op<T>(Sel<T>::tabs(L), u, y, st, F);
}

template <typename T>
void residual(pmg_mesh* m, int l, const T* F, const T* u, T* y, hipStream_t st) {
    residual<T>(m->lv[l], F, u, y, st);
}

template <typename T> const T* jdiag(const Level& L);
template <> const double* jdiag<double>(const Level& L) { return L.jd64; }
template <> const float* jdiag<float>(const Level& L) { return L.jd32; }
template <typename T> const T* jdown(const Level& L);
template <> const double* jdown<double>(const Level& L) { return L.Jd64; }
template <> const float* jdown<float>(const Level& L) { return L.Jd32; }
template <typename T> const T* const* hweights(const Level& L);
template <> const double* const* hweights<double>(const Level& L) { return L.ht64; }
template <> const float* const* hweights<float>(const Level& L) { return L.ht32; }

// u += omega Smoother(r) on one level: the star smoother of Alg. 2, or on
// degree-1 levels its equivalent point form (each star is a single vertex,
// so the local solve is a division by the diagonal).
template <typename T>
void schwarz_add(Level& L, const T* r, T* u, T omega, hipStream_t st) {
    if (L.blocks && L.p >= 2) launch_block_smoother_add<T>(Sel<T>::tabs(L), r, u, omega, st);
    else launch_smoother_add<T>(Sel<T>::tabs(L), r, u, omega, st);
}

template <typename T>
void smooth_add(Level& L, const T* r, T* u, hipStream_t st) {
    if (L.p == 1 && jdiag<T>(L)) launch_point_smooth<T>(L.lay, jdiag<T>(L), r, u, (T)L.omega, st);
    else schwarz_add<T>(L, r, u, (T)L.omega, st);
}

// Tables and workspaces of the element-centred block smoother on one level
// (built on first request; the FP32 tables share the FP64 workspaces).
int setup_blocks(pmg_mesh* m, Level& L) {
    if (L.t64.bnp || L.p < 2) return 0;
    const int p = L.p, nS = 3 * p - 1, np = 16 * ((nS + 15) / 16);
    int rc;
    for (int d = 0; d < 3; ++d) {
        std::vector<double> S, lam, w;
        const int bcd = (L.lay.dlo(d) ? 1 : 0) | (L.lay.dhi(d) ? 2 : 0) | (L.lay.per(d) ? 4 : 0);
        build_block_tables(p, L.h[d], np, bcd, S, lam, w);
        if ((rc = m->upload(&L.t64.bl_S[d], S)) || (rc = m->upload(&L.t32.bl_S[d], S)) ||
            (rc = m->upload(&L.t64.bl_lam[d], lam)) || (rc = m->upload(&L.t32.bl_lam[d], lam)) ||
            (rc = m->upload(&L.t64.bl_w[d], w)) || (rc = m->upload(&L.t32.bl_w[d], w)))
            return rc;
    }
    const size_t ws = (size_t)L.lay.n[0] * L.lay.n[1] * L.lay.n[2] * 6 * np * np;
    for (int k = 0; k < 2; ++k) {
        double* X = nullptr;
        if ((rc = m->alloc(&X, ws))) return rc;
        L.t64.bwX[k] = X;
        L.t32.bwX[k] = reinterpret_cast<float*>(X);
    }
    L.t64.bnp = L.t32.bnp = np;
    return 0;
}

// Jacobi-preconditioned CG on level 0 (FP64), x = 0 initially: the init
// kernel, then iteration launches (k updates take k + 2 launches: the first
// forms z_0 and w_0, the last finds convergence; launches after convergence
// return at once).  With a tolerance, as many launches are queued as the
// largest update count of the last few solves needs, the host waits for
// the device's completion notice, and further launches follow only if the
// solve has not finished by then; without one, exactly maxit + 2 launches
// are queued and nothing is waited for.  b and x are level-0 skeleton
// arrays.
//
// Queue n iteration launches with ring indices j0 .. j0 + n - 1 as graphs
// of up to COARSE_GRAPH_MAXN launches (captured on first use; the launches
// of one graph run back to back).
int coarse_launch_range(pmg_mesh* m, Level& L0, long j0, long n, hipStream_t st) {
    if (L0.coarse_exec.empty()) L0.coarse_exec.assign((size_t)COARSE_GRAPH_MAXN * COARSE_RING, nullptr);
    while (n > 0) {
        const int k = (int)std::min<long>(n, COARSE_GRAPH_MAXN);
        const int r0 = (int)(j0 % COARSE_RING);
        hipGraphExec_t& ex = L0.coarse_exec[(size_t)(k - 1) * COARSE_RING + r0];
        if (!ex) {
            HIPCHK(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = hipSuccess;
            for (int j = 0; j < k && e == hipSuccess; ++j)
                e = launch_coarse_iter(L0.ca, (r0 + j) % COARSE_RING, j == k - 1, m->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(m->cap_stream, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail(PMG_EHIP, std::string("coarse graph capture: ") +
                                          hipGetErrorString(e != hipSuccess ? e : e2));
            }
            e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return fail(PMG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        HIPCHK(hipGraphLaunch(ex, st));
        j0 += k;
        n -= k;
    }
    return 0;
}

// With `in_graphs` the caller's graphs hold the initialisation (before) and
// the extraction of x (after); otherwise both are launched here.
int coarse_cg(pmg_mesh* m, const double* b, double* x, hipStream_t st, bool in_graphs = false) {
    Level& L0 = *m->act[0];
    CoarseArgs& a = L0.ca;
    auto deliver = [&]() -> int {
        if (!in_graphs) HIPCHK(launch_coarse_extract(a, x, st));
        return 0;
    };
    const bool init_queued = in_graphs;
    if (!init_queued) HIPCHK(launch_coarse_init(a, b, m->coarse_maxit, m->coarse_rtol, st));
    const int64_t id = ++m->coarse_id;
    if (a.N0 == 0) return deliver();
    const long need = (long)std::max(m->coarse_maxit, 0) + 2;  // launches for maxit updates
    int rc;
    if (!(m->coarse_rtol > 0.0)) {
        if ((rc = coarse_launch_range(m, L0, 0, need, st))) return rc;
        return deliver();
    }
    int est = m->coarse_last;
    for (int i = 0; i < std::min(m->coarse_nrec, 4); ++i) est = std::max(est, m->coarse_recent[i]);
    long launched = std::min(need, (long)est + 2);
    if ((rc = coarse_launch_range(m, L0, 0, launched, st))) return rc;
    HostMail* hm = m->hmail;
    while (true) {
        // the finishing launch reports (id, updates); the last queued launch
        // reports (id, updates so far) if the solve goes on
        const int64_t ran_out = (id << 20) | (int64_t)(launched - 1);
        if ((rc = host_wait(st, [&] { return hm->cseq == id || hm->rseq == ran_out; }))) return rc;
        if (hm->cseq == id) {
            m->coarse_last = hm->cit;
            m->coarse_recent[m->coarse_nrec++ % 4] = hm->cit;
            return deliver();
        }
        if (launched >= need) return fail(PMG_EHIP, "coarse solver did not finish within maxit");
        const long more = std::min(need - launched, std::max(2L * COARSE_RING, launched / 8));
        if ((rc = coarse_launch_range(m, L0, launched, more, st))) return rc;
        launched += more;
    }
}

// The coarse solve of the active cycle: the Jacobi CG, or the exact solve by
// fast diagonalization (kernel launches only, so capturable in a graph).
int coarse_solve(pmg_mesh* m, const double* b, double* x, hipStream_t st) {
    if (m->coarse_kind == 1) {
        Level& L0 = *m->act[0];
        launch_fd_solve(L0.lay, L0.fd, m->lam, b, x, st);
        HIPCHK(hipGetLastError());
        return 0;
    }
    return coarse_cg(m, b, x, st);
}

// Read and reset the device-side coarse iteration counter.
int coarse_stats(pmg_mesh* m, hipStream_t st, int* iters) {
    int h = 0;
    HIPCHK(hipMemcpyAsync(&h, m->d_coarse_iters, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemsetAsync(m->d_coarse_iters, 0, sizeof(int), st));
    *iters = h;
    return 0;
}

// Alg. 3 over the active cycle (coarsest level first), with u_L = z (zero on
// entry unless `nonzero_u`) and F_L = r, in three phases: the down-sweep up
// to the restricted right-hand side of the coarsest level (cast to FP64 for
// an FP32 cycle), the coarse CG in FP64, and the up-sweep.  The down- and
// up-sweeps contain kernel launches only (zero fills are kernels too), so
// the solver can capture them as graphs.
template <typename T>
void vc_coarse_io(pmg_mesh* m, const T* r, T* z, const double*& b, double*& x) {
    auto& A = m->act;
    Level& l0 = *A[0];
    const bool dbl = std::is_same<T, double>::value;
    if (A.size() == 1) {
        b = dbl ? reinterpret_cast<const double*>(r) : l0.F64;
        x = dbl ? reinterpret_cast<double*>(z) : l0.u64;
    } else {
        b = dbl ? reinterpret_cast<const double*>(Sel<T>::F(l0)) : l0.F64;
        x = l0.u64;
    }
}

// One grid transfer between active levels lv (fine) and lc (coarse); the
// coarse-side array may be FP64 below an FP32 fine level.
template <typename T, typename TC>
void restrict_to(Level& lv, Level& lc, const T* y, TC* Fc, hipStream_t st) {
    if (lv.kind == 'p') launch_restrict<T>(lv.lay, lc.lay, jdown<T>(lv), y, Fc, Sel<T>::tb(lv), st);
    else launch_hrestrict<T>(lv.lay, lc.lay, hweights<T>(lv), y, Fc, st);
}
template <typename T, typename TC>
void prolong_from(Level& lc, Level& lv, const TC* uc, T* u, hipStream_t st) {
    if (lv.kind == 'p') launch_prolong_add<T>(lc.lay, lv.lay, jdown<T>(lv), uc, u, st);
    else launch_hprolong_add<T>(lc.lay, lv.lay, hweights<T>(lv), uc, u, st);
}

// z_clear: z already holds zeros (the mixed-precision CG clears it in its
// update), so no fill before the first smoothing
template <typename T>
int vc_down(pmg_mesh* m, const T* r, T* z, bool nonzero_u, hipStream_t st, bool z_clear = false) {
    auto& A = m->act;
    const int L = (int)A.size() - 1;
    Level& l0 = *A[0];
    if (L == 0) {
        if (!std::is_same<T, double>::value) launch_cast_scale<T, double>(r, l0.F64, nullptr, 0, l0.lay.len, st);
        return 0;
    }
    if (!nonzero_u && !z_clear) launch_fill_zero<T>(z, A[L]->lay.len, st);
    const T* F = r;
    for (int l = L; l >= 1; --l) {
        Level& lv = *A[l];
        T* u = (l == L) ? z : Sel<T>::u(lv);
        if (l != L) launch_fill_zero<T>(u, lv.lay.len, st);
        bool zero = (l != L) || !nonzero_u;
        T* y = Sel<T>::y(lv);
        for (int i = 0; i < lv.nu; ++i) {
            const T* res = F;
            if (!zero) {
                residual<T>(lv, F, u, y, st);
                res = y;
            }
            smooth_add<T>(lv, res, u, st);
            zero = false;
        }
        residual<T>(lv, F, u, y, st);
        Level& lc = *A[l - 1];
        if (l == 1) {   // into the FP64 right-hand side of the coarse solve
            restrict_to<T, double>(lv, lc, y, l0.F64, st);
            break;
        }
        restrict_to<T, T>(lv, lc, y, Sel<T>::F(lc), st);
        F = Sel<T>::F(lc);
    }
    return 0;
}

template <typename T>
int vc_up(pmg_mesh* m, const T* r, T* z, hipStream_t st) {
    auto& A = m->act;
    const int L = (int)A.size() - 1;
    Level& l0 = *A[0];
    const bool dbl = std::is_same<T, double>::value;
    if (L == 0) {
        if (!dbl) launch_cast_scale<double, T>(l0.u64, z, nullptr, 0, l0.lay.len, st);
        return 0;
    }
    const T* uc = nullptr;
    for (int l = 1; l <= L; ++l) {
        Level& lv = *A[l];
        Level& lc = *A[l - 1];
        T* u = (l == L) ? z : Sel<T>::u(lv);
        const T* F = (l == L) ? r : Sel<T>::F(lv);
        if (l == 1) prolong_from<T, double>(lc, lv, l0.u64, u, st);   // the FP64 coarse solution
        else prolong_from<T, T>(lc, lv, uc, u, st);
        T* y = Sel<T>::y(lv);
        for (int i = 0; i < lv.nu; ++i) {
            residual<T>(lv, F, u, y, st);
            smooth_add<T>(lv, y, u, st);
        }
        uc = u;
    }
    return 0;
}

template <typename T>
int vcycle_impl(pmg_mesh* m, const T* r, T* z, bool nonzero_u, hipStream_t st) {
    int rc;
    if ((rc = vc_down<T>(m, r, z, nonzero_u, st))) return rc;
    const double* b;
    double* x;
    vc_coarse_io<T>(m, r, z, b, x);
    if ((rc = coarse_solve(m, b, x, st))) return rc;
    return vc_up<T>(m, r, z, st);
}

// Capture the launches `body` makes into an executable graph (on the
// mesh's private stream; the graph is later launched on the caller's).
template <typename F>
int capture_graph(pmg_mesh* m, hipGraphExec_t* out, F body) {
    HIPCHK(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = body(m->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(m->cap_stream, &g);
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : fail(PMG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PMG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return 0;
}

int check_mesh(const pmg_mesh* m) {
    if (!m) return fail(PMG_EINVAL, "null mesh");
    return 0;
}

int check_level(const pmg_mesh* m, int level) {
    if (!m) return fail(PMG_EINVAL, "null mesh");
    if (level < 0 || level > m->L) return fail(PMG_EINVAL, "level out of range");
    return 0;
}

// Boundary kinds of the six sides (x1 low, x1 high, x2 low, ..., x3 high;
// PMG_BC_*) as Layout::bc; -1 if invalid.
int encode_bc(const int* kinds, const int n[3], double lambda, std::string& why) {
    if (!kinds) return BC_ALL_DIRICHLET;
    int bc = 0;
    bool any_dir = false;
    for (int d = 0; d < 3; ++d) {
        const int lo = kinds[2 * d], hi = kinds[2 * d + 1];
        for (int k : {lo, hi})
            if (k != PMG_BC_DIRICHLET && k != PMG_BC_NEUMANN && k != PMG_BC_PERIODIC) {
                why = "boundary kind must be PMG_BC_DIRICHLET, PMG_BC_NEUMANN or PMG_BC_PERIODIC";
                return -1;
            }
        if ((lo == PMG_BC_PERIODIC) != (hi == PMG_BC_PERIODIC)) {
            why = "a periodic direction is periodic on both sides";
            return -1;
        }
        if (lo == PMG_BC_PERIODIC) {
            if (n[d] < 3) {
                why = "a periodic direction needs at least 3 elements";
                return -1;
            }
            bc |= 1 << (6 + d);
        }
        if (lo == PMG_BC_DIRICHLET) bc |= 1 << d;
        if (hi == PMG_BC_DIRICHLET) bc |= 1 << (3 + d);
        any_dir = any_dir || lo == PMG_BC_DIRICHLET || hi == PMG_BC_DIRICHLET;
    }
    if (!any_dir && !(lambda > 0.0)) {
        why = "without a Dirichlet side the operator is singular unless lambda > 0";
        return -1;
    }
    return bc;
}

int create(int n1, int n2, int n3, int p, double lambda, const double* hx, const double* hy, const double* hz,
           double stretch, const int* kinds, pmg_mesh** out) {
    if (!out) return fail(PMG_EINVAL, "out is null");
    *out = nullptr;
    if (n1 < 1 || n2 < 1 || n3 < 1) return fail(PMG_EINVAL, "element counts must be >= 1");
    if (p < 1 || p > PMG_MAX_DEGREE) return fail(PMG_EINVAL, "degree out of range");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(PMG_EINVAL, "lambda must be finite and >= 0");
    const int nn0[3] = {n1, n2, n3};
    std::string why;
    const int bc = encode_bc(kinds, nn0, lambda, why);
    if (bc < 0) return fail(PMG_EINVAL, why);
    pmg_mesh* m = new (std::nothrow) pmg_mesh();
    if (!m) return fail(PMG_ENOMEM, "host allocation");
    m->n[0] = n1; m->n[1] = n2; m->n[2] = n3;
    m->p = p;
    m->lam = lambda;
    m->bc = bc;
    // other boundaries than Dirichlet: the exact coarse solve (the Jacobi CG
    // coarse solver and the degree-1 levels assume Dirichlet sides)
    if (bc != BC_ALL_DIRICHLET) m->coarse_kind = 1;
    const int nn[3] = {n1, n2, n3};
    const double* hs[3] = {hx, hy, hz};
    for (int d = 0; d < 3; ++d) {
        m->h[d].resize(nn[d]);
        if (hs[d]) {
            for (int e = 0; e < nn[d]; ++e) {
                if (!(hs[d][e] > 0.0) || !std::isfinite(hs[d][e])) {
                    delete m;
                    return fail(PMG_EINVAL, "element widths must be finite and > 0");
                }
                m->h[d][e] = hs[d][e];
            }
        } else {
            double s = 0.0;
            for (int e = 0; e < nn[d]; ++e) s += std::pow(stretch, e);
            for (int e = 0; e < nn[d]; ++e) m->h[d][e] = std::pow(stretch, e) / s;
        }
    }
    int rc = build_mesh(m);
    if (rc) {
        pmg_destroy_mesh(m);
        return rc;
    }
    *out = m;
    return 0;
}

}  // namespace

extern "C" {

const char* pmg_last_error(void) { return g_err.c_str(); }

int pmg_create_mesh(int n1, int n2, int n3, int p, double lambda, double stretch, pmg_mesh** out) {
    if (!(stretch >= 1.0) || !std::isfinite(stretch)) return fail(PMG_EINVAL, "stretch must be >= 1");
    return create(n1, n2, n3, p, lambda, nullptr, nullptr, nullptr, stretch, nullptr, out);
}

int pmg_create_mesh_widths(int n1, int n2, int n3, int p, double lambda, const double* hx, const double* hy,
                           const double* hz, pmg_mesh** out) {
    if (!hx || !hy || !hz) return fail(PMG_EINVAL, "width arrays must not be null");
    return create(n1, n2, n3, p, lambda, hx, hy, hz, 1.0, nullptr, out);
}

int pmg_create_mesh_bc(int n1, int n2, int n3, int p, double lambda, const double* hx, const double* hy,
                       const double* hz, const int* bc, pmg_mesh** out) {
    if (!hx || !hy || !hz) return fail(PMG_EINVAL, "width arrays must not be null");
    if (!bc) return fail(PMG_EINVAL, "boundary kinds must not be null");
    return create(n1, n2, n3, p, lambda, hx, hy, hz, 1.0, bc, out);
}

void pmg_destroy_mesh(pmg_mesh* m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    for (auto* v : {&m->lv, &m->hlv})
        for (Level& l : *v)
            for (hipGraphExec_t g : l.coarse_exec)
                if (g) (void)hipGraphExecDestroy(g);
    for (hipGraphExec_t g : m->solver_graphs)
        if (g) (void)hipGraphExecDestroy(g);
    for (void* q : m->allocs) (void)hipFree(q);
    if (m->hscal) (void)hipHostFree(m->hscal);
    if (m->hcit) (void)hipHostFree(m->hcit);
    if (m->hmail) (void)hipHostFree((void*)m->hmail);
    if (m->cap_stream) (void)hipStreamDestroy(m->cap_stream);
    delete m;
}

int pmg_num_levels(const pmg_mesh* m, int* L) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (!L) return fail(PMG_EINVAL, "null output");
    *L = m->L;
    return 0;
}

int pmg_level_degree(const pmg_mesh* m, int level, int* p) {
    if (check_level(m, level)) return PMG_EINVAL;
    if (!p) return fail(PMG_EINVAL, "null output");
    *p = m->lv[level].p;
    return 0;
}

int pmg_skeleton_len(const pmg_mesh* m, int level, int64_t* len) {
    if (check_level(m, level)) return PMG_EINVAL;
    if (!len) return fail(PMG_EINVAL, "null output");
    *len = m->lv[level].lay.len;
    return 0;
}

int pmg_grid_len(const pmg_mesh* m, int64_t* len) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (!len) return fail(PMG_EINVAL, "null output");
    const Layout& L = m->lv.back().lay;
    *len = (int64_t)L.N[0] * L.N[1] * L.N[2];
    return 0;
}

int pmg_grid_coords(const pmg_mesh* m, double* x1, double* x2, double* x3) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (!x1 || !x2 || !x3) return fail(PMG_EINVAL, "null output");
    std::vector<double> x, w;
    gll_nodes_weights(m->p, x, w);
    double* out[3] = {x1, x2, x3};
    for (int d = 0; d < 3; ++d) {
        double x0 = 0.0;
        for (int e = 0; e < m->n[d]; ++e) {
            for (int i = 0; i < m->p; ++i) out[d][e * m->p + i] = x0 + 0.5 * m->h[d][e] * (x[i] + 1.0);
            x0 += m->h[d][e];
        }
        out[d][m->n[d] * m->p] = x0;
    }
    return 0;
}

int pmg_grid_to_skeleton(pmg_mesh* m, int dtype, const double* g, void* s, void* stream) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (!g || !s) return fail(PMG_EINVAL, "null pointer");
    const Layout& L = m->lv.back().lay;
    if (dtype == PMG_F64) launch_grid_to_skel<double>(L, g, (double*)s, S(stream));
    else if (dtype == PMG_F32) launch_grid_to_skel<float>(L, g, (float*)s, S(stream));
    else return fail(PMG_EINVAL, "bad dtype");
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_skeleton_to_grid(pmg_mesh* m, int dtype, const void* s, double* g, void* stream) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (!g || !s) return fail(PMG_EINVAL, "null pointer");
    const Layout& L = m->lv.back().lay;
    if (dtype == PMG_F64) launch_skel_to_grid<double>(L, (const double*)s, g, S(stream));
    else if (dtype == PMG_F32) launch_skel_to_grid<float>(L, (const float*)s, g, S(stream));
    else return fail(PMG_EINVAL, "bad dtype");
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_apply_condensed_op(pmg_mesh* m, int level, int dtype, const void* u, void* y, void* stream) {
    if (check_level(m, level)) return PMG_EINVAL;
    if (!u || !y || u == y) return fail(PMG_EINVAL, "null or aliasing pointers");
    Level& L = m->lv[level];
    if (dtype == PMG_F64) launch_condensed_op<double>(L.t64, (const double*)u, (double*)y, S(stream));
    else if (dtype == PMG_F32) launch_condensed_op<float>(L.t32, (const float*)u, (float*)y, S(stream));
    else return fail(PMG_EINVAL, "bad dtype");
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_schwarz_smooth(pmg_mesh* m, int level, int dtype, const void* r, void* du, double omega, void* stream) {
    if (check_level(m, level)) return PMG_EINVAL;
    if (!r || !du || r == du) return fail(PMG_EINVAL, "null or aliasing pointers");
    Level& L = m->lv[level];
    if (dtype == PMG_F64) {
        launch_fill_zero<double>((double*)du, L.lay.len, S(stream));  // a kernel: capturable
        schwarz_add<double>(L, (const double*)r, (double*)du, omega, S(stream));
    } else if (dtype == PMG_F32) {
        launch_fill_zero<float>((float*)du, L.lay.len, S(stream));
        schwarz_add<float>(L, (const float*)r, (float*)du, (float)omega, S(stream));
    } else return fail(PMG_EINVAL, "bad dtype");
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_schwarz_smooth_add(pmg_mesh* m, int level, int dtype, const void* r, void* u, double omega,
                           void* stream) {
    if (check_level(m, level)) return PMG_EINVAL;
    if (!r || !u || r == u) return fail(PMG_EINVAL, "null or aliasing pointers");
    Level& L = m->lv[level];
    if (dtype == PMG_F64) schwarz_add<double>(L, (const double*)r, (double*)u, omega, S(stream));
    else if (dtype == PMG_F32) schwarz_add<float>(L, (const float*)r, (float*)u, (float)omega, S(stream));
    else return fail(PMG_EINVAL, "bad dtype");
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_prolong_add(pmg_mesh* m, int level, int dtype, const void* c, void* f, void* stream) {
    if (check_level(m, level) || level < 1) return fail(PMG_EINVAL, "level must be 1..L");
    if (!c || !f) return fail(PMG_EINVAL, "null pointer");
    Level& lf = m->lv[level];
    Level& lc = m->lv[level - 1];
    if (dtype == PMG_F64) launch_prolong_add<double>(lc.lay, lf.lay, lf.t64.J, (const double*)c, (double*)f, S(stream));
    else if (dtype == PMG_F32) launch_prolong_add<float>(lc.lay, lf.lay, lf.t32.J, (const float*)c, (float*)f, S(stream));
    else return fail(PMG_EINVAL, "bad dtype");
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_restrict(pmg_mesh* m, int level, int dtype, const void* f, void* c, void* stream) {
    if (check_level(m, level) || level < 1) return fail(PMG_EINVAL, "level must be 1..L");
    if (!c || !f) return fail(PMG_EINVAL, "null pointer");
    Level& lf = m->lv[level];
    Level& lc = m->lv[level - 1];
    if (dtype == PMG_F64)
        launch_restrict<double>(lf.lay, lc.lay, lf.t64.J, (const double*)f, (double*)c, lf.tb64, S(stream));
    else if (dtype == PMG_F32)
        launch_restrict<float>(lf.lay, lc.lay, lf.t32.J, (const float*)f, (float*)c, lf.tb32, S(stream));
    else return fail(PMG_EINVAL, "bad dtype");
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_set_cycle(pmg_mesh* m, int nu_mode, double coarse_rtol, int coarse_maxit) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (nu_mode != 0 && nu_mode != 1) return fail(PMG_EINVAL, "nu_mode must be 0 or 1");
    if (!(coarse_rtol >= 0.0) || coarse_maxit < 0 || coarse_maxit > PMG_MAX_COARSE_IT)
        return fail(PMG_EINVAL, "bad coarse parameters");
    m->nu_mode = nu_mode;
    m->coarse_rtol = coarse_rtol;
    m->coarse_maxit = coarse_maxit;
    return rebuild_active(m);
}

int pmg_set_coarse_mg(pmg_mesh* m, int levels, double omega, int nu) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (levels < 0 || levels > 16 || !(omega > 0.0) || !std::isfinite(omega) || nu < 1 || nu > 16)
        return fail(PMG_EINVAL, "bad coarse multigrid parameters");
    if (levels > 0 && m->lv[0].p < 2) return fail(PMG_EUNSUP, "degree-1 levels need p_0 = 2");
    if (levels > 0 && m->bc != BC_ALL_DIRICHLET)
        return fail(PMG_EUNSUP, "degree-1 levels are built for Dirichlet sides only");
    if (levels > 0 && m->coarse_level != 0) return fail(PMG_EUNSUP, "degree-1 levels need the coarse level 0");
    int rc;
    if ((rc = build_h_levels(m, levels))) return rc;
    m->hmg_levels = levels;
    m->hmg_omega = omega;
    m->hmg_nu = nu;
    if ((rc = rebuild_active(m))) return rc;
    HIPCHK(hipDeviceSynchronize());
    return 0;
}

int pmg_set_coarse_solver(pmg_mesh* m, int kind) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (kind != 0 && kind != 1) return fail(PMG_EINVAL, "coarse solver kind must be 0 (CG) or 1 (exact)");
    if (kind == 0 && m->bc != BC_ALL_DIRICHLET)
        return fail(PMG_EUNSUP, "the coarse CG is built for Dirichlet sides only; this mesh keeps the exact solve");
    if (kind == 0 && m->coarse_level != 0) return fail(PMG_EUNSUP, "the coarse CG runs on level 0 only");
    m->coarse_kind = kind;
    int rc;
    if ((rc = rebuild_active(m))) return rc;
    HIPCHK(hipDeviceSynchronize());
    return 0;
}

int pmg_set_coarse_level(pmg_mesh* m, int level) {
    if (check_level(m, level)) return PMG_EINVAL;
    if (level > 0 && m->coarse_kind != 1) return fail(PMG_EUNSUP, "a coarse level above 0 needs the exact coarse solve");
    if (level > 0 && m->hmg_levels > 0) return fail(PMG_EUNSUP, "a coarse level above 0 excludes degree-1 levels");
    m->coarse_level = level;
    int rc;
    if ((rc = rebuild_active(m))) return rc;
    HIPCHK(hipDeviceSynchronize());
    return 0;
}

int pmg_set_smoother(pmg_mesh* m, int kind) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (kind != 0 && kind != 1) return fail(PMG_EINVAL, "smoother kind must be 0 (star) or 1 (element-centred)");
    int rc;
    if (kind == 1)
        for (auto& L : m->lv)
            if ((rc = setup_blocks(m, L))) return rc;
    for (auto& L : m->lv) L.blocks = kind == 1;
    m->smoother_kind = kind;
    if ((rc = rebuild_active(m))) return rc;
    HIPCHK(hipDeviceSynchronize());
    return 0;
}

int pmg_set_damping(pmg_mesh* m, const float* om, int n) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (n < 0 || n > m->L || (n > 0 && !om)) return fail(PMG_EINVAL, "bad damping vector");
    for (int l = 0; l <= m->L; ++l) m->omega[l] = 1.0;
    for (int j = 0; j < n; ++j) {
        if (!(om[j] > 0.0f) || !std::isfinite(om[j])) return fail(PMG_EINVAL, "damping must be > 0");
        m->omega[m->L - j] = om[j];
    }
    return rebuild_active(m);
}

int pmg_vcycle(pmg_mesh* m, int dtype, const void* r, void* z, void* stream) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (!r || !z || r == z) return fail(PMG_EINVAL, "null or aliasing pointers");
    int rc;
    if (dtype == PMG_F64) rc = vcycle_impl<double>(m, (const double*)r, (double*)z, false, S(stream));
    else if (dtype == PMG_F32) rc = vcycle_impl<float>(m, (const float*)r, (float*)z, false, S(stream));
    else return fail(PMG_EINVAL, "bad dtype");
    if (rc) return rc;
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_coarse_solve(pmg_mesh* m, const double* F0, double* u0, int* iters, void* stream) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (!F0 || !u0) return fail(PMG_EINVAL, "null pointer");
    int it = 0, rc;
    if ((rc = coarse_stats(m, S(stream), &it))) return rc;
    if ((rc = coarse_solve(m, F0, u0, S(stream)))) return rc;
    if ((rc = coarse_stats(m, S(stream), &it))) return rc;
    m->coarse_last = it;
    if (iters) *iters = it;
    return 0;
}

// The right-hand side grid as the element kernels read it: on a mesh with a
// periodic direction a copy whose last layers repeat the first ones (the
// values given there are ignored).
static const double* rhs_grid(pmg_mesh* m, const double* f, hipStream_t st) {
    const Layout& L = m->lv.back().lay;
    if (!L.any_per()) return f;
    launch_grid_seam_copy(L, f, m->w_fgrid, st);
    return m->w_fgrid;
}

int pmg_condense_rhs(pmg_mesh* m, const double* f, double* Fh, void* stream) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (!f || !Fh) return fail(PMG_EINVAL, "null pointer");
    launch_condense(m->lv.back().t64, m->m1d[0], m->m1d[1], m->m1d[2], rhs_grid(m, f, S(stream)), Fh, S(stream));
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_recover_interior(pmg_mesh* m, const double* f, const double* uh, double* u, void* stream) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (!f || !uh || !u) return fail(PMG_EINVAL, "null pointer");
    launch_recover(m->lv.back().t64, rhs_grid(m, f, S(stream)), uh, u, S(stream));
    HIPCHK(hipGetLastError());
    return 0;
}

static int solve_common(pmg_mesh* m, const double* f, double* ug, double rtol, int maxit, int mode, int pdt,
                        pmg_stats* st_out, hipStream_t st) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (!f || !ug) return fail(PMG_EINVAL, "null pointer");
    if (!(rtol >= 0.0) || maxit < 0) return fail(PMG_EINVAL, "bad tolerance or iteration limit");
    if (pdt != PMG_F64 && pdt != PMG_F32) return fail(PMG_EINVAL, "bad dtype");
    // with no smoothed level the cycle is the coarse solve alone, which runs
    // in FP64 either way: an FP32 cycle would only round r and z
    if (m->act.size() == 1) pdt = PMG_F64;
    const Layout& Lf = m->lv.back().lay;
    const int64_t n = Lf.len;
    pmg_stats stats;
    std::memset(&stats, 0, sizeof(stats));
    HIPCHK(hipStreamSynchronize(st));
    std::atomic_thread_fence(std::memory_order_acquire);
    m->pub_expected = m->hmail->seq;  // resynchronise the notice count
    launch_fill_zero<int>(m->d_coarse_iters, 1, st);
    hipEvent_t ev[4];
    for (int i = 0; i < 4; ++i) HIPCHK(hipEventCreate(&ev[i]));
    HIPCHK(hipEventRecord(ev[0], st));
    const double* fg = rhs_grid(m, f, st);
    launch_condense(m->lv.back().t64, m->m1d[0], m->m1d[1], m->m1d[2], fg, m->w_F, st);
    HIPCHK(hipEventRecord(ev[1], st));
    int rc = 0, status = 0;
    // r = F, u = 0, s = r, p = 0, delta = 1
    launch_pcg_start(m->w_F, m->w_r, m->w_s, m->w_u, m->w_p, m->scal + SC_DELTA, n, st);
    launch_dot2<double>(m->w_r, m->w_r, nullptr, n, m->partials, m->counter, m->scal + SC_RR, st);
    if ((rc = read_scalars(m, st))) return rc;
    double rr0 = m->hscal[SC_RR], rr = rr0;
    stats.res0 = std::sqrt(rr0);
    stats.res_hist[0] = stats.res0;
    const double eps = rtol * stats.res0;
    int it = 0;
    if (!std::isfinite(rr0)) status = PMG_BREAKDOWN;  // NaN or Inf in the condensed right-hand side
    // FP32 preconditioner: the first cycle's input r / |r| (each later one is
    // written by the update that produces its residual)
    if (mode == 0 && pdt == PMG_F32 && !status)
        launch_cast_down(m->w_r, m->w_r32, m->scal + SC_RR, m->scal + SC_ZS, n, st, m->w_z32);
    while (!status && std::sqrt(rr) > eps && it < maxit) {
        if (mode == 1) {
            // Alg. 4: u <- MultigridCycle(u, F); r = F - H u
            if (m->act.size() == 1) {
                // coarse CG on the whole problem applied to the residual
                if ((rc = vcycle_impl<double>(m, m->w_r, m->w_z, false, st))) return rc;
                launch_axpy<double>(1.0, m->w_z, m->w_u, n, st);
            } else if ((rc = vcycle_impl<double>(m, m->w_F, m->w_u, true, st))) return rc;
            residual<double>(m, m->L, m->w_F, m->w_u, m->w_r, st);
            launch_dot2<double>(m->w_r, m->w_r, nullptr, n, m->partials, m->counter, m->scal + SC_RR, st);
            if ((rc = read_scalars(m, st))) return rc;
            rr = m->hscal[SC_RR];
        } else {
            // Alg. 5: z = MG(0, r) (FP64, or FP32 on r / |r| scaled back by
            // |r|, the norm taken from the device), then the direction and
            // the update.  Everything but the coarse CG iterations is
            // replayed from two graphs captured on first use (the first ends
            // with the coarse CG's initialisation, the second starts with the
            // extraction of its solution).
            const int gi = pdt == PMG_F64 ? 0 : 2;
            const double* cb;
            double* cx;
            if (pdt == PMG_F64) vc_coarse_io<double>(m, m->w_r, m->w_z, cb, cx);
            else vc_coarse_io<float>(m, m->w_r32, m->w_z32, cb, cx);
            if (!m->solver_graphs[gi]) {
                auto part_a = [&](hipStream_t s) -> int {
                    int r2;
                    if (pdt == PMG_F64) r2 = vc_down<double>(m, m->w_r, m->w_z, false, s);
                    else r2 = vc_down<float>(m, m->w_r32, m->w_z32, false, s, true);   // cleared by the update
                    if (r2) return r2;
                    if (m->coarse_kind == 1) {   // the exact coarse solve, inside the graph
                        Level& L0 = *m->act[0];
                        launch_fd_solve(L0.lay, L0.fd, m->lam, cb, cx, s);
                        return 0;
                    }
                    HIPCHK(launch_coarse_init(m->act[0]->ca, cb, m->coarse_maxit, m->coarse_rtol, s));
                    return 0;
                };
                auto part_b = [&](hipStream_t s) -> int {
                    if (m->coarse_kind != 1) HIPCHK(launch_coarse_extract(m->act[0]->ca, cx, s));
                    int r2 = pdt == PMG_F64 ? vc_up<double>(m, m->w_r, m->w_z, s)
                                            : vc_up<float>(m, m->w_r32, m->w_z32, s);
                    if (r2) return r2;
                    // gamma = z . r, gamma0 = z . s, p = beta p + z, q = H p,
                    // q . p, the update (FP32: z = zs z32 taken on the fly, and
                    // the update writes the next cycle's r32)
                    if (pdt == PMG_F64) {
                        launch_dot2<double>(m->w_z, m->w_r, m->w_s, n, m->partials, m->counter, m->scal + SC_GAMMA,
                                            s);
                        launch_pcg_dir(m->w_p, m->w_z, m->scal, n, s);
                    } else {
                        launch_dot_zmix(m->w_z32, m->scal + SC_ZS, m->w_r, m->w_s, n, m->partials, m->counter,
                                        m->scal + SC_GAMMA, s);
                        launch_pcg_dir_mixed(m->w_p, m->w_z32, m->scal + SC_ZS, m->scal, n, s);
                    }
                    launch_condensed_op<double>(m->lv.back().t64, m->w_p, m->w_q, s);
                    launch_dot2<double>(m->w_q, m->w_p, nullptr, n, m->partials, m->counter, m->scal + SC_QP, s);
                    launch_pcg_update(m->w_u, m->w_r, m->w_s, m->w_p, m->w_q, m->scal + SC_GAMMA, m->scal + SC_QP,
                                      n, m->partials, m->counter, m->scal + SC_RR, m->scal + SC_DELTA, s,
                                      pdt == PMG_F64 ? nullptr : m->w_r32, m->scal + SC_ZS,
                                      pdt == PMG_F64 ? nullptr : m->w_z32);
                    launch_publish(m->scal, SC_N, m->d_pubcnt, m->dmail, s);
                    return 0;
                };
                if ((rc = capture_graph(m, &m->solver_graphs[gi], part_a)) ||
                    (rc = capture_graph(m, &m->solver_graphs[gi + 1], part_b)))
                    return rc;
            }
            HIPCHK(hipGraphLaunch(m->solver_graphs[gi], st));
            if (m->coarse_kind != 1 && (rc = coarse_cg(m, cb, cx, st, true))) return rc;
            HIPCHK(hipGraphLaunch(m->solver_graphs[gi + 1], st));
            if ((rc = read_scalars(m, st, true))) return rc;
            rr = m->hscal[SC_RR];
            double qp = m->hscal[SC_QP];
            if (!(qp > 0.0) || !std::isfinite(rr)) {
                status = PMG_BREAKDOWN;
                ++it;
                if (it < PMG_MAX_HIST) stats.res_hist[it] = std::sqrt(rr);
                break;
            }
        }
        ++it;
        if (it < PMG_MAX_HIST) stats.res_hist[it] = std::sqrt(rr);
        if (!std::isfinite(rr)) {
            status = PMG_BREAKDOWN;
            break;
        }
    }
    if (!status && !(std::sqrt(rr) <= eps)) status = PMG_NOT_CONVERGED;
    HIPCHK(hipEventRecord(ev[2], st));
    launch_recover(m->lv.back().t64, fg, m->w_u, ug, st);
    HIPCHK(hipEventRecord(ev[3], st));
    HIPCHK(hipMemcpyAsync(m->hcit, m->d_coarse_iters, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    float t0 = 0, t1 = 0, t2 = 0;
    (void)hipEventElapsedTime(&t0, ev[0], ev[1]);   // a failed query leaves 0
    (void)hipEventElapsedTime(&t1, ev[1], ev[2]);
    (void)hipEventElapsedTime(&t2, ev[2], ev[3]);
    for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ev[i]);
    stats.iters = it;
    stats.status = status;
    stats.rel_res = stats.res0 > 0 ? std::sqrt(rr) / stats.res0 : 0.0;
    stats.coarse_iters = *m->hcit;
    stats.t_pre_ms = t0;
    stats.t_iter_ms = t1;
    stats.t_post_ms = t2;
    if (st_out) *st_out = stats;
    HIPCHK(hipGetLastError());
    return status;
}

int pmg_pcg_solve(pmg_mesh* m, const double* f, double* u, double rtol, int maxit, int pdt, pmg_stats* st,
                  void* stream) {
    return solve_common(m, f, u, rtol, maxit, 0, pdt, st, S(stream));
}

int pmg_mg_solve(pmg_mesh* m, const double* f, double* u, double rtol, int maxit, pmg_stats* st, void* stream) {
    return solve_common(m, f, u, rtol, maxit, 1, PMG_F64, st, S(stream));
}

int pmg_lift_dirichlet(pmg_mesh* m, const double* f, const double* g, double* out, void* stream) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (m->bc != BC_ALL_DIRICHLET) return fail(PMG_EUNSUP, "Dirichlet data by lifting needs Dirichlet sides only");
    if (!f || !g || !out) return fail(PMG_EINVAL, "null pointer");
    if (out == g) return fail(PMG_EINVAL, "out must not alias g");
    launch_lift_dirichlet(m->lv.back().lay.N, m->p, m->lift_tab, f, g, out, S(stream));
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_set_boundary(pmg_mesh* m, const double* g, double* u, void* stream) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (m->bc != BC_ALL_DIRICHLET) return fail(PMG_EUNSUP, "Dirichlet data by lifting needs Dirichlet sides only");
    if (!g || !u) return fail(PMG_EINVAL, "null pointer");
    launch_set_boundary(m->lv.back().lay.N, g, u, S(stream));
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_pcg_solve_dirichlet(pmg_mesh* m, const double* f, const double* g, double* u, double rtol, int maxit,
                            int pdt, pmg_stats* st, void* stream) {
    if (check_mesh(m)) return PMG_EINVAL;
    if (m->bc != BC_ALL_DIRICHLET) return fail(PMG_EUNSUP, "Dirichlet data by lifting needs Dirichlet sides only");
    if (!f || !g || !u) return fail(PMG_EINVAL, "null pointer");
    if (u == g) return fail(PMG_EINVAL, "u must not alias g");
    const int* N = m->lv.back().lay.N;
    int rc;
    if (!m->w_lift && (rc = m->alloc(&m->w_lift, (size_t)N[0] * N[1] * N[2]))) return rc;
    const hipStream_t s = S(stream);
    launch_lift_dirichlet(N, m->p, m->lift_tab, f, g, m->w_lift, s);
    HIPCHK(hipGetLastError());
    rc = solve_common(m, m->w_lift, u, rtol, maxit, 0, pdt, st, s);
    if (rc < 0) return rc;
    launch_set_boundary(N, g, u, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return rc;
}

int pmg_mlp_nparams(int nout) { return 64 * 3 + 64 + 64 * 64 + 64 + nout * 64 + nout; }

int pmg_mlp_forward(const float* prm, const float* x, float* y, float* cache, int batch, int nout, void* stream) {
    if (!prm || !x || !y || !cache || batch < 0 || nout < 1) return fail(PMG_EINVAL, "bad MLP arguments");
    if (batch == 0) return 0;
    launch_mlp_forward(prm, x, y, cache, batch, nout, S(stream));
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_mlp_loss(const float* y, const float* t, const float* mask, float* dy, float* loss, int batch, int nout,
                 void* stream) {
    if (!y || !t || !mask || !dy || !loss || batch < 0 || nout < 1) return fail(PMG_EINVAL, "bad MLP arguments");
    launch_mlp_loss(y, t, mask, dy, loss, batch * nout, S(stream));
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_mlp_backward(const float* prm, const float* x, const float* cache, const float* dy, float* grad, int batch,
                     int nout, void* stream) {
    if (!prm || !x || !cache || !dy || !grad || batch < 0 || nout < 1) return fail(PMG_EINVAL, "bad MLP arguments");
    // per-sample deltas live in a scratch buffer sized like the cache
    float* work = nullptr;
    size_t bytes = (size_t)std::max(batch, 1) * (128 + nout) * sizeof(float);
    HIPCHK(hipMallocAsync((void**)&work, bytes, S(stream)));
    launch_mlp_backward(prm, x, cache, dy, work, grad, batch, nout, S(stream));
    HIPCHK(hipFreeAsync(work, S(stream)));
    HIPCHK(hipGetLastError());
    return 0;
}

// Allocation-free backward pass: the per-sample deltas go to a fixed device
// array instead of a stream-ordered allocation.  Every call on one GPU uses
// that GPU's copy of the array, so calls that overlap on one GPU race.
constexpr size_t kMlpScratchFloats = size_t(1) << 21;  // 8 MiB per GPU
static __device__ __align__(256) float scratch[kMlpScratchFloats];
static std::mutex g_scratch_mu;
static std::vector<float*> g_scratch_dev;  // device address of `scratch`, per device

// Device address of the current device's `scratch` (looked up once per device).
static int scratch_address(float** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(PMG_EHIP, "hipGetSymbolAddress returned a null address for the MLP scratch");
        g_scratch_dev[dev] = static_cast<float*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return 0;
}

int pmg_mlp_backward_noalloc(const float* prm, const float* x, const float* cache, const float* dy, float* grad,
                             int batch, int nout, void* stream) {
    if (!prm || !x || !cache || !dy || !grad || batch < 0 || nout < 1) return fail(PMG_EINVAL, "bad MLP arguments");
    const size_t need = (size_t)std::max(batch, 1) * (128 + (size_t)nout);
    if (need > kMlpScratchFloats)
        return fail(PMG_EUNSUP, "pmg_mlp_backward_noalloc: batch * (128 + nout) = " + std::to_string(need) +
                                    " floats exceeds the fixed scratch of " + std::to_string(kMlpScratchFloats));
    float* work = nullptr;
    int rc = scratch_address(&work);
    if (rc) return rc;
    // every delta the parameter pass reads is written first by the per-sample
    // pass of the same call, so the scratch needs no clearing
    launch_mlp_backward(prm, x, cache, dy, work, grad, batch, nout, S(stream));
    HIPCHK(hipGetLastError());
    return 0;
}

int pmg_mlp_adam(float* prm, const float* g, float* mm, float* vv, int n, float lr, float b1, float b2, float eps,
                 int t, void* stream) {
    if (!prm || !g || !mm || !vv || n < 0 || t < 1) return fail(PMG_EINVAL, "bad Adam arguments");
    if (n == 0) return 0;
    launch_mlp_adam(prm, g, mm, vv, n, lr, b1, b2, eps, t, S(stream));
    HIPCHK(hipGetLastError());
    return 0;
}

}  // extern "C"
