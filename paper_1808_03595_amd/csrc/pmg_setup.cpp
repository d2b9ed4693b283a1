// Host-side set-up of the 1D tables that drive the kernels.
//
// GLL nodes/weights, the standard stiffness matrix, generalized eigenpairs
// of (L, M) with a diagonal M, Lagrange interpolation and the weight
// polynomial; then the per-level tables of elements (condensed operator,
// Sec. 2.2), stars (Alg. 1, with the identity padding of Sec. 3.3) and the
// transfer matrix (Sec. 4.1).
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <stdexcept>

#include "pmg_internal.h"

namespace pmg {

Layout make_layout(int n1, int n2, int n3, int p, int bc) {
    Layout L{};
    L.p = p;
    L.bc = bc;
    L.n[0] = n1; L.n[1] = n2; L.n[2] = n3;
    for (int d = 0; d < 3; ++d) L.N[d] = L.n[d] * p + 1;
    auto pad = [](int v) { return (v + 3) & ~3; };
    // family 0: [i3][i2]; family 1: [i3][i1]; family 2: [i2][i1]
    L.pitch[0] = pad(L.N[1]); L.rows[0] = L.N[2];
    L.pitch[1] = pad(L.N[0]); L.rows[1] = L.N[2];
    L.pitch[2] = pad(L.N[0]); L.rows[2] = L.N[1];
    int64_t o = 0;
    for (int d = 0; d < 3; ++d) {
        L.pstride[d] = (int64_t)L.rows[d] * L.pitch[d];
        L.pstride[d] = (L.pstride[d] + 63) & ~(int64_t)63;
        L.off[d] = o;
        o += (int64_t)(L.n[d] + 1) * L.pstride[d];
    }
    L.len = o;
    return L;
}

// Legendre P_k(x) for k = 0..n by the three-term recurrence.
static void legendre_all(int n, double x, std::vector<double>& P) {
    P.assign(n + 1, 0.0);
    P[0] = 1.0;
    if (n >= 1) P[1] = x;
    for (int k = 2; k <= n; ++k) P[k] = ((2 * k - 1) * x * P[k - 1] - (k - 1) * P[k - 2]) / k;
}

// GLL nodes are the zeros of P_{p+1} - P_{p-1} (proportional to
// (1 - x^2) P_p'), whose derivative is (2p + 1) P_p.  Newton from the
// Chebyshev-Lobatto points; weights 2 / (p (p + 1) P_p(x)^2).
void gll_nodes_weights(int p, std::vector<double>& x, std::vector<double>& w) {
    x.resize(p + 1);
    w.resize(p + 1);
    std::vector<double> P;
    for (int i = 0; i <= p; ++i) {
        double xi = -std::cos(M_PI * i / p);
        if (i > 0 && i < p) {
            for (int it = 0; it < 100; ++it) {
                legendre_all(p + 1, xi, P);
                double dx = (P[p + 1] - P[p - 1]) / ((2 * p + 1) * P[p]);
                xi -= dx;
                if (std::fabs(dx) < 1e-16) break;
            }
        }
        x[i] = xi;
    }
    x[0] = -1.0;
    x[p] = 1.0;
    for (int i = 0; i <= p; ++i) {
        legendre_all(p, x[i], P);
        w[i] = 2.0 / (p * (p + 1.0) * P[p] * P[p]);
    }
}

// L_S = D^T W D with the closed-form GLL differentiation matrix
// D_ij = P_p(x_i) / (P_p(x_j) (x_i - x_j)), D_00 = -p(p+1)/4, D_pp = p(p+1)/4.
void stiffness_std(int p, const std::vector<double>& x, const std::vector<double>& w,
                   std::vector<double>& L) {
    int n = p + 1;
    std::vector<double> Pp(n), P, D(n * n, 0.0);
    for (int i = 0; i < n; ++i) {
        legendre_all(p, x[i], P);
        Pp[i] = P[p];
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (i != j) D[i * n + j] = Pp[i] / (Pp[j] * (x[i] - x[j]));
    D[0] = -p * (p + 1.0) / 4.0;
    D[n * n - 1] = p * (p + 1.0) / 4.0;
    L.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int q = 0; q < n; ++q) s += D[q * n + i] * w[q] * D[q * n + j];
            L[i * n + j] = s;
        }
}

// Cyclic Jacobi rotations for a symmetric n x n matrix A (destroyed).
// Q[i][k] column k is the eigenvector of lam[k]; ascending order.  The
// rotations run in extended precision (long double; the matrix is given in
// it) and skip an entry once
// it is negligible relative to its two diagonal entries, so that even the
// smallest eigenvalues come out correct to the last FP64 bit at large p
// (their absolute size is ~p^-4 of the largest one).
static void jacobi_ext(int n, std::vector<long double>& A, std::vector<double>& Q_out, std::vector<double>& lam) {
    typedef long double R;
    std::vector<R> Q((size_t)n * n, 0.0L);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0L;
    const R tol = 4.0L * std::numeric_limits<R>::epsilon();
    for (int sweep = 0; sweep < 100; ++sweep) {
        bool rotated = false;
        for (int pq = 0; pq < n; ++pq)
            for (int qq = pq + 1; qq < n; ++qq) {
                const R apq = A[(size_t)pq * n + qq];
                const R app = A[(size_t)pq * n + pq], aqq = A[(size_t)qq * n + qq];
                if (std::fabs(apq) <= tol * std::sqrt(std::fabs(app * aqq))) continue;
                rotated = true;
                const R theta = (aqq - app) / (2.0L * apq);
                const R t = (theta >= 0 ? 1.0L : -1.0L) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0L));
                const R c = 1.0L / std::sqrt(t * t + 1.0L), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const R akp = A[(size_t)k * n + pq], akq = A[(size_t)k * n + qq];
                    A[(size_t)k * n + pq] = c * akp - s * akq;
                    A[(size_t)k * n + qq] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const R apk = A[(size_t)pq * n + k], aqk = A[(size_t)qq * n + k];
                    A[(size_t)pq * n + k] = c * apk - s * aqk;
                    A[(size_t)qq * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const R qkp = Q[(size_t)k * n + pq], qkq = Q[(size_t)k * n + qq];
                    Q[(size_t)k * n + pq] = c * qkp - s * qkq;
                    Q[(size_t)k * n + qq] = s * qkp + c * qkq;
                }
            }
        if (!rotated) break;
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return A[(size_t)a * n + a] < A[(size_t)b * n + b]; });
    Q_out.assign((size_t)n * n, 0.0);
    lam.resize(n);
    for (int k = 0; k < n; ++k) {
        lam[k] = (double)A[(size_t)ord[k] * n + ord[k]];
        for (int i = 0; i < n; ++i) Q_out[(size_t)i * n + k] = (double)Q[(size_t)i * n + ord[k]];
    }
}

void sym_eig_jacobi(int n, std::vector<double>& A_in, std::vector<double>& Q_out, std::vector<double>& lam) {
    std::vector<long double> A(A_in.begin(), A_in.end());
    jacobi_ext(n, A, Q_out, lam);
}

// Generalized eigenpairs of (L, diag(m)): S^T L S = diag(lam), S^T M S = I,
// via the symmetric matrix M^-1/2 L M^-1/2 = Q diag(lam) Q^T, S = M^-1/2 Q
// (scaling and back-scaling in extended precision as well).
void gen_eig_diag(int n, const double* L, const double* m, std::vector<double>& S,
                  std::vector<double>& lam) {
    typedef long double R;
    std::vector<R> ms(n);
    for (int i = 0; i < n; ++i) ms[i] = std::sqrt((R)m[i]);
    std::vector<R> A((size_t)n * n);
    std::vector<double> Q;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = (R)L[(size_t)i * n + j] / (ms[i] * ms[j]);
    jacobi_ext(n, A, Q, lam);
    S.resize((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) S[(size_t)i * n + k] = (double)((R)Q[(size_t)i * n + k] / ms[i]);
}

// J[i][j] = l_j(xt[i]) by the barycentric formula on the nodes xf.
void lagrange_interp(const std::vector<double>& xf, const std::vector<double>& xt,
                     std::vector<double>& J) {
    int nf = (int)xf.size(), nt = (int)xt.size();
    std::vector<double> b(nf, 1.0);
    for (int j = 0; j < nf; ++j)
        for (int k = 0; k < nf; ++k)
            if (k != j) b[j] /= (xf[j] - xf[k]);
    J.assign(nt * nf, 0.0);
    for (int i = 0; i < nt; ++i) {
        int hit = -1;
        for (int j = 0; j < nf; ++j)
            if (xt[i] == xf[j]) hit = j;
        if (hit >= 0) {
            J[i * nf + hit] = 1.0;
            continue;
        }
        double den = 0.0;
        for (int j = 0; j < nf; ++j) den += b[j] / (xt[i] - xf[j]);
        for (int j = 0; j < nf; ++j) J[i * nf + j] = (b[j] / (xt[i] - xf[j])) / den;
    }
}

static double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// Degree-pw (odd) polynomial that is 0 at t = 0, 1 at t = 1 and has its
// first (pw-1)/2 derivatives zero at both ends: the smoothstep polynomial
// S_m(t) = t^(m+1) sum_k C(m+k, k) C(2m+1, m-k) (-t)^k, m = (pw-1)/2.
double smoothstep(int pw, double t) {
    int m = (pw - 1) / 2;
    double s = 0.0;
    for (int k = 0; k <= m; ++k) s += binom(m + k, k) * binom(2 * m + 1, m - k) * std::pow(-t, k);
    return std::pow(t, m + 1) * s;
}

// Element-centred blocks (Sec. 3.4) along one direction: for every element
// e of the widths h, the 1D matrices of elements e-1, e, e+1 assembled on
// positions 0..3p with both ends dropped (n_S = 3p - 1 positions), the
// generalized eigenpairs of the coupled part, identity padding (eigenvalue 1)
// at positions in ghost elements and at Dirichlet boundary vertices
// (Sec. 3.3), and the block's 1D weights.  Weights: the block's distance
// function is q(t)/2 on its left element, 1/2 on the centre and q(1-t)/2 on
// the right element (q the degree-7 weight polynomial, t the element
// reference coordinate); a position's weight is the block's value divided by
// the sum over all blocks of the mesh that cover it, so the weights of the
// covering blocks add up to one.  Outputs padded to np per block: S [e][i][k]
// (np x np), lam [e][np], w [e][np] (zero on padding and ghost positions).
void build_block_tables(int p, const std::vector<double>& h, int np, int bc_d, std::vector<double>& Sout,
                        std::vector<double>& lamout, std::vector<double>& wout) {
    // bc_d: bit 0 Dirichlet low end, bit 1 Dirichlet high end, bit 2 periodic
    const bool per = (bc_d >> 2) & 1, dl = !per && (bc_d & 1), dh = !per && ((bc_d >> 1) & 1);
    std::vector<double> x, w, Ls;
    gll_nodes_weights(p, x, w);
    stiffness_std(p, x, w, Ls);
    const int n1 = p + 1, nS = 3 * p - 1, nb = (int)h.size(), W = 3 * p + 1;
    Sout.assign((size_t)nb * np * np, 0.0);
    lamout.assign((size_t)nb * np, 1.0);
    wout.assign((size_t)nb * np, 0.0);
    // distance function of block b at global position g it covers (in a
    // periodic direction g in 0..nb p - 1 and the neighbours wrap round)
    auto phi = [&](int b, int g) -> double {
        int m = g / p, j = g - m * p;
        if (m >= nb) { m = nb - 1; j = p; }
        const double t = 0.5 * (x[j] + 1.0);
        const int rel = per ? ((m - b) % nb + nb) % nb : m - b;
        if (rel == 0) return 0.5;
        if (rel == -1 || (per && rel == nb - 1)) return 0.5 * smoothstep(7, t);
        if (rel == 1) return 0.5 * smoothstep(7, 1.0 - t);
        return 0.0;
    };
    for (int e = 0; e < nb; ++e) {
        std::vector<double> M(W, 0.0), L((size_t)W * W, 0.0);
        std::vector<char> cpl(W, 0);
        for (int j = 0; j < 3; ++j) {
            int el = e - 1 + j;
            if (per) el = (el + nb) % nb;
            if (el < 0 || el >= nb) continue;
            const double he = h[el];
            for (int a = 0; a < n1; ++a) {
                M[j * p + a] += 0.5 * he * w[a];
                cpl[j * p + a] = 1;
                for (int b = 0; b < n1; ++b) L[(size_t)(j * p + a) * W + j * p + b] += (2.0 / he) * Ls[a * n1 + b];
            }
        }
        if (e == 0 && dl) cpl[p] = 0;            // Dirichlet boundary at the block's left face
        if (e == nb - 1 && dh) cpl[2 * p] = 0;   // Dirichlet boundary at the block's right face
        std::vector<int> c;
        for (int i = 1; i < 3 * p; ++i)
            if (cpl[i]) c.push_back(i);
        double* S = &Sout[(size_t)e * np * np];
        double* lam = &lamout[(size_t)e * np];
        for (int i = 0; i < np; ++i) S[(size_t)i * np + i] = i < nS ? 1.0 : 0.0;
        const int nc = (int)c.size();
        if (nc > 0) {
            std::vector<double> Lc((size_t)nc * nc), mc(nc), Sc, lc;
            for (int a = 0; a < nc; ++a) {
                mc[a] = M[c[a]];
                for (int b = 0; b < nc; ++b) Lc[(size_t)a * nc + b] = L[(size_t)c[a] * W + c[b]];
            }
            gen_eig_diag(nc, Lc.data(), mc.data(), Sc, lc);
            for (int a = 0; a < nc; ++a) {
                lam[c[a] - 1] = lc[a];
                for (int b = 0; b < nc; ++b) S[(size_t)(c[a] - 1) * np + (c[b] - 1)] = Sc[(size_t)a * nc + b];
            }
        }
        for (int o = 0; o < nS; ++o) {
            int g = (e - 1) * p + 1 + o;
            double tot = 0.0;
            if (per) {
                const int P = nb * p;
                g = (g % P + P) % P;
                for (int b = 0; b < nb; ++b) {
                    const int rel = ((g - (b - 1) * p) % P + P) % P;
                    if (rel > 0 && rel < 3 * p) tot += phi(b, g);
                }
            } else {
                if (g < 0 || g > nb * p) continue;
                for (int b = std::max(0, g / p - 2); b <= std::min(nb - 1, g / p + 1); ++b)
                    if ((b - 1) * p < g && g < (b + 2) * p) tot += phi(b, g);
            }
            wout[(size_t)e * np + o] = tot > 0.0 ? phi(e, g) / tot : 0.0;
        }
    }
}

// Exact coarse solve by fast diagonalization of the whole mesh: along one
// direction, the assembled 1D GLL mass (diagonal) and stiffness on the
// n p + 1 nodes, the two Dirichlet end nodes removed, and their generalized
// eigenpairs S^T L S = diag(mu), S^T M S = I.  Outputs (m = n p - 1):
// Af[k][i] = S[i][k] (forward transform), Ab[i][k] = S[i][k] (backward), mu.
void build_fd_tables(int p, const std::vector<double>& h, int bc_d, std::vector<double>& Af,
                     std::vector<double>& Ab, std::vector<double>& mu, int& first) {
    std::vector<double> x, w, Ls;
    gll_nodes_weights(p, x, w);
    stiffness_std(p, x, w, Ls);
    const bool per = (bc_d >> 2) & 1, dl = !per && (bc_d & 1), dh = !per && ((bc_d >> 1) & 1);
    // assembled on the n p + 1 nodes, or on the n p distinct ones of a
    // periodic direction (the last element's end node is node 0)
    const int n = (int)h.size(), N = per ? n * p : n * p + 1, n1 = p + 1;
    std::vector<double> M(N, 0.0), L((size_t)N * N, 0.0);
    for (int e = 0; e < n; ++e)
        for (int a = 0; a < n1; ++a) {
            const int ga = (e * p + a) % N;
            M[ga] += 0.5 * h[e] * w[a];
            for (int b = 0; b < n1; ++b) L[(size_t)ga * N + (e * p + b) % N] += (2.0 / h[e]) * Ls[a * n1 + b];
        }
    first = dl ? 1 : 0;
    const int m = N - (dl ? 1 : 0) - (dh ? 1 : 0);
    std::vector<double> Li((size_t)m * m), Mi(m), S;
    for (int a = 0; a < m; ++a) {
        Mi[a] = M[a + first];
        for (int b = 0; b < m; ++b) Li[(size_t)a * m + b] = L[(size_t)(a + first) * N + b + first];
    }
    gen_eig_diag(m, Li.data(), Mi.data(), S, mu);
    Af.assign((size_t)m * m, 0.0);
    Ab.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i)
        for (int k = 0; k < m; ++k) {
            Af[(size_t)k * m + i] = S[(size_t)i * m + k];
            Ab[(size_t)i * m + k] = S[(size_t)i * m + k];
        }
}

void build_level_tables(int p, int pc, const std::vector<double> h[3], HostTables& t, int bc) {
    std::vector<double> x, w, Ls;
    gll_nodes_weights(p, x, w);
    stiffness_std(p, x, w, Ls);
    const int n1 = p + 1, q = p - 1, nS = 2 * p - 1;
    for (int d = 0; d < 3; ++d) {
        const int ne = (int)h[d].size();
        t.el_m[d].clear(); t.el_L[d].clear(); t.el_Sinv[d].clear(); t.el_MS[d].clear();
        t.el_lam[d].clear(); t.el_c0[d].clear(); t.el_cp[d].clear();
        t.st_S[d].clear(); t.st_lam[d].clear();
        for (int e = 0; e < ne; ++e) {
            double he = h[d][e];
            std::vector<double> m(n1), L(n1 * n1);
            for (int i = 0; i < n1; ++i) m[i] = 0.5 * he * w[i];
            for (int i = 0; i < n1 * n1; ++i) L[i] = (2.0 / he) * Ls[i];
            t.el_m[d].insert(t.el_m[d].end(), m.begin(), m.end());
            t.el_L[d].insert(t.el_L[d].end(), L.begin(), L.end());
            if (q >= 1) {
                std::vector<double> LI(q * q), mI(q), S, lam;
                for (int i = 0; i < q; ++i) {
                    mI[i] = m[i + 1];
                    for (int j = 0; j < q; ++j) LI[i * q + j] = L[(i + 1) * n1 + (j + 1)];
                }
                gen_eig_diag(q, LI.data(), mI.data(), S, lam);
                for (int k = 0; k < q; ++k)
                    for (int i = 0; i < q; ++i) t.el_Sinv[d].push_back(S[i * q + k] * mI[i]);
                for (int i = 0; i < q; ++i)
                    for (int k = 0; k < q; ++k) t.el_MS[d].push_back(mI[i] * S[i * q + k]);
                t.el_lam[d].insert(t.el_lam[d].end(), lam.begin(), lam.end());
                for (int k = 0; k < q; ++k) {
                    double c0 = 0.0, cp = 0.0;
                    for (int i = 0; i < q; ++i) {
                        c0 += S[i * q + k] * L[(i + 1) * n1 + 0];
                        cp += S[i * q + k] * L[(i + 1) * n1 + p];
                    }
                    t.el_c0[d].push_back(c0);
                    t.el_cp[d].push_back(cp);
                }
            }
        }
        // stars: block positions -p..p -> 0..2p; keep 1..2p-1.  Sec. 3.3: an
        // element outside the domain is decoupled (identity), and so is a
        // Dirichlet vertex; a Neumann vertex stays coupled; in a periodic
        // direction the element before vertex 0 is the last one (the star of
        // vertex ne duplicates it and is never used)
        const bool per = (bc >> (6 + d)) & 1;
        const bool dlo = !per && ((bc >> d) & 1), dhi = !per && ((bc >> (3 + d)) & 1);
        for (int v = 0; v <= ne; ++v) {
            std::vector<double> M(2 * p + 1, 0.0), L((2 * p + 1) * (2 * p + 1), 0.0);
            std::vector<char> cpl(2 * p + 1, 0);
            auto add_el = [&](int e, int base) {
                double he = h[d][e];
                for (int i = 0; i < n1; ++i) {
                    M[base + i] += 0.5 * he * w[i];
                    cpl[base + i] = 1;
                    for (int j = 0; j < n1; ++j)
                        L[(base + i) * (2 * p + 1) + base + j] += (2.0 / he) * Ls[i * n1 + j];
                }
            };
            if (v >= 1) add_el(v - 1, 0);
            else if (per) add_el(ne - 1, 0);
            if (v <= ne - 1) add_el(v, p);
            if ((v == 0 && dlo) || (v == ne && dhi)) cpl[p] = 0;
            std::vector<int> c;
            for (int i = 1; i < 2 * p; ++i)
                if (cpl[i]) c.push_back(i);
            std::vector<double> S(nS * nS, 0.0), lam(nS, 1.0);
            for (int i = 0; i < nS; ++i) S[i * nS + i] = 1.0;
            int nc = (int)c.size();
            if (nc > 0) {
                std::vector<double> Lc(nc * nc), mc(nc), Sc, lc;
                for (int a = 0; a < nc; ++a) {
                    mc[a] = M[c[a]];
                    for (int b = 0; b < nc; ++b) Lc[a * nc + b] = L[c[a] * (2 * p + 1) + c[b]];
                }
                gen_eig_diag(nc, Lc.data(), mc.data(), Sc, lc);
                for (int a = 0; a < nc; ++a) {
                    lam[c[a] - 1] = lc[a];
                    for (int b = 0; b < nc; ++b) S[(c[a] - 1) * nS + (c[b] - 1)] = Sc[a * nc + b];
                }
            }
            t.st_S[d].insert(t.st_S[d].end(), S.begin(), S.end());
            t.st_lam[d].insert(t.st_lam[d].end(), lam.begin(), lam.end());
        }
    }
    // weights at offsets -(p-1)..(p-1): t = (1 - x_|j|) / 2
    t.st_w.resize(nS);
    for (int j = -(p - 1); j <= p - 1; ++j) t.st_w[j + p - 1] = smoothstep(7, (1.0 - x[std::abs(j)]) / 2.0);
    // copies padded to np = 16 ceil(nS / 16) for the matrix-core smoothers
    const int np = 16 * ((nS + 15) / 16);
    t.np = np;
    for (int d = 0; d < 3; ++d) {
        const int nv = (int)h[d].size() + 1;
        t.st_SP[d].assign((size_t)nv * np * np, 0.0);
        t.st_lamP[d].assign((size_t)nv * np, 1.0);
        for (int v = 0; v < nv; ++v)
            for (int i = 0; i < nS; ++i) {
                t.st_lamP[d][(size_t)v * np + i] = t.st_lam[d][(size_t)v * nS + i];
                for (int k = 0; k < nS; ++k)
                    t.st_SP[d][((size_t)v * np + i) * np + k] = t.st_S[d][(size_t)v * nS * nS + i * nS + k];
            }
    }
    t.st_wP.assign(np, 0.0);
    for (int i = 0; i < nS; ++i) t.st_wP[i] = t.st_w[i];
    t.J.clear();
    if (pc > 0) {
        std::vector<double> xc, wc;
        gll_nodes_weights(pc, xc, wc);
        lagrange_interp(xc, x, t.J);
    }
    // p <= 2: the assembled 1D mass (diagonal) and stiffness (band of
    // half-width p) per direction, one record per global node index
    for (int d = 0; d < 3; ++d) {
        t.ax[d].clear();
        if (p > 2) continue;
        const int ne = (int)h[d].size(), N = ne * p + 1;
        t.ax[d].assign((size_t)N * AXW, 0.0);
        for (int e = 0; e < ne; ++e)
            for (int a = 0; a < n1; ++a) {
                double* rec = &t.ax[d][(size_t)(e * p + a) * AXW];
                rec[0] += t.el_m[d][(size_t)e * n1 + a];
                for (int b = 0; b < n1; ++b) rec[1 + p + (b - a)] += t.el_L[d][(size_t)e * n1 * n1 + a * n1 + b];
            }
    }
}

// Diagonal of the assembled condensed operator on a level, stored in the
// plane layout (1 at unused slots).  Per element: diagonal of H_e at the
// shell nodes minus, at face-interior nodes, the Schur term
// sum_k (c_{d,s}[k_d] Sinv[k'][a'] Sinv[k''][a''])^2 / D[k].
void coarse_diagonal(const Layout& lay, double lam, const std::vector<double> h[3],
                     std::vector<double>& diag) {
    const int p = lay.p, n1 = p + 1, q = p - 1;
    HostTables t;
    build_level_tables(p, 0, h, t);
    diag.assign(lay.len, 0.0);
    std::vector<char> used(lay.len, 0);
    for (int e3 = 0; e3 < lay.n[2]; ++e3)
        for (int e2 = 0; e2 < lay.n[1]; ++e2)
            for (int e1 = 0; e1 < lay.n[0]; ++e1) {
                const int e[3] = {e1, e2, e3};
                const double* m[3];
                const double* L[3];
                const double *Si[3], *lm[3], *c0[3], *cp[3];
                for (int d = 0; d < 3; ++d) {
                    m[d] = &t.el_m[d][e[d] * n1];
                    L[d] = &t.el_L[d][e[d] * n1 * n1];
                    Si[d] = q ? &t.el_Sinv[d][e[d] * q * q] : nullptr;
                    lm[d] = q ? &t.el_lam[d][e[d] * q] : nullptr;
                    c0[d] = q ? &t.el_c0[d][e[d] * q] : nullptr;
                    cp[d] = q ? &t.el_cp[d][e[d] * q] : nullptr;
                }
                for (int a3 = 0; a3 <= p; ++a3)
                    for (int a2 = 0; a2 <= p; ++a2)
                        for (int a1 = 0; a1 <= p; ++a1) {
                            const int a[3] = {a1, a2, a3};
                            bool on[3];
                            int non = 0;
                            for (int d = 0; d < 3; ++d) {
                                on[d] = (a[d] == 0 || a[d] == p);
                                non += on[d];
                            }
                            if (!non) continue;
                            const int g1 = e1 * p + a1, g2 = e2 * p + a2, g3 = e3 * p + a3;
                            if (g1 == 0 || g2 == 0 || g3 == 0 || g1 == lay.N[0] - 1 ||
                                g2 == lay.N[1] - 1 || g3 == lay.N[2] - 1)
                                continue;
                            double v = lam * m[0][a1] * m[1][a2] * m[2][a3] +
                                       m[2][a3] * m[1][a2] * L[0][a1 * n1 + a1] +
                                       m[2][a3] * m[0][a1] * L[1][a2 * n1 + a2] +
                                       m[1][a2] * m[0][a1] * L[2][a3 * n1 + a3];
                            if (non == 1 && q > 0) {
                                int dn = on[0] ? 0 : (on[1] ? 1 : 2);
                                const double* c = (a[dn] == 0) ? c0[dn] : cp[dn];
                                int da = (dn == 0) ? 1 : 0, db = (dn == 2) ? 1 : 2;
                                double s = 0.0;
                                for (int k3 = 0; k3 < q; ++k3)
                                    for (int k2 = 0; k2 < q; ++k2)
                                        for (int k1 = 0; k1 < q; ++k1) {
                                            const int k[3] = {k1, k2, k3};
                                            double g = c[k[dn]] * Si[da][k[da] * q + (a[da] - 1)] *
                                                       Si[db][k[db] * q + (a[db] - 1)];
                                            double D = lam + lm[0][k1] + lm[1][k2] + lm[2][k3];
                                            s += g * g / D;
                                        }
                                v -= s;
                            }
                            int64_t sl = lay.slot(g1, g2, g3, on[0], !on[0] && on[1]);
                            diag[sl] += v;
                            used[sl] = 1;
                        }
            }
    for (int64_t i = 0; i < lay.len; ++i)
        if (!used[i]) diag[i] = 1.0;
}

}  // namespace pmg
