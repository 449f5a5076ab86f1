// Host-side set-up of the direct RZ Poisson solve for geometries in which
// the finite-volume operator separates (Eqs. poisson and epseff with chi = 0
// when the permittivity depends on z only): eigenvectors of the radial
// operator, per-mode tridiagonal factors in z, and the capacitance system
// that imposes Dirichlet values on nodes inside the rectangular block of
// unknowns (the coil turns).
#pragma once
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace pic {

// Eigenvalues and orthonormal eigenvectors of the symmetric tridiagonal
// matrix with diagonal d[0..n-1] and off-diagonal e[0..n-2], by the
// implicit QL iteration with shifts taken from the trailing 2x2 block of
// the active window (Bowdler, Martin, Reinsch and Wilkinson's method).
// On return d holds the eigenvalues and q[r * n + c] the component r of
// eigenvector c.  Returns false if an eigenvalue needs more than 60 sweeps.
inline bool tridiagonal_eigen(std::vector<double> &d, std::vector<double> e, std::vector<double> &q)
{
    const int n = (int)d.size();
    q.assign((size_t)n * n, 0.0);
    for (int r = 0; r < n; ++r) q[(size_t)r * n + r] = 1.0;
    e.resize(n, 0.0);   // e[n-1] = 0 closes the matrix
    for (int lo = 0; lo < n; ++lo) {
        for (int sweep = 0;; ++sweep) {
            // the window [lo, hi] ends at the first negligible off-diagonal
            int hi = lo;
            while (hi < n - 1) {
                const double scale = std::fabs(d[hi]) + std::fabs(d[hi + 1]);
                if (std::fabs(e[hi]) + scale == scale) break;   // below half an ulp of the diagonal
                ++hi;
            }
            if (hi == lo) break;
            if (sweep == 60) return false;
            // shift: the eigenvalue of the leading 2x2 block nearer d[lo]
            const double g0 = (d[lo + 1] - d[lo]) / (2.0 * e[lo]);
            const double rr = std::hypot(g0, 1.0);
            double g = d[hi] - d[lo] + e[lo] / (g0 + (g0 >= 0.0 ? rr : -rr));
            double s = 1.0, c = 1.0, p = 0.0;
            bool early = false;
            // chase the bulge from the bottom of the window to its top
            for (int i = hi - 1; i >= lo; --i) {
                const double f = s * e[i], b = c * e[i];
                const double r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {   // the rotation splits the window
                    d[i + 1] -= p;
                    e[hi] = 0.0;
                    early = true;
                    break;
                }
                s = f / r;
                c = g / r;
                const double t = d[i + 1] - p;
                const double u = (d[i] - t) * s + 2.0 * c * b;
                p = s * u;
                d[i + 1] = t + p;
                g = c * u - b;
                for (int k = 0; k < n; ++k) {
                    const double a0 = q[(size_t)k * n + i], a1 = q[(size_t)k * n + i + 1];
                    q[(size_t)k * n + i + 1] = s * a0 + c * a1;
                    q[(size_t)k * n + i] = c * a0 - s * a1;
                }
            }
            if (early) continue;
            d[lo] -= p;
            e[lo] = g;
            e[hi] = 0.0;
        }
    }
    return true;
}

// Inverse of a symmetric positive definite matrix (row-major m x m) by
// Gauss-Jordan elimination without pivoting.  Returns false if a pivot is
// not positive.
inline bool spd_inverse(std::vector<double> a, int m, std::vector<double> &inv)
{
    inv.assign((size_t)m * m, 0.0);
    for (int r = 0; r < m; ++r) inv[(size_t)r * m + r] = 1.0;
    for (int p = 0; p < m; ++p) {
        const double piv = a[(size_t)p * m + p];
        if (!(piv > 0.0)) return false;
        const double ip = 1.0 / piv;
        for (int c = 0; c < m; ++c) {
            a[(size_t)p * m + c] *= ip;
            inv[(size_t)p * m + c] *= ip;
        }
        for (int r = 0; r < m; ++r) {
            if (r == p) continue;
            const double f = a[(size_t)r * m + p];
            if (f == 0.0) continue;
            for (int c = 0; c < m; ++c) {
                a[(size_t)r * m + c] -= f * a[(size_t)p * m + c];
                inv[(size_t)r * m + c] -= f * inv[(size_t)p * m + c];
            }
        }
    }
    return true;
}

constexpr int DP_MAX_DIRICHLET = 512;   // interior Dirichlet nodes the capacitance system takes
constexpr int DP_MAX_ROWS = 16;          // distinct block rows holding them
constexpr int DP_MAX_NI = 1024;          // block rows (the per-mode solve keeps 8 arrays of them in LDS)

// The block of unknowns is rows i = 1..nz-1 and columns j = 0..nr-1 of the
// node grid; every node outside it is Dirichlet.  On the block the operator
// is A = Z (x) L_R + L_Z (x) D: radial conductances Z_i b_j, axial
// conductances e_i D_j.  With D-orthonormal eigenvectors V of L_R
// (L_R V = D V diag(lambda), V^T D V = I) the transformed unknowns u = V^T
// D x solve one tridiagonal system per mode k: T_k u_k = (V^T b)_k with
// T_k = lambda_k Z + L_Z.  Nodes inside the block that are Dirichlet take
// their values through sources s on them: x = S (b + E s) with
// S = A^{-1}, s = C^{-1} (phi_D - (S b)_D) and C = S_DD; in the transformed
// unknowns the sources add sum_q g_q(k) w_q(k), g_q = T_k^{-1} e_{rows[q]}.
struct SeparablePlan {
    int ni = 0, nj = 0;             // block rows and columns
    std::vector<double> v;          // V, nj x nj: v[j * nj + k]
    std::vector<double> lam;        // nj eigenvalues
    std::vector<double> zrow;       // ni: Z of block row r (node row r + 1)
    std::vector<double> erow;       // ni + 1: axial coupling e of node rows r and r + 1
    int m = 0;                      // interior Dirichlet nodes
    std::vector<int32_t> dnode;     // their node indices
    std::vector<int32_t> drow;      // index into rows
    std::vector<int32_t> rows;      // distinct block rows that hold interior Dirichlet nodes (ascending)
    std::vector<double> cinv;       // m x m inverse of the capacitance matrix
    std::vector<double> g;          // rows x ni x nj: g[(q * ni + r) * nj + k] = (T_k^{-1} e_{rows[q]})_r
};

// Interior Dirichlet nodes and the distinct block rows holding them.
inline void interior_dirichlet(const std::vector<int32_t> &tag, int nr, int nz, int &m, int &nrow)
{
    m = nrow = 0;
    for (int i = 1; i < nz; ++i) {
        bool any = false;
        for (int j = 0; j < nr; ++j)
            if (tag[(size_t)i * (nr + 1) + j] >= 0) {
                ++m;
                any = true;
            }
        nrow += any;
    }
}

// Builds the plan from the level-0 conductances (cw, ce, cs, cn, cc per
// node) and the Dirichlet tags (tag >= 0); returns an empty string on
// success, else why the direct solve does not apply.
inline std::string plan_separable(const std::vector<double> &cw, const std::vector<double> &ce,
                                  const std::vector<double> &cs, const std::vector<double> &cn,
                                  const std::vector<double> &cc, const std::vector<int32_t> &tag, int nr, int nz,
                                  SeparablePlan &p)
{
    const int nr1 = nr + 1;
    if (nr < 2 || nz < 3) return "grid too small";
    if (nz - 1 > DP_MAX_NI) return "more than 1024 rows of unknowns";
    auto node = [&](int i, int j) { return (size_t)i * nr1 + j; };
    for (int j = 0; j <= nr; ++j)
        if (tag[node(0, j)] < 0 || tag[node(nz, j)] < 0) return "a free node on the bottom or top row";
    for (int i = 0; i <= nz; ++i)
        if (tag[node(i, nr)] < 0) return "a free node on the outer radius";
    {
        int m, nrow;
        interior_dirichlet(tag, nr, nz, m, nrow);
        if (m > DP_MAX_DIRICHLET) return "more than 512 Dirichlet nodes inside the block";
        if (nrow > DP_MAX_ROWS) return "Dirichlet nodes inside the block on more than 16 rows";
    }
    const int ni = nz - 1, nj = nr;
    // factors: b_j = ce(1, j), Z_i = ce(i, 0) / b_0; D_j = cn(1, j), e_i = cn(i, 0) / D_0
    std::vector<double> b(nj), Z(nz + 1), D(nj), e(nz);
    for (int j = 0; j < nj; ++j) {
        b[j] = ce[node(1, j)];
        D[j] = cn[node(1, j)];
        if (!(b[j] > 0.0) || !(D[j] > 0.0)) return "a non-positive conductance";
    }
    for (int i = 1; i < nz; ++i) Z[i] = ce[node(i, 0)] / b[0];
    for (int i = 0; i < nz; ++i) e[i] = cn[node(i, 0)] / D[0];
    const double tol = 1e-13;
    auto close = [&](double a, double ref) { return std::fabs(a - ref) <= tol * std::fabs(ref); };
    for (int i = 1; i < nz; ++i)
        for (int j = 0; j < nj; ++j) {
            const size_t n = node(i, j);
            const double bw = j > 0 ? b[j - 1] : 0.0;
            if (!close(ce[n], Z[i] * b[j]) || !(j > 0 ? close(cw[n], Z[i] * bw) : cw[n] == 0.0) ||
                !close(cn[n], e[i] * D[j]) || !close(cs[n], e[i - 1] * D[j]) ||
                !close(cc[n], Z[i] * (bw + b[j]) + D[j] * (e[i - 1] + e[i])))
                return "the permittivity varies within a row of cells";
        }
    // radial modes: M = D^{-1/2} L_R D^{-1/2}, V = D^{-1/2} Q
    std::vector<double> dg(nj), off(nj > 1 ? nj - 1 : 0), Q;
    for (int j = 0; j < nj; ++j) dg[j] = ((j > 0 ? b[j - 1] : 0.0) + b[j]) / D[j];
    for (int j = 0; j + 1 < nj; ++j) off[j] = -b[j] / std::sqrt(D[j] * D[j + 1]);
    if (!tridiagonal_eigen(dg, off, Q)) return "radial eigen-decomposition did not converge";
    p.ni = ni;
    p.nj = nj;
    p.lam = dg;
    for (int k = 0; k < nj; ++k)
        if (!(p.lam[k] > 0.0)) return "radial operator not definite";
    p.v.assign((size_t)nj * nj, 0.0);
    for (int j = 0; j < nj; ++j)
        for (int k = 0; k < nj; ++k) p.v[(size_t)j * nj + k] = Q[(size_t)j * nj + k] / std::sqrt(D[j]);
    p.zrow.assign(ni, 0.0);
    p.erow.assign(ni + 1, 0.0);
    for (int r = 0; r < ni; ++r) p.zrow[r] = Z[r + 1];
    for (int r = 0; r <= ni; ++r) p.erow[r] = e[r];
    // interior Dirichlet nodes
    p.dnode.clear();
    p.drow.clear();
    p.rows.clear();
    std::vector<int32_t> dcol;
    for (int r = 0; r < ni; ++r)
        for (int j = 0; j < nj; ++j) {
            const size_t n = node(r + 1, j);
            if (tag[n] < 0) continue;
            if (p.rows.empty() || p.rows.back() != r) p.rows.push_back(r);
            p.dnode.push_back((int32_t)n);
            p.drow.push_back((int32_t)p.rows.size() - 1);
            dcol.push_back(j);
        }
    p.m = (int)p.dnode.size();
    p.cinv.clear();
    p.g.clear();
    if (p.m == 0) return "";
    const int nrow = (int)p.rows.size();
    // g_q for every mode by the Thomas algorithm (T_k is diagonally dominant)
    p.g.assign((size_t)nrow * ni * nj, 0.0);
    std::vector<double> y(ni), cpr(ni), ivr(ni);
    for (int k = 0; k < nj; ++k) {
        for (int r = 0; r < ni; ++r) {
            const double diag = p.lam[k] * p.zrow[r] + p.erow[r] + p.erow[r + 1];
            // sub-diagonal -erow[r]: w = diag - (-erow[r]) cp_{r-1}
            const double w = diag + (r > 0 ? p.erow[r] * cpr[r - 1] : 0.0);
            ivr[r] = 1.0 / w;
            cpr[r] = r + 1 < ni ? -p.erow[r + 1] * ivr[r] : 0.0;
        }
        for (int q = 0; q < nrow; ++q) {
            double prev = 0.0;
            for (int r = 0; r < ni; ++r) {
                const double rhs = r == p.rows[q] ? 1.0 : 0.0;
                prev = (rhs + (r > 0 ? p.erow[r] * prev : 0.0)) * ivr[r];
                y[r] = prev;
            }
            for (int r = ni - 2; r >= 0; --r) y[r] -= cpr[r] * y[r + 1];
            for (int r = 0; r < ni; ++r) p.g[((size_t)q * ni + r) * nj + k] = y[r];
        }
    }
    // C(a, c) = sum_k V(j_a, k) V(j_c, k) g_{row(c)}(k)_{row(a)}
    std::vector<double> C((size_t)p.m * p.m, 0.0);
    for (int a = 0; a < p.m; ++a)
        for (int c = 0; c < p.m; ++c) {
            const int ra = p.rows[p.drow[a]];
            double s = 0.0;
            for (int k = 0; k < nj; ++k)
                s += p.v[(size_t)dcol[a] * nj + k] * p.v[(size_t)dcol[c] * nj + k] *
                     p.g[((size_t)p.drow[c] * ni + ra) * nj + k];
            C[(size_t)a * p.m + c] = s;
        }
    // symmetrise the rounding
    for (int a = 0; a < p.m; ++a)
        for (int c = 0; c < a; ++c) {
            const double s = 0.5 * (C[(size_t)a * p.m + c] + C[(size_t)c * p.m + a]);
            C[(size_t)a * p.m + c] = C[(size_t)c * p.m + a] = s;
        }
    if (!spd_inverse(C, p.m, p.cinv)) return "capacitance matrix not definite";
    return "";
}

}  // namespace pic
