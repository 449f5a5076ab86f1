// Host check of the direct Poisson solve's set-up (separable.h), run by
// tests/test_separable_host.py on the CPU:
//   separable_check laplace N      -- eigenvalues and orthogonality of the
//       1-D Dirichlet Laplacian (diagonal 2, off-diagonal -1) against
//       lambda_k = 2 - 2 cos(k pi / (N + 1));
//   separable_check coil NR NZ [perturb] -- the coil-cell geometry (quartz
//       window, five turns inside the block): plan, then the solve as the
//       GPU runs it (transform, per-mode parallel cyclic reduction,
//       capacitance sources through the unit responses, back transform)
//       for a seeded random charge and the turn potentials, and the
//       relative residual of the 5-point operator on the free nodes and the
//       mismatch at the turn nodes; with "perturb" one cell's permittivity
//       differs and the plan must refuse.
#include <cstdio>
#include <random>
#include "../paper_2609_15043_amd/csrc/separable.h"
using namespace pic;
static const double TWO_PI = 6.283185307179586;
struct Coeffs { std::vector<double> cw, ce, cs, cn, cc; };
static Coeffs assemble(int nr, int nz, double dr, double dz, const std::vector<double> &eps, double eps0)
{
    const int nr1 = nr + 1, nodes = (nz + 1) * nr1;
    Coeffs c;
    c.cw.assign(nodes, 0.0); c.ce.assign(nodes, 0.0); c.cs.assign(nodes, 0.0); c.cn.assign(nodes, 0.0); c.cc.assign(nodes, 0.0);
    auto cell_eps = [&](int i, int j, double &sum, int &cnt) {
        if (i >= 0 && i < nz && j >= 0 && j < nr) { sum += eps[(size_t)i * nr + j]; ++cnt; }
    };
    for (int i = 0; i <= nz; ++i)
        for (int j = 0; j <= nr; ++j) {
            const int n = i * nr1 + j; const double R = j * dr;
            if (j < nr) {
                const double h = std::min((double)nz * dz, i * dz + 0.5 * dz) - std::max(0.0, i * dz - 0.5 * dz);
                const double area = TWO_PI * (R + 0.5 * dr) * h;
                double s = 0.0; int k = 0; cell_eps(i - 1, j, s, k); cell_eps(i, j, s, k);
                const double cf = eps0 * (s / k) * area / dr; c.ce[n] = cf; c.cw[n + 1] = cf;
            }
            if (i < nz) {
                const double lo = std::max(0.0, R - 0.5 * dr), hi = std::min((double)nr * dr, R + 0.5 * dr);
                const double area = 0.5 * TWO_PI * (hi * hi - lo * lo);
                double s = 0.0; int k = 0; cell_eps(i, j - 1, s, k); cell_eps(i, j, s, k);
                const double cf = eps0 * (s / k) * area / dz; c.cn[n] = cf; c.cs[n + nr1] = cf;
            }
        }
    for (int n = 0; n < nodes; ++n) c.cc[n] = c.cw[n] + c.ce[n] + c.cs[n] + c.cn[n];
    return c;
}
static void pcr(int ni, double lam, const SeparablePlan &p, std::vector<double> &d)
{
    std::vector<double> A(ni), B(ni), C(ni), A1(ni), B1(ni), C1(ni), D1(ni);
    for (int r = 0; r < ni; ++r) {
        A[r] = r > 0 ? -p.erow[r] : 0.0; C[r] = r + 1 < ni ? -p.erow[r + 1] : 0.0;
        B[r] = lam * p.zrow[r] + p.erow[r] + p.erow[r + 1];
    }
    for (int s = 1; s < ni; s <<= 1) {
        for (int r = 0; r < ni; ++r) {
            double an = 0, cn = 0, bn = B[r], dn = d[r];
            if (r - s >= 0) { const double al = -A[r] / B[r - s]; an = al * A[r - s]; bn += al * C[r - s]; dn += al * d[r - s]; }
            if (r + s < ni) { const double ga = -C[r] / B[r + s]; cn = ga * C[r + s]; bn += ga * A[r + s]; dn += ga * d[r + s]; }
            A1[r] = an; B1[r] = bn; C1[r] = cn; D1[r] = dn;
        }
        A.swap(A1); B.swap(B1); C.swap(C1); d.swap(D1);
    }
    for (int r = 0; r < ni; ++r) d[r] /= B[r];
}
static int laplace(int n)
{
    std::vector<double> d(n, 2.0), e(n - 1, -1.0), q;
    if (!tridiagonal_eigen(d, e, q)) { printf("no convergence\n"); return 1; }
    std::sort(d.begin(), d.end());
    double err = 0.0, orth = 0.0;
    for (int k = 0; k < n; ++k) err = std::max(err, std::fabs(d[k] - (2.0 - 2.0 * std::cos((k + 1) * M_PI / (n + 1)))));
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            double s = 0.0;
            for (int r = 0; r < n; ++r) s += q[(size_t)r * n + a] * q[(size_t)r * n + b];
            orth = std::max(orth, std::fabs(s - (a == b ? 1.0 : 0.0)));
        }
    printf("eigen_err %.3e orth %.3e\n", err, orth);
    return 0;
}
int main(int argc, char **argv)
{
    if (std::string(argv[1]) == "laplace") return laplace(atoi(argv[2]));
    const int nr = atoi(argv[2]), nz = atoi(argv[3]);
    const bool perturb = argc > 4 && std::string(argv[4]) == "perturb";
    const double rmax = 0.15, zmax = 0.2, dr = rmax / nr, dz = zmax / nz;
    const int ip = (int)std::lround(0.15 / dz), iw = (int)std::lround((0.15 + 13 * 0.2 / 256) / dz);
    std::vector<double> eps((size_t)nz * nr, 1.0);
    for (int i = ip; i < iw; ++i) for (int j = 0; j < nr; ++j) eps[(size_t)i * nr + j] = 3.8;
    if (perturb) eps[(size_t)(nz / 3) * nr + nr / 2] = 2.0;
    const int nr1 = nr + 1, nodes = (nz + 1) * nr1;
    std::vector<int32_t> tag(nodes, -1);
    for (int j = 0; j <= nr; ++j) { tag[j] = 0; tag[(size_t)nz * nr1 + j] = 0; }
    for (int i = 0; i <= nz; ++i) tag[(size_t)i * nr1 + nr] = 0;
    const double zc = 213 * (0.2 / 256);
    for (int k = 1; k <= 5; ++k) {
        const double r0 = 17 * k * (0.15 / 128);
        for (int i = 0; i <= nz; ++i) for (int j = 0; j <= nr; ++j)
            if (std::fabs(j * dr - r0) <= 1.2e-3 + 1e-12 && std::fabs(i * dz - zc) <= 0.8e-3 + 1e-12) tag[(size_t)i * nr1 + j] = k;
    }
    Coeffs co = assemble(nr, nz, dr, dz, eps, 8.8541878128e-12);
    SeparablePlan p;
    std::string why = plan_separable(co.cw, co.ce, co.cs, co.cn, co.cc, tag, nr, nz, p);
    printf("plan '%s' ni %d nj %d m %d rows %zu\n", why.c_str(), p.ni, p.nj, p.m, p.rows.size());
    if (!why.empty()) return 0;
    const int ni = p.ni, nj = p.nj;
    std::mt19937_64 rng(5);
    std::uniform_real_distribution<double> U(-1, 1);
    std::vector<double> Q(nodes), phi(nodes, 0.0), phiD(nodes, 0.0);
    for (int n = 0; n < nodes; ++n) Q[n] = tag[n] < 0 ? 1e-12 * U(rng) : 0.0;
    const double vt[5] = {300, 240, 180, 120, 60};
    for (int n = 0; n < nodes; ++n) if (tag[n] >= 1) phiD[n] = vt[tag[n] - 1];
    std::vector<double> B((size_t)ni * nj), Uu((size_t)ni * nj);
    for (int r = 0; r < ni; ++r) for (int j = 0; j < nj; ++j) {
        const int i = r + 1; const size_t n = (size_t)i * nr1 + j;
        double b = tag[n] >= 0 ? 0.0 : Q[n];
        if (tag[n] < 0) {
            if (i == 1) b += co.cs[n] * phiD[n - nr1];
            if (i == nz - 1) b += co.cn[n] * phiD[n + nr1];
            if (j == nr - 1) b += co.ce[n] * phiD[n + 1];
        }
        B[(size_t)r * nj + j] = b;
    }
    for (int r = 0; r < ni; ++r) for (int k = 0; k < nj; ++k) {
        double s = 0; for (int j = 0; j < nj; ++j) s += B[(size_t)r * nj + j] * p.v[(size_t)j * nj + k];
        Uu[(size_t)r * nj + k] = s;
    }
    std::vector<double> col(ni);
    for (int k = 0; k < nj; ++k) {
        for (int r = 0; r < ni; ++r) col[r] = Uu[(size_t)r * nj + k];
        pcr(ni, p.lam[k], p, col);
        for (int r = 0; r < ni; ++r) Uu[(size_t)r * nj + k] = col[r];
    }
    if (p.m) {
        const int nrow = (int)p.rows.size();
        std::vector<double> res(p.m), s(p.m, 0.0), W((size_t)nrow * nj, 0.0);
        for (int a = 0; a < p.m; ++a) {
            const int n = p.dnode[a], i = n / nr1, j = n - i * nr1, r = i - 1;
            double x = 0; for (int k = 0; k < nj; ++k) x += p.v[(size_t)j * nj + k] * Uu[(size_t)r * nj + k];
            res[a] = phiD[n] - x;
        }
        for (int a = 0; a < p.m; ++a) for (int c = 0; c < p.m; ++c) s[a] += p.cinv[(size_t)a * p.m + c] * res[c];
        for (int a = 0; a < p.m; ++a) {
            const int n = p.dnode[a], j = n - (n / nr1) * nr1;
            for (int k = 0; k < nj; ++k) W[(size_t)p.drow[a] * nj + k] += s[a] * p.v[(size_t)j * nj + k];
        }
        for (int r = 0; r < ni; ++r) for (int k = 0; k < nj; ++k) {
            double d = 0; for (int q = 0; q < nrow; ++q) d += p.g[((size_t)q * ni + r) * nj + k] * W[(size_t)q * nj + k];
            Uu[(size_t)r * nj + k] += d;
        }
    }
    for (int n = 0; n < nodes; ++n) phi[n] = phiD[n];
    double dmis = 0;
    for (int r = 0; r < ni; ++r) for (int j = 0; j < nj; ++j) {
        const size_t n = (size_t)(r + 1) * nr1 + j;
        double x = 0; for (int k = 0; k < nj; ++k) x += Uu[(size_t)r * nj + k] * p.v[(size_t)j * nj + k];
        if (tag[n] >= 0) { dmis = std::max(dmis, std::fabs(x - phiD[n]) / 300.0); continue; }
        phi[n] = x;
    }
    double rmax_ = 0, scale = 0;
    for (int i = 1; i < nz; ++i) for (int j = 0; j < nr; ++j) {
        const size_t n = (size_t)i * nr1 + j;
        if (tag[n] >= 0) continue;
        double Ax = co.cc[n] * phi[n] - (j > 0 ? co.cw[n] * phi[n - 1] : 0) - co.ce[n] * phi[n + 1] - co.cs[n] * phi[n - nr1] - co.cn[n] * phi[n + nr1];
        double absx = std::fabs(co.cc[n] * phi[n]) + (j > 0 ? std::fabs(co.cw[n] * phi[n - 1]) : 0) + std::fabs(co.ce[n] * phi[n + 1]) + std::fabs(co.cs[n] * phi[n - nr1]) + std::fabs(co.cn[n] * phi[n + nr1]);
        rmax_ = std::max(rmax_, std::fabs(Q[n] - Ax));
        scale = std::max(scale, std::max(std::fabs(Q[n]), absx));
    }
    printf("residual %.3e mismatch %.3e\n", rmax_ / scale, dmis);
    return 0;
}
