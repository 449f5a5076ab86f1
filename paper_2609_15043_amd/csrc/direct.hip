// Direct RZ Poisson solve (Eqs. poisson and epseff with chi = 0) for
// geometries whose finite-volume operator separates: on the block of
// unknowns (rows 1..nz-1, columns 0..nr-1) the operator is
// A = Z (x) L_R + L_Z (x) D, so with D-orthonormal radial eigenvectors V
// (L_R V = D V diag(lambda)) the transformed unknowns solve one tridiagonal
// system per radial mode.  Dirichlet nodes inside the block (the coil turns)
// take their values through the capacitance system C s = phi_D - (S b)_D
// with C = S_DD, S = A^{-1}.  Per solve:
//   k_dp_rhs     right-hand side on the block (node charge plus the wall
//                couplings) and the wall values of phi;
//   k_dp_gemm    B~ = B V (rows of the block times the radial eigenvectors);
//   k_dp_pcr     the tridiagonal system of each mode by parallel cyclic
//                reduction in LDS (one workgroup per mode);
//   k_dp_xd, k_dp_src, k_dp_w: (S b)_D, s = C^{-1} (phi_D - (S b)_D), and
//                the sources transformed by V^T;
//   k_dp_correct the modes' response to those sources (precomputed unit
//                responses g), added;
//   k_dp_gemm    phi = U V^T on the block (Dirichlet nodes get their values).
// FP64 throughout; the work is a few grid-sized passes and two products of
// (nz-1) x nr by nr x nr.
#include "kernels.h"
#include "launch.h"

namespace pic {

// Potential of turn q at the step's phase: the sum over the retained orders.
__device__ __forceinline__ double turn_value(const DirectArgs &a, int q)
{
    double V = a.vc[q] * a.o.cs[0] + a.vs[q] * a.o.sn[0];
    for (int r = 1; r < a.o.n; ++r) V += a.vc[r * MAX_TURNS + q] * a.o.cs[r] + a.vs[r * MAX_TURNS + q] * a.o.sn[r];
    return V;
}

// Dirichlet value of node n at the step's phase: turn k: phi_k(t); a
// grounded node: the manufactured boundary when given, else phi as it is.
__device__ __forceinline__ double dirichlet_value(const DirectArgs &a, int n)
{
    const int k = a.tag[n];
    if (k >= 1) return turn_value(a, k - 1);
    if (a.basis) {
        double s = 0.0;
        for (int q = 0; q < a.nturns; ++q) s += a.basis[(size_t)q * a.nodes + n] * turn_value(a, q);
        return s;
    }
    return a.phi[n];
}

// b on the block: free nodes take Q plus the couplings to Dirichlet walls;
// Dirichlet nodes inside the block take 0 (their equation is replaced by
// the capacitance system).  Nodes outside the block get their phi.
__global__ __launch_bounds__(256) void k_dp_rhs(DirectArgs a)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.nodes) return;
    const int nr1 = a.nr + 1;
    const int i = n / nr1, j = n - i * nr1;
    if (i == 0 || i == a.nz || j == a.nr) {
        a.phi[n] = dirichlet_value(a, n);
        return;
    }
    double b = 0.0;
    if (a.tag[n] < 0) {
        b = a.Q[n];
        if (i == 1) b += a.cs[n] * dirichlet_value(a, n - nr1);
        if (i == a.nz - 1) b += a.cn[n] * dirichlet_value(a, n + nr1);
        if (j == a.nr - 1) b += a.ce[n] * dirichlet_value(a, n + 1);
    }
    a.b[(size_t)(i - 1) * a.nj + j] = b;
}

// C = A op(B) with A m x kk (row-major), op(B) kk x nn: B as stored
// (B[k * nn + c]) or transposed (B[c * kk + k]).  One workgroup of GW waves
// per 16 x 16 tile of C (2 x 2 per lane): wave w takes the w-th of GW
// contiguous parts of kk in slices of GK through its own LDS, the next
// slice's loads issued before the current slice is multiplied; the partial
// sums are added in wave order at the end, so the result does not depend on
// timing.  Splitting kk shortens each lane's chain of dependent FMAs by GW
// and puts GW times as many waves on the chip (the products are small:
// latency, not arithmetic, bounds them).  to_phi: C row r is block row
// r + 1 of phi (columns 0..nr-1), Dirichlet nodes of the block taking their
// values.
constexpr int GT = 16, GK = 32, GW = 4, GE = GT * GK / 64;   // tile, slice, waves, elements per lane and operand
template <bool TRANS_B, bool TO_PHI>
__global__ __launch_bounds__(GW * 64) void k_dp_gemm(const double *A, const double *B, double *C, int m, int nn,
                                                     int kk, DirectArgs a)
{
    __shared__ double As[GW][GT][GK + 1];   // [wave][row][k]
    __shared__ double Bs[GW][GK][GT + 1];   // [wave][k][column]
    __shared__ double red[GW - 1][GT * GT];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, tx = lane % 8, ty = lane / 8;
    const int r0 = blockIdx.y * GT, c0 = blockIdx.x * GT;
    // this wave's part of kk; every wave runs the same number of slices (a
    // slice past the part's end holds zeros)
    const int part = (kk + GW - 1) / GW, nsl = (part + GK - 1) / GK;
    const int kb = wave * part, ke = min(kk, kb + part);
    double ra[GE], rb[GE];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int e = 0; e < GE; ++e) {
            const int idx = e * 64 + lane;
            const int rr = idx / GK, q = idx % GK;   // A: consecutive lanes, consecutive k
            const int gr = r0 + rr, gk = k0 + q;
            ra[e] = (gr < m && gk < ke) ? A[(size_t)gr * kk + gk] : 0.0;
            int bq, bc;
            if (TRANS_B) {   // consecutive lanes, consecutive k of one column
                bc = idx / GK;
                bq = idx % GK;
            } else {         // consecutive lanes, consecutive columns of one k
                bq = idx / GT;
                bc = idx % GT;
            }
            const int hk = k0 + bq, hc = c0 + bc;
            rb[e] = (hk < ke && hc < nn) ? (TRANS_B ? B[(size_t)hc * kk + hk] : B[(size_t)hk * nn + hc]) : 0.0;
        }
    };
    double acc00 = 0.0, acc01 = 0.0, acc10 = 0.0, acc11 = 0.0;
    fetch(kb);
    for (int sl = 0; sl < nsl; ++sl) {
        const int k0 = kb + sl * GK;
#pragma unroll
        for (int e = 0; e < GE; ++e) {
            const int idx = e * 64 + lane;
            As[wave][idx / GK][idx % GK] = ra[e];
            if (TRANS_B)
                Bs[wave][idx % GK][idx / GK] = rb[e];
            else
                Bs[wave][idx / GT][idx % GT] = rb[e];
        }
        __syncthreads();
        if (sl + 1 < nsl) fetch(k0 + GK);
#pragma unroll 16
        for (int q = 0; q < GK; ++q) {
            const double x0 = As[wave][2 * ty][q], x1 = As[wave][2 * ty + 1][q];
            const double y0 = Bs[wave][q][2 * tx], y1 = Bs[wave][q][2 * tx + 1];
            acc00 = fma(x0, y0, acc00);
            acc01 = fma(x0, y1, acc01);
            acc10 = fma(x1, y0, acc10);
            acc11 = fma(x1, y1, acc11);
        }
        __syncthreads();
    }
    const int e0 = 2 * ty * GT + 2 * tx;
    if (wave > 0) {
        double *rw = red[wave - 1];
        rw[e0] = acc00;
        rw[e0 + 1] = acc01;
        rw[e0 + GT] = acc10;
        rw[e0 + GT + 1] = acc11;
    }
    __syncthreads();
    if (wave > 0) return;
    double acc[2][2] = {{acc00, acc01}, {acc10, acc11}};
    for (int v = 0; v < GW - 1; ++v)
        for (int u = 0; u < 2; ++u)
            for (int w = 0; w < 2; ++w) acc[u][w] += red[v][e0 + u * GT + w];
    for (int u = 0; u < 2; ++u)
        for (int w = 0; w < 2; ++w) {
            const int gr = r0 + 2 * ty + u, gc = c0 + 2 * tx + w;
            if (gr >= m || gc >= nn) continue;
            if (TO_PHI) {
                const int n = (gr + 1) * (a.nr + 1) + gc;
                a.phi[n] = a.tag[n] >= 0 ? dirichlet_value(a, n) : acc[u][w];
            } else {
                C[(size_t)gr * nn + gc] = acc[u][w];
            }
        }
}

// Tridiagonal solve of mode k (one workgroup) by parallel cyclic
// reduction in LDS: T_k = lambda_k Z + L_Z with diagonal lambda_k z_r +
// e_r + e_{r+1} and off-diagonals -e_r, -e_{r+1}; each round eliminates the
// neighbours at distance s from every equation (s = 1, 2, 4, ...), after
// which the equations are decoupled.  T_k is diagonally dominant, so no
// pivoting.  Column k of u is the right-hand side and the solution.
__global__ __launch_bounds__(256) void k_dp_pcr(DirectArgs a)
{
    extern __shared__ double sm[];
    const int k = blockIdx.x, ni = a.ni, nj = a.nj;
    double *A0 = sm, *B0 = sm + ni, *C0 = sm + 2 * ni, *D0 = sm + 3 * ni;
    double *A1 = sm + 4 * ni, *B1 = sm + 5 * ni, *C1 = sm + 6 * ni, *D1 = sm + 7 * ni;
    const double lam = a.lam[k];
    for (int r = threadIdx.x; r < ni; r += blockDim.x) {
        const double el = a.erow[r], eh = a.erow[r + 1];
        A0[r] = r > 0 ? -el : 0.0;
        C0[r] = r + 1 < ni ? -eh : 0.0;
        B0[r] = lam * a.zrow[r] + el + eh;
        D0[r] = a.u[(size_t)r * nj + k];
    }
    __syncthreads();
    for (int s = 1; s < ni; s <<= 1) {
        for (int r = threadIdx.x; r < ni; r += blockDim.x) {
            double an = 0.0, cn = 0.0, bn = B0[r], dn = D0[r];
            if (r - s >= 0) {
                const double al = -A0[r] / B0[r - s];
                an = al * A0[r - s];
                bn = fma(al, C0[r - s], bn);
                dn = fma(al, D0[r - s], dn);
            }
            if (r + s < ni) {
                const double ga = -C0[r] / B0[r + s];
                cn = ga * C0[r + s];
                bn = fma(ga, A0[r + s], bn);
                dn = fma(ga, D0[r + s], dn);
            }
            A1[r] = an;
            B1[r] = bn;
            C1[r] = cn;
            D1[r] = dn;
        }
        __syncthreads();
        double *t;
        t = A0, A0 = A1, A1 = t;
        t = B0, B0 = B1, B1 = t;
        t = C0, C0 = C1, C1 = t;
        t = D0, D0 = D1, D1 = t;
    }
    for (int r = threadIdx.x; r < ni; r += blockDim.x) a.u[(size_t)r * nj + k] = D0[r] / B0[r];
}

// The capacitance step, spread over the chip in three kernels (each a
// fixed-order reduction per output, so the result is the same every run):
// k_dp_xd: res_d = phi_D - (V u)_d at each interior Dirichlet node (one
// wave per node); k_dp_src: s = C^{-1} res (one wave per row of C^{-1});
// k_dp_w: w(q, k) = sum over the nodes d of row rows[q] of s_d V(j_d, k)
// (one lane per (q, k); the nodes of a row are a contiguous range).
__device__ __forceinline__ double wave_sum(double x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__global__ __launch_bounds__(64) void k_dp_xd(DirectArgs a)
{
    const int d = blockIdx.x, lane = threadIdx.x, nj = a.nj, nr1 = a.nr + 1;
    const int n = a.dnode[d], i = n / nr1, j = n - i * nr1;
    const double *u = a.u + (size_t)(i - 1) * nj;
    const double *v = a.v + (size_t)j * nj;
    double x = 0.0;
    for (int k = lane; k < nj; k += 64) x = fma(v[k], u[k], x);
    x = wave_sum(x);
    if (lane == 0) a.res[d] = dirichlet_value(a, n) - x;
}

__global__ __launch_bounds__(64) void k_dp_src(DirectArgs a)
{
    const int d = blockIdx.x, lane = threadIdx.x, m = a.m;
    const double *ci = a.cinv + (size_t)d * m;
    double s = 0.0;
    for (int e = lane; e < m; e += 64) s = fma(ci[e], a.res[e], s);
    s = wave_sum(s);
    if (lane == 0) a.src[d] = s;
}

__global__ __launch_bounds__(256) void k_dp_w(DirectArgs a)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x, nj = a.nj, nr1 = a.nr + 1;
    if (t >= a.nrow * nj) return;
    const int q = t / nj, k = t - q * nj;
    const int d0 = a.rowstart[q], d1 = a.rowstart[q + 1];
    double w = 0.0;
    // the row's nodes in batches of 8: all loads of a batch are issued
    // before its FMAs (which keep the node order)
    for (int d = d0; d < d1; d += 8) {
        double sv[8], vv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int dd = d + e < d1 ? d + e : d0;
            const int n = a.dnode[dd], j = n - (n / nr1) * nr1;
            sv[e] = a.src[dd];
            vv[e] = a.v[(size_t)j * nj + k];
        }
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (d + e < d1) w = fma(sv[e], vv[e], w);
    }
    a.w[t] = w;
}

// u += sum_q g_q w_q: the modes' response to the capacitance sources
// (one element of u per lane).
__global__ __launch_bounds__(256) void k_dp_correct(DirectArgs a)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t tot = (size_t)a.ni * a.nj;
    if (t >= tot) return;
    const int k = (int)(t % a.nj);
    double d = 0.0;
    for (int q = 0; q < a.nrow; ++q) d = fma(a.g[(size_t)q * tot + t], a.w[(size_t)q * a.nj + k], d);
    a.u[t] += d;
}

void launch_direct_solve(const DirectArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_dp_rhs, dim3((a.nodes + 255) / 256), dim3(256), 0, st, a);
    const dim3 g((a.nj + GT - 1) / GT, (a.ni + GT - 1) / GT);
    // B~ = B V into u, then the mode solves in place
    hipLaunchKernelGGL((k_dp_gemm<false, false>), g, dim3(GW * 64), 0, st, (const double *)a.b, a.v, a.u, a.ni,
                       a.nj, a.nj, a);
    hipLaunchKernelGGL(k_dp_pcr, dim3(a.nj), dim3(256), 8 * (size_t)a.ni * sizeof(double), st, a);
    if (a.m > 0) {
        hipLaunchKernelGGL(k_dp_xd, dim3(a.m), dim3(64), 0, st, a);
        hipLaunchKernelGGL(k_dp_src, dim3(a.m), dim3(64), 0, st, a);
        hipLaunchKernelGGL(k_dp_w, dim3((a.nrow * a.nj + 255) / 256), dim3(256), 0, st, a);
        const size_t tot = (size_t)a.ni * a.nj;
        hipLaunchKernelGGL(k_dp_correct, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a);
    }
    hipLaunchKernelGGL((k_dp_gemm<true, true>), g, dim3(GW * 64), 0, st, (const double *)a.u, a.v,
                       (double *)nullptr, a.ni, a.nj, a.nj, a);
}

}  // namespace pic
