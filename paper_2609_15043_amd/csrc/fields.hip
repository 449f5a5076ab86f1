// Grid kernels of the RZ PIC/MCC step: field staging for the gather, node
// charge / current from the fixed-point accumulators, the per-step period
// accumulation, the FP64 geometric multigrid for the finite-volume RZ
// Poisson problem, and the turn charges from the operator's face fluxes.
#include "kernels.h"
#include "launch.h"

namespace pic {

// ---------------------------------------------------------------------------
// Staging: E_r, E_z = -grad phi (central inside, one-sided at the box edges,
// E_r = 0 on the axis) and E_theta(t_n) = E_c cos th - E_s^sto sin th, packed
// per node for the gather; the step's deposit accumulators are cleared.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_stage(const double *phi, const double *ec, const double *es, Orders o,
                        typename Field4<T>::type *ef, long long *accJ, long long *accQ, int clear_q, GridC g)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.nodes) return;
    const int i = n / g.nr1, j = n - i * g.nr1;
    double ez, er;
    if (i == 0)
        ez = -(phi[n + g.nr1] - phi[n]) / g.dz;
    else if (i == g.nz)
        ez = -(phi[n] - phi[n - g.nr1]) / g.dz;
    else
        ez = -(phi[n + g.nr1] - phi[n - g.nr1]) / (2.0 * g.dz);
    if (j == 0)
        er = 0.0;
    else if (j == g.nr)
        er = -(phi[n] - phi[n - 1]) / g.dr;
    else
        er = -(phi[n + 1] - phi[n - 1]) / (2.0 * g.dr);
    double et = ec[n] * o.cs[0] - es[n] * o.sn[0];
    for (int m = 1; m < o.n; ++m)   // retained orders m + 1 (arrays order after order)
        et += ec[(size_t)m * g.nodes + n] * o.cs[m] - es[(size_t)m * g.nodes + n] * o.sn[m];
    typename Field4<T>::type f;
    f.x = (T)er;
    f.y = (T)ez;
    f.z = (T)et;
    f.w = (T)0;
    ef[n] = f;
    accJ[n] = 0;
    accJ[g.nodes + n] = 0;
    if (clear_q) {
        accQ[n] = 0;
        accQ[g.nodes + n] = 0;
    }
}

// RF magnetic field of the applied azimuthal field at phase th (Faraday's
// law): with F = (E_c sin th + E_s^sto cos th) / w the zero-mean time
// integral of E_theta(t) = E_c cos - E_s^sto sin, B = -curl(F theta_hat),
// i.e. B_r = dF/dz and B_z = -(1/R) d(R F)/dR; central differences inside,
// one-sided at the box edges, B_z = -2 dF/dR on the axis (F = 0 there).
template <typename T>
__global__ void k_stage_b(const double *ec, const double *es, double cs, double sn, double inv_w,
                          typename Field2<T>::type *eb, GridC g)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.nodes) return;
    const int i = n / g.nr1, j = n - i * g.nr1;
    auto F = [&](int m) { return (ec[m] * sn + es[m] * cs) * inv_w; };
    double br, bz;
    if (i == 0)
        br = (F(n + g.nr1) - F(n)) / g.dz;
    else if (i == g.nz)
        br = (F(n) - F(n - g.nr1)) / g.dz;
    else
        br = (F(n + g.nr1) - F(n - g.nr1)) / (2.0 * g.dz);
    if (j == 0) {
        bz = -2.0 * (F(n + 1) - F(n)) / g.dr;
    } else {
        const double R = j * g.dr;
        if (j == g.nr)
            bz = -(R * F(n) - (R - g.dr) * F(n - 1)) / g.dr / R;
        else
            bz = -((R + g.dr) * F(n + 1) - (R - g.dr) * F(n - 1)) / (2.0 * g.dr) / R;
    }
    typename Field2<T>::type b;
    b.x = (T)br;
    b.y = (T)bz;
    eb[n] = b;
}

// Direct-implicit susceptibility at the nodes from the predicted particles'
// weights accQ_s (fixed point, per species): chi = (dt^2 / 2) / eps0 sum_s
// (q_s^2 / m_s) w_s (accQ_s / 2^kQ) / V_node, i.e. half the squared plasma
// frequency times dt^2 (the D1 scheme's susceptibility in Eq. poisson).
// c0, c1 carry every factor but the node volume.
__global__ void k_chi(const long long *accQ, double c0, double c1, double *chi, GridC g)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.nodes) return;
    const int i = n / g.nr1, j = n - i * g.nr1;
    chi[n] = (c0 * (double)accQ[n] + c1 * (double)accQ[g.nodes + n]) / node_volume(g, i, j);
}

// Level-0 Poisson operator with the susceptibility: every face conductance
// of the chi = 0 operator (base arrays) times 1 + (chi_a + chi_b) / 2 (Eq.
// epseff), the diagonal their sum.
__global__ void k_chi_operator(const double *cw0, const double *ce0, const double *cs0, const double *cn0,
                               const double *chi, double *cw, double *ce, double *cs, double *cn, double *cc, GridC g)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.nodes) return;
    const int i = n / g.nr1, j = n - i * g.nr1;
    const double x = chi[n];
    const double w = j > 0 ? cw0[n] * (1.0 + 0.5 * (x + chi[n - 1])) : 0.0;
    const double e = j < g.nr ? ce0[n] * (1.0 + 0.5 * (x + chi[n + 1])) : 0.0;
    const double s = i > 0 ? cs0[n] * (1.0 + 0.5 * (x + chi[n - g.nr1])) : 0.0;
    const double t = i < g.nz ? cn0[n] * (1.0 + 0.5 * (x + chi[n + g.nr1])) : 0.0;
    cw[n] = w;
    ce[n] = e;
    cs[n] = s;
    cn[n] = t;
    cc[n] = w + e + s + t;
}

void launch_chi(const long long *accQ, double c0, double c1, double *chi, const double *cw0, const double *ce0,
                const double *cs0, const double *cn0, const MGLevel &L0, const GridC &g, hipStream_t st)
{
    hipLaunchKernelGGL(k_chi, dim3((g.nodes + 255) / 256), dim3(256), 0, st, accQ, c0, c1, chi, g);
    hipLaunchKernelGGL(k_chi_operator, dim3((g.nodes + 255) / 256), dim3(256), 0, st, cw0, ce0, cs0, cn0,
                       (const double *)chi, const_cast<double *>(L0.cw), const_cast<double *>(L0.ce),
                       const_cast<double *>(L0.cs), const_cast<double *>(L0.cn), const_cast<double *>(L0.cc), g);
}

// node charge = sum_s q_s w_s (accQ_s / 2^kQ + accS_s), after the step's
// window charge accW_s / 2^kQ (fixed point) has joined the persistent FP64
// window sums accS_s (one add per node and step, in a fixed order)
__global__ void k_finalize_q(const long long *accQ, long long *accW, double *accS, double inv_scale, double cq0,
                             double cq1, double cs0, double cs1, double *Q, int nodes)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nodes) return;
    const long long w0 = accW[n], w1 = accW[nodes + n];
    double s0 = accS[n], s1 = accS[nodes + n];
    if (w0 | w1) {
        s0 += (double)w0 * inv_scale;
        s1 += (double)w1 * inv_scale;
        accS[n] = s0;
        accS[nodes + n] = s1;
        accW[n] = 0;
        accW[nodes + n] = 0;
    }
    Q[n] = (cq0 * (double)accQ[n] + cq1 * (double)accQ[nodes + n]) + (cs0 * s0 + cs1 * s1);
}

__device__ __forceinline__ void neumaier(double &sum, double &comp, double x)
{
    const double t = sum + x;
    if (fabs(sum) >= fabs(x))
        comp += (sum - t) + x;
    else
        comp += (x - t) + sum;
    sum = t;
}

// ---------------------------------------------------------------------------
// Per-step period accumulation (compensated FP64).  A second one-block
// kernel reduces the inductive-power partials in block order and updates
// the turn sums, so the result does not depend on block scheduling.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_harmonic(const long long *accJ, double cj0, double cj1, const double *ec,
                                                  const double *es, Orders o, double *I, double *Jc, double *Jcc,
                                                  double *Js, double *Jsc, double *partial, int nodes)
{
    __shared__ double red[256];
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    double pw = 0.0;
    if (n < nodes) {
        const double cur = cj0 * (double)accJ[n] + cj1 * (double)accJ[nodes + n];
        I[n] = cur;
        double et = ec[n] * o.cs[0] - es[n] * o.sn[0];
        for (int m = 1; m < o.n; ++m)
            et += ec[(size_t)m * nodes + n] * o.cs[m] - es[(size_t)m * nodes + n] * o.sn[m];
        pw = cur * et;
        // the current's harmonic of every retained order (arrays order after order)
        for (int m = 0; m < o.n; ++m) {
            const size_t q = (size_t)m * nodes + n;
            double a = Jc[q], ac = Jcc[q];
            neumaier(a, ac, cur * o.cs[m]);
            Jc[q] = a;
            Jcc[q] = ac;
            double b = Js[q], bc = Jsc[q];
            neumaier(b, bc, cur * o.sn[m]);
            Js[q] = b;
            Jsc[q] = bc;
        }
    }
    red[threadIdx.x] = pw;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Every retained order keeps its own accumulator: the turn-charge
// harmonics of its order, and the same time-domain inductive power and
// V dQ trapezoid (of the total potentials) in each.
__global__ __launch_bounds__(256) void k_harmonic_fold(const double *partial, int nparts, Orders o, HarmState *hs,
                                                       const double *Qk, const double *vc, const double *vs,
                                                       int nturns)
{
    __shared__ double red[256];
    {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nparts; b += 256) acc += partial[b];
        red[threadIdx.x] = acc;
    }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x >= o.n) return;
    const int m = threadIdx.x;
    HarmState *h = hs + m;
    neumaier(h->pind, h->pind_c, red[0]);
    for (int k = 0; k < nturns; ++k) {
        double V = vc[k] * o.cs[0] + vs[k] * o.sn[0];
        for (int r = 1; r < o.n; ++r) V += vc[r * MAX_TURNS + k] * o.cs[r] + vs[r * MAX_TURNS + k] * o.sn[r];
        const double q = Qk[k];
        neumaier(h->qc[k], h->qc_c[k], q * o.cs[m]);
        neumaier(h->qs[k], h->qs_c[k], q * o.sn[m]);
        if (h->samples == 0) {
            h->v_first[k] = V;
            h->q_first[k] = q;
        } else {
            neumaier(h->w[k], h->w_c[k], 0.5 * (V + h->v_prev[k]) * (q - h->q_prev[k]));
        }
        h->v_prev[k] = V;
        h->q_prev[k] = q;
    }
    h->samples += 1;
}

// ---------------------------------------------------------------------------
// Multigrid on a vertex-centred hierarchy (factor-2 coarsening), used as
// the preconditioner of a conjugate-gradient solve.  Level 0 smooths with
// red-black Gauss-Seidel (5-point), the Galerkin levels with four-colour
// Gauss-Seidel (9-point); restriction is P^T, prolongation bilinear P,
// both skipping Dirichlet nodes; the coarse operators are P^T A P.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double apply_op(const MGLevel &L, const double *x, int n, int i, int j)
{
    if (!L.nine) {
        double a = L.cc[n] * x[n];
        if (j > 0) a -= L.cw[n] * x[n - 1];
        if (j < L.nr) a -= L.ce[n] * x[n + 1];
        if (i > 0) a -= L.cs[n] * x[n - L.nr1];
        if (i < L.nz) a -= L.cn[n] * x[n + L.nr1];
        return a;
    }
    double a = 0.0;
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
        if (i + di < 0 || i + di > L.nz) continue;
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
            if (j + dj < 0 || j + dj > L.nr) continue;
            a += L.a[(size_t)((di + 1) * 3 + dj + 1) * L.nodes + n] * x[n + di * L.nr1 + dj];
        }
    }
    return a;
}

// Full-weighting restriction of the finer level's residual to coarse node
// (I, J): weights 1, 1/2, 1/4 on the 3 x 3 fine nodes around (2I, 2J), the
// transpose of the bilinear prolongation below.
__device__ __forceinline__ double restrict_res(const MGLevel &F, int I, int J)
{
    double s = 0.0;
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
        const int i = 2 * I + di;
        if (i < 0 || i > F.nz) continue;
        const double wi = di == 0 ? 1.0 : 0.5;
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
            const int j = 2 * J + dj;
            if (j < 0 || j > F.nr) continue;
            const double wj = dj == 0 ? 1.0 : 0.5;
            s += wi * wj * F.res[i * F.nr1 + j];
        }
    }
    return s;
}

// Bilinear prolongation of the coarse correction to fine node (i, j)
__device__ __forceinline__ double prolong_at(const MGLevel &C, int i, int j)
{
    const int I = i >> 1, J = j >> 1;
    const int c = I * C.nr1 + J;
    if (!(i & 1) && !(j & 1)) return C.phi[c];
    if (!(i & 1)) return 0.5 * (C.phi[c] + C.phi[c + 1]);
    if (!(j & 1)) return 0.5 * (C.phi[c] + C.phi[c + C.nr1]);
    return 0.25 * (C.phi[c] + C.phi[c + 1] + C.phi[c + C.nr1] + C.phi[c + C.nr1 + 1]);
}

// block partial sums of the CG kernels (defined with them below)
__device__ __forceinline__ void block_partial(double v, double *out, bool is_max);

// Tile smoother: each workgroup stages a TZ x TR tile of the correction plus
// a one-node halo in LDS and runs `sweeps` Gauss-Seidel sweeps (red-black on
// the 5-point level, four colours on the Galerkin levels; colours in reverse
// order when SM_REVERSE) on its tile, the halo held at its values from the
// start of the kernel: Gauss-Seidel inside a tile, Jacobi across tiles.
// The result goes to `out`, which must not be L.phi unless SM_ZERO is set:
// a tile that finished early would otherwise change the halo its
// neighbours load, and the V-cycle would depend on the order in which
// workgroups run.  Reversing the colour order for the post-smoother keeps
// the V-cycle a symmetric preconditioner.  The modes fold the V-cycle's
// transfers into the smoothers:
//   SM_ZERO     the correction starts from zero (pre-smoother; L.phi is not
//               read, Dirichlet nodes of out are written 0);
//   SM_RHS      the right-hand side is the full-weighting restriction of
//               the finer level's residual, stored in L.rhs;
//   SM_PROLONG  the coarser level's correction is prolonged and added to
//               the tile (and halo) as it is loaded (post-smoother);
//   SM_RZ       per-block partial of rhs . x over the tile (the CG r.z of
//               the level-0 post-smoother) to partial[2 * block].
// Tiles of 8 x 32 nodes, one per thread: every level is latency-bound, and
// small tiles give it the most workgroups (16 x 64 tiles on level 0 took
// 13 us per sweep pair against 7 us, at the same CG iteration counts).
constexpr int TILE_Z = 8, TILE_R = 32;
__global__ __launch_bounds__(256) void k_mg_smooth_tile(MGLevel L, MGLevel F, MGLevel C, int sweeps, int mode,
                                                        const MGState *st, double *partial, double *out)
{
    constexpr int TILE_PER = TILE_Z * TILE_R / 256;
    __shared__ double xs[(TILE_Z + 2) * (TILE_R + 2)];
    if (st->done) return;
    constexpr int W = TILE_R + 2;
    const int tiles_r = (L.nr1 + TILE_R - 1) / TILE_R;
    const int i0 = (blockIdx.x / tiles_r) * TILE_Z, j0 = (blockIdx.x % tiles_r) * TILE_R;
    for (int e = threadIdx.x; e < (TILE_Z + 2) * W; e += 256) {
        const int i = i0 - 1 + e / W, j = j0 - 1 + e % W;
        double v = 0.0;
        if (i >= 0 && i <= L.nz && j >= 0 && j <= L.nr) {
            const int n = i * L.nr1 + j;
            if (!(mode & SM_ZERO)) v = L.phi[n];
            if ((mode & SM_PROLONG) && !L.dir[n]) v += prolong_at(C, i, j);
        }
        xs[e] = v;
    }
    // owned nodes: coefficients and right-hand side in registers
    const int nc = L.nine ? 4 : 2;
    double coef[TILE_PER][9], rhs[TILE_PER];
    int own[TILE_PER], col[TILE_PER];
#pragma unroll
    for (int q = 0; q < TILE_PER; ++q) {
        const int e = threadIdx.x + 256 * q;
        const int i = i0 + e / TILE_R, j = j0 + e % TILE_R;
        own[q] = -1;
        col[q] = -1;
        rhs[q] = 0.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) coef[q][k] = 0.0;
        if (i > L.nz || j > L.nr) continue;
        const int n = i * L.nr1 + j;
        if (L.dir[n]) {
            if (mode & SM_ZERO) out[n] = 0.0;
            if (mode & SM_RHS) L.rhs[n] = 0.0;
            continue;
        }
        own[q] = n;
        col[q] = L.nine ? ((i & 1) << 1) | (j & 1) : ((i + j) & 1);
        if (mode & SM_RHS) {
            rhs[q] = restrict_res(F, i, j);
            L.rhs[n] = rhs[q];
        } else {
            rhs[q] = L.rhs[n];
        }
        if (L.nine) {
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int di = k / 3 - 1, dj = k % 3 - 1;
                const bool in = i + di >= 0 && i + di <= L.nz && j + dj >= 0 && j + dj <= L.nr;
                coef[q][k] = in ? L.a[(size_t)k * L.nodes + n] : 0.0;
            }
        } else {
            coef[q][4] = L.cc[n];
            coef[q][3] = j > 0 ? -L.cw[n] : 0.0;
            coef[q][5] = j < L.nr ? -L.ce[n] : 0.0;
            coef[q][1] = i > 0 ? -L.cs[n] : 0.0;
            coef[q][7] = i < L.nz ? -L.cn[n] : 0.0;
        }
    }
    __syncthreads();
    for (int sw = 0; sw < sweeps; ++sw)
        for (int cc = 0; cc < nc; ++cc) {
            const int c = (mode & SM_REVERSE) ? nc - 1 - cc : cc;
#pragma unroll
            for (int q = 0; q < TILE_PER; ++q) {
                if (col[q] != c) continue;
                const int e = threadIdx.x + 256 * q;
                const int li = e / TILE_R + 1, lj = e % TILE_R + 1;
                double ax = 0.0;
#pragma unroll
                for (int k = 0; k < 9; ++k) ax += coef[q][k] * xs[(li + k / 3 - 1) * W + lj + k % 3 - 1];
                xs[li * W + lj] += (rhs[q] - ax) / coef[q][4];
            }
            __syncthreads();
        }
    double rz = 0.0;
#pragma unroll
    for (int q = 0; q < TILE_PER; ++q) {
        if (own[q] < 0) continue;
        const int e = threadIdx.x + 256 * q;
        const double x = xs[(e / TILE_R + 1) * W + e % TILE_R + 1];
        out[own[q]] = x;
        rz += rhs[q] * x;
    }
    if (mode & SM_RZ) block_partial(rz, partial + 2 * blockIdx.x, false);
}

// residual of a level after its pre-smoother: res = rhs - A phi on free
// nodes, 0 on Dirichlet nodes
__global__ __launch_bounds__(256) void k_mg_resid(MGLevel L, const MGState *st)
{
    if (st->done) return;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < L.nodes; n += gridDim.x * blockDim.x) {
        if (L.dir[n]) {
            L.res[n] = 0.0;
            continue;
        }
        const int i = n / L.nr1, j = n - i * L.nr1;
        L.res[n] = L.rhs[n] - apply_op(L, L.phi, n, i, j);
    }
}

// right-hand side of the bottom level: restriction of the finer residual
__global__ __launch_bounds__(256) void k_mg_restrict_res(MGLevel F, MGLevel C, const MGState *st)
{
    if (st->done) return;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < C.nodes; n += gridDim.x * blockDim.x) {
        const int I = n / C.nr1, J = n - I * C.nr1;
        C.rhs[n] = C.dir[n] ? 0.0 : restrict_res(F, I, J);
    }
}

// Bottom solve of the preconditioner: phi = Inv rhs with the inverse held in
// FP32 (symmetrised when rounded, so the preconditioner stays symmetric;
// products and sums in FP64).  It is half the bytes of the FP64 inverse,
// which every CG iteration streams; an approximate bottom solve changes
// only how fast CG converges, not the tolerance it converges to.  One wave
// per row, the row streamed in 16-byte loads (rows padded to a multiple of
// four, ld floats) into two independent partial sums.
__global__ __launch_bounds__(256) void k_dense_solve(const float *inv, int ld, MGLevel L, const MGState *st)
{
    if (st->done) return;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= L.nodes) return;
    const int lane = threadIdx.x & 63;
    const float4 *row = reinterpret_cast<const float4 *>(inv + (size_t)r * ld);
    const int n4 = L.nodes >> 2;
    double s0 = 0.0, s1 = 0.0;
    for (int k = lane; k < n4; k += 64) {
        const float4 a = row[k];
        s0 += (double)a.x * L.rhs[4 * k] + (double)a.z * L.rhs[4 * k + 2];
        s1 += (double)a.y * L.rhs[4 * k + 1] + (double)a.w * L.rhs[4 * k + 3];
    }
    for (int k = 4 * n4 + lane; k < L.nodes; k += 64) s0 += (double)inv[(size_t)r * ld + k] * L.rhs[k];
    const double s = wave_total(s0 + s1);
    if (lane == 63) L.phi[r] = s;
}

// FP32 copy of the FP64 inverse (row stride ld), symmetrised: out(r, c) =
// (inv(r, c) + inv(c, r)) / 2 rounded once; the padding columns are 0.
__global__ void k_inverse_f32(const double *inv, int n, int ld, float *out, int ld32)
{
    const int64_t total = (int64_t)n * ld32;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(t / ld32), c = (int)(t - (int64_t)r * ld32);
        out[t] = c < n ? (float)(0.5 * (inv[(size_t)r * ld + c] + inv[(size_t)c * ld + r])) : 0.f;
    }
}

// In-place Gauss-Jordan inversion (row stride ld), one pivot per kernel
// pair: save the scaled pivot row and the pivot column, then update every
// entry.
__global__ void k_gj_save(const double *A, int n, int ld, int k, double *rowk, double *colk)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double p = A[(size_t)k * ld + k];
    rowk[t] = t == k ? 1.0 / p : A[(size_t)k * ld + t] / p;
    colk[t] = A[(size_t)t * ld + k];
}

__global__ void k_gj_update(double *A, int n, int ld, int k, const double *rowk, const double *colk)
{
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)n * n) return;
    const int i = (int)(e / n), j = (int)(e - (size_t)i * n);
    double &a = A[(size_t)i * ld + j];
    if (i == k)
        a = rowk[j];
    else
        a = (j == k ? 0.0 : a) - colk[i] * rowk[j];
}

// ---------------------------------------------------------------------------
// Conjugate gradient on the free nodes of level 0, preconditioned by one
// V-cycle.  Scalars (r.z, alpha, beta, norms) stay on the device.  Each
// reduction writes per-block partials that the NEXT kernel sums (stream
// order makes them visible without device-scope fences), every block the
// same partials in the same order, so all blocks agree bit for bit.  After
// convergence every kernel returns at once, so the host can enqueue a
// budget of iterations without synchronising.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_partial(double v, double *out, bool is_max)
{
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] = is_max ? fmax(red[threadIdx.x], red[threadIdx.x + off]) : red[threadIdx.x] + red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// sum (or max) of the first np partials, same value in every thread
__device__ __forceinline__ double fold_partials(const double *part, int np, int stride, bool is_max)
{
    __shared__ double red[256];
    __shared__ double result;
    double acc = 0.0;
    for (int b = threadIdx.x; b < np; b += blockDim.x) acc = is_max ? fmax(acc, part[b * stride]) : acc + part[b * stride];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] = is_max ? fmax(red[threadIdx.x], red[threadIdx.x + off]) : red[threadIdx.x] + red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) result = red[0];
    __syncthreads();
    return result;
}

// Dirichlet values (turn k nodes: phi_k(t_n)); free nodes start from the
// solution extrapolated in time from the stored previous solutions (prev:
// two arrays, phi^{n-1} then phi^{n-2}): order 1 gives 2 phi^n - phi^{n-1},
// order 2 gives 3 phi^n - 3 phi^{n-1} + phi^{n-2}; the stored solutions then
// shift by one; state reset.
__global__ void k_pcg_begin(MGLevel L, PCGVec v, const int32_t *tag, const double *vc, const double *vs, Orders o,
                            MGState *st, double *prev, int order, const double *basis, int nturns)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n == 0) {
        st->done = 0;
        st->cycles = -1;
        st->ticket = 0;
        st->rz[0] = 0.0;
    }
    if (n >= L.nodes) return;
    const int k = tag[n];
    // turn potential at t_n: the sum over the retained orders
    auto turn = [&](int q) {
        double V = vc[q] * o.cs[0] + vs[q] * o.sn[0];
        for (int r = 1; r < o.n; ++r) V += vc[r * MAX_TURNS + q] * o.cs[r] + vs[r * MAX_TURNS + q] * o.sn[r];
        return V;
    };
    if (k >= 1) {
        v.x[n] = turn(k - 1);
    } else if (k == 0 && basis) {
        // manufactured boundary: linear in the turn potentials
        double s = 0.0;
        for (int q = 0; q < nturns; ++q) s += basis[(size_t)q * L.nodes + n] * turn(q);
        v.x[n] = s;
    } else if (k < 0 && prev) {
        double *prev2 = prev + L.nodes;
        const double cur = v.x[n], p1 = prev[n];
        if (order == 2)
            v.x[n] = 3.0 * cur - 3.0 * p1 + prev2[n];
        else if (order == 1)
            v.x[n] = 2.0 * cur - p1;
        prev2[n] = p1;
        prev[n] = cur;
    }
}

// sum of |terms| of (A x)_n on the 5-point level: the size of the equation,
// including the drive from Dirichlet neighbours
__device__ __forceinline__ double apply_abs(const MGLevel &L, const double *x, int n, int i, int j)
{
    double a = fabs(L.cc[n] * x[n]);
    if (j > 0) a += fabs(L.cw[n] * x[n - 1]);
    if (j < L.nr) a += fabs(L.ce[n] * x[n + 1]);
    if (i > 0) a += fabs(L.cs[n] * x[n - L.nr1]);
    if (i < L.nz) a += fabs(L.cn[n] * x[n + L.nr1]);
    return a;
}

// r = b - A x on free nodes (0 on Dirichlet), z = p = 0; partials of
// max|r| and of the equation scale max(|b|, sum |A_nm x_m|)
__global__ __launch_bounds__(256) void k_pcg_resid(MGLevel L, PCGVec v, double *partial)
{
    double m0 = 0.0, m1 = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < L.nodes; n += gridDim.x * blockDim.x) {
        v.z[n] = 0.0;
        v.p[n] = 0.0;
        if (L.dir[n]) {
            v.r[n] = 0.0;
            continue;
        }
        const int i = n / L.nr1, j = n - i * L.nr1;
        const double r = v.b[n] - apply_op(L, v.x, n, i, j);
        v.r[n] = r;
        m0 = fmax(m0, fabs(r));
        m1 = fmax(m1, fmax(fabs(v.b[n]), apply_abs(L, v.x, n, i, j)));
    }
    block_partial(m0, partial + 2 * blockIdx.x, true);
    block_partial(m1, partial + 2 * blockIdx.x + 1, true);
}

// One block: convergence test on the residual partials (k_pcg_resid at the
// start of a solve, k_pcg_update afterwards); counts the iteration.
// unconv (nullable, given to the last check of a solve): counts the solve
// when its iteration budget ran out before rtol was met
__global__ __launch_bounds__(256) void k_pcg_check(MGState *st, const double *partial, int np, double rtol, int first,
                                                   unsigned long long *unconv)
{
    if (st->done) return;
    const double R = fold_partials(partial, np, 2, true);
    double scale = st->scale;
    if (first) scale = fold_partials(partial + 1, np, 2, true);
    if (threadIdx.x != 0) return;
    if (first) st->scale = scale = scale > 0.0 ? scale : 1.0;
    st->cycles += 1;
    st->rel = R / scale;
    if (R == 0.0 || st->rel <= rtol) st->done = 1;
    else if (unconv) atomicAdd(unconv, 1ull);
}

// partials of r.z when the V-cycle is the dense solve alone (no smoother)
__global__ __launch_bounds__(256) void k_pcg_rz(MGLevel L, PCGVec v, const MGState *st, double *partial)
{
    if (st->done) return;
    double s = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < L.nodes; n += gridDim.x * blockDim.x) s += v.r[n] * v.z[n];
    block_partial(s, partial + 2 * blockIdx.x, false);
}

// rz_k = sum of the r.z partials (from the level-0 post-smoother, even
// slots); p' = z + (rz_k / rz_{k-1}) p (beta = 0 first) into the other p
// buffer; Ap' = A p' on free nodes, with p' at the neighbours formed on
// the fly from z and p; partials of p'.Ap' to the odd slots.
__global__ __launch_bounds__(256) void k_pcg_pmatvec(MGLevel L, PCGVec v, const double *pold, double *pnew,
                                                     MGState *st, double *partial, int nrz)
{
    if (st->done) return;
    const int it = st->cycles;
    const double rz = fold_partials(partial, nrz, 2, false);
    const double beta = it == 0 || st->rz[it] == 0.0 ? 0.0 : rz / st->rz[it];
    if (blockIdx.x == 0 && threadIdx.x == 0) st->rz[it + 1] = rz;
    double s = 0.0;
    const double *z = v.z;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < L.nodes; n += gridDim.x * blockDim.x) {
        const double pn = z[n] + beta * pold[n];
        pnew[n] = pn;
        double ap = 0.0;
        if (!L.dir[n]) {
            const int i = n / L.nr1, j = n - i * L.nr1;
            ap = L.cc[n] * pn;
            if (j > 0) ap -= L.cw[n] * (z[n - 1] + beta * pold[n - 1]);
            if (j < L.nr) ap -= L.ce[n] * (z[n + 1] + beta * pold[n + 1]);
            if (i > 0) ap -= L.cs[n] * (z[n - L.nr1] + beta * pold[n - L.nr1]);
            if (i < L.nz) ap -= L.cn[n] * (z[n + L.nr1] + beta * pold[n + L.nr1]);
        }
        v.Ap[n] = ap;
        s += pn * ap;
    }
    block_partial(s, partial + 2 * blockIdx.x + 1, false);
}

// alpha = rz / p.Ap (odd-slot partials); x += alpha p, r -= alpha Ap;
// partials of max|r| to the even slots
__global__ __launch_bounds__(256) void k_pcg_update(MGLevel L, PCGVec v, const double *p, const MGState *st,
                                                    double *partial, int np)
{
    if (st->done) return;
    const double pap = fold_partials(partial + 1, np, 2, false);
    const double alpha = pap != 0.0 ? st->rz[st->cycles + 1] / pap : 0.0;
    __syncthreads();
    double m = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < L.nodes; n += gridDim.x * blockDim.x) {
        if (L.dir[n]) continue;
        v.x[n] += alpha * p[n];
        const double r = v.r[n] - alpha * v.Ap[n];
        v.r[n] = r;
        m = fmax(m, fabs(r));
    }
    block_partial(m, partial + 2 * blockIdx.x, true);
}

// Q_k = sum over faces (turn-k node p, outside node q) of c (phi_p - phi_q);
// one workgroup, per-thread partial sums per turn, tree reduction in a
// fixed order (the face list is sorted by turn-node index on the host)
// One wave per turn (nturns waves in one workgroup): each lane sums its
// share of the turn's faces in list order, then a fixed butterfly across the
// wave; no barriers.
__global__ __launch_bounds__(1024) void k_face_charge(const double *phi, const int32_t *fp, const int32_t *fq,
                                                      const int32_t *fk, const double *fc, int nfaces, double *Qk,
                                                      int nturns, const double *chi)
{
    const int k = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (k >= nturns) return;
    double s = 0.0;
    for (int f = lane; f < nfaces; f += 64)
        if (fk[f] == k) {
            // the solve's own face coefficient, the susceptibility included (Eq. facecharge)
            const double x = chi ? 1.0 + 0.5 * (chi[fp[f]] + chi[fq[f]]) : 1.0;
            s += fc[f] * x * (phi[fp[f]] - phi[fq[f]]);
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) Qk[k] = s;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
void launch_stage(const double *phi, const double *ec, const double *es, const Orders &o,
                  typename Field4<T>::type *ef, long long *accJ, long long *accQ, bool clear_q, const GridC &g,
                  hipStream_t st)
{
    hipLaunchKernelGGL(k_stage<T>, dim3(nblk(g.nodes, 256)), dim3(256), 0, st, phi, ec, es, o, ef, accJ, accQ,
                       clear_q ? 1 : 0, g);
}
template <typename T>
void launch_stage_b(const double *ec, const double *es, double cs, double sn, double inv_w,
                    typename Field2<T>::type *eb, const GridC &g, hipStream_t st)
{
    hipLaunchKernelGGL(k_stage_b<T>, dim3(nblk(g.nodes, 256)), dim3(256), 0, st, ec, es, cs, sn, inv_w, eb, g);
}
template void launch_stage_b<float>(const double *, const double *, double, double, double, float2 *, const GridC &,
                                    hipStream_t);
template void launch_stage_b<double>(const double *, const double *, double, double, double, double2 *,
                                     const GridC &, hipStream_t);
template void launch_stage<float>(const double *, const double *, const double *, const Orders &, float4 *,
                                  long long *, long long *, bool, const GridC &, hipStream_t);
template void launch_stage<double>(const double *, const double *, const double *, const Orders &, double4 *,
                                   long long *, long long *, bool, const GridC &, hipStream_t);

void launch_finalize_q(const long long *accQ, long long *accW, double *accS, double inv_scale, double cq0, double cq1,
                       double cs0, double cs1, double *Q, int nodes, hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize_q, dim3(nblk(nodes, 256)), dim3(256), 0, st, accQ, accW, accS, inv_scale, cq0, cq1,
                       cs0, cs1, Q, nodes);
}

void launch_harmonic(const long long *accJ, double cj0, double cj1, const double *ec, const double *es,
                     const Orders &o, double *I, double *Jc, double *Jcc, double *Js, double *Jsc, double *partial,
                     HarmState *h, const double *Qk, const double *vc, const double *vs, int nturns, int nodes,
                     hipStream_t st)
{
    const int nb = (int)nblk(nodes, 256);
    hipLaunchKernelGGL(k_harmonic, dim3(nb), dim3(256), 0, st, accJ, cj0, cj1, ec, es, o, I, Jc, Jcc, Js, Jsc,
                       partial, nodes);
    hipLaunchKernelGGL(k_harmonic_fold, dim3(1), dim3(256), 0, st, partial, nb, o, h, Qk, vc, vs, nturns);
}

int harmonic_blocks(int nodes) { return (int)nblk(nodes, 256); }

static unsigned mg_grid(int work) { return nblk(work, 256) < 2048 ? nblk(work, 256) : 2048; }
static unsigned red_grid(int work) { return nblk(work, 256) < 1024 ? nblk(work, 256) : 1024; }

static int smooth_tiles(const MGLevel &L)
{
    return ((L.nz + 1 + TILE_Z - 1) / TILE_Z) * ((L.nr1 + TILE_R - 1) / TILE_R);
}
int smooth_blocks(const MGLevel &L) { return smooth_tiles(L); }
int pcg_partial_size(const MGLevel &L0)
{
    const int t = smooth_tiles(L0), r = (int)red_grid(L0.nodes);
    return 2 * (t > r ? t : r);
}
void launch_mg_smooth_tile(const MGLevel &L, const MGLevel *F, const MGLevel *C, int sweeps, int mode,
                           const MGState *st, double *partial, double *out, hipStream_t s)
{
    const MGLevel none{};
    hipLaunchKernelGGL(k_mg_smooth_tile, dim3(smooth_tiles(L)), dim3(256), 0, s, L, F ? *F : none, C ? *C : none,
                       sweeps, mode, st, partial, out);
}
void launch_mg_resid(const MGLevel &L, const MGState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_mg_resid, dim3(mg_grid(L.nodes)), dim3(256), 0, s, L, st);
}
void launch_mg_restrict_res(const MGLevel &F, const MGLevel &C, const MGState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_mg_restrict_res, dim3(mg_grid(C.nodes)), dim3(256), 0, s, F, C, st);
}
int dense_ld(int n) { return n + (n & 1); }
int dense_ld32(int n) { return (n + 3) & ~3; }
void launch_dense_solve(const float *inv, const MGLevel &L, const MGState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_dense_solve, dim3(nblk(L.nodes, 4)), dim3(256), 0, s, inv, dense_ld32(L.nodes), L, st);
}
void launch_inverse_f32(const double *inv, int n, float *out, hipStream_t s)
{
    const int64_t total = (int64_t)n * dense_ld32(n);
    hipLaunchKernelGGL(k_inverse_f32, dim3(std::min<int64_t>(nblk(total, 256), 4096)), dim3(256), 0, s, inv, n,
                       dense_ld(n), out, dense_ld32(n));
}
void launch_gauss_jordan(double *A, int n, double *rowk, double *colk, hipStream_t s)
{
    const int ld = dense_ld(n);
    for (int k = 0; k < n; ++k) {
        hipLaunchKernelGGL(k_gj_save, dim3(nblk(n, 256)), dim3(256), 0, s, A, n, ld, k, rowk, colk);
        hipLaunchKernelGGL(k_gj_update, dim3(nblk((int64_t)n * n, 256)), dim3(256), 0, s, A, n, ld, k, rowk, colk);
    }
}
int pcg_blocks(int nodes) { return (int)red_grid(nodes); }
void launch_pcg_begin(const MGLevel &L, const PCGVec &v, const int32_t *tag, const double *vc, const double *vs,
                      const Orders &o, MGState *st, double *prev, int order, hipStream_t s, const double *basis,
                      int nturns)
{
    hipLaunchKernelGGL(k_pcg_begin, dim3(nblk(L.nodes, 256)), dim3(256), 0, s, L, v, tag, vc, vs, o, st, prev, order,
                       basis, nturns);
}
void launch_pcg_resid(const MGLevel &L, const PCGVec &v, double *partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_resid, dim3(red_grid(L.nodes)), dim3(256), 0, s, L, v, partial);
}
void launch_pcg_check(MGState *st, const double *partial, int np, double rtol, bool first, hipStream_t s,
                      unsigned long long *unconv)
{
    hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(256), 0, s, st, partial, np, rtol, first ? 1 : 0, unconv);
}
void launch_pcg_rz(const MGLevel &L, const PCGVec &v, const MGState *st, double *partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_rz, dim3(red_grid(L.nodes)), dim3(256), 0, s, L, v, st, partial);
}
void launch_pcg_pmatvec(const MGLevel &L, const PCGVec &v, const double *pold, double *pnew, MGState *st,
                        double *partial, int nrz, hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_pmatvec, dim3(red_grid(L.nodes)), dim3(256), 0, s, L, v, pold, pnew, st, partial, nrz);
}
void launch_pcg_update(const MGLevel &L, const PCGVec &v, const double *p, const MGState *st, double *partial,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_update, dim3(red_grid(L.nodes)), dim3(256), 0, s, L, v, p, st, partial,
                       (int)red_grid(L.nodes));
}
void launch_face_charge(const double *phi, const int32_t *fp, const int32_t *fq, const int32_t *fk, const double *fc,
                        int nfaces, double *Qk, int nturns, hipStream_t s, const double *chi)
{
    hipLaunchKernelGGL(k_face_charge, dim3(1), dim3(64 * (nturns > 0 ? nturns : 1)), 0, s, phi, fp, fq, fk, fc, nfaces,
                       Qk, nturns, chi);
}

}  // namespace pic
