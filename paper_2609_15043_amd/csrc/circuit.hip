// Field-circuit coupling kernels: right-hand sides of the inductive
// (Helmholtz) solves, port projections, the closed-period circuit update
// (harmonic finalisation, power controller, (2N+1) complex network solve,
// relaxation, residuals) and the composition of the next period's
// azimuthal field.  FP64 throughout.
#include "kernels.h"
#include "launch.h"

namespace pic {

// ---------------------------------------------------------------------------
// Inductive operator in symmetric form.  The five-point finite-difference
// L u = u_zz + u_RR + u_R / R - u / R^2 + k^2 u (Eq. helmholtz_op) becomes
// symmetric after multiplying row j by R_j:
//   R_j (-L u) = R_j (2/dz^2 + 2/dR^2 + 1/R_j^2 - k^2) u - R_j/dz^2 (u_S + u_N)
//                - (R_j + dR/2)/dR^2 u_E - (R_j - dR/2)/dR^2 u_W,
// so K u = src (K = L / (mu0 w)) is solved as A_H u = -mu0 w R_j src with the
// same preconditioned-CG / multigrid machinery as the Poisson problem.
// ---------------------------------------------------------------------------

// b = -mu0 w R_j (scale (acc + comp)) / V_node on free nodes; V_node is the
// node's control volume clipped to the domain.
__global__ void k_helm_rhs(const double *acc, const double *comp, double scale, const uint8_t *dir, double mw,
                           double *b, GridC g)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.nodes) return;
    if (dir[n]) {
        b[n] = 0.0;
        return;
    }
    const int i = n / g.nr1, j = n - i * g.nr1;
    const double R = j * g.dr;
    const double lo = fmax(R - 0.5 * g.dr, 0.0), hi = fmin(R + 0.5 * g.dr, g.nr * g.dr);
    const double zl = fmax((i - 0.5) * g.dz, 0.0), zh = fmin((i + 0.5) * g.dz, g.nz * g.dz);
    const double vol = 3.141592653589793 * (hi * hi - lo * lo) * (zh - zl);
    b[n] = -mw * R * (scale * (acc[n] + comp[n])) / vol;
}

// b = -mu0 w R_j g_k on the nodes of turn k (tag k + 1), 0 elsewhere
__global__ void k_unit_rhs(const int32_t *tag, int turn, double gval, const uint8_t *dir, double mw, double *b,
                           GridC g)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.nodes) return;
    const int j = n % g.nr1;
    b[n] = (!dir[n] && tag[n] == turn + 1) ? -mw * (j * g.dr) * gval : 0.0;
}

// out[k * ostride + f] = sum over the nodes of turn k of g_k F_f 2 pi R dz dR
// (Eqs. zvac, vpind).  One thread per (turn, field) pair, nodes in list
// order, so the sums are reproducible.
__global__ void k_project(const double *fields, int nf, int64_t stride, const int32_t *list, const int32_t *lturn,
                          int nlist, const double *gval, int nturns, double *out, int ostride, GridC g)
{
    const int t = threadIdx.x;
    if (t >= nturns * nf) return;
    const int k = t / nf, f = t - k * nf;
    const double *F = fields + (int64_t)f * stride;
    double s = 0.0;
    for (int e = 0; e < nlist; ++e) {
        if (lturn[e] != k) continue;
        const int n = list[e];
        const int j = n % g.nr1;
        s += F[n] * (6.283185307179586 * (j * g.dr) * g.dz * g.dr);
    }
    out[k * ostride + f] = gval[k] * s;
}

// ---------------------------------------------------------------------------
// Closed-period circuit update in one workgroup.
// mode 0: first state (zero load responses), Z_vac reciprocity;
// mode 1: finalise the period's harmonics and powers, controller, target
//         network solve, relaxation, residuals;
// mode 2: finalise the period's harmonics and powers only (prescribed
//         turn potentials and field).
// New turn potentials V_c = Re V_k, V_s = -Im V_k go to vc / vs.
// ---------------------------------------------------------------------------
struct Cx {
    double re, im;
};
__device__ __forceinline__ Cx cmul(Cx a, Cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ Cx csub(Cx a, Cx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ Cx cdiv(Cx a, Cx b)
{
    // scaled division (Smith's method) to keep intermediate products in range
    if (fabs(b.re) >= fabs(b.im)) {
        const double r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    }
    const double r = b.re / b.im, d = b.re * r + b.im;
    return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
__device__ __forceinline__ double cabs1(Cx a) { return fabs(a.re) + fabs(a.im); }

// entry (r, col) of the network matrix (Eq. blockmatrix)
__device__ Cx net_entry(const CircuitDev &c, int r, int col)
{
    const int N = c.N;
    Cx v{0.0, 0.0};
    if (r == 0) {
        if (col == 0) v = {c.zs_re, c.zs_im};
        if (col == 1 + N) v.re = 1.0;
        return v;
    }
    if (r <= N) {   // KCL of node k
        const int k = r - 1;
        if (col == (k == 0 ? 0 : k)) v.re += 1.0;            // I_in,k
        if (col == 1 + k) v.re -= 1.0;                       // -I_k
        if (col == 1 + N + k) v.im -= c.omega * c.cstray[k];
        return v;
    }
    const int k = r - 1 - N;   // KVL of segment k
    if (col >= 1 && col <= N) {
        const int l = col - 1;
        // -Z_turn,kl = -(R_rf,k delta_kl - i mvac_kl)
        v.re = -(k == l ? c.rrf[k] : 0.0);
        v.im = c.mvac[k * MAX_TURNS + l];
    }
    if (col == 1 + N + k) v.re += 1.0;
    if (col == 2 + N + k && k + 1 < N) v.re -= 1.0;
    return v;
}

__global__ __launch_bounds__(64) void k_circuit(CircuitDev *cdp, const HarmState *h, double *vc, double *vs,
                                                int mode)
{
    __shared__ double Are[MAX_X][MAX_X], Aim[MAX_X][MAX_X];
    __shared__ double bre[MAX_X], bim[MAX_X];
    __shared__ int piv;
    const int t = threadIdx.x;
    CircuitDev &c = *cdp;
    const int N = c.N, M = 2 * N + 1;

    if (t == 0 && mode != 0) {
        // period finalisation (Eqs. fourier, icap, pind, pcap, pcap_phasor)
        const double two_n = 2.0 / c.nrf;
        double wsum = 0.0, pph = 0.0;
        for (int k = 0; k < N; ++k) {
            const double qc = two_n * (h->qc[k] + h->qc_c[k]), qs = two_n * (h->qs[k] + h->qs_c[k]);
            c.qc[k] = qc;
            c.qs[k] = qs;
            c.icap_re[k] = c.omega * qs;
            c.icap_im[k] = c.omega * qc;
            const double Wk = (h->w[k] + h->w_c[k]) + 0.5 * (h->v_first[k] + h->v_prev[k]) * (h->q_first[k] - h->q_prev[k]);
            c.wk[k] = Wk;
            wsum += Wk;
            // 1/2 Re(V conj(I_cap)) with V = V_c - i V_s
            pph += 0.5 * (vc[k] * c.icap_re[k] - vs[k] * c.icap_im[k]);
        }
        c.samples = h->samples;
        c.p_ind = (h->pind + h->pind_c) / c.nrf;
        c.p_cap = c.freq * wsum;
        c.p_cap_ph = pph;
    }
    if (mode == 2) return;

    if (t == 0 && mode == 1) {
        // loads of the completed period (Eq. vpind) and its powers (Eqs. pport, pbalance)
        for (int k = 0; k < N; ++k) {
            c.vp_re[k] = -c.proj[2 * k];
            c.vp_im[k] = -c.proj[2 * k + 1];
        }
        c.p_port = 0.5 * (c.x_re[1 + N] * c.x_re[0] + c.x_im[1 + N] * c.x_im[0]);
        double pcu = 0.0;
        for (int k = 0; k < N; ++k) pcu += 0.5 * c.rrf[k] * (c.x_re[1 + k] * c.x_re[1 + k] + c.x_im[1 + k] * c.x_im[1 + k]);
        c.p_cu = pcu;
        const double bal = c.p_ind + c.p_cap + pcu;
        c.eps_bal = c.p_port != 0.0 ? fabs(c.p_port - bal) / fabs(c.p_port) : INFINITY;
        c.vg_old = c.vg_amp;
        if (c.controller) {   // Eqs. pfilter, ptrend, pcontrol, limiter, bounds
            const double prev = c.have_pf ? c.pf_prev : c.p_port;
            const double pf = c.gamma * c.p_port + (1.0 - c.gamma) * prev;
            const double pc = fmax(pf + c.n_trend * (pf - prev), c.eps_p);
            const double vold = c.vg_amp;
            double vn = vold + c.alpha_v * (vold * sqrt(c.p_target / pc) - vold);
            vn = fmin(fmax(vn, (1.0 - c.f_step) * vold), (1.0 + c.f_step) * vold);
            vn = fmin(fmax(vn, c.v_min), c.v_max);
            c.vg_amp = vn;
            c.pf_prev = pf;
            c.have_pf = 1;
            c.pf = pf;
            c.pc = pc;
        }
    }
    __syncthreads();

    // assemble the network and its right-hand side
    const Cx vg1{cos(c.vg_phase), sin(c.vg_phase)};
    for (int e = t; e < M * M; e += blockDim.x) {
        const int r = e / M, col = e - r * M;
        const Cx v = net_entry(c, r, col);
        Are[r][col] = v.re;
        Aim[r][col] = v.im;
    }
    for (int r = t; r < M; r += blockDim.x) {
        Cx v{0.0, 0.0};
        if (r == 0) {
            // init with the target-power start solves for V_g = 1 first
            const double a = (mode == 0 && c.vg_from_target) ? 1.0 : c.vg_amp;
            v = {a * vg1.re, a * vg1.im};
        } else if (mode == 1 && r <= N) {
            v = {c.icap_re[r - 1], c.icap_im[r - 1]};
        } else if (mode == 1) {
            v = {c.vp_re[r - 1 - N], c.vp_im[r - 1 - N]};
        }
        bre[r] = v.re;
        bim[r] = v.im;
    }
    __syncthreads();

    // Gaussian elimination with partial pivoting (largest |re| + |im|)
    for (int col = 0; col < M; ++col) {
        if (t == 0) {
            int p = col;
            double best = cabs1({Are[col][col], Aim[col][col]});
            for (int r = col + 1; r < M; ++r) {
                const double m = cabs1({Are[r][col], Aim[r][col]});
                if (m > best) {
                    best = m;
                    p = r;
                }
            }
            piv = best > 0.0 ? p : -1;
            if (best == 0.0) c.singular = 1;
        }
        __syncthreads();
        const int p = piv;
        if (p < 0) return;
        if (p != col) {
            for (int k = t; k < M; k += blockDim.x) {
                double x = Are[p][k];
                Are[p][k] = Are[col][k];
                Are[col][k] = x;
                x = Aim[p][k];
                Aim[p][k] = Aim[col][k];
                Aim[col][k] = x;
            }
            if (t == 0) {
                double x = bre[p];
                bre[p] = bre[col];
                bre[col] = x;
                x = bim[p];
                bim[p] = bim[col];
                bim[col] = x;
            }
        }
        __syncthreads();
        // multipliers of the rows below, then the row updates
        const Cx d{Are[col][col], Aim[col][col]};
        for (int r = col + 1 + t; r < M; r += blockDim.x) {
            const Cx f = cdiv({Are[r][col], Aim[r][col]}, d);
            for (int k = col + 1; k < M; ++k) {
                const Cx u = csub({Are[r][k], Aim[r][k]}, cmul(f, {Are[col][k], Aim[col][k]}));
                Are[r][k] = u.re;
                Aim[r][k] = u.im;
            }
            const Cx u = csub({bre[r], bim[r]}, cmul(f, {bre[col], bim[col]}));
            bre[r] = u.re;
            bim[r] = u.im;
            Are[r][col] = 0.0;
            Aim[r][col] = 0.0;
        }
        __syncthreads();
    }
    if (t != 0) return;
    Cx x[MAX_X];
    for (int r = M - 1; r >= 0; --r) {
        Cx s{bre[r], bim[r]};
        for (int k = r + 1; k < M; ++k) s = csub(s, cmul({Are[r][k], Aim[r][k]}, x[k]));
        x[r] = cdiv(s, {Are[r][r], Aim[r][r]});
    }
    if (mode == 0) {
        if (c.vg_from_target) {
            // linear network: x(V_g) = V_g x(1); P_port scales with V_g^2
            const double p1 = 0.5 * (x[1 + N].re * x[0].re + x[1 + N].im * x[0].im);
            c.vg_amp = sqrt(c.p_target / p1);
            for (int r = 0; r < M; ++r) x[r] = {c.vg_amp * x[r].re, c.vg_amp * x[r].im};
        }
        for (int r = 0; r < M; ++r) {
            c.x_re[r] = c.xt_re[r] = x[r].re;
            c.x_im[r] = c.xt_im[r] = x[r].im;
        }
        double num = 0.0, den = 0.0;   // Eq. reciprocity
        for (int k = 0; k < N; ++k)
            for (int l = 0; l < N; ++l) {
                num = fmax(num, fabs(c.mvac[k * MAX_TURNS + l] - c.mvac[l * MAX_TURNS + k]));
                den = fmax(den, fabs(c.mvac[k * MAX_TURNS + l]));
            }
        c.eps_rec = den > 0.0 ? num / den : 0.0;
    } else {
        // relaxation (Eq. relaxation)
        for (int r = 0; r < M; ++r) {
            c.xt_re[r] = x[r].re;
            c.xt_im[r] = x[r].im;
            c.x_re[r] = (1.0 - c.alpha) * c.x_re[r] + c.alpha * x[r].re;
            c.x_im[r] = (1.0 - c.alpha) * c.x_im[r] + c.alpha * x[r].im;
        }
        // residuals of the new state against this period's loads (Eqs. kclres, kvlres)
        double rk = 0.0, rv = 0.0;
        for (int r = 0; r < M; ++r) {
            Cx s{0.0, 0.0};
            if (r == 0) s = {c.vg_amp * vg1.re, c.vg_amp * vg1.im};
            else if (r <= N) s = {c.icap_re[r - 1], c.icap_im[r - 1]};
            else s = {c.vp_re[r - 1 - N], c.vp_im[r - 1 - N]};
            for (int k = 0; k < M; ++k) s = csub(s, cmul(net_entry(c, r, k), {c.x_re[k], c.x_im[k]}));
            const double m = sqrt(s.re * s.re + s.im * s.im);
            if (r >= 1 && r <= N) rk = fmax(rk, m);
            else rv = fmax(rv, m);
        }
        const double is = sqrt(c.x_re[0] * c.x_re[0] + c.x_im[0] * c.x_im[0]);
        c.kcl = rk / (is > 0.0 ? is : 1.0);
        c.kvl = rv / c.vg_amp;
    }
    for (int k = 0; k < N; ++k) {
        vc[k] = c.x_re[1 + N + k];
        vs[k] = -c.x_im[1 + N + k];
    }
}

// E_c = E_c^p + sum I_s,k U_k, E_s^sto = E_s^sto,p + sum I_c,k U_k with
// I_k = I_c,k - i I_s,k of the applied state (Eq. compose)
__global__ void k_compose(const double *ecp, const double *esp, const double *U, int64_t stride,
                          const CircuitDev *cd, double *ec, double *es, int nodes)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nodes) return;
    double a = ecp[n], b = esp[n];
    const int N = cd->N;
    for (int k = 0; k < N; ++k) {
        const double u = U[(int64_t)k * stride + n];
        a += -cd->x_im[1 + k] * u;
        b += cd->x_re[1 + k] * u;
    }
    ec[n] = a;
    es[n] = b;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

void launch_helm_rhs(const double *acc, const double *comp, double scale, const uint8_t *dir, double mw, double *b,
                     const GridC &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_helm_rhs, dim3(nb256(g.nodes)), dim3(256), 0, s, acc, comp, scale, dir, mw, b, g);
}
void launch_unit_rhs(const int32_t *tag, int turn, double gval, const uint8_t *dir, double mw, double *b,
                     const GridC &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_unit_rhs, dim3(nb256(g.nodes)), dim3(256), 0, s, tag, turn, gval, dir, mw, b, g);
}
void launch_project(const double *fields, int nf, int64_t stride, const int32_t *list, const int32_t *lturn, int nlist,
                    const double *gval, int nturns, double *out, int ostride, const GridC &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_project, dim3(1), dim3(256), 0, s, fields, nf, stride, list, lturn, nlist, gval, nturns, out,
                       ostride, g);
}
void launch_circuit(CircuitDev *cd, const HarmState *h, double *vc, double *vs, int mode, hipStream_t s)
{
    hipLaunchKernelGGL(k_circuit, dim3(1), dim3(64), 0, s, cd, h, vc, vs, mode);
}
void launch_compose(const double *ecp, const double *esp, const double *U, int64_t stride, const CircuitDev *cd,
                    double *ec, double *es, int nodes, hipStream_t s)
{
    hipLaunchKernelGGL(k_compose, dim3(nb256(nodes)), dim3(256), 0, s, ecp, esp, U, stride, cd, ec, es, nodes);
}

}  // namespace pic
