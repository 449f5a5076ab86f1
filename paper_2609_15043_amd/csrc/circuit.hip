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
// integral of the node's weight (node_volume).
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
    b[n] = -mw * (j * g.dr) * (scale * (acc[n] + comp[n])) / node_volume(g, i, j);
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
//         turn potentials and field);
// mode 3: finalise and measure only (the surrogate stages follow).
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

// Shared memory of one network solve.
struct NetSmem {
    double Are[MAX_X][MAX_X], Aim[MAX_X][MAX_X];
    double bre[MAX_X], bim[MAX_X];
    int piv;
};

// The whole workgroup solves A x = b (Eq. blockmatrix) for source V_g and
// loads (icap, vp) by Gaussian elimination with partial pivoting (largest
// |re| + |im|); thread 0 writes x.  Returns false (every thread) when
// singular.
__device__ bool network_solve(const CircuitDev &c, Cx vg, const double *icap_re, const double *icap_im,
                              const double *vp_re, const double *vp_im, double *x_re, double *x_im, NetSmem &S)
{
    const int t = threadIdx.x, N = c.N, M = 2 * N + 1;
    for (int e = t; e < M * M; e += blockDim.x) {
        const int r = e / M, col = e - r * M;
        const Cx v = net_entry(c, r, col);
        S.Are[r][col] = v.re;
        S.Aim[r][col] = v.im;
    }
    for (int r = t; r < M; r += blockDim.x) {
        Cx v{0.0, 0.0};
        if (r == 0)
            v = vg;
        else if (r <= N)
            v = {icap_re[r - 1], icap_im[r - 1]};
        else
            v = {vp_re[r - 1 - N], vp_im[r - 1 - N]};
        S.bre[r] = v.re;
        S.bim[r] = v.im;
    }
    __syncthreads();
    for (int col = 0; col < M; ++col) {
        if (t == 0) {
            int p = col;
            double best = cabs1({S.Are[col][col], S.Aim[col][col]});
            for (int r = col + 1; r < M; ++r) {
                const double m = cabs1({S.Are[r][col], S.Aim[r][col]});
                if (m > best) {
                    best = m;
                    p = r;
                }
            }
            S.piv = best > 0.0 ? p : -1;
        }
        __syncthreads();
        const int p = S.piv;
        if (p < 0) return false;
        if (p != col) {
            for (int k = t; k < M; k += blockDim.x) {
                double x = S.Are[p][k];
                S.Are[p][k] = S.Are[col][k];
                S.Are[col][k] = x;
                x = S.Aim[p][k];
                S.Aim[p][k] = S.Aim[col][k];
                S.Aim[col][k] = x;
            }
            if (t == 0) {
                double x = S.bre[p];
                S.bre[p] = S.bre[col];
                S.bre[col] = x;
                x = S.bim[p];
                S.bim[p] = S.bim[col];
                S.bim[col] = x;
            }
        }
        __syncthreads();
        const Cx d{S.Are[col][col], S.Aim[col][col]};
        for (int r = col + 1 + t; r < M; r += blockDim.x) {
            const Cx f = cdiv({S.Are[r][col], S.Aim[r][col]}, d);
            for (int k = col + 1; k < M; ++k) {
                const Cx u = csub({S.Are[r][k], S.Aim[r][k]}, cmul(f, {S.Are[col][k], S.Aim[col][k]}));
                S.Are[r][k] = u.re;
                S.Aim[r][k] = u.im;
            }
            const Cx u = csub({S.bre[r], S.bim[r]}, cmul(f, {S.bre[col], S.bim[col]}));
            S.bre[r] = u.re;
            S.bim[r] = u.im;
            S.Are[r][col] = 0.0;
            S.Aim[r][col] = 0.0;
        }
        __syncthreads();
    }
    if (t == 0) {
        Cx x[MAX_X];
        for (int r = M - 1; r >= 0; --r) {
            Cx s{S.bre[r], S.bim[r]};
            for (int k = r + 1; k < M; ++k) s = csub(s, cmul({S.Are[r][k], S.Aim[r][k]}, x[k]));
            x[r] = cdiv(s, {S.Are[r][r], S.Aim[r][r]});
        }
        for (int r = 0; r < M; ++r) {
            x_re[r] = x[r].re;
            x_im[r] = x[r].im;
        }
    }
    __syncthreads();
    return true;
}

// max residuals of state x against source vg and loads (Eqs. kclres, kvlres)
__device__ void network_residuals(CircuitDev &c, Cx vg, const double *icap_re, const double *icap_im,
                                  const double *vp_re, const double *vp_im)
{
    const int N = c.N, M = 2 * N + 1;
    double rk = 0.0, rv = 0.0;
    for (int r = 0; r < M; ++r) {
        Cx s{0.0, 0.0};
        if (r == 0)
            s = vg;
        else if (r <= N)
            s = {icap_re[r - 1], icap_im[r - 1]};
        else
            s = {vp_re[r - 1 - N], vp_im[r - 1 - N]};
        for (int k = 0; k < M; ++k) s = csub(s, cmul(net_entry(c, r, k), {c.x_re[k], c.x_im[k]}));
        const double m = sqrt(s.re * s.re + s.im * s.im);
        if (r >= 1 && r <= N)
            rk = fmax(rk, m);
        else
            rv = fmax(rv, m);
    }
    const double is = sqrt(c.x_re[0] * c.x_re[0] + c.x_im[0] * c.x_im[0]);
    c.kcl = rk / (is > 0.0 ? is : 1.0);
    c.kvl = rv / sqrt(vg.re * vg.re + vg.im * vg.im);
}

// period finalisation (Eqs. fourier, icap, pind, pcap, pcap_phasor), thread 0
__device__ void finalize_period(CircuitDev &c, const HarmState *h, const double *vc, const double *vs)
{
    const int N = c.N;
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

// loads of the completed period (Eq. vpind) and its powers (Eqs. pport,
// pbalance, power_imbalance), thread 0.  Prescribed loads (a circuit
// override) replace the measured V_p and I_cap; the powers stay measured.
__device__ void measure_period(CircuitDev &c)
{
    const int N = c.N;
    for (int k = 0; k < N; ++k) {
        c.vp_re[k] = -c.proj[2 * k];
        c.vp_im[k] = -c.proj[2 * k + 1];
    }
    if (c.ovr_loads) {
        for (int k = 0; k < N; ++k) {
            c.vp_re[k] = c.ovr_vp_re[k];
            c.vp_im[k] = c.ovr_vp_im[k];
            c.icap_re[k] = c.ovr_icap_re[k];
            c.icap_im[k] = c.ovr_icap_im[k];
        }
        c.ovr_loads = 0;
    }
    c.p_port = 0.5 * (c.x_re[1 + N] * c.x_re[0] + c.x_im[1 + N] * c.x_im[0]);
    double pcu = 0.0;
    for (int k = 0; k < N; ++k) pcu += 0.5 * c.rrf[k] * (c.x_re[1 + k] * c.x_re[1 + k] + c.x_im[1 + k] * c.x_im[1 + k]);
    c.p_cu = pcu;
    const double bal = c.p_ind + c.p_cap + pcu;
    c.eps_bal = c.p_port != 0.0 ? fabs(c.p_port - bal) / fabs(c.p_port) : INFINITY;
    c.vg_old = c.vg_amp;
}

// filtered, trend-extrapolated power controller (Eqs. pfilter, ptrend,
// pcontrol, limiter, bounds) fed with the measured port power p; thread 0
__device__ void controller_step(CircuitDev &c, double p)
{
    if (!c.controller) return;
    const double prev = c.have_pf ? c.pf_prev : p;
    const double pf = c.gamma * p + (1.0 - c.gamma) * prev;
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

__device__ __forceinline__ Cx vg_phasor(const CircuitDev &c, double amp)
{
    return {amp * cos(c.vg_phase), amp * sin(c.vg_phase)};
}

// relaxation (Eq. relaxation) of the applied state towards the target, then
// the residuals against the loads used; thread 0
__device__ void relax_and_check(CircuitDev &c, const double *icap_re, const double *icap_im, const double *vp_re,
                                const double *vp_im)
{
    const int M = 2 * c.N + 1;
    for (int r = 0; r < M; ++r) {
        c.x_re[r] = (1.0 - c.alpha) * c.x_re[r] + c.alpha * c.xt_re[r];
        c.x_im[r] = (1.0 - c.alpha) * c.x_im[r] + c.alpha * c.xt_im[r];
    }
    network_residuals(c, vg_phasor(c, c.vg_amp), icap_re, icap_im, vp_re, vp_im);
}

__device__ void write_turn_potentials(const CircuitDev &c, double *vc, double *vs)
{
    for (int k = 0; k < c.N; ++k) {
        vc[k] = c.x_re[1 + c.N + k];
        vs[k] = -c.x_im[1 + c.N + k];
    }
}

__global__ __launch_bounds__(64) void k_circuit(CircuitDev *cdp, const HarmState *h, double *vc, double *vs,
                                                int mode)
{
    __shared__ NetSmem S;
    const int t = threadIdx.x;
    CircuitDev &c = *cdp;
    const int N = c.N, M = 2 * N + 1;
    if (t == 0 && mode != 0) finalize_period(c, h, vc, vs);
    if (mode == 2) return;
    if (t == 0 && (mode == 1 || mode == 3)) measure_period(c);
    if (mode == 3) return;
    if (t == 0 && mode == 1) controller_step(c, c.p_port);
    __syncthreads();
    if (mode == 0) {
        // first state: zero load responses; with the target-power start the
        // network is solved for V_g = 1 and scaled (it is linear in V_g)
        __shared__ double zero[MAX_TURNS];
        if (t < MAX_TURNS) zero[t] = 0.0;
        __syncthreads();
        const double a = c.vg_from_target ? 1.0 : c.vg_amp;
        if (!network_solve(c, vg_phasor(c, a), zero, zero, zero, zero, c.xt_re, c.xt_im, S)) {
            if (t == 0) c.singular = 1;
            return;
        }
        if (t != 0) return;
        double scale = 1.0;
        if (c.vg_from_target) {
            const double p1 = 0.5 * (c.xt_re[1 + N] * c.xt_re[0] + c.xt_im[1 + N] * c.xt_im[0]);
            c.vg_amp = sqrt(c.p_target / p1);
            scale = c.vg_amp;
        }
        for (int r = 0; r < M; ++r) {
            c.x_re[r] = c.xt_re[r] = scale * c.xt_re[r];
            c.x_im[r] = c.xt_im[r] = scale * c.xt_im[r];
        }
        double num = 0.0, den = 0.0;   // Eq. reciprocity
        for (int k = 0; k < N; ++k)
            for (int l = 0; l < N; ++l) {
                num = fmax(num, fabs(c.mvac[k * MAX_TURNS + l] - c.mvac[l * MAX_TURNS + k]));
                den = fmax(den, fabs(c.mvac[k * MAX_TURNS + l]));
            }
        c.eps_rec = den > 0.0 ? num / den : 0.0;
        write_turn_potentials(c, vc, vs);
        return;
    }
    // mode 1: target network solve with this period's loads, relaxation
    if (!network_solve(c, vg_phasor(c, c.vg_amp), c.icap_re, c.icap_im, c.vp_re, c.vp_im, c.xt_re, c.xt_im, S)) {
        if (t == 0) c.singular = 1;
        return;
    }
    if (t != 0) return;
    relax_and_check(c, c.icap_re, c.icap_im, c.vp_re, c.vp_im);
    write_turn_potentials(c, vc, vs);
}

// ---------------------------------------------------------------------------
// Surrogate-assisted update.  y = (V_p, I_cap) measured over the completed
// period; yhat(x) the network's prediction for circuit state x.
// stage 0: prediction at x^n -> correction y - yhat(x^n) and its scaled
//          error (V_p by |V_g|, I_cap by |I_f|); above err_max the plain
//          update runs here instead (controller, target solve, relaxation);
//          else the inner iteration starts at x^n.
// stage 1: one inner step: loads yhat(x_i) + correction, controller on the
//          iterate's port power (limited to the period's step bounds),
//          target solve, relaxation; converged when the step is below
//          tol |x|.
// stage 2: the converged iterate becomes the applied state; an iterate
//          that ran away from the period's state (|x_i|^2 > 1e6 |x^n|^2
//          or non-finite) is discarded for the plain update.
// ---------------------------------------------------------------------------
__device__ void features(const CircuitDev &c, const double *xr, const double *xi, float *f)
{
    const int N = c.N;
    for (int k = 0; k < N; ++k) {
        f[2 * k] = (float)xr[1 + k];
        f[2 * k + 1] = (float)xi[1 + k];
        f[2 * N + 2 * k] = (float)xr[1 + N + k];
        f[2 * N + 2 * k + 1] = (float)xi[1 + N + k];
    }
    f[4 * N] = (float)c.pressure;
    for (int m = 0; m < 8; ++m) f[4 * N + 1 + m] = (float)c.moments[m];
}

__global__ void k_features(const CircuitDev *cd, float *f, int iterate)
{
    if (threadIdx.x != 0) return;
    const CircuitDev &c = *cd;
    if (iterate && c.sur_done) return;
    features(c, iterate ? c.xi_re : c.x_re, iterate ? c.xi_im : c.x_im, f);
}

__global__ __launch_bounds__(64) void k_surrogate(CircuitDev *cdp, const float *pred, double *vc, double *vs, int stage)
{
    __shared__ NetSmem S;
    __shared__ double lre[MAX_TURNS], lim[MAX_TURNS], vre[MAX_TURNS], vim[MAX_TURNS];
    __shared__ int mode;   // 0 plain fallback, 1 inner step, -1 nothing
    const int t = threadIdx.x;
    CircuitDev &c = *cdp;
    const int N = c.N, M = 2 * N + 1;
    if (t == 0) {
        mode = -1;
        if (stage == 0) {
            const double sv = sqrt(c.vg_amp * c.vg_amp), si = sqrt(c.x_re[0] * c.x_re[0] + c.x_im[0] * c.x_im[0]);
            double num = 0.0, den = 0.0;
            for (int k = 0; k < N; ++k) {
                const double y[4] = {c.vp_re[k], c.vp_im[k], c.icap_re[k], c.icap_im[k]};
                const double yh[4] = {pred[2 * k], pred[2 * k + 1], pred[2 * N + 2 * k], pred[2 * N + 2 * k + 1]};
                for (int q = 0; q < 4; ++q) {
                    const double sc = q < 2 ? 1.0 / (sv > 0.0 ? sv : 1.0) : 1.0 / (si > 0.0 ? si : 1.0);
                    num += (yh[q] - y[q]) * (yh[q] - y[q]) * sc * sc;
                    den += y[q] * y[q] * sc * sc;
                }
                c.sur_corr[2 * k] = c.vp_re[k] - yh[0];
                c.sur_corr[2 * k + 1] = c.vp_im[k] - yh[1];
                c.sur_corr[2 * N + 2 * k] = c.icap_re[k] - yh[2];
                c.sur_corr[2 * N + 2 * k + 1] = c.icap_im[k] - yh[3];
            }
            c.sur_err = den > 0.0 ? sqrt(num / den) : INFINITY;
            c.sur_iters = 0;
            c.sur_step = 0.0;
            if (!(c.sur_err <= c.sur_err_max)) {
                c.sur_used = 0;
                c.sur_done = 1;
                controller_step(c, c.p_port);
                mode = 0;
            } else {
                c.sur_used = 1;
                c.sur_done = 0;
                for (int r = 0; r < M; ++r) {
                    c.xi_re[r] = c.x_re[r];
                    c.xi_im[r] = c.x_im[r];
                    c.xa_re[r] = 0.0;
                    c.xa_im[r] = 0.0;
                }
                c.vg_iter = c.vg_amp;
                c.vg_acc = 0.0;
                c.sur_navg = 0;
            }
        } else if (stage == 1 && !c.sur_done) {
            mode = 1;
            for (int k = 0; k < N; ++k) {
                vre[k] = pred[2 * k] + c.sur_corr[2 * k];
                vim[k] = pred[2 * k + 1] + c.sur_corr[2 * k + 1];
                lre[k] = pred[2 * N + 2 * k] + c.sur_corr[2 * N + 2 * k];
                lim[k] = pred[2 * N + 2 * k + 1] + c.sur_corr[2 * N + 2 * k + 1];
            }
            if (c.controller) {
                // port power of the iterate; the amplitude stays within the
                // period's controller bounds
                const double pp = 0.5 * (c.xi_re[1 + N] * c.xi_re[0] + c.xi_im[1 + N] * c.xi_im[0]);
                const double pc = fmax(pp, c.eps_p), v = c.vg_iter;
                double vn = v + c.alpha_v * (v * sqrt(c.p_target / pc) - v);
                vn = fmin(fmax(vn, (1.0 - c.f_step) * c.vg_old), (1.0 + c.f_step) * c.vg_old);
                c.vg_iter = fmin(fmax(vn, c.v_min), c.v_max);
            }
        }
    }
    __syncthreads();
    if (mode == 0) {
        // plain update with the measured loads
        if (!network_solve(c, vg_phasor(c, c.vg_amp), c.icap_re, c.icap_im, c.vp_re, c.vp_im, c.xt_re, c.xt_im, S)) {
            if (t == 0) c.singular = 1;
            return;
        }
        if (t != 0) return;
        relax_and_check(c, c.icap_re, c.icap_im, c.vp_re, c.vp_im);
        write_turn_potentials(c, vc, vs);
        return;
    }
    if (mode == 1) {
        if (!network_solve(c, vg_phasor(c, c.vg_iter), lre, lim, vre, vim, c.xt_re, c.xt_im, S)) {
            if (t == 0) {
                c.singular = 1;
                c.sur_done = 1;
            }
            return;
        }
        if (t != 0) return;
        double dn = 0.0, xn = 0.0;
        for (int r = 0; r < M; ++r) {
            const double nr = (1.0 - c.alpha) * c.xi_re[r] + c.alpha * c.xt_re[r];
            const double ni = (1.0 - c.alpha) * c.xi_im[r] + c.alpha * c.xt_im[r];
            dn += (nr - c.xi_re[r]) * (nr - c.xi_re[r]) + (ni - c.xi_im[r]) * (ni - c.xi_im[r]);
            xn += nr * nr + ni * ni;
            c.xi_re[r] = nr;
            c.xi_im[r] = ni;
        }
        c.sur_iters += 1;
        c.sur_step = sqrt(dn / (xn > 0.0 ? xn : 1.0));
        if (c.sur_iters <= SUR_MAX_ITER) c.sur_hist[c.sur_iters - 1] = c.sur_step;
        // an iterate far outside the period's state means the predicted load
        // map does not contract here: the plain update runs instead
        double x0 = 0.0;
        for (int r = 0; r < M; ++r) x0 += c.x_re[r] * c.x_re[r] + c.x_im[r] * c.x_im[r];
        if (!(c.sur_step < 1e300) || xn > 1e6 * x0) {
            c.sur_used = 2;
            c.sur_done = 1;
        }
        if (c.sur_step < c.sur_tol || c.sur_iters >= c.sur_max_iter) c.sur_done = 1;
        // BF16 activations make the predicted loads a step function of the
        // state: iterates that circle the fixed point instead of settling
        // on it are averaged over the second half
        if (c.sur_used == 1 && !(c.sur_step < c.sur_tol) && c.sur_iters > c.sur_max_iter / 2) {
            for (int r = 0; r < M; ++r) {
                c.xa_re[r] += c.xi_re[r];
                c.xa_im[r] += c.xi_im[r];
            }
            c.vg_acc += c.vg_iter;
            c.sur_navg += 1;
        }
        return;
    }
    if (stage == 2 && c.sur_used == 2) {
        // diverged inner iteration: plain update with the measured loads
        if (t == 0) controller_step(c, c.p_port);
        __syncthreads();
        if (!network_solve(c, vg_phasor(c, c.vg_amp), c.icap_re, c.icap_im, c.vp_re, c.vp_im, c.xt_re, c.xt_im, S)) {
            if (t == 0) c.singular = 1;
            return;
        }
        if (t != 0) return;
        relax_and_check(c, c.icap_re, c.icap_im, c.vp_re, c.vp_im);
        write_turn_potentials(c, vc, vs);
        c.sur_used = 0;
        return;
    }
    if (stage == 2 && t == 0 && c.sur_used == 1) {
        // the last iterate when it met the tolerance, else the mean of the
        // second half's iterates
        const bool mean = !(c.sur_step < c.sur_tol) && c.sur_navg > 0;
        const double na = mean ? (double)c.sur_navg : 1.0;
        for (int r = 0; r < M; ++r) {
            c.x_re[r] = mean ? c.xa_re[r] / na : c.xi_re[r];
            c.x_im[r] = mean ? c.xa_im[r] / na : c.xi_im[r];
        }
        c.vg_amp = mean ? c.vg_acc / na : c.vg_iter;
        // the filter restarts from the port power of the new state
        c.pf_prev = 0.5 * (c.x_re[1 + N] * c.x_re[0] + c.x_im[1 + N] * c.x_im[0]);
        c.have_pf = 1;
        // residuals against the loads the iterate converged with
        double vre2[MAX_TURNS], vim2[MAX_TURNS], lre2[MAX_TURNS], lim2[MAX_TURNS];
        for (int k = 0; k < N; ++k) {
            vre2[k] = pred[2 * k] + c.sur_corr[2 * k];
            vim2[k] = pred[2 * k + 1] + c.sur_corr[2 * k + 1];
            lre2[k] = pred[2 * N + 2 * k] + c.sur_corr[2 * N + 2 * k];
            lim2[k] = pred[2 * N + 2 * k + 1] + c.sur_corr[2 * N + 2 * k + 1];
        }
        network_residuals(c, vg_phasor(c, c.vg_amp), lre2, lim2, vre2, vim2);
        write_turn_potentials(c, vc, vs);
    }
}

// ---------------------------------------------------------------------------
// Multiharmonic circuit: the same network at every retained order m (its
// own record cd[m - 1]: impedances at m w, vacuum coupling from the unit
// fields of order m, loads from the order-m harmonics).  The source of order
// m is V_g,m = rho_m exp(i phi_m) V_g with the fundamental's amplitude V_g;
// the controller acts on the total port power.
// mode 0: first states with zero load responses; with the target-power
//         start V_g puts p_target into the vacuum networks together (they
//         are linear in V_g: solved for V_g = 1, then scaled);
// mode 1: after every order's finalisation and measurement (k_circuit
//         mode 3): totals, controller, each order's target solve,
//         relaxation and residuals.
// Turn potentials of order m go to vc / vs + (m - 1) MAX_TURNS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double port_power(const CircuitDev &c, const double *xr, const double *xi)
{
    return 0.5 * (xr[1 + c.N] * xr[0] + xi[1 + c.N] * xi[0]);
}

__global__ __launch_bounds__(64) void k_circuit_orders(CircuitDev *cd, int M, double *vc, double *vs, int mode)
{
    __shared__ NetSmem S;
    __shared__ double zero[MAX_TURNS];
    const int t = threadIdx.x;
    CircuitDev &f = cd[0];
    const int N = f.N, X = 2 * N + 1;
    if (mode == 0) {
        if (t < MAX_TURNS) zero[t] = 0.0;
        __syncthreads();
        const double base = f.vg_from_target ? 1.0 : f.vg_amp;
        double p1 = 0.0;
        for (int m = 0; m < M; ++m) {
            CircuitDev &c = cd[m];
            if (!network_solve(c, vg_phasor(c, base * c.vg_ratio), zero, zero, zero, zero, c.xt_re, c.xt_im, S)) {
                if (t == 0) f.singular = c.singular = 1;
                return;
            }
            if (t == 0) p1 += port_power(c, c.xt_re, c.xt_im);
        }
        if (t != 0) return;
        double scale = 1.0;
        if (f.vg_from_target) {
            f.vg_amp = sqrt(f.p_target / p1);
            scale = f.vg_amp;
        }
        for (int m = 0; m < M; ++m) {
            CircuitDev &c = cd[m];
            if (m > 0) c.vg_amp = f.vg_amp * c.vg_ratio;
            for (int r = 0; r < X; ++r) {
                c.x_re[r] = c.xt_re[r] = scale * c.xt_re[r];
                c.x_im[r] = c.xt_im[r] = scale * c.xt_im[r];
            }
            double num = 0.0, den = 0.0;   // Eq. reciprocity, per order
            for (int k = 0; k < N; ++k)
                for (int l = 0; l < N; ++l) {
                    num = fmax(num, fabs(c.mvac[k * MAX_TURNS + l] - c.mvac[l * MAX_TURNS + k]));
                    den = fmax(den, fabs(c.mvac[k * MAX_TURNS + l]));
                }
            c.eps_rec = den > 0.0 ? num / den : 0.0;
            write_turn_potentials(c, vc + m * MAX_TURNS, vs + m * MAX_TURNS);
        }
        return;
    }
    if (t == 0) {
        double pp = 0.0, pcu = 0.0;
        for (int m = 0; m < M; ++m) {
            pp += cd[m].p_port;
            pcu += cd[m].p_cu;
        }
        f.tot_p_port = pp;
        f.tot_p_cu = pcu;
        controller_step(f, pp);
        for (int m = 1; m < M; ++m) cd[m].vg_amp = f.vg_amp * cd[m].vg_ratio;
    }
    __syncthreads();
    for (int m = 0; m < M; ++m) {
        CircuitDev &c = cd[m];
        if (!network_solve(c, vg_phasor(c, c.vg_amp), c.icap_re, c.icap_im, c.vp_re, c.vp_im, c.xt_re, c.xt_im, S)) {
            if (t == 0) f.singular = c.singular = 1;
            return;
        }
        if (t == 0) {
            relax_and_check(c, c.icap_re, c.icap_im, c.vp_re, c.vp_im);
            write_turn_potentials(c, vc + m * MAX_TURNS, vs + m * MAX_TURNS);
        }
        __syncthreads();
    }
    if (t != 0) return;
    // totals: the time-domain P_ind and P_cap of any order's accumulator
    // are those of the whole waveform (the fundamental's record holds them)
    double pph = 0.0, kcl = 0.0, kvl = 0.0;
    for (int m = 0; m < M; ++m) {
        pph += cd[m].p_cap_ph;
        kcl = fmax(kcl, cd[m].kcl);
        kvl = fmax(kvl, cd[m].kvl);
    }
    f.tot_p_cap_ph = pph;
    f.tot_kcl = kcl;
    f.tot_kvl = kvl;
    const double bal = f.p_ind + f.p_cap + f.tot_p_cu;
    f.tot_eps_bal = f.tot_p_port != 0.0 ? fabs(f.tot_p_port - bal) / fabs(f.tot_p_port) : INFINITY;
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
void launch_features(const CircuitDev *cd, float *f, bool iterate, hipStream_t s)
{
    hipLaunchKernelGGL(k_features, dim3(1), dim3(64), 0, s, cd, f, iterate ? 1 : 0);
}
void launch_surrogate(CircuitDev *cd, const float *pred, double *vc, double *vs, int stage, hipStream_t s)
{
    hipLaunchKernelGGL(k_surrogate, dim3(1), dim3(64), 0, s, cd, pred, vc, vs, stage);
}
void launch_circuit_orders(CircuitDev *cd, int M, double *vc, double *vs, int mode, hipStream_t s)
{
    hipLaunchKernelGGL(k_circuit_orders, dim3(1), dim3(64), 0, s, cd, M, vc, vs, mode);
}
void launch_compose(const double *ecp, const double *esp, const double *U, int64_t stride, const CircuitDev *cd,
                    double *ec, double *es, int nodes, hipStream_t s)
{
    hipLaunchKernelGGL(k_compose, dim3(nb256(nodes)), dim3(256), 0, s, ecp, esp, U, stride, cd, ec, es, nodes);
}

}  // namespace pic
