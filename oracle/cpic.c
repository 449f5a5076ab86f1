/*
 * Plain FP64 CPU oracle for the particle part of the axisymmetric (z, R)
 * PIC/MCC step: loading, gather, Boris push with the cylindrical move,
 * azimuthal current deposit, null-collision Monte Carlo collisions and the
 * charge deposit.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the HIP kernels are
 * checked against; it shares no code with them and nothing in the product
 * path may call it.  It is deliberately slow and literal: one loop over
 * particles per operation, absolute positions (R, z) in metres, FP64
 * throughout.
 *
 * What it follows (paper: Chen et al., phasor-PIC for bidirectional circuit
 * coupling of ICPs):
 *   - E_theta(t_n) is rebuilt from the two stored arrays with the phase
 *     theta_n = 2 pi (n mod N_RF) / N_RF (Sec. 2.1, Eq. et_reconstruct);
 *     the caller passes the node values already rebuilt.
 *   - The particle modules themselves are inherited by the paper from earlier
 *     PIC/MCC work and not written out there (Sec. 2.1, first paragraph);
 *     the readings used here are the textbook ones: volume (R^2-linear)
 *     radial weights, leapfrog/Boris kick, Cartesian
 *     move + rotation back to (r, theta), null-collision MCC with Philox
 *     counters keyed by (particle id, step).
 */
#define _USE_MATH_DEFINES
#include <math.h>
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from the     */
/* published description: 10 rounds of two 32x32->64 multiplies with a    */
/* Weyl-sequence key schedule.                                             */
/* ---------------------------------------------------------------------- */
#define PHILOX_MUL_A 0xD2511F53u
#define PHILOX_MUL_B 0xCD9E8D57u
#define PHILOX_WEYL_A 0x9E3779B9u
#define PHILOX_WEYL_B 0xBB67AE85u

void ora_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL_A;
            k1 += PHILOX_WEYL_B;
        }
        uint64_t pa = (uint64_t)PHILOX_MUL_A * (uint64_t)c[0];
        uint64_t pb = (uint64_t)PHILOX_MUL_B * (uint64_t)c[2];
        uint32_t n0 = (uint32_t)(pb >> 32) ^ c[1] ^ k0;
        uint32_t n1 = (uint32_t)pb;
        uint32_t n2 = (uint32_t)(pa >> 32) ^ c[3] ^ k1;
        uint32_t n3 = (uint32_t)pa;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    memcpy(out, c, sizeof c);
}

/* n blocks, counters given row-wise (n x 4) */
void ora_philox_many(int64_t n, const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out)
{
    uint32_t key[2] = {k0, k1};
    for (int64_t p = 0; p < n; ++p) ora_philox4x32_10(ctr + 4 * p, key, out + 4 * p);
}

/* one block for particle `id` of species `sp` at step `n`, purpose `use` */
static void draw(uint32_t seed, int sp, uint32_t id, uint32_t n, uint32_t use, uint32_t out[4])
{
    uint32_t ctr[4] = {id, n, use, 0u};
    uint32_t key[2] = {seed, (uint32_t)sp};
    ora_philox4x32_10(ctr, key, out);
}

/* uniform on the open interval (0, 1) */
static double u01(uint32_t x) { return ((double)x + 0.5) / 4294967296.0; }

/* two standard normals from two uniforms (Box-Muller) */
static void box_muller(uint32_t a, uint32_t b, double *g0, double *g1)
{
    double r = sqrt(-2.0 * log(u01(a)));
    double t = 2.0 * M_PI * u01(b);
    *g0 = r * cos(t);
    *g1 = r * sin(t);
}

/* isotropic unit vector, (r, theta, z) components */
static void iso_dir(uint32_t a, uint32_t b, double d[3])
{
    double ct = 1.0 - 2.0 * u01(a);
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double ph = 2.0 * M_PI * u01(b);
    d[0] = st * cos(ph);
    d[1] = st * sin(ph);
    d[2] = ct;
}

/* Gap to the next null-collision candidate.  Candidates of one particle
 * form a Bernoulli process in the step index with probability P per step,
 * so the gaps are i.i.d. Geometric(P) on {1, 2, ...}:
 * G = 1 + floor(log(u) / log(1 - P)), with lq = log(1 - P) < 0. */
static int64_t geo_gap(uint32_t x, double lq)
{
    double g = floor(log(u01(x)) / lq);
    if (g > 2.0e9) g = 2.0e9;
    return 1 + (int64_t)g;
}

static int32_t clamp_step(int64_t s) { return s > 2147483647 ? 2147483647 : (int32_t)s; }

/* ---------------------------------------------------------------------- */
/* Geometry and parameters                                                 */
/* ---------------------------------------------------------------------- */
typedef struct {
    int32_t nr, nz;      /* cells in R and z */
    int32_t ip;          /* node row of the top of the particle region */
    int32_t window;      /* 1: charge leaving through z = zp stays on that row */
    double dr, dz, rmax, zp;
} ora_grid;

typedef struct {
    double q, m, w, dt;  /* charge, mass, macro weight, time step */
    double b[3];         /* uniform magnetic field (B_r, B_theta, B_z) */
} ora_species;

typedef struct {
    int32_t kind;        /* 0 analytic fits, 1 constant */
    double el_a, el_b, exc_a, exc_th, iz_a, iz_th;
    double iel_a, iel_p, icx_a, icx_p;
    double e_cap_ev, i_gcap, nu_margin;
} ora_xs;

typedef struct {
    double ngas;         /* neutral density (m^-3) */
    double tgas_ev;      /* neutral temperature (eV) */
    double qe;           /* elementary charge (eV <-> J) */
    double me, mi;       /* electron and ion (= neutral) mass */
} ora_gas;

static int64_t node(const ora_grid *g, int i, int j) { return (int64_t)i * (g->nr + 1) + j; }

/* Radial index and R^2-linear weight of the upper node; axial index and
 * linear weight of the upper node. */
static void weights(const ora_grid *g, double R, double z, int *j, int *i, double *wr1, double *wz1)
{
    int jj = (int)floor(R / g->dr);
    int ii = (int)floor(z / g->dz);
    if (jj > g->nr - 1) jj = g->nr - 1;
    if (jj < 0) jj = 0;
    if (ii > g->nz - 1) ii = g->nz - 1;
    if (ii < 0) ii = 0;
    double r0 = jj * g->dr, r1 = (jj + 1) * g->dr;
    *wr1 = (R * R - r0 * r0) / (r1 * r1 - r0 * r0);
    *wz1 = (z - ii * g->dz) / g->dz;
    *j = jj;
    *i = ii;
}

/* ---------------------------------------------------------------------- */
/* Loading: uniform in volume, Maxwellian velocities                       */
/* ---------------------------------------------------------------------- */
/* next[p]: the first null-collision candidate step, G - 1 from word 2 of
 * the second load block (lq = log(1 - P_null) of this species). */
void ora_load(int64_t n, uint32_t seed, int sp, double rmax, double zlo, double zhi, double vth,
              double lq, double *R, double *z, double *vr, double *vt, double *vz, uint32_t *id,
              int32_t *next)
{
    for (int64_t p = 0; p < n; ++p) {
        uint32_t a[4], b[4];
        draw(seed, sp, (uint32_t)p, 0u, 0u, a);
        draw(seed, sp, (uint32_t)p, 0u, 1u, b);
        R[p] = rmax * sqrt(u01(a[0]));
        z[p] = zlo + (zhi - zlo) * u01(a[1]);
        double g0, g1, g2, g3;
        box_muller(a[2], a[3], &g0, &g1);
        box_muller(b[0], b[1], &g2, &g3);
        vr[p] = vth * g0;
        vt[p] = vth * g1;
        vz[p] = vth * g2;
        id[p] = (uint32_t)p;
        next[p] = clamp_step(geo_gap(b[2], lq) - 1);
    }
}

/* ---------------------------------------------------------------------- */
/* Gather + Boris push + move + J_theta deposit + absorption               */
/* ---------------------------------------------------------------------- */
/*
 * alive[p]: 1 live, 0 dead (skipped).  On output, particles that left the
 * particle region get alive = 0; absorbed[p] tells where: 1 wall, 2 window.
 * Inode accumulates q w vbar_theta W_node(x^n) (vbar = mean of the two half
 * step velocities in the frame at x^n); surf accumulates the charge left on
 * the window row.  Br, Bz (nullable): node values of the RF magnetic field
 * at t_n, gathered with the same weights and added to the uniform field of
 * the species block in the Boris rotation.
 */
void ora_gather_push(const ora_grid *g, const ora_species *s, int64_t n,
                     double *R, double *z, double *vr, double *vt, double *vz,
                     int32_t *alive, int32_t *absorbed,
                     const double *Er, const double *Ez, const double *Et,
                     const double *Br, const double *Bz,
                     double *Inode, double *surf)
{
    const double qm = s->q / s->m;
    const double h = 0.5 * qm * s->dt;
    const double tv[3] = {h * s->b[0], h * s->b[1], h * s->b[2]};
    const double t2 = tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2];
    const double sv[3] = {2 * tv[0] / (1 + t2), 2 * tv[1] / (1 + t2), 2 * tv[2] / (1 + t2)};
    const double qw = s->q * s->w;
    for (int64_t p = 0; p < n; ++p) {
        absorbed[p] = 0;
        if (!alive[p]) continue;
        int j, i;
        double wr1, wz1;
        weights(g, R[p], z[p], &j, &i, &wr1, &wz1);
        const double W[4] = {(1 - wz1) * (1 - wr1), (1 - wz1) * wr1, wz1 * (1 - wr1), wz1 * wr1};
        const int64_t nd[4] = {node(g, i, j), node(g, i, j + 1), node(g, i + 1, j), node(g, i + 1, j + 1)};
        double e[3] = {0, 0, 0};
        for (int k = 0; k < 4; ++k) {
            e[0] += W[k] * Er[nd[k]];
            e[1] += W[k] * Et[nd[k]];
            e[2] += W[k] * Ez[nd[k]];
        }
        /* rotation vector t = (q/m) B dt / 2 and s = 2 t / (1 + t^2) */
        double tp[3] = {tv[0], tv[1], tv[2]}, sp[3] = {sv[0], sv[1], sv[2]};
        double tt = t2;
        if (Br && Bz) {
            double b[2] = {0, 0};
            for (int k = 0; k < 4; ++k) {
                b[0] += W[k] * Br[nd[k]];
                b[1] += W[k] * Bz[nd[k]];
            }
            tp[0] = h * (s->b[0] + b[0]);
            tp[2] = h * (s->b[2] + b[1]);
            tt = tp[0] * tp[0] + tp[1] * tp[1] + tp[2] * tp[2];
            for (int c = 0; c < 3; ++c) sp[c] = 2 * tp[c] / (1 + tt);
        }
        /* half kick, rotation, half kick: (r, theta, z) right-handed */
        double v[3] = {vr[p] + h * e[0], vt[p] + h * e[1], vz[p] + h * e[2]};
        if (tt > 0) {
            double c1[3] = {v[1] * tp[2] - v[2] * tp[1], v[2] * tp[0] - v[0] * tp[2], v[0] * tp[1] - v[1] * tp[0]};
            double vp[3] = {v[0] + c1[0], v[1] + c1[1], v[2] + c1[2]};
            double c2[3] = {vp[1] * sp[2] - vp[2] * sp[1], vp[2] * sp[0] - vp[0] * sp[2], vp[0] * sp[1] - vp[1] * sp[0]};
            v[0] += c2[0]; v[1] += c2[1]; v[2] += c2[2];
        }
        v[0] += h * e[0];
        v[1] += h * e[1];
        v[2] += h * e[2];
        /* azimuthal current at x^n with the time-centred v_theta */
        const double vbar = 0.5 * (vt[p] + v[1]);
        for (int k = 0; k < 4; ++k) Inode[nd[k]] += qw * vbar * W[k];
        /* Cartesian move in the plane through the particle, then rotate
         * the velocity back to the local (r, theta) frame */
        const double X = R[p] + v[0] * s->dt;
        const double Y = v[1] * s->dt;
        const double znew = z[p] + v[2] * s->dt;
        const double Rnew = sqrt(X * X + Y * Y);
        double c = 1.0, sn = 0.0;
        if (Rnew > 0) { c = X / Rnew; sn = Y / Rnew; }
        const double vrn = c * v[0] + sn * v[1];
        const double vtn = -sn * v[0] + c * v[1];
        int out = 0;
        if (znew < 0) {
            out = 1;
        } else if (znew >= g->zp) {
            out = 1;
            if (g->window) {
                const double ts = (g->zp - z[p]) / v[2];
                const double xs = R[p] + v[0] * ts, ys = v[1] * ts;
                const double Rs = sqrt(xs * xs + ys * ys);
                if (Rs < g->rmax) {
                    int js = (int)floor(Rs / g->dr);
                    if (js > g->nr - 1) js = g->nr - 1;
                    const double r0 = js * g->dr, r1 = (js + 1) * g->dr;
                    const double w1 = (Rs * Rs - r0 * r0) / (r1 * r1 - r0 * r0);
                    surf[node(g, g->ip, js)] += qw * (1 - w1);
                    surf[node(g, g->ip, js + 1)] += qw * w1;
                    out = 2;
                }
            }
        } else if (Rnew >= g->rmax) {
            out = 1;
        }
        R[p] = Rnew;
        z[p] = znew;
        vr[p] = vrn;
        vt[p] = vtn;
        vz[p] = v[2];
        if (out) {
            alive[p] = 0;
            absorbed[p] = out;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Ion-induced secondary electron emission at the grounded metal walls     */
/* (the inherited GEC module the paper names without its yields; read here */
/* as a constant yield per absorbed ion and a flux-weighted Maxwellian      */
/* electron).  For the m absorbed ions given in ascending id order, at     */
/* their positions before the step's move (R0, z0) and with the wall they  */
/* crossed (1 bottom z = 0, 2 top z = zp without a window, 3 outer         */
/* R = rmax), block (id, n, 4, 0) of the ion stream decides the emission,  */
/* u0 < gamma, and draws the electron's velocity: normal speed             */
/* sigma sqrt(-2 ln u1) into the domain (the normal component of a         */
/* Maxwellian flux through the wall), two tangential components            */
/* sigma sqrt(-2 ln u2) (cos, sin)(2 pi u3), sigma = sqrt(T e / m_e).      */
/* Block (id, n, 5, 0) draws the electron's first collision candidate      */
/* n + G.  Emitted electrons are written in order; returns their count.    */
/* ---------------------------------------------------------------------- */
int64_t ora_see(uint32_t seed, uint32_t n, double gamma, double sigma, double lq_e, int64_t m,
                const uint32_t *id, const double *R0, const double *z0, const int32_t *wall,
                double *R, double *z, double *v, int32_t *next)
{
    int64_t k = 0;
    for (int64_t p = 0; p < m; ++p) {
        uint32_t b[4], c[4];
        draw(seed, 1, id[p], n, 4u, b);
        if (!(u01(b[0]) < gamma)) continue;
        const double vn = sigma * sqrt(-2.0 * log(u01(b[1])));
        const double rt = sigma * sqrt(-2.0 * log(u01(b[2])));
        const double t1 = rt * cos(2.0 * M_PI * u01(b[3])), t2 = rt * sin(2.0 * M_PI * u01(b[3]));
        double *o = v + 3 * k;
        if (wall[p] == 1) {          /* bottom: +z */
            o[0] = t1; o[1] = t2; o[2] = vn;
        } else if (wall[p] == 2) {   /* top: -z */
            o[0] = t1; o[1] = t2; o[2] = -vn;
        } else {                     /* outer: -R */
            o[0] = -vn; o[1] = t1; o[2] = t2;
        }
        draw(seed, 1, id[p], n, 5u, c);
        next[k] = clamp_step((int64_t)n + geo_gap(c[0], lq_e));
        R[k] = R0[p];
        z[k] = z0[p];
        ++k;
    }
    return k;
}

/* ---------------------------------------------------------------------- */
/* Charge deposit at the current positions                                 */
/* ---------------------------------------------------------------------- */
void ora_deposit(const ora_grid *g, int64_t n, const double *R, const double *z,
                 const int32_t *alive, double qw, double *Qnode)
{
    for (int64_t p = 0; p < n; ++p) {
        if (!alive[p]) continue;
        int j, i;
        double wr1, wz1;
        weights(g, R[p], z[p], &j, &i, &wr1, &wz1);
        Qnode[node(g, i, j)] += qw * (1 - wz1) * (1 - wr1);
        Qnode[node(g, i, j + 1)] += qw * (1 - wz1) * wr1;
        Qnode[node(g, i + 1, j)] += qw * wz1 * (1 - wr1);
        Qnode[node(g, i + 1, j + 1)] += qw * wz1 * wr1;
    }
}

/* ---------------------------------------------------------------------- */
/* Cross sections                                                          */
/* ---------------------------------------------------------------------- */
static double threshold_shape(double eps, double th)
{
    if (eps <= th) return 0.0;
    double x = eps / th;
    return 4.0 * (x - 1.0) / (x * x);
}

/* electron: sig[0] elastic, sig[1] excitation, sig[2] ionization (m^2) */
void ora_sigma_e(const ora_xs *x, double eps, double sig[3])
{
    if (x->kind == 1) {
        sig[0] = x->el_a;
        sig[1] = eps > x->exc_th ? x->exc_a : 0.0;
        sig[2] = eps > x->iz_th ? x->iz_a : 0.0;
        return;
    }
    sig[0] = x->el_a / sqrt(1.0 + eps / x->el_b);
    sig[1] = x->exc_a * threshold_shape(eps, x->exc_th);
    sig[2] = x->iz_a * threshold_shape(eps, x->iz_th);
}

/* ion: sig[0] elastic, sig[1] charge exchange, at centre-of-mass energy */
void ora_sigma_i(const ora_xs *x, double ecm, double sig[2])
{
    if (x->kind == 1) {
        sig[0] = x->iel_a;
        sig[1] = x->icx_a;
        return;
    }
    sig[0] = x->iel_a * pow(1.0 + ecm, -x->iel_p);
    sig[1] = x->icx_a * pow(1.0 + ecm, -x->icx_p);
}

/* Maximum total collision frequency over the scanned range (times the
 * margin), the null-collision probability per step and log(1 - P).
 * out_nu[2], out_p[2], out_lq[2] for (electron, ion). */
void ora_null_setup(const ora_xs *x, const ora_gas *gs, double dt, int64_t nscan,
                    double *out_nu, double *out_p, double *out_lq)
{
    double best_e = 0.0, best_i = 0.0;
    for (int64_t k = 0; k <= nscan; ++k) {
        double eps = x->e_cap_ev * (double)k / (double)nscan;
        double sig[3];
        ora_sigma_e(x, eps, sig);
        double v = sqrt(2.0 * eps * gs->qe / gs->me);
        double nu = gs->ngas * (sig[0] + sig[1] + sig[2]) * v;
        if (nu > best_e) best_e = nu;
        double gg = x->i_gcap * (double)k / (double)nscan;
        double ecm = 0.25 * gs->mi * gg * gg / gs->qe;
        double si[2];
        ora_sigma_i(x, ecm, si);
        double nui = gs->ngas * (si[0] + si[1]) * gg;
        if (nui > best_i) best_i = nui;
    }
    out_nu[0] = best_e * x->nu_margin;
    out_nu[1] = best_i * x->nu_margin;
    for (int s = 0; s < 2; ++s) {
        out_p[s] = -expm1(-out_nu[s] * dt);
        out_lq[s] = -out_nu[s] * dt;   /* log(1 - P) = -nu_max dt exactly */
    }
}

/* ---------------------------------------------------------------------- */
/* Null-collision MCC on v^{n+1/2}                                          */
/* ---------------------------------------------------------------------- */
/*
 * A particle is a candidate at step n iff next[p] == n; its block
 * (id, n, 1, 0) then gives the next gap from word x0 (next = n + G).
 *
 * Electron-neutral (neutral at rest): at a candidate,
 * R = u(x1) nu_max against the cumulative nu_el, nu_exc, nu_iz; every real
 * collision picks an isotropic lab direction from (x2, x3).  Ionization
 * shares eps - E_iz uniformly (block purpose 2, word 0), the secondary's
 * direction uses words 1, 2 of that block and the new ion is a neutral
 * Maxwellian from block purpose 3.
 *
 * Ion-neutral: neutral velocity from block purpose 2 (Box-Muller of words
 * 0,1 and 2,3); at a candidate R = u(x1) nu_max against nu_el,
 * nu_cx with g = |v_i - v_n|; charge exchange takes the neutral velocity,
 * elastic scattering is isotropic in the centre-of-mass frame.
 *
 * counts[0..3]: candidates, process 1, process 2, process 3 (ions: no 3rd);
 * counts[4]: candidates whose total frequency exceeded nu_max.
 * Births (electrons only) go to the b_* arrays, at most bcap of them; a
 * newborn's first candidate is step + G with G from word 3 of block
 * purpose 2 (electron, lq_e) or 3 (ion, lq_i).  Returns the number of
 * births or -1 on overflow.
 */
int64_t ora_mcc(int sp, uint32_t seed, uint32_t step, const ora_xs *x, const ora_gas *gs,
                double numax, double lq, double lq_ion, int64_t n,
                const double *R, const double *z, double *vr, double *vt, double *vz,
                const uint32_t *id, const int32_t *alive, int32_t *next,
                int64_t bcap, uint32_t *b_parent, double *b_R, double *b_z,
                double *b_ve, double *b_vi, int32_t *b_next, int64_t *counts)
{
    int64_t nb = 0;
    const double vg = sqrt(gs->tgas_ev * gs->qe / gs->mi);
    for (int64_t p = 0; p < n; ++p) {
        if (!alive[p]) continue;
        if (next[p] != (int32_t)step) continue;
        uint32_t b0[4];
        draw(seed, sp, id[p], step, 1u, b0);
        next[p] = clamp_step((int64_t)step + geo_gap(b0[0], lq));
        counts[0]++;
        double v[3] = {vr[p], vt[p], vz[p]};
        if (sp == 0) {
            double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            double speed = sqrt(v2);
            double eps = 0.5 * gs->me * v2 / gs->qe;
            double sig[3];
            ora_sigma_e(x, eps, sig);
            double nu_el = gs->ngas * sig[0] * speed;
            double nu_ex = gs->ngas * sig[1] * speed;
            double nu_iz = gs->ngas * sig[2] * speed;
            if (nu_el + nu_ex + nu_iz > numax) counts[4]++;
            double Rv = u01(b0[1]) * numax;
            double d[3];
            iso_dir(b0[2], b0[3], d);
            if (Rv < nu_el) {
                counts[1]++;
                double cchi = speed > 0 ? (v[0] * d[0] + v[1] * d[1] + v[2] * d[2]) / speed : 1.0;
                double e1 = eps * (1.0 - 2.0 * gs->me / gs->mi * (1.0 - cchi));
                double s1 = sqrt(2.0 * e1 * gs->qe / gs->me);
                vr[p] = s1 * d[0]; vt[p] = s1 * d[1]; vz[p] = s1 * d[2];
            } else if (Rv < nu_el + nu_ex) {
                counts[2]++;
                double e1 = eps - x->exc_th;
                double s1 = sqrt(2.0 * e1 * gs->qe / gs->me);
                vr[p] = s1 * d[0]; vt[p] = s1 * d[1]; vz[p] = s1 * d[2];
            } else if (Rv < nu_el + nu_ex + nu_iz) {
                counts[3]++;
                uint32_t b2[4], b3[4];
                draw(seed, sp, id[p], step, 2u, b2);
                draw(seed, sp, id[p], step, 3u, b3);
                double erem = eps - x->iz_th;
                double esec = u01(b2[0]) * erem;
                double epri = erem - esec;
                double s1 = sqrt(2.0 * epri * gs->qe / gs->me);
                vr[p] = s1 * d[0]; vt[p] = s1 * d[1]; vz[p] = s1 * d[2];
                if (nb >= bcap) return -1;
                double d2[3];
                iso_dir(b2[1], b2[2], d2);
                double s2 = sqrt(2.0 * esec * gs->qe / gs->me);
                double g0, g1, g2, g3;
                box_muller(b3[0], b3[1], &g0, &g1);
                box_muller(b3[2], b3[3], &g2, &g3);
                b_parent[nb] = id[p];
                b_R[nb] = R[p];
                b_z[nb] = z[p];
                b_ve[3 * nb + 0] = s2 * d2[0];
                b_ve[3 * nb + 1] = s2 * d2[1];
                b_ve[3 * nb + 2] = s2 * d2[2];
                b_vi[3 * nb + 0] = vg * g0;
                b_vi[3 * nb + 1] = vg * g1;
                b_vi[3 * nb + 2] = vg * g2;
                b_next[2 * nb + 0] = clamp_step((int64_t)step + geo_gap(b2[3], lq));
                b_next[2 * nb + 1] = clamp_step((int64_t)step + geo_gap(b3[3], lq_ion));
                nb++;
            }
        } else {
            uint32_t b2[4];
            draw(seed, sp, id[p], step, 2u, b2);
            double g0, g1, g2, g3;
            box_muller(b2[0], b2[1], &g0, &g1);
            box_muller(b2[2], b2[3], &g2, &g3);
            double vn[3] = {vg * g0, vg * g1, vg * g2};
            double gv[3] = {v[0] - vn[0], v[1] - vn[1], v[2] - vn[2]};
            double gm = sqrt(gv[0] * gv[0] + gv[1] * gv[1] + gv[2] * gv[2]);
            double ecm = 0.25 * gs->mi * gm * gm / gs->qe;
            double sig[2];
            ora_sigma_i(x, ecm, sig);
            double nu_el = gs->ngas * sig[0] * gm;
            double nu_cx = gs->ngas * sig[1] * gm;
            if (nu_el + nu_cx > numax) counts[4]++;
            double Rv = u01(b0[1]) * numax;
            if (Rv < nu_el) {
                counts[1]++;
                double d[3];
                iso_dir(b0[2], b0[3], d);
                for (int c = 0; c < 3; ++c) v[c] = 0.5 * (v[c] + vn[c]) + 0.5 * gm * d[c];
                vr[p] = v[0]; vt[p] = v[1]; vz[p] = v[2];
            } else if (Rv < nu_el + nu_cx) {
                counts[2]++;
                vr[p] = vn[0]; vt[p] = vn[1]; vz[p] = vn[2];
            }
        }
    }
    return nb;
}

/* ---------------------------------------------------------------------- */
/* Direct-implicit step (the paper's electrostatic scheme, Sec. 2.3, after */
/* Langdon, Cohen & Friedman's direct implicit method; the paper inherits  */
/* the particle update and does not write it out).  The D1 time filter is  */
/* used: with a = (q/m) E_es,                                              */
/*   v^{n+1/2} = v^{n-1/2} + (dt/2) (a^{n+1} + abar^{n-1})                 */
/*               + dt (q/m) E_theta(t_n) theta_hat,                        */
/*   abar^n    = (a^{n+1} + abar^{n-1}) / 2,  x^{n+1} = x^n + dt v^{n+1/2}.*/
/* The predictor moves with everything but a^{n+1} (positions x~, whose    */
/* charge and susceptibility the implicit field solve uses); the corrector */
/* adds (dt^2/2) a^{n+1}(x~) to the position and (dt/2) a^{n+1}(x~) to the */
/* velocity.  abar is a 3-vector in the particle's local (r, theta, z)     */
/* frame and turns with the velocity when the move rotates that frame.     */
/* No magnetic field in this mode.                                         */
/* ---------------------------------------------------------------------- */
static void window_charge(const ora_grid *g, double Rs, double qw, double *surf)
{
    int js = (int)floor(Rs / g->dr);
    if (js > g->nr - 1) js = g->nr - 1;
    const double r0 = js * g->dr, r1 = (js + 1) * g->dr;
    const double w1 = (Rs * Rs - r0 * r0) / (r1 * r1 - r0 * r0);
    surf[node(g, g->ip, js)] += qw * (1 - w1);
    surf[node(g, g->ip, js + 1)] += qw * w1;
}

/* Predictor of step n: kick by (dt/2) abar and the inductive field, J_theta
 * at x^n with the time-centred v_theta, Cartesian move to x~ with v and abar
 * turned into the new frame, absorption and window charge as in the
 * explicit push. */
void ora_di_predict(const ora_grid *g, const ora_species *s, int64_t n,
                    double *R, double *z, double *vr, double *vt, double *vz,
                    double *ar, double *at, double *az,
                    int32_t *alive, int32_t *absorbed, const double *Et,
                    double *Inode, double *surf)
{
    const double h = 0.5 * s->q / s->m * s->dt;
    const double qw = s->q * s->w;
    for (int64_t p = 0; p < n; ++p) {
        absorbed[p] = 0;
        if (!alive[p]) continue;
        int j, i;
        double wr1, wz1;
        weights(g, R[p], z[p], &j, &i, &wr1, &wz1);
        const double W[4] = {(1 - wz1) * (1 - wr1), (1 - wz1) * wr1, wz1 * (1 - wr1), wz1 * wr1};
        const int64_t nd[4] = {node(g, i, j), node(g, i, j + 1), node(g, i + 1, j), node(g, i + 1, j + 1)};
        double et = 0;
        for (int k = 0; k < 4; ++k) et += W[k] * Et[nd[k]];
        const double u[3] = {vr[p] + 0.5 * s->dt * ar[p], vt[p] + 0.5 * s->dt * at[p] + 2 * h * et,
                             vz[p] + 0.5 * s->dt * az[p]};
        const double vbar = 0.5 * (vt[p] + u[1]);
        for (int k = 0; k < 4; ++k) Inode[nd[k]] += qw * vbar * W[k];
        const double X = R[p] + u[0] * s->dt, Y = u[1] * s->dt;
        const double znew = z[p] + u[2] * s->dt;
        const double Rnew = sqrt(X * X + Y * Y);
        double c = 1.0, sn = 0.0;
        if (Rnew > 0) { c = X / Rnew; sn = Y / Rnew; }
        const double a0 = ar[p], a1 = at[p];
        int out = 0;
        if (znew < 0) {
            out = 1;
        } else if (znew >= g->zp) {
            out = 1;
            if (g->window) {
                const double ts = (g->zp - z[p]) / u[2];
                const double xs = R[p] + u[0] * ts, ys = u[1] * ts;
                const double Rs = sqrt(xs * xs + ys * ys);
                if (Rs < g->rmax) {
                    window_charge(g, Rs, qw, surf);
                    out = 2;
                }
            }
        } else if (Rnew >= g->rmax) {
            out = 1;
        }
        R[p] = Rnew;
        z[p] = znew;
        vr[p] = c * u[0] + sn * u[1];
        vt[p] = -sn * u[0] + c * u[1];
        vz[p] = u[2];
        ar[p] = c * a0 + sn * a1;
        at[p] = -sn * a0 + c * a1;
        if (out) {
            alive[p] = 0;
            absorbed[p] = out;
        }
    }
}

/* Corrector of step n: a = (q/m) (E_r, E_z)^{n+1} gathered at x~; position
 * += (dt^2/2) a (radially and axially: the frame does not turn), velocity
 * += (dt/2) a, abar = (a + abar) / 2.  A corrected radius below zero passes
 * through the axis: R -> -R with the radial and azimuthal components of v
 * and abar reversed.  Absorption as in the push, the window crossing taken
 * on the correction segment. */
void ora_di_correct(const ora_grid *g, const ora_species *s, int64_t n,
                    double *R, double *z, double *vr, double *vt, double *vz,
                    double *ar, double *at, double *az,
                    int32_t *alive, int32_t *absorbed, const double *Er, const double *Ez, double *surf)
{
    const double qm = s->q / s->m, dt = s->dt;
    const double qw = s->q * s->w;
    for (int64_t p = 0; p < n; ++p) {
        absorbed[p] = 0;
        if (!alive[p]) continue;
        int j, i;
        double wr1, wz1;
        weights(g, R[p], z[p], &j, &i, &wr1, &wz1);
        const double W[4] = {(1 - wz1) * (1 - wr1), (1 - wz1) * wr1, wz1 * (1 - wr1), wz1 * wr1};
        const int64_t nd[4] = {node(g, i, j), node(g, i, j + 1), node(g, i + 1, j), node(g, i + 1, j + 1)};
        double er = 0, ez = 0;
        for (int k = 0; k < 4; ++k) {
            er += W[k] * Er[nd[k]];
            ez += W[k] * Ez[nd[k]];
        }
        const double a_r = qm * er, a_z = qm * ez;
        const double z0 = z[p];
        double Rn = R[p] + 0.5 * dt * dt * a_r;
        const double zn = z0 + 0.5 * dt * dt * a_z;
        double v0 = vr[p] + 0.5 * dt * a_r, v1 = vt[p], v2 = vz[p] + 0.5 * dt * a_z;
        double b0 = 0.5 * (a_r + ar[p]), b1 = 0.5 * at[p], b2 = 0.5 * (a_z + az[p]);
        if (Rn < 0) {
            Rn = -Rn;
            v0 = -v0;
            v1 = -v1;
            b0 = -b0;
            b1 = -b1;
        }
        int out = 0;
        if (zn < 0) {
            out = 1;
        } else if (zn >= g->zp) {
            out = 1;
            if (g->window) {
                const double f = (g->zp - z0) / (zn - z0);
                const double Rs = fabs(R[p] + f * 0.5 * dt * dt * a_r);
                if (Rs < g->rmax) {
                    window_charge(g, Rs, qw, surf);
                    out = 2;
                }
            }
        } else if (Rn >= g->rmax) {
            out = 1;
        }
        R[p] = Rn;
        z[p] = zn;
        vr[p] = v0;
        vt[p] = v1;
        vz[p] = v2;
        ar[p] = b0;
        at[p] = b1;
        az[p] = b2;
        if (out) {
            alive[p] = 0;
            absorbed[p] = out;
        }
    }
}
