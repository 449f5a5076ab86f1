/*
 * phasorpic: the per-timestep axisymmetric (z, R) PIC/MCC cycle of the
 * phasor-PIC method (Chen et al., "Phasor-particle-in-cell algorithm for
 * bidirectional external-circuit coupling of inductively coupled plasma"),
 * as HIP kernels for MI355X (gfx950) behind a plain C ABI.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns a pic_status (int32_t); PIC_OK == 0.  Argument errors
 *   are reported synchronously.  Work is enqueued asynchronously on the HIP
 *   stream given to pic_init; errors raised on the device (capacity
 *   overflow, solver non-convergence) surface at the next synchronising
 *   call (pic_sync, the getters, circuit_period_update) and then stick
 *   until pic_clear_error.  pic_last_error() explains the last failure.
 * - Grid: nr x nz cells; node (i, j) sits at z = i dz, R = j dR with
 *   dz = zmax / nz, dR = rmax / nr; node arrays are (nz+1) x (nr+1), R index
 *   fastest (linear index i * (nr+1) + j); cell arrays are nz x nr.
 * - Species 0 are electrons, species 1 Ar+ ions.  Particles live in the box
 *   0 <= R < rmax, 0 <= z < zp with zp = ip dz.
 * - Memory: the caller owns all device memory.  pic_workspace_bytes() sizes
 *   one device buffer that the caller allocates (e.g. a torch uint8 tensor)
 *   and passes to pic_init; the library carves every device array it uses
 *   out of it and never frees it.  Host pointers in pic_config are read
 *   during pic_init only.  The opaque pic_ctx is host memory owned by the
 *   library and released by pic_destroy.
 * - Threading: one host thread per context; a context is not thread-safe.
 * - Step order of one PIC step n (the paper's workflow, Sec. 2.5):
 *       pic_gather_push(n); harmonic_accumulate(n); mcc_collide(n);
 *       pic_deposit(n+1); [circuit_period_update() when (n+1) % N_RF == 0];
 *       poisson_solve_rz(n+1, ...)
 *   and with the direct-implicit update (pic_config.implicit), where the
 *   particles' correction follows the field solve:
 *       pic_gather_push(n); harmonic_accumulate(n); pic_deposit(n+1);
 *       [circuit_period_update()]; poisson_solve_rz(n+1, ...); mcc_collide(n)
 */
#ifndef PHASORPIC_H
#define PHASORPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pic_status;

enum {
    PIC_OK = 0,
    PIC_EINVAL = -1,    /* bad configuration, shape or argument */
    PIC_ENOMEM = -2,    /* workspace, particle or birth capacity too small */
    PIC_EDEVICE = -3,   /* HIP runtime error */
    PIC_ENOTCONV = -4,  /* Poisson multigrid missed rtol within max_cycles */
    PIC_EPHASE = -5,    /* phase closure or sample count != N_RF: update rejected */
    PIC_ESTATE = -6     /* call-order violation */
};

enum { PIC_FP64 = 0, PIC_MIXED = 1 };
/* poisson_solve_rz operators */
enum { PIC_OP_POISSON = 0, PIC_OP_HELMHOLTZ_C = 1, PIC_OP_HELMHOLTZ_S = 2 };
/* Poisson solver (pic_config.poisson_solver): AUTO takes the direct solve
 * when the operator separates (below) and multigrid-CG otherwise; DIRECT
 * fails pic_init with PIC_EINVAL when it does not separate. */
enum { PIC_POISSON_AUTO = 0, PIC_POISSON_MULTIGRID = 1, PIC_POISSON_DIRECT = 2 };
enum { PIC_FIELD_FULL = 0, PIC_FIELD_MQS = 1 };   /* inductive operator with / without displacement term */
enum { PIC_RRF_GIVEN = 0, PIC_RRF_SKIN = 1 };     /* turn RF resistance: given / round-wire skin model */
#define PIC_MAX_TURNS 16

/* grids readable with pic_get_grid (all FP64 node arrays) */
enum {
    PIC_GRID_PHI = 0,      /* electrostatic potential phi^n (V) */
    PIC_GRID_CHARGE = 1,   /* node charge of the last pic_deposit, incl. window charge (C) */
    PIC_GRID_CURRENT = 2,  /* azimuthal node current I^n = sum q w vbar_theta W (A m) */
    PIC_GRID_ER = 3,       /* staged E_r of the last pic_gather_push (V/m) */
    PIC_GRID_EZ = 4,       /* staged E_z (V/m) */
    PIC_GRID_ETHETA = 5,   /* staged E_theta(t_n) (V/m) */
    PIC_GRID_SURFACE = 6,  /* window surface charge accumulated up to the last pic_deposit (C) */
    PIC_GRID_JC = 7,       /* running sum of I^n cos(theta_n) of the open period */
    PIC_GRID_JS = 8,       /* running sum of I^n sin(theta_n) of the open period */
    PIC_GRID_EC = 9,       /* E_c of the applied azimuthal field (V/m; the fundamental's with nharm > 0) */
    PIC_GRID_ES = 10,      /* stored sine array E_s^sto = -E_s of the applied field (V/m; likewise) */
    PIC_GRID_EC_PLASMA = 11,  /* plasma-only E_c^p of the last circuit update (fundamental) */
    PIC_GRID_ES_PLASMA = 12,  /* plasma-only E_s^sto,p of the last circuit update */
    PIC_GRID_BR = 13,      /* staged RF B_r of the last pic_gather_push (T), cfg->rf_bfield only */
    PIC_GRID_BZ = 14,      /* staged RF B_z (T) */
    PIC_GRID_CHI = 15,     /* direct-implicit susceptibility of the last pic_deposit, cfg->implicit only */
    PIC_GRID_UNIT = 16     /* + k: unit-current field U_k of turn k+1 (V/m per A) */
};

typedef struct pic_config {
    /* grid */
    int32_t nr, nz;          /* cells in R and z; multigrid wants both even, ideally 2^k */
    int32_t ip;              /* node row of the top of the particle region */
    int32_t window;          /* 1: charge leaving through row ip stays there (dielectric) */
    double rmax, zmax;       /* m */
    /* time: N_RF = nint(1 / (freq dt)) (Sec. 2.1, Eq. nrf) */
    double dt, freq;
    /* arithmetic: PIC_FP64, or PIC_MIXED (int cell + FP32 offsets and velocities) */
    int32_t precision;
    uint32_t seed;           /* Philox key word 0; key word 1 is the species */
    /* species: charge (C), mass (kg), macro weight, initial temperature (eV) */
    double q[2], m[2], w[2], temp_ev[2];
    int64_t np_init[2];      /* particles loaded by pic_init (if load != 0) */
    int64_t capacity[2];     /* particle slots per species */
    double bfield[3];        /* uniform (B_r, B_theta, B_z) in the Boris rotation (T) */
    /* gas and cross sections */
    double ngas;             /* neutral density (m^-3) */
    double tgas_ev;          /* neutral temperature (eV) */
    double qe;               /* elementary charge, for eV conversions */
    double eps0;             /* vacuum permittivity used by the Poisson operator */
    int32_t xs_kind;         /* 0 smooth analytic fits, 1 constant cross sections */
    int32_t nscan;           /* points of the nu_max scan */
    /* el_a el_b exc_a exc_th iz_a iz_th iel_a iel_p icx_a icx_p e_cap_ev i_gcap nu_margin */
    double xs[13];
    /* geometry and materials (host arrays, copied by pic_init) */
    int32_t nturns;          /* coil turns with Dirichlet potentials */
    int32_t fuse;            /* 1: pic_gather_push runs the fused push+MCC+deposit pass */
    const double *eps_cell;  /* nz*nr relative permittivity */
    const int32_t *node_tag; /* (nz+1)*(nr+1): -1 free, 0 grounded, k >= 1 turn k */
    const double *ec;        /* node E_c of the azimuthal field (V/m); NULL = 0 */
    const double *es_sto;    /* node stored sine array (= -E_s) (V/m); NULL = 0 */
    const double *turn_vc;   /* nturns: V_c,k of the turn potentials (V) */
    const double *turn_vs;   /* nturns: V_s,k */
    /* Poisson multigrid and scheduling */
    double mg_rtol;          /* residual tolerance relative to the equation's scale: the largest
                                over free nodes of max(|b_n|, sum_m |A_nm x_m|) for the start
                                value x (Dirichlet values included) */
    int32_t mg_max_cycles;   /* V-cycles per solve at most */
    int32_t sort_every;      /* steps between cell sorts of the particle arrays (>= 1) */
    int32_t load;            /* 1: load the initial uniform Maxwellian plasma */
    int32_t birth_capacity;  /* ionization events buffered per step */
    /* field-circuit coupling (Secs. 2.2 and 2.4).  circuit == 0 keeps the
     * prescribed ec / es_sto / turn_vc / turn_vs; circuit == 1 derives them
     * from the unit-current fields and the network, and updates them at
     * every closed period.  Turn k's nodes (tag k) are its source region
     * Omega_k for the inductive solve and its Dirichlet conductor for the
     * Poisson solve. */
    int32_t circuit;
    int32_t field_mode;      /* PIC_FIELD_FULL or PIC_FIELD_MQS */
    double mu0;              /* vacuum permeability used by the inductive operator */
    const double *turn_sign; /* s_k (+1 or -1), nturns; NULL = +1 */
    double r_g, r_m, l_m, c_m;   /* generator R, series matching R, L, C (c_m <= 0: no capacitor) */
    const double *c_stray;   /* out-of-domain shunt capacitance per node (F), nturns; NULL = 0 */
    int32_t rrf_mode;        /* PIC_RRF_GIVEN (r_rf) or PIC_RRF_SKIN (Eq. skin) */
    const double *r_rf;      /* nturns (ohm), rrf_mode == PIC_RRF_GIVEN */
    double rho20, alpha_cu, temp_c;   /* copper resistivity at 20 C, its coefficient, temperature (C) */
    double vg_amp, vg_phase; /* Thevenin peak amplitude (V) and phase (rad) */
    int32_t vg_from_target;  /* 1: start from the amplitude that puts p_target into the vacuum network */
    int32_t controller;      /* 1: closed-loop power control (Eqs. pfilter, ptrend, pcontrol) */
    double p_target, gamma, n_trend, eps_p, alpha_v, f_step, v_min, v_max;
    double alpha;            /* state relaxation, 0 < alpha <= 1 (Eq. relaxation) */
    double helm_rtol;        /* inductive solves: residual tolerance relative to the equation's scale */
    int32_t helm_max_cycles; /* ... and their iteration limit */
    int32_t sort_every_ion;  /* steps between cell sorts of the ion arrays (ions move a small fraction of a
                                cell per step); 0: sort_every */
    /* manufactured boundaries (host arrays of nturns x nodes, copied by pic_init; NULL = 0), as in the
     * paper's joint benchmark (Sec. 3.3): a grounded node n (tag 0) of the Poisson problem takes
     * sum_k dir_basis[k * nodes + n] V_k(t_n), with V_k(t_n) the turn potentials of Eq. dirichlet,
     * and the unit-current field U_k takes unit_bvals[k * nodes + n] on the Dirichlet nodes of the
     * inductive operator (axis, outer boundary, metal) */
    const double *dir_basis;
    const double *unit_bvals;
    /* 1: the RF magnetic field of the applied azimuthal field enters the Boris rotation (with bfield):
     * by Faraday's law, with F = (E_c sin th_n + E_s^sto cos th_n) / w, B_r = dF/dz and
     * B_z = -(1/R) d(R F)/dR at t_n, staged per node by central differences and gathered with the
     * particle weights (the paper leaves the push's magnetic field unstated) */
    int32_t rf_bfield;
    /* 1: direct-implicit electrostatic update (Sec. 2.3: the charge and the susceptibility chi of
     * Eqs. poisson and epseff from predicted positions), with the D1 time filter of the direct
     * implicit method the paper cites (see the step order above).  Per step:
     *   pic_gather_push(n): predictor -- the electrostatic kick is each particle's filtered half kick
     *     (dt/2) abar^{n-1}, the inductive kick dt (q/m) E_theta(t_n) explicit, J_theta^n deposited,
     *     move to the predicted positions x~, whose charge is deposited;
     *   harmonic_accumulate(n);
     *   pic_deposit(n+1): rho~ and chi = (dt^2 / 2) sum_s q_s^2 n_s / (m_s eps0) at the nodes from
     *     x~, and the level-0 operator with face coefficients eps_r (1 + (chi_a + chi_b) / 2);
     *   [circuit_period_update()];
     *   poisson_solve_rz(n+1): phi^{n+1} with chi (the coarse multigrid levels keep the chi = 0
     *     operator as CG preconditioner; Q_k with the same face coefficients, Eq. facecharge);
     *   mcc_collide(n): corrector -- x += dt (dt/2) a^{n+1}(x~), v += (dt/2) a^{n+1}, abar =
     *     (a^{n+1} + abar) / 2 -- then the collisions of v^{n+1/2} at x^{n+1} and the births.
     * No magnetic field (bfield, rf_bfield) in this mode. */
    int32_t implicit;
    /* PIC_POISSON_*.  The direct solve applies when every node of the bottom row, the top row and the
     * outer radius is Dirichlet, the permittivity of every row of cells is uniform in R (so the
     * finite-volume operator on the block of remaining nodes is Z (x) L_R + L_Z (x) D), at most 512
     * Dirichlet nodes lie inside that block, and the update is explicit (implicit == 0: chi changes
     * the operator every step).  It transforms the block by the radial eigenvectors, solves one
     * tridiagonal system in z per radial mode, and imposes the interior Dirichlet values (the turns)
     * through their capacitance matrix: one pass, FP64, with no iteration and no tolerance. */
    int32_t poisson_solver;
    /* Multiharmonic circuit (the outlook of the paper's conclusions): nharm orders above the fundamental
     * (0..3) are retained, order m = 2..nharm+1 at frequency m freq.  Each order runs the circuit
     * network of Sec. 2.2 at m w -- its own unit fields, Z_vac, source and matching impedance and skin
     * resistance at m w, plasma-only fields from the order-m current harmonic J^(m) = (2 / N_RF)
     * sum_n I^n (cos, sin)(m th_n), and I_cap^(m) = i m w Q^(m) from the turn-charge harmonic of order
     * m -- and the fields, turn potentials and gathers take the sum over the orders, E_theta(t_n) =
     * sum_m E_c^(m) cos(m th_n) - E_s^sto,(m) sin(m th_n) and phi_k(t_n) = sum_m V_c,k^(m) cos(m th_n)
     * + V_s,k^(m) sin(m th_n).  The source of order m is harm_ratio[m-2] exp(i harm_phase[m-2]) times
     * the fundamental's V_g; the controller and the target-power start act on the total port power
     * (sum over the orders).  Requires circuit = 1 and field_mode = PIC_FIELD_MQS (one inductive
     * operator for every order); excludes rf_bfield, pic_set_source, prescribed loads and the
     * surrogate.  harm_ratio > 0 and finite phases for the first nharm entries. */
    int32_t nharm;
    double harm_ratio[3];
    double harm_phase[3];    /* rad */
    /* Ion-induced secondary electron emission at the grounded metal walls (the GEC cell's inherited
     * module, Sec. 3.4; its yields are not given): each ion absorbed at the bottom (z = 0), at the top
     * (z = zp, metal when window == 0) or at the outer wall (R = rmax) emits an electron with probability
     * see_gamma (0 = off; [0, 1]) -- Philox block (ion id, n, 4, 0) of the ion stream, word 0 below
     * see_gamma.  The electron starts at the ion's position before the step's move, with a
     * flux-weighted Maxwellian velocity at see_temp_ev (eV): normal speed sigma sqrt(-2 ln u1) into
     * the domain, tangential components sigma sqrt(-2 ln u2) (cos, sin)(2 pi u3), sigma = sqrt(T e /
     * m_e); block (id, n, 5, 0) draws its first collision candidate.  mcc_collide(n) appends the
     * step's emitted electrons after its ionization births, in ascending parent-ion id order, with
     * ids continuing the electron counter, and deposits their charge in the fused mode.  At most 65536
     * ions per step reach a metal wall (PIC_ENOMEM beyond).  Not with implicit. */
    double see_gamma;
    double see_temp_ev;
} pic_config;

typedef struct pic_solve_info {
    int32_t cycles;          /* V-cycles run by the last solve */
    int32_t converged;       /* 1 if rel_residual <= rtol */
    double rel_residual;     /* max |residual| / equation scale after the last cycle */
} pic_solve_info;

typedef struct pic_stats {
    int64_t slots[2];        /* particle slots in use (live + not yet compacted) */
    int64_t live[2];         /* live particles */
    int64_t next_id[2];      /* next particle id per species */
    int64_t candidates[2];   /* MCC candidates since init */
    int64_t events[2][3];    /* real collisions by process since init */
    int64_t births;          /* ionization births since init */
    int64_t absorbed[2];     /* particles absorbed since init */
    int64_t over_numax[2];   /* candidates whose total frequency exceeded nu_max */
    int64_t window_out;      /* deposit contributions outside the LDS window (fallback atomics) */
    int64_t samples;         /* harmonic samples in the open period */
    int32_t nrf;             /* N_RF */
    int32_t phase_closed;    /* Eq. phaseclosure holds */
    double numax[2];         /* null-collision frequency per species (1/s) */
    double pnull[2];         /* null-collision probability per step */
    double pind_sum;         /* open-period sum of sum_nodes I E_theta (W) */
    double qc[16], qs[16];   /* open-period sums of Q_k cos, Q_k sin (first 16 turns) */
    double wk[16];           /* open-period trapezoid sums of V dQ (first 16 turns) */
    double qk[16];           /* Q_k of the last Poisson solve (C) */
    /* HIP-event timing since pic_timing(ctx, 1) (milliseconds, launches) */
    double pass_ms;          /* particle pass, summed over launches (one launch per species and step) */
    int64_t pass_count;      /* launches timed */
    double poisson_ms;       /* whole poisson_solve_rz */
    int64_t poisson_count;
    double sort_ms;          /* cell sorts of both species */
    int64_t sort_count;
    double circuit_ms;       /* circuit_period_update's device work */
    int64_t circuit_count;
    int64_t mg_cycles;       /* V-cycles of the last solve */
    double mg_rel;           /* its final relative residual */
    int64_t mg_unconverged;  /* Poisson solves since init that used up their iteration budget before
                                rtol (the stepping path's budget adapts to the recent counts; a solve
                                given an info record runs max_cycles and returns PIC_ENOTCONV instead) */
    int64_t see_emitted;     /* secondary electrons emitted since init (cfg->see_gamma) */
} pic_stats;

typedef struct pic_ctx pic_ctx;
typedef struct mlp_ctx mlp_ctx;

/* Bytes of device workspace pic_init needs for this configuration. */
pic_status pic_workspace_bytes(const pic_config *cfg, size_t *bytes);

/* Validates the configuration (grid, tags, phase closure flag, species),
 * carves the workspace, sets up the null-collision constants, loads the
 * plasma when cfg->load (uniform in volume, Maxwellian, Philox-keyed by
 * particle id), sorts it by cell, deposits rho^0 and solves phi^0.
 * Follows Sec. 2.1 (time structure), Sec. 2.3 (Poisson problem) and the
 * workflow's initialisation (Sec. 2.5).  workspace: device pointer of at
 * least pic_workspace_bytes(cfg) bytes; stream: a hipStream_t (NULL = the
 * default stream).  On success *out owns a new context. */
pic_status pic_init(const pic_config *cfg, void *workspace, size_t workspace_bytes, void *stream,
                    pic_ctx **out);

/* Step n, particle part: stages E_r, E_z from phi^n and E_theta(t_n) =
 * E_c cos th_n - E_s^sto sin th_n (Eq. et_reconstruct), gathers at x^n with
 * R^2-linear radial and linear axial weights, Boris-pushes v^{n-1/2} ->
 * v^{n+1/2}, moves to x^{n+1} in the particle's Cartesian plane and rotates
 * (v_r, v_theta) back, deposits the azimuthal current I^n with the gather
 * weights and vbar_theta = (v^{n-1/2} + v^{n+1/2})/2, and removes particles
 * that leave the box (window crossings leave their charge on row ip).
 * With cfg->fuse the same pass also runs the collisions and the charge
 * deposit of the new positions.  Requires n == last step + 1 (first n = 0);
 * sorts the electron arrays by cell first when n % sort_every == 0, the ion
 * arrays when n % sort_every_ion == 0 (sort_every when 0). */
pic_status pic_gather_push(pic_ctx *ctx, int64_t n);

/* Null-collision MCC of step n on v^{n+1/2} at x^{n+1}: particles whose
 * candidate step is n draw Philox4x32-10 block (id, n, 1, 0) keyed by
 * (seed, species), select elastic / excitation / ionization (electrons) or
 * elastic / charge exchange (ions) against nu_max, and schedule their next
 * candidate.  Ionization births are appended in parent-id order.  Capacity
 * overflow -> PIC_ENOMEM at the next sync. */
pic_status mcc_collide(pic_ctx *ctx, int64_t n);

/* Node charge rho^{n1} at x^{n1}: q w times the gather weights, summed in
 * exact 64-bit fixed point, plus the accumulated window surface charge. */
pic_status pic_deposit(pic_ctx *ctx, int64_t n1);

/* Field solves on the grid, FP64: multigrid-preconditioned CG, or for a
 * separable Poisson operator the direct solve (pic_config.poisson_solver).
 *
 * op = PIC_OP_POISSON: the finite-volume RZ Poisson problem
 * sum_f eps0 eps_f A_f (phi_p - phi_nb) / d_f = Q_p (Eqs. poisson with
 * chi = 0, epseff, areas; Neumann axis, Eq. axis_electrostatic_bc) with
 * Dirichlet 0 on grounded nodes and phi_k(t_n) = V_c,k cos th_n +
 * V_s,k sin th_n on turn k (Eq. dirichlet); the multigrid-CG solve is
 * warm-started from the last phi (extrapolated in time along a running
 * sequence of steps).  Then the turn charges Q_k(t_n) from the operator's
 * face fluxes (Eq. facecharge).
 *
 * op = PIC_OP_HELMHOLTZ_C / _S (coupled contexts only, else PIC_EINVAL):
 * one of the two real plasma-only inductive solves of the period update
 * (Sec. 2.2, Eq. helmholtz_two_real), K E_c^p = J_s / V and K E_s^sto,p =
 * J_c / V, with the harmonics J_c, J_s = (2 / N_RF) sum_n I^n (cos, sin)
 * th_n accumulated so far in the open period (after N_RF samples exactly
 * the fields circuit_period_update computes); the result replaces
 * PIC_GRID_EC_PLASMA / _ES_PLASMA.  n is ignored.
 *
 * rtol <= 0 / max_cycles <= 0 take the config values (mg_* for Poisson,
 * helm_* for the inductive solves).  info (nullable): when given the call
 * synchronises, fills it and returns PIC_ENOTCONV if rtol was not met;
 * without it a Poisson solve runs an iteration budget adapted to the
 * recent solves and a short solve is only counted (pic_stats.
 * mg_unconverged), while the inductive solves always synchronise and
 * return PIC_ENOTCONV when they miss rtol.  The direct Poisson solve
 * ignores rtol and max_cycles except that info, when given, reports its
 * relative residual (cycles = 0) and PIC_ENOTCONV if that exceeds rtol. */
pic_status poisson_solve_rz(pic_ctx *ctx, int64_t n, int32_t op, double rtol, int32_t max_cycles,
                            pic_solve_info *info);

/* Period accumulation of step n (Eqs. fourier, pind, pcap): J_c += I^n
 * cos th_n, J_s += I^n sin th_n on nodes, Q_c,k / Q_s,k with Q_k(t_n),
 * P_ind sum of sum_nodes I^n E_theta(t_n), the trapezoid of V_k dQ_k and the
 * sample count; FP64 with compensated (Neumaier) sums.  Must follow
 * pic_gather_push(n); calling it twice for one step is PIC_ESTATE. */
pic_status harmonic_accumulate(pic_ctx *ctx, int64_t n);

/* Closed-period report (Eqs. fourier, icap, pind, pcap, pcap_phasor) and,
 * with cfg->circuit, the circuit update (Eqs. vpind, pport, pbalance,
 * power_imbalance, pcontrol, blockmatrix, relaxation, kclres, kvlres).
 * Phasors are peak values under Re[x exp(+i w t)]; x = (I_f, I_1..I_N,
 * V_1..V_N). */
typedef struct pic_period_report {
    int32_t accepted;        /* 0: sample count != N_RF, nothing changed */
    int32_t samples;
    double p_ind;            /* W */
    double p_cap;            /* W, periodic trapezoid */
    double p_cap_ph;         /* W, phasor cross-check */
    double qc[16], qs[16];   /* charge harmonics Q_c,k, Q_s,k */
    double icap_re[16], icap_im[16];  /* I_cap,k = w Q_s,k + i w Q_c,k */
    /* circuit update (cfg->circuit != 0) */
    double p_port;           /* 1/2 Re(V_1 conj(I_f)) of the completed period's state */
    double p_cu;             /* copper loss of that state */
    double eps_bal;          /* |P_port - (P_ind + P_cap + P_Cu)| / |P_port| */
    double kcl, kvl;         /* max residuals of the new state, / |I_f| and / |V_g| */
    double vg_old, vg_amp;   /* Thevenin amplitude before / after the controller */
    double pf, pc;           /* filtered and trend-extrapolated power (controller on) */
    double vp_re[16], vp_im[16];      /* plasma reaction voltages V_p,k */
    double xt_re[33], xt_im[33];      /* target network solution */
    double x_re[33], x_im[33];        /* relaxed state applied in the next period */
    int32_t helm_cycles[2];  /* CG iterations of the two plasma-only inductive solves */
    double helm_rel[2];      /* and their final relative residuals */
    double xp_re[33], xp_im[33];      /* state applied during the completed period */
    double pressure;         /* gas pressure (Pa) */
    /* plasma moments at the end of the period: <n_e>, <n_i> (m^-3, over the
     * particle box), max n_e (m^-3, nodes), <eps_e>, <eps_i> (eV), electron
     * centroid R, z (m), ionizations during the period (real particles:
     * macro-particle births times the electron weight) */
    double moments[8];
    int32_t sur_used;        /* 1: the surrogate-assisted update was applied */
    int32_t sur_iters;       /* its inner fixed-point iterations */
    double sur_err;          /* scaled prediction error at the applied state */
    double sur_steps[64];    /* |x_{i+1} - x_i| / |x_{i+1}| of each inner iterate (first sur_iters) */
    double vg_phase;         /* phase of the Thevenin source V_g (rad) */
} pic_period_report;

/* Surrogate-assisted circuit update (the learned predictor of the load
 * responses).  With a network attached, circuit_period_update predicts
 * yhat(x^n) = (V_p, I_cap) from the applied state, pressure and moments,
 * and compares it with the measured y_n (V_p scaled by |V_g|, I_cap by
 * |I_f|).  Above err_max the plain update runs; otherwise the state
 * iterates x_{i+1} = relax(network(yhat(x_i) + y_n - yhat(x^n), V_g,i)),
 * with the controller acting on each iterate's port power inside the
 * period's step bounds, until the relative step is below tol or max_iter,
 * and the converged state is applied.  When max_iter iterates pass without
 * meeting tol, the state and source amplitude applied are the means of the
 * iterates of the second half (the BF16 activations make the predictions a
 * step function of the state, so the iterates circle the fixed point). */
typedef struct pic_surrogate_config {
    double err_max;          /* e.g. 0.02 */
    double tol;              /* e.g. 1e-6 */
    int32_t max_iter;        /* e.g. 50; at most 64 */
} pic_surrogate_config;

/* Inductive-port data of a coupled context (pic_get_circuit). */
typedef struct pic_circuit_info {
    int32_t nturns;
    double omega;
    double zvac_im[16 * 16];  /* Im Z_vac,kl (row-major, stride 16); Re Z_vac = 0 */
    double eps_rec;           /* reciprocity error of Z_vac (Eq. reciprocity) */
    double r_rf[16];          /* turn RF resistances */
    double zs_re, zs_im;      /* source + matching branch impedance */
    double g[16];             /* shape-function value s_k / A_k of each turn (1/m^2) */
    double area[16];          /* A_k = N_k dz dR */
    double vg_amp, vg_phase;  /* current Thevenin amplitude and phase */
    double x_re[33], x_im[33];  /* applied state */
} pic_circuit_info;

/* What a caller may impose on one period update (all fields optional). */
typedef struct pic_circuit_override {
    /* context without circuit coupling: the next period's turn potentials
     * (nturns each) and azimuthal field (node arrays); NULL keeps them */
    const double *new_vc, *new_vs;
    const double *new_ec, *new_es_sto;
    /* coupled context: prescribed load responses (loads != 0) replace the
     * measured plasma reaction voltages and capacitive currents of the
     * closed period in the controller and the network solve (Eqs.
     * blockmatrix, relaxation) -- a prescribed load or an external
     * predictor; the powers of the report stay the measured ones, its
     * V_p / I_cap are the prescribed values.  Not with a surrogate attached. */
    int32_t loads;
    double vp_re[16], vp_im[16];      /* V_p,k (V) */
    double icap_re[16], icap_im[16];  /* I_cap,k (A) */
} pic_circuit_override;

/* Closes the RF period: synchronises and requires phase closure and
 * exactly N_RF samples (otherwise PIC_EPHASE: the update is rejected, the
 * circuit state and fields stay as they are, and the accumulators restart
 * empty).  Finalises the harmonics and powers into *report (nullable) and
 * copies J_c, J_s (x 2/N_RF) into the caller's host arrays jc, js when
 * non-NULL.  Without cfg->circuit it then installs what ovr (nullable)
 * gives for the next period.  With cfg->circuit the update of Sec. 2.4 runs
 * on the device: two plasma-only inductive solves K E_c^p = J_s / V_node,
 * K E_s^sto,p = J_c / V_node (Eq. helmholtz_two_real), V_p,k (Eq. vpind),
 * I_cap,k (Eq. icap) -- or the loads ovr prescribes --, the power
 * controller, the (2N+1) complex network solve with partial pivoting, the
 * relaxation, the residuals, and the next period's turn potentials and
 * field (Eq. compose).  PIC_EINVAL for an override that does not fit the
 * context (turn data on a coupled one, loads on an uncoupled one or with a
 * surrogate, or loads with cfg->nharm > 0); PIC_ENOTCONV if an inductive
 * solve misses helm_rtol.  The accumulators are reset.
 *
 * With cfg->nharm > 0 every retained order runs that update at its own
 * frequency (two inductive solves per order, its own loads and network),
 * the controller acts on the total port power, and *report holds the
 * fundamental's harmonics, loads and states with the totals over the orders
 * in p_port, p_cu, p_cap_ph, eps_bal and kcl / kvl (largest); p_ind and
 * p_cap are time-domain powers of the whole waveform; jc, js receive the
 * fundamental's harmonics. */
pic_status circuit_period_update(pic_ctx *ctx, const pic_circuit_override *ovr, pic_period_report *report,
                                 double *jc, double *js);

/* The last circuit update's fields of retained order `order` (1 = the
 * fundamental .. cfg->nharm + 1): its charge harmonics and I_cap^(m), p_port
 * and p_cu of its own network state, p_cap_ph, V_p^(m), the target, applied
 * and previous states, its source amplitude and phase and its residuals; the
 * time-domain p_ind, p_cap are those of the whole waveform.  accepted = 0
 * before the first update.  Synchronises.  PIC_EINVAL without
 * cfg->circuit or for an order outside 1..nharm + 1. */
pic_status circuit_order_report(pic_ctx *ctx, int32_t order, pic_period_report *report);

/* Set the Thevenin source amplitude (V, > 0) and phase (rad) used by the
 * next circuit update of a coupled context (the controller, when on, starts
 * from this amplitude).  For scans of the operating point.  PIC_EINVAL with
 * cfg->nharm > 0 (the orders' sources follow from the configuration). */
pic_status pic_set_source(pic_ctx *ctx, double vg_amp, double vg_phase);

/* Attach (net != NULL) or detach (NULL) a surrogate network: n_in = 4 N + 9
 * (turn current and voltage phasors, pressure, the eight moments), n_out =
 * 4 N (V_p and I_cap phasors), N <= 5, same stream as the context.  The
 * network stays owned by the caller and must outlive the attachment.
 * PIC_EINVAL with cfg->nharm > 0. */
pic_status pic_attach_surrogate(pic_ctx *ctx, mlp_ctx *net, const pic_surrogate_config *cfg);

/* Copy the inductive-port data and the applied circuit state of a coupled
 * context (synchronising); PIC_EINVAL without cfg->circuit. */
pic_status pic_get_circuit(pic_ctx *ctx, pic_circuit_info *info);

/* Synchronise the stream and report any sticky device-side error. */
pic_status pic_sync(pic_ctx *ctx);
pic_status pic_clear_error(pic_ctx *ctx);

/* Host copies of one species' live particles (synchronising), in the
 * oracle's representation: R, z (m), v_r, v_theta, v_z (m/s), id, next
 * candidate step; arrays of capacity cap; *count receives the live count
 * (PIC_ENOMEM if it exceeds cap; any pointer may be NULL). */
pic_status pic_get_particles(pic_ctx *ctx, int32_t species, int64_t cap, double *R, double *z,
                             double *vr, double *vt, double *vz, uint32_t *id, int32_t *next,
                             int64_t *count);

/* Replace one species' particles (host arrays of length n) and re-sort.
 * next_id becomes max(id) + 1 unless a larger value is already set. */
pic_status pic_set_particles(pic_ctx *ctx, int32_t species, int64_t n, const double *R,
                             const double *z, const double *vr, const double *vt, const double *vz,
                             const uint32_t *id, const int32_t *next);

/* Make n the next step for pic_gather_push (restart from a saved state,
 * or a test that starts mid-period). */
pic_status pic_set_step(pic_ctx *ctx, int64_t n);

/* Replace phi (host node array); the next pic_gather_push stages from it. */
pic_status pic_set_phi(pic_ctx *ctx, const double *phi);

/* Restart (the restart check of the paper's appendix: a run stopped and
 * resumed reproduces the uninterrupted one).  pic_checkpoint copies the
 * whole time-dependent state at a step boundary -- both species' particle
 * slots in storage order, counters, phi and the two previous solutions of
 * the start-value extrapolation, the window charge, the turn charges, the
 * open period's accumulators, the applied turn potentials and azimuthal
 * field, the plasma-only fields and the circuit state -- into the caller's
 * host buffer buf of cap bytes; with buf == NULL it only sets *bytes to
 * the size needed.  PIC_ESTATE between the calls of a step, PIC_ENOMEM if
 * cap is too small.  pic_restore loads such a buffer into a context made
 * by pic_init with the same configuration (what pic_init derives from the
 * configuration alone is not stored); PIC_EINVAL for a buffer from another
 * configuration.  Then pic_gather_push continues with the step after the
 * checkpoint.  The continuation is bit-identical to the uninterrupted run
 * until the next cell sort (which orders the particles within a cell by
 * atomics).  An attached surrogate stays attached. */
pic_status pic_checkpoint(pic_ctx *ctx, void *buf, size_t cap, size_t *bytes);
pic_status pic_restore(pic_ctx *ctx, const void *buf, size_t bytes);

/* Copy one FP64 node grid (PIC_GRID_*) to host (synchronising). */
pic_status pic_get_grid(pic_ctx *ctx, int32_t which, double *out);

/* Enable (1) or disable (0) HIP-event timing of the particle pass, the
 * Poisson solve and the sort on the context's stream; enabling resets the
 * totals reported in pic_stats. */
pic_status pic_timing(pic_ctx *ctx, int32_t enable);

/* Counters and open-period accumulators (synchronising). */
pic_status pic_get_stats(pic_ctx *ctx, pic_stats *out);

/* Release the context (not the caller's workspace). */
void pic_destroy(pic_ctx *ctx);

/* The message of the context's last failure; with ctx == NULL, why the
 * last pic_workspace_bytes or pic_init on the calling thread failed ("null
 * context" if it did not).  The string stays valid until the next call on
 * that context (or, for NULL, the next pic_workspace_bytes / pic_init on the
 * thread). */
const char *pic_last_error(const pic_ctx *ctx);

/* ------------------------------------------------------------------------
 * Surrogate network of the coil-plasma response (the learned predictor of
 * the circuit update): n_in (<= 32) standardised inputs -> three GELU
 * hidden layers of width `hidden` -> n_out (<= 32) standardised outputs.
 * BF16 weights and activations on the matrix cores with FP32
 * accumulation; FP32 master weights trained by Adam on mean-squared
 * error.  Inputs and outputs are padded to 32 columns internally.
 * Flat FP32 parameter vector (padded):
 *   W1 [hidden x 32], b1 [hidden], W2 [hidden x hidden], b2, W3, b3,
 *   W4 [32 x hidden], b4 [32]   (W row-major, rows = outputs).
 * ------------------------------------------------------------------------ */
typedef struct mlp_config {
    int32_t n_in, n_out;      /* 1..32 */
    int32_t hidden;           /* multiple of 64 */
    int32_t max_batch;        /* rows per call at most */
    double lr, beta1, beta2, eps;   /* Adam */
    /* standardisation x_std = (x - mean) / std, y = y_std * std + mean (host
     * arrays of n_in / n_out, read by mlp_init; NULL = 0 / 1) */
    const float *in_mean, *in_std, *out_mean, *out_std;
} mlp_config;

pic_status mlp_workspace_bytes(const mlp_config *cfg, size_t *bytes);
/* workspace: device memory of mlp_workspace_bytes; parameters start at 0
 * (load them with mlp_set_params). */
pic_status mlp_init(const mlp_config *cfg, void *workspace, size_t workspace_bytes, void *stream,
                    mlp_ctx **out);
pic_status mlp_param_count(const mlp_ctx *ctx, int64_t *n);
/* Host FP32 parameter vector in, Adam moments and step count reset. */
pic_status mlp_set_params(mlp_ctx *ctx, const float *host);
pic_status mlp_get_params(mlp_ctx *ctx, float *host);
/* y[batch x n_out] (device, FP32) = network(x[batch x n_in]) (device, FP32). */
pic_status mlp_forward(mlp_ctx *ctx, const float *x, int32_t batch, float *y);
/* mlp_forward for callers that cannot allocate device memory or let the
 * library touch the context's workspace activations: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same
 * result as mlp_forward (same kernels and arithmetic), but the input,
 * hidden activations and output staging live in a static device array of
 * the library (307,200 bytes per device, held until the process ends; its
 * address is looked up once per device by mlp_init), so the call allocates
 * nothing.  Limits: batch 1..64 and hidden <= 256, else PIC_EINVAL with
 * nothing launched.  x, y as for mlp_forward (device FP32, caller-owned).
 * Every call on a device shares that device's array: calls that overlap on
 * one device (two streams, two threads) race and must be serialised by
 * the caller; the array keeps the last call's contents and needs no
 * clearing (every element read is written first in the same call). */
pic_status mlp_forward_noalloc(mlp_ctx *ctx, const float *x, int32_t batch, float *y);
/* One training step on a batch (device arrays x[batch x n_in], t[batch x
 * n_out]): forward, mean-squared error over batch x n_out standardised
 * targets, backward (7 products), Adam.  loss (host, nullable): the batch
 * loss before the update; giving it synchronises. */
pic_status mlp_train_step(mlp_ctx *ctx, const float *x, const float *t, int32_t batch, float *loss);
/* Gradient of the last training step (host FP32, parameter layout). */
pic_status mlp_get_grads(mlp_ctx *ctx, float *host);
pic_status mlp_sync(mlp_ctx *ctx);
void mlp_destroy(mlp_ctx *ctx);
const char *mlp_last_error(const mlp_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* PHASORPIC_H */
