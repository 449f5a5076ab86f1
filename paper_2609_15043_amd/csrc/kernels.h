// Kernel argument blocks and launch entry points shared between the
// kernel translation units and the host library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace pic {

// LDS deposit window of one particle block (node slots, 64-bit fixed point
// in either precision): whole node rows around the block's particles, so
// particles that drifted a few cells since the last sort still land in LDS.
// 2304 slots: eight padded rows of a 256-cell radial grid, and four blocks
// of the fused pass per CU.
#ifndef PIC_WIN_NODES
#define PIC_WIN_NODES 2304
#endif
template <typename T> struct Win {
    static constexpr int N = PIC_WIN_NODES;
};
constexpr int BLOCK = 256;
// a wave reduction only for a cell holding at least half the wave (so at
// most two per deposit); smaller groups add their own values to the window.
// Measured on the large workload: pass 0.721 ms per launch with 16 lanes and
// 4 groups, 0.710 ms with 32 and 2 (8 lanes: 0.731; 48: 0.711)
#ifndef PIC_DEPOSIT_GROUPS
#define PIC_DEPOSIT_GROUPS 2
#endif
constexpr int DEPOSIT_GROUPS = PIC_DEPOSIT_GROUPS;   // wave reductions per run deposit before lanes add their own
#ifndef PIC_DEPOSIT_MIN_LANES
#define PIC_DEPOSIT_MIN_LANES 32
#endif
constexpr int DEPOSIT_MIN_LANES = PIC_DEPOSIT_MIN_LANES;   // smallest group worth a wave reduction
constexpr int RUN = 4;                  // consecutive particles per lane per vector load
// 8 runs per wave: with the streamed particle data non-temporal, longer
// blocks amortise the window set-up and flush better (pass 0.735 -> 0.720 ms
// on the large workload against 4 runs; 12 and 16 runs were slower)
#ifndef PIC_PASS_RUNS
#define PIC_PASS_RUNS 8
#endif
// the FP64 pass (3 waves per SIMD, plain stream accesses) is fastest at 4
#ifndef PIC_PASS_RUNS_F64
#define PIC_PASS_RUNS_F64 4
#endif
// runs per wave per block and particles per pass block, per precision
template <typename T> struct PassShape {
    static constexpr int runs = sizeof(T) == 4 ? PIC_PASS_RUNS : PIC_PASS_RUNS_F64;
    static constexpr int chunk = BLOCK * RUN * runs;
};
// particle capacities are padded to a multiple of both chunks
constexpr int PAD = PassShape<float>::chunk > PassShape<double>::chunk ? PassShape<float>::chunk
                                                                        : PassShape<double>::chunk;
static_assert(PAD % PassShape<float>::chunk == 0 && PAD % PassShape<double>::chunk == 0,
              "the padding must hold whole chunks of either precision");

// Counter slots (int64) in the device statistics block.
enum StatSlot {
    ST_CAND0 = 0, ST_CAND1,
    ST_EV00, ST_EV01, ST_EV02,          // electron elastic, excitation, ionization
    ST_EV10, ST_EV11, ST_EV12,          // ion elastic, charge exchange, (unused)
    ST_BIRTHS,
    ST_ABS0, ST_ABS1,
    ST_OVER0, ST_OVER1,
    ST_WINOUT,
    ST_MGUNCONV,                        // Poisson solves that ended before rtol
    ST_SEE,                             // secondary electrons emitted
    ST_NSTAT
};

// Device flags (int32) of the error word.
enum ErrFlag { ERR_BIRTH_OVERFLOW = 1, ERR_CAPACITY = 2, ERR_MG_NOTCONV = 4, ERR_QUEUE_OVERFLOW = 8, ERR_SEE_OVERFLOW = 16 };

struct GridC {
    int nr, nz, nr1, nodes, ncells, ip, window;
    double dr, dz;
    float inv_nr;      // 1 / nr, for the cell -> (i, j) split
};

// Integral of node (i, j)'s weight over the domain: pi (R_{j+1}^2 -
// R_{j-1}^2) / 2 radially for the R^2-linear weight (neighbour radii clipped
// to [0, R_max], so pi dR^2 / 2 on the axis), times dz axially (dz / 2 on
// the end rows).  I / V and q w W / V are then the current and particle
// densities the gather/deposit weight sees.
__device__ __forceinline__ double node_volume(const GridC &g, int i, int j)
{
    const double hi = (double)min(j + 1, g.nr) * g.dr, lo = (double)max(j - 1, 0) * g.dr;
    const double h = (i == 0 || i == g.nz) ? 0.5 * g.dz : g.dz;
    return 1.5707963267948966 * (hi * hi - lo * lo) * h;
}

// cell -> (i, j) with i = floor(cell / nr): (cell + 1/2) / nr is at least
// 1/(2 nr) from an integer and the FP32 product errs by < nz 2^-23, so the
// truncation is exact while nz nr < 2^22 (checked on the host).
__device__ __forceinline__ void split_cell(const GridC &g, int cell, int &i, int &j)
{
    i = (int)(((float)cell + 0.5f) * g.inv_nr);
    j = cell - i * g.nr;
}

struct SpeciesC {
    int s;
    double h;          // (q/m) dt / 2
    double dtr, dtz;   // dt / dR, dt / dz
    int has_b;
    double bt[3], bs[3];  // Boris t and s vectors
    double jscale;     // fixed-point scale of vbar W / vref
    double qscale;     // fixed-point scale of W
    double vref;
    double inv_vref;
    // the same constants rounded to FP32, for the FP32 particle pass (read
    // from the kernel arguments as they are, with no conversion per use)
    float hf, dtrf, dtzf, inv_vreff, jscalef, qscalef, btf[3], bsf[3];
};

// a species constant in the pass's working precision
template <typename T> __device__ __forceinline__ T sc_val(double d, float f);
template <> __device__ __forceinline__ float sc_val<float>(double, float f) { return f; }
template <> __device__ __forceinline__ double sc_val<double>(double d, float) { return d; }

struct MccC {
    uint32_t seed;
    int xs_kind;
    double numax[2];
    double lq[2];      // log(1 - P_null) = -nu_max dt
    double ngas, qe, me, mi, vg;
    double xs[13];
};

// Birth records (structure of arrays), one per ionization event.
template <typename T> struct Births {
    uint32_t *parent;
    int32_t *rank;     // ranks being counted (number of smaller parent ids); zero between steps
    int32_t *cell;
    T *dr, *dz;
    T *ve;             // 3 per record
    T *vi;             // 3 per record
    int32_t *next;     // 2 per record (electron, ion)
    int32_t *count;    // device counter
    int32_t cap;
};

// Queue of this step's null-collision candidates of one species (indices
// into its particle arrays), filled by the streaming pass.
struct CandQueue {
    int32_t *idx;
    void *vel;         // the candidates' v_r, v_theta, v_z after the push (3 x cap, particle precision)
    int32_t *count;
    int32_t cap;
};

// Ions absorbed at a metal wall during the step (ion-induced secondary
// emission): parent id, cell and offsets before the move, the wall (1 bottom,
// 2 top without a window, 3 outer).  count[0]: records queued by the pass,
// count[1]: emitters among them.  cap == 0: emission off.
template <typename T> struct SeeQueue {
    uint32_t *parent;
    int32_t *cell;
    T *dr, *dz;
    int32_t *wall;
    int32_t *rank;          // ranks being counted; zero between steps
    int32_t *count;
    int32_t cap;
    uint32_t pad;
    unsigned long long thr; // emit iff Philox word 0 < thr, i.e. (x + 1/2) 2^-32 < gamma
    double sigma;           // sqrt(T e / m_e) of the emitted electrons
};

template <typename T> struct PassArgs {
    Parts<T> p;
    CandQueue q;
    const int64_t *count;              // slots in use of this species
    const typename Field4<T>::type *ef;
    const typename Field2<T>::type *eb;   // RF magnetic field per node, or none
    long long *accJ;                   // this species' current accumulator
    long long *accQ;                   // this species' charge accumulator
    long long *accW;                   // this species' window charge of the step (weights, fixed point)
    unsigned long long *stats;
    int32_t *err;
    GridC g;
    SpeciesC sc;
    MccC mc;
    Births<T> b;
    SeeQueue<T> see;
    int32_t step;
};

// Both species' arguments of the streaming pass, launched as one grid whose
// first nb0 blocks take the electrons' chunks.
template <typename T> struct PassPair {
    PassArgs<T> a[2];
    int32_t nb0;
};

// One multigrid level (device arrays).  Level 0 is the 5-point finite-
// volume operator (A x)_p = cc x_p - cw x_W - ce x_E - cs x_S - cn x_N; the
// coarser levels are Galerkin products P^T A P with 9-point stencils
// (A x)_p = sum_k a[k][p] x_{p + off(k)}, k = 3 (di + 1) + (dj + 1).
struct MGLevel {
    int nr, nz, nr1, nodes;
    int nine;
    double *phi, *rhs;       // correction and its right-hand side
    double *res;             // residual after the pre-smoother (levels above the bottom)
    const double *cw, *ce, *cs, *cn, *cc;
    const double *a;         // 9 * nodes (nine == 1)
    const uint8_t *dir;      // 1: Dirichlet (correction fixed at 0)
};

constexpr int MAX_LEVELS = 14;
struct MGLevels {
    int n;
    MGLevel L[MAX_LEVELS];
    const double *coarse_inv;   // dense inverse of the bottom operator (Dirichlet rows identity)
    const float *coarse_inv32;  // the same, symmetrised and rounded to FP32 (rows of dense_ld32 floats)
};

// Device-resident state of one preconditioned-CG solve.
constexpr int MAX_CG = 64;
struct MGState {
    int32_t done;
    int32_t cycles;          // CG iterations (one V-cycle each)
    uint32_t ticket;
    int32_t pad;
    double rel;              // max |r| / scale
    double scale;            // max(|b|, |diag x|) at the start of the solve
    double rz[MAX_CG + 1];   // r.z of each iteration
};

constexpr int MAX_TURNS = 16;
// Retained orders of the multiharmonic circuit (order m at frequency m f):
// arrays of per-order data are stored order after order (the fundamental
// first), and a step's phase reaches the kernels as cos, sin of m th_n.
constexpr int MAX_HARM = 4;
struct Orders {
    int n;                          // retained orders (1: fundamental only)
    double cs[MAX_HARM], sn[MAX_HARM];
};
constexpr int SUR_MAX_ITER = 64;        // inner iterations of the surrogate-assisted update at most
// Open-period accumulators (compensated sums: value + correction).
struct HarmState {
    int32_t samples, pad;
    double pind, pind_c;
    double qc[MAX_TURNS], qc_c[MAX_TURNS], qs[MAX_TURNS], qs_c[MAX_TURNS];
    double w[MAX_TURNS], w_c[MAX_TURNS];
    double v_first[MAX_TURNS], q_first[MAX_TURNS], v_prev[MAX_TURNS], q_prev[MAX_TURNS];
};

// Field-circuit coupling (device-resident; one update per closed period).
// Turn currents and voltages are peak phasors under Re[x exp(+i w t)]; the
// network unknowns are x = (I_f, I_1..I_N, V_1..V_N).
constexpr int MAX_X = 2 * MAX_TURNS + 1;
struct CircuitDev {
    int32_t N, nrf, controller, vg_from_target;
    int32_t have_pf, pad;
    double omega, freq, alpha;
    double zs_re, zs_im;                    // source + matching branch impedance
    double rrf[MAX_TURNS], cstray[MAX_TURNS];
    double mvac[MAX_TURNS * MAX_TURNS];     // sum g_k U_l dV; Z_vac = -i mvac
    double p_target, gamma, n_trend, eps_p, alpha_v, f_step, v_min, v_max;
    double vg_amp, vg_phase, pf_prev;
    double x_re[MAX_X], x_im[MAX_X];        // applied state
    double proj[2 * MAX_TURNS];             // sum g_k E_c^p dV, sum g_k E_s^sto,p dV
    // results of the last update
    double xt_re[MAX_X], xt_im[MAX_X];      // target state
    double vp_re[MAX_TURNS], vp_im[MAX_TURNS];
    double qc[MAX_TURNS], qs[MAX_TURNS], icap_re[MAX_TURNS], icap_im[MAX_TURNS], wk[MAX_TURNS];
    double p_port, p_cu, p_ind, p_cap, p_cap_ph, eps_bal, kcl, kvl, eps_rec, pf, pc, vg_old;
    int32_t samples, singular;
    // surrogate-assisted update: plasma moments of the completed period,
    // the correction y_n - yhat(x^n), the inner fixed-point iterate
    double pressure;
    double moments[8];          // <n_e>, <n_i>, max n_e, <eps_e>, <eps_i> (eV), R_e, z_e (m), ionizations (real particles)
    double births_prev;
    int32_t sur_max_iter, sur_iters, sur_used, sur_done;
    double sur_err_max, sur_tol, sur_err;
    double sur_corr[4 * MAX_TURNS];         // (V_p re, im) x N then (I_cap re, im) x N
    double xi_re[MAX_X], xi_im[MAX_X];      // inner iterate
    double vg_iter, sur_step;
    // sums of the second half's iterates (applied as their mean when the
    // inner iteration ends without meeting its tolerance)
    double xa_re[MAX_X], xa_im[MAX_X];
    double vg_acc;
    int32_t sur_navg, pad2;
    double sur_hist[SUR_MAX_ITER];          // relative step of each inner iterate
    // prescribed load responses of the next update (circuit override)
    int32_t ovr_loads, order;               // order: m of this network (1 = fundamental)
    // multiharmonic circuit: this order's source amplitude relative to the
    // fundamental's (its phase offset is folded into vg_phase); in the
    // fundamental's record, the totals over the retained orders of the last
    // update (port power, copper loss, phasor capacitive power, imbalance,
    // largest KCL / KVL residual)
    double vg_ratio;
    double tot_p_port, tot_p_cu, tot_p_cap_ph, tot_eps_bal, tot_kcl, tot_kvl;
    double ovr_vp_re[MAX_TURNS], ovr_vp_im[MAX_TURNS], ovr_icap_re[MAX_TURNS], ovr_icap_im[MAX_TURNS];
};

// Direct Poisson solve of a separable operator (direct.hip): the grid and
// phase, the level-0 conductances, the plan's device arrays and the work
// arrays.  Block row r is node row r + 1; block column j is node column j.
constexpr int DP_MAX_DIRICHLET_DEV = 512;   // interior Dirichlet nodes at most
struct DirectArgs {
    int nr, nz, nodes, ni, nj, m, nrow, nturns;
    Orders o;                               // the step's phase per retained order
    const int32_t *tag;
    const double *vc, *vs, *basis;
    double *phi;
    const double *Q;
    const double *cw, *ce, *cs, *cn;
    const double *v;                        // nj x nj radial eigenvectors, v[j * nj + k]
    const double *lam;                      // nj radial eigenvalues
    const double *zrow;                     // ni: radial conductance factor of block row r
    const double *erow;                     // ni + 1: axial coupling of node rows r and r + 1
    const double *cinv;                     // m x m inverse capacitance matrix
    const double *g;                        // nrow x ni x nj: responses of the modes to unit sources on rows[q]
    const int32_t *dnode, *drow, *rows;     // interior Dirichlet nodes, their row index, the distinct rows
    const int32_t *rowstart;                // nrow + 1: the nodes of row q are dnode[rowstart[q] .. rowstart[q+1])
    double *b, *u, *w;                      // ni x nj right-hand side, ni x nj modes, nrow x nj sources
    double *res, *src;                      // m: phi_D - (S b)_D, and the capacitance sources
};

// features of the surrogate network: (I_k re, im), (V_k re, im), pressure,
// the eight moments; outputs: (V_p,k re, im), (I_cap,k re, im)
constexpr int SUR_MAX_TURNS = 5;

// per-block sums of the plasma moments (electrons: count, energy, R, z;
// ions: count, energy)
constexpr int MOM_SUMS = 6;

}  // namespace pic
