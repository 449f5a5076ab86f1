// Host-side launchers of the kernels (implemented next to the kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "../../include/phasorpic.h"

namespace pic {

template <typename T>
void launch_load(const Parts<T> &p, int64_t n, uint32_t seed, int s, double rmax, double zp, double vth, double lq,
                 const GridC &g, hipStream_t st);
template <typename T>
void launch_place(const Parts<T> &p, int64_t n, const double *R, const double *z, const double *vr,
                  const double *vt, const double *vz, const uint32_t *id, const int32_t *next, const GridC &g,
                  hipStream_t st);
template <typename T>
void launch_unplace(const Parts<T> &p, const int64_t *count, int64_t cap, const int64_t *index, double *R, double *z,
                    double *vr, double *vt, double *vz, uint32_t *id, int32_t *next, const GridC &g, hipStream_t st);
void launch_count_live(const int32_t *cell, const int64_t *count, unsigned long long *out, hipStream_t st);
void launch_live_index(const int32_t *cell, const int64_t *count, int64_t *index, int64_t *nlive, hipStream_t st);
template <typename T>
void launch_pass(const PassArgs<T> &e, const PassArgs<T> &i, int64_t cap_e, int64_t cap_i, bool push, bool depq,
                 hipStream_t st);
template <typename T>
void launch_correct(const PassArgs<T> &e, const PassArgs<T> &i, int64_t cap_e, int64_t cap_i, hipStream_t st);
template <typename T> void launch_collide(const PassArgs<T> &a, hipStream_t st);
template <typename T>
void launch_births(const Births<T> &b, const Parts<T> &pe, const Parts<T> &pi, int64_t *count, int64_t *next_id,
                   int64_t cap_e, int64_t cap_i, long long *accQe, long long *accQi, bool deposit, double qscale,
                   const GridC &g, int32_t *err, unsigned long long *stats, int32_t *q0, int32_t *q1, hipStream_t st);
template <typename T>
void launch_see(const SeeQueue<T> &q, const Parts<T> &pe, int64_t *count, int64_t *next_id, int64_t cap_e,
                long long *accQe, bool deposit, double qscale, const GridC &g, int32_t *err, unsigned long long *stats,
                uint32_t seed, int32_t step, double lq_e, hipStream_t st);
template <typename T>
void launch_sort(const Parts<T> &src, const Parts<T> &dst, int64_t *count, int64_t *count_old, int32_t *hist,
                 int32_t *cursor, int64_t *scanpart, int ncells, int64_t cap, hipStream_t st);
int sort_scan_blocks(int ncells);

template <typename T>
void launch_stage_b(const double *ec, const double *es, double cs, double sn, double inv_w,
                    typename Field2<T>::type *eb, const GridC &g, hipStream_t st);
template <typename T>
void launch_stage(const double *phi, const double *ec, const double *es, const Orders &o,
                  typename Field4<T>::type *ef, long long *accJ, long long *accQ, bool clear_q, const GridC &g,
                  hipStream_t st);
void launch_chi(const long long *accQ, double c0, double c1, double *chi, const double *cw0, const double *ce0,
                const double *cs0, const double *cn0, const MGLevel &L0, const GridC &g, hipStream_t st);
void launch_finalize_q(const long long *accQ, long long *accW, double *accS, double inv_scale, double cq0, double cq1,
                       double cs0, double cs1, double *Q, int nodes, hipStream_t st);
void launch_harmonic(const long long *accJ, double cj0, double cj1, const double *ec, const double *es,
                     const Orders &o, double *I, double *Jc, double *Jcc, double *Js, double *Jsc, double *partial,
                     HarmState *h, const double *Qk, const double *vc, const double *vs, int nturns, int nodes,
                     hipStream_t st);
int harmonic_blocks(int nodes);

struct PCGVec {
    double *x, *b, *r, *z, *p, *Ap;
};
int pcg_partial_size(const MGLevel &L0);
// tile smoother modes (combinable); the smoothed correction is written to
// out, which may be L.phi only with SM_ZERO (otherwise the halo is read there)
constexpr int SM_REVERSE = 1, SM_ZERO = 2, SM_RHS = 4, SM_PROLONG = 8, SM_RZ = 16;
int smooth_blocks(const MGLevel &L);
void launch_mg_smooth_tile(const MGLevel &L, const MGLevel *F, const MGLevel *C, int sweeps, int mode,
                           const MGState *st, double *partial, double *out, hipStream_t s);
void launch_mg_resid(const MGLevel &L, const MGState *st, hipStream_t s);
void launch_mg_restrict_res(const MGLevel &F, const MGLevel &C, const MGState *st, hipStream_t s);
void launch_dense_solve(const float *inv, const MGLevel &L, const MGState *st, hipStream_t s);
int dense_ld32(int n);
void launch_inverse_f32(const double *inv, int n, float *out, hipStream_t s);
// dense inverse of the bottom level: n rows of stride dense_ld(n) (even, so
// that rows start 16-byte aligned)
int dense_ld(int n);
void launch_gauss_jordan(double *A, int n, double *rowk, double *colk, hipStream_t s);
int pcg_blocks(int nodes);
void launch_pcg_begin(const MGLevel &L, const PCGVec &v, const int32_t *tag, const double *vc, const double *vs,
                      const Orders &o, MGState *st, double *prev, int order, hipStream_t s,
                      const double *basis = nullptr, int nturns = 0);
void launch_direct_solve(const DirectArgs &a, hipStream_t st);
void launch_pcg_resid(const MGLevel &L, const PCGVec &v, double *partial, hipStream_t s);
void launch_pcg_check(MGState *st, const double *partial, int np, double rtol, bool first, hipStream_t s,
                      unsigned long long *unconv = nullptr);
void launch_pcg_rz(const MGLevel &L, const PCGVec &v, const MGState *st, double *partial, hipStream_t s);
void launch_pcg_pmatvec(const MGLevel &L, const PCGVec &v, const double *pold, double *pnew, MGState *st,
                        double *partial, int nrz, hipStream_t s);
void launch_pcg_update(const MGLevel &L, const PCGVec &v, const double *p, const MGState *st, double *partial,
                       hipStream_t s);
void launch_helm_rhs(const double *acc, const double *comp, double scale, const uint8_t *dir, double mw, double *b,
                     const GridC &g, hipStream_t s);
void launch_unit_rhs(const int32_t *tag, int turn, double gval, const uint8_t *dir, double mw, double *b,
                     const GridC &g, hipStream_t s);
void launch_project(const double *fields, int nf, int64_t stride, const int32_t *list, const int32_t *lturn, int nlist,
                    const double *gval, int nturns, double *out, int ostride, const GridC &g, hipStream_t s);
void launch_circuit(CircuitDev *cd, const HarmState *h, double *vc, double *vs, int mode, hipStream_t s);
void launch_circuit_orders(CircuitDev *cd, int M, double *vc, double *vs, int mode, hipStream_t s);
void launch_features(const CircuitDev *cd, float *f, bool iterate, hipStream_t s);
void launch_surrogate(CircuitDev *cd, const float *pred, double *vc, double *vs, int stage, hipStream_t s);
template <typename T>
void launch_moments(const Parts<T> &pe, const Parts<T> &pi, const int64_t *count, const long long *accQe,
                    double qscale, double we, double wi, double me, double mi, double qe, double *partial,
                    int np, CircuitDev *cd, const unsigned long long *stats, const GridC &g, hipStream_t st);
int moments_blocks();
void launch_compose(const double *ecp, const double *esp, const double *U, int64_t stride, const CircuitDev *cd,
                    double *ec, double *es, int nodes, hipStream_t s);
void mlp_shape(const mlp_ctx *c, int *n_in, int *n_out, void **stream);
void launch_face_charge(const double *phi, const int32_t *fp, const int32_t *fq, const int32_t *fk, const double *fc,
                        int nfaces, double *Qk, int nturns, hipStream_t s,
                        const double *chi = nullptr);

}  // namespace pic
