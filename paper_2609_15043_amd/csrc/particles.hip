// Particle kernels of the RZ PIC/MCC step: loading, the gather / Boris push
// / move / current deposit pass (optionally fused with the collisions and
// the charge deposit), ionization births, and the counting sort by cell.
//
// Data layout: structure of arrays per species (cell index, in-cell offsets,
// velocity, id, next collision-candidate step), kept sorted by cell every
// few steps so that the 64 lanes of a wave stream contiguous memory and
// mostly share one cell.  Deposits are reduced across the wave (segmented
// by cell), accumulated in an LDS window of node values per block, and
// flushed with one 64-bit fixed-point atomic per touched node.
#include "kernels.h"
#include "launch.h"

namespace pic {

constexpr double PI = 3.141592653589793238462643;

// ---------------------------------------------------------------------------
// Small FP64 helpers of the collision model
// ---------------------------------------------------------------------------
__device__ __forceinline__ double above_threshold(double eps, double th)
{
    if (eps <= th) return 0.0;
    const double x = eps / th;
    return 4.0 * (x - 1.0) / (x * x);
}

// e-Ar: elastic, excitation, ionization cross sections at energy eps (eV)
__device__ __forceinline__ void sigma_electron(const MccC &m, double eps, double &sel, double &sex, double &siz)
{
    if (m.xs_kind == 1) {
        sel = m.xs[0];
        sex = eps > m.xs[3] ? m.xs[2] : 0.0;
        siz = eps > m.xs[5] ? m.xs[4] : 0.0;
        return;
    }
    sel = m.xs[0] / sqrt(1.0 + eps / m.xs[1]);
    sex = m.xs[2] * above_threshold(eps, m.xs[3]);
    siz = m.xs[4] * above_threshold(eps, m.xs[5]);
}

// Ar+-Ar: elastic and charge exchange at centre-of-mass energy (eV)
__device__ __forceinline__ void sigma_ion(const MccC &m, double ecm, double &sel, double &scx)
{
    if (m.xs_kind == 1) {
        sel = m.xs[6];
        scx = m.xs[8];
        return;
    }
    sel = m.xs[6] * pow(1.0 + ecm, -m.xs[7]);
    scx = m.xs[8] * pow(1.0 + ecm, -m.xs[9]);
}

// step of the next candidate after a draw at `step`: step + G,
// G = 1 + floor(log u / log(1 - P)), clamped to int32
__device__ __forceinline__ int32_t next_candidate(int64_t step, uint32_t x, double lq)
{
    double g = floor(log(unit(x)) / lq);
    g = fmin(g, 2.0e9);
    const int64_t s = step + 1 + (int64_t)g;
    return s > 2147483647ll ? 2147483647 : (int32_t)s;
}

__device__ __forceinline__ void isotropic(uint32_t a, uint32_t b, double d[3])
{
    const double ct = 1.0 - 2.0 * unit(a);
    const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double sp, cp;
    sincos(2.0 * PI * unit(b), &sp, &cp);
    d[0] = st * cp;
    d[1] = st * sp;
    d[2] = ct;
}

__device__ __forceinline__ void normal_pair(uint32_t a, uint32_t b, double &g0, double &g1)
{
    const double r = sqrt(-2.0 * log(unit(a)));
    double s, c;
    sincos(2.0 * PI * unit(b), &s, &c);
    g0 = r * c;
    g1 = r * s;
}

// (R, z) in metres -> (cell, offsets); R and z are inside the box
template <typename T>
__device__ __forceinline__ void place(const GridC &g, double R, double z, int32_t &cell, T &dr, T &dz)
{
    const double x = R / g.dr, y = z / g.dz;
    int j = (int)floor(x), i = (int)floor(y);
    j = min(max(j, 0), g.nr - 1);
    i = min(max(i, 0), g.nz - 1);
    double a = x - j, b = y - i;
    T ta = (T)a, tb = (T)b;
    if (ta >= (T)1) ta = (T)0.9999999;
    if (tb >= (T)1) tb = (T)0.9999999;
    cell = i * g.nr + j;
    dr = ta;
    dz = tb;
}

// ---------------------------------------------------------------------------
// Loading: uniform in volume (R = Rmax sqrt(u)), Maxwellian velocities,
// Philox blocks (id, 0, 0, 0) and (id, 0, 1, 0) keyed by (seed, species).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_load(Parts<T> p, int64_t n, uint32_t seed, int s, double rmax, double zp, double vth,
                       double lq, GridC g)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const U4 a = philox10(U4{(uint32_t)k, 0u, 0u, 0u}, seed, (uint32_t)s);
    const U4 b = philox10(U4{(uint32_t)k, 0u, 1u, 0u}, seed, (uint32_t)s);
    const double R = rmax * sqrt(unit(a.x));
    const double z = zp * unit(a.y);
    double g0, g1, g2, g3;
    normal_pair(a.z, a.w, g0, g1);
    normal_pair(b.x, b.y, g2, g3);
    int32_t cell;
    T dr, dz;
    place<T>(g, R, z, cell, dr, dz);
    p.cell[k] = cell;
    p.dr[k] = dr;
    p.dz[k] = dz;
    p.vr[k] = (T)(vth * g0);
    p.vt[k] = (T)(vth * g1);
    p.vz[k] = (T)(vth * g2);
    p.id[k] = (uint32_t)k;
    p.next[k] = next_candidate(-1, b.z, lq);   // first candidate: G - 1
    if (p.fr) p.fr[k] = p.ft[k] = p.fz[k] = (T)0;
}

// Host-given particles (R, z in metres) -> store
template <typename T>
__global__ void k_place(Parts<T> p, int64_t n, const double *R, const double *z, const double *vr,
                        const double *vt, const double *vz, const uint32_t *id, const int32_t *next, GridC g)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int32_t cell;
    T dr, dz;
    place<T>(g, R[k], z[k], cell, dr, dz);
    p.cell[k] = cell;
    p.dr[k] = dr;
    p.dz[k] = dz;
    p.vr[k] = (T)vr[k];
    p.vt[k] = (T)vt[k];
    p.vz[k] = (T)vz[k];
    p.id[k] = id[k];
    p.next[k] = next[k];
    if (p.fr) p.fr[k] = p.ft[k] = p.fz[k] = (T)0;
}

// store -> host representation (only live particles, order of the store)
template <typename T>
__global__ void k_unplace(Parts<T> p, const int64_t *count, const int64_t *live_index, double *R, double *z,
                          double *vr, double *vt, double *vz, uint32_t *id, int32_t *next, GridC g)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= *count) return;
    const int32_t c = p.cell[k];
    if (c < 0) return;
    const int64_t o = live_index[k];
    const int i = c / g.nr, j = c - i * g.nr;
    R[o] = ((double)j + (double)p.dr[k]) * g.dr;
    z[o] = ((double)i + (double)p.dz[k]) * g.dz;
    vr[o] = (double)p.vr[k];
    vt[o] = (double)p.vt[k];
    vz[o] = (double)p.vz[k];
    id[o] = p.id[k];
    next[o] = p.next[k];
}

// ---------------------------------------------------------------------------
// LDS window of node values of one pass block.  Row mode: `rows` whole node
// rows from row ib, stored with a padded row stride ws = 8 (mod 64).  With
// the grid's own stride nr + 1 a node row sits one bank after the row below
// it, so the nodes around a few neighbouring cells all fall in a handful of
// banks and the adds of a wave whose particles spread over those cells
// queue there; with the padded stride adjacent rows are 8 banks apart.
// Linear mode (a row too long for three to fit): nodes [base, base + N).
// ---------------------------------------------------------------------------
struct WinMap {
    int ib, rows, ws, base;   // rows == 0: linear mode
};

__device__ __forceinline__ int win_stride(int nr1) { return nr1 + ((8 - nr1) & 63); }

// window slot of node (r, c), or -1 outside the window
template <int N> __device__ __forceinline__ int win_off(const WinMap &w, int r, int c, int nr1)
{
    if (w.rows) {
        const int d = r - w.ib;
        return (unsigned)d < (unsigned)w.rows ? d * w.ws + c : -1;
    }
    const int o = r * nr1 + c - w.base;
    return (unsigned)o < (unsigned)N ? o : -1;
}

// One node value, in the accumulator's 64-bit fixed point, to the window
// (an integer LDS add: exact, independent of order, and on this hardware
// an order of magnitude faster than a floating-point LDS add) or, outside
// the window, to the global accumulator.
template <typename T>
__device__ __forceinline__ void deposit_node(const WinMap &w, int r, int c, T v, long long *win, long long *acc,
                                             int nr1, T scale, int &nout)
{
    const long long f = to_fixed_fast(v, scale);
    const int o = win_off<Win<T>::N>(w, r, c, nr1);
    if (o >= 0) {
        atomicAdd(reinterpret_cast<unsigned long long *>(&win[o]), static_cast<unsigned long long>(f));
    } else {
        atomic_add_i64(&acc[r * nr1 + c], f);
        ++nout;
    }
}

// Four node values of one particle in cell (i, j) straight into the window
// (or the global accumulator outside it): the per-lane path.
template <typename T>
__device__ __forceinline__ void deposit_lane(int i, int j, T v0, T v1, T v2, T v3, long long *win, const WinMap &w,
                                             long long *acc, int nr1, T scale, int &nout)
{
    deposit_node<T>(w, i, j, v0, win, acc, nr1, scale, nout);
    deposit_node<T>(w, i, j + 1, v1, win, acc, nr1, scale, nout);
    deposit_node<T>(w, i + 1, j, v2, win, acc, nr1, scale, nout);
    deposit_node<T>(w, i + 1, j + 1, v3, win, acc, nr1, scale, nout);
}

// ---------------------------------------------------------------------------
// Wave-collective deposit of four node values around the lower-left node
// (i, j) of each lane's run.  Lanes are grouped by cell (segmented by
// ballot); each group's four node sums (wave scan, total in lane 63) are
// formed in the working precision and converted to 64-bit fixed point one
// value at a time (deposit_node) as they are added to the block's LDS
// window, or, for a node outside the window, to the global fixed-point
// accumulator.  The integer adds are exact and independent of order, so a
// node's total depends only on which particles share a wave: the in-wave
// sums round in the working precision in the particle order the cell sort
// leaves, and the sort orders the particles within a cell by atomics, so
// two runs may differ in the last bits.  Called by all 64 lanes.
// ---------------------------------------------------------------------------
// lane 63's value in every lane (a wave total after wave_total)
__device__ __forceinline__ float lane63(float v)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double lane63(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (long long)(uint32_t)lo);
}

template <typename T>
__device__ __forceinline__ void deposit4(bool valid, int i, int j, T v0, T v1, T v2, T v3, long long *win,
                                         const WinMap &w, long long *acc, int nr1, T scale, int &nout)
{
    const int key = i * nr1 + j;
    uint64_t todo = ballot(valid);
    const int lane = lane_id();
    // wave reductions for groups of at least DEPOSIT_MIN_LANES lanes (at most
    // DEPOSIT_GROUPS of them); the lanes of smaller groups (a wave whose
    // particles drifted apart since the sort) add their own values, an
    // integer LDS add being cheaper than a reduction for a few lanes
    for (int it = 0; todo && it < DEPOSIT_GROUPS; ++it) {
        const int lead = __ffsll((unsigned long long)todo) - 1;
        const int k = __builtin_amdgcn_readlane(key, lead);
        const bool m = valid && key == k;
        const uint64_t mm = ballot(m);
        if (__popcll(mm) < DEPOSIT_MIN_LANES) break;
        const int ki = __builtin_amdgcn_readlane(i, lead), kj = __builtin_amdgcn_readlane(j, lead);
        const T s0 = lane63(wave_total(m ? v0 : (T)0));
        const T s1 = lane63(wave_total(m ? v1 : (T)0));
        const T s2 = lane63(wave_total(m ? v2 : (T)0));
        const T s3 = lane63(wave_total(m ? v3 : (T)0));
        // the four node sums are added by lanes 0..3 at once
        if (lane < 4) {
            const T v = lane == 0 ? s0 : lane == 1 ? s1 : lane == 2 ? s2 : s3;
            if (v != (T)0) deposit_node<T>(w, ki + (lane >> 1), kj + (lane & 1), v, win, acc, nr1, scale, nout);
        }
        todo &= ~mm;
    }
    if (todo >> lane & 1ull) deposit_lane<T>(i, j, v0, v1, v2, v3, win, w, acc, nr1, scale, nout);
}

__device__ __forceinline__ void count_wave(bool c, unsigned long long *sstat, int slot)
{
    const uint64_t m = ballot(c);
    if (m && lane_id() == __ffsll((unsigned long long)m) - 1) atomicAdd(&sstat[slot], (unsigned long long)__popcll(m));
}

// ---------------------------------------------------------------------------
// Collision of one candidate (FP64 inside).  Velocity in/out in the local
// frame at the particle's position.  Returns the process index or -1.
// ---------------------------------------------------------------------------
template <typename T>
__device__ int collide(const MccC &mc, int s, uint32_t id, int32_t step, T &vr, T &vt, T &vz, int32_t &next,
                       bool &over, bool &born, double ve[3], double vi[3], int32_t nb[2])
{
    const U4 b0 = philox10(U4{id, (uint32_t)step, 1u, 0u}, mc.seed, (uint32_t)s);
    next = next_candidate(step, b0.x, mc.lq[s]);
    double v[3] = {(double)vr, (double)vt, (double)vz};
    int ev = -1;
    if (s == 0) {
        const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        const double speed = sqrt(v2);
        const double eps = 0.5 * mc.me * v2 / mc.qe;
        double sel, sex, siz;
        sigma_electron(mc, eps, sel, sex, siz);
        const double nel = mc.ngas * sel * speed, nex = mc.ngas * sex * speed, niz = mc.ngas * siz * speed;
        over = nel + nex + niz > mc.numax[0];
        const double Rv = unit(b0.y) * mc.numax[0];
        double d[3];
        isotropic(b0.z, b0.w, d);
        double e1 = -1.0;
        if (Rv < nel) {
            const double cchi = speed > 0.0 ? (v[0] * d[0] + v[1] * d[1] + v[2] * d[2]) / speed : 1.0;
            e1 = eps * (1.0 - 2.0 * mc.me / mc.mi * (1.0 - cchi));
            ev = 0;
        } else if (Rv < nel + nex) {
            e1 = eps - mc.xs[3];
            ev = 1;
        } else if (Rv < nel + nex + niz) {
            const U4 b2 = philox10(U4{id, (uint32_t)step, 2u, 0u}, mc.seed, 0u);
            const U4 b3 = philox10(U4{id, (uint32_t)step, 3u, 0u}, mc.seed, 0u);
            const double erem = eps - mc.xs[5];
            const double esec = unit(b2.x) * erem;
            e1 = erem - esec;
            double d2[3];
            isotropic(b2.y, b2.z, d2);
            const double s2 = sqrt(2.0 * esec * mc.qe / mc.me);
            double g0, g1, g2, g3;
            normal_pair(b3.x, b3.y, g0, g1);
            normal_pair(b3.z, b3.w, g2, g3);
            ve[0] = s2 * d2[0];
            ve[1] = s2 * d2[1];
            ve[2] = s2 * d2[2];
            vi[0] = mc.vg * g0;
            vi[1] = mc.vg * g1;
            vi[2] = mc.vg * g2;
            nb[0] = next_candidate(step, b2.w, mc.lq[0]);
            nb[1] = next_candidate(step, b3.w, mc.lq[1]);
            born = true;
            ev = 2;
        }
        if (ev >= 0) {
            const double s1 = sqrt(2.0 * e1 * mc.qe / mc.me);
            vr = (T)(s1 * d[0]);
            vt = (T)(s1 * d[1]);
            vz = (T)(s1 * d[2]);
        }
    } else {
        const U4 b2 = philox10(U4{id, (uint32_t)step, 2u, 0u}, mc.seed, 1u);
        double g0, g1, g2, g3;
        normal_pair(b2.x, b2.y, g0, g1);
        normal_pair(b2.z, b2.w, g2, g3);
        const double vn[3] = {mc.vg * g0, mc.vg * g1, mc.vg * g2};
        const double gv[3] = {v[0] - vn[0], v[1] - vn[1], v[2] - vn[2]};
        const double gm = sqrt(gv[0] * gv[0] + gv[1] * gv[1] + gv[2] * gv[2]);
        const double ecm = 0.25 * mc.mi * gm * gm / mc.qe;
        double sel, scx;
        sigma_ion(mc, ecm, sel, scx);
        const double nel = mc.ngas * sel * gm, ncx = mc.ngas * scx * gm;
        over = nel + ncx > mc.numax[1];
        const double Rv = unit(b0.y) * mc.numax[1];
        if (Rv < nel) {
            double d[3];
            isotropic(b0.z, b0.w, d);
            vr = (T)(0.5 * (v[0] + vn[0]) + 0.5 * gm * d[0]);
            vt = (T)(0.5 * (v[1] + vn[1]) + 0.5 * gm * d[1]);
            vz = (T)(0.5 * (v[2] + vn[2]) + 0.5 * gm * d[2]);
            ev = 0;
        } else if (Rv < nel + ncx) {
            vr = (T)vn[0];
            vt = (T)vn[1];
            vz = (T)vn[2];
            ev = 1;
        }
    }
    return ev;
}

// ---------------------------------------------------------------------------
// 16-byte vector access to four consecutive particles of one lane.
// ---------------------------------------------------------------------------
// The particle stream is touched once per pass: its loads and stores carry
// the non-temporal hint, so the lines it moves leave the caches first and
// the staged field nodes (gathered many times per block) stay.  Measured on
// the large workload: pass 0.789 -> 0.737 ms per launch, step 1.093 ->
// 1.019 ms over 200 steps.
#ifndef PIC_STREAM_NT
#define PIC_STREAM_NT 1
#endif
template <typename V> __device__ __forceinline__ V ldv(const V *p)
{
    if constexpr (PIC_STREAM_NT != 0) return __builtin_nontemporal_load(p);
    else return *p;
}
template <typename V> __device__ __forceinline__ void stv(V *p, V v)
{
    if constexpr (PIC_STREAM_NT != 0) __builtin_nontemporal_store(v, p);
    else *p = v;
}
__device__ __forceinline__ void ld4(const float *p, float (&o)[4])
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 v = ldv(reinterpret_cast<const f4 *>(p));
    o[0] = v.x, o[1] = v.y, o[2] = v.z, o[3] = v.w;
}
// FP64 stream: plain loads and stores (pass 1.428 ms per launch against 1.453
// with the hint on both and 1.470 with it on the loads alone; its two
// 16-byte stores per run wrote 9 % more to HBM with the hint)
#ifndef PIC_STREAM_NT_F64_LOAD
#define PIC_STREAM_NT_F64_LOAD 0
#endif
#ifndef PIC_STREAM_NT_F64_STORE
#define PIC_STREAM_NT_F64_STORE 0
#endif
__device__ __forceinline__ void ld4(const double *p, double (&o)[4])
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 *q = reinterpret_cast<const d2 *>(p);
    d2 u, v;
    if constexpr (PIC_STREAM_NT_F64_LOAD != 0) {
        u = ldv(q);
        v = ldv(q + 1);
    } else {
        u = q[0];
        v = q[1];
    }
    o[0] = u.x, o[1] = u.y, o[2] = v.x, o[3] = v.y;
}
__device__ __forceinline__ void ld4(const int32_t *p, int32_t (&o)[4])
{
    typedef int i4 __attribute__((ext_vector_type(4)));
    const i4 v = ldv(reinterpret_cast<const i4 *>(p));
    o[0] = v.x, o[1] = v.y, o[2] = v.z, o[3] = v.w;
}
__device__ __forceinline__ void st4(float *p, const float (&o)[4])
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    stv(reinterpret_cast<f4 *>(p), f4{o[0], o[1], o[2], o[3]});
}
__device__ __forceinline__ void st4(double *p, const double (&o)[4])
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 *q = reinterpret_cast<d2 *>(p);
    if constexpr (PIC_STREAM_NT_F64_STORE != 0) {
        stv(q, d2{o[0], o[1]});
        stv(q + 1, d2{o[2], o[3]});
    } else {
        q[0] = d2{o[0], o[1]};
        q[1] = d2{o[2], o[3]};
    }
}
__device__ __forceinline__ void st4(int32_t *p, const int32_t (&o)[4])
{
    typedef int i4 __attribute__((ext_vector_type(4)));
    stv(reinterpret_cast<i4 *>(p), i4{o[0], o[1], o[2], o[3]});
}

// R^2-linear radial and linear axial weights of the four cell nodes
template <typename T>
__device__ __forceinline__ void node_weights(int j, T dr, T dz, T &w00, T &w01, T &w10, T &w11)
{
    const T fj = (T)j;
    const T wr1 = quot(dr * ((T)2 * fj + dr), (T)2 * fj + (T)1);
    w00 = ((T)1 - dz) * ((T)1 - wr1);
    w01 = ((T)1 - dz) * wr1;
    w10 = dz * ((T)1 - wr1);
    w11 = dz * wr1;
}

// ---------------------------------------------------------------------------
// The particle pass.  Each lane takes runs of four consecutive particles
// (16-byte vector loads; a wave reads 1 KiB contiguous per instruction).
// PUSH: gather + Boris + move + J deposit + absorption, and this step's
// collision candidates (next == step) go to a queue; DEPQ: charge deposit
// at the (new) positions.  Fused: both in one streaming pass.  Deposits
// accumulate in registers over the run (particles of one cell), then one
// wave reduction per run; the collisions run in k_collide over the queue.
// ---------------------------------------------------------------------------
// At least PIC_PASS_WAVES_PER_EU waves per SIMD for the FP32 pass and 3 for
// the FP64 one (the register budget is held to fit them)
#ifndef PIC_PASS_WAVES_PER_EU
#define PIC_PASS_WAVES_PER_EU 4
#endif
template <typename T> struct PassOcc {
    static constexpr int min_waves = sizeof(T) == 4 ? PIC_PASS_WAVES_PER_EU : 3;
};
#define PIC_PASS_OCCUPANCY __attribute__((amdgpu_waves_per_eu(PassOcc<T>::min_waves, 8)))
// RFB: the RF magnetic field staged per node (eb) joins the uniform field
// in the Boris rotation, with the rotation vector formed per particle.
// DI: the predictor of the direct-implicit update: the electrostatic kick is
// the particle's filtered half kick (dt/2) abar^{n-1} (arrays fr, ft, fz),
// the inductive kick dt (q/m) E_theta(t_n) is explicit, and the filter turns
// with the velocity at the move; no collision candidates (the corrector
// takes them).
#ifndef PIC_PASS_GATHER_AHEAD
#define PIC_PASS_GATHER_AHEAD 1
#endif
#ifndef PIC_PASS_PREFETCH_RUN
#define PIC_PASS_PREFETCH_RUN 1
#endif
#ifndef PIC_PASS_WINDOW_FROM_RUN
#define PIC_PASS_WINDOW_FROM_RUN 1
#endif
template <typename T, bool PUSH, bool DEPQ, bool RFB, bool DI>
__global__ __launch_bounds__(BLOCK) PIC_PASS_OCCUPANCY void k_pass(PassPair<T> pp)
{
    // FP64: no registers to spare; RF magnetic field: its node loads would
    // still wait per particle, and the ahead registers slowed that pass
    constexpr bool GATHER_AHEAD = PIC_PASS_GATHER_AHEAD != 0 && sizeof(T) == 4 && !RFB;
    constexpr int RUNS = PassShape<T>::runs, CHUNK = PassShape<T>::chunk;
    // one grid for both species: blocks [0, nb0) take the electrons' chunks,
    // the rest the ions', so the ions' blocks fill the CUs as the electrons'
    // drain instead of waiting for a second launch
    const int sp = (int)blockIdx.x >= pp.nb0 ? 1 : 0;
    const PassArgs<T> &a = pp.a[sp];
    const int64_t bid = (int64_t)blockIdx.x - (sp ? pp.nb0 : 0);
    using F4 = typename Field4<T>::type;
    constexpr int WIN = Win<T>::N;
    __shared__ long long winJ[PUSH ? WIN : 1];   // fixed point, the accumulators' scales
    __shared__ long long winQ[DEPQ ? WIN : 1];
    __shared__ unsigned long long sstat[ST_NSTAT];
    __shared__ WinMap s_w;
    constexpr int CAND_LDS = PUSH ? 512 : 1;
    __shared__ int32_t s_cand[CAND_LDS];
    __shared__ int s_ncand, s_qbase;

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int64_t n = *a.count;
    // chunks in reverse order: the tail of the arrays (births appended since
    // the last sort, in no cell order) is the slowest to deposit, so its
    // blocks start first and overlap the streaming of the sorted bulk
    const int64_t nchunks = (n + CHUNK - 1) / CHUNK;
    if (bid >= nchunks) return;
    const int64_t c0 = (nchunks - 1 - bid) * CHUNK;
    const int64_t c1 = min(c0 + (int64_t)CHUNK, n);
    const GridC g = a.g;
    const int s = a.sc.s;
    if (tid == 0) s_ncand = 0;

    const int64_t wbase = c0 + (int64_t)(tid >> 6) * (RUN * RUNS * 64);
    int32_t cell[RUN], nxt[RUN];
    T dr[RUN], dz[RUN], vr[RUN], vt[RUN], vz[RUN];
    T kr[DI ? RUN : 1], kt[DI ? RUN : 1], kz[DI ? RUN : 1];   // direct-implicit filter
    // a run's particles; the next run's loads are issued right after this
    // run's stores (its registers are free then), so that their latency
    // overlaps this run's deposit reductions
    auto load_run = [&](int64_t q) {
        ld4(a.p.cell + q, cell);
        ld4(a.p.dr + q, dr);
        ld4(a.p.dz + q, dz);
        if (PUSH) {
            ld4(a.p.vr + q, vr);
            ld4(a.p.vt + q, vt);
            ld4(a.p.vz + q, vz);
            ld4(a.p.next + q, nxt);
            if constexpr (DI) {
                ld4(a.p.fr + q, kr);
                ld4(a.p.ft + q, kt);
                ld4(a.p.fz + q, kz);
            }
        }
    };
    // the first run's loads do not depend on the window: issued first, their
    // latency overlaps the window set-up below
    load_run(wbase + RUN * lane);

    if (tid < 64) {
        // window centre: mean row of 64 particles (one hot particle far from
        // the rest cannot shift it by much).  Taken from the first particle
        // of each lane's first run, already loaded by wave 0, rather than from
        // 64 extra scattered loads across the chunk (one 128-byte line each,
        // about 1 B per particle of extra traffic)
        int cl;
        if constexpr (PIC_PASS_WINDOW_FROM_RUN != 0) {
            cl = c0 + RUN * tid < c1 ? cell[0] : -1;
        } else {
            const int64_t q = c0 + (int64_t)tid * (CHUNK / 64);
            cl = q < c1 ? a.p.cell[q] : -1;
        }
        int ci = 0, cj = 0;
        if (cl >= 0) split_cell(g, cl, ci, cj);
        const float sr = wave_total(cl >= 0 ? (float)ci : 0.f);
        const float sc = wave_total(cl >= 0 ? (float)cj : 0.f);
        const float sn = wave_total(cl >= 0 ? 1.f : 0.f);
        if (tid == 63) {
        const int i = sn > 0.f ? (int)(sr / sn) : 0;
        const int j = sn > 0.f ? (int)(sc / sn) : 0;
        WinMap w;
        w.ws = win_stride(g.nr1);
        const int nrows = g.nodes / g.nr1;   // node rows of the grid
        w.rows = min(WIN / w.ws, nrows);
        if (w.rows >= min(3, nrows)) {
            w.ib = max(0, min(i - (w.rows - 1) / 2, nrows - w.rows));
            w.base = 0;
        } else {
            w.rows = 0;
            w.ib = 0;
            const int base = i * g.nr1 + j + g.nr1 / 2 + 1 - WIN / 2;
            w.base = max(min(base, g.nodes - WIN), 0);
        }
        s_w = w;
        }
    }
    for (int k = tid; k < WIN; k += BLOCK) {
        if (PUSH) winJ[k] = 0;
        if (DEPQ) winQ[k] = 0;
    }
    if (tid < ST_NSTAT) sstat[tid] = 0;
    __syncthreads();
    const WinMap w = s_w;
    const T jscale = sc_val<T>(a.sc.jscale, a.sc.jscalef), qscale = sc_val<T>(a.sc.qscale, a.sc.qscalef);   // powers of two
    int nout = 0;   // this lane's deposits outside the window

    for (int r = 0; r < RUNS; ++r) {
        const int64_t q0 = wbase + (int64_t)r * (RUN * 64) + RUN * lane;
        if (!PIC_PASS_PREFETCH_RUN && r > 0) load_run(q0);
        bool live[RUN];
#pragma unroll
        for (int k = 0; k < RUN; ++k) live[k] = q0 + k < c1 && cell[k] >= 0;

        // lane's run sums around its key nodes (old cell for J, new for Q)
        int iJ = -1, jJ = 0, iQ = -1, jQ = 0;   // each run's first cell (row, column)
        T aJ[4] = {0, 0, 0, 0}, aQ[4] = {0, 0, 0, 0};
        uint32_t abs_bits = 0;    // bit k: particle k of the run was absorbed
        uint32_t cand_bits = 0;
        bool moved = false;   // a particle of the run changed cell (or was absorbed)
        // field nodes one particle ahead: the next particle's four node loads
        // are in flight while this one is pushed and deposited, so a run
        // waits on one cache round trip instead of four
        F4 n00, n01, n10, n11;
        auto gather_nodes = [&](int k) {
            int key = 0;   // a dead slot reads node 0 and ignores it
            if (live[k]) {
                int i, j;
                split_cell(g, cell[k], i, j);
                key = i * g.nr1 + j;
            }
            n00 = a.ef[key];
            n01 = a.ef[key + 1];
            n10 = a.ef[key + g.nr1];
            n11 = a.ef[key + g.nr1 + 1];
        };
        if constexpr (PUSH && GATHER_AHEAD) gather_nodes(0);
#pragma unroll
        for (int k = 0; k < RUN; ++k) {
            F4 c00, c01, c10, c11;
            if constexpr (PUSH && GATHER_AHEAD) {
                c00 = n00, c01 = n01, c10 = n10, c11 = n11;
                if (k + 1 < RUN) gather_nodes(k + 1);
            }
            if (PUSH && live[k]) {
                int i, j;
                split_cell(g, cell[k], i, j);
                T w00, w01, w10, w11;
                node_weights<T>(j, dr[k], dz[k], w00, w01, w10, w11);
                const int key = i * g.nr1 + j;
                F4 f00, f01, f10, f11;
                if constexpr (GATHER_AHEAD) {
                    f00 = c00, f01 = c01, f10 = c10, f11 = c11;
                } else {
                    f00 = a.ef[key], f01 = a.ef[key + 1], f10 = a.ef[key + g.nr1], f11 = a.ef[key + g.nr1 + 1];
                }
                const T er = w00 * f00.x + w01 * f01.x + w10 * f10.x + w11 * f11.x;
                const T ez = w00 * f00.y + w01 * f01.y + w10 * f10.y + w11 * f11.y;
                const T et = w00 * f00.z + w01 * f01.z + w10 * f10.z + w11 * f11.z;
                const T h = sc_val<T>(a.sc.h, a.sc.hf);
                T ur = vr[k] + h * er, ut = vt[k] + h * et, uz = vz[k] + h * ez;
                if constexpr (DI) {
                    // electrostatic part from the filter, inductive part explicit
                    ur = vr[k] + kr[k];
                    ut = vt[k] + kt[k] + (T)2 * h * et;
                    uz = vz[k] + kz[k];
                } else if constexpr (RFB) {
                    using F2 = typename Field2<T>::type;
                    const F2 b00 = a.eb[key], b01 = a.eb[key + 1], b10 = a.eb[key + g.nr1], b11 = a.eb[key + g.nr1 + 1];
                    const T br = w00 * b00.x + w01 * b01.x + w10 * b10.x + w11 * b11.x;
                    const T bz = w00 * b00.y + w01 * b01.y + w10 * b10.y + w11 * b11.y;
                    // t = (q/m) (B_uniform + B_rf) dt / 2, s = 2 t / (1 + t^2)
                    const T t0 = sc_val<T>(a.sc.bt[0], a.sc.btf[0]) + h * br, t1 = sc_val<T>(a.sc.bt[1], a.sc.btf[1]),
                            t2 = sc_val<T>(a.sc.bt[2], a.sc.btf[2]) + h * bz;
                    const T f = quot((T)2, (T)1 + (t0 * t0 + t1 * t1 + t2 * t2));
                    const T s0 = f * t0, s1 = f * t1, s2 = f * t2;
                    const T pr = ur + (ut * t2 - uz * t1), pt = ut + (uz * t0 - ur * t2), pz = uz + (ur * t1 - ut * t0);
                    ur += pt * s2 - pz * s1;
                    ut += pz * s0 - pr * s2;
                    uz += pr * s1 - pt * s0;
                } else if (a.sc.has_b) {
                    const T t0 = sc_val<T>(a.sc.bt[0], a.sc.btf[0]), t1 = sc_val<T>(a.sc.bt[1], a.sc.btf[1]),
                            t2 = sc_val<T>(a.sc.bt[2], a.sc.btf[2]);
                    const T s0 = sc_val<T>(a.sc.bs[0], a.sc.bsf[0]), s1 = sc_val<T>(a.sc.bs[1], a.sc.bsf[1]),
                            s2 = sc_val<T>(a.sc.bs[2], a.sc.bsf[2]);
                    const T pr = ur + (ut * t2 - uz * t1), pt = ut + (uz * t0 - ur * t2), pz = uz + (ur * t1 - ut * t0);
                    ur += pt * s2 - pz * s1;
                    ut += pz * s0 - pr * s2;
                    uz += pr * s1 - pt * s0;
                }
                if constexpr (!DI) {
                    ur += h * er;
                    ut += h * et;
                    uz += h * ez;
                }
                // azimuthal current at x^n with the time-centred v_theta
                const T jv = (T)0.5 * (vt[k] + ut) * sc_val<T>(a.sc.inv_vref, a.sc.inv_vreff);
                if (iJ < 0) iJ = i, jJ = j;
                if (i == iJ && j == jJ) {
                    aJ[0] += jv * w00;
                    aJ[1] += jv * w01;
                    aJ[2] += jv * w10;
                    aJ[3] += jv * w11;
                } else {
                    deposit_lane<T>(i, j, jv * w00, jv * w01, jv * w10, jv * w11, winJ, w, a.accJ, g.nr1,
                                    jscale, nout);
                }
                // Cartesian move in the particle's plane, in cell units
                const T fj = (T)j;
                const T ar = dr[k] + ur * sc_val<T>(a.sc.dtr, a.sc.dtrf);
                const T X = fj + ar;
                const T Y = ut * sc_val<T>(a.sc.dtr, a.sc.dtrf);
                const T hyp = root(X * X + Y * Y);
                const T rel = X > (T)0 ? ar + quot(Y * Y, X + hyp) : hyp - fj;   // R' - j
                T c = (T)1, sn = (T)0;
                if (hyp > (T)0) {
                    c = quot(X, hyp);
                    sn = quot(Y, hyp);
                }
                const T vrn = c * ur + sn * ut;
                const T vtn = -sn * ur + c * ut;
                if constexpr (DI) {
                    const T k0 = kr[k], k1 = kt[k];
                    kr[k] = c * k0 + sn * k1;
                    kt[k] = -sn * k0 + c * k1;
                }
                const T fr = floor(rel);
                int jn = j + (int)fr;
                T drn = rel - fr;
                if (drn >= (T)1) {
                    drn -= (T)1;
                    jn += 1;
                }
                const T bz = dz[k] + uz * sc_val<T>(a.sc.dtz, a.sc.dtzf);
                const T fz = floor(bz);
                int in = i + (int)fz;
                T dzn = bz - fz;
                if (dzn >= (T)1) {
                    dzn -= (T)1;
                    in += 1;
                }
                int absorbed = 0;
                if (!(hyp == hyp) || !(bz == bz) || in < 0) {
                    absorbed = 1;   // below the bottom wall (or a non-finite state)
                } else if (in >= g.ip) {
                    absorbed = 1;
                    if (g.window && uz > (T)0) {
                        // crossing of z = zp within the step (FP64)
                        const double frac = ((double)g.ip - ((double)i + (double)dz[k])) / ((double)uz * a.sc.dtz);
                        const double xs = (double)j + (double)dr[k] + (double)ur * a.sc.dtr * frac;
                        const double ys = (double)ut * a.sc.dtr * frac;
                        const double Rs = sqrt(xs * xs + ys * ys);
                        if (Rs < (double)g.nr) {
                            int js = (int)floor(Rs);
                            js = min(js, g.nr - 1);
                            const double w1 = (Rs * Rs - (double)js * js) / (2.0 * js + 1.0);
                            const int nd = g.ip * g.nr1 + js;
                            // fixed point, like the node charge: integer adds
                            // are exact and independent of order
                            atomic_add_i64(&a.accW[nd], to_fixed(1.0 - w1, a.sc.qscale));
                            atomic_add_i64(&a.accW[nd + 1], to_fixed(w1, a.sc.qscale));
                            absorbed = 2;
                        }
                    }
                } else if (jn >= g.nr || jn < 0) {
                    absorbed = 1;
                }
                if (absorbed == 1 && a.see.cap > 0 && hyp == hyp && bz == bz) {
                    // an ion at a metal wall: queued for secondary emission
                    // with its position before the move
                    const int slot = atomicAdd(a.see.count, 1);
                    if (slot < a.see.cap) {
                        a.see.parent[slot] = a.p.id[q0 + k];
                        a.see.cell[slot] = i * g.nr + j;
                        a.see.dr[slot] = dr[k];
                        a.see.dz[slot] = dz[k];
                        a.see.wall[slot] = in < 0 ? 1 : (in >= g.ip && !g.window ? 2 : 3);
                    } else {
                        atomicOr(a.err, (int)ERR_SEE_OVERFLOW);
                    }
                }
                if (absorbed) abs_bits |= 1u << k;
                live[k] = absorbed == 0;
                const int32_t cn = live[k] ? in * g.nr + jn : -1;
                moved |= cn != cell[k];
                cell[k] = cn;
                dr[k] = drn;
                dz[k] = dzn;
                vr[k] = vrn;
                vt[k] = vtn;
                vz[k] = uz;
                if (!DI && live[k] && nxt[k] == a.step) cand_bits |= 1u << k;
            }
            if (DEPQ && live[k]) {
                int i, j;
                split_cell(g, cell[k], i, j);
                T w00, w01, w10, w11;
                node_weights<T>(j, dr[k], dz[k], w00, w01, w10, w11);
                if (iQ < 0) iQ = i, jQ = j;
                if (i == iQ && j == jQ) {
                    aQ[0] += w00;
                    aQ[1] += w01;
                    aQ[2] += w10;
                    aQ[3] += w11;
                } else {
                    deposit_lane<T>(i, j, w00, w01, w10, w11, winQ, w, a.accQ, g.nr1, qscale, nout);
                }
            }
        }
        if constexpr (PUSH) {
            // the cell array is written only where it changed: ions cross a
            // cell edge every ~1e4 steps, electrons every ~20
            if (moved) st4(a.p.cell + q0, cell);
            st4(a.p.dr + q0, dr);
            st4(a.p.dz + q0, dz);
            st4(a.p.vr + q0, vr);
            st4(a.p.vt + q0, vt);
            st4(a.p.vz + q0, vz);
            if constexpr (DI) {
                st4(a.p.fr + q0, kr);
                st4(a.p.ft + q0, kt);
                st4(a.p.fz + q0, kz);
            }
            // this step's collision candidates -> block-local list (LDS), one
            // global reservation per block at the end
            // candidates of the lanes below this one and of the whole wave,
            // from one ballot per run position (no shuffles)
            int before = 0, wtot = 0;
#pragma unroll
            for (int k = 0; k < RUN; ++k) {
                const uint64_t bk = ballot(cand_bits >> k & 1u);
                before += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bk >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)bk, 0u));
                wtot += (int)__popcll(bk);
            }
            int slot0 = 0;
            if (wtot) {
                if (lane == 63) slot0 = atomicAdd(&s_ncand, wtot);
                slot0 = __builtin_amdgcn_readlane(slot0, 63);
            }
            int slot = slot0 + before;
#pragma unroll
            for (int k = 0; k < RUN; ++k) {
                if (!(cand_bits >> k & 1u)) continue;
                if (slot < CAND_LDS) {
                    s_cand[slot] = (int32_t)(q0 + k);
                } else {
                    const int gs = atomicAdd(a.q.count, 1);
                    if (gs < a.q.cap) {
                        T *qv = static_cast<T *>(a.q.vel);
                        a.q.idx[gs] = (int32_t)(q0 + k);
                        qv[gs] = vr[k];
                        qv[a.q.cap + gs] = vt[k];
                        qv[2 * a.q.cap + gs] = vz[k];
                    } else
                        atomicOr(a.err, (int)ERR_QUEUE_OVERFLOW);
                }
                ++slot;
            }
        }
        if (PIC_PASS_PREFETCH_RUN && r + 1 < RUNS) load_run(q0 + RUN * 64);
        if constexpr (PUSH) {
            deposit4<T>(iJ >= 0, iJ, jJ, aJ[0], aJ[1], aJ[2], aJ[3], winJ, w, a.accJ, g.nr1, jscale, nout);
            // absorbed count of the wave, from one ballot per run position
            int tot = 0;
#pragma unroll
            for (int k = 0; k < RUN; ++k) tot += (int)__popcll(ballot(abs_bits >> k & 1u));
            if (lane == 0 && tot) atomicAdd(&sstat[ST_ABS0 + s], (unsigned long long)tot);
        }
        if constexpr (DEPQ)
            deposit4<T>(iQ >= 0, iQ, jQ, aQ[0], aQ[1], aQ[2], aQ[3], winQ, w, a.accQ, g.nr1, qscale, nout);
    }
    {
        int tot = nout;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
        if (lane == 0 && tot) atomicAdd(&sstat[ST_WINOUT], (unsigned long long)tot);
    }
    __syncthreads();
    if constexpr (PUSH) {
        const int nc = min(s_ncand, CAND_LDS);
        if (tid == 0) s_qbase = nc ? atomicAdd(a.q.count, nc) : 0;
        __syncthreads();
        // queue records: index and the velocity after the push (written by
        // this block above, read back from L2), so that the collisions read
        // them contiguously instead of from scattered particle slots
        T *qv = static_cast<T *>(a.q.vel);
        for (int k = tid; k < nc; k += BLOCK) {
            const int gs = s_qbase + k;
            if (gs < a.q.cap) {
                const int32_t p = s_cand[k];
                a.q.idx[gs] = p;
                qv[gs] = a.p.vr[p];
                qv[a.q.cap + gs] = a.p.vt[p];
                qv[2 * a.q.cap + gs] = a.p.vz[p];
            } else
                atomicOr(a.err, (int)ERR_QUEUE_OVERFLOW);
        }
    }
    // flush: row mode walks the rows (the padding is skipped), linear mode
    // the slots
    const int nrow = w.rows ? w.rows : 1, ncol = w.rows ? g.nr1 : WIN;
    for (int r = 0; r < nrow; ++r) {
        for (int c = tid; c < ncol; c += BLOCK) {
            const int k = r * w.ws + c;   // ws is unused (0 rows) in linear mode
            const int node = w.rows ? (w.ib + r) * g.nr1 + c : w.base + c;
            if (PUSH) {
                const long long v = winJ[w.rows ? k : c];
                if (v) atomic_add_i64(&a.accJ[node], v);
            }
            if (DEPQ) {
                const long long v = winQ[w.rows ? k : c];
                if (v) atomic_add_i64(&a.accQ[node], v);
            }
        }
    }
    if (tid < ST_NSTAT && sstat[tid]) atomicAdd(&a.stats[tid], sstat[tid]);
}

// ---------------------------------------------------------------------------
// Corrector of the direct-implicit update, step n: the new electrostatic
// field E^{n+1} (staged per node from phi^{n+1}) gathered at the predicted
// position x~ gives the half kick h E = (dt/2) a^{n+1}; the position moves by
// dt h E (radially and axially: the frame does not turn), the velocity by
// h E, and the filter becomes (h E + filter) / 2.  A radius corrected below
// zero passes through the axis (radial and azimuthal components reversed).
// Absorption as in the push, the window crossing taken on the correction
// segment; the step's collision candidates are queued here (the velocity
// is final only now).  Four consecutive particle slots per lane; one grid
// for both species, the first nb0 blocks the electrons'.
// ---------------------------------------------------------------------------
template <typename T> __global__ __launch_bounds__(256) void k_correct(PassPair<T> pp)
{
    const int sp = (int)blockIdx.x >= pp.nb0 ? 1 : 0;
    const PassArgs<T> &a = pp.a[sp];
    // four consecutive particles per lane (16-byte vector loads and stores;
    // capacities are whole chunks, so the four slots exist)
    const int64_t b0 = 4 * ((int64_t)blockIdx.x - (sp ? pp.nb0 : 0)) * blockDim.x;
    const int64_t p0 = b0 + 4 * (int64_t)threadIdx.x;
    const int64_t n = *a.count;
    if (b0 >= n) return;   // the whole block past the live slots
    using F4 = typename Field4<T>::type;
    const GridC g = a.g;
    // every lane reaches the block-aggregated counts at the end
    bool absd[4] = {false, false, false, false}, cand[4] = {false, false, false, false};
    T vr[4], vt[4], vz[4];
    if (p0 < n) {
        int32_t cell[4], nxt[4];
        T dr[4], dz[4], fr[4], ft[4], fz[4];
        ld4(a.p.cell + p0, cell);
        ld4(a.p.dr + p0, dr);
        ld4(a.p.dz + p0, dz);
        ld4(a.p.vr + p0, vr);
        ld4(a.p.vt + p0, vt);
        ld4(a.p.vz + p0, vz);
        ld4(a.p.fr + p0, fr);
        ld4(a.p.ft + p0, ft);
        ld4(a.p.fz + p0, fz);
        ld4(a.p.next + p0, nxt);
        // field nodes one particle ahead, as in the pass (the next particle's
        // node loads are in flight while this one is corrected)
        F4 n00, n01, n10, n11;
        auto gather_nodes = [&](int k) {
            int key = 0;   // a dead slot reads node 0 and ignores it
            if (p0 + k < n && cell[k] >= 0) {
                int i, j;
                split_cell(g, cell[k], i, j);
                key = i * g.nr1 + j;
            }
            n00 = a.ef[key];
            n01 = a.ef[key + 1];
            n10 = a.ef[key + g.nr1];
            n11 = a.ef[key + g.nr1 + 1];
        };
        gather_nodes(0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const F4 f00 = n00, f01 = n01, f10 = n10, f11 = n11;
            if (k + 1 < 4) gather_nodes(k + 1);
            if (p0 + k >= n || cell[k] < 0) continue;
            int i, j;
            split_cell(g, cell[k], i, j);
            const T dr0 = dr[k], dz0 = dz[k];
            T w00, w01, w10, w11;
            node_weights<T>(j, dr0, dz0, w00, w01, w10, w11);
            const T er = w00 * f00.x + w01 * f01.x + w10 * f10.x + w11 * f11.x;
            const T ez = w00 * f00.y + w01 * f01.y + w10 * f10.y + w11 * f11.y;
            const T h = sc_val<T>(a.sc.h, a.sc.hf);
            const T kr = h * er, kz = h * ez;
            const T dtr = sc_val<T>(a.sc.dtr, a.sc.dtrf), dtz = sc_val<T>(a.sc.dtz, a.sc.dtzf);
            T rel = (T)j + (dr0 + kr * dtr);
            const T bz = dz0 + kz * dtz;
            vr[k] += kr;
            vz[k] += kz;
            fr[k] = (T)0.5 * (kr + fr[k]);
            ft[k] = (T)0.5 * ft[k];
            fz[k] = (T)0.5 * (kz + fz[k]);
            if (rel < (T)0) {
                rel = -rel;
                vr[k] = -vr[k];
                vt[k] = -vt[k];
                fr[k] = -fr[k];
                ft[k] = -ft[k];
            }
            const T fj = floor(rel);
            int jn = (int)fj;
            T drn = rel - fj;
            if (drn >= (T)1) {
                drn -= (T)1;
                jn += 1;
            }
            const T fzz = floor(bz);
            int in = i + (int)fzz;
            T dzn = bz - fzz;
            if (dzn >= (T)1) {
                dzn -= (T)1;
                in += 1;
            }
            // absorption as one flat predicate and the cell as a plain select
            // (a nested if/else chain here let the compiler store the column
            // index in place of -1 for particles past the outer wall)
            const bool finite = rel == rel && bz == bz;
            const bool absorbed = !finite || in < 0 || in >= g.ip || jn >= g.nr;
            if (finite && in >= g.ip && g.window && kz > (T)0) {
                // crossing of z = zp on the correction segment (FP64)
                const double frac = ((double)g.ip - ((double)i + (double)dz0)) / ((double)kz * a.sc.dtz);
                const double Rs = fabs((double)j + (double)dr0 + frac * (double)kr * a.sc.dtr);
                if (Rs < (double)g.nr) {
                    int js = (int)floor(Rs);
                    js = min(js, g.nr - 1);
                    const double w1 = (Rs * Rs - (double)js * js) / (2.0 * js + 1.0);
                    const int nd = g.ip * g.nr1 + js;
                    atomic_add_i64(&a.accW[nd], to_fixed(1.0 - w1, a.sc.qscale));
                    atomic_add_i64(&a.accW[nd + 1], to_fixed(w1, a.sc.qscale));
                }
            }
            cell[k] = absorbed ? -1 : in * g.nr + jn;
            dr[k] = drn;
            dz[k] = dzn;
            absd[k] = absorbed;
            cand[k] = !absorbed && nxt[k] == a.step;
        }
        st4(a.p.cell + p0, cell);
        st4(a.p.dr + p0, dr);
        st4(a.p.dz + p0, dz);
        st4(a.p.vr + p0, vr);
        st4(a.p.vt + p0, vt);
        st4(a.p.vz + p0, vz);
        st4(a.p.fr + p0, fr);
        st4(a.p.ft + p0, ft);
        st4(a.p.fz + p0, fz);
    }
    // absorbed count and queue slots: one global atomic per block (a counter
    // taken per lane, or per wave and run position, serialises the grid on
    // one address); the lane's candidates take consecutive slots after those
    // of the lanes below it
    __shared__ int s_wq[4];
    __shared__ unsigned s_wa[4];
    __shared__ int s_qbase;
    const int wv = (int)threadIdx.x >> 6;
    int before = 0, wtot = 0;
    unsigned atot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t cm = ballot(cand[k]);
        before += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(cm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)cm, 0u));
        wtot += (int)__popcll(cm);
        atot += (unsigned)__popcll(ballot(absd[k]));
    }
    if (lane_id() == 0) {
        s_wq[wv] = wtot;
        s_wa[wv] = atot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        unsigned ab = 0;
        for (int w = 0; w < 4; ++w) {
            const int c = s_wq[w];
            s_wq[w] = tot;
            tot += c;
            ab += s_wa[w];
        }
        s_qbase = tot ? atomicAdd(a.q.count, tot) : 0;
        if (ab) atomicAdd(&a.stats[ST_ABS0 + a.sc.s], (unsigned long long)ab);
    }
    __syncthreads();
    int gs = s_qbase + s_wq[wv] + before;
    T *qv = static_cast<T *>(a.q.vel);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!cand[k]) continue;
        if (gs < a.q.cap) {
            a.q.idx[gs] = (int32_t)(p0 + k);
            qv[gs] = vr[k];
            qv[a.q.cap + gs] = vt[k];
            qv[2 * a.q.cap + gs] = vz[k];
        } else {
            atomicOr(a.err, (int)ERR_QUEUE_OVERFLOW);
        }
        ++gs;
    }
}

// ---------------------------------------------------------------------------
// Collisions of the queued candidates of step `step` (velocity at x^{n+1}
// after the push); births recorded for the ionizations.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_collide(PassArgs<T> a)
{
    __shared__ unsigned long long sstat[ST_NSTAT];
    const int s = a.sc.s;
    const int nq = min(*a.q.count, a.q.cap);
    if ((int64_t)blockIdx.x * blockDim.x >= nq) return;
    if (threadIdx.x < ST_NSTAT) sstat[threadIdx.x] = 0;
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = t < nq;
    int64_t p = act ? a.q.idx[t] : 0;
    bool over = false, born = false;
    int ev = -1;
    double ve[3], vi[3];
    int32_t nb[2];
    T vr = 0, vt = 0, vz = 0;
    int32_t next = 0;
    if (act) {
        const T *qv = static_cast<const T *>(a.q.vel);
        vr = qv[t];
        vt = qv[a.q.cap + t];
        vz = qv[2 * a.q.cap + t];
        ev = collide<T>(a.mc, s, a.p.id[p], a.step, vr, vt, vz, next, over, born, ve, vi, nb);
        if (ev >= 0) {   // a null collision leaves the velocity as it is
            a.p.vr[p] = vr;
            a.p.vt[p] = vt;
            a.p.vz[p] = vz;
        }
        a.p.next[p] = next;
    }
    count_wave(act, sstat, ST_CAND0 + s);
    count_wave(ev == 0, sstat, (s == 0 ? ST_EV00 : ST_EV10));
    count_wave(ev == 1, sstat, (s == 0 ? ST_EV01 : ST_EV11));
    count_wave(ev == 2, sstat, ST_EV02);
    count_wave(over, sstat, ST_OVER0 + s);
    const uint64_t bm = ballot(born);
    if (bm) {
        const int lead = __ffsll((unsigned long long)bm) - 1;
        int slot0 = 0;
        if (lane_id() == lead) slot0 = atomicAdd(a.b.count, __popcll(bm));
        slot0 = __builtin_amdgcn_readlane(slot0, lead);
        if (born) {
            const int slot = slot0 + __builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
            if (slot < a.b.cap) {
                a.b.parent[slot] = a.p.id[p];
                a.b.cell[slot] = a.p.cell[p];
                a.b.dr[slot] = a.p.dr[p];
                a.b.dz[slot] = a.p.dz[p];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    a.b.ve[3 * slot + c] = (T)ve[c];
                    a.b.vi[3 * slot + c] = (T)vi[c];
                }
                a.b.next[2 * slot] = nb[0];
                a.b.next[2 * slot + 1] = nb[1];
            } else {
                atomicOr(a.err, (int)ERR_BIRTH_OVERFLOW);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < ST_NSTAT && sstat[threadIdx.x]) atomicAdd(&a.stats[threadIdx.x], sstat[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// Births: rank by parent id (ids then follow parent-id order, as in a
// sequential sort), append to both species, deposit their charge.  A parent
// ionizes at most once per step, so the ids are distinct and a birth's rank
// is the number of smaller parent ids, counted against all of them: the ids
// are cut into BIRTH_SLICES slices, each workgroup stages one slice in LDS
// and adds its counts for 256 records to the rank array (every lane reads
// the same LDS words, four ids at a time).
// ---------------------------------------------------------------------------
constexpr int BIRTH_SLICES = 16;
constexpr int BIRTH_STAGE = 4096;   // ids staged at a time (a longer slice loops)

__global__ __launch_bounds__(256) void k_birth_rank(const uint32_t *parent, const int32_t *bcount, int cap,
                                                    int32_t *rank)
{
    __shared__ __attribute__((aligned(16))) uint32_t ids[BIRTH_STAGE];
    const int B = min(*bcount, cap);
    if ((int)blockIdx.x * 256 >= B) return;
    const int len = (B + BIRTH_SLICES - 1) / BIRTH_SLICES;
    const int k0 = (int)blockIdx.y * len, k1 = min(B, k0 + len);
    if (k0 >= k1) return;
    const int t = blockIdx.x * 256 + threadIdx.x;
    const uint32_t mine = t < B ? parent[t] : 0u;
    int cnt = 0;
    for (int c0 = k0; c0 < k1; c0 += BIRTH_STAGE) {
        const int n = min(BIRTH_STAGE, k1 - c0);
        __syncthreads();
        for (int e = threadIdx.x; e < n; e += 256) ids[e] = parent[c0 + e];
        __syncthreads();
        const uint4 *v4 = reinterpret_cast<const uint4 *>(ids);
        const int n4 = n >> 2;
        for (int e = 0; e < n4; ++e) {
            const uint4 v = v4[e];
            cnt += (int)(v.x < mine) + (int)(v.y < mine) + (int)(v.z < mine) + (int)(v.w < mine);
        }
        for (int e = n4 << 2; e < n; ++e) cnt += (int)(ids[e] < mine);
    }
    if (t < B && cnt) atomicAdd(&rank[t], cnt);
}

template <typename T>
__global__ __launch_bounds__(256) void k_births(Births<T> b, Parts<T> pe, Parts<T> pi, const int64_t *count,
                                                const int64_t *next_id, int64_t cap_e, int64_t cap_i,
                                                long long *accQe, long long *accQi, int deposit, double qscale,
                                                GridC g, int32_t *err)
{
    const int B = min(*b.count, b.cap);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B) return;
    const int rank = b.rank[t];
    b.rank[t] = 0;   // zero again for the next step
    const int64_t ne = count[0], ni = count[1];
    if (ne + B > cap_e || ni + B > cap_i) {
        atomicOr(err, (int)ERR_CAPACITY);
        return;
    }
    const int64_t oe = ne + rank, oi = ni + rank;
    const int32_t c = b.cell[t];
    const T dr = b.dr[t], dz = b.dz[t];
    pe.cell[oe] = c;
    pe.dr[oe] = dr;
    pe.dz[oe] = dz;
    pe.vr[oe] = b.ve[3 * t];
    pe.vt[oe] = b.ve[3 * t + 1];
    pe.vz[oe] = b.ve[3 * t + 2];
    pe.id[oe] = (uint32_t)(next_id[0] + rank);
    pe.next[oe] = b.next[2 * t];
    pi.cell[oi] = c;
    pi.dr[oi] = dr;
    pi.dz[oi] = dz;
    pi.vr[oi] = b.vi[3 * t];
    pi.vt[oi] = b.vi[3 * t + 1];
    pi.vz[oi] = b.vi[3 * t + 2];
    pi.id[oi] = (uint32_t)(next_id[1] + rank);
    pi.next[oi] = b.next[2 * t + 1];
    if (pe.fr) {
        pe.fr[oe] = pe.ft[oe] = pe.fz[oe] = (T)0;
        pi.fr[oi] = pi.ft[oi] = pi.fz[oi] = (T)0;
    }
    if (deposit) {
        const int ii = c / g.nr, jj = c - ii * g.nr;
        const T fj = (T)jj;
        const T wr1 = dr * ((T)2 * fj + dr) / ((T)2 * fj + (T)1);
        const T w[4] = {((T)1 - dz) * ((T)1 - wr1), ((T)1 - dz) * wr1, dz * ((T)1 - wr1), dz * wr1};
        const int k0 = ii * g.nr1 + jj;
        const int nd[4] = {k0, k0 + 1, k0 + g.nr1, k0 + g.nr1 + 1};
        for (int q = 0; q < 4; ++q) {
            const long long f = to_fixed((double)w[q], qscale);
            atomic_add_i64(&accQe[nd[q]], f);
            atomic_add_i64(&accQi[nd[q]], f);
        }
    }
}

// ---------------------------------------------------------------------------
// Ion-induced secondary electron emission (constant yield gamma per ion
// absorbed at a metal wall; flux-weighted Maxwellian electron).  Block (ion
// id, n, 4, 0) of the ion stream decides (word 0 below gamma) and draws the
// velocity: normal speed sigma sqrt(-2 ln u1) into the domain, tangential
// sigma sqrt(-2 ln u2) (cos, sin)(2 pi u3); block (id, n, 5, 0) the first
// candidate.  The electrons are appended after the step's ionization births
// in ascending parent-ion id order (k_birth_rank over the queued ids, the
// non-emitters' ids replaced by the largest value) at the position the ion
// had before the move, and their charge is deposited with `deposit`.
// ---------------------------------------------------------------------------
template <typename T> __global__ void k_see_decide(SeeQueue<T> q, uint32_t seed, int32_t step)
{
    const int S = min(q.count[0], q.cap);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S) return;
    const U4 b = philox10(U4{q.parent[t], (uint32_t)step, 4u, 0u}, seed, 1u);
    if ((unsigned long long)b.x < q.thr)
        atomicAdd(&q.count[1], 1);
    else
        q.parent[t] = 0xFFFFFFFFu;
}

template <typename T>
__global__ void k_see_births(SeeQueue<T> q, Parts<T> pe, const int64_t *count, const int64_t *next_id, int64_t cap_e,
                             long long *accQe, int deposit, double qscale, GridC g, int32_t *err, uint32_t seed,
                             int32_t step, double lq_e)
{
    const int S = min(q.count[0], q.cap);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S) return;
    const int rank = q.rank[t];
    q.rank[t] = 0;   // zero again for the next step
    const uint32_t id = q.parent[t];
    if (id == 0xFFFFFFFFu) return;
    const int E = q.count[1];
    if (count[0] + E > cap_e) {
        atomicOr(err, (int)ERR_CAPACITY);
        return;
    }
    const U4 b = philox10(U4{id, (uint32_t)step, 4u, 0u}, seed, 1u);
    const U4 c = philox10(U4{id, (uint32_t)step, 5u, 0u}, seed, 1u);
    const double vn = q.sigma * sqrt(-2.0 * log(unit(b.y)));
    const double rt = q.sigma * sqrt(-2.0 * log(unit(b.z)));
    double sp, cp;
    sincos(2.0 * PI * unit(b.w), &sp, &cp);
    const double t1 = rt * cp, t2 = rt * sp;
    const int wall = q.wall[t];
    double v[3];
    if (wall == 1) {
        v[0] = t1, v[1] = t2, v[2] = vn;
    } else if (wall == 2) {
        v[0] = t1, v[1] = t2, v[2] = -vn;
    } else {
        v[0] = -vn, v[1] = t1, v[2] = t2;
    }
    const int64_t o = count[0] + rank;
    const int32_t cl = q.cell[t];
    const T dr = q.dr[t], dz = q.dz[t];
    pe.cell[o] = cl;
    pe.dr[o] = dr;
    pe.dz[o] = dz;
    pe.vr[o] = (T)v[0];
    pe.vt[o] = (T)v[1];
    pe.vz[o] = (T)v[2];
    pe.id[o] = (uint32_t)(next_id[0] + rank);
    pe.next[o] = next_candidate(step, c.x, lq_e);
    if (pe.fr) pe.fr[o] = pe.ft[o] = pe.fz[o] = (T)0;
    if (deposit) {
        const int ii = cl / g.nr, jj = cl - ii * g.nr;
        const T fj = (T)jj;
        const T wr1 = dr * ((T)2 * fj + dr) / ((T)2 * fj + (T)1);
        const T w[4] = {((T)1 - dz) * ((T)1 - wr1), ((T)1 - dz) * wr1, dz * ((T)1 - wr1), dz * wr1};
        const int k0 = ii * g.nr1 + jj;
        const int nd[4] = {k0, k0 + 1, k0 + g.nr1, k0 + g.nr1 + 1};
        for (int e = 0; e < 4; ++e) atomic_add_i64(&accQe[nd[e]], to_fixed((double)w[e], qscale));
    }
}

__global__ void k_see_commit(int32_t *qcount, int64_t *count, int64_t *next_id, int64_t cap_e,
                             unsigned long long *stats)
{
    const int E = qcount[1];
    if (E > 0 && count[0] + E <= cap_e) {
        count[0] += E;
        next_id[0] += E;
        stats[ST_SEE] += (unsigned long long)E;
    }
    qcount[0] = 0;
    qcount[1] = 0;
}

// Commit of the step's births, and the collision queues emptied for the
// next pass (every push pass is followed by the collisions and this commit).
__global__ void k_births_commit(int32_t *bcount, int32_t cap, int64_t *count, int64_t *next_id,
                                int64_t cap_e, int64_t cap_i, unsigned long long *stats, int32_t *q0, int32_t *q1)
{
    const int B = min(*bcount, cap);
    if (B > 0 && count[0] + B <= cap_e && count[1] + B <= cap_i) {
        count[0] += B;
        count[1] += B;
        next_id[0] += B;
        next_id[1] += B;
        stats[ST_BIRTHS] += (unsigned long long)B;
    }
    *bcount = 0;
    *q0 = 0;
    *q1 = 0;
}

// ---------------------------------------------------------------------------
// Counting sort by cell (absorbed particles dropped).  The arrays are
// nearly sorted (particles move a fraction of a cell per step), so each
// block of SORT_PER particles counts its cells in an LDS window of
// SORT_WIN cells around its first particle and touches the global
// histogram / cursors once per window cell it uses; particles outside the
// window (births appended since the last sort) go to global atomics.  The
// window, [c - 512, c + 1536) around the block's first cell c, holds the
// block's cells and a move of one row (256 cells at 256 radial cells) either
// way.
// ---------------------------------------------------------------------------
constexpr int SORT_PER = 1024;
constexpr int SORT_WIN = 2048;
#ifndef PIC_SORT_GROUPS
#define PIC_SORT_GROUPS 4
#endif
#ifndef PIC_SORT_MIN_LANES
#define PIC_SORT_MIN_LANES 8
#endif
constexpr int SORT_GROUPS = PIC_SORT_GROUPS;        // wave-aggregated cells per wave before own adds
constexpr int SORT_MIN_LANES = PIC_SORT_MIN_LANES;  // smallest group worth a wave aggregation
constexpr int SCAN_BLOCK = 1024;

__device__ __forceinline__ int sort_window_lo(const int32_t *cell, int64_t p0, int64_t n, int ncells)
{
    int c = -1;
    for (int k = 0; k < 64 && c < 0 && p0 + k < n; ++k) {
        const int v = cell[p0 + k];
        if (v >= 0 && v < ncells) c = v;
    }
    return c < 0 ? 0 : max(0, c - SORT_WIN / 4);
}

__global__ __launch_bounds__(256) void k_sort_hist(const int32_t *cell, const int64_t *count, int32_t *hist, int ncells)
{
    __shared__ int bins[SORT_WIN];
    __shared__ int s_lo;
    const int64_t n = *count;
    const int64_t p0 = (int64_t)blockIdx.x * SORT_PER;
    if (p0 >= n) return;
    if (threadIdx.x == 0) s_lo = sort_window_lo(cell, p0, n, ncells);
    for (int k = threadIdx.x; k < SORT_WIN; k += blockDim.x) bins[k] = 0;
    __syncthreads();
    const int lo = s_lo;
    for (int q = 0; q < SORT_PER / 256; ++q) {
        const int64_t p = p0 + q * 256 + threadIdx.x;
        const int32_t c = p < n ? cell[p] : -1;
        const bool live = c >= 0 && c < ncells;
        uint64_t todo = ballot(live);
        for (int it = 0; todo && it < SORT_GROUPS; ++it) {
            const int lead = __ffsll((unsigned long long)todo) - 1;
            const int k = __builtin_amdgcn_readlane(c, lead);
            const uint64_t mm = ballot(live && c == k);
            if (__popcll(mm) < SORT_MIN_LANES) break;
            if (lane_id() == lead) {
                const int b = k - lo;
                if (b >= 0 && b < SORT_WIN)
                    atomicAdd(&bins[b], (int)__popcll(mm));
                else
                    atomicAdd(&hist[k], (int)__popcll(mm));
            }
            todo &= ~mm;
        }
        if (todo >> lane_id() & 1ull) {
            // small groups (particles spread over many cells): own adds
            const int b = c - lo;
            if (b >= 0 && b < SORT_WIN)
                atomicAdd(&bins[b], 1);
            else
                atomicAdd(&hist[c], 1);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < SORT_WIN; k += blockDim.x)
        if (bins[k]) atomicAdd(&hist[lo + k], bins[k]);
}

// exclusive scan of hist in blocks of SCAN_BLOCK cells (block totals to part)
__global__ __launch_bounds__(1024) void k_scan_blocks(const int32_t *hist, int ncells, int32_t *cursor, int64_t *part)
{
    __shared__ int64_t v[SCAN_BLOCK];
    const int i = blockIdx.x * SCAN_BLOCK + threadIdx.x;
    const int64_t h = i < ncells ? hist[i] : 0;
    v[threadIdx.x] = h;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        const int64_t a = threadIdx.x >= off ? v[threadIdx.x - off] : 0;
        __syncthreads();
        v[threadIdx.x] += a;
        __syncthreads();
    }
    if (i < ncells) cursor[i] = (int32_t)(v[threadIdx.x] - h);
    if (threadIdx.x == SCAN_BLOCK - 1) part[blockIdx.x] = v[threadIdx.x];
}

// single block: exclusive scan of the block totals; count_old <- count,
// count <- live total
__global__ __launch_bounds__(1024) void k_scan_top(int64_t *part, int nblocks, int64_t *count, int64_t *count_old)
{
    __shared__ int64_t v[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    for (int b0 = 0; b0 < nblocks; b0 += 1024) {
        __syncthreads();
        const int b = b0 + threadIdx.x;
        const int64_t h = b < nblocks ? part[b] : 0;
        v[threadIdx.x] = h;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int64_t a = threadIdx.x >= off ? v[threadIdx.x - off] : 0;
            __syncthreads();
            v[threadIdx.x] += a;
            __syncthreads();
        }
        if (b < nblocks) part[b] = carry + v[threadIdx.x] - h;
        __syncthreads();
        if (threadIdx.x == 1023) carry += v[1023];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        *count_old = *count;
        *count = carry;
    }
}

// cursor += block offset; histogram cleared for the next sort
__global__ void k_scan_add(int32_t *cursor, int32_t *hist, int ncells, const int64_t *part)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncells) return;
    cursor[i] += (int32_t)part[i / SCAN_BLOCK];
    hist[i] = 0;
}

// Scatter of one block of SORT_PER particles.  The in-window particles are
// staged in LDS in destination order (block-local scan of the window cells'
// counts), so that consecutive lanes write consecutive slots of each cell's
// reserved range and the stores fill whole lines: written in source order,
// electrons that changed cell since the last sort left short runs in several
// cells per store, and the scatter wrote 2.3x the bytes it moved.
template <typename T>
__global__ __launch_bounds__(256) void k_sort_scatter(Parts<T> src, Parts<T> dst, const int64_t *count_old,
                                                      int32_t *cursor, int ncells)
{
    __shared__ int bins[SORT_WIN];
    __shared__ int s_lo, s_wt[BLOCK / 64];
    __shared__ int32_t sg_cell[SORT_PER], sg_next[SORT_PER];
    __shared__ uint32_t sg_id[SORT_PER];
    __shared__ int32_t sg_src[SORT_PER];   // source slot (for the direct-implicit filter arrays)
    __shared__ T sg_dr[SORT_PER], sg_dz[SORT_PER], sg_vr[SORT_PER], sg_vt[SORT_PER], sg_vz[SORT_PER];
    constexpr int Q = SORT_PER / 256;
    constexpr int BPT = SORT_WIN / 256;   // window cells per thread in the scan
    const int64_t n = *count_old;
    const int64_t p0 = (int64_t)blockIdx.x * SORT_PER;
    if (p0 >= n) return;
    const int tid = threadIdx.x, lane = lane_id();
    if (tid == 0) s_lo = sort_window_lo(src.cell, p0, n, ncells);
    for (int k = tid; k < SORT_WIN; k += blockDim.x) bins[k] = 0;
    int32_t c[Q], nx[Q];
    uint32_t id[Q];
    T dr[Q], dz[Q], vr[Q], vt[Q], vz[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t p = p0 + q * 256 + tid;
        const bool in = p < n;
        c[q] = in ? src.cell[p] : -1;
        dr[q] = in ? src.dr[p] : (T)0;
        dz[q] = in ? src.dz[p] : (T)0;
        vr[q] = in ? src.vr[p] : (T)0;
        vt[q] = in ? src.vt[p] : (T)0;
        vz[q] = in ? src.vz[p] : (T)0;
        id[q] = in ? src.id[p] : 0u;
        nx[q] = in ? src.next[p] : 0;
    }
    __syncthreads();
    const int lo = s_lo;
    int pos[Q];
    bool inwin[Q];
    // 1. offsets inside the block (window cells) or global positions (others)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const bool live = c[q] >= 0 && c[q] < ncells;
        pos[q] = -1;
        inwin[q] = live && c[q] - lo >= 0 && c[q] - lo < SORT_WIN;
        uint64_t todo = ballot(live);
        for (int it = 0; todo && it < SORT_GROUPS; ++it) {
            const int lead = __ffsll((unsigned long long)todo) - 1;
            const int k = __builtin_amdgcn_readlane(c[q], lead);
            const uint64_t mm = ballot(live && c[q] == k);
            if (__popcll(mm) < SORT_MIN_LANES) break;
            int b0 = 0;
            if (lane == lead) {
                const int b = k - lo;
                if (b >= 0 && b < SORT_WIN)
                    b0 = atomicAdd(&bins[b], (int)__popcll(mm));
                else
                    b0 = atomicAdd(&cursor[k], (int)__popcll(mm));
            }
            b0 = __builtin_amdgcn_readlane(b0, lead);
            if (live && c[q] == k)
                pos[q] = b0 + __builtin_amdgcn_mbcnt_hi((uint32_t)(mm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mm, 0u));
            todo &= ~mm;
        }
        if (todo >> lane & 1ull) {
            // small groups: own reservation (offset in the window cell's
            // block-local count, or a global position outside the window)
            const int b = c[q] - lo;
            pos[q] = (b >= 0 && b < SORT_WIN) ? atomicAdd(&bins[b], 1) : atomicAdd(&cursor[c[q]], 1);
        }
    }
    __syncthreads();
    // 2. block-local exclusive scan of the window counts: bins = start
    int cnt[BPT], start[BPT];
    int sum = 0;
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        cnt[i] = bins[tid * BPT + i];
        start[i] = sum;
        sum += cnt[i];
    }
    int pre = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(pre, off);
        if (lane >= off) pre += v;
    }
    if (lane == 63) s_wt[tid >> 6] = pre;
    __syncthreads();
    int excl = pre - sum;
    for (int w = 0; w < (tid >> 6); ++w) excl += s_wt[w];
    int nin = 0;
    for (int w = 0; w < BLOCK / 64; ++w) nin += s_wt[w];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        start[i] += excl;
        bins[tid * BPT + i] = start[i];
    }
    __syncthreads();
    // 3. stage the in-window particles in destination order; the others go
    // to their global positions now
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (pos[q] < 0) continue;
        if (inwin[q]) {
            const int L = bins[c[q] - lo] + pos[q];
            sg_cell[L] = c[q];
            sg_dr[L] = dr[q];
            sg_dz[L] = dz[q];
            sg_vr[L] = vr[q];
            sg_vt[L] = vt[q];
            sg_vz[L] = vz[q];
            sg_id[L] = id[q];
            sg_next[L] = nx[q];
            sg_src[L] = q * 256 + tid;
        } else {
            const int64_t o = pos[q];
            dst.cell[o] = c[q];
            dst.dr[o] = dr[q];
            dst.dz[o] = dz[q];
            dst.vr[o] = vr[q];
            dst.vt[o] = vt[q];
            dst.vz[o] = vz[q];
            dst.id[o] = id[q];
            dst.next[o] = nx[q];
            if (src.fr) {
                const int64_t sp = p0 + q * 256 + tid;
                dst.fr[o] = src.fr[sp];
                dst.ft[o] = src.ft[sp];
                dst.fz[o] = src.fz[sp];
            }
        }
    }
    __syncthreads();
    // 4. one global reservation per window cell the block uses: bins = the
    // cell's global base minus its local start
#pragma unroll
    for (int i = 0; i < BPT; ++i)
        if (cnt[i]) bins[tid * BPT + i] = atomicAdd(&cursor[lo + tid * BPT + i], cnt[i]) - start[i];
    __syncthreads();
    // 5. move in destination order
    for (int k = tid; k < nin; k += BLOCK) {
        const int32_t cc = sg_cell[k];
        const int64_t o = (int64_t)bins[cc - lo] + k;
        dst.cell[o] = cc;
        dst.dr[o] = sg_dr[k];
        dst.dz[o] = sg_dz[k];
        dst.vr[o] = sg_vr[k];
        dst.vt[o] = sg_vt[k];
        dst.vz[o] = sg_vz[k];
        dst.id[o] = sg_id[k];
        dst.next[o] = sg_next[k];
        if (src.fr) {
            const int64_t sp = p0 + sg_src[k];
            dst.fr[o] = src.fr[sp];
            dst.ft[o] = src.ft[sp];
            dst.fz[o] = src.fz[sp];
        }
    }
}

// live-index prefix for the getters: index[k] = number of live slots < k
__global__ __launch_bounds__(1024) void k_live_index(const int32_t *cell, const int64_t *count, int64_t *index,
                                                     int64_t *nlive)
{
    __shared__ int64_t part[1024];
    const int64_t n = *count;
    const int t = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t lo = min((int64_t)t * per, n), hi = min(lo + per, n);
    int64_t sum = 0;
    for (int64_t k = lo; k < hi; ++k) sum += cell[k] >= 0;
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - sum;
    for (int64_t k = lo; k < hi; ++k) {
        index[k] = run;
        run += cell[k] >= 0;
    }
    if (t == 1023) *nlive = part[1023];
}

// number of live slots (cell >= 0) among the first *count
__global__ __launch_bounds__(256) void k_count_live(const int32_t *cell, const int64_t *count, unsigned long long *out)
{
    __shared__ unsigned long long red[256];
    const int64_t n = *count;
    unsigned long long c = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        c += cell[k] >= 0;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0]) atomicAdd(out, red[0]);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_count_live(const int32_t *cell, const int64_t *count, unsigned long long *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_count_live, dim3(1024), dim3(256), 0, st, cell, count, out);
}

template <typename T>
void launch_load(const Parts<T> &p, int64_t n, uint32_t seed, int s, double rmax, double zp, double vth, double lq,
                 const GridC &g, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_load<T>, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, seed, s, rmax, zp, vth, lq, g);
}

template <typename T>
void launch_place(const Parts<T> &p, int64_t n, const double *R, const double *z, const double *vr,
                  const double *vt, const double *vz, const uint32_t *id, const int32_t *next, const GridC &g,
                  hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_place<T>, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, R, z, vr, vt, vz, id, next, g);
}

template <typename T>
void launch_unplace(const Parts<T> &p, const int64_t *count, int64_t cap, const int64_t *index, double *R, double *z,
                    double *vr, double *vt, double *vz, uint32_t *id, int32_t *next, const GridC &g, hipStream_t st)
{
    hipLaunchKernelGGL(k_unplace<T>, dim3(blocks_for(cap, 256)), dim3(256), 0, st, p, count, index, R, z, vr, vt, vz,
                       id, next, g);
}

void launch_live_index(const int32_t *cell, const int64_t *count, int64_t *index, int64_t *nlive, hipStream_t st)
{
    hipLaunchKernelGGL(k_live_index, dim3(1), dim3(1024), 0, st, cell, count, index, nlive);
}

template <typename T>
void launch_pass(const PassArgs<T> &e, const PassArgs<T> &i, int64_t cap_e, int64_t cap_i, bool push, bool depq,
                 hipStream_t st)
{
    PassPair<T> pp;
    pp.a[0] = e;
    pp.a[1] = i;
    pp.nb0 = blocks_for(cap_e, PassShape<T>::chunk);
    const dim3 grid(pp.nb0 + blocks_for(cap_i, PassShape<T>::chunk)), blk(BLOCK);
    const bool rfb = e.eb != nullptr, di = e.p.fr != nullptr;
    if (push && depq && di)
        hipLaunchKernelGGL((k_pass<T, true, true, false, true>), grid, blk, 0, st, pp);
    else if (push && di)
        hipLaunchKernelGGL((k_pass<T, true, false, false, true>), grid, blk, 0, st, pp);
    else if (push && depq && rfb)
        hipLaunchKernelGGL((k_pass<T, true, true, true, false>), grid, blk, 0, st, pp);
    else if (push && depq)
        hipLaunchKernelGGL((k_pass<T, true, true, false, false>), grid, blk, 0, st, pp);
    else if (push && rfb)
        hipLaunchKernelGGL((k_pass<T, true, false, true, false>), grid, blk, 0, st, pp);
    else if (push)
        hipLaunchKernelGGL((k_pass<T, true, false, false, false>), grid, blk, 0, st, pp);
    else if (depq)
        hipLaunchKernelGGL((k_pass<T, false, true, false, false>), grid, blk, 0, st, pp);
}

template <typename T>
void launch_correct(const PassArgs<T> &e, const PassArgs<T> &i, int64_t cap_e, int64_t cap_i, hipStream_t st)
{
    PassPair<T> pp;
    pp.a[0] = e;
    pp.a[1] = i;
    // four particles per lane (the arrays are padded to whole pass chunks,
    // so the last lane's four slots exist)
    pp.nb0 = blocks_for((cap_e + 3) / 4, 256);
    hipLaunchKernelGGL(k_correct<T>, dim3(pp.nb0 + blocks_for((cap_i + 3) / 4, 256)), dim3(256), 0, st, pp);
}

template <typename T> void launch_collide(const PassArgs<T> &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_collide<T>, dim3(blocks_for(a.q.cap, 256)), dim3(256), 0, st, a);
}

template <typename T>
void launch_births(const Births<T> &b, const Parts<T> &pe, const Parts<T> &pi, int64_t *count, int64_t *next_id,
                   int64_t cap_e, int64_t cap_i, long long *accQe, long long *accQi, bool deposit, double qscale,
                   const GridC &g, int32_t *err, unsigned long long *stats, int32_t *q0, int32_t *q1, hipStream_t st)
{
    hipLaunchKernelGGL(k_birth_rank, dim3(blocks_for(b.cap, 256), BIRTH_SLICES), dim3(256), 0, st, b.parent, b.count,
                       b.cap, b.rank);
    hipLaunchKernelGGL(k_births<T>, dim3(blocks_for(b.cap, 256)), dim3(256), 0, st, b, pe, pi, count, next_id, cap_e,
                       cap_i, accQe, accQi, deposit ? 1 : 0, qscale, g, err);
    hipLaunchKernelGGL(k_births_commit, dim3(1), dim3(1), 0, st, b.count, b.cap, count, next_id, cap_e, cap_i, stats,
                       q0, q1);
}

template <typename T>
void launch_see(const SeeQueue<T> &q, const Parts<T> &pe, int64_t *count, int64_t *next_id, int64_t cap_e,
                long long *accQe, bool deposit, double qscale, const GridC &g, int32_t *err, unsigned long long *stats,
                uint32_t seed, int32_t step, double lq_e, hipStream_t st)
{
    const unsigned nb = blocks_for(q.cap, 256);
    hipLaunchKernelGGL(k_see_decide<T>, dim3(nb), dim3(256), 0, st, q, seed, step);
    hipLaunchKernelGGL(k_birth_rank, dim3(nb, BIRTH_SLICES), dim3(256), 0, st, q.parent, q.count, q.cap, q.rank);
    hipLaunchKernelGGL(k_see_births<T>, dim3(nb), dim3(256), 0, st, q, pe, count, next_id, cap_e, accQe,
                       deposit ? 1 : 0, qscale, g, err, seed, step, lq_e);
    hipLaunchKernelGGL(k_see_commit, dim3(1), dim3(1), 0, st, q.count, count, next_id, cap_e, stats);
}

template <typename T>
void launch_sort(const Parts<T> &src, const Parts<T> &dst, int64_t *count, int64_t *count_old, int32_t *hist,
                 int32_t *cursor, int64_t *scanpart, int ncells, int64_t cap, hipStream_t st)
{
    const unsigned nb = blocks_for(cap, SORT_PER), ns = blocks_for(ncells, SCAN_BLOCK);
    hipLaunchKernelGGL(k_sort_hist, dim3(nb), dim3(256), 0, st, src.cell, count, hist, ncells);
    hipLaunchKernelGGL(k_scan_blocks, dim3(ns), dim3(SCAN_BLOCK), 0, st, hist, ncells, cursor, scanpart);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, scanpart, (int)ns, count, count_old);
    hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(ncells, 256)), dim3(256), 0, st, cursor, hist, ncells, scanpart);
    hipLaunchKernelGGL(k_sort_scatter<T>, dim3(nb), dim3(256), 0, st, src, dst, count_old, cursor, ncells);
}
int sort_scan_blocks(int ncells) { return (int)blocks_for(ncells, SCAN_BLOCK); }

#define PIC_INSTANTIATE(T)                                                                                          \
    template void launch_load<T>(const Parts<T> &, int64_t, uint32_t, int, double, double, double, double,          \
                                 const GridC &, hipStream_t);                                                       \
    template void launch_place<T>(const Parts<T> &, int64_t, const double *, const double *, const double *,        \
                                  const double *, const double *, const uint32_t *, const int32_t *, const GridC &, \
                                  hipStream_t);                                                                     \
    template void launch_unplace<T>(const Parts<T> &, const int64_t *, int64_t, const int64_t *, double *,          \
                                    double *, double *, double *, double *, uint32_t *, int32_t *, const GridC &,   \
                                    hipStream_t);                                                                   \
    template void launch_pass<T>(const PassArgs<T> &, const PassArgs<T> &, int64_t, int64_t, bool, bool,          \
                                 hipStream_t);                                                                      \
    template void launch_collide<T>(const PassArgs<T> &, hipStream_t);                                              \
    template void launch_correct<T>(const PassArgs<T> &, const PassArgs<T> &, int64_t, int64_t, hipStream_t);       \
    template void launch_births<T>(const Births<T> &, const Parts<T> &, const Parts<T> &, int64_t *, int64_t *,     \
                                   int64_t, int64_t, long long *, long long *, bool, double, const GridC &,         \
                                   int32_t *, unsigned long long *, int32_t *, int32_t *, hipStream_t);             \
    template void launch_sort<T>(const Parts<T> &, const Parts<T> &, int64_t *, int64_t *, int32_t *, int32_t *,    \
                                 int64_t *, int, int64_t, hipStream_t);                                             \
    template void launch_see<T>(const SeeQueue<T> &, const Parts<T> &, int64_t *, int64_t *, int64_t, long long *,   \
                                bool, double, const GridC &, int32_t *, unsigned long long *, uint32_t, int32_t,     \
                                double, hipStream_t);

PIC_INSTANTIATE(float)
PIC_INSTANTIATE(double)

}  // namespace pic

namespace pic {

// ---------------------------------------------------------------------------
// Plasma moments of the current particle state (once per closed period):
// per-block FP64 sums over live electrons (count, kinetic energy, R, z) and
// ions (count, kinetic energy), then one workgroup folds them in block
// order, adds the electron node-density maximum from this step's charge
// accumulator and the period's ionizations (real particles).
// ---------------------------------------------------------------------------
constexpr int MOM_BLOCKS = 512;

template <typename T>
__global__ __launch_bounds__(256) void k_moments(Parts<T> pe, Parts<T> pi, const int64_t *count, double me, double mi,
                                                 double inv_qe, GridC g, double *partial)
{
    __shared__ double red[MOM_SUMS][256];
    double s[MOM_SUMS] = {0, 0, 0, 0, 0, 0};
    for (int sp = 0; sp < 2; ++sp) {
        const Parts<T> &p = sp ? pi : pe;
        const int64_t n = count[sp];
        const double hm = 0.5 * (sp ? mi : me) * inv_qe;
        for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
            const int c = p.cell[k];
            if (c < 0) continue;
            const double vr = p.vr[k], vt = p.vt[k], vz = p.vz[k];
            const double e = hm * (vr * vr + vt * vt + vz * vz);
            if (sp == 0) {
                int i, j;
                split_cell(g, c, i, j);
                s[0] += 1.0;
                s[1] += e;
                s[2] += (j + (double)p.dr[k]) * g.dr;
                s[3] += (i + (double)p.dz[k]) * g.dz;
            } else {
                s[4] += 1.0;
                s[5] += e;
            }
        }
    }
    for (int q = 0; q < MOM_SUMS; ++q) red[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int q = 0; q < MOM_SUMS; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x < MOM_SUMS) partial[blockIdx.x * MOM_SUMS + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_moments_fold(const double *partial, int np, const long long *accQe,
                                                      double qscale, double we, double wi, CircuitDev *cd,
                                                      const unsigned long long *stats, GridC g)
{
    __shared__ double red[256];
    __shared__ double sums[MOM_SUMS];
    if (threadIdx.x < MOM_SUMS) {
        double a = 0.0;
        for (int b = 0; b < np; ++b) a += partial[b * MOM_SUMS + threadIdx.x];
        sums[threadIdx.x] = a;
    }
    // electron node density maximum: |accQ_e| / qscale * w_e / V_node
    double m = 0.0;
    for (int n = threadIdx.x; n < g.nodes; n += blockDim.x) {
        const int i = n / g.nr1, j = n - i * g.nr1;
        m = fmax(m, fabs((double)accQe[n]) / qscale * we / node_volume(g, i, j));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    CircuitDev &c = *cd;
    const double vol = 3.141592653589793 * (g.nr * g.dr) * (g.nr * g.dr) * (g.ip * g.dz);
    const double ne = sums[0], ni = sums[4];
    c.moments[0] = ne * we / vol;
    c.moments[1] = ni * wi / vol;
    c.moments[2] = red[0];
    c.moments[3] = ne > 0 ? sums[1] / ne : 0.0;
    c.moments[4] = ni > 0 ? sums[5] / ni : 0.0;
    c.moments[5] = ne > 0 ? sums[2] / ne : 0.0;
    c.moments[6] = ne > 0 ? sums[3] / ne : 0.0;
    const double births = (double)stats[ST_BIRTHS];
    // ionizations of the period in real particles (births times the
    // electron weight): independent of how many macro-particles carry them
    c.moments[7] = (births - c.births_prev) * we;
    c.births_prev = births;
}

int moments_blocks() { return MOM_BLOCKS; }

template <typename T>
void launch_moments(const Parts<T> &pe, const Parts<T> &pi, const int64_t *count, const long long *accQe,
                    double qscale, double we, double wi, double me, double mi, double qe, double *partial, int np,
                    CircuitDev *cd, const unsigned long long *stats, const GridC &g, hipStream_t st)
{
    hipLaunchKernelGGL(k_moments<T>, dim3(np), dim3(256), 0, st, pe, pi, count, me, mi, 1.0 / qe, g, partial);
    hipLaunchKernelGGL(k_moments_fold, dim3(1), dim3(256), 0, st, partial, np, accQe, qscale, we, wi, cd, stats, g);
}
template void launch_moments<float>(const Parts<float> &, const Parts<float> &, const int64_t *, const long long *,
                                    double, double, double, double, double, double, double *, int, CircuitDev *,
                                    const unsigned long long *, const GridC &, hipStream_t);
template void launch_moments<double>(const Parts<double> &, const Parts<double> &, const int64_t *,
                                     const long long *, double, double, double, double, double, double, double *, int,
                                     CircuitDev *, const unsigned long long *, const GridC &, hipStream_t);

}  // namespace pic
