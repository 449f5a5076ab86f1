// Host side of the phasorpic C ABI: configuration checks, workspace
// carving, null-collision constants, the multigrid hierarchy of the
// finite-volume RZ Poisson operator, and the per-call kernel orchestration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/phasorpic.h"
#include "kernels.h"
#include "launch.h"
#include "separable.h"

using namespace pic;

namespace {

constexpr double TWO_PI = 6.283185307179586476925287;

// Bump allocator over the caller's workspace (dry run when base == nullptr).
struct Carver {
    uint8_t *base;
    size_t off = 0;
    template <typename U> U *take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        U *p = base ? reinterpret_cast<U *>(base + off) : nullptr;
        off += count * sizeof(U);
        return p;
    }
};

template <typename T> void carve_parts(Carver &c, Parts<T> &p, int64_t cap, bool implicit)
{
    cap = (cap + PAD - 1) / PAD * PAD;   // the pass reads and writes whole blocks of particles
    p.cell = c.take<int32_t>(cap);
    p.dr = c.take<T>(cap);
    p.dz = c.take<T>(cap);
    p.vr = c.take<T>(cap);
    p.vt = c.take<T>(cap);
    p.vz = c.take<T>(cap);
    p.id = c.take<uint32_t>(cap);
    p.next = c.take<int32_t>(cap);
    p.fr = p.ft = p.fz = nullptr;
    if (implicit) {
        p.fr = c.take<T>(cap);
        p.ft = c.take<T>(cap);
        p.fz = c.take<T>(cap);
    }
}

// queue of the ions absorbed at metal walls in one step (secondary emission)
constexpr int SEE_CAP = 65536;
template <typename T> void carve_see(Carver &c, SeeQueue<T> &q, const pic_config &f)
{
    q = SeeQueue<T>{};
    if (!(f.see_gamma > 0.0)) return;
    q.parent = c.take<uint32_t>(SEE_CAP);
    q.cell = c.take<int32_t>(SEE_CAP);
    q.dr = c.take<T>(SEE_CAP);
    q.dz = c.take<T>(SEE_CAP);
    q.wall = c.take<int32_t>(SEE_CAP);
    q.rank = c.take<int32_t>(SEE_CAP);
    q.count = c.take<int32_t>(2);
    q.cap = SEE_CAP;
    // emit iff word x < thr: (x + 1/2) 2^-32 < gamma <=> x < ceil(gamma 2^32 - 1/2)
    const double y = f.see_gamma * 4294967296.0 - 0.5;
    q.thr = y <= 0.0 ? 0ull : (unsigned long long)std::ceil(y);
    q.sigma = std::sqrt(f.see_temp_ev * f.qe / f.m[0]);
}

template <typename T> void carve_births(Carver &c, Births<T> &b, int cap)
{
    b.parent = c.take<uint32_t>(cap);
    b.rank = c.take<int32_t>(cap);
    b.cell = c.take<int32_t>(cap);
    b.dr = c.take<T>(cap);
    b.dz = c.take<T>(cap);
    b.ve = c.take<T>(3 * (size_t)cap);
    b.vi = c.take<T>(3 * (size_t)cap);
    b.next = c.take<int32_t>(2 * (size_t)cap);
    b.count = c.take<int32_t>(1);
    b.cap = cap;
}

struct HostLevel {
    int nr, nz;
    std::vector<double> eps;   // nz * nr
    std::vector<uint8_t> dir;  // nodes
};

// largest level solved by its dense inverse (nodes)
#ifndef PIC_BOTTOM_NODES
#define PIC_BOTTOM_NODES 2200
#endif
constexpr int BOTTOM_NODES = PIC_BOTTOM_NODES;

int64_t ceil_log2(double x)
{
    int64_t k = 0;
    while (std::ldexp(1.0, (int)k) < x) ++k;
    return k;
}

}  // namespace

struct pic_ctx {
    pic_config cfg{};
    std::vector<double> eps_cell, ec, es, vc, vs;
    std::vector<int32_t> tag;
    hipStream_t stream = nullptr;
    GridC g{};
    bool mixed = false;
    int nrf = 0;
    bool closed = false;
    std::string err;
    int64_t last_push = -1;
    int64_t last_harm = -1;
    int64_t last_mcc = -1;
    int64_t last_dep = 0;
    bool pushed_since_sort = false;

    // particles (ping-pong per species)
    Parts<float> pf[2][2];
    Parts<double> pd[2][2];
    int cur[2] = {0, 0};
    Births<float> bf{};
    SeeQueue<float> sqf{};       // ions at metal walls of the step (secondary emission; cap 0: off)
    SeeQueue<double> sqd{};
    Births<double> bd{};
    CandQueue cq[2]{};
    int64_t *ctl = nullptr;      // count[2], count_old[2], next_id[2], nlive, pad
    unsigned long long *stats = nullptr;
    int32_t *errw = nullptr;
    int32_t *hist = nullptr, *cursor = nullptr;
    int64_t *scanpart = nullptr;   // block totals of the sort's scan
    int64_t *live_index = nullptr;
    double *stage = nullptr;     // 5 doubles + id + next per staged particle
    int64_t stage_cap = 0;

    // grids
    void *ef = nullptr;
    void *eb = nullptr;           // staged RF magnetic field (B_r, B_z) per node, when the config asks for it
    long long *accJ = nullptr, *accQ = nullptr;
    double *accS = nullptr;       // window surface charge per species (weights, FP64, persistent)
    long long *accW = nullptr;    // the step's window charge per species (fixed point, folded into accS)
    double *phi = nullptr, *Q = nullptr, *I = nullptr, *d_ec = nullptr, *d_es = nullptr;
    int32_t *d_tag = nullptr;
    double *dbasis = nullptr;     // manufactured Dirichlet basis, nturns x nodes (or none)
    // direct-implicit update: node susceptibility and the chi = 0 level-0 conductances
    double *chi = nullptr, *cw0 = nullptr, *ce0 = nullptr, *cs0 = nullptr, *cn0 = nullptr;
    double *d_vc = nullptr, *d_vs = nullptr;
    double *Jc = nullptr, *Jcc = nullptr, *Js = nullptr, *Jsc = nullptr, *hpartial = nullptr;
    HarmState *harm = nullptr;

    // multigrid
    MGLevels lv{};
    int lb = 0;
    MGState *mgs = nullptr;
    double *mgpartial = nullptr;
    double *pr = nullptr, *pz = nullptr, *pp = nullptr, *pAp = nullptr;   // CG vectors
    double *pp2 = nullptr;   // second search-direction buffer (alternates with pp)
    double *phi_prev = nullptr;   // phi of the two previous solves (initial-guess extrapolation)
    int run = 0;                  // consecutive solves of the running sequence before this one
    int64_t last_solve = -2;
    // adaptive iteration budget: each solve's state lands in pinned host
    // memory asynchronously; the next solve budgets the recent count + 1
    MGState *mg_host = nullptr;   // pinned ring
    int mg_ring = 0;
    int mg_budget = 8;
    // direct-implicit solves still to run at the full budget: the ring holds
    // counts of solves with chi only after four of them (the solve at the
    // load has chi = 0 and needs far fewer iterations)
    int di_full = 4;
    // a circuit update moves the turn potentials by a whole period's
    // correction: the solves until the start-value extrapolation again spans
    // only solutions after the jump run max_cycles, and the extrapolation
    // restarts from the first of them
    // direct solve of a separable operator (poisson_solver), when it applies
    bool direct = false;
    bool direct_carved = false;   // the workspace holds the plan's arrays
    DirectArgs da{};
    int mg_fresh = 0;             // solves left at max_cycles
    bool mg_restart = false;      // the stored solutions predate the jump
    int32_t *fp = nullptr, *fq = nullptr, *fk = nullptr;
    double *fc = nullptr, *Qk = nullptr;
    int nfaces = 0;

    // field-circuit coupling
    MGLevels hlv{};               // inductive-operator hierarchy (level work arrays shared with lv)
    MGState *hgs = nullptr;
    int32_t *htag = nullptr;      // inductive Dirichlet structure as a tag array: 0 fixed at 0, -1 free
    double *U = nullptr;          // unit-current fields, nturns * nodes
    double *Ep = nullptr;         // plasma-only E_c^p and E_s^sto,p (2 * nodes)
    double *hb = nullptr;         // right-hand side of an inductive solve
    CircuitDev *cd = nullptr;     // device circuit state (also the period finalisation), one per retained order
    CircuitDev cdh{};             // host copy of the fundamental's after the last update
    // retained orders m = 1..M of the multiharmonic circuit (1: the
    // fundamental alone); per-order arrays (cd, harm, U, Ep, d_ec / d_es,
    // d_vc / d_vs, J_c / J_s) hold the orders one after the other
    int M = 1;
    std::vector<double> xp_ord;   // state applied during the completed period, per order (re then im, MAX_X each)
    int32_t *plist = nullptr, *pturn = nullptr;   // turn nodes in node order, their turn index
    double *gval = nullptr;       // s_k / A_k
    int nlist = 0;
    std::vector<double> area;
    int helm_cycles[2]{};
    double helm_rel[2]{};
    // surrogate network (owned by the caller) and its device buffers
    mlp_ctx *net = nullptr;
    float *feat = nullptr, *pred = nullptr;
    double *mompart = nullptr;

    // HIP-event timing: ring of (start, stop) pairs per timed region
    struct Timer {
        static constexpr int RING = 64;
        hipEvent_t ev[RING][2]{};
        int head = 0, pending = 0;
        double ms = 0.0;
        int64_t count = 0;
    };
    bool timing = false;
    Timer t_pass, t_poisson, t_sort, t_circuit;

    // constants
    SpeciesC sc[2]{};
    MccC mc{};
    double qscale = 1.0, jscale = 1.0;
    double numax[2]{}, pnull[2]{}, lq[2]{};
};

static void timer_start(pic_ctx &c, pic_ctx::Timer &t)
{
    if (!c.timing) return;
    auto &e = t.ev[t.head];
    if (!e[0]) {
        (void)hipEventCreate(&e[0]);
        (void)hipEventCreate(&e[1]);
    }
    if (t.pending == pic_ctx::Timer::RING) {   // oldest pair still unread: read it now
        float ms = 0.f;
        (void)hipEventSynchronize(e[1]);
        (void)hipEventElapsedTime(&ms, e[0], e[1]);
        t.ms += ms;
        t.count += 1;
        t.pending -= 1;
    }
    (void)hipEventRecord(e[0], c.stream);
}

static void timer_stop(pic_ctx &c, pic_ctx::Timer &t)
{
    if (!c.timing) return;
    (void)hipEventRecord(t.ev[t.head][1], c.stream);
    t.head = (t.head + 1) % pic_ctx::Timer::RING;
    t.pending += 1;
}

static void timer_drain(pic_ctx::Timer &t)
{
    const int R = pic_ctx::Timer::RING;
    for (int k = t.pending; k > 0; --k) {
        auto &e = t.ev[(t.head - k + R) % R];
        float ms = 0.f;
        (void)hipEventSynchronize(e[1]);
        (void)hipEventElapsedTime(&ms, e[0], e[1]);
        t.ms += ms;
        t.count += 1;
    }
    t.pending = 0;
}

static pic_status fail(pic_ctx *c, pic_status s, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

static hipError_t cpy(hipStream_t st, void *dst, const void *src, size_t bytes, hipMemcpyKind kind)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, st);
    return e != hipSuccess ? e : hipStreamSynchronize(st);
}

static hipError_t mset(hipStream_t st, void *dst, int v, size_t bytes)
{
    hipError_t e = hipMemsetAsync(dst, v, bytes, st);
    return e != hipSuccess ? e : hipStreamSynchronize(st);
}

#define HIPCHK(ctx, expr)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail(ctx, PIC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

// ---------------------------------------------------------------------------
// Geometry: finite-volume conductances of the RZ Poisson operator on a level
// (face areas of the axisymmetric control volumes, face permittivity = mean
// of the cells sharing the face), and the Dirichlet structure.
// ---------------------------------------------------------------------------
struct Coeffs {
    std::vector<double> cw, ce, cs, cn, cc;
};

static Coeffs assemble(int nr, int nz, double dr, double dz, const std::vector<double> &eps, double eps0)
{
    const int nr1 = nr + 1, nodes = (nz + 1) * nr1;
    Coeffs c;
    c.cw.assign(nodes, 0.0);
    c.ce.assign(nodes, 0.0);
    c.cs.assign(nodes, 0.0);
    c.cn.assign(nodes, 0.0);
    c.cc.assign(nodes, 0.0);
    auto cell_eps = [&](int i, int j, double &sum, int &cnt) {
        if (i >= 0 && i < nz && j >= 0 && j < nr) {
            sum += eps[(size_t)i * nr + j];
            ++cnt;
        }
    };
    for (int i = 0; i <= nz; ++i) {
        for (int j = 0; j <= nr; ++j) {
            const int n = i * nr1 + j;
            const double R = j * dr;
            if (j < nr) {   // face between (i, j) and (i, j+1)
                const double h = std::min((double)nz * dz, i * dz + 0.5 * dz) - std::max(0.0, i * dz - 0.5 * dz);
                const double area = TWO_PI * (R + 0.5 * dr) * h;
                double s = 0.0;
                int k = 0;
                cell_eps(i - 1, j, s, k);
                cell_eps(i, j, s, k);
                const double cf = eps0 * (s / k) * area / dr;
                c.ce[n] = cf;
                c.cw[n + 1] = cf;
            }
            if (i < nz) {   // face between (i, j) and (i+1, j)
                const double lo = std::max(0.0, R - 0.5 * dr), hi = std::min((double)nr * dr, R + 0.5 * dr);
                const double area = 0.5 * TWO_PI * (hi * hi - lo * lo);
                double s = 0.0;
                int k = 0;
                cell_eps(i, j - 1, s, k);
                cell_eps(i, j, s, k);
                const double cf = eps0 * (s / k) * area / dz;
                c.cn[n] = cf;
                c.cs[n + nr1] = cf;
            }
        }
    }
    for (int n = 0; n < nodes; ++n) c.cc[n] = c.cw[n] + c.ce[n] + c.cs[n] + c.cn[n];
    return c;
}

// Galerkin coarse operator A_c = P^T A P of a 9-point (or 5-point, as 9-point
// with zero corners) fine operator, P bilinear and zero on fine Dirichlet
// nodes.  Entry k = 3 (di + 1) + (dj + 1) of node n sits at a[k * nodes + n].
// A coarse node none of whose interpolation support is free becomes a
// Dirichlet (fixed-zero) node.
struct Stencil9 {
    int nr, nz;
    std::vector<double> a;
    std::vector<uint8_t> dir;
};

static Stencil9 galerkin(const Stencil9 &F)
{
    Stencil9 C;
    C.nr = F.nr / 2;
    C.nz = F.nz / 2;
    const int nr1f = F.nr + 1, nr1c = C.nr + 1;
    const size_t nf = (size_t)(F.nz + 1) * nr1f, nc = (size_t)(C.nz + 1) * nr1c;
    C.a.assign(9 * nc, 0.0);
    std::vector<uint8_t> support(nc, 0);
    auto interp = [](int i, int *idx, double *w) {
        if (i % 2 == 0) {
            idx[0] = i / 2;
            w[0] = 1.0;
            return 1;
        }
        idx[0] = (i - 1) / 2;
        idx[1] = (i + 1) / 2;
        w[0] = w[1] = 0.5;
        return 2;
    };
    for (int i = 0; i <= F.nz; ++i)
        for (int j = 0; j <= F.nr; ++j) {
            const size_t p = (size_t)i * nr1f + j;
            if (F.dir[p]) continue;
            int Ii[2], Jj[2];
            double wi[2], wj[2];
            const int ni = interp(i, Ii, wi), nj = interp(j, Jj, wj);
            for (int a = 0; a < ni; ++a)
                for (int b = 0; b < nj; ++b) support[(size_t)Ii[a] * nr1c + Jj[b]] = 1;
            for (int k = 0; k < 9; ++k) {
                const int di = k / 3 - 1, dj = k % 3 - 1;
                const int i2 = i + di, j2 = j + dj;
                if (i2 < 0 || i2 > F.nz || j2 < 0 || j2 > F.nr) continue;
                const size_t q = (size_t)i2 * nr1f + j2;
                if (F.dir[q]) continue;
                const double v = F.a[(size_t)k * nf + p];
                if (v == 0.0) continue;
                int I2[2], J2[2];
                double w2i[2], w2j[2];
                const int mi = interp(i2, I2, w2i), mj = interp(j2, J2, w2j);
                for (int a = 0; a < ni; ++a)
                    for (int b = 0; b < nj; ++b)
                        for (int c2 = 0; c2 < mi; ++c2)
                            for (int d2 = 0; d2 < mj; ++d2) {
                                const int oi = I2[c2] - Ii[a], oj = J2[d2] - Jj[b];
                                const size_t row = (size_t)Ii[a] * nr1c + Jj[b];
                                C.a[(size_t)((oi + 1) * 3 + (oj + 1)) * nc + row] += wi[a] * wj[b] * v * w2i[c2] * w2j[d2];
                            }
            }
        }
    C.dir.assign(nc, 0);
    for (size_t n = 0; n < nc; ++n)
        if (!support[n]) {
            C.dir[n] = 1;
            for (int k = 0; k < 9; ++k) C.a[(size_t)k * nc + n] = k == 4 ? 1.0 : 0.0;
        }
    return C;
}

// ---------------------------------------------------------------------------
// Null-collision constants: nu_max = margin * max over the scanned range of
// n_g sigma_T v (electrons: energy 0..e_cap; ions: relative speed 0..g_cap),
// P_null = 1 - exp(-nu_max dt), log(1 - P_null) = -nu_max dt.
// ---------------------------------------------------------------------------
static double host_threshold_shape(double eps, double th)
{
    if (eps <= th) return 0.0;
    const double x = eps / th;
    return 4.0 * (x - 1.0) / (x * x);
}

static void null_constants(const pic_config &c, double numax[2], double pnull[2], double lq[2])
{
    const double *x = c.xs;
    double be = 0.0, bi = 0.0;
    const int N = c.nscan > 0 ? c.nscan : 200000;
    for (int k = 0; k <= N; ++k) {
        const double eps = x[10] * (double)k / (double)N;
        double sel, sex, siz;
        if (c.xs_kind == 1) {
            sel = x[0];
            sex = eps > x[3] ? x[2] : 0.0;
            siz = eps > x[5] ? x[4] : 0.0;
        } else {
            sel = x[0] / std::sqrt(1.0 + eps / x[1]);
            sex = x[2] * host_threshold_shape(eps, x[3]);
            siz = x[4] * host_threshold_shape(eps, x[5]);
        }
        const double v = std::sqrt(2.0 * eps * c.qe / c.m[0]);
        be = std::max(be, c.ngas * (sel + sex + siz) * v);
        const double gr = x[11] * (double)k / (double)N;
        const double ecm = 0.25 * c.m[1] * gr * gr / c.qe;
        double iel, icx;
        if (c.xs_kind == 1) {
            iel = x[6];
            icx = x[8];
        } else {
            iel = x[6] * std::pow(1.0 + ecm, -x[7]);
            icx = x[8] * std::pow(1.0 + ecm, -x[9]);
        }
        bi = std::max(bi, c.ngas * (iel + icx) * gr);
    }
    numax[0] = be * x[12];
    numax[1] = bi * x[12];
    for (int s = 0; s < 2; ++s) {
        pnull[s] = -std::expm1(-numax[s] * c.dt);
        lq[s] = -numax[s] * c.dt;
    }
}

// ---------------------------------------------------------------------------
// Workspace layout (shared by the size query and pic_init)
// ---------------------------------------------------------------------------
static int mg_levels(int nr, int nz)
{
    int n = 1;
    while (nr % 2 == 0 && nz % 2 == 0 && std::min(nr, nz) >= 4 && n < MAX_LEVELS) {
        nr /= 2;
        nz /= 2;
        ++n;
    }
    return n;
}

static_assert(DP_MAX_DIRICHLET == DP_MAX_DIRICHLET_DEV, "interior Dirichlet limit differs between host and device");

// the configuration may take the direct Poisson solve (whether the operator
// separates is decided at pic_init)
static bool direct_candidate(const pic_config &f)
{
    return f.poisson_solver != PIC_POISSON_MULTIGRID && !f.implicit && f.nr >= 2 && f.nz >= 3;
}

// retained orders of the circuit (the fundamental and nharm above it)
static int norders(const pic_config &f) { return 1 + (f.nharm > 0 ? f.nharm : 0); }

static void layout(pic_ctx &c, Carver &cv)
{
    const pic_config &f = c.cfg;
    const int nodes = (f.nz + 1) * (f.nr + 1), ncells = f.nz * f.nr;
    for (int s = 0; s < 2; ++s)
        for (int b = 0; b < 2; ++b) {
            if (c.mixed)
                carve_parts(cv, c.pf[s][b], f.capacity[s], f.implicit != 0);
            else
                carve_parts(cv, c.pd[s][b], f.capacity[s], f.implicit != 0);
        }
    const int bcap = f.birth_capacity > 0 ? f.birth_capacity : 65536;
    if (c.mixed) {
        carve_births(cv, c.bf, bcap);
        carve_see(cv, c.sqf, f);
    } else {
        carve_births(cv, c.bd, bcap);
        carve_see(cv, c.sqd, f);
    }
    for (int s = 0; s < 2; ++s) {
        const double expect = c.pnull[s] * (double)f.capacity[s];
        const int64_t qc = std::min<int64_t>(f.capacity[s], (int64_t)(4.0 * expect + 16.0 * std::sqrt(expect + 1.0)) + 4096);
        c.cq[s].cap = (int32_t)qc;
        c.cq[s].idx = cv.take<int32_t>(qc);
        c.cq[s].vel = cv.take<uint8_t>(3 * (size_t)qc * (c.mixed ? sizeof(float) : sizeof(double)));
        c.cq[s].count = cv.take<int32_t>(1);
    }
    c.ctl = cv.take<int64_t>(8);
    c.stats = cv.take<unsigned long long>(ST_NSTAT);
    c.errw = cv.take<int32_t>(1);
    c.hist = cv.take<int32_t>(ncells + 1);
    c.cursor = cv.take<int32_t>(ncells + 1);
    c.scanpart = cv.take<int64_t>(sort_scan_blocks(ncells) + 1);
    const int64_t capmax = std::max(f.capacity[0], f.capacity[1]);
    c.live_index = cv.take<int64_t>(capmax);
    c.stage_cap = std::min<int64_t>(capmax, 1 << 20);
    c.stage = cv.take<double>(6 * (size_t)c.stage_cap);
    c.ef = c.mixed ? (void *)cv.take<float4>(nodes) : (void *)cv.take<double4>(nodes);
    if (f.rf_bfield) c.eb = c.mixed ? (void *)cv.take<float2>(nodes) : (void *)cv.take<double2>(nodes);
    c.accJ = cv.take<long long>(2 * (size_t)nodes);
    c.accQ = cv.take<long long>(2 * (size_t)nodes);
    c.accS = cv.take<double>(2 * (size_t)nodes);
    c.accW = cv.take<long long>(2 * (size_t)nodes);
    c.phi = cv.take<double>(nodes);
    c.Q = cv.take<double>(nodes);
    c.I = cv.take<double>(nodes);
    const int M = norders(f);
    c.d_ec = cv.take<double>((size_t)M * nodes);
    c.d_es = cv.take<double>((size_t)M * nodes);
    c.d_tag = cv.take<int32_t>(nodes);
    if (f.dir_basis && f.nturns > 0) c.dbasis = cv.take<double>((size_t)f.nturns * nodes);
    if (f.implicit) {
        c.chi = cv.take<double>(nodes);
        c.cw0 = cv.take<double>(nodes);
        c.ce0 = cv.take<double>(nodes);
        c.cs0 = cv.take<double>(nodes);
        c.cn0 = cv.take<double>(nodes);
    }
    c.d_vc = cv.take<double>((size_t)M * MAX_TURNS);
    c.d_vs = cv.take<double>((size_t)M * MAX_TURNS);
    if (direct_candidate(f)) {
        // direct solve of a separable operator (whether it separates is
        // decided at pic_init; the interior Dirichlet nodes size the plan)
        int m, nrow;
        interior_dirichlet(c.tag, f.nr, f.nz, m, nrow);
        if (m <= DP_MAX_DIRICHLET && nrow <= DP_MAX_ROWS && f.nz - 1 <= DP_MAX_NI) {
            const int ni = f.nz - 1, nj = f.nr;
            DirectArgs &d = c.da;
            d.v = cv.take<double>((size_t)nj * nj);
            d.lam = cv.take<double>(nj);
            d.zrow = cv.take<double>(ni);
            d.erow = cv.take<double>(ni + 1);
            d.cinv = cv.take<double>((size_t)m * m);
            d.g = cv.take<double>((size_t)nrow * ni * nj);
            d.dnode = cv.take<int32_t>(m);
            d.drow = cv.take<int32_t>(m);
            d.rows = cv.take<int32_t>(nrow);
            d.rowstart = cv.take<int32_t>(nrow + 1);
            d.res = cv.take<double>(m);
            d.src = cv.take<double>(m);
            d.b = cv.take<double>((size_t)ni * nj);
            d.u = cv.take<double>((size_t)ni * nj);
            d.w = cv.take<double>((size_t)std::max(nrow, 1) * nj);
            c.direct_carved = true;
        }
    }
    c.Jc = cv.take<double>((size_t)M * nodes);
    c.Jcc = cv.take<double>((size_t)M * nodes);
    c.Js = cv.take<double>((size_t)M * nodes);
    c.Jsc = cv.take<double>((size_t)M * nodes);
    c.hpartial = cv.take<double>(harmonic_blocks(nodes));
    c.harm = cv.take<HarmState>(M);
    // multigrid: level 0 holds the CG correction (z) and residual (r); the
    // hierarchy stops at the first level of at most BOTTOM_NODES nodes, which
    // is solved with a dense inverse (inverted in FP64, applied from an FP32 copy)
    int nl = mg_levels(f.nr, f.nz);
    {
        int nr_ = f.nr, nz_ = f.nz, l = 0;
        while (l < nl - 1 && (nz_ + 1) * (nr_ + 1) > BOTTOM_NODES) {
            nr_ /= 2;
            nz_ /= 2;
            ++l;
        }
        nl = l + 1;
    }
    c.lv.n = nl;
    c.lb = nl - 1;
    c.pr = cv.take<double>(nodes);
    c.pz = cv.take<double>(nodes);
    c.pp = cv.take<double>(nodes);
    c.pAp = cv.take<double>(nodes);
    c.pp2 = cv.take<double>(nodes);
    int nr = f.nr, nz = f.nz;
    for (int l = 0; l < nl; ++l) {
        MGLevel &L = c.lv.L[l];
        L.nr = nr;
        L.nz = nz;
        L.nr1 = nr + 1;
        L.nodes = (nz + 1) * (nr + 1);
        L.nine = l > 0;
        L.phi = l == 0 ? c.pz : cv.take<double>(L.nodes);
        L.rhs = l == 0 ? c.pr : cv.take<double>(L.nodes);
        L.res = l < nl - 1 ? cv.take<double>(L.nodes) : nullptr;
        if (l == 0) {
            L.cw = cv.take<double>(L.nodes);
            L.ce = cv.take<double>(L.nodes);
            L.cs = cv.take<double>(L.nodes);
            L.cn = cv.take<double>(L.nodes);
            L.cc = cv.take<double>(L.nodes);
            L.a = nullptr;
        } else {
            L.cw = L.ce = L.cs = L.cn = L.cc = nullptr;
            L.a = cv.take<double>(9 * (size_t)L.nodes);
        }
        L.dir = cv.take<uint8_t>(L.nodes);
        nr /= 2;
        nz /= 2;
    }
    c.phi_prev = cv.take<double>(2 * (size_t)nodes);
    {
        const MGLevel &Lc = c.lv.L[nl - 1];
        c.lv.coarse_inv = cv.take<double>((size_t)Lc.nodes * dense_ld(Lc.nodes));
        c.lv.coarse_inv32 = cv.take<float>((size_t)Lc.nodes * dense_ld32(Lc.nodes));
    }
    c.mgs = cv.take<MGState>(1);
    c.mgpartial = cv.take<double>(pcg_partial_size(c.lv.L[0]));
    // face list upper bound: 4 faces per turn node
    int nturn_nodes = 0;
    if (!c.tag.empty())
        for (int32_t t : c.tag) nturn_nodes += t >= 1;
    const int fmax = 4 * nturn_nodes + 1;
    c.fp = cv.take<int32_t>(fmax);
    c.fq = cv.take<int32_t>(fmax);
    c.fk = cv.take<int32_t>(fmax);
    c.fc = cv.take<double>(fmax);
    c.Qk = cv.take<double>(MAX_TURNS);
    c.cd = cv.take<CircuitDev>(M);
    c.gval = cv.take<double>(MAX_TURNS);
    c.plist = cv.take<int32_t>(nturn_nodes + 1);
    c.pturn = cv.take<int32_t>(nturn_nodes + 1);
    c.feat = cv.take<float>(32);
    c.pred = cv.take<float>(32);
    c.mompart = cv.take<double>((size_t)moments_blocks() * MOM_SUMS);
    if (f.circuit) {
        c.hgs = cv.take<MGState>(1);
        c.htag = cv.take<int32_t>(nodes);
        c.U = cv.take<double>((size_t)M * f.nturns * nodes);
        c.Ep = cv.take<double>(2 * (size_t)M * nodes);
        c.hb = cv.take<double>(nodes);
        c.hlv.n = nl;
        for (int l = 0; l < nl; ++l) {
            const MGLevel &P = c.lv.L[l];
            MGLevel &L = c.hlv.L[l];
            L = P;   // same geometry and work arrays, own operator
            if (l == 0) {
                L.cw = cv.take<double>(L.nodes);
                L.ce = cv.take<double>(L.nodes);
                L.cs = cv.take<double>(L.nodes);
                L.cn = cv.take<double>(L.nodes);
                L.cc = cv.take<double>(L.nodes);
            } else {
                L.a = cv.take<double>(9 * (size_t)L.nodes);
            }
            L.dir = cv.take<uint8_t>(L.nodes);
        }
        const MGLevel &Lc = c.hlv.L[nl - 1];
        c.hlv.coarse_inv = cv.take<double>((size_t)Lc.nodes * dense_ld(Lc.nodes));
        c.hlv.coarse_inv32 = cv.take<float>((size_t)Lc.nodes * dense_ld32(Lc.nodes));
    }
}

static pic_status check_config(const pic_config *f, pic_ctx *c)
{
    if (!f) return fail(c, PIC_EINVAL, "null config");
    if (f->nr < 2 || f->nz < 2) return fail(c, PIC_EINVAL, "grid too small (%d x %d)", f->nr, f->nz);
    if (f->ip < 1 || f->ip > f->nz) return fail(c, PIC_EINVAL, "ip = %d outside 1..nz", f->ip);
    if (!(f->rmax > 0) || !(f->zmax > 0) || !(f->dt > 0) || !(f->freq > 0))
        return fail(c, PIC_EINVAL, "rmax, zmax, dt, freq must be positive");
    if (f->precision != PIC_FP64 && f->precision != PIC_MIXED) return fail(c, PIC_EINVAL, "bad precision");
    for (int s = 0; s < 2; ++s) {
        if (f->capacity[s] < 1 || f->capacity[s] >= (int64_t)1 << 31)
            return fail(c, PIC_EINVAL, "capacity[%d] outside 1 .. 2^31-1", s);
        if (f->load && f->np_init[s] > f->capacity[s]) return fail(c, PIC_ENOMEM, "np_init > capacity");
        if (!(f->m[s] > 0)) return fail(c, PIC_EINVAL, "mass must be positive");
    }
    if (f->nturns < 0 || f->nturns > MAX_TURNS) return fail(c, PIC_EINVAL, "nturns outside 0..%d", MAX_TURNS);
    if (f->nturns > 0 && !f->circuit && (!f->turn_vc || !f->turn_vs))
        return fail(c, PIC_EINVAL, "turn voltages missing");
    if (f->circuit) {
        if (f->nturns < 1) return fail(c, PIC_EINVAL, "circuit coupling needs at least one turn");
        if (!(f->alpha > 0.0 && f->alpha <= 1.0)) return fail(c, PIC_EINVAL, "relaxation alpha outside (0, 1]");
        if (!(f->mu0 > 0.0) || !(f->eps0 > 0.0)) return fail(c, PIC_EINVAL, "mu0, eps0 must be positive");
        if (f->field_mode != PIC_FIELD_FULL && f->field_mode != PIC_FIELD_MQS) return fail(c, PIC_EINVAL, "bad field_mode");
        if (f->rrf_mode == PIC_RRF_GIVEN && !f->r_rf) return fail(c, PIC_EINVAL, "r_rf missing");
        if (f->rrf_mode != PIC_RRF_GIVEN && f->rrf_mode != PIC_RRF_SKIN) return fail(c, PIC_EINVAL, "bad rrf_mode");
        if (!(f->helm_rtol > 0.0) || f->helm_max_cycles < 1 || f->helm_max_cycles > MAX_CG)
            return fail(c, PIC_EINVAL, "helm_rtol > 0 and helm_max_cycles in 1..%d required", MAX_CG);
        if (f->controller && !(f->p_target > 0.0 && f->v_min > 0.0 && f->v_max >= f->v_min && f->f_step >= 0.0))
            return fail(c, PIC_EINVAL, "controller settings invalid");
        if (f->vg_from_target && !(f->p_target > 0.0)) return fail(c, PIC_EINVAL, "p_target must be positive");
    }
    if (!f->eps_cell || !f->node_tag) return fail(c, PIC_EINVAL, "eps_cell and node_tag are required");
    if (f->sort_every < 1) return fail(c, PIC_EINVAL, "sort_every must be >= 1");
    if (f->sort_every_ion < 0) return fail(c, PIC_EINVAL, "sort_every_ion must be >= 0");
    if (f->birth_capacity < 0) return fail(c, PIC_EINVAL, "birth_capacity < 0");
    if (f->implicit && (f->rf_bfield || f->bfield[0] != 0.0 || f->bfield[1] != 0.0 || f->bfield[2] != 0.0))
        return fail(c, PIC_EINVAL, "the direct-implicit update runs without magnetic field");
    if (!(f->see_gamma >= 0.0 && f->see_gamma <= 1.0))
        return fail(c, PIC_EINVAL, "see_gamma must lie in [0, 1]");
    if (f->see_gamma > 0.0) {
        if (!(f->see_temp_ev > 0.0 && std::isfinite(f->see_temp_ev)))
            return fail(c, PIC_EINVAL, "see_temp_ev must be positive");
        if (f->implicit) return fail(c, PIC_EINVAL, "secondary emission runs with the explicit step only");
    }
    if (f->nharm < 0 || f->nharm > MAX_HARM - 1)
        return fail(c, PIC_EINVAL, "nharm outside 0..%d", MAX_HARM - 1);
    if (f->nharm > 0) {
        if (!f->circuit) return fail(c, PIC_EINVAL, "the multiharmonic circuit needs circuit coupling");
        if (f->field_mode != PIC_FIELD_MQS)
            return fail(c, PIC_EINVAL, "the multiharmonic circuit needs the magnetoquasistatic inductive operator");
        if (f->rf_bfield) return fail(c, PIC_EINVAL, "the RF magnetic field is formed from the fundamental only");
        for (int q = 0; q < f->nharm; ++q)
            if (!(f->harm_ratio[q] > 0.0 && std::isfinite(f->harm_ratio[q])) || !std::isfinite(f->harm_phase[q]))
                return fail(c, PIC_EINVAL, "harm_ratio[%d] must be positive and harm_phase[%d] finite", q, q);
    }
    return PIC_OK;
}

static pic_status prepare_host(pic_ctx &c, const pic_config *f)
{
    c.cfg = *f;
    c.mixed = f->precision == PIC_MIXED;
    const int nodes = (f->nz + 1) * (f->nr + 1), ncells = f->nz * f->nr;
    c.eps_cell.assign(f->eps_cell, f->eps_cell + ncells);
    c.tag.assign(f->node_tag, f->node_tag + nodes);
    c.ec.assign(nodes, 0.0);
    c.es.assign(nodes, 0.0);
    if (f->ec) c.ec.assign(f->ec, f->ec + nodes);
    if (f->es_sto) c.es.assign(f->es_sto, f->es_sto + nodes);
    c.M = norders(*f);
    c.vc.assign((size_t)c.M * MAX_TURNS, 0.0);
    c.vs.assign((size_t)c.M * MAX_TURNS, 0.0);
    c.ec.resize((size_t)c.M * nodes, 0.0);
    c.es.resize((size_t)c.M * nodes, 0.0);
    c.xp_ord.assign((size_t)c.M * 2 * MAX_X, 0.0);
    for (int k = 0; k < f->nturns; ++k) {
        c.vc[k] = f->turn_vc ? f->turn_vc[k] : 0.0;
        c.vs[k] = f->turn_vs ? f->turn_vs[k] : 0.0;
    }
    for (int n = 0; n < nodes; ++n)
        if (c.tag[n] > f->nturns || c.tag[n] < -1) return fail(&c, PIC_EINVAL, "node tag %d invalid", c.tag[n]);
    // the particle box must be free of Dirichlet nodes inside (rows 1..ip-1, cols 0..nr-1)
    for (int i = 1; i < f->ip; ++i)
        for (int j = 0; j < f->nr; ++j)
            if (c.tag[i * (f->nr + 1) + j] != -1)
                return fail(&c, PIC_EINVAL, "Dirichlet node (%d, %d) inside the particle region", i, j);
    c.g.nr = f->nr;
    c.g.nz = f->nz;
    c.g.nr1 = f->nr + 1;
    c.g.nodes = nodes;
    c.g.ncells = ncells;
    c.g.ip = f->ip;
    c.g.window = f->window;
    c.g.dr = f->rmax / f->nr;
    c.g.dz = f->zmax / f->nz;
    c.g.inv_nr = 1.0f / (float)f->nr;
    if ((int64_t)f->nr * f->nz >= (1 << 22)) return fail(&c, PIC_EINVAL, "grid too large (nr nz >= 2^22)");
    {
        int nr_ = f->nr, nz_ = f->nz, nl = mg_levels(f->nr, f->nz);
        for (int l = 0; l < nl - 1 && (nz_ + 1) * (nr_ + 1) > BOTTOM_NODES; ++l) {
            nr_ /= 2;
            nz_ /= 2;
        }
        if ((nz_ + 1) * (nr_ + 1) > 4 * BOTTOM_NODES)
            return fail(&c, PIC_EINVAL, "grid %d x %d does not coarsen to a small bottom level (use even, ideally "
                                        "power-of-two cell counts)", f->nr, f->nz);
    }
    null_constants(*f, c.numax, c.pnull, c.lq);
    const double nf = 1.0 / (f->freq * f->dt);
    c.nrf = (int)std::lround(nf);
    c.closed = std::fabs(f->freq * f->dt * c.nrf - 1.0) < 1e-10;
    return PIC_OK;
}

// message of the last failed pic_workspace_bytes / pic_init of this thread
// (pic_last_error(NULL))
static thread_local std::string init_error;

extern "C" pic_status pic_workspace_bytes(const pic_config *cfg, size_t *bytes)
{
    if (!bytes) return PIC_EINVAL;
    pic_ctx c;
    init_error.clear();
    pic_status st = check_config(cfg, &c);
    if (!st) st = prepare_host(c, cfg);
    if (st) {
        init_error = c.err;
        return st;
    }
    Carver cv{nullptr};
    layout(c, cv);
    *bytes = cv.off + 256;
    return PIC_OK;
}

// ---------------------------------------------------------------------------
// Templated orchestration
// ---------------------------------------------------------------------------
template <typename T> static Parts<T> &parts(pic_ctx &c, int s, int b);
template <> Parts<float> &parts<float>(pic_ctx &c, int s, int b) { return c.pf[s][b]; }
template <> Parts<double> &parts<double>(pic_ctx &c, int s, int b) { return c.pd[s][b]; }
template <typename T> static Births<T> &births(pic_ctx &c);
template <> Births<float> &births<float>(pic_ctx &c) { return c.bf; }
template <> Births<double> &births<double>(pic_ctx &c) { return c.bd; }
template <typename T> static SeeQueue<T> &see_queue(pic_ctx &c);
template <> SeeQueue<float> &see_queue<float>(pic_ctx &c) { return c.sqf; }
template <> SeeQueue<double> &see_queue<double>(pic_ctx &c) { return c.sqd; }

template <typename T> static PassArgs<T> pass_args(pic_ctx &c, int s, int64_t step)
{
    PassArgs<T> a{};
    a.p = parts<T>(c, s, c.cur[s]);
    a.q = c.cq[s];
    a.count = c.ctl + s;
    a.ef = reinterpret_cast<const typename Field4<T>::type *>(c.ef);
    a.eb = reinterpret_cast<const typename Field2<T>::type *>(c.eb);
    a.accJ = c.accJ + (size_t)s * c.g.nodes;
    a.accQ = c.accQ + (size_t)s * c.g.nodes;
    a.accW = c.accW + (size_t)s * c.g.nodes;
    a.stats = c.stats;
    a.err = c.errw;
    a.g = c.g;
    a.sc = c.sc[s];
    a.mc = c.mc;
    a.b = births<T>(c);
    if (s == 1) a.see = see_queue<T>(c);   // ions only; cap 0 keeps emission off
    a.step = (int32_t)step;
    return a;
}

template <typename T> static void sort_species(pic_ctx &c, int s)
{
    const int from = c.cur[s], to = 1 - from;
    timer_start(c, c.t_sort);
    launch_sort<T>(parts<T>(c, s, from), parts<T>(c, s, to), c.ctl + s, c.ctl + 2 + s, c.hist, c.cursor, c.scanpart,
                   c.g.ncells, c.cfg.capacity[s], c.stream);
    timer_stop(c, c.t_sort);
    c.cur[s] = to;
}

// cos, sin of m th_n for the retained orders m = 1..M (Eq. et_reconstruct
// at every order's frequency)
static Orders step_orders(const pic_ctx &c, int64_t n)
{
    const double th = TWO_PI * (double)(n % c.nrf) / (double)c.nrf;
    Orders o{};
    o.n = c.M;
    for (int m = 0; m < c.M; ++m) {
        o.cs[m] = std::cos((m + 1) * th);
        o.sn[m] = std::sin((m + 1) * th);
    }
    return o;
}

template <typename T> static void stage(pic_ctx &c, int64_t n)
{
    const double th = TWO_PI * (double)(n % c.nrf) / (double)c.nrf;
    launch_stage<T>(c.phi, c.d_ec, c.d_es, step_orders(c, n),
                    reinterpret_cast<typename Field4<T>::type *>(c.ef), c.accJ, c.accQ, true, c.g, c.stream);
    if (c.eb)
        launch_stage_b<T>(c.d_ec, c.d_es, std::cos(th), std::sin(th), 1.0 / (TWO_PI * c.cfg.freq),
                          reinterpret_cast<typename Field2<T>::type *>(c.eb), c.g, c.stream);
}

template <typename T> static void run_pass(pic_ctx &c, int64_t n, bool push, bool depq)
{
    const bool timed = push;   // one timer pair around the launch of both species
    if (timed) timer_start(c, c.t_pass);
    launch_pass<T>(pass_args<T>(c, 0, n), pass_args<T>(c, 1, n), c.cfg.capacity[0], c.cfg.capacity[1], push, depq,
                   c.stream);
    if (timed) timer_stop(c, c.t_pass);
}

template <typename T> static void run_collide(pic_ctx &c, int64_t n)
{
    for (int s = 0; s < 2; ++s) launch_collide<T>(pass_args<T>(c, s, n), c.stream);
}

template <typename T> static void run_births(pic_ctx &c, bool deposit, int64_t n = 0)
{
    launch_births<T>(births<T>(c), parts<T>(c, 0, c.cur[0]), parts<T>(c, 1, c.cur[1]), c.ctl, c.ctl + 4,
                     c.cfg.capacity[0], c.cfg.capacity[1], c.accQ, c.accQ + c.g.nodes, deposit, c.qscale, c.g,
                     c.errw, c.stats, c.cq[0].count, c.cq[1].count, c.stream);
    // secondary electrons of the step's ions at metal walls, after the
    // ionization births
    const SeeQueue<T> &q = see_queue<T>(c);
    if (q.cap > 0)
        launch_see<T>(q, parts<T>(c, 0, c.cur[0]), c.ctl, c.ctl + 4, c.cfg.capacity[0], c.accQ, deposit, c.qscale,
                      c.g, c.errw, c.stats, c.cfg.seed, (int32_t)n, c.lq[0], c.stream);
}

// with_chi: the direct-implicit susceptibility of the deposited (predicted)
// particles joins the operator; the initial solve at the loaded positions is
// the plain Poisson problem (no push precedes it)
static void finalize_charge(pic_ctx &c, bool with_chi)
{
    const pic_config &f = c.cfg;
    launch_finalize_q(c.accQ, c.accW, c.accS, 1.0 / c.qscale, f.q[0] * f.w[0] / c.qscale, f.q[1] * f.w[1] / c.qscale,
                      f.q[0] * f.w[0], f.q[1] * f.w[1], c.Q, c.g.nodes, c.stream);
    if (c.chi && with_chi) {
        // susceptibility of the deposited (predicted) particles and the
        // level-0 operator with it; the coarse levels keep the chi = 0
        // Galerkin operators as the preconditioner of the CG
        const double k = 0.5 * f.dt * f.dt / f.eps0 / c.qscale;
        launch_chi(c.accQ, k * f.q[0] * f.q[0] / f.m[0] * f.w[0], k * f.q[1] * f.q[1] / f.m[1] * f.w[1], c.chi,
                   c.cw0, c.ce0, c.cs0, c.cn0, c.lv.L[0], c.g, c.stream);
    }
}

// V-cycle on the correction (level 0: right-hand side = the CG residual r,
// correction = z): two red-black sweeps on the 5-point fine level, one
// four-colour sweep on the Galerkin levels, dense-inverse solve on the bottom level
// (dense inverse, one multi-block product).  The pre-smoothers start from
// zero, the coarse ones with the right-hand side restricted from the finer
// level's residual; the post-smoothers add the prolonged coarse correction
// as they load their tiles, the level-0 one leaving the partials of r.z.
#ifndef PIC_MG_NU0
#define PIC_MG_NU0 2
#endif
#ifndef PIC_MG_NU
#define PIC_MG_NU 1
#endif
static void vcycle(pic_ctx &c, const MGLevels &lv, const MGState *st)
{
    const int lb = c.lb;
    // Each level above the bottom keeps two corrections: the pre-smoothed one
    // (read as the post-smoother's start and halo) and the post-smoothed one,
    // so no smoother launch reads what a neighbouring tile of the same launch
    // writes.  Level 0: pre-smoothed in the A p buffer (idle during the
    // V-cycle), post-smoothed into z (= L[0].phi, Dirichlet entries 0 since
    // the start of the solve).  Levels l >= 1: pre-smoothed in phi,
    // post-smoothed into res, free once restricted (Dirichlet entries 0).
    MGLevel pre[MAX_LEVELS], post[MAX_LEVELS];
    for (int l = 0; l <= lb; ++l) {
        pre[l] = post[l] = lv.L[l];
        if (l == 0 && lb > 0) pre[0].phi = c.pAp;
        if (l > 0 && l < lb) post[l].phi = lv.L[l].res;
    }
    for (int l = 0; l < lb; ++l) {
        const int nu = l == 0 ? PIC_MG_NU0 : PIC_MG_NU;
        launch_mg_smooth_tile(pre[l], l > 0 ? &pre[l - 1] : nullptr, nullptr, nu, SM_ZERO | (l > 0 ? SM_RHS : 0), st,
                              nullptr, pre[l].phi, c.stream);
        launch_mg_resid(pre[l], st, c.stream);
    }
    if (lb > 0) launch_mg_restrict_res(pre[lb - 1], pre[lb], st, c.stream);
    launch_dense_solve(lv.coarse_inv32, lv.L[lb], st, c.stream);
    for (int l = lb - 1; l >= 0; --l) {
        const int nu = l == 0 ? PIC_MG_NU0 : PIC_MG_NU;
        launch_mg_smooth_tile(pre[l], nullptr, &post[l + 1], nu, SM_REVERSE | SM_PROLONG | (l == 0 ? SM_RZ : 0), st,
                              c.mgpartial, post[l].phi, c.stream);
    }
}

// preconditioned-CG iteration k of a solve (no-ops once st->done); the
// search direction alternates between two buffers (the p update and the
// product A p are one kernel)
static void pcg_iteration(pic_ctx &c, const MGLevels &lv, MGState *st, const PCGVec &v, double rtol, int k,
                          unsigned long long *unconv = nullptr)
{
    const MGLevel &L0 = lv.L[0];
    vcycle(c, lv, st);
    int nrz = smooth_blocks(L0);
    if (c.lb == 0) {
        launch_pcg_rz(L0, v, st, c.mgpartial, c.stream);
        nrz = pcg_blocks(L0.nodes);
    }
    const double *pold = (k & 1) ? c.pp2 : c.pp;
    double *pnew = (k & 1) ? c.pp : c.pp2;
    launch_pcg_pmatvec(L0, v, pold, pnew, st, c.mgpartial, nrz, c.stream);
    launch_pcg_update(L0, v, pnew, st, c.mgpartial, c.stream);
    launch_pcg_check(st, c.mgpartial, pcg_blocks(L0.nodes), rtol, false, c.stream, unconv);
}

// Preconditioned CG on the free nodes (x = phi, b = node charge), one
// V-cycle per iteration; scalars stay on the device.
static pic_status solve_direct(pic_ctx &c, int64_t n, double rtol, pic_solve_info *info);

static pic_status solve(pic_ctx &c, int64_t n, double rtol, int max_cycles, pic_solve_info *info, bool full = false)
{
    if (c.direct && !c.chi) return solve_direct(c, n, rtol, info);
    const double th = TWO_PI * (double)(n % c.nrf) / (double)c.nrf;
    timer_start(c, c.t_poisson);
    const MGLevel &L0 = c.lv.L[0];
    const PCGVec v{c.phi, c.Q, c.pr, c.pz, c.pp, c.pAp};
    // budget from the latest finished solves (pinned ring, read without waiting)
    int budget = max_cycles;
    if (!info && !full && c.mg_host) {
        int seen = 0;
        bool short_run = false;
        for (int k = 0; k < 4; ++k) {
            const volatile MGState *h = c.mg_host + k;
            if (h->ticket == 0xFFFFFFFFu) continue;   // never written
            seen = std::max(seen, (int)h->cycles);
            if (!h->done) short_run = true;
        }
        if (short_run) {
            c.mg_budget = std::min(max_cycles, c.mg_budget + 4);
        } else if (seen > 0) {
            c.mg_budget = std::min(max_cycles, seen + 1);
        }
        budget = std::max(2, std::min(max_cycles, c.mg_budget));
        // after a circuit update (or a restore) the recent counts say
        // nothing about this start value: full budget (iterations past
        // convergence are no-ops)
        // the direct-implicit operator changes with chi every step while the
        // coarse levels precondition with the chi = 0 operator: one
        // iteration beyond the explicit margin, and the full budget until a
        // finished solve has been seen or after one that ran short (a full
        // budget every step spent most of the solve in iterations past
        // convergence, each a dozen launches that find the solve done)
        if (c.cfg.implicit) {
            budget = (c.di_full <= 0 && seen > 0 && !short_run) ? std::min(max_cycles, budget + 1) : max_cycles;
            c.di_full = std::max(0, c.di_full - 1);
        }
        if (c.mg_fresh > 0) budget = max_cycles;
    }
    c.mg_fresh = std::max(0, c.mg_fresh - 1);
    // extrapolate only across consecutive steps of a running sequence: linear
    // once two previous solutions are stored, quadratic once three are
    c.run = (n == c.last_solve + 1 && !full && !info && !c.mg_restart) ? c.run + 1 : 0;
    c.mg_restart = false;
    const int order = c.run >= 3 ? 2 : c.run >= 2 ? 1 : 0;
    launch_pcg_begin(L0, v, c.d_tag, c.d_vc, c.d_vs, step_orders(c, n), c.mgs, c.phi_prev, order, c.stream,
                     c.dbasis, c.cfg.nturns);
    c.last_solve = n;
    const int np = pcg_blocks(L0.nodes);
    budget = std::min(budget, MAX_CG);
    launch_pcg_resid(L0, v, c.mgpartial, c.stream);
    launch_pcg_check(c.mgs, c.mgpartial, np, rtol, true, c.stream);
    // the last iteration's check counts the solve if it ends short of rtol
    // (pic_stats.mg_unconverged)
    for (int k = 0; k < budget; ++k)
        pcg_iteration(c, c.lv, c.mgs, v, rtol, k, k == budget - 1 ? c.stats + ST_MGUNCONV : nullptr);
    if (c.cfg.nturns > 0)
        launch_face_charge(c.phi, c.fp, c.fq, c.fk, c.fc, c.nfaces, c.Qk, c.cfg.nturns, c.stream, c.chi);
    timer_stop(c, c.t_poisson);
    if (c.mg_host) {
        (void)hipMemcpyAsync(c.mg_host + c.mg_ring, c.mgs, sizeof(MGState), hipMemcpyDeviceToHost, c.stream);
        c.mg_ring = (c.mg_ring + 1) % 4;
    }
    if (info) {
        MGState s;
        HIPCHK(&c, hipMemcpyAsync(&s, c.mgs, sizeof s, hipMemcpyDeviceToHost, c.stream));
        HIPCHK(&c, hipStreamSynchronize(c.stream));
        info->cycles = s.cycles;
        info->converged = s.done;
        info->rel_residual = s.rel;
        if (!s.done) return fail(&c, PIC_ENOTCONV, "multigrid-CG: rel residual %.3e after %d iterations", s.rel,
                                 s.cycles);
    }
    return PIC_OK;
}

// Device copy of a separable plan; the direct solve's fixed arguments.
static pic_status upload_direct(pic_ctx &c, const SeparablePlan &sp)
{
    DirectArgs &d = c.da;
    const pic_config &f = c.cfg;
    const MGLevel &L0 = c.lv.L[0];
    d.nr = f.nr;
    d.nz = f.nz;
    d.nodes = c.g.nodes;
    d.ni = sp.ni;
    d.nj = sp.nj;
    d.m = sp.m;
    d.nrow = (int)sp.rows.size();
    d.nturns = f.nturns;
    d.tag = c.d_tag;
    d.vc = c.d_vc;
    d.vs = c.d_vs;
    d.basis = c.dbasis;
    d.phi = c.phi;
    d.Q = c.Q;
    d.cw = L0.cw;
    d.ce = L0.ce;
    d.cs = L0.cs;
    d.cn = L0.cn;
    auto up = [&](const void *dst, const void *src, size_t bytes) {
        return bytes ? cpy(c.stream, const_cast<void *>(dst), src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    if (!c.direct_carved) return fail(&c, PIC_EINVAL, "direct Poisson solve: workspace holds no plan");
    HIPCHK(&c, up(d.v, sp.v.data(), sp.v.size() * 8));
    HIPCHK(&c, up(d.lam, sp.lam.data(), sp.lam.size() * 8));
    HIPCHK(&c, up(d.zrow, sp.zrow.data(), sp.zrow.size() * 8));
    HIPCHK(&c, up(d.erow, sp.erow.data(), sp.erow.size() * 8));
    HIPCHK(&c, up(d.cinv, sp.cinv.data(), sp.cinv.size() * 8));
    HIPCHK(&c, up(d.g, sp.g.data(), sp.g.size() * 8));
    HIPCHK(&c, up(d.dnode, sp.dnode.data(), sp.dnode.size() * 4));
    HIPCHK(&c, up(d.drow, sp.drow.data(), sp.drow.size() * 4));
    HIPCHK(&c, up(d.rows, sp.rows.data(), sp.rows.size() * 4));
    {
        std::vector<int32_t> rs(sp.rows.size() + 1, 0);
        for (int32_t r : sp.drow) ++rs[r + 1];
        for (size_t q = 0; q < sp.rows.size(); ++q) rs[q + 1] += rs[q];
        HIPCHK(&c, up(d.rowstart, rs.data(), rs.size() * 4));
    }
    c.direct = true;
    return PIC_OK;
}

// The direct solve of step n (phase th_n): phi on every node, then the turn
// charges; info gets the relative residual from the multigrid's residual
// and check kernels (scale as for the iterative solve).
static pic_status solve_direct(pic_ctx &c, int64_t n, double rtol, pic_solve_info *info)
{
    timer_start(c, c.t_poisson);
    DirectArgs a = c.da;
    a.o = step_orders(c, n);
    launch_direct_solve(a, c.stream);
    c.last_solve = n;
    c.run = 0;
    c.mg_fresh = 0;
    c.mg_restart = false;
    if (c.cfg.nturns > 0)
        launch_face_charge(c.phi, c.fp, c.fq, c.fk, c.fc, c.nfaces, c.Qk, c.cfg.nturns, c.stream, c.chi);
    timer_stop(c, c.t_poisson);
    if (info) {
        const MGLevel &L0 = c.lv.L[0];
        const PCGVec v{c.phi, c.Q, c.pr, c.pz, c.pp, c.pAp};
        launch_pcg_begin(L0, v, c.d_tag, c.d_vc, c.d_vs, a.o, c.mgs, nullptr, 0, c.stream, c.dbasis,
                         c.cfg.nturns);
        launch_pcg_resid(L0, v, c.mgpartial, c.stream);
        launch_pcg_check(c.mgs, c.mgpartial, pcg_blocks(L0.nodes), rtol, true, c.stream);
        MGState s;
        HIPCHK(&c, hipMemcpyAsync(&s, c.mgs, sizeof s, hipMemcpyDeviceToHost, c.stream));
        HIPCHK(&c, hipStreamSynchronize(c.stream));
        info->cycles = 0;
        info->converged = s.done;
        info->rel_residual = s.rel;
        if (!s.done) return fail(&c, PIC_ENOTCONV, "direct Poisson solve: rel residual %.3e", s.rel);
    }
    return PIC_OK;
}

// Multigrid hierarchy of a level-0 five-point operator (co) with Dirichlet
// mask dir: level-0 coefficients, Galerkin coarse levels and the dense
// inverse of the coarsest level, all copied into lv's device arrays.
static pic_status build_levels(pic_ctx &c, MGLevels &lv, const Coeffs &co, const std::vector<uint8_t> &dir)
{
    const pic_config &f = c.cfg;
    const int nodes = c.g.nodes;
    MGLevel &L0 = lv.L[0];
    const size_t nb = (size_t)nodes * sizeof(double);
    HIPCHK(&c, cpy(c.stream, (void *)L0.cw, co.cw.data(), nb, hipMemcpyHostToDevice));
    HIPCHK(&c, cpy(c.stream, (void *)L0.ce, co.ce.data(), nb, hipMemcpyHostToDevice));
    HIPCHK(&c, cpy(c.stream, (void *)L0.cs, co.cs.data(), nb, hipMemcpyHostToDevice));
    HIPCHK(&c, cpy(c.stream, (void *)L0.cn, co.cn.data(), nb, hipMemcpyHostToDevice));
    HIPCHK(&c, cpy(c.stream, (void *)L0.cc, co.cc.data(), nb, hipMemcpyHostToDevice));
    HIPCHK(&c, cpy(c.stream, (void *)L0.dir, dir.data(), nodes, hipMemcpyHostToDevice));
    Stencil9 S;
    S.nr = f.nr;
    S.nz = f.nz;
    S.dir = dir;
    S.a.assign(9 * (size_t)nodes, 0.0);
    for (int n = 0; n < nodes; ++n) {
        S.a[(size_t)4 * nodes + n] = co.cc[n];
        S.a[(size_t)3 * nodes + n] = -co.cw[n];
        S.a[(size_t)5 * nodes + n] = -co.ce[n];
        S.a[(size_t)1 * nodes + n] = -co.cs[n];
        S.a[(size_t)7 * nodes + n] = -co.cn[n];
    }
    for (int l = 1; l < lv.n; ++l) {
        S = galerkin(S);
        MGLevel &L = lv.L[l];
        HIPCHK(&c, cpy(c.stream, (void *)L.a, S.a.data(), S.a.size() * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(&c, cpy(c.stream, (void *)L.dir, S.dir.data(), S.dir.size(), hipMemcpyHostToDevice));
        HIPCHK(&c, mset(c.stream, L.phi, 0, (size_t)L.nodes * sizeof(double)));
        HIPCHK(&c, mset(c.stream, L.rhs, 0, (size_t)L.nodes * sizeof(double)));
    }
    // dense inverse of the bottom level, computed on the device by
    // Gauss-Jordan elimination (no pivoting: the free block is symmetric
    // positive definite and Dirichlet rows are identity rows)
    {
        const int m = (S.nz + 1) * (S.nr + 1), nr1 = S.nr + 1;
        std::vector<double> A((size_t)m * m, 0.0);
        for (int n = 0; n < m; ++n) {
            const int i = n / nr1, j = n - i * nr1;
            if (S.dir[n]) {
                A[(size_t)n * m + n] = 1.0;
                continue;
            }
            for (int k = 0; k < 9; ++k) {
                const int di = k / 3 - 1, dj = k % 3 - 1;
                if (i + di < 0 || i + di > S.nz || j + dj < 0 || j + dj > S.nr) continue;
                const int q = n + di * nr1 + dj;
                if (S.dir[q]) continue;
                A[(size_t)n * m + q] = S.a[(size_t)k * m + n];
            }
            if (!(A[(size_t)n * m + n] > 0.0)) return fail(&c, PIC_EINVAL, "bottom multigrid level not definite");
        }
        HIPCHK(&c, hipMemcpy2DAsync((void *)lv.coarse_inv, (size_t)dense_ld(m) * sizeof(double), A.data(),
                                    (size_t)m * sizeof(double), (size_t)m * sizeof(double), m, hipMemcpyHostToDevice,
                                    c.stream));
        launch_gauss_jordan(const_cast<double *>(lv.coarse_inv), m, c.pp, c.pAp, c.stream);
        launch_inverse_f32(lv.coarse_inv, m, const_cast<float *>(lv.coarse_inv32), c.stream);
        HIPCHK(&c, hipStreamSynchronize(c.stream));
    }
    return PIC_OK;
}

// K u = src for one inductive field x (free nodes), b = -mu0 w R src in
// hb: CG on the R-weighted symmetric operator with multigrid preconditioning,
// in chunks of iterations with a convergence check between chunks.
static pic_status helm_solve(pic_ctx &c, double *x, int *cycles, double *rel, double rtol = 0.0, int maxc = 0)
{
    const MGLevel &L0 = c.hlv.L[0];
    const PCGVec v{x, c.hb, c.pr, c.pz, c.pp, c.pAp};
    if (rtol <= 0.0) rtol = c.cfg.helm_rtol;
    maxc = std::min(maxc > 0 ? maxc : c.cfg.helm_max_cycles, MAX_CG);
    launch_pcg_begin(L0, v, c.htag, nullptr, nullptr, Orders{1, {0.0}, {0.0}}, c.hgs, nullptr, 0, c.stream);
    launch_pcg_resid(L0, v, c.mgpartial, c.stream);
    launch_pcg_check(c.hgs, c.mgpartial, pcg_blocks(L0.nodes), rtol, true, c.stream);
    MGState s{};
    int run = 0;
    for (;;) {
        HIPCHK(&c, cpy(c.stream, &s, c.hgs, sizeof s, hipMemcpyDeviceToHost));
        if (s.done || run >= maxc) break;
        const int chunk = std::min(run == 0 ? 4 : 8, maxc - run);
        for (int k = 0; k < chunk; ++k) pcg_iteration(c, c.hlv, c.hgs, v, rtol, run + k);
        run += chunk;
    }
    if (cycles) *cycles = s.cycles;
    if (rel) *rel = s.rel;
    if (!s.done)
        return fail(&c, PIC_ENOTCONV, "inductive solve: rel residual %.3e after %d iterations", s.rel, s.cycles);
    return PIC_OK;
}

// Five-point inductive operator in R-weighted symmetric form (see
// circuit.hip): Dirichlet on the axis, the outer boundary and metal
// (tag 0); turn nodes are free source nodes.
static void helm_operator(const pic_ctx &c, Coeffs &co, std::vector<uint8_t> &dir)
{
    const pic_config &f = c.cfg;
    const int nr = f.nr, nz = f.nz, nr1 = nr + 1, nodes = (nz + 1) * nr1;
    const double dr = c.g.dr, dz = c.g.dz, w = TWO_PI * f.freq;
    co.cw.assign(nodes, 0.0);
    co.ce.assign(nodes, 0.0);
    co.cs.assign(nodes, 0.0);
    co.cn.assign(nodes, 0.0);
    co.cc.assign(nodes, 1.0);
    dir.assign(nodes, 1);
    for (int i = 1; i < nz; ++i)
        for (int j = 1; j < nr; ++j) {
            const int n = i * nr1 + j;
            if (c.tag[n] == 0) continue;
            dir[n] = 0;
            double k2 = 0.0;
            if (f.field_mode == PIC_FIELD_FULL) {
                // node permittivity: mean of the four cells touching the node
                const double e = 0.25 * (c.eps_cell[(size_t)(i - 1) * nr + j - 1] + c.eps_cell[(size_t)(i - 1) * nr + j] +
                                         c.eps_cell[(size_t)i * nr + j - 1] + c.eps_cell[(size_t)i * nr + j]);
                k2 = f.mu0 * f.eps0 * e * w * w;
            }
            const double R = j * dr;
            co.cc[n] = R * (2.0 / (dz * dz) + 2.0 / (dr * dr) + 1.0 / (R * R) - k2);
            co.cs[n] = co.cn[n] = R / (dz * dz);
            co.ce[n] = (R + 0.5 * dr) / (dr * dr);
            co.cw[n] = (R - 0.5 * dr) / (dr * dr);
        }
}

// Next period's azimuthal field of every order from its plasma-only part
// and the applied turn currents (Eq. compose)
static void compose_fields(pic_ctx &c)
{
    const int nodes = c.g.nodes;
    const size_t un = (size_t)c.cfg.nturns * nodes;
    for (int m = 0; m < c.M; ++m) {
        const double *ep = c.Ep + (size_t)2 * m * nodes;
        launch_compose(ep, ep + nodes, c.U + m * un, nodes, c.cd + m, c.d_ec + (size_t)m * nodes,
                       c.d_es + (size_t)m * nodes, nodes, c.stream);
    }
}

// Initialisation of the coupling (Sec. 2.2 and the workflow's
// initialisation): shape functions, unit fields, Z_vac, network constants,
// the first applied state, its turn potentials and azimuthal field.
static pic_status circuit_init(pic_ctx &c)
{
    const pic_config &f = c.cfg;
    const int N = f.nturns, nodes = c.g.nodes, nr1 = f.nr + 1;
    const double w = TWO_PI * f.freq, dr = c.g.dr, dz = c.g.dz;
    CircuitDev &h = c.cdh;
    std::memset(&h, 0, sizeof h);
    h.N = N;
    h.nrf = c.nrf;
    h.omega = w;
    h.freq = f.freq;
    // turn node list, shape functions g_k = s_k / A_k (Eq. shape)
    std::vector<int32_t> list, lturn;
    std::vector<int> count(N, 0);
    std::vector<double> rsum(N, 0.0);
    for (int n = 0; n < nodes; ++n)
        if (c.tag[n] >= 1) {
            list.push_back(n);
            lturn.push_back(c.tag[n] - 1);
            count[c.tag[n] - 1] += 1;
            rsum[c.tag[n] - 1] += (n % nr1) * dr;
        }
    c.nlist = (int)list.size();
    std::vector<double> g(MAX_TURNS, 0.0);
    c.area.assign(N, 0.0);
    for (int k = 0; k < N; ++k) {
        if (count[k] == 0) return fail(&c, PIC_EINVAL, "turn %d has no nodes", k + 1);
        const double s = f.turn_sign ? f.turn_sign[k] : 1.0;
        if (s != 1.0 && s != -1.0) return fail(&c, PIC_EINVAL, "turn_sign[%d] must be +1 or -1", k);
        c.area[k] = count[k] * dz * dr;
        g[k] = s / c.area[k];
        double norm = 0.0;
        for (int e = 0; e < c.nlist; ++e)
            if (lturn[e] == k) norm += g[k] * dz * dr;
        if (std::fabs(norm - s) > 1e-12) return fail(&c, PIC_EINVAL, "turn %d: shape normalisation fails", k + 1);
    }
    if (c.nlist) {
        HIPCHK(&c, cpy(c.stream, c.plist, list.data(), list.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(&c, cpy(c.stream, c.pturn, lturn.data(), lturn.size() * 4, hipMemcpyHostToDevice));
    }
    HIPCHK(&c, cpy(c.stream, c.gval, g.data(), MAX_TURNS * 8, hipMemcpyHostToDevice));
    h.order = 1;
    h.vg_ratio = 1.0;
    if (!f.circuit) {
        HIPCHK(&c, cpy(c.stream, c.cd, &h, sizeof h, hipMemcpyHostToDevice));
        return PIC_OK;
    }
    // network constants (Eqs. zsource, skin, zturn_field) of order m (1 =
    // the fundamental) at its angular frequency m w
    const double rho = f.rho20 * (1.0 + f.alpha_cu * (f.temp_c - 20.0));
    auto network_constants = [&](CircuitDev &o, int m) {
        const double wm = m == 1 ? w : TWO_PI * (f.freq * m);
        o.omega = wm;
        o.alpha = f.alpha;
        o.zs_re = f.r_g + f.r_m;
        o.zs_im = wm * f.l_m - (f.c_m > 0.0 ? 1.0 / (wm * f.c_m) : 0.0);
        const double delta = std::sqrt(2.0 * rho / (wm * f.mu0));
        for (int k = 0; k < N; ++k) {
            if (f.rrf_mode == PIC_RRF_SKIN) {
                const double rw = std::sqrt(c.area[k] / M_PI), rmean = rsum[k] / count[k];
                const double inner = std::max(rw - delta, 0.0);
                o.rrf[k] = rho * TWO_PI * rmean / (M_PI * (rw * rw - inner * inner));
            } else {
                o.rrf[k] = f.r_rf[k];
            }
            o.cstray[k] = f.c_stray ? f.c_stray[k] : 0.0;
        }
    };
    network_constants(h, 1);
    h.controller = f.controller;
    h.vg_from_target = f.vg_from_target;
    h.p_target = f.p_target;
    h.gamma = f.gamma;
    h.n_trend = f.n_trend;
    h.eps_p = f.eps_p;
    h.alpha_v = f.alpha_v;
    h.f_step = f.f_step;
    h.v_min = f.v_min;
    h.v_max = f.v_max;
    h.vg_amp = f.vg_amp;
    h.vg_phase = f.vg_phase;
    h.pressure = f.ngas * f.tgas_ev * f.qe;
    HIPCHK(&c, cpy(c.stream, c.cd, &h, sizeof h, hipMemcpyHostToDevice));
    // the orders above the fundamental: the same network at m w without a
    // controller of their own; the source of order m is rho_m exp(i phi_m)
    // times the fundamental's
    for (int m = 2; m <= c.M; ++m) {
        CircuitDev o = h;
        network_constants(o, m);
        o.order = m;
        o.controller = 0;
        o.vg_from_target = 0;
        o.vg_ratio = f.harm_ratio[m - 2];
        o.vg_amp = f.vg_amp * o.vg_ratio;
        o.vg_phase = f.vg_phase + f.harm_phase[m - 2];
        HIPCHK(&c, cpy(c.stream, c.cd + (m - 1), &o, sizeof o, hipMemcpyHostToDevice));
    }
    // inductive operator hierarchy
    Coeffs co;
    std::vector<uint8_t> dir;
    helm_operator(c, co, dir);
    pic_status st = build_levels(c, c.hlv, co, dir);
    if (st) return st;
    std::vector<int32_t> htag(nodes);
    for (int n = 0; n < nodes; ++n) htag[n] = dir[n] ? 0 : -1;
    HIPCHK(&c, cpy(c.stream, c.htag, htag.data(), nodes * 4, hipMemcpyHostToDevice));
    const size_t un = (size_t)N * nodes;
    HIPCHK(&c, mset(c.stream, c.U, 0, c.M * un * 8));
    // manufactured boundary values of the unit fields (the solves keep the
    // Dirichlet entries of their start value)
    if (f.unit_bvals) {
        std::vector<double> ub(un, 0.0);
        for (int k = 0; k < N; ++k)
            for (int n = 0; n < nodes; ++n)
                if (dir[n]) ub[(size_t)k * nodes + n] = f.unit_bvals[(size_t)k * nodes + n];
        for (int m = 0; m < c.M; ++m)
            HIPCHK(&c, cpy(c.stream, c.U + m * un, ub.data(), ub.size() * 8, hipMemcpyHostToDevice));
    }
    HIPCHK(&c, mset(c.stream, c.Ep, 0, 2 * (size_t)c.M * nodes * 8));
    HIPCHK(&c, mset(c.stream, c.hgs, 0, sizeof(MGState)));
    // unit-current fields K U_k = g_k (Eq. unitfield) at every order's
    // frequency (the magnetoquasistatic operator is the same for all; the
    // right-hand side scales with m w), and Z_vac of every order (Eq. zvac)
    for (int m = 1; m <= c.M; ++m) {
        const double mw = f.mu0 * (m == 1 ? w : TWO_PI * (f.freq * m));
        double *Um = c.U + (m - 1) * un;
        for (int k = 0; k < N; ++k) {
            launch_unit_rhs(c.d_tag, k, g[k], c.hlv.L[0].dir, mw, c.hb, c.g, c.stream);
            st = helm_solve(c, Um + (size_t)k * nodes, nullptr, nullptr);
            if (st) return st;
        }
        launch_project(Um, N, nodes, c.plist, c.pturn, c.nlist, c.gval, N,
                       reinterpret_cast<double *>(reinterpret_cast<char *>(c.cd + (m - 1)) + offsetof(CircuitDev, mvac)),
                       MAX_TURNS, c.g, c.stream);
    }
    // first state, turn potentials and field
    if (c.M == 1)
        launch_circuit(c.cd, c.harm, c.d_vc, c.d_vs, 0, c.stream);
    else
        launch_circuit_orders(c.cd, c.M, c.d_vc, c.d_vs, 0, c.stream);
    compose_fields(c);
    HIPCHK(&c, cpy(c.stream, &h, c.cd, sizeof h, hipMemcpyDeviceToHost));
    if (h.singular) return fail(&c, PIC_EINVAL, "singular circuit network");
    return PIC_OK;
}

template <typename T> static pic_status init_impl(pic_ctx &c)
{
    const pic_config &f = c.cfg;
    hipStream_t st = c.stream;
    const int nodes = c.g.nodes;
    // zero every counter / accumulator region
    HIPCHK(&c, hipMemsetAsync(c.ctl, 0, 8 * sizeof(int64_t), st));
    HIPCHK(&c, hipMemsetAsync(c.stats, 0, ST_NSTAT * sizeof(unsigned long long), st));
    HIPCHK(&c, hipMemsetAsync(c.errw, 0, sizeof(int32_t), st));
    HIPCHK(&c, hipMemsetAsync(c.hist, 0, (c.g.ncells + 1) * sizeof(int32_t), st));
    HIPCHK(&c, hipMemsetAsync(births<T>(c).count, 0, sizeof(int32_t), st));
    HIPCHK(&c, hipMemsetAsync(births<T>(c).rank, 0, (size_t)births<T>(c).cap * sizeof(int32_t), st));
    if (see_queue<T>(c).cap > 0) {
        HIPCHK(&c, hipMemsetAsync(see_queue<T>(c).count, 0, 2 * sizeof(int32_t), st));
        HIPCHK(&c, hipMemsetAsync(see_queue<T>(c).rank, 0, (size_t)see_queue<T>(c).cap * sizeof(int32_t), st));
    }
    for (int s2 = 0; s2 < 2; ++s2) HIPCHK(&c, hipMemsetAsync(c.cq[s2].count, 0, sizeof(int32_t), st));
    HIPCHK(&c, hipMemsetAsync(c.accS, 0, 2 * (size_t)nodes * sizeof(double), st));
    HIPCHK(&c, hipMemsetAsync(c.accW, 0, 2 * (size_t)nodes * sizeof(long long), st));
    HIPCHK(&c, hipMemsetAsync(c.phi, 0, nodes * sizeof(double), st));
    HIPCHK(&c, hipMemsetAsync(c.I, 0, nodes * sizeof(double), st));
    const size_t mn = (size_t)c.M * nodes;
    HIPCHK(&c, hipMemsetAsync(c.Jc, 0, mn * sizeof(double), st));
    HIPCHK(&c, hipMemsetAsync(c.Jcc, 0, mn * sizeof(double), st));
    HIPCHK(&c, hipMemsetAsync(c.Js, 0, mn * sizeof(double), st));
    HIPCHK(&c, hipMemsetAsync(c.Jsc, 0, mn * sizeof(double), st));
    HIPCHK(&c, hipMemsetAsync(c.harm, 0, c.M * sizeof(HarmState), st));
    HIPCHK(&c, hipMemsetAsync(c.Qk, 0, MAX_TURNS * sizeof(double), st));
    HIPCHK(&c, hipMemsetAsync(c.mgs, 0, sizeof(MGState), st));
    HIPCHK(&c, hipMemcpyAsync(c.d_ec, c.ec.data(), mn * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(&c, hipMemcpyAsync(c.d_es, c.es.data(), mn * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(&c, hipMemcpyAsync(c.d_tag, c.tag.data(), nodes * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (c.dbasis)
        HIPCHK(&c, hipMemcpyAsync(c.dbasis, f.dir_basis, (size_t)f.nturns * nodes * sizeof(double),
                                  hipMemcpyHostToDevice, st));
    HIPCHK(&c, hipMemcpyAsync(c.d_vc, c.vc.data(), c.M * MAX_TURNS * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(&c, hipMemcpyAsync(c.d_vs, c.vs.data(), c.M * MAX_TURNS * sizeof(double), hipMemcpyHostToDevice, st));

    // multigrid hierarchy: finite-volume fine operator, Galerkin coarse levels
    {
        const Coeffs co = assemble(f.nr, f.nz, c.g.dr, c.g.dz, c.eps_cell, f.eps0);
        std::vector<uint8_t> dir(nodes);
        for (int n = 0; n < nodes; ++n) dir[n] = c.tag[n] >= 0;
        // turn face list (Eq. facecharge): faces from a turn-k node to a node outside turn k
        {
            std::vector<int32_t> hp, hq, hk;
            std::vector<double> hc;
            const int nr1 = f.nr + 1;
            for (int n = 0; n < nodes; ++n) {
                const int k = c.tag[n];
                if (k < 1) continue;
                const int i = n / nr1, j = n - i * nr1;
                const int nb[4] = {j > 0 ? n - 1 : -1, j < f.nr ? n + 1 : -1, i > 0 ? n - nr1 : -1,
                                   i < f.nz ? n + nr1 : -1};
                const double cf[4] = {co.cw[n], co.ce[n], co.cs[n], co.cn[n]};
                for (int q = 0; q < 4; ++q) {
                    if (nb[q] < 0 || c.tag[nb[q]] == k || cf[q] == 0.0) continue;
                    hp.push_back(n);
                    hq.push_back(nb[q]);
                    hk.push_back(k - 1);
                    hc.push_back(cf[q]);
                }
            }
            c.nfaces = (int)hp.size();
            if (c.nfaces) {
                HIPCHK(&c, cpy(c.stream, c.fp, hp.data(), hp.size() * 4, hipMemcpyHostToDevice));
                HIPCHK(&c, cpy(c.stream, c.fq, hq.data(), hq.size() * 4, hipMemcpyHostToDevice));
                HIPCHK(&c, cpy(c.stream, c.fk, hk.data(), hk.size() * 4, hipMemcpyHostToDevice));
                HIPCHK(&c, cpy(c.stream, c.fc, hc.data(), hc.size() * 8, hipMemcpyHostToDevice));
            }
        }
        pic_status bs = build_levels(c, c.lv, co, dir);
        if (bs) return bs;
        if (f.poisson_solver == PIC_POISSON_DIRECT && !direct_candidate(f))
            return fail(&c, PIC_EINVAL, "direct Poisson solve requested for a direct-implicit or tiny grid");
        if (direct_candidate(f)) {
            SeparablePlan sp;
            // (plan_separable also refuses what the layout did not carve for)
            const std::string why = plan_separable(co.cw, co.ce, co.cs, co.cn, co.cc, c.tag, f.nr, f.nz, sp);
            if (why.empty()) {
                pic_status ds = upload_direct(c, sp);
                if (ds) return ds;
            } else if (f.poisson_solver == PIC_POISSON_DIRECT) {
                return fail(&c, PIC_EINVAL, "direct Poisson solve: %s", why.c_str());
            }
        }
        if (c.chi) {
            // chi = 0 conductances, from which every step's operator is formed
            const size_t nb = (size_t)nodes * sizeof(double);
            HIPCHK(&c, cpy(c.stream, c.cw0, co.cw.data(), nb, hipMemcpyHostToDevice));
            HIPCHK(&c, cpy(c.stream, c.ce0, co.ce.data(), nb, hipMemcpyHostToDevice));
            HIPCHK(&c, cpy(c.stream, c.cs0, co.cs.data(), nb, hipMemcpyHostToDevice));
            HIPCHK(&c, cpy(c.stream, c.cn0, co.cn.data(), nb, hipMemcpyHostToDevice));
            HIPCHK(&c, mset(c.stream, c.chi, 0, nb));
        }
        for (double *v : {c.pr, c.pz, c.pp, c.pp2, c.pAp, c.phi_prev, c.phi_prev + nodes})
            HIPCHK(&c, mset(c.stream, v, 0, (size_t)nodes * sizeof(double)));
    }
    {
        pic_status cs = circuit_init(c);
        if (cs) return cs;
    }

    // fixed-point scales
    const double cells = (double)f.nr * f.ip;
    const double ppc = (double)std::max(f.capacity[0], f.capacity[1]) / std::max(1.0, cells);
    const int64_t kq = 62 - ceil_log2(256.0 * ppc + 1024.0);
    c.qscale = std::ldexp(1.0, (int)kq);
    c.jscale = std::ldexp(1.0, (int)(kq - 6));

    // species and collision constants (null-collision constants: prepare_host)
    for (int s = 0; s < 2; ++s) {
        SpeciesC &sc = c.sc[s];
        sc.s = s;
        sc.h = 0.5 * f.q[s] / f.m[s] * f.dt;
        sc.dtr = f.dt / c.g.dr;
        sc.dtz = f.dt / c.g.dz;
        double t2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            sc.bt[k] = sc.h * f.bfield[k];
            t2 += sc.bt[k] * sc.bt[k];
        }
        for (int k = 0; k < 3; ++k) sc.bs[k] = 2.0 * sc.bt[k] / (1.0 + t2);
        sc.has_b = t2 > 0.0;
        sc.jscale = c.jscale;
        sc.qscale = c.qscale;
        sc.vref = std::sqrt(std::max(f.temp_ev[s], 1e-3) * f.qe / f.m[s]);
        sc.inv_vref = 1.0 / sc.vref;
        sc.hf = (float)sc.h;
        sc.dtrf = (float)sc.dtr;
        sc.dtzf = (float)sc.dtz;
        sc.inv_vreff = (float)sc.inv_vref;
        sc.jscalef = (float)sc.jscale;
        sc.qscalef = (float)sc.qscale;
        for (int k = 0; k < 3; ++k) {
            sc.btf[k] = (float)sc.bt[k];
            sc.bsf[k] = (float)sc.bs[k];
        }
    }
    c.mc.seed = f.seed;
    c.mc.xs_kind = f.xs_kind;
    for (int s = 0; s < 2; ++s) {
        c.mc.numax[s] = c.numax[s];
        c.mc.lq[s] = c.lq[s];
    }
    c.mc.ngas = f.ngas;
    c.mc.qe = f.qe;
    c.mc.me = f.m[0];
    c.mc.mi = f.m[1];
    c.mc.vg = std::sqrt(f.tgas_ev * f.qe / f.m[1]);
    for (int k = 0; k < 13; ++k) c.mc.xs[k] = f.xs[k];

    // plasma
    if (f.load) {
        for (int s = 0; s < 2; ++s) {
            const double vth = std::sqrt(f.temp_ev[s] * f.qe / f.m[s]);
            launch_load<T>(parts<T>(c, s, c.cur[s]), f.np_init[s], f.seed, s, f.rmax, f.ip * c.g.dz, vth, c.lq[s],
                           c.g, st);
        }
        int64_t h[8] = {f.np_init[0], f.np_init[1], 0, 0, f.np_init[0], f.np_init[1], 0, 0};
        HIPCHK(&c, hipMemcpyAsync(c.ctl, h, sizeof h, hipMemcpyHostToDevice, st));
        HIPCHK(&c, hipStreamSynchronize(st));
        for (int s = 0; s < 2; ++s) sort_species<T>(c, s);
    }
    stage<T>(c, 0);
    run_pass<T>(c, 0, false, true);
    finalize_charge(c, false);
    pic_status s = solve(c, 0, f.mg_rtol, f.mg_max_cycles, nullptr, true);
    if (s) return s;
    HIPCHK(&c, hipStreamSynchronize(st));
    return PIC_OK;
}

extern "C" pic_status pic_init(const pic_config *cfg, void *workspace, size_t workspace_bytes, void *stream,
                               pic_ctx **out)
{
    if (!out) return PIC_EINVAL;
    *out = nullptr;
    init_error.clear();
    pic_ctx *c = new pic_ctx();
    pic_status st = check_config(cfg, c);
    if (!st) st = prepare_host(*c, cfg);
    if (st) {
        init_error = c->err;
        delete c;
        return st;
    }
    Carver dry{nullptr};
    layout(*c, dry);
    if (!workspace || workspace_bytes < dry.off) {
        init_error = "workspace smaller than pic_workspace_bytes()";
        delete c;
        return PIC_ENOMEM;
    }
    Carver cv{reinterpret_cast<uint8_t *>(workspace)};
    layout(*c, cv);
    c->stream = reinterpret_cast<hipStream_t>(stream);
    if (hipHostMalloc((void **)&c->mg_host, 4 * sizeof(MGState), hipHostMallocDefault) == hipSuccess) {
        for (int k = 0; k < 4; ++k) {
            std::memset(c->mg_host + k, 0, sizeof(MGState));
            c->mg_host[k].ticket = 0xFFFFFFFFu;
        }
    } else {
        c->mg_host = nullptr;
    }
    st = c->mixed ? init_impl<float>(*c) : init_impl<double>(*c);
    if (st) {
        init_error = c->err;
        pic_destroy(c);
        return st;
    }
    *out = c;
    return PIC_OK;
}

static pic_status sticky(pic_ctx *c)
{
    int32_t e = 0;
    HIPCHK(c, hipMemcpyAsync(&e, c->errw, sizeof e, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (e & ERR_BIRTH_OVERFLOW) return fail(c, PIC_ENOMEM, "birth buffer overflow (raise birth_capacity)");
    if (e & ERR_SEE_OVERFLOW) return fail(c, PIC_ENOMEM, "more than 65536 ions reached a metal wall in one step");
    if (e & ERR_CAPACITY) return fail(c, PIC_ENOMEM, "particle capacity exceeded");
    if (e & ERR_QUEUE_OVERFLOW) return fail(c, PIC_ENOMEM, "collision-candidate queue overflow");
    return PIC_OK;
}

extern "C" pic_status pic_gather_push(pic_ctx *c, int64_t n)
{
    if (!c) return PIC_EINVAL;
    if (n != c->last_push + 1) return fail(c, PIC_ESTATE, "pic_gather_push(%lld) after step %lld", (long long)n,
                                           (long long)c->last_push);
    if (n > 2147483000ll) return fail(c, PIC_EINVAL, "step index too large");
    if (c->cfg.implicit && c->last_push >= 0 && c->last_mcc != c->last_push)
        return fail(c, PIC_ESTATE, "pic_gather_push(%lld) before the corrector of step %lld (mcc_collide)",
                    (long long)n, (long long)c->last_push);
    const bool fuse = c->cfg.fuse != 0;
    const int every_ion = c->cfg.sort_every_ion > 0 ? c->cfg.sort_every_ion : c->cfg.sort_every;
    const bool sort_e = n > 0 && n % c->cfg.sort_every == 0, sort_i = n > 0 && n % every_ion == 0;
    if (c->mixed) {
        if (sort_e) sort_species<float>(*c, 0);
        if (sort_i) sort_species<float>(*c, 1);
        stage<float>(*c, n);
        run_pass<float>(*c, n, true, fuse);
    } else {
        if (sort_e) sort_species<double>(*c, 0);
        if (sort_i) sort_species<double>(*c, 1);
        stage<double>(*c, n);
        run_pass<double>(*c, n, true, fuse);
    }
    c->last_push = n;
    return hipGetLastError() == hipSuccess ? PIC_OK : fail(c, PIC_EDEVICE, "kernel launch failed");
}

// Direct-implicit step n after the field solve: E^{n+1} staged from
// phi^{n+1}, the corrector (positions, velocities, filter, absorption,
// collision candidates), then the collisions and births (their charge
// joins the next step's predicted deposit).
template <typename T> static void implicit_correct_collide(pic_ctx &c, int64_t n)
{
    // the corrector takes E_r, E_z only
    launch_stage<T>(c.phi, c.d_ec, c.d_es, Orders{1, {1.0}, {0.0}},
                    reinterpret_cast<typename Field4<T>::type *>(c.ef), c.accJ, c.accQ, false, c.g, c.stream);
    launch_correct<T>(pass_args<T>(c, 0, n), pass_args<T>(c, 1, n), c.cfg.capacity[0], c.cfg.capacity[1], c.stream);
    run_collide<T>(c, n);
    run_births<T>(c, false);
}

extern "C" pic_status mcc_collide(pic_ctx *c, int64_t n)
{
    if (!c) return PIC_EINVAL;
    if (n != c->last_push || c->last_mcc == n) return fail(c, PIC_ESTATE, "mcc_collide(%lld) out of order", (long long)n);
    if (c->cfg.implicit) {
        if (c->last_solve != n + 1 || c->last_dep != n + 1)
            return fail(c, PIC_ESTATE, "direct-implicit mcc_collide(%lld) before pic_deposit and poisson_solve_rz(%lld)",
                        (long long)n, (long long)(n + 1));
        if (c->mixed)
            implicit_correct_collide<float>(*c, n);
        else
            implicit_correct_collide<double>(*c, n);
        c->last_mcc = n;
        return hipGetLastError() == hipSuccess ? PIC_OK : fail(c, PIC_EDEVICE, "kernel launch failed");
    }
    const bool fuse = c->cfg.fuse != 0;
    if (c->mixed) {
        run_collide<float>(*c, n);
        run_births<float>(*c, fuse, n);
    } else {
        run_collide<double>(*c, n);
        run_births<double>(*c, fuse, n);
    }
    c->last_mcc = n;
    return hipGetLastError() == hipSuccess ? PIC_OK : fail(c, PIC_EDEVICE, "kernel launch failed");
}

extern "C" pic_status pic_deposit(pic_ctx *c, int64_t n1)
{
    if (!c) return PIC_EINVAL;
    // explicit: after the collisions of step n1 - 1; direct-implicit: before them
    // (the corrector follows the field solve)
    const bool ok = c->cfg.implicit ? (n1 == c->last_push + 1 && c->last_mcc != c->last_push && c->last_dep != n1)
                                    : (n1 == c->last_push + 1 && c->last_mcc == c->last_push);
    if (!ok) return fail(c, PIC_ESTATE, "pic_deposit(%lld) out of order", (long long)n1);
    c->last_dep = n1;
    if (!c->cfg.fuse) {
        if (c->mixed)
            run_pass<float>(*c, n1 - 1, false, true);
        else
            run_pass<double>(*c, n1 - 1, false, true);
    }
    finalize_charge(*c, true);
    return hipGetLastError() == hipSuccess ? PIC_OK : fail(c, PIC_EDEVICE, "kernel launch failed");
}

// one plasma-only inductive field from the open period's harmonics:
// which = 0: K E_c^p = J_s / V, which = 1: K E_s^sto,p = J_c / V
// Plasma-only field of order m (0: the fundamental) from that order's
// current harmonic, at its frequency (m + 1) w
static pic_status plasma_field(pic_ctx &c, int which, double rtol, int max_cycles, int *cycles, double *rel, int m = 0)
{
    const double mw = c.cfg.mu0 * (m == 0 ? TWO_PI * c.cfg.freq : TWO_PI * (c.cfg.freq * (m + 1)));
    const uint8_t *hdir = c.hlv.L[0].dir;
    const size_t o = (size_t)m * c.g.nodes;
    if (which == 0)
        launch_helm_rhs(c.Js + o, c.Jsc + o, 2.0 / c.nrf, hdir, mw, c.hb, c.g, c.stream);
    else
        launch_helm_rhs(c.Jc + o, c.Jcc + o, 2.0 / c.nrf, hdir, mw, c.hb, c.g, c.stream);
    return helm_solve(c, c.Ep + (size_t)(2 * m + which) * c.g.nodes, cycles, rel, rtol, max_cycles);
}

extern "C" pic_status poisson_solve_rz(pic_ctx *c, int64_t n, int32_t op, double rtol, int32_t max_cycles,
                                       pic_solve_info *info)
{
    if (!c) return PIC_EINVAL;
    if (op == PIC_OP_POISSON) {
        if (rtol <= 0) rtol = c->cfg.mg_rtol;
        if (max_cycles <= 0) max_cycles = c->cfg.mg_max_cycles;
        return solve(*c, n, rtol, max_cycles, info);
    }
    if (op != PIC_OP_HELMHOLTZ_C && op != PIC_OP_HELMHOLTZ_S) return fail(c, PIC_EINVAL, "unknown operator %d", op);
    if (!c->cfg.circuit) return fail(c, PIC_EINVAL, "inductive solves need a coupled context");
    pic_status st = sticky(c);
    if (st) return st;
    if (rtol <= 0) rtol = c->cfg.helm_rtol;
    if (max_cycles <= 0) max_cycles = c->cfg.helm_max_cycles;
    int cyc = 0;
    double rel = 0.0;
    st = plasma_field(*c, op == PIC_OP_HELMHOLTZ_C ? 0 : 1, rtol, std::min<int>(max_cycles, MAX_CG), &cyc, &rel);
    if (info) {
        info->cycles = cyc;
        info->converged = st == PIC_OK;
        info->rel_residual = rel;
    }
    return st;
}

extern "C" pic_status harmonic_accumulate(pic_ctx *c, int64_t n)
{
    if (!c) return PIC_EINVAL;
    if (n != c->last_push || c->last_harm == n)
        return fail(c, PIC_ESTATE, "harmonic_accumulate(%lld) out of order", (long long)n);
    const pic_config &f = c->cfg;
    const double cj0 = f.q[0] * f.w[0] * c->sc[0].vref / c->jscale, cj1 = f.q[1] * f.w[1] * c->sc[1].vref / c->jscale;
    launch_harmonic(c->accJ, cj0, cj1, c->d_ec, c->d_es, step_orders(*c, n), c->I, c->Jc, c->Jcc, c->Js, c->Jsc,
                    c->hpartial, c->harm, c->Qk, c->d_vc, c->d_vs, f.nturns, c->g.nodes, c->stream);
    c->last_harm = n;
    return hipGetLastError() == hipSuccess ? PIC_OK : fail(c, PIC_EDEVICE, "kernel launch failed");
}

// Surrogate-assisted update (see pic_attach_surrogate): measurement, the
// prediction at the applied state, then the inner fixed point with one
// network prediction per iterate.
static pic_status surrogate_update(pic_ctx &c)
{
    launch_circuit(c.cd, c.harm, c.d_vc, c.d_vs, 3, c.stream);
    launch_features(c.cd, c.feat, false, c.stream);
    pic_status st = mlp_forward(c.net, c.feat, 1, c.pred);
    if (st) return fail(&c, st, "surrogate forward: %s", mlp_last_error(c.net));
    launch_surrogate(c.cd, c.pred, c.d_vc, c.d_vs, 0, c.stream);
    const int maxit = c.cdh.sur_max_iter;
    int32_t done = 0;
    for (int it = 0; it < maxit; ++it) {
        if (it % 5 == 0) {
            HIPCHK(&c, cpy(c.stream, &done, reinterpret_cast<char *>(c.cd) + offsetof(CircuitDev, sur_done), 4,
                           hipMemcpyDeviceToHost));
            if (done) break;
        }
        launch_features(c.cd, c.feat, true, c.stream);
        st = mlp_forward(c.net, c.feat, 1, c.pred);
        if (st) return fail(&c, st, "surrogate forward: %s", mlp_last_error(c.net));
        launch_surrogate(c.cd, c.pred, c.d_vc, c.d_vs, 1, c.stream);
    }
    launch_surrogate(c.cd, c.pred, c.d_vc, c.d_vs, 2, c.stream);
    return PIC_OK;
}

extern "C" pic_status pic_set_source(pic_ctx *c, double vg_amp, double vg_phase)
{
    if (!c) return PIC_EINVAL;
    if (!c->cfg.circuit) return fail(c, PIC_EINVAL, "context without circuit coupling");
    if (c->M > 1) return fail(c, PIC_EINVAL, "the multiharmonic circuit sets its sources from the configuration");
    if (!(vg_amp > 0.0)) return fail(c, PIC_EINVAL, "vg_amp must be positive");
    char *d = reinterpret_cast<char *>(c->cd);
    HIPCHK(c, cpy(c->stream, d + offsetof(CircuitDev, vg_amp), &vg_amp, 8, hipMemcpyHostToDevice));
    HIPCHK(c, cpy(c->stream, d + offsetof(CircuitDev, vg_phase), &vg_phase, 8, hipMemcpyHostToDevice));
    return PIC_OK;
}

extern "C" pic_status pic_attach_surrogate(pic_ctx *c, mlp_ctx *net, const pic_surrogate_config *sc)
{
    if (!c) return PIC_EINVAL;
    if (!net) {
        c->net = nullptr;
        return PIC_OK;
    }
    if (!c->cfg.circuit) return fail(c, PIC_EINVAL, "surrogate needs a coupled context");
    if (c->M > 1) return fail(c, PIC_EINVAL, "the surrogate predicts the fundamental's loads only");
    if (!sc || !(sc->err_max > 0.0) || !(sc->tol > 0.0) || sc->max_iter < 1 || sc->max_iter > SUR_MAX_ITER)
        return fail(c, PIC_EINVAL, "surrogate settings invalid (max_iter 1..%d)", SUR_MAX_ITER);
    const int N = c->cfg.nturns;
    if (N > SUR_MAX_TURNS) return fail(c, PIC_EINVAL, "surrogate supports at most %d turns", SUR_MAX_TURNS);
    int n_in = 0, n_out = 0;
    void *nst = nullptr;
    mlp_shape(net, &n_in, &n_out, &nst);
    if (n_in != 4 * N + 9 || n_out != 4 * N)
        return fail(c, PIC_EINVAL, "surrogate network has %d -> %d, needs %d -> %d", n_in, n_out, 4 * N + 9, 4 * N);
    if (nst != (void *)c->stream) return fail(c, PIC_EINVAL, "surrogate network must use the context's stream");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->cdh.sur_err_max = sc->err_max;
    c->cdh.sur_tol = sc->tol;
    c->cdh.sur_max_iter = sc->max_iter;
    char *d = reinterpret_cast<char *>(c->cd);
    HIPCHK(c, cpy(c->stream, d + offsetof(CircuitDev, sur_max_iter), &c->cdh.sur_max_iter, 4, hipMemcpyHostToDevice));
    HIPCHK(c, cpy(c->stream, d + offsetof(CircuitDev, sur_err_max), &c->cdh.sur_err_max, 8, hipMemcpyHostToDevice));
    HIPCHK(c, cpy(c->stream, d + offsetof(CircuitDev, sur_tol), &c->cdh.sur_tol, 8, hipMemcpyHostToDevice));
    c->net = net;
    return PIC_OK;
}

static pic_status reset_period(pic_ctx *c)
{
    const size_t mn = (size_t)c->M * c->g.nodes;
    HIPCHK(c, mset(c->stream, c->Jc, 0, mn * 8));
    HIPCHK(c, mset(c->stream, c->Jcc, 0, mn * 8));
    HIPCHK(c, mset(c->stream, c->Js, 0, mn * 8));
    HIPCHK(c, mset(c->stream, c->Jsc, 0, mn * 8));
    HIPCHK(c, mset(c->stream, c->harm, 0, c->M * sizeof(HarmState)));
    return PIC_OK;
}

extern "C" pic_status circuit_period_update(pic_ctx *c, const pic_circuit_override *ovr, pic_period_report *rep,
                                            double *jc, double *js)
{
    if (!c) return PIC_EINVAL;
    const bool coupled = c->cfg.circuit != 0;
    const double *new_vc = ovr ? ovr->new_vc : nullptr, *new_vs = ovr ? ovr->new_vs : nullptr;
    const double *new_ec = ovr ? ovr->new_ec : nullptr, *new_es = ovr ? ovr->new_es_sto : nullptr;
    const bool loads = ovr && ovr->loads;
    if (coupled && (new_vc || new_vs || new_ec || new_es))
        return fail(c, PIC_EINVAL, "a coupled context derives turn potentials and field itself");
    if (loads && !coupled) return fail(c, PIC_EINVAL, "prescribed loads need a coupled context");
    if (loads && c->net) return fail(c, PIC_EINVAL, "prescribed loads and an attached surrogate exclude each other");
    if (loads && c->M > 1) return fail(c, PIC_EINVAL, "prescribed loads are for a single-frequency circuit");
    pic_status st = sticky(c);
    if (st) return st;
    int32_t samples = 0;
    HIPCHK(c, cpy(c->stream, &samples, reinterpret_cast<char *>(c->harm) + offsetof(HarmState, samples), 4,
                  hipMemcpyDeviceToHost));
    const int N = c->nrf, K = c->cfg.nturns, nodes = c->g.nodes;
    if (rep) {
        std::memset(rep, 0, sizeof *rep);
        rep->samples = samples;
    }
    if (!c->closed || samples != N) {
        st = reset_period(c);
        if (st) return st;
        if (!c->closed) return fail(c, PIC_EPHASE, "phase closure |f dt N_RF - 1| >= 1e-10: period update rejected");
        return fail(c, PIC_EPHASE, "%d samples in the period, N_RF = %d: update rejected", samples, N);
    }
    timer_start(*c, c->t_circuit);
    if (coupled) {
        // plasma-only fields from the current harmonics of every order
        // (Eq. helmholtz_two_real at the order's frequency), projected on
        // the turns
        for (int m = 0; m < c->M; ++m) {
            for (int q = 0; q < 2; ++q) {
                int cyc = 0;
                double rel = 0.0;
                st = plasma_field(*c, q, 0.0, 0, m == 0 ? &c->helm_cycles[q] : &cyc, m == 0 ? &c->helm_rel[q] : &rel,
                                  m);
                if (st) return st;
            }
            launch_project(c->Ep + (size_t)2 * m * nodes, 2, nodes, c->plist, c->pturn, c->nlist, c->gval, K,
                           reinterpret_cast<double *>(reinterpret_cast<char *>(c->cd + m) + offsetof(CircuitDev, proj)),
                           2, c->g, c->stream);
        }
        // plasma moments of the completed period (surrogate features, report)
        {
            const pic_config &f = c->cfg;
            if (c->mixed)
                launch_moments<float>(c->pf[0][c->cur[0]], c->pf[1][c->cur[1]], c->ctl, c->accQ, c->qscale, f.w[0],
                                      f.w[1], f.m[0], f.m[1], f.qe, c->mompart, moments_blocks(), c->cd, c->stats,
                                      c->g, c->stream);
            else
                launch_moments<double>(c->pd[0][c->cur[0]], c->pd[1][c->cur[1]], c->ctl, c->accQ, c->qscale, f.w[0],
                                       f.w[1], f.m[0], f.m[1], f.qe, c->mompart, moments_blocks(), c->cd, c->stats,
                                       c->g, c->stream);
        }
        // the state applied during the completed period, for the report
        for (int m = 0; m < c->M; ++m)
            HIPCHK(c, cpy(c->stream, c->xp_ord.data() + (size_t)2 * MAX_X * m,
                          reinterpret_cast<char *>(c->cd + m) + offsetof(CircuitDev, x_re),
                          sizeof(c->cdh.x_re) + sizeof(c->cdh.x_im), hipMemcpyDeviceToHost));
        const double *xp = c->xp_ord.data();
        if (loads) {
            // prescribed loads, taken by the update kernel in place of the measured ones
            CircuitDev &h = c->cdh;
            h.ovr_loads = 1;
            for (int k = 0; k < MAX_TURNS; ++k) {
                h.ovr_vp_re[k] = k < K ? ovr->vp_re[k] : 0.0;
                h.ovr_vp_im[k] = k < K ? ovr->vp_im[k] : 0.0;
                h.ovr_icap_re[k] = k < K ? ovr->icap_re[k] : 0.0;
                h.ovr_icap_im[k] = k < K ? ovr->icap_im[k] : 0.0;
            }
            const size_t o0 = offsetof(CircuitDev, ovr_loads), o1 = offsetof(CircuitDev, ovr_icap_im) + sizeof h.ovr_icap_im;
            HIPCHK(c, cpy(c->stream, reinterpret_cast<char *>(c->cd) + o0, reinterpret_cast<const char *>(&h) + o0,
                          o1 - o0, hipMemcpyHostToDevice));
        }
        if (c->net) {
            st = surrogate_update(*c);
            if (st) return st;
        } else if (c->M == 1) {
            launch_circuit(c->cd, c->harm, c->d_vc, c->d_vs, 1, c->stream);
        } else {
            // every order finalises its harmonics and measures its loads,
            // then the joint update (controller on the total port power)
            for (int m = 0; m < c->M; ++m)
                launch_circuit(c->cd + m, c->harm + m, c->d_vc + m * MAX_TURNS, c->d_vs + m * MAX_TURNS, 3,
                               c->stream);
            launch_circuit_orders(c->cd, c->M, c->d_vc, c->d_vs, 1, c->stream);
        }
        compose_fields(*c);
        if (rep)
            for (int r = 0; r < 2 * K + 1; ++r) {
                rep->xp_re[r] = xp[r];
                rep->xp_im[r] = xp[MAX_X + r];
            }
    } else {
        launch_circuit(c->cd, c->harm, c->d_vc, c->d_vs, 2, c->stream);
    }
    timer_stop(*c, c->t_circuit);
    CircuitDev &h = c->cdh;
    HIPCHK(c, cpy(c->stream, &h, c->cd, sizeof h, hipMemcpyDeviceToHost));
    if (coupled && h.singular) return fail(c, PIC_EDEVICE, "singular circuit network");
    if (rep) {
        rep->accepted = 1;
        rep->p_ind = h.p_ind;
        rep->p_cap = h.p_cap;
        rep->p_cap_ph = h.p_cap_ph;
        for (int k = 0; k < K; ++k) {
            rep->qc[k] = h.qc[k];
            rep->qs[k] = h.qs[k];
            rep->icap_re[k] = h.icap_re[k];
            rep->icap_im[k] = h.icap_im[k];
        }
        if (coupled) {
            rep->p_port = h.p_port;
            rep->p_cu = h.p_cu;
            rep->eps_bal = h.eps_bal;
            rep->kcl = h.kcl;
            rep->kvl = h.kvl;
            if (c->M > 1) {   // totals over the retained orders
                rep->p_port = h.tot_p_port;
                rep->p_cu = h.tot_p_cu;
                rep->p_cap_ph = h.tot_p_cap_ph;
                rep->eps_bal = h.tot_eps_bal;
                rep->kcl = h.tot_kcl;
                rep->kvl = h.tot_kvl;
            }
            rep->vg_old = h.vg_old;
            rep->vg_amp = h.vg_amp;
            rep->vg_phase = h.vg_phase;
            rep->pf = h.pf;
            rep->pc = h.pc;
            for (int k = 0; k < K; ++k) {
                rep->vp_re[k] = h.vp_re[k];
                rep->vp_im[k] = h.vp_im[k];
            }
            for (int r = 0; r < 2 * K + 1; ++r) {
                rep->xt_re[r] = h.xt_re[r];
                rep->xt_im[r] = h.xt_im[r];
                rep->x_re[r] = h.x_re[r];
                rep->x_im[r] = h.x_im[r];
            }
            for (int q = 0; q < 2; ++q) {
                rep->helm_cycles[q] = c->helm_cycles[q];
                rep->helm_rel[q] = c->helm_rel[q];
            }
            rep->pressure = h.pressure;
            for (int q = 0; q < 8; ++q) rep->moments[q] = h.moments[q];
            rep->sur_used = c->net ? h.sur_used : 0;
            rep->sur_iters = c->net ? h.sur_iters : 0;
            rep->sur_err = c->net ? h.sur_err : 0.0;
            if (c->net && h.sur_used)
                for (int q = 0; q < std::min(h.sur_iters, SUR_MAX_ITER); ++q) rep->sur_steps[q] = h.sur_hist[q];
        }
    }
    if (jc || js) {
        std::vector<double> a(nodes), b(nodes);
        if (jc) {
            HIPCHK(c, cpy(c->stream, a.data(), c->Jc, nodes * 8, hipMemcpyDeviceToHost));
            HIPCHK(c, cpy(c->stream, b.data(), c->Jcc, nodes * 8, hipMemcpyDeviceToHost));
            for (int n = 0; n < nodes; ++n) jc[n] = 2.0 / N * (a[n] + b[n]);
        }
        if (js) {
            HIPCHK(c, cpy(c->stream, a.data(), c->Js, nodes * 8, hipMemcpyDeviceToHost));
            HIPCHK(c, cpy(c->stream, b.data(), c->Jsc, nodes * 8, hipMemcpyDeviceToHost));
            for (int n = 0; n < nodes; ++n) js[n] = 2.0 / N * (a[n] + b[n]);
        }
    }
    if (!coupled) {
        if (new_vc)
            for (int k = 0; k < K; ++k) c->vc[k] = new_vc[k];
        if (new_vs)
            for (int k = 0; k < K; ++k) c->vs[k] = new_vs[k];
        HIPCHK(c, cpy(c->stream, c->d_vc, c->vc.data(), MAX_TURNS * 8, hipMemcpyHostToDevice));
        HIPCHK(c, cpy(c->stream, c->d_vs, c->vs.data(), MAX_TURNS * 8, hipMemcpyHostToDevice));
        if (new_ec) {
            c->ec.assign(new_ec, new_ec + nodes);
            HIPCHK(c, cpy(c->stream, c->d_ec, new_ec, nodes * 8, hipMemcpyHostToDevice));
        }
        if (new_es) {
            c->es.assign(new_es, new_es + nodes);
            HIPCHK(c, cpy(c->stream, c->d_es, new_es, nodes * 8, hipMemcpyHostToDevice));
        }
    }
    // the turn potentials move by a whole period's correction: the next
    // Poisson solves restart the start-value extrapolation at full budget
    // (three of them: until the quadratic extrapolation again spans only
    // solutions after the jump)
    c->mg_fresh = 3;
    c->mg_restart = true;
    return reset_period(c);
}

extern "C" pic_status circuit_order_report(pic_ctx *c, int32_t order, pic_period_report *rep)
{
    if (!c || !rep) return PIC_EINVAL;
    if (!c->cfg.circuit) return fail(c, PIC_EINVAL, "context without circuit coupling");
    if (order < 1 || order > c->M) return fail(c, PIC_EINVAL, "order %d outside 1..%d", order, c->M);
    pic_status st = sticky(c);
    if (st) return st;
    CircuitDev h;
    HIPCHK(c, cpy(c->stream, &h, c->cd + (order - 1), sizeof h, hipMemcpyDeviceToHost));
    std::memset(rep, 0, sizeof *rep);
    const int K = c->cfg.nturns;
    rep->samples = h.samples;
    rep->accepted = h.samples == c->nrf;
    rep->p_ind = h.p_ind;
    rep->p_cap = h.p_cap;
    rep->p_cap_ph = h.p_cap_ph;
    rep->p_port = h.p_port;
    rep->p_cu = h.p_cu;
    rep->eps_bal = h.eps_bal;
    rep->kcl = h.kcl;
    rep->kvl = h.kvl;
    rep->vg_old = h.vg_old;
    rep->vg_amp = h.vg_amp;
    rep->vg_phase = h.vg_phase;
    for (int k = 0; k < K; ++k) {
        rep->qc[k] = h.qc[k];
        rep->qs[k] = h.qs[k];
        rep->icap_re[k] = h.icap_re[k];
        rep->icap_im[k] = h.icap_im[k];
        rep->vp_re[k] = h.vp_re[k];
        rep->vp_im[k] = h.vp_im[k];
    }
    const double *xp = c->xp_ord.data() + (size_t)2 * MAX_X * (order - 1);
    for (int r = 0; r < 2 * K + 1; ++r) {
        rep->xt_re[r] = h.xt_re[r];
        rep->xt_im[r] = h.xt_im[r];
        rep->x_re[r] = h.x_re[r];
        rep->x_im[r] = h.x_im[r];
        rep->xp_re[r] = xp[r];
        rep->xp_im[r] = xp[MAX_X + r];
    }
    rep->pressure = h.pressure;
    return PIC_OK;
}

// ---------------------------------------------------------------------------
// Checkpoint / restore of the whole time-dependent state at a step boundary
// (the restart of the paper's Appendix A checks).  Everything pic_init
// derives from the configuration alone (operators, multigrid hierarchies,
// unit fields, Z_vac, null-collision constants) is rebuilt by pic_init of
// the restoring context and not stored.
// ---------------------------------------------------------------------------
namespace {
constexpr uint64_t CKPT_MAGIC = 0x3143504349504850ull;   // "PHPICPC1"
struct CkptHead {
    uint64_t magic;
    int32_t precision, nr, nz, nturns, circuit, nrf;
    int64_t capacity[2], count[2];
    int64_t last_push, last_harm, last_mcc, last_solve;
    int32_t run, mg_budget, mg_fresh, mg_restart;
    int32_t norders, pad;
    double qscale, jscale;
    uint64_t total;
};
struct Seg {
    void *p;
    size_t n;
};
}  // namespace

// device arrays of the state, in storage order (count[s] particle slots)
static std::vector<Seg> state_segments(pic_ctx &c, const int64_t count[2])
{
    std::vector<Seg> v;
    const int nodes = c.g.nodes;
    const size_t es = c.mixed ? sizeof(float) : sizeof(double);
    for (int s = 0; s < 2; ++s) {
        void *p[6];
        int32_t *cell, *next;
        uint32_t *id;
        if (c.mixed) {
            const Parts<float> &q = c.pf[s][c.cur[s]];
            cell = q.cell, id = q.id, next = q.next;
            p[0] = q.dr, p[1] = q.dz, p[2] = q.vr, p[3] = q.vt, p[4] = q.vz;
        } else {
            const Parts<double> &q = c.pd[s][c.cur[s]];
            cell = q.cell, id = q.id, next = q.next;
            p[0] = q.dr, p[1] = q.dz, p[2] = q.vr, p[3] = q.vt, p[4] = q.vz;
        }
        const size_t n = (size_t)count[s];
        v.push_back({cell, n * 4});
        for (int k = 0; k < 5; ++k) v.push_back({p[k], n * es});
        v.push_back({id, n * 4});
        v.push_back({next, n * 4});
        if (c.cfg.implicit) {
            void *f[3];
            if (c.mixed)
                f[0] = c.pf[s][c.cur[s]].fr, f[1] = c.pf[s][c.cur[s]].ft, f[2] = c.pf[s][c.cur[s]].fz;
            else
                f[0] = c.pd[s][c.cur[s]].fr, f[1] = c.pd[s][c.cur[s]].ft, f[2] = c.pd[s][c.cur[s]].fz;
            for (int k = 0; k < 3; ++k) v.push_back({f[k], n * es});
        }
    }
    const size_t nb = (size_t)nodes * sizeof(double);
    v.push_back({c.ctl, 8 * sizeof(int64_t)});
    v.push_back({c.stats, ST_NSTAT * sizeof(unsigned long long)});
    v.push_back({c.phi, nb});
    v.push_back({c.phi_prev, 2 * nb});
    v.push_back({c.Q, nb});
    v.push_back({c.I, nb});
    v.push_back({c.accS, 2 * nb});
    v.push_back({c.Qk, MAX_TURNS * sizeof(double)});
    const size_t M = c.M;
    v.push_back({c.Jc, M * nb});
    v.push_back({c.Jcc, M * nb});
    v.push_back({c.Js, M * nb});
    v.push_back({c.Jsc, M * nb});
    v.push_back({c.harm, M * sizeof(HarmState)});
    v.push_back({c.d_vc, M * MAX_TURNS * sizeof(double)});
    v.push_back({c.d_vs, M * MAX_TURNS * sizeof(double)});
    v.push_back({c.d_ec, M * nb});
    v.push_back({c.d_es, M * nb});
    if (c.cfg.circuit) {
        v.push_back({c.Ep, 2 * M * nb});
        v.push_back({c.cd, M * sizeof(CircuitDev)});
    }
    return v;
}

extern "C" pic_status pic_checkpoint(pic_ctx *c, void *buf, size_t cap, size_t *bytes)
{
    if (!c || !bytes) return PIC_EINVAL;
    pic_status st = sticky(c);
    if (st) return st;
    if (c->last_push != c->last_solve - 1 || c->last_mcc != c->last_push)
        return fail(c, PIC_ESTATE, "checkpoint between the calls of a step (last push %lld, solve %lld)",
                    (long long)c->last_push, (long long)c->last_solve);
    CkptHead h{};
    h.magic = CKPT_MAGIC;
    h.precision = c->cfg.precision;
    h.nr = c->cfg.nr;
    h.nz = c->cfg.nz;
    h.nturns = c->cfg.nturns;
    h.circuit = c->cfg.circuit;
    h.nrf = c->nrf;
    h.norders = c->M;
    HIPCHK(c, cpy(c->stream, h.count, c->ctl, 2 * sizeof(int64_t), hipMemcpyDeviceToHost));
    for (int s = 0; s < 2; ++s) h.capacity[s] = c->cfg.capacity[s];
    h.last_push = c->last_push;
    h.last_harm = c->last_harm;
    h.last_mcc = c->last_mcc;
    h.last_solve = c->last_solve;
    h.run = c->run;
    h.mg_budget = c->mg_budget;
    h.mg_fresh = c->mg_fresh;
    h.mg_restart = c->mg_restart;
    h.qscale = c->qscale;
    h.jscale = c->jscale;
    const std::vector<Seg> segs = state_segments(*c, h.count);
    size_t total = sizeof h;
    for (const Seg &s : segs) total += s.n;
    h.total = total;
    *bytes = total;
    if (!buf) return PIC_OK;
    if (cap < total) return fail(c, PIC_ENOMEM, "checkpoint needs %zu bytes, buffer has %zu", total, cap);
    char *o = static_cast<char *>(buf);
    std::memcpy(o, &h, sizeof h);
    o += sizeof h;
    for (const Seg &s : segs) {
        if (s.n) HIPCHK(c, hipMemcpyAsync(o, s.p, s.n, hipMemcpyDeviceToHost, c->stream));
        o += s.n;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

extern "C" pic_status pic_restore(pic_ctx *c, const void *buf, size_t bytes)
{
    if (!c || !buf) return PIC_EINVAL;
    CkptHead h;
    if (bytes < sizeof h) return fail(c, PIC_EINVAL, "checkpoint too short");
    std::memcpy(&h, buf, sizeof h);
    if (h.magic != CKPT_MAGIC) return fail(c, PIC_EINVAL, "not a checkpoint of this library");
    if (h.total != bytes) return fail(c, PIC_EINVAL, "checkpoint of %llu bytes given %zu", (unsigned long long)h.total, bytes);
    const pic_config &f = c->cfg;
    if (h.precision != f.precision || h.nr != f.nr || h.nz != f.nz || h.nturns != f.nturns || h.circuit != f.circuit ||
        h.nrf != c->nrf || h.norders != c->M || h.qscale != c->qscale || h.jscale != c->jscale)
        return fail(c, PIC_EINVAL, "checkpoint taken with another configuration");
    for (int s = 0; s < 2; ++s)
        if (h.count[s] > f.capacity[s]) return fail(c, PIC_ENOMEM, "checkpoint holds %lld slots of species %d, capacity %lld",
                                                    (long long)h.count[s], s, (long long)f.capacity[s]);
    pic_status st = sticky(c);
    if (st) return st;
    const std::vector<Seg> segs = state_segments(*c, h.count);
    size_t total = sizeof h;
    for (const Seg &s : segs) total += s.n;
    if (total != bytes) return fail(c, PIC_EINVAL, "checkpoint layout does not match this context");
    const char *in = static_cast<const char *>(buf) + sizeof h;
    for (const Seg &s : segs) {
        if (s.n) HIPCHK(c, hipMemcpyAsync(s.p, in, s.n, hipMemcpyHostToDevice, c->stream));
        in += s.n;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->last_push = h.last_push;
    c->last_harm = h.last_harm;
    c->last_mcc = h.last_mcc;
    c->last_solve = h.last_solve;
    c->run = h.run;
    c->mg_budget = h.mg_budget;
    c->mg_fresh = std::max(h.mg_fresh, 1);
    c->di_full = 4;   // the ring does not travel with the checkpoint
    c->mg_restart = h.mg_restart != 0;
    // host mirrors of what the device arrays now hold
    const size_t M = c->M;
    HIPCHK(c, cpy(c->stream, c->vc.data(), c->d_vc, M * MAX_TURNS * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(c, cpy(c->stream, c->vs.data(), c->d_vs, M * MAX_TURNS * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(c, cpy(c->stream, c->ec.data(), c->d_ec, M * c->g.nodes * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(c, cpy(c->stream, c->es.data(), c->d_es, M * c->g.nodes * sizeof(double), hipMemcpyDeviceToHost));
    if (f.circuit) {
        // the surrogate settings belong to the attachment, not the state
        const int32_t mi = c->cdh.sur_max_iter;
        const double em = c->cdh.sur_err_max, tl = c->cdh.sur_tol;
        HIPCHK(c, cpy(c->stream, &c->cdh, c->cd, sizeof(CircuitDev), hipMemcpyDeviceToHost));
        c->cdh.sur_max_iter = mi;
        c->cdh.sur_err_max = em;
        c->cdh.sur_tol = tl;
        char *d = reinterpret_cast<char *>(c->cd);
        HIPCHK(c, cpy(c->stream, d + offsetof(CircuitDev, sur_max_iter), &mi, 4, hipMemcpyHostToDevice));
        HIPCHK(c, cpy(c->stream, d + offsetof(CircuitDev, sur_err_max), &em, 8, hipMemcpyHostToDevice));
        HIPCHK(c, cpy(c->stream, d + offsetof(CircuitDev, sur_tol), &tl, 8, hipMemcpyHostToDevice));
    }
    return PIC_OK;
}

extern "C" pic_status pic_get_circuit(pic_ctx *c, pic_circuit_info *o)
{
    if (!c || !o) return PIC_EINVAL;
    if (!c->cfg.circuit) return fail(c, PIC_EINVAL, "context without circuit coupling");
    HIPCHK(c, cpy(c->stream, &c->cdh, c->cd, sizeof(CircuitDev), hipMemcpyDeviceToHost));
    const CircuitDev &h = c->cdh;
    std::memset(o, 0, sizeof *o);
    const int K = c->cfg.nturns;
    o->nturns = K;
    o->omega = h.omega;
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < K; ++l) o->zvac_im[k * 16 + l] = -h.mvac[k * MAX_TURNS + l];
    o->eps_rec = h.eps_rec;
    std::vector<double> g(MAX_TURNS);
    HIPCHK(c, cpy(c->stream, g.data(), c->gval, MAX_TURNS * 8, hipMemcpyDeviceToHost));
    for (int k = 0; k < K; ++k) {
        o->r_rf[k] = h.rrf[k];
        o->g[k] = g[k];
        o->area[k] = c->area[k];
    }
    o->zs_re = h.zs_re;
    o->zs_im = h.zs_im;
    o->vg_amp = h.vg_amp;
    o->vg_phase = h.vg_phase;
    for (int r = 0; r < 2 * K + 1; ++r) {
        o->x_re[r] = h.x_re[r];
        o->x_im[r] = h.x_im[r];
    }
    return PIC_OK;
}

extern "C" pic_status pic_sync(pic_ctx *c)
{
    if (!c) return PIC_EINVAL;
    return sticky(c);
}

extern "C" pic_status pic_clear_error(pic_ctx *c)
{
    if (!c) return PIC_EINVAL;
    HIPCHK(c, hipMemsetAsync(c->errw, 0, sizeof(int32_t), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->err.clear();
    return PIC_OK;
}

template <typename T>
static pic_status get_parts(pic_ctx *c, int s, int64_t cap, double *R, double *z, double *vr, double *vt, double *vz,
                            uint32_t *id, int32_t *next, int64_t *count)
{
    hipStream_t st = c->stream;
    const Parts<T> &p = parts<T>(*c, s, c->cur[s]);
    launch_live_index(p.cell, c->ctl + s, c->live_index, c->ctl + 6, st);
    int64_t slots = 0, nlive = 0;
    HIPCHK(c, hipMemcpyAsync(&slots, c->ctl + s, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(&nlive, c->ctl + 6, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (count) *count = nlive;
    if (nlive > cap) return fail(c, PIC_ENOMEM, "%lld live particles > cap %lld", (long long)nlive, (long long)cap);
    // chunks of slots whose live particles fit the staging area
    int64_t k0 = 0;
    std::vector<int64_t> idx(2);
    while (k0 < slots) {
        const int64_t k1 = std::min(slots, k0 + c->stage_cap);
        int64_t lo = 0, hi = 0;
        HIPCHK(c, cpy(c->stream, &lo, c->live_index + k0, 8, hipMemcpyDeviceToHost));
        if (k1 < slots)
            HIPCHK(c, cpy(c->stream, &hi, c->live_index + k1, 8, hipMemcpyDeviceToHost));
        else
            hi = nlive;
        const int64_t m = hi - lo;
        // shift the index so this chunk writes at 0 .. m
        double *sR = c->stage, *sz = sR + c->stage_cap, *svr = sz + c->stage_cap, *svt = svr + c->stage_cap,
               *svz = svt + c->stage_cap;
        uint32_t *sid = reinterpret_cast<uint32_t *>(svz + c->stage_cap);
        int32_t *snx = reinterpret_cast<int32_t *>(sid + c->stage_cap);
        Parts<T> q = p;
        q.cell += k0;
        q.dr += k0;
        q.dz += k0;
        q.vr += k0;
        q.vt += k0;
        q.vz += k0;
        q.id += k0;
        q.next += k0;
        // temporary count = chunk length in ctl[7]
        const int64_t len = k1 - k0;
        HIPCHK(c, cpy(c->stream, c->ctl + 7, &len, 8, hipMemcpyHostToDevice));
        // rebased index: live_index[k0 + k] - lo
        std::vector<int64_t> li(len);
        HIPCHK(c, cpy(c->stream, li.data(), c->live_index + k0, len * 8, hipMemcpyDeviceToHost));
        for (auto &v : li) v -= lo;
        HIPCHK(c, cpy(c->stream, c->live_index + k0, li.data(), len * 8, hipMemcpyHostToDevice));
        launch_unplace<T>(q, c->ctl + 7, len, c->live_index + k0, sR, sz, svr, svt, svz, sid, snx, c->g, st);
        HIPCHK(c, hipStreamSynchronize(st));
        if (m > 0) {
            if (R) HIPCHK(c, cpy(c->stream, R + lo, sR, m * 8, hipMemcpyDeviceToHost));
            if (z) HIPCHK(c, cpy(c->stream, z + lo, sz, m * 8, hipMemcpyDeviceToHost));
            if (vr) HIPCHK(c, cpy(c->stream, vr + lo, svr, m * 8, hipMemcpyDeviceToHost));
            if (vt) HIPCHK(c, cpy(c->stream, vt + lo, svt, m * 8, hipMemcpyDeviceToHost));
            if (vz) HIPCHK(c, cpy(c->stream, vz + lo, svz, m * 8, hipMemcpyDeviceToHost));
            if (id) HIPCHK(c, cpy(c->stream, id + lo, sid, m * 4, hipMemcpyDeviceToHost));
            if (next) HIPCHK(c, cpy(c->stream, next + lo, snx, m * 4, hipMemcpyDeviceToHost));
        }
        k0 = k1;
    }
    return PIC_OK;
}

extern "C" pic_status pic_get_particles(pic_ctx *c, int32_t s, int64_t cap, double *R, double *z, double *vr,
                                        double *vt, double *vz, uint32_t *id, int32_t *next, int64_t *count)
{
    if (!c || s < 0 || s > 1) return PIC_EINVAL;
    pic_status st = sticky(c);
    if (st) return st;
    return c->mixed ? get_parts<float>(c, s, cap, R, z, vr, vt, vz, id, next, count)
                    : get_parts<double>(c, s, cap, R, z, vr, vt, vz, id, next, count);
}

template <typename T>
static pic_status set_parts(pic_ctx *c, int s, int64_t n, const double *R, const double *z, const double *vr,
                            const double *vt, const double *vz, const uint32_t *id, const int32_t *next)
{
    hipStream_t st = c->stream;
    Parts<T> p = parts<T>(*c, s, c->cur[s]);
    uint32_t maxid = 0;
    for (int64_t k = 0; k < n; ++k) maxid = std::max(maxid, id[k]);
    for (int64_t k0 = 0; k0 < n; k0 += c->stage_cap) {
        const int64_t m = std::min(c->stage_cap, n - k0);
        double *sR = c->stage, *sz = sR + c->stage_cap, *svr = sz + c->stage_cap, *svt = svr + c->stage_cap,
               *svz = svt + c->stage_cap;
        uint32_t *sid = reinterpret_cast<uint32_t *>(svz + c->stage_cap);
        int32_t *snx = reinterpret_cast<int32_t *>(sid + c->stage_cap);
        HIPCHK(c, cpy(c->stream, sR, R + k0, m * 8, hipMemcpyHostToDevice));
        HIPCHK(c, cpy(c->stream, sz, z + k0, m * 8, hipMemcpyHostToDevice));
        HIPCHK(c, cpy(c->stream, svr, vr + k0, m * 8, hipMemcpyHostToDevice));
        HIPCHK(c, cpy(c->stream, svt, vt + k0, m * 8, hipMemcpyHostToDevice));
        HIPCHK(c, cpy(c->stream, svz, vz + k0, m * 8, hipMemcpyHostToDevice));
        HIPCHK(c, cpy(c->stream, sid, id + k0, m * 4, hipMemcpyHostToDevice));
        HIPCHK(c, cpy(c->stream, snx, next + k0, m * 4, hipMemcpyHostToDevice));
        Parts<T> q = p;
        q.cell += k0;
        q.dr += k0;
        q.dz += k0;
        q.vr += k0;
        q.vt += k0;
        q.vz += k0;
        q.id += k0;
        q.next += k0;
        launch_place<T>(q, m, sR, sz, svr, svt, svz, sid, snx, c->g, st);
        HIPCHK(c, hipStreamSynchronize(st));
    }
    int64_t h[2];
    HIPCHK(c, cpy(c->stream, h, c->ctl + 4, 16, hipMemcpyDeviceToHost));
    h[s] = std::max<int64_t>(h[s], (int64_t)maxid + 1);
    HIPCHK(c, cpy(c->stream, c->ctl + 4, h, 16, hipMemcpyHostToDevice));
    HIPCHK(c, cpy(c->stream, c->ctl + s, &n, 8, hipMemcpyHostToDevice));
    sort_species<T>(*c, s);
    HIPCHK(c, hipStreamSynchronize(st));
    return PIC_OK;
}

extern "C" pic_status pic_set_particles(pic_ctx *c, int32_t s, int64_t n, const double *R, const double *z,
                                        const double *vr, const double *vt, const double *vz, const uint32_t *id,
                                        const int32_t *next)
{
    if (!c || s < 0 || s > 1 || n < 0) return PIC_EINVAL;
    if (n > c->cfg.capacity[s]) return fail(c, PIC_ENOMEM, "n > capacity");
    if (n > 0 && (!R || !z || !vr || !vt || !vz || !id || !next)) return fail(c, PIC_EINVAL, "null array");
    const double zp = c->g.ip * c->g.dz, rmax = c->cfg.rmax;
    for (int64_t k = 0; k < n; ++k)
        if (!(R[k] >= 0 && R[k] < rmax && z[k] >= 0 && z[k] < zp))
            return fail(c, PIC_EINVAL, "particle %lld outside the particle region", (long long)k);
    return c->mixed ? set_parts<float>(c, s, n, R, z, vr, vt, vz, id, next)
                    : set_parts<double>(c, s, n, R, z, vr, vt, vz, id, next);
}

extern "C" pic_status pic_set_step(pic_ctx *c, int64_t n)
{
    if (!c || n < 0) return PIC_EINVAL;
    c->last_push = n - 1;
    c->last_mcc = n - 1;
    c->last_harm = n - 1;
    return PIC_OK;
}

extern "C" pic_status pic_set_phi(pic_ctx *c, const double *phi)
{
    if (!c || !phi) return PIC_EINVAL;
    c->run = 0;
    HIPCHK(c, hipMemcpyAsync(c->phi, phi, c->g.nodes * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

template <typename T> static void bfield_component(pic_ctx *c, int comp, double *out)
{
    std::vector<typename Field2<T>::type> f(c->g.nodes);
    (void)cpy(c->stream, f.data(), c->eb, f.size() * sizeof(f[0]), hipMemcpyDeviceToHost);
    for (int n = 0; n < c->g.nodes; ++n) out[n] = comp == 0 ? (double)f[n].x : (double)f[n].y;
}

template <typename T> static void field_component(pic_ctx *c, int comp, double *out)
{
    std::vector<typename Field4<T>::type> f(c->g.nodes);
    (void)cpy(c->stream, f.data(), c->ef, f.size() * sizeof(f[0]), hipMemcpyDeviceToHost);
    for (int n = 0; n < c->g.nodes; ++n) out[n] = comp == 0 ? (double)f[n].x : comp == 1 ? (double)f[n].y : (double)f[n].z;
}

extern "C" pic_status pic_get_grid(pic_ctx *c, int32_t which, double *out)
{
    if (!c || !out) return PIC_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int nodes = c->g.nodes;
    switch (which) {
    case PIC_GRID_PHI: HIPCHK(c, cpy(c->stream, out, c->phi, nodes * 8, hipMemcpyDeviceToHost)); break;
    case PIC_GRID_CHARGE: HIPCHK(c, cpy(c->stream, out, c->Q, nodes * 8, hipMemcpyDeviceToHost)); break;
    case PIC_GRID_CURRENT: HIPCHK(c, cpy(c->stream, out, c->I, nodes * 8, hipMemcpyDeviceToHost)); break;
    case PIC_GRID_ER:
    case PIC_GRID_EZ:
    case PIC_GRID_ETHETA:
        if (c->mixed)
            field_component<float>(c, which - PIC_GRID_ER, out);
        else
            field_component<double>(c, which - PIC_GRID_ER, out);
        break;
    case PIC_GRID_CHI:
        if (!c->chi) return fail(c, PIC_EINVAL, "the configuration has no direct-implicit update");
        HIPCHK(c, cpy(c->stream, out, c->chi, nodes * 8, hipMemcpyDeviceToHost));
        break;
    case PIC_GRID_BR:
    case PIC_GRID_BZ:
        if (!c->eb) return fail(c, PIC_EINVAL, "the configuration has no RF magnetic field");
        if (c->mixed)
            bfield_component<float>(c, which - PIC_GRID_BR, out);
        else
            bfield_component<double>(c, which - PIC_GRID_BR, out);
        break;
    case PIC_GRID_SURFACE: {
        std::vector<double> a(2 * (size_t)nodes);
        HIPCHK(c, cpy(c->stream, a.data(), c->accS, a.size() * 8, hipMemcpyDeviceToHost));
        const pic_config &f = c->cfg;
        for (int n = 0; n < nodes; ++n) out[n] = f.q[0] * f.w[0] * a[n] + f.q[1] * f.w[1] * a[nodes + n];
        break;
    }
    case PIC_GRID_JC:
    case PIC_GRID_JS: {
        std::vector<double> a(nodes), b(nodes);
        HIPCHK(c, cpy(c->stream, a.data(), which == PIC_GRID_JC ? c->Jc : c->Js, nodes * 8, hipMemcpyDeviceToHost));
        HIPCHK(c, cpy(c->stream, b.data(), which == PIC_GRID_JC ? c->Jcc : c->Jsc, nodes * 8, hipMemcpyDeviceToHost));
        for (int n = 0; n < nodes; ++n) out[n] = a[n] + b[n];
        break;
    }
    case PIC_GRID_EC: HIPCHK(c, cpy(c->stream, out, c->d_ec, nodes * 8, hipMemcpyDeviceToHost)); break;
    case PIC_GRID_ES: HIPCHK(c, cpy(c->stream, out, c->d_es, nodes * 8, hipMemcpyDeviceToHost)); break;
    case PIC_GRID_EC_PLASMA:
    case PIC_GRID_ES_PLASMA:
        if (!c->cfg.circuit) return fail(c, PIC_EINVAL, "context without circuit coupling");
        HIPCHK(c, cpy(c->stream, out, c->Ep + (which == PIC_GRID_ES_PLASMA ? nodes : 0), nodes * 8,
                      hipMemcpyDeviceToHost));
        break;
    default:
        if (which >= PIC_GRID_UNIT && which < PIC_GRID_UNIT + c->cfg.nturns && c->cfg.circuit) {
            HIPCHK(c, cpy(c->stream, out, c->U + (size_t)(which - PIC_GRID_UNIT) * nodes, nodes * 8,
                          hipMemcpyDeviceToHost));
            break;
        }
        return fail(c, PIC_EINVAL, "unknown grid %d", which);
    }
    return PIC_OK;
}

extern "C" pic_status pic_timing(pic_ctx *c, int32_t enable)
{
    if (!c) return PIC_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto *t : {&c->t_pass, &c->t_poisson, &c->t_sort, &c->t_circuit}) {
        timer_drain(*t);
        t->ms = 0.0;
        t->count = 0;
    }
    c->timing = enable != 0;
    return PIC_OK;
}

extern "C" pic_status pic_get_stats(pic_ctx *c, pic_stats *o)
{
    if (!c || !o) return PIC_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::memset(o, 0, sizeof *o);
    for (auto *t : {&c->t_pass, &c->t_poisson, &c->t_sort, &c->t_circuit}) timer_drain(*t);
    o->pass_ms = c->t_pass.ms;
    o->pass_count = c->t_pass.count;
    o->poisson_ms = c->t_poisson.ms;
    o->poisson_count = c->t_poisson.count;
    o->sort_ms = c->t_sort.ms;
    o->sort_count = c->t_sort.count;
    o->circuit_ms = c->t_circuit.ms;
    o->circuit_count = c->t_circuit.count;
    {
        MGState ms;
        HIPCHK(c, cpy(c->stream, &ms, c->mgs, sizeof ms, hipMemcpyDeviceToHost));
        o->mg_cycles = ms.cycles;
        o->mg_rel = ms.rel;
    }
    int64_t ctl[8];
    unsigned long long st[ST_NSTAT];
    HIPCHK(c, cpy(c->stream, ctl, c->ctl, sizeof ctl, hipMemcpyDeviceToHost));
    HIPCHK(c, cpy(c->stream, st, c->stats, sizeof st, hipMemcpyDeviceToHost));
    for (int s = 0; s < 2; ++s) {
        o->slots[s] = ctl[s];
        o->next_id[s] = ctl[4 + s];
        const int32_t *cell = c->mixed ? c->pf[s][c->cur[s]].cell : c->pd[s][c->cur[s]].cell;
        HIPCHK(c, hipMemsetAsync(c->ctl + 6, 0, 8, c->stream));
        launch_count_live(cell, c->ctl + s, reinterpret_cast<unsigned long long *>(c->ctl + 6), c->stream);
        int64_t nl = 0;
        HIPCHK(c, hipMemcpyAsync(&nl, c->ctl + 6, 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        o->live[s] = nl;
        o->candidates[s] = (int64_t)st[ST_CAND0 + s];
        o->absorbed[s] = (int64_t)st[ST_ABS0 + s];
        o->over_numax[s] = (int64_t)st[ST_OVER0 + s];
        o->numax[s] = c->numax[s];
        o->pnull[s] = c->pnull[s];
    }
    o->events[0][0] = (int64_t)st[ST_EV00];
    o->events[0][1] = (int64_t)st[ST_EV01];
    o->events[0][2] = (int64_t)st[ST_EV02];
    o->events[1][0] = (int64_t)st[ST_EV10];
    o->events[1][1] = (int64_t)st[ST_EV11];
    o->births = (int64_t)st[ST_BIRTHS];
    o->window_out = (int64_t)st[ST_WINOUT];
    o->mg_unconverged = (int64_t)st[ST_MGUNCONV];
    o->see_emitted = (int64_t)st[ST_SEE];
    HarmState h;
    HIPCHK(c, cpy(c->stream, &h, c->harm, sizeof h, hipMemcpyDeviceToHost));
    o->samples = h.samples;
    o->nrf = c->nrf;
    o->phase_closed = c->closed ? 1 : 0;
    o->pind_sum = h.pind + h.pind_c;
    double qk[MAX_TURNS];
    HIPCHK(c, cpy(c->stream, qk, c->Qk, sizeof qk, hipMemcpyDeviceToHost));
    for (int k = 0; k < MAX_TURNS; ++k) {
        o->qc[k] = h.qc[k] + h.qc_c[k];
        o->qs[k] = h.qs[k] + h.qs_c[k];
        o->wk[k] = h.w[k] + h.w_c[k];
        o->qk[k] = qk[k];
    }
    return PIC_OK;
}

extern "C" void pic_destroy(pic_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto *t : {&c->t_pass, &c->t_poisson, &c->t_sort, &c->t_circuit})
        for (auto &e : t->ev)
            for (auto &x : e)
                if (x) (void)hipEventDestroy(x);
    if (c->mg_host) (void)hipHostFree(c->mg_host);
    delete c;
}

extern "C" const char *pic_last_error(const pic_ctx *c)
{
    if (c) return c->err.c_str();
    return init_error.empty() ? "null context" : init_error.c_str();
}
