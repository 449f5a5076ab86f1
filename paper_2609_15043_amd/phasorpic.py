"""ctypes binding of libphasorpic (include/phasorpic.h): argument marshalling
only.  Every step of the method runs in the library's HIP kernels; this
module fails loudly when the library is missing.  PyTorch provides the
device workspace and the stream.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphasorpic.so")

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EDEVICE, PIC_ENOTCONV, PIC_EPHASE, PIC_ESTATE = 0, -1, -2, -3, -4, -5, -6
PIC_FP64, PIC_MIXED = 0, 1
PIC_OP_POISSON, PIC_OP_HELMHOLTZ_C, PIC_OP_HELMHOLTZ_S = 0, 1, 2
PIC_POISSON_AUTO, PIC_POISSON_MULTIGRID, PIC_POISSON_DIRECT = 0, 1, 2
PIC_FIELD_FULL, PIC_FIELD_MQS = 0, 1
PIC_RRF_GIVEN, PIC_RRF_SKIN = 0, 1
(PIC_GRID_PHI, PIC_GRID_CHARGE, PIC_GRID_CURRENT, PIC_GRID_ER, PIC_GRID_EZ, PIC_GRID_ETHETA,
 PIC_GRID_SURFACE, PIC_GRID_JC, PIC_GRID_JS, PIC_GRID_EC, PIC_GRID_ES, PIC_GRID_EC_PLASMA,
 PIC_GRID_ES_PLASMA, PIC_GRID_BR, PIC_GRID_BZ, PIC_GRID_CHI) = range(16)
PIC_GRID_UNIT = 16

_D, _I32, _I64, _U32 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
_PD, _PI32, _PU32 = ctypes.POINTER(_D), ctypes.POINTER(_I32), ctypes.POINTER(_U32)


class PicConfig(ctypes.Structure):
    _fields_ = [
        ("nr", _I32), ("nz", _I32), ("ip", _I32), ("window", _I32),
        ("rmax", _D), ("zmax", _D), ("dt", _D), ("freq", _D),
        ("precision", _I32), ("seed", _U32),
        ("q", _D * 2), ("m", _D * 2), ("w", _D * 2), ("temp_ev", _D * 2),
        ("np_init", _I64 * 2), ("capacity", _I64 * 2), ("bfield", _D * 3),
        ("ngas", _D), ("tgas_ev", _D), ("qe", _D), ("eps0", _D),
        ("xs_kind", _I32), ("nscan", _I32), ("xs", _D * 13),
        ("nturns", _I32), ("fuse", _I32),
        ("eps_cell", _PD), ("node_tag", _PI32), ("ec", _PD), ("es_sto", _PD),
        ("turn_vc", _PD), ("turn_vs", _PD),
        ("mg_rtol", _D), ("mg_max_cycles", _I32), ("sort_every", _I32), ("load", _I32),
        ("birth_capacity", _I32),
        ("circuit", _I32), ("field_mode", _I32), ("mu0", _D), ("turn_sign", _PD),
        ("r_g", _D), ("r_m", _D), ("l_m", _D), ("c_m", _D), ("c_stray", _PD),
        ("rrf_mode", _I32), ("r_rf", _PD), ("rho20", _D), ("alpha_cu", _D), ("temp_c", _D),
        ("vg_amp", _D), ("vg_phase", _D), ("vg_from_target", _I32), ("controller", _I32),
        ("p_target", _D), ("gamma", _D), ("n_trend", _D), ("eps_p", _D), ("alpha_v", _D), ("f_step", _D),
        ("v_min", _D), ("v_max", _D), ("alpha", _D), ("helm_rtol", _D), ("helm_max_cycles", _I32),
        ("sort_every_ion", _I32), ("dir_basis", _PD), ("unit_bvals", _PD), ("rf_bfield", _I32),
        ("implicit", _I32), ("poisson_solver", _I32),
        ("nharm", _I32), ("harm_ratio", _D * 3), ("harm_phase", _D * 3),
        ("see_gamma", _D), ("see_temp_ev", _D),
    ]


class PicSolveInfo(ctypes.Structure):
    _fields_ = [("cycles", _I32), ("converged", _I32), ("rel_residual", _D)]


class PicStats(ctypes.Structure):
    _fields_ = [
        ("slots", _I64 * 2), ("live", _I64 * 2), ("next_id", _I64 * 2), ("candidates", _I64 * 2),
        ("events", (_I64 * 3) * 2), ("births", _I64), ("absorbed", _I64 * 2), ("over_numax", _I64 * 2),
        ("window_out", _I64), ("samples", _I64), ("nrf", _I32), ("phase_closed", _I32),
        ("numax", _D * 2), ("pnull", _D * 2), ("pind_sum", _D),
        ("qc", _D * 16), ("qs", _D * 16), ("wk", _D * 16), ("qk", _D * 16),
        ("pass_ms", _D), ("pass_count", _I64), ("poisson_ms", _D), ("poisson_count", _I64),
        ("sort_ms", _D), ("sort_count", _I64), ("circuit_ms", _D), ("circuit_count", _I64),
        ("mg_cycles", _I64), ("mg_rel", _D), ("mg_unconverged", _I64), ("see_emitted", _I64),
    ]


class PicPeriodReport(ctypes.Structure):
    _fields_ = [("accepted", _I32), ("samples", _I32), ("p_ind", _D), ("p_cap", _D), ("p_cap_ph", _D),
                ("qc", _D * 16), ("qs", _D * 16), ("icap_re", _D * 16), ("icap_im", _D * 16),
                ("p_port", _D), ("p_cu", _D), ("eps_bal", _D), ("kcl", _D), ("kvl", _D),
                ("vg_old", _D), ("vg_amp", _D), ("pf", _D), ("pc", _D),
                ("vp_re", _D * 16), ("vp_im", _D * 16), ("xt_re", _D * 33), ("xt_im", _D * 33),
                ("x_re", _D * 33), ("x_im", _D * 33), ("helm_cycles", _I32 * 2), ("helm_rel", _D * 2),
                ("xp_re", _D * 33), ("xp_im", _D * 33), ("pressure", _D), ("moments", _D * 8),
                ("sur_used", _I32), ("sur_iters", _I32), ("sur_err", _D), ("sur_steps", _D * 64),
                ("vg_phase", _D)]


class PicSurrogateConfig(ctypes.Structure):
    _fields_ = [("err_max", _D), ("tol", _D), ("max_iter", _I32)]


class PicCircuitOverride(ctypes.Structure):
    _fields_ = [("new_vc", _PD), ("new_vs", _PD), ("new_ec", _PD), ("new_es_sto", _PD), ("loads", _I32),
                ("vp_re", _D * 16), ("vp_im", _D * 16), ("icap_re", _D * 16), ("icap_im", _D * 16)]


class PicCircuitInfo(ctypes.Structure):
    _fields_ = [("nturns", _I32), ("omega", _D), ("zvac_im", _D * 256), ("eps_rec", _D), ("r_rf", _D * 16),
                ("zs_re", _D), ("zs_im", _D), ("g", _D * 16), ("area", _D * 16), ("vg_amp", _D),
                ("vg_phase", _D), ("x_re", _D * 33), ("x_im", _D * 33)]


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"phasorpic status {status}: {msg}")
        self.status = status


_LIB = None

# exported C symbols, in header order
SYMBOLS = ["pic_workspace_bytes", "pic_init", "pic_gather_push", "mcc_collide", "pic_deposit",
           "poisson_solve_rz", "harmonic_accumulate", "circuit_period_update", "circuit_order_report",
           "pic_set_source",
           "pic_attach_surrogate",
           "pic_get_circuit", "pic_sync",
           "pic_clear_error", "pic_get_particles", "pic_set_particles", "pic_set_step", "pic_set_phi",
           "pic_checkpoint", "pic_restore",
           "pic_get_grid", "pic_timing", "pic_get_stats", "pic_destroy", "pic_last_error"]


def lib():
    """Load libphasorpic.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: build it with paper_2609_15043_amd/build.py "
                               "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.pic_workspace_bytes.argtypes = [ctypes.POINTER(PicConfig), ctypes.POINTER(ctypes.c_size_t)]
        L.pic_init.argtypes = [ctypes.POINTER(PicConfig), P, ctypes.c_size_t, P, ctypes.POINTER(P)]
        for name in ("pic_gather_push", "mcc_collide", "pic_deposit", "harmonic_accumulate", "pic_set_step"):
            getattr(L, name).argtypes = [P, _I64]
        L.poisson_solve_rz.argtypes = [P, _I64, _I32, _D, _I32, ctypes.POINTER(PicSolveInfo)]
        L.circuit_period_update.argtypes = [P, ctypes.POINTER(PicCircuitOverride), ctypes.POINTER(PicPeriodReport),
                                            _PD, _PD]
        L.circuit_order_report.argtypes = [P, _I32, ctypes.POINTER(PicPeriodReport)]
        L.pic_get_circuit.argtypes = [P, ctypes.POINTER(PicCircuitInfo)]
        L.pic_attach_surrogate.argtypes = [P, P, ctypes.POINTER(PicSurrogateConfig)]
        L.pic_set_source.argtypes = [P, _D, _D]
        L.pic_sync.argtypes = [P]
        L.pic_clear_error.argtypes = [P]
        L.pic_get_particles.argtypes = [P, _I32, _I64, _PD, _PD, _PD, _PD, _PD, _PU32, _PI32,
                                        ctypes.POINTER(_I64)]
        L.pic_set_particles.argtypes = [P, _I32, _I64, _PD, _PD, _PD, _PD, _PD, _PU32, _PI32]
        L.pic_set_phi.argtypes = [P, _PD]
        L.pic_checkpoint.argtypes = [P, ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        L.pic_restore.argtypes = [P, ctypes.c_void_p, ctypes.c_size_t]
        L.pic_get_grid.argtypes = [P, _I32, _PD]
        L.pic_get_stats.argtypes = [P, ctypes.POINTER(PicStats)]
        L.pic_timing.argtypes = [P, _I32]
        L.pic_destroy.argtypes = [P]
        L.pic_destroy.restype = None
        L.pic_last_error.argtypes = [P]
        L.pic_last_error.restype = ctypes.c_char_p
        for name in SYMBOLS:
            if name not in ("pic_destroy", "pic_last_error"):
                getattr(L, name).restype = _I32
        _LIB = L
    return _LIB


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t)) if a is not None else None


# ---------------------------------------------------------------------------
# Configuration from a workload description
# ---------------------------------------------------------------------------
def config_from_workload(wl, precision="mixed", fuse=True, load=True, mg_rtol=None, mg_max_cycles=30,
                         sort_every=16, sort_every_ion=0, birth_capacity=65536, nscan=200_000, helm_rtol=1e-12,
                         helm_max_cycles=60, poisson_solver="auto"):
    """(PicConfig, keep-alive list).  precision: 'fp64' or 'mixed'.  A
    workload with a ``circuit`` couples its turns to the external network.
    poisson_solver: 'auto', 'multigrid' or 'direct' (PIC_POISSON_*)."""
    keep = []
    c = PicConfig()
    c.nr, c.nz, c.ip, c.window = wl.nr, wl.nz, wl.ip, 1 if wl.window else 0
    c.rmax, c.zmax, c.dt, c.freq = wl.rmax, wl.zmax, wl.dt, wl.freq
    c.precision = PIC_MIXED if precision == "mixed" else PIC_FP64
    c.seed = wl.seed
    for s in range(2):
        c.q[s], c.m[s], c.w[s], c.temp_ev[s] = wl.charge[s], wl.mass[s], wl.weight[s], wl.temp_ev[s]
        c.np_init[s] = wl.np_init[s]
        c.capacity[s] = wl.capacity[s]
    for k in range(3):
        c.bfield[k] = wl.bfield[k]
    c.ngas, c.tgas_ev, c.qe, c.eps0 = wl.ngas, wl.tgas_ev, W.QE, wl.eps0
    x = wl.xs
    c.xs_kind, c.nscan = x.kind, nscan
    for k, v in enumerate((x.el_a, x.el_b, x.exc_a, x.exc_th, x.iz_a, x.iz_th, x.iel_a, x.iel_p, x.icx_a,
                           x.icx_p, x.e_cap_ev, x.i_gcap, x.nu_margin)):
        c.xs[k] = v
    eps = np.ascontiguousarray(wl.eps_cell, dtype=np.float64)
    tag = np.ascontiguousarray(wl.node_tag, dtype=np.int32)
    ec = np.ascontiguousarray(wl.ec, dtype=np.float64)
    es = np.ascontiguousarray(wl.es_sto, dtype=np.float64)
    vc = np.ascontiguousarray(wl.turn_vc, dtype=np.float64)
    vs = np.ascontiguousarray(wl.turn_vs, dtype=np.float64)
    keep += [eps, tag, ec, es, vc, vs]
    c.nturns, c.fuse = wl.nturns, 1 if fuse else 0
    c.eps_cell, c.node_tag, c.ec, c.es_sto = _ptr(eps, _D), _ptr(tag, _I32), _ptr(ec, _D), _ptr(es, _D)
    c.turn_vc, c.turn_vs = _ptr(vc, _D), _ptr(vs, _D)
    for name in ("dir_basis", "unit_bvals"):
        a = getattr(wl, name)
        if a is not None:
            a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
            assert a.size == wl.nturns * wl.nodes
            keep.append(a)
            setattr(c, name, _ptr(a, _D))
    if mg_rtol is None:
        mg_rtol = 1e-13 if precision == "fp64" else 1e-9
    c.mg_rtol, c.mg_max_cycles, c.sort_every, c.load = mg_rtol, mg_max_cycles, sort_every, 1 if load else 0
    c.sort_every_ion = sort_every_ion
    c.rf_bfield = 1 if wl.rf_bfield else 0
    c.implicit = 1 if wl.implicit else 0
    c.see_gamma, c.see_temp_ev = wl.see_gamma, wl.see_temp_ev
    c.poisson_solver = {"auto": PIC_POISSON_AUTO, "multigrid": PIC_POISSON_MULTIGRID,
                        "direct": PIC_POISSON_DIRECT}[poisson_solver]
    c.birth_capacity = birth_capacity
    cp = wl.circuit
    if cp is not None:
        N = wl.nturns
        sign = np.ascontiguousarray(np.ones(N) if cp.turn_sign is None else cp.turn_sign, dtype=np.float64)
        cst = np.ascontiguousarray(np.zeros(N) if cp.c_stray is None else cp.c_stray, dtype=np.float64)
        rrf = np.ascontiguousarray(np.zeros(N) if cp.r_rf is None else cp.r_rf, dtype=np.float64)
        keep += [sign, cst, rrf]
        c.circuit, c.field_mode, c.mu0 = 1, cp.field_mode, cp.mu0
        c.turn_sign, c.c_stray, c.r_rf = _ptr(sign, _D), _ptr(cst, _D), _ptr(rrf, _D)
        c.r_g, c.r_m, c.l_m, c.c_m = cp.r_g, cp.r_m, cp.l_m, cp.c_m
        c.rrf_mode, c.rho20, c.alpha_cu, c.temp_c = cp.rrf_mode, cp.rho20, cp.alpha_cu, cp.temp_c
        c.vg_amp, c.vg_phase, c.vg_from_target = cp.vg_amp, cp.vg_phase, 1 if cp.vg_from_target else 0
        c.controller = 1 if cp.controller else 0
        c.p_target, c.gamma, c.n_trend, c.eps_p = cp.p_target, cp.gamma, cp.n_trend, cp.eps_p
        c.alpha_v, c.f_step, c.v_min, c.v_max = cp.alpha_v, cp.f_step, cp.v_min, cp.v_max
        c.alpha = cp.alpha
        c.helm_rtol, c.helm_max_cycles = helm_rtol, helm_max_cycles
        # orders above the fundamental of a multiharmonic circuit: (ratio, phase) each
        c.nharm = len(cp.harmonics)
        for q, (a, ph) in enumerate(cp.harmonics):
            c.harm_ratio[q], c.harm_phase[q] = a, ph
    return c, keep


# ---------------------------------------------------------------------------
# The entry points, same names as the C ABI
# ---------------------------------------------------------------------------
class Context:
    """A pic_ctx together with the torch workspace it lives in."""

    def __init__(self, handle, workspace, keep, cfg):
        self.handle = handle
        self.workspace = workspace
        self.keep = keep
        self.cfg = cfg
        self.nodes = (cfg.nz + 1) * (cfg.nr + 1)
        self.shape = (cfg.nz + 1, cfg.nr + 1)

    def check(self, st):
        if st != PIC_OK:
            raise PicError(st, lib().pic_last_error(self.handle).decode())
        return st

    def __del__(self):
        try:
            if self.handle:
                lib().pic_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def pic_workspace_bytes(cfg):
    n = ctypes.c_size_t()
    st = lib().pic_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n))
    if st:
        raise PicError(st, "pic_workspace_bytes: " + lib().pic_last_error(None).decode())
    return n.value


def pic_init(cfg, keep=(), device="cuda", stream=None):
    import torch
    nbytes = pic_workspace_bytes(cfg)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    if stream is None:
        stream = torch.cuda.current_stream(ws.device).cuda_stream
    h = ctypes.c_void_p()
    st = lib().pic_init(ctypes.byref(cfg), ctypes.c_void_p(ws.data_ptr()), nbytes, ctypes.c_void_p(stream),
                        ctypes.byref(h))
    if st:
        raise PicError(st, "pic_init: " + lib().pic_last_error(None).decode())
    return Context(h, ws, list(keep), cfg)


def pic_gather_push(ctx, n):
    return ctx.check(lib().pic_gather_push(ctx.handle, n))


def mcc_collide(ctx, n):
    return ctx.check(lib().mcc_collide(ctx.handle, n))


def pic_deposit(ctx, n1):
    return ctx.check(lib().pic_deposit(ctx.handle, n1))


def poisson_solve_rz(ctx, n, rtol=0.0, max_cycles=0, info=False, op=PIC_OP_POISSON):
    if not info:
        return ctx.check(lib().poisson_solve_rz(ctx.handle, n, op, rtol, max_cycles, None))
    inf = PicSolveInfo()
    st = lib().poisson_solve_rz(ctx.handle, n, op, rtol, max_cycles, ctypes.byref(inf))
    if st not in (PIC_OK, PIC_ENOTCONV):
        ctx.check(st)
    return dict(status=st, cycles=inf.cycles, converged=inf.converged, rel_residual=inf.rel_residual)


def harmonic_accumulate(ctx, n):
    return ctx.check(lib().harmonic_accumulate(ctx.handle, n))


def circuit_period_update(ctx, new_vc=None, new_vs=None, new_ec=None, new_es_sto=None, want_j=False,
                          loads=None):
    """Returns (status, report dict, jc, js).  new_*: the next period's
    turn potentials and field of an uncoupled context; loads = (V_p, I_cap)
    complex arrays prescribed for a coupled context's update."""
    rep = PicPeriodReport()
    arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in
            (new_vc, new_vs, new_ec, new_es_sto)]
    jc = np.zeros(ctx.shape) if want_j else None
    js = np.zeros(ctx.shape) if want_j else None
    ovr = None
    if any(a is not None for a in arrs) or loads is not None:
        ovr = PicCircuitOverride()
        ovr.new_vc, ovr.new_vs, ovr.new_ec, ovr.new_es_sto = (_ptr(a, _D) for a in arrs)
        if loads is not None:
            vp, icap = (np.asarray(a, dtype=complex) for a in loads)
            ovr.loads = 1
            for k in range(len(vp)):
                ovr.vp_re[k], ovr.vp_im[k] = vp[k].real, vp[k].imag
                ovr.icap_re[k], ovr.icap_im[k] = icap[k].real, icap[k].imag
    st = lib().circuit_period_update(ctx.handle, ctypes.byref(ovr) if ovr is not None else None, ctypes.byref(rep),
                                     _ptr(jc, _D), _ptr(js, _D))
    out = _report_dict(ctx, rep)
    if ctx.cfg.circuit and ctx.cfg.nharm > 0 and st == PIC_OK:
        out["orders"] = [circuit_order_report(ctx, m) for m in range(1, ctx.cfg.nharm + 2)]
    return st, out, jc, js


def _report_dict(ctx, rep):
    K = ctx.cfg.nturns
    out = dict(accepted=rep.accepted, samples=rep.samples, p_ind=rep.p_ind, p_cap=rep.p_cap, p_cap_ph=rep.p_cap_ph,
               qc=np.array(rep.qc[:K]), qs=np.array(rep.qs[:K]),
               icap=np.array(rep.icap_re[:K]) + 1j * np.array(rep.icap_im[:K]))
    if ctx.cfg.circuit:
        M = 2 * K + 1
        out.update(p_port=rep.p_port, p_cu=rep.p_cu, eps_bal=rep.eps_bal, kcl=rep.kcl, kvl=rep.kvl,
                   vg_old=rep.vg_old, vg_amp=rep.vg_amp, pf=rep.pf, pc=rep.pc,
                   vg=rep.vg_amp * complex(math.cos(rep.vg_phase), math.sin(rep.vg_phase)),
                   vp=np.array(rep.vp_re[:K]) + 1j * np.array(rep.vp_im[:K]),
                   x_target=np.array(rep.xt_re[:M]) + 1j * np.array(rep.xt_im[:M]),
                   x=np.array(rep.x_re[:M]) + 1j * np.array(rep.x_im[:M]),
                   helm_cycles=tuple(rep.helm_cycles), helm_rel=tuple(rep.helm_rel),
                   x_prev=np.array(rep.xp_re[:M]) + 1j * np.array(rep.xp_im[:M]), pressure=rep.pressure,
                   moments=np.array(rep.moments[:]), sur_used=rep.sur_used, sur_iters=rep.sur_iters,
                   sur_err=rep.sur_err, sur_steps=np.array(rep.sur_steps[:min(rep.sur_iters, 64)]))
    return out


def circuit_order_report(ctx, order):
    """The last update's report fields of retained order `order` (1 = the
    fundamental) of a multiharmonic circuit, as a dict like the period
    report's."""
    rep = PicPeriodReport()
    ctx.check(lib().circuit_order_report(ctx.handle, order, ctypes.byref(rep)))
    return _report_dict(ctx, rep)


def pic_set_source(ctx, vg_amp, vg_phase=0.0):
    return ctx.check(lib().pic_set_source(ctx.handle, vg_amp, vg_phase))


def pic_attach_surrogate(ctx, net, err_max=0.02, tol=1e-6, max_iter=50):
    """Attach an Mlp (or None to detach) to a coupled context."""
    sc = PicSurrogateConfig(err_max, tol, max_iter)
    ctx.check(lib().pic_attach_surrogate(ctx.handle, net.handle if net is not None else None, ctypes.byref(sc)))
    ctx.keep.append(net)


def surrogate_features(rep, N):
    """Network input of a period report: (I_k re, im), (V_k re, im) of the
    state applied during the period, pressure, the eight moments."""
    x = rep["x_prev"]
    f = []
    for k in range(N):
        f += [x[1 + k].real, x[1 + k].imag]
    for k in range(N):
        f += [x[1 + N + k].real, x[1 + N + k].imag]
    return np.array(f + [rep["pressure"]] + list(rep["moments"]))


def surrogate_targets(rep, N):
    """Network output of a period report: (V_p,k re, im), (I_cap,k re, im)."""
    f = []
    for k in range(N):
        f += [rep["vp"][k].real, rep["vp"][k].imag]
    for k in range(N):
        f += [rep["icap"][k].real, rep["icap"][k].imag]
    return np.array(f)


def pic_get_circuit(ctx):
    """Dict with Z_vac (complex K x K), eps_rec, R_rf, Z_source, g, A, V_g and the applied state x."""
    info = PicCircuitInfo()
    ctx.check(lib().pic_get_circuit(ctx.handle, ctypes.byref(info)))
    K = info.nturns
    zim = np.array(info.zvac_im).reshape(16, 16)[:K, :K]
    M = 2 * K + 1
    return dict(omega=info.omega, zvac=1j * zim, eps_rec=info.eps_rec, r_rf=np.array(info.r_rf[:K]),
                zs=complex(info.zs_re, info.zs_im), g=np.array(info.g[:K]), area=np.array(info.area[:K]),
                vg_amp=info.vg_amp, vg_phase=info.vg_phase,
                x=np.array(info.x_re[:M]) + 1j * np.array(info.x_im[:M]))


def pic_sync(ctx):
    return ctx.check(lib().pic_sync(ctx.handle))


def pic_clear_error(ctx):
    return ctx.check(lib().pic_clear_error(ctx.handle))


def pic_set_step(ctx, n):
    return ctx.check(lib().pic_set_step(ctx.handle, n))


def pic_set_phi(ctx, phi):
    a = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
    assert a.size == ctx.nodes
    return ctx.check(lib().pic_set_phi(ctx.handle, _ptr(a, _D)))


def pic_checkpoint(ctx):
    """The context's state at a step boundary as a bytes object."""
    n = ctypes.c_size_t()
    ctx.check(lib().pic_checkpoint(ctx.handle, None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    ctx.check(lib().pic_checkpoint(ctx.handle, buf, n.value, ctypes.byref(n)))
    return buf.raw[:n.value]


def pic_restore(ctx, data):
    buf = ctypes.create_string_buffer(bytes(data), len(data))
    return ctx.check(lib().pic_restore(ctx.handle, buf, len(data)))


def pic_get_grid(ctx, which):
    out = np.zeros(ctx.nodes)
    ctx.check(lib().pic_get_grid(ctx.handle, which, _ptr(out, _D)))
    return out.reshape(ctx.shape)


def pic_timing(ctx, enable=True):
    return ctx.check(lib().pic_timing(ctx.handle, 1 if enable else 0))


def pic_get_stats(ctx):
    s = PicStats()
    ctx.check(lib().pic_get_stats(ctx.handle, ctypes.byref(s)))
    return s


def pic_get_particles(ctx, s):
    """Dict of live particles (R, z, vr, vt, vz, id, next), sorted by id."""
    st = pic_get_stats(ctx)
    cap = int(st.slots[s])
    R, z, vr, vt, vz = (np.zeros(cap) for _ in range(5))
    ids = np.zeros(cap, np.uint32)
    nxt = np.zeros(cap, np.int32)
    cnt = _I64()
    ctx.check(lib().pic_get_particles(ctx.handle, s, cap, _ptr(R, _D), _ptr(z, _D), _ptr(vr, _D), _ptr(vt, _D),
                                      _ptr(vz, _D), _ptr(ids, _U32), _ptr(nxt, _I32), ctypes.byref(cnt)))
    n = cnt.value
    o = np.argsort(ids[:n], kind="stable")
    return dict(id=ids[:n][o], R=R[:n][o], z=z[:n][o], vr=vr[:n][o], vt=vt[:n][o], vz=vz[:n][o], next=nxt[:n][o])


def pic_set_particles(ctx, s, d):
    n = len(d["R"])
    a = {k: np.ascontiguousarray(d[k], dtype=np.float64) for k in ("R", "z", "vr", "vt", "vz")}
    ids = np.ascontiguousarray(d["id"], dtype=np.uint32)
    nxt = np.ascontiguousarray(d["next"], dtype=np.int32)
    return ctx.check(lib().pic_set_particles(ctx.handle, s, n, _ptr(a["R"], _D), _ptr(a["z"], _D),
                                             _ptr(a["vr"], _D), _ptr(a["vt"], _D), _ptr(a["vz"], _D),
                                             _ptr(ids, _U32), _ptr(nxt, _I32)))


def step(ctx, n):
    """One whole PIC step n in the library's order (without the period update)."""
    pic_gather_push(ctx, n)
    harmonic_accumulate(ctx, n)
    if ctx.cfg.implicit:
        pic_deposit(ctx, n + 1)
        poisson_solve_rz(ctx, n + 1)
        mcc_collide(ctx, n)
        return
    mcc_collide(ctx, n)
    pic_deposit(ctx, n + 1)
    poisson_solve_rz(ctx, n + 1)


def nrf(wl):
    return int(round(1.0 / (wl.freq * wl.dt)))


# ---------------------------------------------------------------------------
# Surrogate network (mlp_* calls)
# ---------------------------------------------------------------------------
class MlpConfig(ctypes.Structure):
    _fields_ = [("n_in", _I32), ("n_out", _I32), ("hidden", _I32), ("max_batch", _I32),
                ("lr", _D), ("beta1", _D), ("beta2", _D), ("eps", _D),
                ("in_mean", ctypes.POINTER(ctypes.c_float)), ("in_std", ctypes.POINTER(ctypes.c_float)),
                ("out_mean", ctypes.POINTER(ctypes.c_float)), ("out_std", ctypes.POINTER(ctypes.c_float))]


MLP_SYMBOLS = ["mlp_workspace_bytes", "mlp_init", "mlp_param_count", "mlp_set_params", "mlp_get_params",
               "mlp_forward", "mlp_forward_noalloc", "mlp_train_step", "mlp_get_grads", "mlp_sync", "mlp_destroy",
               "mlp_last_error"]
SYMBOLS += MLP_SYMBOLS

_MLP_BOUND = False
_PF = ctypes.POINTER(ctypes.c_float)


def _mlp_lib():
    global _MLP_BOUND
    L = lib()
    if not _MLP_BOUND:
        P = ctypes.c_void_p
        L.mlp_workspace_bytes.argtypes = [ctypes.POINTER(MlpConfig), ctypes.POINTER(ctypes.c_size_t)]
        L.mlp_init.argtypes = [ctypes.POINTER(MlpConfig), P, ctypes.c_size_t, P, ctypes.POINTER(P)]
        L.mlp_param_count.argtypes = [P, ctypes.POINTER(_I64)]
        L.mlp_set_params.argtypes = [P, _PF]
        L.mlp_get_params.argtypes = [P, _PF]
        L.mlp_get_grads.argtypes = [P, _PF]
        L.mlp_forward.argtypes = [P, P, _I32, P]
        L.mlp_forward_noalloc.argtypes = [P, P, _I32, P]
        L.mlp_train_step.argtypes = [P, P, P, _I32, _PF]
        L.mlp_sync.argtypes = [P]
        L.mlp_destroy.argtypes = [P]
        L.mlp_destroy.restype = None
        L.mlp_last_error.argtypes = [P]
        L.mlp_last_error.restype = ctypes.c_char_p
        for name in MLP_SYMBOLS:
            if name not in ("mlp_destroy", "mlp_last_error"):
                getattr(L, name).restype = _I32
        _MLP_BOUND = True
    return L


class Mlp:
    """An mlp_ctx with its torch workspace.  x, t, y are torch FP32 device
    tensors; parameters move as numpy FP32 vectors."""

    def __init__(self, n_in=W.MLP_IN, n_out=W.MLP_OUT, hidden=W.MLP_HIDDEN, max_batch=4096, lr=1e-3,
                 beta1=0.9, beta2=0.999, eps=1e-8, norm=None, device="cuda"):
        import torch
        L = _mlp_lib()
        c = MlpConfig()
        c.n_in, c.n_out, c.hidden, c.max_batch = n_in, n_out, hidden, max_batch
        c.lr, c.beta1, c.beta2, c.eps = lr, beta1, beta2, eps
        self._keep = []
        if norm is not None:
            arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in norm]
            self._keep += arrs
            c.in_mean, c.in_std, c.out_mean, c.out_std = (a.ctypes.data_as(_PF) for a in arrs)
        n = ctypes.c_size_t()
        st = L.mlp_workspace_bytes(ctypes.byref(c), ctypes.byref(n))
        if st:
            raise PicError(st, "mlp_workspace_bytes: bad configuration")
        self.ws = torch.empty(n.value, dtype=torch.uint8, device=device)
        stream = torch.cuda.current_stream(self.ws.device).cuda_stream
        h = ctypes.c_void_p()
        st = L.mlp_init(ctypes.byref(c), ctypes.c_void_p(self.ws.data_ptr()), n.value, ctypes.c_void_p(stream),
                        ctypes.byref(h))
        if st:
            raise PicError(st, "mlp_init failed")
        self.handle, self.cfg = h, c
        cnt = _I64()
        self.check(L.mlp_param_count(h, ctypes.byref(cnt)))
        self.n_params = cnt.value

    def check(self, st):
        if st != PIC_OK:
            raise PicError(st, _mlp_lib().mlp_last_error(self.handle).decode())
        return st

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == self.n_params
        self.check(_mlp_lib().mlp_set_params(self.handle, a.ctypes.data_as(_PF)))

    def get_params(self):
        a = np.zeros(self.n_params, np.float32)
        self.check(_mlp_lib().mlp_get_params(self.handle, a.ctypes.data_as(_PF)))
        return a

    def get_grads(self):
        a = np.zeros(self.n_params, np.float32)
        self.check(_mlp_lib().mlp_get_grads(self.handle, a.ctypes.data_as(_PF)))
        return a

    def forward(self, x, y=None):
        import torch
        x = x.contiguous()
        if y is None:
            y = torch.empty((x.shape[0], self.cfg.n_out), dtype=torch.float32, device=x.device)
        self.check(_mlp_lib().mlp_forward(self.handle, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                          ctypes.c_void_p(y.data_ptr())))
        return y

    def forward_noalloc(self, x, y=None):
        """mlp_forward_noalloc: the same network output, activations in the
        library's static device scratch (batch <= 64)."""
        import torch
        x = x.contiguous()
        if y is None:
            y = torch.empty((x.shape[0], self.cfg.n_out), dtype=torch.float32, device=x.device)
        self.check(_mlp_lib().mlp_forward_noalloc(self.handle, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                                  ctypes.c_void_p(y.data_ptr())))
        return y

    def train_step(self, x, t, want_loss=True):
        x, t = x.contiguous(), t.contiguous()
        loss = ctypes.c_float()
        self.check(_mlp_lib().mlp_train_step(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                             x.shape[0], ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def sync(self):
        self.check(_mlp_lib().mlp_sync(self.handle))

    def __del__(self):
        try:
            if self.handle:
                _mlp_lib().mlp_destroy(self.handle)
                self.handle = None
        except Exception:
            pass
