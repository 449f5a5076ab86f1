"""Plain FP64 CPU oracle of the RZ PIC/MCC step (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use this package.  It shares no code with the HIP path; the
two meet only in ``paper_2609_15043_amd.workloads`` (input descriptions).

Per step n (ordering of the paper's workflow, Sec. 2.5 and its algorithm
figure; the particle modules are inherited by the paper and read in their
textbook forms):

1. E_r, E_z at nodes from phi^n by central differences (E_R = 0 on the axis,
   Eq. axis_electrostatic_bc); E_theta(t_n) = E_c cos th - E_s^sto sin th
   (Eq. et_reconstruct).
2. gather at x^n, Boris kick, Cartesian move, J_theta^n deposit (cpic.c).
3. harmonic accumulation of J^n, Q_k(t_n), V_k(t_n) and the inductive power
   (Eqs. fourier, pind, pcap).
4. null-collision MCC on v^{n+1/2} at x^{n+1}; births sorted by parent id.
5. charge deposit rho^{n+1} plus the window surface charge.
6. Poisson for phi^{n+1} with the turn Dirichlet values phi_k(t_{n+1})
   (Eqs. poisson with chi = 0, epseff, areas, dirichlet) solved by a sparse
   direct factorization, and the turn charges Q_k(t_{n+1}) from the face
   fluxes of the same operator (Eq. facecharge).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib_path():
    return os.path.join(_HERE, "libcpic.so")


def build(force=False):
    """Compile cpic.c with gcc into oracle/libcpic.so."""
    out = lib_path()
    src = os.path.join(_HERE, "cpic.c")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        import subprocess
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


class Grid(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("nz", ctypes.c_int32), ("ip", ctypes.c_int32),
                ("window", ctypes.c_int32), ("dr", ctypes.c_double), ("dz", ctypes.c_double),
                ("rmax", ctypes.c_double), ("zp", ctypes.c_double)]


class Species(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("m", ctypes.c_double), ("w", ctypes.c_double),
                ("dt", ctypes.c_double), ("b", ctypes.c_double * 3)]


class XS(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32)] + [(n, ctypes.c_double) for n in (
        "el_a", "el_b", "exc_a", "exc_th", "iz_a", "iz_th", "iel_a", "iel_p", "icx_a", "icx_p",
        "e_cap_ev", "i_gcap", "nu_margin")]


class Gas(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("ngas", "tgas_ev", "qe", "me", "mi")]


def _p(a, t):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(t))


_D = ctypes.c_double
_U32 = ctypes.c_uint32
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64


def lib():
    global _LIB
    if _LIB is None:
        path = lib_path()
        if not os.path.exists(path):
            build()
        L = ctypes.CDLL(path)
        L.ora_philox_many.argtypes = [_I64, ctypes.POINTER(_U32), _U32, _U32, ctypes.POINTER(_U32)]
        L.ora_load.argtypes = [_I64, _U32, ctypes.c_int, _D, _D, _D, _D, _D] + \
            [ctypes.POINTER(_D)] * 5 + [ctypes.POINTER(_U32), ctypes.POINTER(_I32)]
        L.ora_gather_push.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Species), _I64] + \
            [ctypes.POINTER(_D)] * 5 + [ctypes.POINTER(_I32)] * 2 + [ctypes.POINTER(_D)] * 7
        L.ora_deposit.argtypes = [ctypes.POINTER(Grid), _I64, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                  ctypes.POINTER(_I32), _D, ctypes.POINTER(_D)]
        L.ora_sigma_e.argtypes = [ctypes.POINTER(XS), _D, ctypes.POINTER(_D)]
        L.ora_sigma_i.argtypes = [ctypes.POINTER(XS), _D, ctypes.POINTER(_D)]
        L.ora_null_setup.argtypes = [ctypes.POINTER(XS), ctypes.POINTER(Gas), _D, _I64,
                                     ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D)]
        L.ora_mcc.argtypes = [ctypes.c_int, _U32, _U32, ctypes.POINTER(XS), ctypes.POINTER(Gas), _D, _D, _D,
                              _I64, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D),
                              ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_U32),
                              ctypes.POINTER(_I32), ctypes.POINTER(_I32), _I64, ctypes.POINTER(_U32),
                              ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D),
                              ctypes.POINTER(_I32), ctypes.POINTER(_I64)]
        L.ora_mcc.restype = _I64
        di = [ctypes.POINTER(Grid), ctypes.POINTER(Species), _I64] + [ctypes.POINTER(_D)] * 8 + \
            [ctypes.POINTER(_I32)] * 2
        L.ora_di_predict.argtypes = di + [ctypes.POINTER(_D)] * 3
        L.ora_di_correct.argtypes = di + [ctypes.POINTER(_D)] * 3
        L.ora_see.argtypes = [_U32, _U32, _D, _D, _D, _I64, ctypes.POINTER(_U32), ctypes.POINTER(_D),
                              ctypes.POINTER(_D), ctypes.POINTER(_I32), ctypes.POINTER(_D), ctypes.POINTER(_D),
                              ctypes.POINTER(_D), ctypes.POINTER(_I32)]
        L.ora_see.restype = _I64
        _LIB = L
    return _LIB


# ---------------------------------------------------------------------------
# Philox and loading
# ---------------------------------------------------------------------------
def philox(ctr, key):
    """Philox4x32-10 blocks for counters ctr (n x 4 uint32) under key (k0, k1)."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().ora_philox_many(len(ctr), _p(ctr, _U32), _U32(key[0]), _U32(key[1]), _p(out, _U32))
    return out


def xs_struct(xs):
    x = XS()
    x.kind = xs.kind
    for n in ("el_a", "el_b", "exc_a", "exc_th", "iz_a", "iz_th", "iel_a", "iel_p", "icx_a", "icx_p",
              "e_cap_ev", "i_gcap", "nu_margin"):
        setattr(x, n, getattr(xs, n))
    return x


def gas_struct(wl):
    from paper_2609_15043_amd import workloads as W
    g = Gas()
    g.ngas, g.tgas_ev, g.qe, g.me, g.mi = wl.ngas, wl.tgas_ev, W.QE, W.ME, W.M_AR
    return g


NSCAN = 200_000


def null_setup(wl, nscan=NSCAN):
    """(nu_max[2], P_null[2], log(1 - P_null)[2]) for electrons and ions."""
    nu = np.zeros(2)
    pn = np.zeros(2)
    lq = np.zeros(2)
    x, g = xs_struct(wl.xs), gas_struct(wl)
    lib().ora_null_setup(ctypes.byref(x), ctypes.byref(g), wl.dt, nscan, _p(nu, _D), _p(pn, _D), _p(lq, _D))
    return nu, pn, lq


def sigma_e(xs, eps):
    out = np.zeros(3)
    lib().ora_sigma_e(ctypes.byref(xs_struct(xs)), float(eps), _p(out, _D))
    return out


def sigma_i(xs, ecm):
    out = np.zeros(2)
    lib().ora_sigma_i(ctypes.byref(xs_struct(xs)), float(ecm), _p(out, _D))
    return out


class Particles:
    """One species: absolute positions (R, z) in metres, velocities in the
    local (r, theta, z) frame, ids and a live flag."""

    def __init__(self, n):
        self.R = np.zeros(n)
        self.z = np.zeros(n)
        self.vr = np.zeros(n)
        self.vt = np.zeros(n)
        self.vz = np.zeros(n)
        self.id = np.zeros(n, np.uint32)
        self.alive = np.ones(n, np.int32)
        self.next = np.zeros(n, np.int32)
        # filtered electrostatic acceleration of the direct-implicit update
        # (local frame), zero unless that update runs
        self.ar = np.zeros(n)
        self.at = np.zeros(n)
        self.az = np.zeros(n)

    @property
    def n(self):
        return len(self.R)

    def append(self, R, z, v, ids, nxt):
        self.R = np.concatenate([self.R, R])
        self.z = np.concatenate([self.z, z])
        self.vr = np.concatenate([self.vr, v[:, 0]])
        self.vt = np.concatenate([self.vt, v[:, 1]])
        self.vz = np.concatenate([self.vz, v[:, 2]])
        self.id = np.concatenate([self.id, ids.astype(np.uint32)])
        self.alive = np.concatenate([self.alive, np.ones(len(R), np.int32)])
        self.next = np.concatenate([self.next, nxt.astype(np.int32)])
        for k in ("ar", "at", "az"):
            setattr(self, k, np.concatenate([getattr(self, k), np.zeros(len(R))]))

    def compact(self):
        m = self.alive.astype(bool)
        for k in ("R", "z", "vr", "vt", "vz", "id", "alive", "next", "ar", "at", "az"):
            setattr(self, k, getattr(self, k)[m].copy())

    def live(self):
        """Dict of the live particles, sorted by id."""
        m = self.alive.astype(bool)
        o = np.argsort(self.id[m], kind="stable")
        return {k: getattr(self, k)[m][o] for k in ("id", "R", "z", "vr", "vt", "vz", "next", "ar", "at", "az")}


def load_species(wl, s, lq=None):
    from paper_2609_15043_amd import workloads as W
    if lq is None:
        lq = null_setup(wl)[2][s]
    n = wl.np_init[s]
    P = Particles(n)
    vth = math.sqrt(wl.temp_ev[s] * W.QE / wl.mass[s])
    lib().ora_load(n, _U32(wl.seed), s, wl.rmax, 0.0, wl.zp, vth, float(lq), _p(P.R, _D), _p(P.z, _D),
                   _p(P.vr, _D), _p(P.vt, _D), _p(P.vz, _D), _p(P.id, _U32), _p(P.next, _I32))
    return P


# ---------------------------------------------------------------------------
# Grid operators
# ---------------------------------------------------------------------------
def theta(n, nrf):
    """Phase of step n (Eq. et_reconstruct)."""
    return 2.0 * math.pi * (n % nrf) / nrf


def n_rf(freq, dt):
    """N_RF = nint(1 / (f dt)) and whether the phase closes (Eqs. nrf, phaseclosure)."""
    N = int(round(1.0 / (freq * dt)))
    return N, abs(freq * dt * N - 1.0) < 1e-10


def rf_bfield(ec, es_sto, dr, dz, omega, th):
    """RF magnetic field (B_r, B_z) at phase th of the applied azimuthal
    field E_theta(t) = E_c cos(wt) - E_s^sto sin(wt), from Faraday's law
    dB/dt = -curl E (the paper leaves the push's magnetic field unstated;
    this is the field that its own E_theta implies).  With the time
    integral F = (E_c sin(wt) + E_s^sto cos(wt)) / w of E_theta (zero
    mean), B = -curl(F theta_hat):
        B_r = dF/dz,    B_z = -(1/R) d(R F)/dR.
    Node values by central differences inside, one-sided at the domain
    edges; on the axis (1/R) d(R F)/dR -> 2 dF/dR, with F = 0 there."""
    F = (np.asarray(ec) * math.sin(th) + np.asarray(es_sto) * math.cos(th)) / omega
    nz1, nr1 = F.shape
    Br = np.zeros_like(F)
    Bz = np.zeros_like(F)
    Br[1:-1, :] = (F[2:, :] - F[:-2, :]) / (2 * dz)
    Br[0, :] = (F[1, :] - F[0, :]) / dz
    Br[-1, :] = (F[-1, :] - F[-2, :]) / dz
    R = np.arange(nr1) * dr
    RF = R[None, :] * F
    Bz[:, 1:-1] = -(RF[:, 2:] - RF[:, :-2]) / (2 * dr) / R[None, 1:-1]
    Bz[:, -1] = -(RF[:, -1] - RF[:, -2]) / dr / R[-1]
    Bz[:, 0] = -2.0 * (F[:, 1] - F[:, 0]) / dr
    return np.ascontiguousarray(Br), np.ascontiguousarray(Bz)


def e_from_phi(phi, dr, dz):
    """Node E_r, E_z = -grad phi: central differences inside, one-sided at
    the domain edges, E_r = 0 on the axis."""
    nz1, nr1 = phi.shape
    Ez = np.zeros_like(phi)
    Er = np.zeros_like(phi)
    Ez[1:-1, :] = -(phi[2:, :] - phi[:-2, :]) / (2 * dz)
    Ez[0, :] = -(phi[1, :] - phi[0, :]) / dz
    Ez[-1, :] = -(phi[-1, :] - phi[-2, :]) / dz
    Er[:, 1:-1] = -(phi[:, 2:] - phi[:, :-2]) / (2 * dr)
    Er[:, -1] = -(phi[:, -1] - phi[:, -2]) / dr
    Er[:, 0] = 0.0
    return Er, Ez


def poisson_faces(nr, nz, dr, dz, eps_cell, eps0):
    """All control-volume faces of the finite-volume RZ Poisson operator.

    Returns a list of (node_a, node_b, conductance) with
    conductance = eps0 * eps_f * A_f / d_f (Eqs. epseff with chi = 0, areas).
    Face areas: A_z = 2 pi R_j dR (pi dR^2 / 4 on the axis), A_R(+-) =
    2 pi (R_j +- dR/2) dz; rows 0 and nz have half-height control volumes.
    eps_f is the mean relative permittivity of the cells sharing the face.
    """
    faces = []
    nr1 = nr + 1

    def nid(i, j):
        return i * nr1 + j

    def eps_mean(cells):
        vals = [eps_cell[i, j] for (i, j) in cells if 0 <= i < nz and 0 <= j < nr]
        return sum(vals) / len(vals)

    for i in range(nz + 1):
        for j in range(nr + 1):
            Rj = j * dr
            # axial face between node (i, j) and (i+1, j)
            if i < nz:
                lo = max(0.0, Rj - dr / 2)
                hi = min(nr * dr, Rj + dr / 2)
                area = math.pi * (hi * hi - lo * lo)
                ef = eps_mean([(i, j - 1), (i, j)])
                faces.append((nid(i, j), nid(i + 1, j), eps0 * ef * area / dz))
            # radial face between node (i, j) and (i, j+1)
            if j < nr:
                zlo = max(0.0, i * dz - dz / 2)
                zhi = min(nz * dz, i * dz + dz / 2)
                area = 2 * math.pi * (Rj + dr / 2) * (zhi - zlo)
                ef = eps_mean([(i - 1, j), (i, j)])
                faces.append((nid(i, j), nid(i, j + 1), eps0 * ef * area / dr))
    return faces


class Poisson:
    """Direct solver of sum_f c_f (phi_p - phi_nb) = Q_p on free nodes with
    Dirichlet values on tagged nodes (tag >= 0): 0 on grounded metal, the
    turn potential on turn k."""

    def __init__(self, nr, nz, dr, dz, eps_cell, tag, eps0):
        self.nr, self.nz = nr, nz
        self.tag = tag.reshape(-1)
        n = (nr + 1) * (nz + 1)
        self.faces = poisson_faces(nr, nz, dr, dz, eps_cell, eps0)
        free = self.tag < 0
        self.free = free
        idx = -np.ones(n, np.int64)
        idx[free] = np.arange(free.sum())
        self.idx = idx
        rows, cols, vals = [], [], []
        diag = np.zeros(free.sum())
        # coupling of free nodes to Dirichlet nodes: rhs += c * phi_D
        self.dir_a, self.dir_b, self.dir_c = [], [], []
        for a, b, c in self.faces:
            for p, q in ((a, b), (b, a)):
                if free[p]:
                    diag[idx[p]] += c
                    if free[q]:
                        rows.append(idx[p]); cols.append(idx[q]); vals.append(-c)
                    else:
                        self.dir_a.append(idx[p]); self.dir_b.append(q); self.dir_c.append(c)
        m = free.sum()
        A = sp.coo_matrix((vals, (rows, cols)), shape=(m, m)).tocsc() + sp.diags(diag).tocsc()
        self.A = A.tocsc()
        self.lu = spla.splu(self.A)
        self.dir_a = np.array(self.dir_a, np.int64)
        self.dir_b = np.array(self.dir_b, np.int64)
        self.dir_c = np.array(self.dir_c)
        fa = np.array([f[0] for f in self.faces], np.int64)
        fb = np.array([f[1] for f in self.faces], np.int64)
        fc = np.array([f[2] for f in self.faces])
        self.fa, self.fb, self.fc = fa, fb, fc

    def dirichlet_values(self, turn_phi, ground=None):
        """Node array of Dirichlet values (free nodes 0).  Tag-0 nodes take
        `ground` (a node array, default 0), turn-k nodes the turn potential."""
        v = np.zeros(len(self.tag))
        if ground is not None:
            g = np.asarray(ground, dtype=np.float64).reshape(-1)
            v[self.tag == 0] = g[self.tag == 0]
        for k, ph in enumerate(turn_phi, start=1):
            v[self.tag == k] = ph
        return v

    def solve(self, Q, turn_phi, ground=None, chi=None):
        """phi on all nodes for node charge Q (C) and turn potentials.  chi
        (node array, optional): the direct-implicit susceptibility; every
        face conductance is multiplied by 1 + (chi_a + chi_b) / 2 (Eq.
        epseff) and the system is assembled and factored for this call."""
        vD = self.dirichlet_values(turn_phi, ground)
        rhs = Q.reshape(-1)[self.free].copy()
        if chi is None:
            lu, dc = self.lu, self.dir_c
        else:
            f = self.face_factor(chi)
            lu, dc = self._factor(self.fc * f)
        np.add.at(rhs, self.dir_a, dc * vD[self.dir_b])
        phi = vD.copy()
        phi[self.free] = lu.solve(rhs)
        return phi.reshape(self.nz + 1, self.nr + 1)

    def face_factor(self, chi):
        """1 + (chi_a + chi_b) / 2 of every face (Eq. epseff)."""
        c = np.asarray(chi, dtype=np.float64).reshape(-1)
        return 1.0 + 0.5 * (c[self.fa] + c[self.fb])

    def _factor(self, cond):
        """Sparse LU of the free-node system with face conductances cond, and
        the conductances of the free-to-Dirichlet couplings (in the order of
        dir_a / dir_b)."""
        free, idx = self.free, self.idx
        m = int(free.sum())
        fa, fb = self.fa, self.fb
        diag = np.zeros(m)
        rows, cols, vals, dcs = [], [], [], []
        for a, b, c in zip(fa, fb, cond):
            for p, q in ((a, b), (b, a)):
                if free[p]:
                    diag[idx[p]] += c
                    if free[q]:
                        rows.append(idx[p]); cols.append(idx[q]); vals.append(-c)
                    else:
                        dcs.append(c)
        A = sp.coo_matrix((vals, (rows, cols)), shape=(m, m)).tocsc() + sp.diags(diag).tocsc()
        return spla.splu(A.tocsc()), np.array(dcs)

    def turn_charges(self, phi, nturns, chi=None):
        """Q_k = sum over faces between a turn-k node and a node outside the
        turn of c_f (phi_k - phi_nb) (Eq. facecharge), with the same face
        coefficients as the solve (chi included when given)."""
        ph = phi.reshape(-1)
        fc = self.fc if chi is None else self.fc * self.face_factor(chi)
        Qk = np.zeros(nturns)
        ta, tb = self.tag[self.fa], self.tag[self.fb]
        for k in range(1, nturns + 1):
            m1 = (ta == k) & (tb != k)
            m2 = (tb == k) & (ta != k)
            Qk[k - 1] = np.sum(fc[m1] * (ph[self.fa[m1]] - ph[self.fb[m1]])) + \
                np.sum(fc[m2] * (ph[self.fb[m2]] - ph[self.fa[m2]]))
        return Qk


# ---------------------------------------------------------------------------
# Period accumulators (Eqs. fourier, icap, pind, pcap, pcap_phasor)
# ---------------------------------------------------------------------------
class Harmonics:
    """Harmonic and power accumulators over one RF period: the projections
    on cos(m th_n), sin(m th_n) of order m (the fundamental by default), the
    time-domain inductive power and the trapezoid of V_k dQ_k.  freq is the
    fundamental's: the period sampled is 1 / freq for every order, and the
    order's charge harmonic gives I_cap at its own angular frequency
    2 pi m freq."""

    def __init__(self, shape, nturns, nrf, freq, order=1):
        self.shape, self.N, self.nrf, self.freq, self.order = shape, nturns, nrf, freq, order
        self.reset()

    def reset(self):
        self.Jc = np.zeros(self.shape)
        self.Js = np.zeros(self.shape)
        self.Qc = np.zeros(self.N)
        self.Qs = np.zeros(self.N)
        self.W = np.zeros(self.N)
        self.pind = 0.0
        self.samples = 0
        self.first = None
        self.prev = None

    def add(self, n, I, Et, Qk, Vk):
        """Sample of step n: node current I^n, node E_theta(t_n), turn
        charges Q_k(t_n) and turn potentials V_k(t_n)."""
        th = theta(n, self.nrf) * self.order
        c, s = math.cos(th), math.sin(th)
        self.Jc += I * c
        self.Js += I * s
        self.Qc += Qk * c
        self.Qs += Qk * s
        self.pind += float(np.sum(I * Et))
        Vk = np.asarray(Vk, dtype=np.float64)
        Qk = np.asarray(Qk, dtype=np.float64)
        if self.prev is None:
            self.first = (Vk.copy(), Qk.copy())
        else:
            Vp, Qp = self.prev
            self.W += 0.5 * (Vk + Vp) * (Qk - Qp)
        self.prev = (Vk.copy(), Qk.copy())
        self.samples += 1

    def finalize(self, Vc, Vs):
        """Closed-period quantities, or None when the sample count is not
        N_RF (the update is then rejected).  Vc, Vs: turn voltage phasor
        components held during the period (V_k = Vc - i Vs)."""
        if self.samples != self.nrf:
            return None
        N = self.nrf
        V0, Q0 = self.first
        Vl, Ql = self.prev
        W = self.W + 0.5 * (V0 + Vl) * (Q0 - Ql)          # periodic closure
        w = 2 * math.pi * (self.freq * self.order)
        Qc, Qs = 2.0 / N * self.Qc, 2.0 / N * self.Qs
        Icap = w * Qs + 1j * w * Qc
        Vhat = np.asarray(Vc) - 1j * np.asarray(Vs)
        return dict(Jc=2.0 / N * self.Jc, Js=2.0 / N * self.Js, Qc=Qc, Qs=Qs, Icap=Icap,
                    P_ind=self.pind / N, W=W, P_cap=self.freq * float(np.sum(W)),
                    P_cap_ph=0.5 * float(np.real(np.sum(Vhat * np.conj(Icap)))))


# ---------------------------------------------------------------------------
# The step
# ---------------------------------------------------------------------------
class OraclePIC:
    """Whole-step FP64 oracle for a Workload (see module docstring)."""

    def __init__(self, wl, load=True):
        from paper_2609_15043_amd import workloads as W
        self.wl = wl
        self.W = W
        self.grid = Grid(wl.nr, wl.nz, wl.ip, 1 if wl.window else 0, wl.dr, wl.dz, wl.rmax, wl.zp)
        self.sp = []
        for s in range(2):
            S = Species()
            S.q, S.m, S.w, S.dt = wl.charge[s], wl.mass[s], wl.weight[s], wl.dt
            for c in range(3):
                S.b[c] = wl.bfield[c]
            self.sp.append(S)
        self.nrf, self.closed = n_rf(wl.freq, wl.dt)
        self.numax, self.pnull, self.lq = null_setup(wl)
        self.xs, self.gas = xs_struct(wl.xs), gas_struct(wl)
        shape = (wl.nz + 1, wl.nr + 1)
        self.shape = shape
        self.poisson = Poisson(wl.nr, wl.nz, wl.dr, wl.dz, wl.eps_cell, wl.node_tag, W.EPS0)
        # applied turn potentials and azimuthal field: prescribed, or from the
        # field-circuit coupling (oracle/circuit.py)
        self.fc = None
        self.last_report = None
        self.surrogate = None          # callable features -> predicted (V_p, I_cap) vector, or None
        self.sur_cfg = dict(err_max=0.02, tol=1e-6, max_iter=50)
        self.births_total = 0
        self.births_prev = 0
        self.see_pending = None          # ions of the step at metal walls (secondary emission)
        # retained source harmonics (orders 2..M) of a coupled cell
        self.M = 1 + (len(wl.circuit.harmonics) if wl.circuit is not None else 0)
        if wl.circuit is not None and self.M > 1:
            from .circuit import MultiHarmonicCircuit
            self.fc = MultiHarmonicCircuit(wl.nr, wl.nz, wl.dr, wl.dz, wl.node_tag, wl.eps_cell, wl.freq, W.EPS0,
                                           wl.circuit)
            self.vc, self.vs, self.ec, self.es = self.fc.turn_vc, self.fc.turn_vs, self.fc.Ec, self.fc.Es
        elif wl.circuit is not None:
            from .circuit import FieldCircuit
            self.fc = FieldCircuit(wl.nr, wl.nz, wl.dr, wl.dz, wl.node_tag, wl.eps_cell, wl.freq, W.EPS0,
                                   wl.circuit)
            self.vc, self.vs, self.ec, self.es = self.fc.turn_vc, self.fc.turn_vs, self.fc.Ec, self.fc.Es
        else:
            self.vc, self.vs = np.asarray(wl.turn_vc, np.float64), np.asarray(wl.turn_vs, np.float64)
            self.ec, self.es = np.asarray(wl.ec, np.float64), np.asarray(wl.es_sto, np.float64)
        self.surf = np.zeros(shape)
        self.implicit = bool(wl.implicit)
        self.chi = np.zeros(shape)
        self.parts = [load_species(wl, s, self.lq[s]) if load else Particles(0) for s in range(2)]
        self.next_id = [wl.np_init[0], wl.np_init[1]]
        self.counts = np.zeros((2, 5), np.int64)
        self.n = 0
        self.Q = self.deposit()
        self.phi = self.poisson.solve(self.Q, self.turn_phi(0))
        self.Qk = self.poisson.turn_charges(self.phi, wl.nturns)
        self.I = np.zeros(shape)
        self.reset_harmonics()

    # -- fields -----------------------------------------------------------
    def turn_phi(self, n):
        th = theta(n, self.nrf)
        if self.M > 1:   # sum over the retained orders m: V_c^(m) cos(m th) + V_s^(m) sin(m th)
            return sum(vc * math.cos(m * th) + vs * math.sin(m * th)
                       for m, (vc, vs) in enumerate(zip(self.vc, self.vs), start=1))
        return self.vc * math.cos(th) + self.vs * math.sin(th)

    def etheta(self, n):
        th = theta(n, self.nrf)
        if self.M > 1:
            return sum(ec * math.cos(m * th) - es * math.sin(m * th)
                       for m, (ec, es) in enumerate(zip(self.ec, self.es), start=1))
        return self.ec * math.cos(th) - self.es * math.sin(th)

    # -- particle operations ------------------------------------------------
    def gather_push(self, n):
        Er, Ez = e_from_phi(self.phi, self.wl.dr, self.wl.dz)
        Et = self.etheta(n)
        Er, Ez, Et = (np.ascontiguousarray(a, dtype=np.float64) for a in (Er, Ez, Et))
        Br = Bz = None
        if self.wl.rf_bfield:
            assert self.M == 1, "the RF magnetic field is formed from the fundamental only"
            Br, Bz = rf_bfield(self.ec, self.es, self.wl.dr, self.wl.dz, 2 * math.pi * self.wl.freq,
                               theta(n, self.nrf))
        self.I = np.zeros(self.shape)
        self.absorbed = []
        self.see_pending = None
        for s in range(2):
            P = self.parts[s]
            ab = np.zeros(P.n, np.int32)
            if s == 1 and self.wl.see_gamma > 0:
                R0, z0 = P.R.copy(), P.z.copy()
            lib().ora_gather_push(ctypes.byref(self.grid), ctypes.byref(self.sp[s]), P.n,
                                  _p(P.R, _D), _p(P.z, _D), _p(P.vr, _D), _p(P.vt, _D), _p(P.vz, _D),
                                  _p(P.alive, _I32), _p(ab, _I32), _p(Er, _D), _p(Ez, _D), _p(Et, _D),
                                  _p(Br, _D), _p(Bz, _D), _p(self.I, _D), _p(self.surf, _D))
            self.absorbed.append(ab)
            if s == 1 and self.wl.see_gamma > 0:
                # ions absorbed at a metal wall (code 1; 2 is the window):
                # the wall from the position after the move
                k = np.nonzero(ab == 1)[0]
                zn = P.z[k]
                wall = np.where(zn < 0, 1, np.where(zn >= self.wl.zp, 3 if self.wl.window else 2, 3))
                self.see_pending = (P.id[k].copy(), R0[k], z0[k], wall.astype(np.int32))

    def mcc(self, n):
        births = []
        for s in range(2):
            P = self.parts[s]
            bcap = max(16, P.n // 4)
            bp = np.zeros(bcap, np.uint32)
            bR, bz = np.zeros(bcap), np.zeros(bcap)
            bve, bvi = np.zeros((bcap, 3)), np.zeros((bcap, 3))
            bnx = np.zeros((bcap, 2), np.int32)
            cnt = np.zeros(5, np.int64)
            nb = lib().ora_mcc(s, _U32(self.wl.seed), _U32(n), ctypes.byref(self.xs), ctypes.byref(self.gas),
                               float(self.numax[s]), float(self.lq[s]), float(self.lq[1]), P.n, _p(P.R, _D),
                               _p(P.z, _D), _p(P.vr, _D), _p(P.vt, _D), _p(P.vz, _D), _p(P.id, _U32),
                               _p(P.alive, _I32), _p(P.next, _I32), bcap, _p(bp, _U32), _p(bR, _D),
                               _p(bz, _D), _p(bve, _D), _p(bvi, _D), _p(bnx, _I32), _p(cnt, _I64))
            if nb < 0:
                raise RuntimeError("oracle birth buffer overflow")
            self.counts[s] += cnt
            births.append((bp[:nb], bR[:nb], bz[:nb], bve[:nb], bvi[:nb], bnx[:nb]))
        # births: electron-impact ionization only; ids in order of parent id
        bp, bR, bz, bve, bvi, bnx = births[0]
        o = np.argsort(bp, kind="stable")
        bp, bR, bz, bve, bvi, bnx = bp[o], bR[o], bz[o], bve[o], bvi[o], bnx[o]
        nb = len(bp)
        if nb:
            ide = np.arange(self.next_id[0], self.next_id[0] + nb, dtype=np.uint64)
            idi = np.arange(self.next_id[1], self.next_id[1] + nb, dtype=np.uint64)
            self.parts[0].append(bR, bz, bve, ide, bnx[:, 0])
            self.parts[1].append(bR.copy(), bz.copy(), bvi, idi, bnx[:, 1])
            self.next_id[0] += nb
            self.next_id[1] += nb
        self.last_births = (bp, ide if nb else np.zeros(0), idi if nb else np.zeros(0))
        self.births_total += nb
        self.secondary_emission(n)

    def secondary_emission(self, n):
        """Electrons emitted by the ions absorbed at metal walls during step
        n (cpic.c ora_see), in ascending parent-ion id order after the
        step's ionization births; ids continue the electron counter."""
        self.see_absorbed, self.see_emitted = np.zeros(0, np.uint32), 0
        if self.see_pending is None or len(self.see_pending[0]) == 0:
            return
        pid, R0, z0, wall = self.see_pending
        o = np.argsort(pid, kind="stable")
        pid, R0, z0, wall = (np.ascontiguousarray(a[o]) for a in (pid, R0, z0, wall))
        m = len(pid)
        R, z, v, nx = np.zeros(m), np.zeros(m), np.zeros((m, 3)), np.zeros(m, np.int32)
        sigma = math.sqrt(self.wl.see_temp_ev * self.W.QE / self.W.ME)
        k = lib().ora_see(_U32(self.wl.seed), _U32(n), float(self.wl.see_gamma), sigma, float(self.lq[0]), m,
                          _p(pid, _U32), _p(R0, _D), _p(z0, _D), _p(wall, _I32), _p(R, _D), _p(z, _D),
                          _p(v, _D), _p(nx, _I32))
        if k:
            ids = np.arange(self.next_id[0], self.next_id[0] + k, dtype=np.uint64)
            self.parts[0].append(R[:k], z[:k], v[:k], ids, nx[:k])
            self.next_id[0] += k
        self.see_total = getattr(self, "see_total", 0) + k
        self.see_absorbed, self.see_emitted = pid, k

    def deposit(self):
        Q = np.zeros(self.shape)
        for s in range(2):
            P = self.parts[s]
            qw = self.sp[s].q * self.sp[s].w
            lib().ora_deposit(ctypes.byref(self.grid), P.n, _p(P.R, _D), _p(P.z, _D), _p(P.alive, _I32),
                              qw, _p(Q, _D))
        return Q + self.surf

    def solve(self, n1):
        chi = self.chi if self.implicit else None
        self.phi = self.poisson.solve(self.Q, self.turn_phi(n1), self._ground(), chi=chi)
        self.Qk = self.poisson.turn_charges(self.phi, self.wl.nturns, chi=chi)

    def _ground(self):
        """Dirichlet values of the grounded nodes: 0, or the manufactured
        boundary sum_k basis_k V_k(t) (the workload's dir_basis)."""
        return None

    # -- direct-implicit update (Sec. 2.3; D1 filter, see cpic.c) ------------
    def susceptibility(self):
        """chi at the nodes from the predicted particles: (dt^2 / 2) / eps0
        sum_s (q_s^2 / m_s) n_s, n_s the node density of species s (weights
        over the node volume), i.e. half the squared plasma frequency times
        dt^2 (Eq. poisson's chi, here the D1 scheme's)."""
        from .circuit import node_volume
        wl = self.wl
        acc = np.zeros(self.shape)
        for s in range(2):
            P = self.parts[s]
            lib().ora_deposit(ctypes.byref(self.grid), P.n, _p(P.R, _D), _p(P.z, _D), _p(P.alive, _I32),
                              self.sp[s].q ** 2 / self.sp[s].m * self.sp[s].w, _p(acc, _D))
        return 0.5 * wl.dt ** 2 / wl.eps0 * acc / node_volume(wl.nr, wl.nz, wl.dr, wl.dz)

    def predict(self, n):
        Et = np.ascontiguousarray(self.etheta(n), dtype=np.float64)
        self.I = np.zeros(self.shape)
        self.absorbed = []
        for s in range(2):
            P = self.parts[s]
            ab = np.zeros(P.n, np.int32)
            lib().ora_di_predict(ctypes.byref(self.grid), ctypes.byref(self.sp[s]), P.n,
                                 _p(P.R, _D), _p(P.z, _D), _p(P.vr, _D), _p(P.vt, _D), _p(P.vz, _D),
                                 _p(P.ar, _D), _p(P.at, _D), _p(P.az, _D), _p(P.alive, _I32), _p(ab, _I32),
                                 _p(Et, _D), _p(self.I, _D), _p(self.surf, _D))
            self.absorbed.append(ab)

    def correct(self):
        Er, Ez = (np.ascontiguousarray(a) for a in e_from_phi(self.phi, self.wl.dr, self.wl.dz))
        for s in range(2):
            P = self.parts[s]
            ab = np.zeros(P.n, np.int32)
            lib().ora_di_correct(ctypes.byref(self.grid), ctypes.byref(self.sp[s]), P.n,
                                 _p(P.R, _D), _p(P.z, _D), _p(P.vr, _D), _p(P.vt, _D), _p(P.vz, _D),
                                 _p(P.ar, _D), _p(P.at, _D), _p(P.az, _D), _p(P.alive, _I32), _p(ab, _I32),
                                 _p(Er, _D), _p(Ez, _D), _p(self.surf, _D))

    # -- harmonics ----------------------------------------------------------------
    def reset_harmonics(self):
        self.harm = Harmonics(self.shape, self.wl.nturns, self.nrf, self.wl.freq)
        # orders 2..M of a multiharmonic circuit
        self.harm_hi = [Harmonics(self.shape, self.wl.nturns, self.nrf, self.wl.freq, order=m)
                        for m in range(2, getattr(self, "M", 1) + 1)]

    def harmonic(self, n):
        I, Et, Vk = self.I, self.etheta(n), self.turn_phi(n)
        self.harm.add(n, I, Et, self.Qk, Vk)
        for h in self.harm_hi:
            h.add(n, I, Et, self.Qk, Vk)

    def moments(self):
        """Plasma moments of the current particles: <n_e>, <n_i> over the
        particle box (m^-3), the largest electron node density (m^-3, node
        weights over the node control volume), <eps_e>, <eps_i> (eV), the
        electron centroid R, z (m) and the ionizations since the last call
        in real particles (macro-particle births times the electron weight,
        so that the value does not depend on the macro-particle count)."""
        from .circuit import node_volume
        wl = self.wl
        vol = math.pi * wl.rmax ** 2 * wl.zp
        out = []
        for s in range(2):
            P = self.parts[s]
            a = P.alive.astype(bool)
            out.append((a.sum(), P, a))
        (ne, Pe, ae), (ni, Pi, ai) = out
        we, wi = self.sp[0].w, self.sp[1].w
        Wn = np.zeros(self.shape)
        lib().ora_deposit(ctypes.byref(self.grid), Pe.n, _p(Pe.R, _D), _p(Pe.z, _D), _p(Pe.alive, _I32), we,
                          _p(Wn, _D))
        nmax = float(np.max(Wn / node_volume(wl.nr, wl.nz, wl.dr, wl.dz)))
        me, mi = self.sp[0].m, self.sp[1].m

        def energy(P, a, m):
            v2 = P.vr[a] ** 2 + P.vt[a] ** 2 + P.vz[a] ** 2
            return float(np.mean(0.5 * m * v2 / self.W.QE)) if a.any() else 0.0

        ion = self.births_total - self.births_prev
        self.births_prev = self.births_total
        return np.array([ne * we / vol, ni * wi / vol, nmax, energy(Pe, ae, me), energy(Pi, ai, mi),
                         float(np.mean(Pe.R[ae])) if ne else 0.0, float(np.mean(Pe.z[ae])) if ne else 0.0,
                         float(ion) * we])

    def period_update(self):
        """Close the RF period: finalise the harmonics and, when coupled,
        update the circuit (plainly, or surrogate-assisted when a predictor
        is set) and the next period's turn potentials and field.  Returns
        the report (None and restart of the accumulators when the sample
        count is not N_RF)."""
        if self.M > 1:
            hs = [h.finalize(vc, vs) for h, vc, vs in zip([self.harm] + self.harm_hi, self.vc, self.vs)]
            self.reset_harmonics()
            if any(h is None for h in hs):
                return None
            rep = self.fc.update(hs)
            rep["moments"] = self.moments()
            rep["pressure"] = self.wl.pressure_pa
            self.vc, self.vs, self.ec, self.es = self.fc.turn_vc, self.fc.turn_vs, self.fc.Ec, self.fc.Es
            r = {**hs[0], **rep, "harmonics": hs}
            self.last_report = r
            return r
        r = self.harm.finalize(self.vc, self.vs)
        self.reset_harmonics()
        if r is None:
            return None
        if self.fc is not None:
            mom = self.moments()
            pressure = self.wl.pressure_pa
            if self.surrogate is not None:
                rep = self.fc.update_surrogate(r, pressure, mom, self.surrogate, **self.sur_cfg)
            else:
                rep = self.fc.update(r)
            rep["moments"] = mom
            rep["pressure"] = pressure
            self.vc, self.vs, self.ec, self.es = self.fc.turn_vc, self.fc.turn_vs, self.fc.Ec, self.fc.Es
            r = {**r, **rep}
        self.last_report = r
        return r

    # -- one whole step -----------------------------------------------------------
    def step(self):
        if self.implicit:
            assert self.wl.see_gamma == 0, "secondary emission runs with the explicit step only"
            return self.step_implicit()
        n = self.n
        self.gather_push(n)
        self.harmonic(n)
        self.mcc(n)
        self.Q = self.deposit()
        if self.fc is not None and (n + 1) % self.nrf == 0:
            self.period_update()
        self.solve(n + 1)
        self.n = n + 1
        for P in self.parts:
            P.compact()

    def step_implicit(self):
        """Direct-implicit step n: predictor (with J_theta^n), harmonics,
        charge and susceptibility at the predicted positions, the period
        update when due, the Poisson solve with chi, corrector, MCC on the
        corrected v^{n+1/2} at x^{n+1} (births join with zero filtered
        acceleration)."""
        n = self.n
        self.predict(n)
        self.harmonic(n)
        self.Q = self.deposit()
        self.chi = self.susceptibility()
        if self.fc is not None and (n + 1) % self.nrf == 0:
            self.period_update()
        self.solve(n + 1)
        self.correct()
        self.mcc(n)
        self.n = n + 1
        for P in self.parts:
            P.compact()

    def live(self, s):
        return self.parts[s].live()


# ---------------------------------------------------------------------------
# Direct access for pins
# ---------------------------------------------------------------------------
def make_grid(nr, nz, rmax, zmax, zp=None, window=False):
    zp = zmax if zp is None else zp
    dz = zmax / nz
    return Grid(nr, nz, int(round(zp / dz)), 1 if window else 0, rmax / nr, dz, rmax, zp)


def make_species(q, m, w, dt, b=(0.0, 0.0, 0.0)):
    S = Species()
    S.q, S.m, S.w, S.dt = q, m, w, dt
    for c in range(3):
        S.b[c] = b[c]
    return S


def gather_push_raw(grid, species, P, Er, Ez, Et):
    """One gather/push/move of Particles P in place; returns (I_node, surf, absorbed)."""
    shape = (grid.nz + 1, grid.nr + 1)
    I = np.zeros(shape)
    surf = np.zeros(shape)
    ab = np.zeros(P.n, np.int32)
    Er, Ez, Et = (np.ascontiguousarray(np.broadcast_to(a, shape), dtype=np.float64) for a in (Er, Ez, Et))
    lib().ora_gather_push(ctypes.byref(grid), ctypes.byref(species), P.n, _p(P.R, _D), _p(P.z, _D),
                          _p(P.vr, _D), _p(P.vt, _D), _p(P.vz, _D), _p(P.alive, _I32), _p(ab, _I32),
                          _p(Er, _D), _p(Ez, _D), _p(Et, _D), None, None, _p(I, _D), _p(surf, _D))
    return I, surf, ab


def see_raw(seed, n, gamma, sigma, lq_e, ids, R0, z0, wall):
    """ora_see on arrays (ids in the order given); returns (R, z, v, next)
    of the emitted electrons."""
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    R0, z0 = (np.ascontiguousarray(a, dtype=np.float64) for a in (R0, z0))
    wall = np.ascontiguousarray(wall, dtype=np.int32)
    m = len(ids)
    R, z, v, nx = np.zeros(m), np.zeros(m), np.zeros((m, 3)), np.zeros(m, np.int32)
    k = lib().ora_see(_U32(seed), _U32(n), float(gamma), float(sigma), float(lq_e), m, _p(ids, _U32), _p(R0, _D),
                      _p(z0, _D), _p(wall, _I32), _p(R, _D), _p(z, _D), _p(v, _D), _p(nx, _I32))
    return R[:k], z[:k], v[:k], nx[:k]


def deposit_raw(grid, P, qw):
    Q = np.zeros((grid.nz + 1, grid.nr + 1))
    lib().ora_deposit(ctypes.byref(grid), P.n, _p(P.R, _D), _p(P.z, _D), _p(P.alive, _I32), qw, _p(Q, _D))
    return Q


def mcc_raw(sp, seed, step, xs, gas, numax, lq, lq_ion, P, bcap=None):
    """MCC on Particles P in place at step `step` (candidates: P.next ==
    step); returns (counts[5], births dict)."""
    bcap = bcap or max(16, P.n)
    bp = np.zeros(bcap, np.uint32)
    bR, bz = np.zeros(bcap), np.zeros(bcap)
    bve, bvi = np.zeros((bcap, 3)), np.zeros((bcap, 3))
    bnx = np.zeros((bcap, 2), np.int32)
    cnt = np.zeros(5, np.int64)
    nb = lib().ora_mcc(sp, _U32(seed), _U32(step), ctypes.byref(xs), ctypes.byref(gas), float(numax),
                       float(lq), float(lq_ion), P.n, _p(P.R, _D), _p(P.z, _D), _p(P.vr, _D), _p(P.vt, _D),
                       _p(P.vz, _D), _p(P.id, _U32), _p(P.alive, _I32), _p(P.next, _I32), bcap,
                       _p(bp, _U32), _p(bR, _D), _p(bz, _D), _p(bve, _D), _p(bvi, _D), _p(bnx, _I32),
                       _p(cnt, _I64))
    if nb < 0:
        raise RuntimeError("birth buffer overflow")
    return cnt, dict(parent=bp[:nb], R=bR[:nb], z=bz[:nb], ve=bve[:nb], vi=bvi[:nb], next=bnx[:nb])
