"""Pins of the oracle's field-circuit coupling (oracle/circuit.py) against
what the paper and the mathematics fix:

* Test 1 (single ideal solenoid): the field-derived inductance and the
  series-circuit current of the paper's results table for that test;
* Test 2 (two coaxial solenoids): both columns of its results table -- the
  ideal-sheet inductances and two-loop phasors from the closed forms, and
  the field-derived self and mutual inductances and loop phasors, every
  printed digit;
* Test 3 (five nested current sheets): the printed relative errors of the
  extracted inductance and capacitance matrices, the spectral radius of the
  period recurrence, the continuous reference phasors (Eqs. t7C, t7M,
  t7network) and the field-circuit phasors after 30 periods, the power
  identity (Eq. t7power) with the printed reactive powers, and the
  perturbation checks of its appendix;
* closed forms and invariants: the shape normalisation (Eq. shape), the
  skin-resistance limits (Eq. skin), network residuals (Eqs. kclres,
  kvlres), the controller's fixed point and limiter (Eqs. pfilter, ptrend,
  pcontrol), and V_p = Z_vac I for a plasma current shaped like a turn
  (Eqs. helmholtz_two_real, vpind, zvac).
"""
import math
import os

import numpy as np
import pytest

from oracle import circuit as C
from oracle import pic as O


# ---------------------------------------------------------------------------
# Test 1: single ideal solenoid (a = 10 mm, length 1 m, padding b = 0.12 m,
# h = 1 mm, 1000 source nodes on the radial line R = a, MQS, 13.56 MHz,
# mu0 = 4 pi 1e-7; series R = 0.1 ohm driven by 1 V)
# ---------------------------------------------------------------------------
def _solenoid():
    h, nz, nr = 1e-3, 1240, 120
    mu0 = 4e-7 * math.pi
    w = 2 * math.pi * 13.56e6
    tag = np.full((nz + 1, nr + 1), -1, np.int32)
    tag[0, :] = tag[nz, :] = 0
    tag[:, nr] = 0
    tag[121:1121, 10] = 1
    helm = C.Helmholtz(nr, nz, h, h, tag == 0, w, mu0)
    g, area = C.shape_functions(tag, 1, h, h)
    U = helm.solve(g[0].reshape(nz + 1, nr + 1))
    Z = C.z_vac(g, U[None], C.projection_weights(nr, nz, h, h))
    return Z[0, 0], w, mu0


def test_solenoid_inductance_and_current():
    Z, w, mu0 = _solenoid()
    assert abs(Z.real) < 1e-15
    L = Z.imag / w
    # analytic ideal solenoid mu0 pi a^2 / length
    assert abs(mu0 * math.pi * 0.01 ** 2 / 1.0 - T1["L_ana_nH"] * 1e-9) < 5e-16
    # field-derived model value 0.388541 nH (Im Z 0.0331037 ohm); the finite
    # padding and ends put it 1.6 % below the ideal value
    assert abs(L - T1["L_num_nH"] * 1e-9) / (T1["L_num_nH"] * 1e-9) < 2e-4, L
    assert abs(Z.imag - T1["ImZ_num_ohm"]) / T1["ImZ_num_ohm"] < 2e-4
    I = 1.0 / (0.1 + Z)
    assert abs(abs(I) - T1["I_num_abs_A"]) < 2e-3
    assert abs(math.degrees(np.angle(I)) - T1["I_num_deg"]) < 0.01


# ---------------------------------------------------------------------------
# Test 2: two coaxial ideal solenoids (a1 = 10 mm, a2 = 20 mm, length 1 m,
# padding b = 0.12 m, h = 1 mm, MQS, 13.56 MHz); an isolated primary loop (1 V
# behind R1 = 0.1 ohm) and a passive secondary loop (R2 = 0.1 ohm, C = 10 nF)
# coupled only through Z_vac,12
# ---------------------------------------------------------------------------
def _t2_loops(Z, w, R1=0.1, R2=0.1, Cap=10e-9, U=1.0):
    """The two-loop phasors (Eqs. S2loops, S2zab, S2solution, S2ports)."""
    ZA = R1 + Z[0, 0]
    ZB = Z[1, 1] + R2 - 1j / (w * Cap)
    Zm = Z[0, 1]
    det = ZA * ZB - Zm * Zm
    I1, I2 = U * ZB / det, -Zm * U / det
    return dict(I1=I1, I2=I2, U1=Z[0, 0] * I1 + Z[0, 1] * I2, U2=Z[1, 0] * I1 + Z[1, 1] * I2)


def _t2_check(L, k, ph, col):
    """Compare inductances (nH), coupling and phasors with one column of the
    results table, to one unit in the last printed digit."""
    t = _scalars("test2_solenoids.txt")
    for name in ("L1", "L2", "M"):
        assert abs(L[name] - t[f"{name}_{col}_nH"]) <= 1e-6, (name, col, L[name])
    assert abs(k - t[f"k_{col}"]) <= 1e-6, (col, k)
    for name, x in ph.items():
        mag, deg = abs(x), math.degrees(np.angle(x))
        ulp = 10.0 ** (math.floor(math.log10(t[f"{name}_{col}_abs"])) - 5)   # six significant digits
        assert abs(mag - t[f"{name}_{col}_abs"]) <= ulp, (name, col, mag)
        assert abs(deg - t[f"{name}_{col}_deg"]) <= 1e-4, (name, col, deg)


def test_two_solenoids_analytical_column():
    """Eq. S2ind (mu0 pi a^2 / L for both self terms and the mutual term,
    k = a1 / a2) with mu0 = 4 pi 1e-7, through the loop equations."""
    w, mu0 = 2 * math.pi * 13.56e6, 4e-7 * math.pi
    L1, L2 = mu0 * math.pi * 0.01 ** 2 / 1.0, mu0 * math.pi * 0.02 ** 2 / 1.0
    M = L1
    Z = 1j * w * np.array([[L1, M], [M, L2]])
    _t2_check(dict(L1=L1 * 1e9, L2=L2 * 1e9, M=M * 1e9), M / math.sqrt(L1 * L2), _t2_loops(Z, w), "ana")


def test_two_solenoids_field_derived_column():
    """The oracle's unit solves and projections (Eqs. unitfield, zvac,
    S2Mnum) on the benchmark's grid give the model column: self and mutual
    inductances, coupling and the four loop phasors, every printed digit,
    with mu0 = 1.2566e-6 (the paper's stated constant of its Test 3; with
    4 pi 1e-7 the inductances come out 2.9e-5 higher).  Z_vac is symmetric
    (reciprocity) and purely reactive in the lossless vacuum."""
    from paper_2609_15043_amd import workloads as W
    wl = W.test2()
    nr, nz, h = wl.nr, wl.nz, wl.dr
    tag = wl.node_tag
    w, mu0 = 2 * math.pi * wl.freq, wl.circuit.mu0
    assert mu0 == 1.2566e-6
    helm = C.Helmholtz(nr, nz, h, h, tag == 0, w, mu0)
    g, _ = C.shape_functions(tag, 2, h, h)
    U = np.stack([helm.solve(g[k].reshape(nz + 1, nr + 1)) for k in range(2)])
    Z = C.z_vac(g, U, C.projection_weights(nr, nz, h, h))
    assert np.max(np.abs(Z.real)) < 1e-15
    assert abs(Z[0, 1] - Z[1, 0]) <= 1e-12 * abs(Z[0, 1])
    L = Z.imag / w * 1e9
    _t2_check(dict(L1=L[0, 0], L2=L[1, 1], M=L[0, 1]), L[0, 1] / math.sqrt(L[0, 0] * L[1, 1]), _t2_loops(Z, w), "num")


# ---------------------------------------------------------------------------
# Test 3: five nested sheets a = 8, 20, 32, 48, 64 mm in a shield b = 80 mm,
# source length 100 mm, eps_r = 9, eps0 = 8.8542e-12, mu0 = 1.2566e-6,
# 13.56 MHz, V_g = 100 V behind R_g = 50 ohm, R_rf = 20 ohm per segment,
# h = 1 mm, (N_z, N_R) = (102, 81) nodes, manufactured axial boundaries
# ---------------------------------------------------------------------------
T3_EPS0, T3_MU0, T3_F = 8.8542e-12, 1.2566e-6, 13.56e6
T3_A = np.array([8, 20, 32, 48, 64]) * 1e-3
T3_B, T3_ELL, T3_ER = 0.08, 0.1, 9.0

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _scalars(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if len(line) >= 2:
                out[line[0]] = float(line[1])
    return out


def _phasor_table():
    """The paper's Test 3 phasor table: (field-circuit, continuous) for
    x = I_f, I_1..5, V_1..5."""
    field, cont = [], []
    with open(os.path.join(GOLDEN, "test3_phasors.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            field.append(float(t[2]) + 1j * float(t[3]))
            cont.append(float(t[4]) + 1j * float(t[5]))
    return np.array(field), np.array(cont)


T3_FIELD, T3_CONT = _phasor_table()
T3 = _scalars("test3_scalars.txt")
T1 = _scalars("test1_solenoid.txt")


def _t3_continuous():
    a6 = np.append(T3_A, T3_B)
    c = 2 * math.pi * T3_EPS0 * T3_ER * T3_ELL / np.log(a6[1:] / a6[:-1])
    Cm = np.zeros((5, 5))
    for k in range(5):
        Cm[k, k] = c[k] + (c[k - 1] if k else 0.0)
        if k < 4:
            Cm[k, k + 1] = Cm[k + 1, k] = -c[k]
    M = np.array([[T3_MU0 * math.pi / T3_ELL * min(T3_A[k], T3_A[l]) ** 2 * (1 - max(T3_A[k], T3_A[l]) ** 2 / T3_B ** 2)
                   for l in range(5)] for k in range(5)])
    return Cm, M


def _t3_unit_field(k, R, w):
    """Closed-form unit-current field of sheet k (Eq. t7unitfield)."""
    a = T3_A[k]
    inside = (1 - a ** 2 / T3_B ** 2) * R
    outside = a ** 2 * (1 / np.maximum(R, 1e-300) - R / T3_B ** 2)
    return -w * T3_MU0 / (2 * T3_ELL) * np.where(R <= a, inside, outside)


def _t3_potential(V, R):
    """Closed-form electrostatic potential of sheet voltages V (Eq. t7potential)."""
    a6 = np.append(T3_A, T3_B)
    Vx = np.append(np.asarray(V, complex), 0.0)
    out = np.full(R.shape, Vx[0], complex)
    for k in range(5):
        m = (R > a6[k]) & (R <= a6[k + 1])
        out[m] = (Vx[k] * np.log(a6[k + 1] / R[m]) + Vx[k + 1] * np.log(R[m] / a6[k])) / np.log(a6[k + 1] / a6[k])
    return out


class _Test3:
    def __init__(self, h=1e-3, er=T3_ER):
        self.h = h
        self.nr = int(round(T3_B / h))
        nsrc = int(round(T3_ELL / h))
        self.nz = nsrc + 1
        self.w = 2 * math.pi * T3_F
        self.R = np.arange(self.nr + 1) * h
        tag = np.full((self.nz + 1, self.nr + 1), -1, np.int32)
        tag[0, :] = tag[self.nz, :] = 0
        tag[:, self.nr] = 0
        self.jk = np.rint(T3_A / h).astype(int)
        for k in range(5):
            tag[1:self.nz, self.jk[k]] = k + 1
        self.tag = tag
        ub = np.zeros((5, self.nz + 1, self.nr + 1))
        for k in range(5):
            ub[k, 0, :] = ub[k, self.nz, :] = _t3_unit_field(k, self.R, self.w)
        prm = type("P", (), dict(mu0=T3_MU0, field_mode=C.FIELD_MQS, turn_sign=None, rrf_mode=C.RRF_GIVEN,
                                 r_rf=[20.0] * 5, c_stray=None, r_g=50.0, r_m=0.0, l_m=0.0, c_m=0.0,
                                 vg_amp=100.0, vg_phase=0.0, vg_from_target=False, controller=False,
                                 alpha=1.0))()
        self.fc = C.FieldCircuit(self.nr, self.nz, h, h, tag, np.full((self.nz, self.nr), er), T3_F, T3_EPS0, prm,
                                 unit_bvals=ub)
        self.poisson = O.Poisson(self.nr, self.nz, h, h, np.full((self.nz, self.nr), er), tag, T3_EPS0)
        # axial boundary rows carry the closed-form potential of the applied voltages
        self.basis = np.stack([_t3_potential(np.eye(5)[k], self.R).real for k in range(5)])

    def phi(self, V):
        """Potential for real sheet potentials V (the axial rows follow Eq. t7potential)."""
        ground = np.zeros((self.nz + 1, self.nr + 1))
        prof = np.asarray(V) @ self.basis
        ground[0, :] = ground[self.nz, :] = prof
        ground[:, self.nr] = 0.0
        return self.poisson.solve(np.zeros_like(ground), V, ground)

    def charges(self, V):
        return self.poisson.turn_charges(self.phi(V), 5)

    def cap_matrix(self):
        return np.stack([self.charges(np.eye(5)[k]) for k in range(5)], axis=1)

    def harmonics(self, nrf=400):
        """One RF period with the applied state: the charges sampled at nrf
        phases, finalised harmonics (no circuit update)."""
        fc = self.fc
        harm = O.Harmonics((1, 1), 5, nrf, T3_F)
        Vc, Vs = fc.turn_vc, fc.turn_vs
        for n in range(nrf):
            th = 2 * math.pi * n / nrf
            V = Vc * math.cos(th) + Vs * math.sin(th)
            harm.add(n, np.zeros((1, 1)), np.zeros((1, 1)), self.charges(V), V)
        h = harm.finalize(Vc, Vs)
        shape = (self.nz + 1, self.nr + 1)
        h["Jc"], h["Js"] = np.zeros(shape), np.zeros(shape)
        return h

    def period(self, nrf=400):
        """One RF period with the applied state, then the circuit update."""
        h = self.harmonics(nrf)
        return h, self.fc.update(h)


@pytest.fixture(scope="module")
def t3():
    return _Test3()


def _scaled_err(x, ref):
    S = np.r_[np.full(6, abs(ref[0])), np.full(5, 100.0)]
    return np.linalg.norm((x - ref) / S) / np.linalg.norm(ref / S)


def test_t3_continuous_reference_reproduces_table():
    Cm, M = _t3_continuous()
    w = 2 * math.pi * T3_F
    A = C.network_matrix(50.0, 20.0 * np.eye(5) + 1j * w * M, np.zeros(5), w)
    # the capacitive current i w C V moved into the matrix
    A[1:6, 6:11] -= 1j * w * Cm
    x = np.linalg.solve(A, C.network_rhs(100.0, np.zeros(5), np.zeros(5)))
    assert np.max(np.abs(x - T3_CONT) / np.abs(T3_CONT)) < 1e-8
    # the period recurrence of the continuous matrices: spectral radius 0.359062
    A0 = C.network_matrix(50.0, 20.0 * np.eye(5) + 1j * w * M, np.zeros(5), w)
    T = np.zeros((11, 5))
    T[1:6] = np.eye(5)
    G = np.linalg.solve(A0, T @ (1j * w * Cm) @ np.hstack([np.zeros((5, 6)), np.eye(5)]))
    assert abs(max(abs(np.linalg.eigvals(G))) - T3["rho_G"]) < 1e-6


def test_t3_unit_fields_and_inductance_matrix(t3):
    fc = t3.fc
    _, M = _t3_continuous()
    Mh = fc.Zvac.imag / fc.omega
    assert np.max(np.abs(fc.Zvac.real)) < 1e-12 * np.max(np.abs(fc.Zvac))
    err = np.linalg.norm(Mh - M) / np.linalg.norm(M)
    assert abs(err - T3["M_rel_err"]) < 0.01 * T3["M_rel_err"], err
    eta = np.linalg.norm(Mh - Mh.T) / np.linalg.norm(Mh)
    assert abs(eta - T3["eta_M"]) < 0.01 * T3["eta_M"], eta
    # midplane unit fields against Eq. t7unitfield, cylindrically weighted
    mid = t3.nz // 2
    e = []
    for k in range(5):
        ref = _t3_unit_field(k, t3.R, fc.omega)
        m = ref != 0
        e.append(math.sqrt(np.sum(t3.R[m] * (fc.U[k, mid][m] - ref[m]) ** 2) / np.sum(t3.R[m] * ref[m] ** 2)))
    assert abs(max(e) - T3["U_field_err"]) < 0.01 * T3["U_field_err"], e


def test_t3_capacitance_matrix(t3):
    Cm, _ = _t3_continuous()
    Ch = t3.cap_matrix()
    err = np.linalg.norm(Ch - Cm) / np.linalg.norm(Cm)
    assert abs(err - T3["C_rel_err"]) < 0.01 * T3["C_rel_err"], err
    # zero conductor potentials give zero conductor charge
    assert np.max(np.abs(t3.charges(np.zeros(5)))) == 0.0
    # eps_r 9 -> 1 scales the extracted capacitance by 1/9
    Ch1 = _Test3(er=1.0).cap_matrix()
    assert np.max(np.abs(Ch1 * 9.0 - Ch)) / np.max(np.abs(Ch)) < 1e-12


def test_t3_coupled_periods_reproduce_table(t3):
    fc = t3.fc
    w = fc.omega
    Ch = t3.cap_matrix()
    # the first applied state is the network without capacitive feedback;
    # the semidiscrete recurrence has spectral radius 0.359069
    T = np.zeros((11, 5))
    T[1:6] = np.eye(5)
    G = np.linalg.solve(fc.A, T @ (1j * w * Ch) @ np.hstack([np.zeros((5, 6)), np.eye(5)]))
    assert abs(max(abs(np.linalg.eigvals(G))) - T3["rho_G_h"]) < 1e-6
    x = fc.x.copy()
    # first period through the time-sampled charges: I_cap = i w C_h V exactly
    h, rep = t3.period()
    V = x[6:]
    assert np.max(np.abs(h["Icap"] - 1j * w * Ch @ V)) < 1e-12 * np.max(np.abs(h["Icap"]))
    # a lossless linear capacitor network: P_cap from the trapezoid equals the
    # sinc-scaled phasor value (Eq. pcap_quadrature)
    th = 2 * math.pi / 400
    assert abs(h["P_cap"] - math.sin(th) / th * h["P_cap_ph"]) < 1e-10 * abs(h["P_cap_ph"])
    # alpha = 1: the applied state solves the assembled network exactly
    assert rep["kcl"] < 1e-13 and rep["kvl"] < 1e-13
    # periods 2..29 from the recurrence, the sampled path being the same
    # linear map (checked above); the 30th period sampled again, for the
    # power defects of the final completed period
    for _ in range(28):
        icap = 1j * w * Ch @ fc.x[6:]
        xt = np.linalg.solve(fc.A, C.network_rhs(fc.vg, icap, np.zeros(5)))
        fc.x = xt
    h30, rep30 = t3.period()
    xf = fc.x
    assert np.max(np.abs(xf - T3_FIELD)) < 6e-9 * np.max(np.abs(T3_FIELD[6:])), np.abs(xf - T3_FIELD)
    assert abs(_scaled_err(xf, T3_CONT) - T3["state_err_cont"]) < 0.01 * T3["state_err_cont"]
    assert abs(np.max(np.abs(xf - T3_CONT) / np.abs(T3_CONT)) - T3["max_phasor_err"]) < 0.01 * T3["max_phasor_err"]
    # power identity (Eq. t7power) at the fixed point with the extracted
    # matrices, and the printed reactive powers
    Mh = fc.Zvac.imag / w
    I, Vv, If = xf[1:6], xf[6:], xf[0]
    WM = np.conj(I) @ Mh @ I
    WC = np.conj(Vv) @ Ch @ Vv
    Sg = 0.5 * 100.0 * np.conj(If)
    rhs = 0.5 * 50.0 * abs(If) ** 2 + 0.5 * 20.0 * np.sum(np.abs(I) ** 2) + 0.5j * w * (WM - np.conj(WC))
    assert abs(Sg - rhs) / abs(Sg) < 1e-10
    assert abs(w / 2 * WM.real - T3["Q_L"]) < 2e-5
    assert abs(-w / 2 * WC.real - T3["Q_C"]) < 2e-5
    # capacitive power and the two normalised power defects of the final
    # completed period (Sec. 3.3 text): P_cap 1.34e-5 W, eta_cap 1.004e-6,
    # eta_coil 4.51e-7
    eta_cap = abs(h30["P_cap"]) / (abs(T3["Q_L"]) + abs(T3["Q_C"]))
    eta_coil = abs(rep30["p_port"] - rep30["p_cu"]) / abs(rep30["p_port"])
    assert abs(h30["P_cap"] - T3["P_cap_W"]) < 0.01 * T3["P_cap_W"]
    assert abs(eta_cap - T3["eta_cap"]) < 0.01 * T3["eta_cap"]
    assert abs(eta_coil - T3["eta_coil"]) < 0.01 * T3["eta_coil"]


def _exact_loads(fc, Ch):
    """A stand-in for the surrogate that predicts the loads exactly: no
    plasma reaction voltage, I_cap = i w C_h V of the state's turn voltages
    (feature layout: I_k re, im, then V_k re, im, pressure, moments)."""
    def predict(f):
        V = f[10:20:2] + 1j * f[11:20:2]
        ic = 1j * fc.omega * Ch @ V
        return np.concatenate([np.zeros(10), np.column_stack([ic.real, ic.imag]).ravel()])
    return predict


@pytest.mark.parametrize("offset", [0.0, 0.01])
def test_t3_surrogate_update_with_exact_loads_lands_on_the_coupled_fixed_point(offset):
    # with the exact load map the inner fixed point is the stationary state of
    # the coupled network, which the paper tabulates (Table t7phasors, h = 1 mm);
    # a constant prediction offset (1 %, inside the 2 % gate) is cancelled
    # exactly by the correction y_n - yhat(x^n)
    t3 = _Test3()
    fc = t3.fc
    Ch = t3.cap_matrix()
    exact = _exact_loads(fc, Ch)
    off = offset * exact(fc.features(fc.x, 0.0, np.zeros(8)))
    rep = fc.update_surrogate(t3.harmonics(), 0.0, np.zeros(8), lambda f: exact(f) + off, tol=1e-12, max_iter=60)
    assert rep["sur_used"] == 1 and abs(rep["sur_err"] - offset) < 1e-9 and rep["sur_iters"] < 60
    assert np.max(np.abs(fc.x - T3_FIELD)) < 6e-9 * np.max(np.abs(T3_FIELD[6:]))


def test_t3_surrogate_update_beyond_the_error_gate_is_the_plain_update():
    a, b = _Test3(), _Test3()
    exact = _exact_loads(a.fc, a.cap_matrix())
    rep = a.fc.update_surrogate(a.harmonics(), 0.0, np.zeros(8), lambda f: 1.05 * exact(f))
    b.fc.update(b.harmonics())
    assert rep["sur_used"] == 0 and abs(rep["sur_err"] - 0.05) < 1e-9
    assert np.array_equal(a.fc.x, b.fc.x)


def test_t3_surrogate_update_applies_the_second_half_mean_when_tol_is_not_met():
    # alpha = 1 and exact loads: the inner iterates are the coupled recurrence
    # x_(i+1) = A^-1 b(V_i); six iterates with a tolerance never met apply the
    # mean of iterates 4 to 6
    t3 = _Test3()
    fc = t3.fc
    Ch = t3.cap_matrix()
    xs = [fc.x.copy()]
    for _ in range(6):
        icap = 1j * fc.omega * Ch @ xs[-1][6:]
        xs.append(np.linalg.solve(fc.A, C.network_rhs(fc.vg, icap, np.zeros(5))))
    rep = fc.update_surrogate(t3.harmonics(), 0.0, np.zeros(8), _exact_loads(fc, Ch), tol=1e-300, max_iter=6)
    assert rep["sur_used"] == 1 and rep["sur_iters"] == 6
    mean = np.mean(xs[4:7], axis=0)
    assert np.max(np.abs(fc.x - mean)) < 1e-10 * np.max(np.abs(mean))
    # the iterates have not settled: the last one still differs from the mean
    assert np.max(np.abs(xs[6] - mean)) > 1e-6 * np.max(np.abs(mean))


def test_t3_rotation_equivariance():
    a, b = _Test3(), _Test3()
    b.fc.p.vg_phase = math.radians(37.0)
    b.fc.vg = 100.0 * complex(math.cos(b.fc.p.vg_phase), math.sin(b.fc.p.vg_phase))
    b.fc.x = np.linalg.solve(b.fc.A, C.network_rhs(b.fc.vg, np.zeros(5), np.zeros(5)))
    for _ in range(2):
        a.period(nrf=64)
        b.period(nrf=64)
    rot = complex(math.cos(math.radians(37.0)), math.sin(math.radians(37.0)))
    assert np.max(np.abs(b.fc.x - rot * a.fc.x)) < 1e-12 * np.max(np.abs(a.fc.x))


# ---------------------------------------------------------------------------
# Closed forms and invariants
# ---------------------------------------------------------------------------
def test_shape_normalisation_and_signs():
    tag = np.full((9, 9), -1, np.int32)
    tag[3:5, 2:5] = 1
    tag[6, 6] = 2
    g, area = C.shape_functions(tag, 2, 1e-3, 2e-3, sign=[1, -1])
    assert np.allclose(area, [6 * 2e-6, 2e-6])
    assert abs(g[0].sum() * 2e-6 - 1) < 1e-15 and abs(g[1].sum() * 2e-6 + 1) < 1e-15
    with pytest.raises(ValueError):
        C.shape_functions(tag, 3, 1e-3, 2e-3)


def test_skin_resistance_limits():
    w, mu0 = 2 * math.pi * 13.56e6, 4e-7 * math.pi
    rho = 1.68e-8 * (1 + 3.93e-3 * 80.0)
    delta = math.sqrt(2 * rho / (w * mu0))
    # wire thinner than the skin depth: DC resistance of the full section
    A = math.pi * (0.5 * delta) ** 2
    r = C.skin_resistance(0.05, A, w, mu0, 1.68e-8, 3.93e-3, 100.0)
    assert abs(r - rho * 2 * math.pi * 0.05 / A) < 1e-12 * r
    # thick wire: conducting annulus of depth delta
    rw = 50 * delta
    r = C.skin_resistance(0.05, math.pi * rw ** 2, w, mu0, 1.68e-8, 3.93e-3, 100.0)
    ann = math.pi * (2 * rw * delta - delta ** 2)
    assert abs(r - rho * 2 * math.pi * 0.05 / ann) < 1e-12 * r


def _random_network(N=4, seed=3):
    rng = np.random.default_rng(seed)
    w = 2 * math.pi * 13.56e6
    B = rng.normal(size=(N, N))
    M = (B @ B.T + N * np.eye(N)) * 1e-7
    Zt = 1j * w * M + np.diag(rng.uniform(0.1, 1.0, N))
    cs = rng.uniform(0, 5e-12, N)
    Zs = C.z_source(w, 50.0, 1.0, 1e-7, 2e-10)
    icap = rng.normal(size=N) + 1j * rng.normal(size=N)
    vp = rng.normal(size=N) + 1j * rng.normal(size=N)
    return w, Zs, Zt, cs, icap, vp


def test_network_solution_zeroes_the_residuals():
    w, Zs, Zt, cs, icap, vp = _random_network()
    N = len(cs)
    A = C.network_matrix(Zs, Zt, cs, w)
    x = np.linalg.solve(A, C.network_rhs(150.0, icap, vp))
    rI, rV = C.network_residuals(x, 150.0, Zs, Zt, cs, w, icap, vp)
    assert np.max(np.abs(rI)) < 1e-13 * abs(x[0]) and np.max(np.abs(rV)) < 1e-13 * 150.0
    # a perturbed state leaves a residual of the perturbation's size
    y = x.copy()
    y[1 + N] += 1.0
    rI, rV = C.network_residuals(y, 150.0, Zs, Zt, cs, w, icap, vp)
    assert abs(rV[0] + 1.0) < 1e-12
    # series matching branch
    assert Zs == complex(51.0, w * 1e-7 - 1 / (w * 2e-10))
    assert C.z_source(w, 50.0, 0.0, 0.0, 0.0) == 50.0


def test_controller_fixed_point_and_limits():
    mk = lambda **kw: C.Controller(**{**dict(p_target=60.0, gamma=0.3, n_trend=1.0, eps_p=1e-3, alpha_v=0.5,
                                             f_step=0.1, v_min=1.0, v_max=5000.0), **kw})
    c = mk()
    v, pf, pc = c.step(200.0, 60.0)
    assert v == 200.0 and pf == 60.0 and pc == 60.0
    assert mk().step(200.0, 1e-9)[0] == pytest.approx(220.0, rel=1e-15)      # +10 % step limit
    assert mk().step(200.0, 1e9)[0] == pytest.approx(180.0, rel=1e-15)       # -10 % step limit
    assert mk(v_max=210.0).step(200.0, 1e-9)[0] == 210.0
    assert mk(v_min=190.0).step(200.0, 1e9)[0] == 190.0
    # a load drawing P = k V^2: without filter, trend and step limit the
    # controller lands on the target in one step
    c = mk(gamma=1.0, n_trend=0.0, alpha_v=1.0, f_step=10.0)
    k = 60.0 / 300.0 ** 2
    v = 120.0
    v = c.step(v, k * v * v)[0]
    assert abs(k * v * v - 60.0) < 1e-12
    # the trend term extrapolates a rising filtered power
    c = mk(gamma=1.0, f_step=10.0, alpha_v=1.0)
    c.step(100.0, 30.0)
    v, pf, pc = c.step(100.0, 40.0)
    assert pc == 50.0 and v == pytest.approx(100.0 * math.sqrt(60.0 / 50.0), rel=1e-15)


def test_plasma_current_shaped_like_a_turn_induces_z_vac():
    """A plasma current with the spatial shape of turn l and phasor I gives
    V_p,k = Z_vac,kl I (Eqs. helmholtz_two_real, vpind, zvac): checks the
    cosine/sine bookkeeping of J and E and the sign of the projection."""
    from paper_2609_15043_amd import workloads as W
    wl = W.cell(n_per_species=10)
    fc = C.FieldCircuit(wl.nr, wl.nz, wl.dr, wl.dz, wl.node_tag, wl.eps_cell, wl.freq, W.EPS0, wl.circuit)
    Iph = 1.7 - 0.6j                       # I = I_c - i I_s
    l = 2
    shape = (wl.nz + 1, wl.nr + 1)
    gl = fc.g[l].reshape(shape)
    # node currents I_node = J V_node with J(t) = Re(I g_l e^{iwt}): J_c = I_c g_l, J_s = I_s g_l
    Jc, Js = Iph.real * gl * fc.vnode, -Iph.imag * gl * fc.vnode
    fc.plasma_fields(Jc, Js)
    vp = C.v_p_ind(fc.g, fc.Ec_p, fc.Es_p, fc.wts)
    ref = fc.Zvac[:, l] * Iph
    assert np.max(np.abs(vp - ref)) < 1e-12 * np.max(np.abs(ref))
    # and composing the turn-l field gives the same node field as the plasma current
    Ec, Es = C.compose(np.zeros(shape), np.zeros(shape), fc.U, np.eye(5)[l] * Iph)
    assert np.max(np.abs(Ec - fc.Ec_p)) < 1e-12 * np.max(np.abs(Ec))
    assert np.max(np.abs(Es - fc.Es_p)) < 1e-12 * np.max(np.abs(Es))


def test_helmholtz_operator_reproduces_cylindrical_modes():
    """K applied to sin(pi z / Z) J1(k R) (a Bessel mode vanishing on the
    axis and at R = R0) equals -(pi^2/Z^2 + k^2) u / (mu0 w) to second order
    in h away from the axis (R >= R0/4; next to the axis the 1/R factor
    leaves a first-order local error): the truncation error drops by ~4 per
    halving of h."""
    from scipy import special
    errs = []
    for n in (32, 64, 128):
        Zl, R0 = 0.2, 0.1
        k = special.jn_zeros(1, 1)[0] / R0
        h_r, h_z = R0 / n, Zl / (2 * n)
        tag = np.full((2 * n + 1, n + 1), -1, np.int32)
        tag[0, :] = tag[2 * n, :] = 0
        tag[:, n] = 0
        H = C.Helmholtz(n, 2 * n, h_r, h_z, tag == 0, 1e7, 1e-6)
        z = np.arange(2 * n + 1) * h_z
        R = np.arange(n + 1) * h_r
        u = np.outer(np.sin(math.pi * z / Zl), special.j1(k * R))
        Ku = H.apply_K(u)
        ref = -(math.pi ** 2 / Zl ** 2 + k ** 2) * u / (1e-6 * 1e7)
        m = ~H.dmask.reshape(u.shape) & (R[None, :] >= R0 / 4)
        errs.append(np.max(np.abs(Ku - ref)[m]) / np.max(np.abs(ref)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs
