"""Pins of the oracle's grid part: the finite-volume RZ Poisson operator
(Eqs. poisson with chi = 0, epseff, areas, axis_electrostatic_bc), the turn
charge extraction (Eq. facecharge), and the period accumulators (Eqs.
fourier, icap, pind, pcap, pcap_phasor, pcap_quadrature)."""
import math

import numpy as np
import pytest

from oracle import pic
from paper_2609_15043_amd import workloads as W


def _gl(n=6):
    return np.polynomial.legendre.leggauss(n)


def _integrate(f, a, b, n=6):
    if b <= a:
        return 0.0
    x, w = _gl(n)
    t = 0.5 * (b - a) * x + 0.5 * (b + a)
    return 0.5 * (b - a) * np.sum(w * f(t))


def _mms_charge(nr, nz, rmax, zmax, dphi_dR, dphi_dz, eps_of_z, z_split):
    """Exact charge in each control volume: -eps0 times the outward flux of
    eps grad(phi) through its faces, by Gauss-Legendre quadrature on each
    smooth piece (faces crossing z_split are integrated in two parts)."""
    dr, dz = rmax / nr, zmax / nz
    Q = np.zeros((nz + 1, nr + 1))
    for i in range(1, nz):
        for j in range(0, nr):
            R = j * dr
            rlo, rhi = max(0.0, R - dr / 2), R + dr / 2
            zlo, zhi = i * dz - dz / 2, i * dz + dz / 2
            flux = 0.0
            for zf, sgn in ((zhi, 1.0), (zlo, -1.0)):
                flux += sgn * eps_of_z(zf) * _integrate(lambda r: dphi_dz(r, zf) * 2 * math.pi * r, rlo, rhi)
            pieces = [(zlo, zhi)]
            if zlo < z_split < zhi:
                pieces = [(zlo, z_split), (z_split, zhi)]
            for (a, b) in pieces:
                em = eps_of_z(0.5 * (a + b))
                flux += em * _integrate(lambda z: dphi_dR(rhi, z), a, b) * 2 * math.pi * rhi
                if rlo > 0:
                    flux -= em * _integrate(lambda z: dphi_dR(rlo, z), a, b) * 2 * math.pi * rlo
            Q[i, j] = -W.EPS0 * flux
    return Q


def _mms_error(nr, nz, dielectric):
    rmax, zmax = 0.1, 0.2
    k = math.pi / (2 * rmax)
    zd = zmax / 2
    e1, e2 = (1.0, 3.8) if dielectric else (1.0, 1.0)
    # f(z) = z below z_d; quadratic in (Z - z) above, continuous value and
    # continuous eps f' at z_d; zero at z = 0 and z = Z.
    L = zmax - zd
    # gamma L + delta L^2 = zd ; -gamma - 2 delta L = e1/e2
    A = np.array([[L, L * L], [-1.0, -2 * L]])
    gam, dlt = np.linalg.solve(A, [zd, e1 / e2])

    def f(z):
        return np.where(z < zd, z, gam * (zmax - z) + dlt * (zmax - z) ** 2)

    def fp(z):
        return np.where(z < zd, 1.0, -gam - 2 * dlt * (zmax - z))

    phi = lambda R, z: f(z) * np.cos(k * R)
    dR = lambda R, z: -k * f(z) * np.sin(k * R)
    dZ = lambda R, z: fp(z) * np.cos(k * R)
    eps_z = lambda z: e1 if z < zd else e2
    Q = _mms_charge(nr, nz, rmax, zmax, dR, dZ, eps_z, zd)
    eps_cell = np.ones((nz, nr))
    eps_cell[nz // 2:, :] = e2
    eps_cell[: nz // 2, :] = e1
    tag = np.full((nz + 1, nr + 1), -1, np.int32)
    tag[0, :] = tag[nz, :] = 0
    tag[:, nr] = 0
    P = pic.Poisson(nr, nz, rmax / nr, zmax / nz, eps_cell, tag, W.EPS0)
    Rn = np.arange(nr + 1) * rmax / nr
    zn = np.arange(nz + 1) * zmax / nz
    exact = phi(Rn[None, :], zn[:, None])
    num = P.solve(Q, [], ground=exact)
    return np.max(np.abs(num - exact)) / np.max(np.abs(exact))


@pytest.mark.parametrize("dielectric", [False, True])
def test_poisson_mms_second_order(dielectric):
    """Manufactured solution with the axis (Neumann), Dirichlet walls and,
    optionally, a dielectric jump eps_r 1 -> 3.8 at mid height: the nodal
    error falls by ~4 per grid halving."""
    errs = [_mms_error(n, 2 * n, dielectric) for n in (8, 16, 32)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 2e-3
    assert min(orders) > 1.8, (errs, orders)


def test_discrete_gauss_law_and_turn_charges():
    """Summing every equation of the solved system: the free charge plus the
    charge on all conductors (turns and grounded metal, from the operator's
    face fluxes) is zero; with zero potentials and no charge every turn
    charge vanishes; turn charges are linear in the turn potentials."""
    wl = W.cell()
    P = pic.Poisson(wl.nr, wl.nz, wl.dr, wl.dz, wl.eps_cell, wl.node_tag, W.EPS0)
    rng = np.random.default_rng(0)
    Q = np.zeros((wl.nz + 1, wl.nr + 1))
    Q[1:wl.ip, :-1] = rng.normal(0, 1e-13, (wl.ip - 1, wl.nr))
    V = np.array([300.0, -120.0, 50.0, 10.0, 200.0])
    phi = P.solve(Q, V)
    Qk = P.turn_charges(phi, 5)
    ph = phi.reshape(-1)
    tag = wl.node_tag.reshape(-1)
    ga = (tag[P.fa] == 0) & (tag[P.fb] != 0)
    gb = (tag[P.fb] == 0) & (tag[P.fa] != 0)
    Qg = np.sum(P.fc[ga] * (ph[P.fa[ga]] - ph[P.fb[ga]])) + np.sum(P.fc[gb] * (ph[P.fb[gb]] - ph[P.fa[gb]]))
    free_Q = Q.reshape(-1)[tag < 0].sum()
    scale = np.abs(Qk).sum() + abs(Qg)
    assert abs(free_Q + Qk.sum() + Qg) < 1e-12 * scale
    assert np.all(P.turn_charges(P.solve(0 * Q, 0 * V), 5) == 0)
    # linearity: Q_k(V1 + V2) = Q_k(V1) + Q_k(V2) at zero space charge
    V2 = np.array([-40.0, 70.0, 0.0, 15.0, -5.0])
    a = P.turn_charges(P.solve(0 * Q, V), 5)
    b = P.turn_charges(P.solve(0 * Q, V2), 5)
    c = P.turn_charges(P.solve(0 * Q, V + V2), 5)
    np.testing.assert_allclose(c, a + b, rtol=1e-9, atol=1e-12 * np.abs(c).max())
    # a capacitance matrix from unit potentials is symmetric (reciprocity of
    # the symmetric FV operator)
    C = np.stack([P.turn_charges(P.solve(0 * Q, np.eye(5)[k]), 5) for k in range(5)], 1)
    np.testing.assert_allclose(C, C.T, rtol=1e-9, atol=1e-9 * np.abs(C).max())
    assert np.all(np.diag(C) > 0) and np.all(C - np.diag(np.diag(C)) <= 0)


def test_e_from_phi_axis_and_linear_potential():
    """E = -grad phi is exact for a linear potential; E_r = 0 on the axis."""
    nr, nz, dr, dz = 6, 9, 0.01, 0.02
    R = np.arange(nr + 1) * dr
    z = np.arange(nz + 1) * dz
    phi = 3.0 * z[:, None] - 7.0 * R[None, :] + 1.0
    Er, Ez = pic.e_from_phi(phi, dr, dz)
    np.testing.assert_allclose(Ez, -3.0, rtol=1e-12)
    np.testing.assert_allclose(Er[:, 1:], 7.0, rtol=1e-12)
    assert np.all(Er[:, 0] == 0)


# ---------------------------------------------------------------------------
# Period accumulators
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N", [3, 7, 400, 2000])
def test_fourier_projection_of_a_sinusoid_is_exact(N):
    """X_n = A cos th_n + B sin th_n projects to (X_c, X_s) = (A, B) and the
    charge phasor to I_cap = i w Q_hat = w Q_s + i w Q_c (Eqs. fourier, icap)."""
    H = pic.Harmonics((2, 3), 2, N, 13.56e6)
    A = np.array([[1.0, -2.0, 0.5], [3.0, 0.0, -1.0]])
    B = np.array([[0.3, 4.0, -2.5], [0.0, 1.0, 2.0]])
    qa, qb = np.array([1e-12, -3e-12]), np.array([2e-12, 5e-13])
    for n in range(5 * N, 6 * N):
        th = 2 * math.pi * (n % N) / N
        H.add(n, A * math.cos(th) + B * math.sin(th), np.zeros((2, 3)), qa * math.cos(th) + qb * math.sin(th),
              np.zeros(2))
    r = H.finalize([0.0, 0.0], [0.0, 0.0])
    np.testing.assert_allclose(r["Jc"], A, atol=1e-14 * N)
    np.testing.assert_allclose(r["Js"], B, atol=1e-14 * N)
    w = 2 * math.pi * 13.56e6
    np.testing.assert_allclose(r["Icap"], w * qb + 1j * w * qa, rtol=1e-12)


@pytest.mark.parametrize("N", [5, 64, 2000])
def test_pcap_quadrature_identity(N):
    """For a purely fundamental turn voltage and ANY charge samples, the
    periodic trapezoid P_cap equals sin(2pi/N)/(2pi/N) times the phasor
    power (Eq. pcap_quadrature); a lossless capacitor Q = C V gives 0."""
    rng = np.random.default_rng(N)
    K = 3
    Vc, Vs = rng.normal(0, 100, K), rng.normal(0, 100, K)
    f = 13.56e6
    H = pic.Harmonics((1, 1), K, N, f)
    H2 = pic.Harmonics((1, 1), K, N, f)
    Cm = np.array([[2.0, -0.5, -0.1], [-0.5, 3.0, -0.4], [-0.1, -0.4, 1.5]]) * 1e-12
    for n in range(N):
        th = 2 * math.pi * n / N
        V = Vc * math.cos(th) + Vs * math.sin(th)
        H.add(n, np.zeros((1, 1)), np.zeros((1, 1)), rng.normal(0, 1e-10, K), V)
        H2.add(n, np.zeros((1, 1)), np.zeros((1, 1)), Cm @ V, V)
    r = H.finalize(Vc, Vs)
    x = 2 * math.pi / N
    assert r["P_cap"] == pytest.approx(math.sin(x) / x * r["P_cap_ph"], rel=1e-10, abs=1e-18)
    r2 = H2.finalize(Vc, Vs)
    scale = 0.5 * 2 * math.pi * f * np.abs(Cm).sum() * (np.abs(Vc) + np.abs(Vs)).max() ** 2
    assert abs(r2["P_cap"]) < 1e-12 * scale and abs(r2["P_cap_ph"]) < 1e-12 * scale


def test_sample_count_gate_and_pind():
    """The update is rejected unless exactly N_RF samples were taken; P_ind
    is the period mean of sum_nodes I E_theta (Eq. pind)."""
    N = 10
    H = pic.Harmonics((2, 2), 1, N, 1.0)
    tot = 0.0
    rng = np.random.default_rng(1)
    for n in range(N - 1):
        I, E = rng.normal(size=(2, 2)), rng.normal(size=(2, 2))
        tot += float((I * E).sum())
        H.add(n, I, E, np.zeros(1), np.zeros(1))
    assert H.finalize([0.0], [0.0]) is None
    I, E = rng.normal(size=(2, 2)), rng.normal(size=(2, 2))
    tot += float((I * E).sum())
    H.add(N - 1, I, E, np.zeros(1), np.zeros(1))
    r = H.finalize([0.0], [0.0])
    assert r["P_ind"] == pytest.approx(tot / N, rel=1e-14)


def test_phase_closure():
    """N_RF = nint(1/(f dt)) with closure |f dt N - 1| < 1e-10 (Eqs. nrf,
    phaseclosure): the 5e-11 s step at 13.56 MHz does not close, 1/(2000 f)
    does."""
    assert pic.n_rf(13.56e6, 5e-11) == (1475, False)
    assert pic.n_rf(13.56e6, 1 / (2000 * 13.56e6)) == (2000, True)
