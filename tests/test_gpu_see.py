"""GPU parity of ion-induced secondary electron emission (the GEC cell's
inherited module: constant yield per ion absorbed at a metal wall,
flux-weighted Maxwellian electron at the ion's position before the move)
against the oracle, through the C ABI.

The small instance with hot ions (200 eV), dt = 1 ns and 1e13 m^-3 sends some
thirty ions a step to the bottom, top and outer walls; with a yield of 0.5
about half of them emit.  Three whole steps from the same particles: every
particle of both species (ids, candidate steps, positions, velocities), the
emitted count, the node charge and the potential, at the single-step bars
(1e-12 FP64 with every discrete outcome exact; 1e-5 FP32-mixed).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    d = float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if np.size(a) else 0.0
    s = float(np.max(np.abs(b))) if np.size(b) else 0.0
    return d / s if s > 0 else d


def _workload(gamma):
    from paper_2609_15043_amd import workloads as W
    wl = W.small(n_per_species=100_000)
    wl.dt, wl.n0 = 1e-9, 1e13
    wl.temp_ev = (3.0, 200.0)
    wl.see_gamma, wl.see_temp_ev = gamma, 2.0
    return wl


def _compare(g, o, prec, label):
    if prec == "fp64":
        assert np.array_equal(g["id"], o["id"]), f"{label}: id sets differ ({len(g['id'])} vs {len(o['id'])})"
        gi = oi = np.arange(len(o["id"]))
    else:
        common, gi, oi = np.intersect1d(g["id"], o["id"], assume_unique=True, return_indices=True)
        mism = len(g["id"]) + len(o["id"]) - 2 * len(common)
        assert mism <= max(2, 1e-4 * len(o["id"])), f"{label}: {mism} ids differ"
    nx = int(np.sum(g["next"][gi] != o["next"][oi]))
    assert nx <= (0 if prec == "fp64" else max(2, 1e-4 * len(oi))), f"{label}: {nx} candidate steps differ"
    errs = {}
    for k in ("R", "z", "vr", "vt", "vz"):
        a, b = g[k][gi], o[k][oi]
        if prec == "mixed":
            keep = np.abs(a - b) <= 1e-3 * np.max(np.abs(b))
            assert np.sum(~keep) <= max(2, 1e-4 * len(b)), f"{label}: {np.sum(~keep)} outliers in {k}"
            a, b = a[keep], b[keep]
        errs[k] = rel(a, b)
        assert errs[k] <= TOL[prec], f"{label}: {k} rel err {errs[k]:.3e}"
    return errs


@pytest.mark.parametrize("prec,fuse", [("fp64", True), ("fp64", False), ("mixed", True)])
def test_secondary_emission_steps_match_oracle(prec, fuse):
    _need_gpu()
    import paper_2609_15043_amd.phasorpic as pp
    from oracle import pic as O
    wl = _workload(0.5)
    say(f"[gpu] secondary emission, small hot-ion instance, gamma 0.5, {prec} fuse={fuse}")
    ora = O.OraclePIC(wl)
    cfg, keep = pp.config_from_workload(wl, precision=prec, fuse=fuse, load=False)
    ctx = pp.pic_init(cfg, keep)
    for s in range(2):
        pp.pic_set_particles(ctx, s, ora.live(s))
    pp.pic_set_phi(ctx, ora.phi)
    pp.pic_set_step(ctx, 0)
    emitted = 0
    for n in range(3):
        pp.pic_gather_push(ctx, n)
        pp.harmonic_accumulate(ctx, n)
        pp.mcc_collide(ctx, n)
        pp.pic_deposit(ctx, n + 1)
        info = pp.poisson_solve_rz(ctx, n + 1, info=True)
        ora.step()
        emitted += ora.see_emitted
        st = pp.pic_get_stats(ctx)
        res = {}
        for s in range(2):
            res.update({f"{k}{s}": v for k, v in _compare(pp.pic_get_particles(ctx, s), ora.live(s), prec,
                                                          f"step {n} s={s}").items()})
        res["Q"] = rel(pp.pic_get_grid(ctx, pp.PIC_GRID_CHARGE), ora.Q)
        res["phi"] = rel(pp.pic_get_grid(ctx, pp.PIC_GRID_PHI), ora.phi)
        say(f"    step {n}: emitted {ora.see_emitted} of {len(ora.see_absorbed)} ions at metal walls "
            f"(GPU total {st.see_emitted}); " + " ".join(f"{k}={v:.1e}" for k, v in res.items()))
        assert info["converged"], info
        if prec == "fp64":
            assert st.see_emitted == emitted
        else:
            assert abs(st.see_emitted - emitted) <= 2
        for k, v in res.items():
            assert v <= TOL[prec], (n, k, v)
    assert emitted > 30


def test_secondary_emission_off_is_the_plain_step():
    """see_gamma = 0 carves no queue and leaves the step as it was: the same
    particles after a step as a context without the option."""
    _need_gpu()
    import paper_2609_15043_amd.phasorpic as pp
    from oracle import pic as O
    say("[gpu] secondary emission off")
    wl = _workload(0.0)
    ora = O.OraclePIC(wl)
    cfg, keep = pp.config_from_workload(wl, precision="fp64", load=False)
    ctx = pp.pic_init(cfg, keep)
    for s in range(2):
        pp.pic_set_particles(ctx, s, ora.live(s))
    pp.pic_set_phi(ctx, ora.phi)
    pp.pic_set_step(ctx, 0)
    pp.pic_gather_push(ctx, 0)
    pp.harmonic_accumulate(ctx, 0)
    pp.mcc_collide(ctx, 0)
    pp.pic_deposit(ctx, 1)
    pp.poisson_solve_rz(ctx, 1)
    ora.step()
    assert pp.pic_get_stats(ctx).see_emitted == 0
    for s in range(2):
        _compare(pp.pic_get_particles(ctx, s), ora.live(s), "fp64", f"s={s}")
