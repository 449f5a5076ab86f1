"""Full-size parity in the configuration the benchmark times: the large
workload (256 x 512 cells, 3.2e7 electrons + 3.2e7 Ar+, argon 50 mTorr,
quartz window, coil turns as Dirichlet conductors), fused pass, electron
sort every 16 steps and ion sort every 32, in both precisions the benchmark
runs (FP32-mixed particles, and the plain FP64 path).

Both sides load their own particles (the same counter-based draws keyed by
particle id) and solve phi^0, then take one whole step.  The oracle (FP64,
C particle loops, sparse direct Poisson) processes every particle, so the
whole state is compared, not a sample: the loaded particles, phi^0, and
after the step every particle, the candidate and event counts, the node
charge, the window surface charge and phi^1.  Prescribed inductive field
(the circuit update is tested on the coil cell).

Tolerances as for the single-step cases: mixed 1e-5 normwise per array
(particles, I, Q, the window charge and phi) and at most 1e-4 of the
particles on the other side of an FP32 rounding decision; FP64 1e-12 with
every discrete outcome exact.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


TOL = {"mixed": (1e-5, 1e-5), "fp64": (1e-12, 1e-12)}


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_large_step_matches_oracle(prec):
    _need_gpu()
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    from oracle import pic as O
    from test_gpu_parity import _compare_particles, rel
    wl = W.large(circuit=False)
    tp, tg = TOL[prec]
    say(f"[gpu] large workload, {prec}, fused: load, phi0 and one step against the oracle (6.4e7 particles)")
    ora = O.OraclePIC(wl)
    cfg, keep = pp.config_from_workload(wl, precision=prec, fuse=True, load=True, sort_every=16,
                                        sort_every_ion=32)
    ctx = pp.pic_init(cfg, keep)
    res = {}
    for s in range(2):
        errs, mism = _compare_particles(pp.pic_get_particles(ctx, s), ora.live(s), prec, f"load s={s}")
        res.update({f"load_{k}{s}": v for k, v in errs.items()})
    res["phi0"] = rel(pp.pic_get_grid(ctx, pp.PIC_GRID_PHI), ora.phi)
    assert res["phi0"] <= tg, res["phi0"]
    say("    load and phi0: " + " ".join(f"{k}={v:.1e}" for k, v in res.items()))

    n0 = 0
    pp.pic_gather_push(ctx, n0)
    pp.harmonic_accumulate(ctx, n0)
    gI = pp.pic_get_grid(ctx, pp.PIC_GRID_CURRENT)
    pp.mcc_collide(ctx, n0)
    pp.pic_deposit(ctx, n0 + 1)
    info = pp.poisson_solve_rz(ctx, n0 + 1, info=True)
    ora.step()
    res = {"I": rel(gI, ora.I)}
    assert res["I"] <= tp, res["I"]
    for s in range(2):
        errs, mism = _compare_particles(pp.pic_get_particles(ctx, s), ora.live(s), prec, f"step s={s}")
        res.update({f"{k}{s}": v for k, v in errs.items()})
        res[f"idmismatch{s}"] = mism
    st = pp.pic_get_stats(ctx)
    for s in range(2):
        slack = 0 if prec == "fp64" else max(2, 1e-4 * ora.counts[s][0])
        assert abs(st.candidates[s] - ora.counts[s][0]) <= slack, s
        for k in range(2 if s else 3):
            assert abs(st.events[s][k] - ora.counts[s][k + 1]) <= slack, (s, k)
    res["Q"] = rel(pp.pic_get_grid(ctx, pp.PIC_GRID_CHARGE), ora.Q)
    res["surf"] = rel(pp.pic_get_grid(ctx, pp.PIC_GRID_SURFACE), ora.surf)
    res["phi"] = rel(pp.pic_get_grid(ctx, pp.PIC_GRID_PHI), ora.phi)
    say("    step: " + " ".join(f"{k}={v:.1e}" if isinstance(v, float) else f"{k}={v}" for k, v in res.items())
        + f" mg_cycles={info['cycles']} candidates {st.candidates[0]}/{st.candidates[1]}")
    assert info["converged"], info
    for k in ("Q", "surf", "phi"):
        assert res[k] <= tg, (k, res[k])
    assert st.mg_unconverged == 0
