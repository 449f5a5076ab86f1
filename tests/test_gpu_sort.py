"""The cell sort keeps every particle and its state: three steps with both
species sorted before every push, against the oracle (which never sorts;
its particle order plays no part in what a step computes).

Coil cell (128 x 256 cells) with 2e6 particles per species, so that a
species spans about 2000 sort chunks of 1024 particles, several per CU and
more than fit on the device at once.  The first sort takes the load order (random cells per chunk: nearly every particle
goes to its global position directly), the later ones an array that is
sorted but for one step's moves and births (nearly every particle is staged
in the block's cell window).  Tolerances as for one step: FP64 1e-12 with
every discrete outcome exact, mixed 1e-5 normwise with at most 1e-4 of the
particles on the other side of an FP32 rounding decision.
"""
import sys

import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sorted_steps_match_oracle(prec):
    _need_gpu()
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    from oracle import pic as O
    from test_gpu_parity import _compare_particles, rel
    tol = {"fp64": 1e-11, "mixed": 1e-4}[prec]
    wl = W.cell(n_per_species=2_000_000, circuit=False)
    say(f"[gpu] coil cell 2e6/species {prec}: 3 steps, both species sorted before each push after the first")
    cfg, keep = pp.config_from_workload(wl, precision=prec, load=True, sort_every=1, sort_every_ion=1)
    ctx = pp.pic_init(cfg, keep)
    pp.pic_timing(ctx, True)
    ora = O.OraclePIC(wl)
    for n in range(3):
        pp.step(ctx, n)
        ora.step()
    st = pp.pic_get_stats(ctx)
    assert st.sort_count == 4, st.sort_count
    res = {}
    for s in range(2):
        errs, mism = _compare_particles(pp.pic_get_particles(ctx, s), ora.live(s), prec, f"s={s}")
        res.update({f"{k}{s}": v for k, v in errs.items()})
        res[f"idmismatch{s}"] = mism
    res["Q"] = rel(pp.pic_get_grid(ctx, pp.PIC_GRID_CHARGE), ora.Q)
    res["phi"] = rel(pp.pic_get_grid(ctx, pp.PIC_GRID_PHI), ora.phi)
    say("    " + " ".join(f"{k}={v:.1e}" if isinstance(v, float) else f"{k}={v}" for k, v in res.items()))
    assert res["Q"] <= tol, res["Q"]
    assert res["phi"] <= tol, res["phi"]
