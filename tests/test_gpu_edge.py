"""Edge cases on the GPU: a grid whose multigrid hierarchy is not a power of
two, and the error paths of the C ABI (call order, incomplete RF period,
birth buffer and particle capacity exhausted).  The error conditions are
produced from the host (call sequences and small capacities); every kernel
exits normally and the library reports the condition through its status.
"""
import dataclasses
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


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_single_step_ragged_grid(prec):
    """One step on 40 x 70 cells with 50,001 particles per species, against
    the oracle at the single-step tolerances."""
    _need_gpu()
    from test_gpu_parity import _step_case
    _step_case("ragged", prec, True, n0=173)


def _ctx(wl, **kw):
    import paper_2609_15043_amd.phasorpic as pp
    cfg, keep = pp.config_from_workload(wl, precision="mixed", load=True, **kw)
    return pp.pic_init(cfg, keep)


def test_call_order_violations_are_rejected():
    _need_gpu()
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    say("[gpu] call-order violations")
    ctx = _ctx(W.small(n_per_species=10_000))
    with pytest.raises(pp.PicError) as e:
        pp.mcc_collide(ctx, 0)          # before the push of step 0
    assert e.value.status == pp.PIC_ESTATE
    pp.pic_gather_push(ctx, 0)
    with pytest.raises(pp.PicError) as e:
        pp.pic_gather_push(ctx, 0)      # the same step twice
    assert e.value.status == pp.PIC_ESTATE
    with pytest.raises(pp.PicError) as e:
        pp.pic_gather_push(ctx, 2)      # a step skipped
    assert e.value.status == pp.PIC_ESTATE
    pp.harmonic_accumulate(ctx, 0)
    with pytest.raises(pp.PicError) as e:
        pp.harmonic_accumulate(ctx, 0)  # two samples for one step
    assert e.value.status == pp.PIC_ESTATE
    # a rejected call leaves the context usable
    pp.mcc_collide(ctx, 0)
    pp.pic_deposit(ctx, 1)
    pp.poisson_solve_rz(ctx, 1)
    pp.pic_gather_push(ctx, 1)
    pp.pic_sync(ctx)


def test_incomplete_period_is_rejected_and_state_kept():
    _need_gpu()
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    say("[gpu] period update before N_RF samples")
    wl = W.cell(n_per_species=1000)
    wl.dt = 1.0 / (16 * wl.freq)
    cfg, keep = pp.config_from_workload(wl, precision="fp64", load=False)
    ctx = pp.pic_init(cfg, keep)
    before = pp.pic_get_circuit(ctx)["x"].copy()
    for n in range(5):
        pp.step(ctx, n)
        pp.poisson_solve_rz(ctx, n + 1)
    st, rep, _, _ = pp.circuit_period_update(ctx)
    assert st == pp.PIC_EPHASE and not rep["accepted"]
    assert np.array_equal(pp.pic_get_circuit(ctx)["x"], before)


def _hot_small(n, te=40.0):
    from paper_2609_15043_amd import workloads as W
    wl = W.small(n_per_species=n)
    return dataclasses.replace(wl, temp_ev=(te, wl.temp_ev[1]))


def _run_until_error(ctx, steps):
    import paper_2609_15043_amd.phasorpic as pp
    for n in range(steps):
        pp.step(ctx, n)
        pp.poisson_solve_rz(ctx, n + 1)
        pp.pic_sync(ctx)


def test_birth_buffer_overflow_reports_enomem():
    """Hot electrons (40 eV) ionize a few hundred times per step; a buffer of
    16 births overflows at once."""
    _need_gpu()
    import paper_2609_15043_amd.phasorpic as pp
    say("[gpu] birth buffer overflow")
    ctx = _ctx(_hot_small(100_000), birth_capacity=16)
    with pytest.raises(pp.PicError) as e:
        _run_until_error(ctx, 5)
    assert e.value.status == pp.PIC_ENOMEM and "birth" in str(e.value)


def test_particle_capacity_overflow_reports_enomem():
    """Capacity equal to the initial count (plus the library's chunk
    padding): the births exhaust it within tens of steps."""
    _need_gpu()
    import paper_2609_15043_amd.phasorpic as pp
    say("[gpu] particle capacity overflow")
    wl = _hot_small(100_000)
    wl = dataclasses.replace(wl, capacity_factor=1.0)
    ctx = _ctx(wl)
    with pytest.raises(pp.PicError) as e:
        _run_until_error(ctx, 200)
    assert e.value.status == pp.PIC_ENOMEM and "capacity" in str(e.value)


def test_direct_poisson_solver_refuses_a_non_separable_operator():
    """poisson_solver = direct needs permittivity uniform along every row of
    cells: one cell off that makes pic_init fail with PIC_EINVAL and says
    why; 'auto' takes multigrid-CG for the same workload."""
    _need_gpu()
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    wl = W.small(n_per_species=1000)
    wl.eps_cell = wl.eps_cell.copy()
    wl.eps_cell[10, 5] = 2.0
    say("[gpu] direct Poisson solve on a non-separable operator")
    cfg, keep = pp.config_from_workload(wl, precision="fp64", load=False, poisson_solver="direct")
    with pytest.raises(pp.PicError) as e:
        pp.pic_init(cfg, keep)
    say(f"    {e.value}")
    assert e.value.status == pp.PIC_EINVAL and "permittivity" in str(e.value)
    # auto: multigrid-CG (it iterates from a zero start; the direct solve reports no cycles)
    cfg, keep = pp.config_from_workload(wl, precision="fp64", load=True)
    ctx = pp.pic_init(cfg, keep)
    pp.pic_set_phi(ctx, np.zeros((wl.nz + 1, wl.nr + 1)))
    info = pp.poisson_solve_rz(ctx, 0, info=True)
    say(f"    auto on the same workload: {info}")
    assert info["converged"] and info["cycles"] > 0
