"""The multigrid-preconditioned CG gives the same bits every time.

The tile smoother holds each tile's halo at its values from the start of the
launch (Gauss-Seidel inside a tile, Jacobi across tiles), so the V-cycle is a
fixed symmetric operator.  That needs the post-smoother to write a buffer
other than the one whose halo it loads: when it wrote in place, a tile that
finished early changed the halo of a neighbour that started late, and the
result depended on the order in which workgroups ran (in one run out of
several, the inductive solve of the coil cell then missed its tolerance).

Two contexts built from the same configuration must agree bit for bit
(the Poisson solve forced to multigrid-CG here; the direct solve of a
separable operator has no order-dependent step and is checked the same way).
Without plasma every solve's input is fixed by the geometry and the coil
(the particles' deposit is not: the sort leaves the order of particles in a
cell free, and wave sums round before the fixed-point conversion), so the
coil cell (128 x 256 cells) and the large grid (256 x 512 cells, a few
hundred smoother tiles per launch on the finest levels) are run without
plasma: the inductive unit fields of the five turns, the fields they compose
and phi^0 driven by the turn potentials, each solved to 1e-12 in FP64.
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


def _grids(ctx, which):
    import paper_2609_15043_amd.phasorpic as pp
    return {w: np.array(pp.pic_get_grid(ctx, w), copy=True) for w in which}


def _twice(wl, precision, which, solver="multigrid"):
    import paper_2609_15043_amd.phasorpic as pp
    out = []
    for _ in range(2):
        cfg, keep = pp.config_from_workload(wl, precision=precision, load=False, poisson_solver=solver)
        ctx = pp.pic_init(cfg, keep)
        out.append(_grids(ctx, which))
        del ctx
    return out


@pytest.mark.parametrize("name,solver", [("cell", "multigrid"), ("large", "multigrid"), ("large", "direct")])
def test_solves_bitwise_repeatable(name, solver):
    _need_gpu()
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    wl = getattr(W, name)(n_per_species=1000)
    which = [pp.PIC_GRID_UNIT + k for k in range(wl.nturns)] + [pp.PIC_GRID_EC, pp.PIC_GRID_ES, pp.PIC_GRID_PHI]
    say(f"[gpu] {name} ({wl.nr}x{wl.nz} cells), fp64, no plasma, Poisson {solver}: inductive fields and phi0 of "
        "two contexts")
    a, b = _twice(wl, "fp64", which, solver)
    for w in which:
        d = float(np.max(np.abs(a[w] - b[w])))
        say(f"    grid {w}: max |value| {float(np.max(np.abs(a[w]))):.3e}, max |difference| {d:.3e}")
    for w in which:
        assert np.any(a[w] != 0.0), w
        assert np.array_equal(a[w], b[w]), w
