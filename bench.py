"""Throughput of the RZ PIC/MCC step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large|cell|small]
                [--precision mixed|fp64] [--fp64-steps K64] [--no-cpu-baseline] [--no-stationary] [--no-mlp]

A step is one pass of the whole per-step cycle through the C ABI:
pic_gather_push (stage + sort by cell, electrons every 16 steps and ions
every 32 + fused gather/push/MCC/deposit pass), harmonic_accumulate, mcc_collide (births), pic_deposit (node
charge), circuit_period_update at every closed RF period, and
poisson_solve_rz (FP64 multigrid + turn charges).  Inputs are resident in
HBM before the timed region starts.  By default two RF periods (4000 steps,
two circuit updates) of the large workload in each precision.  Prints one
JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s and % HBM peak (FP32-mixed vs FP64); wall-s to stationary circuit"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0   # dense BF16 MFMA peak of MI355X
# algorithmic bytes per particle-step of the particle pass: read cell, two
# offsets, three velocity components and the next-candidate step; write
# cell, offsets and velocity (the id and next step are touched only at
# collision candidates).
BYTES_PER_PARTICLE_STEP = {"mixed": 4 + 2 * 4 + 3 * 4 + 4 + 4 + 2 * 4 + 3 * 4,
                           "fp64": 4 + 2 * 8 + 3 * 8 + 4 + 4 + 2 * 8 + 3 * 8}


def workload(name, scale=1):
    from paper_2609_15043_amd import workloads as W
    wl = W.by_name(name)
    if scale != 1:
        wl = W.by_name(name, n_per_species=wl.np_init[0] // scale)
    return wl


def describe(wl, prec):
    return (f"{wl.name}: R={wl.rmax} m z={wl.zmax} m, {wl.nr}x{wl.nz} cells (R x z), "
            f"{wl.np_init[0]:.3g} e + {wl.np_init[1]:.3g} Ar+, argon {wl.pressure_pa / 133.322 * 1e3:.0f} mTorr, "
            f"dt={wl.dt:.4g} s, {'quartz window + 5-turn coil, ' if wl.window else ''}"
            f"{'FP32-mixed' if prec == 'mixed' else 'FP64'} particles, FP64 multigrid")


def run_gpu(wl, prec, steps, warmup, fuse=True):
    import torch
    import paper_2609_15043_amd.phasorpic as pp
    cfg, keep = pp.config_from_workload(wl, precision=prec, fuse=fuse, load=True, sort_every=SORT_EVERY,
                                        sort_every_ion=SORT_EVERY_ION)
    ctx = pp.pic_init(cfg, keep)
    nrf = pp.nrf(wl)
    n = 0

    def one(n):
        pp.pic_gather_push(ctx, n)
        pp.harmonic_accumulate(ctx, n)
        if not wl.implicit:
            pp.mcc_collide(ctx, n)
        pp.pic_deposit(ctx, n + 1)
        if (n + 1) % nrf == 0:
            st, rep, _, _ = pp.circuit_period_update(ctx)
            if st != 0:
                raise RuntimeError(f"period update status {st}")
        pp.poisson_solve_rz(ctx, n + 1)
        if wl.implicit:   # corrector, collisions and births after the solve with chi
            pp.mcc_collide(ctx, n)

    for _ in range(warmup):
        one(n)
        n += 1
    pp.pic_sync(ctx)
    s0 = pp.pic_get_stats(ctx)
    live0 = s0.live[0] + s0.live[1]
    pp.pic_timing(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one(n)
        n += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pp.pic_sync(ctx)
    s1 = pp.pic_get_stats(ctx)
    live1 = s1.live[0] + s1.live[1]
    wall = t1 - t0
    mean_live = 0.5 * (live0 + live1)
    out = dict(wall=wall, steps=steps, live0=live0, live1=live1, mean_live=mean_live,
               rate=mean_live * steps / wall, ms_per_step=1e3 * wall / steps,
               pass_launch_ms=s1.pass_ms / max(1, s1.pass_count), pass_count=s1.pass_count,
               pass_ms=s1.pass_ms / max(1, s1.pass_count),
               poisson_ms=s1.poisson_ms / max(1, s1.poisson_count),
               sort_ms=s1.sort_ms / max(1, s1.sort_count), sort_count=s1.sort_count,
               mg_cycles=int(s1.mg_cycles), mg_rel=s1.mg_rel, window_out=int(s1.window_out),
               mg_unconverged=int(s1.mg_unconverged - s0.mg_unconverged),
               births=int(s1.births - s0.births))
    del ctx
    torch.cuda.empty_cache()
    return out


# cell sorts: electrons every 16 steps, ions (a small fraction of a cell per
# step) every 32
SORT_EVERY, SORT_EVERY_ION = 16, 32

PASS_SOURCES = ("paper_2609_15043_amd/csrc/particles.hip", "paper_2609_15043_amd/csrc/kernels.h",
                "paper_2609_15043_amd/csrc/device.h", "paper_2609_15043_amd/build.py")


def pass_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in PASS_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name, prec, particles_per_launch):
    """HBM bytes of one pass launch from the committed FETCH_SIZE / WRITE_SIZE
    counter summary, scaled by the copy-kernel calibration and to this run's
    particles per launch.  None when the summary is missing or was taken on
    other pass sources than the ones built now."""
    path = os.path.join(ROOT, "profiles", f"k_pass_hbm_traffic_{name}_{prec}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("pass_source_sha256") != pass_source_hash():
        return None
    per_particle = float(kv["hbm_bytes_per_particle_launch"])
    return per_particle * particles_per_launch


def stationary_index(reps, p_target, tol=0.01, window=10):
    """First period i from which, for `window` periods, the port power stays
    within tol of the target and the applied state within tol of its value
    at i (None if no such period): stationarity held over a window, so that
    one period that happens to pass the test does not count."""
    for i in range(len(reps) - window + 1):
        xi = reps[i]["x"]
        ni = float(np.linalg.norm(xi))
        if all(abs(reps[j]["p_port"] - p_target) / p_target <= tol
               and float(np.linalg.norm(reps[j]["x"] - xi)) <= tol * ni for j in range(i, i + window)):
            return i
    return None


def feature_scale(A):
    """Standard deviation of each column of A, 1 where the column is constant
    to rounding: a scale of ~1e-16 would turn a one-ulp difference from the
    mean into an input of order one."""
    mu, sd = A.mean(0), A.std(0)
    return np.where(sd > 1e-9 * np.maximum(np.abs(mu), 1.0), sd, 1.0)


def stationary_circuit(targets=(60.0, 100.0), plain_periods=100, sur_periods=40, adam_steps=5000):
    """Wall-seconds to the stationary circuit state: the plain FP64 GPU run
    against the surrogate-assisted run (FP64 as well: without plasma the two
    precisions run the same FP64 field and circuit arithmetic), at each port
    power target.  A stand-in for the plasma-loaded cell (hundreds of RF
    periods of 2000 steps): the coil cell without plasma at 13.56 MHz, 16
    steps per RF period, controller driving the port power to its target.
    The network is trained first on the method's own (state, response) pairs
    from 240 periods at scanned source settings: amplitudes 2000-5600 V,
    which span about 20-150 W of port power on this cell, and phases within
    0.5 rad (their cost is reported, not counted in either run).
    Stationary: see stationary_index."""
    import torch
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    wl = W.cell(n_per_species=1000)
    wl.dt = 1.0 / (16 * wl.freq)
    nrf, N = 16, wl.nturns

    def periods_of(ctx, periods, source=None):
        reps, times = [], []
        n = 0
        t0 = time.perf_counter()
        for p in range(periods):
            if source is not None:
                pp.pic_set_source(ctx, *source(p))
            for _ in range(nrf):
                pp.pic_gather_push(ctx, n)
                pp.harmonic_accumulate(ctx, n)
                pp.mcc_collide(ctx, n)
                pp.pic_deposit(ctx, n + 1)
                if (n + 1) % nrf == 0:
                    st, rep, _, _ = pp.circuit_period_update(ctx)   # synchronises
                    if st != 0:
                        raise RuntimeError(f"period update status {st}")
                    reps.append(rep)
                    times.append(time.perf_counter() - t0)
                pp.poisson_solve_rz(ctx, n + 1)
                n += 1
        return reps, times

    # training pairs from the method itself, scanning the source
    t0 = time.perf_counter()
    cfg, keep = pp.config_from_workload(wl, precision="fp64", load=False)
    ctx = pp.pic_init(cfg, keep)
    rng = np.random.default_rng(21)
    scan = [(float(rng.uniform(2000.0, 5600.0)), float(rng.uniform(-0.5, 0.5))) for _ in range(240)]
    reps, _ = periods_of(ctx, 240, source=lambda p: scan[p])
    del ctx
    X = np.array([pp.surrogate_features(r, N) for r in reps])
    Y = np.array([pp.surrogate_targets(r, N) for r in reps])
    norm = (X.mean(0), feature_scale(X), Y.mean(0), feature_scale(Y))
    net = pp.Mlp(norm=norm, lr=1e-3, max_batch=256)
    net.set_params(W.mlp_init_params(seed=22))
    xd = torch.from_numpy(X.astype(np.float32)).cuda()
    yd = torch.from_numpy(Y.astype(np.float32)).cuda()
    for it in range(adam_steps):
        loss = net.train_step(xd, yd, want_loss=(it == adam_steps - 1))
    net.sync()
    t_train = time.perf_counter() - t0
    def leg(r, prec):
        i = r["i"]
        return {"precision": prec, "periods": None if i is None else i + 1,
                "wall_s": None if i is None else r["times"][i], "surrogate_periods": r["used"]}

    out = []
    for target in targets:
        wl.circuit.p_target = target
        runs = {}
        # both runs FP64; the surrogate-assisted run differs only in the period update
        for mode, periods in (("plain", plain_periods), ("surrogate", sur_periods)):
            cfg, keep = pp.config_from_workload(wl, precision="fp64", load=False)
            ctx = pp.pic_init(cfg, keep)
            if mode == "surrogate":
                pp.pic_attach_surrogate(ctx, net, err_max=0.02, tol=1e-6, max_iter=50)
            reps, times = periods_of(ctx, periods)
            runs[mode] = dict(reps=reps, times=times, i=stationary_index(reps, target),
                              used=sum(r["sur_used"] for r in reps))
            del ctx
        x_ref = runs["plain"]["reps"][-1]["x"]
        dev = float(np.linalg.norm(runs["surrogate"]["reps"][-1]["x"] - x_ref) / np.linalg.norm(x_ref))
        final = {k: runs["plain"]["reps"][-1][k] for k in ("p_port", "p_cu", "p_ind", "p_cap", "eps_bal")}
        out.append({"p_target_w": target, "plain_final_powers_w": final, "plain": leg(runs["plain"], "fp64"),
                    "surrogate_assisted": leg(runs["surrogate"], "fp64"), "final_state_deviation": dev})
    return {"workload": f"{wl.name} coil cell without plasma, {wl.nr}x{wl.nz} cells, 13.56 MHz, 16 steps per RF "
                        f"period, port power targets " + ", ".join(f"{t:g}" for t in targets) + " W",
            "criterion": "first period from which, for 10 periods, the port power stays within 1 % of the target "
                         "and the applied state within 1 % of its value at that period",
            "runs": out,
            "training": {"pairs": len(X), "adam_steps": adam_steps, "final_loss": float(loss), "wall_s": t_train}}


def stationary_q27(reps, p_target, tol=0.01, window=10):
    """First period i (0-based) such that over the window [i, i + window)
    every period's port power lies within tol of the target, and for every
    turn the window mean of |I_k| and of |V_k| moves by less than tol
    against the preceding window [i - window, i); None if no such period.
    The plasma keeps evolving (density, temperature), so stationarity is
    judged on window means rather than on single periods."""
    N = (len(reps[0]["x"]) - 1) // 2
    mags = np.array([np.abs(r["x"][1:]) for r in reps])   # |I_k|, |V_k| per period
    for i in range(window, len(reps) - window + 1):
        if not all(abs(reps[j]["p_port"] - p_target) / p_target <= tol for j in range(i, i + window)):
            continue
        cur, prev = mags[i:i + window].mean(0), mags[i - window:i].mean(0)
        if np.all(np.abs(cur - prev) <= tol * np.abs(cur)):
            return i
    return None


def settled_index(reps, p_target, tol=0.01, min_tail=10):
    """The settling rule of the paper's GEC runs (Sec. 3.4): the first period
    (0-based) from which the port power stays within tol of the target in
    every period to the end of the run, with at least min_tail periods
    left; None if there is none."""
    ok = [abs(r["p_port"] - p_target) / p_target <= tol for r in reps]
    first = None
    for i in range(len(reps) - 1, -1, -1):
        if not ok[i]:
            break
        first = i
    if first is None or len(reps) - first < min_tail:
        return None
    return first


PLASMA_N0 = 1e14          # m^-3: Debye length (1 mm at 3 eV) about the cell size
PLASMA_NRF = 400          # steps per RF period
PLASMA_VG_START = 300.0   # V


def plasma_cell(seed, nps, p_target, pressure_mtorr=20.0):
    """The coupled coil cell (128 x 256 cells, quartz window, 5 turns)
    loaded with plasma at PLASMA_N0, PLASMA_NRF steps per RF period, the
    controller driving the port power towards p_target from PLASMA_VG_START."""
    from paper_2609_15043_amd import workloads as W
    wl = W.cell(seed=seed, n_per_species=nps, vg_start=PLASMA_VG_START, n0=PLASMA_N0)
    wl.dt = 1.0 / (PLASMA_NRF * wl.freq)
    wl.pressure_pa = pressure_mtorr * 1e-3 * W.TORR
    wl.capacity_factor = 3.0
    wl.circuit.p_target = float(p_target)
    return wl


def _plasma_periods(ctx, periods, nrf, after_period=None):
    """Whole RF periods of the explicit cycle with the period update; the
    reports and the wall time at the end of each period (after_period(rep),
    when given, runs at each period's end and is timed with it)."""
    import paper_2609_15043_amd.phasorpic as pp
    reps, times = [], []
    n = 0
    t0 = time.perf_counter()
    for _ in range(periods):
        for _ in range(nrf):
            pp.pic_gather_push(ctx, n)
            pp.harmonic_accumulate(ctx, n)
            pp.mcc_collide(ctx, n)
            pp.pic_deposit(ctx, n + 1)
            if (n + 1) % nrf == 0:
                st, rep, _, _ = pp.circuit_period_update(ctx)   # synchronises
                if st != 0:
                    raise RuntimeError(f"period update status {st}")
                reps.append(rep)
                if after_period is not None:
                    after_period(rep)
                times.append(time.perf_counter() - t0)
            pp.poisson_solve_rz(ctx, n + 1)
            n += 1
    return reps, times


class OnlineRefinement:
    """The surrogate-assisted run's own (state, response) pairs join the
    training set as the periods close: after each period update the
    network takes `steps` Adam steps over the base set and the run's pairs
    so far (normalisation fixed by the base set).  The plasma keeps
    evolving during the run (the density grows by about half a per cent
    per period here), which carries its state out of the base set's range;
    the pairs the run measures keep the network's prediction at the states
    it visits within the fallback threshold."""

    def __init__(self, net, X, Y, N, steps=100):
        import torch
        self.net, self.N, self.steps = net, N, steps
        self.X, self.Y = [X.astype(np.float32)], [Y.astype(np.float32)]
        self.torch = torch

    def __call__(self, rep):
        import paper_2609_15043_amd.phasorpic as pp
        torch = self.torch
        self.X.append(pp.surrogate_features(rep, self.N)[None, :].astype(np.float32))
        self.Y.append(pp.surrogate_targets(rep, self.N)[None, :].astype(np.float32))
        xd = torch.from_numpy(np.concatenate(self.X)).cuda()
        yd = torch.from_numpy(np.concatenate(self.Y)).cuda()
        for _ in range(self.steps):
            self.net.train_step(xd, yd, want_loss=False)
        self.net.sync()


def plasma_training_pairs(runs=12, periods=10, nps=2_000_000, power_w=(1.0, 7.5), pressure_mtorr=(5.0, 50.0)):
    """The network's training set from PIC periods with plasma: `runs` runs
    of the plasma cell, run r with port power target ~ U(power_w) and
    pressure ~ logU(pressure_mtorr) drawn by numpy's generator seeded
    1000 + r and its particles loaded with seed 1000 + r, each `periods` RF
    periods from the start (the controller transient sweeps the state);
    every period gives one (state, response) pair.  Returns X, Y and a
    summary."""
    import paper_2609_15043_amd.phasorpic as pp
    t0 = time.perf_counter()
    X, Y = [], []
    for r in range(runs):
        u = np.random.default_rng(1000 + r).uniform(size=2)
        pt = power_w[0] + (power_w[1] - power_w[0]) * u[0]
        lo, hi = math.log(pressure_mtorr[0]), math.log(pressure_mtorr[1])
        wl = plasma_cell(1000 + r, nps, pt, math.exp(lo + (hi - lo) * u[1]))
        cfg, keep = pp.config_from_workload(wl, precision="fp64", load=True)
        ctx = pp.pic_init(cfg, keep)
        reps, _ = _plasma_periods(ctx, periods, pp.nrf(wl))
        del ctx
        X += [pp.surrogate_features(rep, wl.nturns) for rep in reps]
        Y += [pp.surrogate_targets(rep, wl.nturns) for rep in reps]
    return np.array(X), np.array(Y), {"runs": runs, "periods_per_run": periods, "particles_per_species": nps,
                                      "pairs": len(X), "port_power_w": list(power_w),
                                      "pressure_mtorr": list(pressure_mtorr), "data_wall_s": time.perf_counter() - t0}


def train_plasma_surrogate(X, Y, adam_steps=5000, extra_rows=256):
    """Adam on the GPU over the whole training set (inputs and outputs
    standardised by the set's own means and scales).  Returns the network
    and a summary."""
    import torch
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    t0 = time.perf_counter()
    norm = (X.mean(0), feature_scale(X), Y.mean(0), feature_scale(Y))
    net = pp.Mlp(norm=norm, lr=1e-3, max_batch=max(256, len(X) + extra_rows))
    net.set_params(W.mlp_init_params(seed=22))
    xd = torch.from_numpy(X.astype(np.float32)).cuda()
    yd = torch.from_numpy(Y.astype(np.float32)).cuda()
    for it in range(adam_steps):
        loss = net.train_step(xd, yd, want_loss=(it == adam_steps - 1))
    net.sync()
    return net, {"adam_steps": adam_steps, "final_loss": float(loss), "train_wall_s": time.perf_counter() - t0}





def stationary_plasma(targets=(3.0, 5.0), periods=70, nps=2_000_000, window=10, refine_steps=100, training=None):
    """Wall-seconds to the stationary circuit on the plasma-loaded coil cell:
    the plain FP64 GPU run against the surrogate-assisted run in FP32-mixed
    and in FP64, at each port power target, 20 mTorr, nps electrons + nps
    Ar+ (seed 0).  The network is trained first on plasma_training_pairs
    (its cost reported, not counted in either run); each surrogate-assisted
    run starts from those weights and refines them online on its own
    periods (OnlineRefinement, counted in its wall time).  Stationary: the
    settling rule (settled_index: the port power within 1 % of the target
    in every period to the end); also reported, the first period of
    stationary_q27's window-mean criterion, which the plasma's own drift
    makes noisy.  Reported per run: periods and wall-seconds to
    stationary, periods in which the surrogate's update was applied, and
    over the last `window` periods the mean port, inductive and capacitive
    powers, the field-versus-circuit power imbalance and the electron
    density and temperature; the deviation of each run's final window-mean
    state from the plain run's over the same periods (every run lasts
    `periods` periods: the plasma density keeps growing, so states are
    compared at the same time)."""
    import paper_2609_15043_amd.phasorpic as pp
    if training is None:
        X, Y, dinfo = plasma_training_pairs()
        net, tinfo = train_plasma_surrogate(X, Y, extra_rows=periods)
        training = dict(net=net, X=X, Y=Y, info={**dinfo, **tinfo})
    net, X, Y = training["net"], training["X"], training["Y"]
    theta0 = net.get_params()
    out = []
    for target in targets:
        runs = {}
        for mode, prec in (("plain", "fp64"), ("surrogate", "mixed"), ("surrogate", "fp64")):
            wl = plasma_cell(0, nps, target)
            cfg, keep = pp.config_from_workload(wl, precision=prec, load=True)
            ctx = pp.pic_init(cfg, keep)
            refine = None
            if mode == "surrogate":
                net.set_params(theta0)
                pp.pic_attach_surrogate(ctx, net, err_max=0.02, tol=1e-6, max_iter=50)
                refine = OnlineRefinement(net, X, Y, wl.nturns, refine_steps) if refine_steps else None
            reps, times = _plasma_periods(ctx, periods, pp.nrf(wl), after_period=refine)
            st = pp.pic_get_stats(ctx)
            del ctx
            i = settled_index(reps, target)
            iq = stationary_q27(reps, target, window=window)
            tail = reps[-window:]
            runs[f"{mode}_{prec}"] = {
                "periods": None if i is None else i + 1, "wall_s": None if i is None else times[i],
                "periods_window_means": None if iq is None else iq + 1,
                "wall_s_run": times[-1], "surrogate_periods": int(sum(r["sur_used"] for r in reps)),
                "final": {k: float(np.mean([r[k] for r in tail])) for k in ("p_port", "p_ind", "p_cap", "p_cu",
                                                                            "eps_bal")},
                "final_n_e": float(np.mean([r["moments"][0] for r in tail])),
                "final_T_e_ev": float(np.mean([2.0 / 3.0 * r["moments"][3] for r in tail])),
                "mg_unconverged": int(st.mg_unconverged),
                "_x": np.mean([r["x"] for r in tail], axis=0)}
        x_ref = runs["plain_fp64"]["_x"]
        for k in runs:
            runs[k]["final_state_deviation"] = float(np.linalg.norm(runs[k].pop("_x") - x_ref) / np.linalg.norm(x_ref))
        out.append({"p_target_w": target, **runs})
    net.set_params(theta0)
    return {"workload": f"plasma-loaded coil cell 128x256, argon 20 mTorr, {nps:.3g} e + {nps:.3g} Ar+ at "
                        f"{PLASMA_N0:g} m^-3, 13.56 MHz at {PLASMA_NRF} steps per RF period, controller from "
                        f"{PLASMA_VG_START:g} V, port power targets " + ", ".join(f"{t:g}" for t in targets) + " W",
            "criterion": "settling rule: first period from which the port power stays within 1 % of the target in "
                         "every period to the end of the run (at least 10 periods); periods_window_means: first "
                         f"period from which, for {window} periods, the port power stays within 1 % and every turn's "
                         f"window-mean |I_k| and |V_k| moves by under 1 % against the preceding {window} periods",
            "periods_per_run": periods, "online_refinement_adam_steps_per_period": refine_steps,
            "runs": out, "training": training["info"]}


def surrogate_mlp(batch=4096, steps=200, warmup=20):
    """The surrogate network's kernels at their training configuration: MLP
    29-256-256-256-20 (GELU; BF16 operands, FP32 accumulation on MFMA),
    batch 4096, Adam lr 1e-3.  Forward alone, then whole training steps
    (forward, MSE backward, Adam), timed with HIP events on the stream the
    network runs on (torch's current stream, fixed at its creation).
    FLOPs are those of the unpadded layer shapes: forward 2 B sum(in x out);
    a training step adds the weight gradients (as many) and the activation
    gradients of every layer but the first."""
    import torch
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    dims = [W.MLP_IN, W.MLP_HIDDEN, W.MLP_HIDDEN, W.MLP_HIDDEN, W.MLP_OUT]
    macs = [a * b for a, b in zip(dims[:-1], dims[1:])]
    fwd_flop = 2.0 * batch * sum(macs)
    train_flop = 2.0 * fwd_flop + 2.0 * batch * sum(macs[1:])
    net = pp.Mlp(max_batch=batch, lr=1e-3)
    net.set_params(W.mlp_init_params(seed=22))
    g = torch.Generator().manual_seed(23)
    x = torch.randn(batch, W.MLP_IN, generator=g).cuda()
    t = torch.randn(batch, W.MLP_OUT, generator=g).cuda()
    y = torch.empty(batch, W.MLP_OUT, device="cuda")

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    fwd_ms = timed(lambda: net.forward(x, y))
    train_ms = timed(lambda: net.train_step(x, t, want_loss=False))
    net.sync()
    tf = train_flop / (train_ms * 1e-3) / 1e12
    return {"model": "MLP 29-256-256-256-20, GELU, BF16 MFMA with FP32 accumulation, Adam lr 1e-3",
            "batch": batch, "steps": steps,
            "forward": {"ms": fwd_ms, "gflop": fwd_flop / 1e9, "tflops": fwd_flop / (fwd_ms * 1e-3) / 1e12},
            "train_step": {"ms": train_ms, "gflop": train_flop / 1e9, "tflops": tf},
            "roofline": {"bound": "mfma", "achieved": tf, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / BF16_PEAK_TFLOPS, "kernel": "whole training step (11 products + GELU, "
                                                               "loss and Adam kernels)"}}


def _oracle_run(args):
    """One oracle instance (a worker of the all-core baseline, or the
    single-core run): nsteps whole steps of the workload at 1/scale of its
    particles, seed as given; returns (live particles, wall seconds)."""
    name, scale, nsteps, seed = args
    from oracle import pic as O
    wl = workload(name, scale)
    wl.seed = seed
    ora = O.OraclePIC(wl)
    live = sum(int(p.alive.sum()) for p in ora.parts)
    t0 = time.perf_counter()
    for _ in range(nsteps):
        ora.step()
    return live, time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(name, scale, nsteps, workers=None):
    """The oracle as it stands, on a bounded sample: same grid and physics,
    1/scale of the particles, nsteps whole steps (init not timed), on one
    host core; then on every core it may use (min(16, cpu count): the box's
    CPU share): one independent oracle instance per core on its own seed,
    the aggregate rate being all their particle-steps over the wall time of
    the whole set (the particles are independent, so this is the plain
    oracle's all-core throughput without changing its code)."""
    import multiprocessing as mp
    live, dt = _oracle_run((name, scale, nsteps, 0))
    wl = workload(name, scale)
    out = dict(value=live * nsteps / dt, unit="particle-steps/s", cores=1, kind="oracle", cpu_model=cpu_model(),
               sample=f"{wl.name} grid and gas with {wl.np_init[0]:.3g} e + {wl.np_init[1]:.3g} Ar+ "
                      f"(1/{scale} of the workload), {nsteps} whole steps, {dt:.1f} s on one host core "
                      f"(plain C particle loops + sparse direct Poisson)")
    workers = workers or min(16, os.cpu_count() or 1)
    if workers > 1:
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(workers) as pool:
            res = pool.map(_oracle_run, [(name, scale, nsteps, 1 + k) for k in range(workers)])
        wall = time.perf_counter() - t0
        # the workers' own step loops (their set-up excluded): the slowest one
        slow = max(r[1] for r in res)
        out["all_cores"] = dict(value=sum(r[0] for r in res) * nsteps / slow, cores=workers,
                                wall_s=slow, pool_wall_s=wall,
                                sample=f"{workers} oracle instances as above (seeds 1..{workers}) at once")
    return out


def accuracy(name="large"):
    """The FP32-mixed path against FP64 on the bench workload: both contexts
    load the same particles (counter-based draws keyed by particle id) and
    take one whole step; the FP64 path matches the oracle to 1e-12 (the
    parity tests), so these differences are the mixed path's errors.  Per
    quantity max |mixed - FP64| / max |FP64|: phi^0, then after the step E_r,
    E_z (from phi^0), the current I, Q^1, phi^1, the turn charges and every
    particle's R, z, v present in both (ids that differ counted).  Then the
    closed-period powers: the coupled coil cell (2e6 + 2e6 at 1e14 m^-3, 2000
    steps per period, source from 300 V) over one RF period in both
    precisions from the same load: P_ind, P_cap and the port power (the two
    trajectories separate by rounding within the period, so these
    differences are statistical)."""
    import torch
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    wl = workload(name)
    ctxs = {}
    grids = {}
    for prec in ("fp64", "mixed"):
        cfg, keep = pp.config_from_workload(wl, precision=prec, load=True, sort_every=SORT_EVERY,
                                            sort_every_ion=SORT_EVERY_ION)
        ctx = pp.pic_init(cfg, keep)
        g = {"phi0": pp.pic_get_grid(ctx, pp.PIC_GRID_PHI)}
        pp.pic_gather_push(ctx, 0)
        g["Er"] = pp.pic_get_grid(ctx, pp.PIC_GRID_ER)
        g["Ez"] = pp.pic_get_grid(ctx, pp.PIC_GRID_EZ)
        pp.harmonic_accumulate(ctx, 0)
        g["I"] = pp.pic_get_grid(ctx, pp.PIC_GRID_CURRENT)
        pp.mcc_collide(ctx, 0)
        pp.pic_deposit(ctx, 1)
        pp.poisson_solve_rz(ctx, 1)
        g["Q1"] = pp.pic_get_grid(ctx, pp.PIC_GRID_CHARGE)
        g["phi1"] = pp.pic_get_grid(ctx, pp.PIC_GRID_PHI)
        g["Qk"] = np.array(pp.pic_get_stats(ctx).qk[:wl.nturns])
        ctxs[prec] = ctx
        grids[prec] = g
    def rel(a, b):
        return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))
    out = {k: rel(grids["mixed"][k], grids["fp64"][k]) for k in grids["fp64"]}
    mism = 0
    for s in range(2):
        a, b = pp.pic_get_particles(ctxs["mixed"], s), pp.pic_get_particles(ctxs["fp64"], s)
        common, ia, ib = np.intersect1d(a["id"], b["id"], assume_unique=True, return_indices=True)
        mism += len(a["id"]) + len(b["id"]) - 2 * len(common)
        for k in ("R", "z", "vr", "vt", "vz"):
            out[f"{k}_{'e' if s == 0 else 'i'}"] = rel(a[k][ia], b[k][ib])
        del a, b
    out["particle_ids_differing"] = int(mism)
    del ctxs
    torch.cuda.empty_cache()
    # closed-period powers on the coupled cell
    reps = {}
    for prec in ("fp64", "mixed"):
        wl = W.cell(seed=0, n_per_species=2_000_000, vg_start=300.0, n0=1e14)
        cfg, keep = pp.config_from_workload(wl, precision=prec, load=True)
        ctx = pp.pic_init(cfg, keep)
        nrf = pp.nrf(wl)
        for n in range(nrf):
            pp.pic_gather_push(ctx, n)
            pp.harmonic_accumulate(ctx, n)
            pp.mcc_collide(ctx, n)
            pp.pic_deposit(ctx, n + 1)
            if n + 1 == nrf:
                st, reps[prec], _, _ = pp.circuit_period_update(ctx)
            pp.poisson_solve_rz(ctx, n + 1)
        del ctx
    for k in ("p_ind", "p_cap", "p_port"):
        out[f"{k}_period1"] = abs(reps["mixed"][k] - reps["fp64"][k]) / abs(reps["fp64"][k])
    out["workload"] = (f"{name}: one step from the same load (particles, phi, E, I, Q, Q_k); closed-period "
                       f"powers: coupled coil cell 2e6 + 2e6 at 1e14 m^-3, one RF period of 2000 steps")
    return out


def next_steps(name, steps, warmup):
    """The widened rows on the benchmark workload, FP32-mixed, each timed like
    the main run over `steps` steps: the direct-implicit update (predictor,
    chi, multigrid-CG with chi, corrector), the RF magnetic field in the push,
    the multiharmonic circuit (a second order at half the fundamental's
    amplitude, magnetoquasistatic operator; the first period update falls
    after 2000 steps, so the timed steps take the order sums in the gathers,
    the harmonics and the Poisson boundary values) and secondary emission
    (yield 0.1).  For the explicit legs the pass moves the same 52 B per
    particle as the main run."""
    import dataclasses
    from paper_2609_15043_amd import workloads as W
    out = {}
    legs = [("direct_implicit", dict(implicit=True)), ("rf_bfield", dict(rf_bfield=True)),
            ("multiharmonic", dict(harmonics=((0.5, 0.7),))), ("secondary_emission", dict(see_gamma=0.1))]
    for leg, kw in legs:
        wl = workload(name)
        if "harmonics" in kw:
            wl.circuit = dataclasses.replace(wl.circuit, field_mode=W.FIELD_MQS, harmonics=kw["harmonics"])
        else:
            for k, v in kw.items():
                setattr(wl, k, v)
        r = run_gpu(wl, "mixed", steps, warmup)
        q = {"value": r["rate"], "unit": "particle-steps/s", "ms_per_step": r["ms_per_step"], "steps": steps,
             "pass_ms": r["pass_ms"], "poisson_ms": r["poisson_ms"], "mg_cycles_last_solve": r["mg_cycles"],
             "mg_unconverged": r["mg_unconverged"]}
        if leg != "direct_implicit":
            q["pass_hbm_frac"] = BYTES_PER_PARTICLE_STEP["mixed"] * r["mean_live"] / (r["pass_ms"] * 1e-3) / 1e9 \
                / HBM_PEAK_GBS
        out[leg] = q
        print(f"[bench] next step {leg}: {r['rate']:.4g} particle-steps/s, {r['ms_per_step']:.3f} ms/step, "
              f"pass {r['pass_ms']:.3f} ms, poisson {r['poisson_ms']:.3f} ms", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)   # two RF periods of the large workload
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--fp64-steps", type=int, default=4000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stationary", action="store_true", help="skip the wall-seconds-to-stationary leg")
    ap.add_argument("--no-mlp", action="store_true", help="skip the surrogate network's kernel timing")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the mixed-against-FP64 accuracy block")
    ap.add_argument("--next-steps", type=int, default=400, metavar="STEPS",
                    help="timed steps of each widened row (direct-implicit, RF magnetic field, multiharmonic, "
                         "secondary emission); 0 skips them")
    ap.add_argument("--cpu-scale", type=int, default=4)
    ap.add_argument("--cpu-steps", type=int, default=15)
    ap.add_argument("--split", action="store_true", help="unfused pass (parity-isolation mode)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of this many MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the particle decomposition "
              "across GPUs is designed but not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2609_15043_amd import workloads as W  # noqa: F401

    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 1.0, out=b)   # one elementwise kernel: reads a, writes b
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {args.calibrate_copy} MiB read + {args.calibrate_copy} MiB written",
              file=sys.stderr, flush=True)
        del a, b
    wl = workload(args.workload)
    prec = args.precision
    print(f"[bench] {describe(wl, prec)}; {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr,
          flush=True)
    r = run_gpu(wl, prec, args.steps, args.warmup, fuse=not args.split)
    print(f"[bench] {prec}: {r['rate']:.4g} particle-steps/s, {r['ms_per_step']:.3f} ms/step, "
          f"pass {r['pass_ms']:.3f} ms, poisson {r['poisson_ms']:.3f} ms ({r['mg_cycles']} cycles), "
          f"sort {r['sort_ms']:.3f} ms, window fallbacks {r['window_out']}", file=sys.stderr, flush=True)
    other = None
    if args.fp64_steps > 0:
        p2 = "fp64" if prec == "mixed" else "mixed"
        print(f"[bench] {p2}: {args.fp64_steps} timed steps", file=sys.stderr, flush=True)
        r2 = run_gpu(wl, p2, args.fp64_steps, args.warmup, fuse=not args.split)
        print(f"[bench] {p2}: {r2['rate']:.4g} particle-steps/s, {r2['ms_per_step']:.3f} ms/step, "
              f"pass {r2['pass_ms']:.3f} ms", file=sys.stderr, flush=True)
        bpp2 = BYTES_PER_PARTICLE_STEP[p2]
        other = {"precision": p2, "value": r2["rate"], "unit": "particle-steps/s",
                 "ms_per_step": r2["ms_per_step"], "steps": r2["steps"],
                 "pass_ms": r2["pass_ms"], "pass_hbm_frac": bpp2 * r2["mean_live"] / (r2["pass_ms"] * 1e-3) / 1e9
                 / HBM_PEAK_GBS,
                 # counter-measured HBM bytes of one pass launch (committed summary), or None
                 "pass_traffic": measured_traffic(wl.name, p2, r2["mean_live"])}
    bpp = BYTES_PER_PARTICLE_STEP[prec]
    # one launch moves both species: every live particle
    launch_bytes = bpp * r["mean_live"]
    achieved = launch_bytes / (r["pass_launch_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(wl.name, prec, r["mean_live"])
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_pass (fused gather/push/MCC-candidate/deposit pass), one launch for both species per step, "
                          "HIP events on the library stream over the timed steps",
                "launch_ms": r["pass_launch_ms"], "launches": r["pass_count"],
                "bytes_per_launch": launch_bytes, "bytes_per_particle_step": bpp}
    # whole step: the same algorithmic particle bytes over the step's wall
    # time (multigrid, sort, collisions and births included)
    step_bytes = bpp * r["mean_live"]
    step_gbs = step_bytes / (r["ms_per_step"] * 1e-3) / 1e9
    step_hbm = {"achieved": step_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": step_gbs / HBM_PEAK_GBS,
                "bytes_per_step": step_bytes}
    mlp = None
    if not args.no_mlp:
        mlp = surrogate_mlp()
        print(f"[bench] surrogate MLP, batch {mlp['batch']}: forward {mlp['forward']['ms']:.3f} ms "
              f"({mlp['forward']['tflops']:.1f} TFLOP/s), training step {mlp['train_step']['ms']:.3f} ms "
              f"({mlp['train_step']['tflops']:.1f} TFLOP/s)", file=sys.stderr, flush=True)
    stat = stat_vac = None
    if not args.no_stationary:
        print("[bench] wall-s to stationary circuit, plasma-loaded cell: training pairs from PIC periods, then "
              "plain FP64 vs surrogate-assisted FP32-mixed and FP64", file=sys.stderr, flush=True)
        stat = stationary_plasma()
        t = stat["training"]
        print(f"[bench] training set: {t['pairs']} pairs from {t['runs']} runs in {t['data_wall_s']:.1f} s, "
              f"{t['adam_steps']} Adam steps in {t['train_wall_s']:.2f} s", file=sys.stderr, flush=True)
        for run in stat["runs"]:
            for k in ("plain_fp64", "surrogate_mixed", "surrogate_fp64"):
                q = run[k]
                print(f"[bench] {run['p_target_w']:g} W {k}: settled after {q['periods']} periods "
                      f"({q['wall_s']} s; window means {q['periods_window_means']}), surrogate used in "
                      f"{q['surrogate_periods']}, final P_ind {q['final']['p_ind']:.3f} W P_cap "
                      f"{q['final']['p_cap']:.3f} W eps_bal {q['final']['eps_bal']:.2e}, state deviation "
                      f"{q['final_state_deviation']:.2e}", file=sys.stderr, flush=True)
        print("[bench] wall-s to stationary circuit, coil cell without plasma (extra)", file=sys.stderr, flush=True)
        stat_vac = stationary_circuit()
    acc = None
    if not args.no_accuracy:
        print("[bench] accuracy: FP32-mixed against FP64 from the same load", file=sys.stderr, flush=True)
        acc = accuracy(args.workload)
        print("[bench] accuracy: " + " ".join(f"{k} {v:.2e}" for k, v in acc.items() if isinstance(v, float)),
              file=sys.stderr, flush=True)
    nxt = None
    if args.next_steps > 0:
        nxt = next_steps(args.workload, args.next_steps, args.warmup)
    cpu = None
    if not args.no_cpu_baseline:
        print(f"[bench] cpu baseline: oracle on 1/{args.cpu_scale} of {wl.name}, {args.cpu_steps} steps",
              file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.workload, args.cpu_scale, args.cpu_steps)
    line = {
        "metric": METRIC, "value": r["rate"], "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32-mixed" if prec == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": describe(wl, prec), "particles": r["mean_live"], "grid": [wl.nr, wl.nz],
                   "parallelism": "1 GPU", "sort_every": SORT_EVERY, "sort_every_ion": SORT_EVERY_ION,
                   "fused": not args.split},
        "roofline": roofline, "step_hbm": step_hbm, "stationary_circuit": stat,
        "stationary_circuit_vacuum": stat_vac, "surrogate_mlp": mlp,
        "cpu_baseline": cpu, "accuracy": acc, "next_steps": nxt,
        "breakdown_ms": {"pass": r["pass_ms"], "poisson": r["poisson_ms"], "sort_per_species": r["sort_ms"],
                         "window_fallback_atomics": r["window_out"],
                         "species_sorts_per_step": r["sort_count"] / max(1, r["steps"]),
                         "mg_cycles_last_solve": r["mg_cycles"], "mg_unconverged": r["mg_unconverged"]},
        "other_precision": other,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
