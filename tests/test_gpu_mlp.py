"""GPU parity of the surrogate network (BF16 matrix-core kernels through
the C ABI) against the FP64 oracle with BF16 storage emulation
(oracle/mlp.py), on seeded synthetic batches.

Both sides round to BF16 at the same storage points; the GPU accumulates
in FP32 and evaluates GELU in FP32, so an element that lands within FP32
error of a BF16 rounding boundary may round the other way (one BF16 ulp,
2^-8 relative).  Bar: relative Frobenius error <= 1e-3 for outputs and
gradients (per parameter block), 1e-4 for the loss.
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


def fro(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _data(B, seed=0, n_in=29, n_out=20):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(B, n_in)) * rng.uniform(0.5, 2.0, n_in) + rng.normal(size=n_in)
    A = rng.normal(size=(n_in, n_out)) / np.sqrt(n_in)
    t = np.tanh(x @ A) * 3.0 + 1.0
    return x.astype(np.float32), t.astype(np.float32)


def _norm(x, t):
    return (x.mean(0), x.std(0), t.mean(0), t.std(0))


@pytest.mark.parametrize("B", [4096, 37, 5, 1])
def test_forward_matches_oracle(B):
    _need_gpu()
    import torch
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    from oracle import mlp as M
    say(f"[gpu] mlp forward B={B}")
    x, t = _data(max(B, 64), seed=1)
    x, t = x[:B], t[:B]
    norm = _norm(*_data(4096, seed=1))
    theta = W.mlp_init_params(seed=2)
    net = pp.Mlp(norm=norm)
    net.set_params(theta)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    ora = M.MLP(theta.astype(np.float64), 256, 29, 20, bf16_storage=True,
                norm=tuple(np.asarray(a, np.float32).astype(np.float64) for a in norm))
    yo = ora.predict(x.astype(np.float64))
    e = fro(y, yo)
    say(f"    output rel Frobenius {e:.2e}")
    assert e <= 1e-3


def test_gradients_and_adam_match_oracle():
    _need_gpu()
    import torch
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    from oracle import mlp as M
    say("[gpu] mlp gradients and Adam, B=4096")
    x, t = _data(4096, seed=3)
    norm = _norm(x, t)
    theta = W.mlp_init_params(seed=4)
    net = pp.Mlp(norm=norm, lr=1e-3)
    net.set_params(theta)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    loss = net.train_step(xd, td)
    g = net.get_grads()
    ora = M.MLP(theta.astype(np.float64), 256, 29, 20, bf16_storage=True,
                norm=tuple(np.asarray(a, np.float32).astype(np.float64) for a in norm))
    lo, go = ora.loss_and_grad(x.astype(np.float64), t.astype(np.float64))
    say(f"    loss gpu {loss:.6e} oracle {lo:.6e}")
    assert abs(loss - lo) / lo <= 1e-4
    gp, gop = M.unpack(g, 256), M.unpack(go, 256)
    errs = {k: fro(gp[k], gop[k]) for k in gp}
    say("    grads " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= 1e-3, (k, v)
    # padding stays exactly zero
    assert np.all(gp["W1"][:, 29:] == 0) and np.all(gp["W4"][20:] == 0) and np.all(gp["b4"][20:] == 0)
    # one Adam step: the update lr * g / (|g| + eps) agrees except where the
    # two gradients straddle zero
    ora.adam_step(go, 1e-3)
    d_gpu = net.get_params().astype(np.float64) - theta
    d_ora = ora.theta - theta
    bad = np.abs(d_gpu - d_ora) > 1e-2 * 1e-3
    say(f"    Adam step: {bad.mean():.2e} of entries differ by more than 1% of lr")
    assert bad.mean() < 1e-2


def test_training_matches_oracle_and_learns():
    _need_gpu()
    import torch
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    from oracle import mlp as M
    say("[gpu] mlp 30 training steps, B=1024")
    x, t = _data(1024, seed=5)
    norm = _norm(x, t)
    theta = W.mlp_init_params(seed=6)
    net = pp.Mlp(norm=norm, lr=2e-3)
    net.set_params(theta)
    ora = M.MLP(theta.astype(np.float64), 256, 29, 20, bf16_storage=True,
                norm=tuple(np.asarray(a, np.float32).astype(np.float64) for a in norm))
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    lg, lo = [], []
    for _ in range(30):
        lg.append(net.train_step(xd, td))
        lo.append(ora.train_step(x.astype(np.float64), t.astype(np.float64), 2e-3)[0])
    say(f"    loss gpu {lg[0]:.4f} -> {lg[-1]:.4f}, oracle {lo[0]:.4f} -> {lo[-1]:.4f}")
    assert lg[-1] < 0.3 * lg[0]
    assert np.max(np.abs(np.array(lg) - lo) / np.array(lo)) < 0.02
