"""mlp_forward_noalloc (activations in the library's static device scratch)
against mlp_forward (activations in the context's workspace), through the C
ABI: the same kernels and arithmetic, so the outputs must agree bit for bit.
Two calls in a row, the second with a smaller batch, so the second reads a
scratch array that still holds the first call's larger contents; then the
limits (batch above 64 or a hidden width above 256) are refused with
nothing launched."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_forward_noalloc_matches_forward():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    say("[gpu] mlp_forward_noalloc against mlp_forward, batches 64 then 5")
    rng = np.random.default_rng(4)
    norm = (rng.normal(0, 1, 29), rng.uniform(0.5, 2.0, 29), rng.normal(0, 1, 20), rng.uniform(0.5, 2.0, 20))
    net = pp.Mlp(norm=norm, max_batch=256)
    net.set_params(W.mlp_init_params(seed=21))
    for batch in (64, 5):
        x = torch.tensor(rng.normal(0, 1, (batch, 29)), dtype=torch.float32, device="cuda")
        y_ref = net.forward(x)
        y_na = net.forward_noalloc(x)
        torch.cuda.synchronize()
        a, b = y_na.cpu().numpy(), y_ref.cpu().numpy()
        say(f"    batch {batch}: max |noalloc - forward| = {np.max(np.abs(a - b)):.3e}, |y| max {np.max(np.abs(b)):.3e}")
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b)
    # limits: refused on the host, no kernel launched
    x = torch.zeros((65, 29), dtype=torch.float32, device="cuda")
    with pytest.raises(pp.PicError) as e:
        net.forward_noalloc(x)
    assert e.value.status == pp.PIC_EINVAL and "64" in str(e.value)
    wide = pp.Mlp(hidden=320, max_batch=8)
    with pytest.raises(pp.PicError) as e:
        wide.forward_noalloc(torch.zeros((2, 29), dtype=torch.float32, device="cuda"))
    assert e.value.status == pp.PIC_EINVAL
