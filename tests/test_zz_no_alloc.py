"""The forward pass that allocates nothing (kamx_mlp_forward_noalloc, through
the C ABI) against the ordinary forward (kamx_mlp_forward): the same bits on
two calls in a row, the second with a smaller batch, so stale activations
of the first call in the shared per-GPU workspace must not leak into the
second; a batch beyond the workspace is rejected before any work."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_16536_amd import kamx  # noqa: E402


def _net(n_in, n_out, max_batch, seed):
    net = kamx.MLP(n_in, n_out, n_hidden=256, max_batch=max_batch, seed=seed)
    rng = np.random.default_rng(seed)
    net.set_normalization(rng.normal(0, 1, n_in), rng.uniform(0.5, 2.0, n_in), rng.normal(0, 1, n_out),
                          rng.uniform(0.5, 2.0, n_out))
    return net, rng


def test_noalloc_forward_equals_forward_twice_shrinking():
    net, rng = _net(667, 224, 4096, 5)
    for batch in (4096, 100):
        x = torch.as_tensor(rng.normal(0.0, 3.0, (batch, 667)), dtype=torch.float32, device="cuda")
        ref = net.forward(x)
        out = torch.full((batch, 224), float("nan"), dtype=torch.float32, device="cuda")
        net.forward_noalloc(x, out)
        torch.cuda.synchronize()
        print(f"batch {batch}: max |noalloc - forward| = {(out - ref).abs().max().item():.3e}", flush=True)
        assert torch.equal(out, ref), batch
    net.close()


def test_noalloc_forward_two_networks_and_limits():
    """A second network of other sizes after the first (the workspace is
    shared), its batch above that network's own capacity but within the
    workspace, and the rejection of a batch the workspace cannot hold."""
    a, rng = _net(100, 50, 64, 9)
    x = torch.as_tensor(rng.normal(0.0, 1.0, (2000, 100)), dtype=torch.float32, device="cuda")
    out = torch.empty((2000, 50), dtype=torch.float32, device="cuda")
    a.forward_noalloc(x, out)
    # the ordinary forward in chunks of the network's capacity (rows are independent)
    ref = torch.cat([a.forward(x[i:i + 64]) for i in range(0, 2000, 64)])
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    big = torch.empty((8000, 667), dtype=torch.float32, device="cuda")
    b, _ = _net(667, 224, 64, 3)
    with pytest.raises(kamx.KamxError, match="workspace"):
        b.forward_noalloc(big, torch.empty((8000, 224), dtype=torch.float32, device="cuda"))
    a.close()
    b.close()
