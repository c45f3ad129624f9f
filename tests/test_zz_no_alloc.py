"""The forward pass that allocates nothing (fbc_mlp_forward_noalloc) against the network's
own forward pass (fbc_mlp_forward), through the C ABI: two calls in a row, the second on a
smaller input, each bitwise equal to the existing entry point (same kernels, same order)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.normal(size=(n, 8)).astype(np.float32)).cuda()


def test_noalloc_forward_matches_forward_on_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_08798_amd import MLP
    from paper_2105_08798_amd.fbc import FbcError
    net = MLP(max_batch=6000, seed=5)
    nmax = net.noalloc_max_rows()
    assert nmax == (64 << 20) // (4 * 4 * (3 * 128 + 12))
    for n, seed in ((6000, 1), (1500, 2)):
        x = _inputs(n, seed)
        ref = torch.empty((n, 12), dtype=torch.float32, device="cuda")
        got = torch.full((n, 12), float("nan"), dtype=torch.float32, device="cuda")
        net.forward(x, ref)
        net.forward_noalloc(x, got)
        torch.cuda.synchronize()
        print(f"[noalloc] n={n}: max |diff| {(got - ref).abs().max().item():.1e}", flush=True)
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref)
    # beyond the static workspace: rejected before any device work
    x = _inputs(nmax + 1, 3)
    y = torch.zeros((nmax + 1, 12), dtype=torch.float32, device="cuda")
    with pytest.raises(FbcError) as ei:
        net.forward_noalloc(x, y)
    assert ei.value.code == -1
    assert torch.count_nonzero(y).item() == 0
    net.close()
