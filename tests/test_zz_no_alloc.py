"""The allocation-free net forward (sdpm_net_forward_noalloc, static device
scratch) against the allocating one (sdpm_net_forward, caller buffers) on
the same inputs through the C ABI: bit-identical outputs on two calls in a
row, the second on a smaller mesh (the static array then holds the first
call's larger activations beyond what the second reads), and sizes beyond
the array rejected."""
import numpy as np
import pytest

from helpers import log

pytestmark = pytest.mark.gpu


def _forward_pair(P, torch, n, seed):
    from paper_1709_04703_amd.train import init_params
    rng = np.random.Generator(np.random.PCG64(seed))
    r = torch.as_tensor(rng.normal(size=n**3).astype(np.float32)).cuda()
    phi = torch.as_tensor(rng.normal(size=n**3).astype(np.float32)).cuda()
    params = torch.as_tensor(init_params(seed)).cuda()
    act0 = torch.zeros((n**3, 16), dtype=torch.int16, device="cuda")
    P.net_prep(n, r, phi, 0.7, 1.3, 0.2, act0)
    a = torch.zeros_like(act0)
    b = torch.zeros_like(act0)
    ref = torch.zeros(n**3, dtype=torch.float32, device="cuda")
    P.net_forward(n, params, act0, a, b, ref)
    got = torch.full((n**3,), float("nan"), dtype=torch.float32, device="cuda")
    P.net_forward_noalloc(n, params, act0, got)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_forward_matches_allocating_forward():
    import torch
    import paper_1709_04703_amd as P
    for n, seed in ((64, 5), (32, 6)):
        log(f"net_forward_noalloc n={n}")
        got, ref = _forward_pair(P, torch, n, seed)
        assert np.isfinite(ref).all()
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), n


def test_noalloc_forward_rejects_sizes_beyond_its_scratch():
    import torch
    import paper_1709_04703_amd as P
    n = 128
    act0 = torch.zeros((16, 16), dtype=torch.int16, device="cuda")
    out = torch.zeros(16, dtype=torch.float32, device="cuda")
    params = torch.zeros(P.NET_PARAMS, dtype=torch.float32, device="cuda")
    with pytest.raises(P.SdpmError) as e:
        P.net_forward_noalloc(n, params, act0, out)
    assert "exceeds" in str(e.value)
