"""The network's forward pass without device allocation
(cgks_mlp_forward_noalloc) against cgks_mlp_forward, through the C ABI.

Both run the same kernels, so the outputs must agree bit for bit; two calls
in a row, the second smaller, check that a call leaves nothing behind in the
shared fixed workspace that the next one depends on."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _pair(m, X):
    import torch
    n = X.shape[0]
    ref = torch.full((n, 4), float("nan"), device="cuda")
    out = torch.full((n, 4), float("nan"), device="cuda")
    m.forward_noalloc(X, out)
    m.forward(X, ref)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_forward_equals_forward_twice_shrinking():
    import torch
    from paper_2509_06347_amd import cgks
    torch.cuda.set_device(0)
    print("noalloc forward: seed 7, rows 16384 then 777", flush=True)
    m = cgks.MLP(seed=7, stream=torch.cuda.current_stream().cuda_stream)
    g = torch.Generator().manual_seed(3)
    for n in (cgks.MLP.NOALLOC_MAX_ROWS, 777):
        X = (2.0 * torch.randn(n, 5, generator=g)).cuda()
        out, ref = _pair(m, X)
        assert np.isfinite(ref).all()
        assert np.array_equal(out, ref), f"n={n}: max diff {np.abs(out - ref).max():.3e}"
    m.close()


def test_noalloc_forward_rejects_rows_beyond_the_workspace():
    import torch
    from paper_2509_06347_amd import cgks
    torch.cuda.set_device(0)
    m = cgks.MLP(seed=1, stream=torch.cuda.current_stream().cuda_stream)
    n = cgks.MLP.NOALLOC_MAX_ROWS + 1
    X = torch.zeros(n, 5, device="cuda")
    Y = torch.full((n, 4), 7.0, device="cuda")
    with pytest.raises(cgks.CgksError) as e:
        m.forward_noalloc(X, Y)
    assert e.value.code == cgks.ELIMIT
    torch.cuda.synchronize()
    assert bool((Y == 7.0).all())          # nothing ran
    Y0 = torch.zeros(0, 4, device="cuda")
    m.forward_noalloc(torch.zeros(0, 5, device="cuda"), Y0)   # zero rows: a no-op
    m.close()
