"""The bandwidth probe (the lattice update's memory pattern without its
arithmetic) writes f * 0.5 + 1e-3 * (sum of the node's values) to every
output array, in both layouts: checked against the same expression on the
host, so that the bytes it is timed on are the bytes it was asked to move."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("streams", [1, 4, 19])
@pytest.mark.parametrize("tiled", [0, 1])
@pytest.mark.parametrize("dtype", ["float32", "float16"])
def test_stream_probe_values(streams, tiled, dtype):
    import torch
    from paper_2308_05007_amd import binding as B
    B.lib()
    n = 256 * 5
    rng = np.random.default_rng(streams + 10 * tiled)
    h = rng.uniform(-1, 1, streams * n).astype(np.float32)
    if dtype == "float16":
        h = h.astype(np.float16).astype(np.float32)  # representable inputs
    src = torch.from_numpy(h).cuda().to(getattr(torch, dtype))
    dst = torch.full_like(src, float("nan"))
    B.stream_probe(streams, tiled, src, dst)
    torch.cuda.synchronize()
    g = dst.float().cpu().numpy()
    if tiled:
        v = h.reshape(n // 256, streams, 256)
        ref = v * np.float32(0.5) + v.sum(axis=1, dtype=np.float32, keepdims=True) * np.float32(1e-3)
    else:
        v = h.reshape(streams, n)
        ref = v * np.float32(0.5) + v.sum(axis=0, dtype=np.float32, keepdims=True) * np.float32(1e-3)
    # the sum's order differs between the host and the kernel; halves round
    # the result to 11 significant bits
    tol = 1e-6 * streams if dtype == "float32" else 2.0 ** -11 * (np.abs(ref).max() + 1e-3 * streams)
    assert np.abs(g - ref.reshape(-1)).max() <= tol
    assert np.isfinite(g).all()
