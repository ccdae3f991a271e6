"""The allocation-free Gram entry point (gplhr_gram_noalloc) against the
allocating one (gplhr_gram), through the C ABI: two calls in a row on the
shared per-GPU scratch array, the second with a smaller input, in both
precisions; and both against the FP64 definition X^H Y on the CPU."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _rand(rng, n, w, dtype):
    import torch
    X = (rng.standard_normal((n, w)) + 1j * rng.standard_normal((n, w))) / np.sqrt(2)
    return torch.as_tensor(X).to(dtype).to("cuda")


@pytest.mark.parametrize("dtype_name", ["complex128", "complex64"])
def test_gram_noalloc_matches_gram(device, dtype_name):
    import torch
    from paper_1506_06829_amd import gplhr as G
    dtype = getattr(torch, dtype_name)
    rng = np.random.default_rng(77)
    # the widest shape first (its partials fill the most scratch), then a
    # smaller one that reuses the array the first call left behind
    for n, bx, by in [(300007, 64, 64), (4099, 10, 7)]:
        X = _rand(rng, n, bx, dtype)
        Y = _rand(rng, n, by, dtype)
        out = torch.full((by, bx), float("nan"), dtype=torch.complex128, device="cuda")
        Gn = G.gram_noalloc(X, Y, out).cpu().numpy()
        Ga = G.gram(X, Y).cpu().numpy()
        torch.cuda.synchronize()
        Xh = X.to(torch.complex128).cpu().numpy()
        Yh = Y.to(torch.complex128).cpu().numpy()
        ref = Xh.conj().T @ Yh
        # FP64 accumulation: each entry within 1e-12 (about 1e4 unit
        # roundoffs) of the sum of the absolute products it adds up
        bound = 1e-12 * (np.abs(Xh).T @ np.abs(Yh))
        print(f"gram_noalloc {dtype_name} n={n} {bx}x{by}: |noalloc - gram| = "
              f"{np.abs(Gn - Ga).max():.2e}, |noalloc - X^H Y| = {np.abs(Gn - ref).max():.2e}",
              flush=True)
        assert np.all(np.isfinite(Gn))
        assert np.all(np.abs(Gn - Ga) <= bound)
        assert np.all(np.abs(Gn - ref) <= bound)
