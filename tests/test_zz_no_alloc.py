"""The allocation-free entry point nusht_density_map_noalloc, called through the C ABI,
against nusht_density_map (which allocates its count buffer): identical maps on two calls in
a row, the second with fewer points and a smaller map (the fixed count buffer keeps the first
call's counts until the second call clears them), and the size limit."""
import ctypes

import numpy as np
import pytest

from paper_2406_14542_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _call(lib, name, th, ph, nt, nph, out):
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return getattr(lib, name)(th.data_ptr(), ph.data_ptr(), th.numel(), nt, nph, out.data_ptr(),
                              stream)


def test_noalloc_density_map_matches_allocating_entry_point():
    import paper_2406_14542_amd as P
    lib = P.lib()
    print("[no-alloc density map]", flush=True)
    rng = np.random.default_rng(77)
    cases = [(200_000, 64, 128, 11), (3_000, 16, 40, 12)]   # second call: smaller input
    for n, nt, nph, seed in cases:
        th, ph, _ = inputs.holey_points(np.random.default_rng(seed), n)
        ph = ph + rng.uniform(-10, 10, n)          # phi outside [0, 2 pi) wraps
        tht = torch.from_numpy(th).cuda()
        pht = torch.from_numpy(ph).cuda()
        ref = torch.full((nt, nph), -1.0, dtype=torch.float32, device="cuda")
        got = torch.full((nt, nph), -2.0, dtype=torch.float32, device="cuda")
        assert _call(lib, "nusht_density_map", tht, pht, nt, nph, ref) == P.NUSHT_OK
        assert _call(lib, "nusht_density_map_noalloc", tht, pht, nt, nph, got) == P.NUSHT_OK
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(r, g), (n, nt, nph, np.abs(r - g).max())
        # the counts add up to the number of points
        a = np.arange(nt)
        area = (np.cos(np.pi * a / nt) - np.cos(np.pi * (a + 1) / nt)) * (2 * np.pi / nph)
        counts = g.astype(np.float64) * (n * area / (4 * np.pi))[:, None]
        assert abs(counts.sum() - n) < 1e-3 * n
    # beyond the fixed buffer: an error, no launch
    big = torch.empty((300, 300), dtype=torch.float32, device="cuda")
    assert _call(lib, "nusht_density_map_noalloc", tht, pht, 300, 300, big) == P.NUSHT_EINVAL
