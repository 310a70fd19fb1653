"""The allocation-free weight gradient (unet_conv3x3_wgrad_noalloc) against
the entry point that takes a caller-allocated scratch buffer, through the
C ABI: two calls in a row, the second on a smaller input, each bitwise equal
to unet_conv3x3_wgrad (the same kernels; fixed-order sums).  The second call
reuses the library-held array that the first left filled."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_08666_amd import surrogate
    surrogate.lib()
    return surrogate


def _bits(a):
    import torch
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
    b = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return torch.from_numpy(b.view(np.int16)).cuda()


@pytest.mark.parametrize("shape", [[(2, 40, 33, 32, 64), (1, 12, 9, 16, 24)]])
def test_noalloc_wgrad_matches_scratch_entry_point(S, shape):
    import torch
    L = S.lib()
    rng = np.random.default_rng(17)
    for n, h, w, cin, cout in shape:
        print(f"[no-alloc] wgrad n={n} h={h} w={w} cin={cin} cout={cout}", flush=True)
        x = _bits(rng.normal(size=(n, h, w, cin)))
        dy = _bits(rng.normal(size=(n, h, w, cout)))
        part = torch.zeros(int(L.unet_wgrad_scratch_floats(n, h, w, cin, cout, 9)), dtype=torch.float32,
                           device="cuda")
        outs = []
        for noalloc in (False, True):
            dw = torch.full((cout, 3, 3, cin), 7.0, dtype=torch.float32, device="cuda")
            db = torch.full((cout,), 7.0, dtype=torch.float32, device="cuda")
            if noalloc:
                st = L.unet_conv3x3_wgrad_noalloc(x.data_ptr(), n, h, w, cin, cin, 0, dy.data_ptr(), cout, cout, 0,
                                                  dw.data_ptr(), db.data_ptr(), 0, None)
            else:
                st = L.unet_conv3x3_wgrad(x.data_ptr(), n, h, w, cin, cin, 0, dy.data_ptr(), cout, cout, 0,
                                          dw.data_ptr(), db.data_ptr(), part.data_ptr(), 0, None)
            assert st == 0
            torch.cuda.synchronize()
            outs.append((dw.cpu().numpy(), db.cpu().numpy()))
        assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
        assert np.abs(outs[1][0]).max() > 0
