"""lgs_bin_sort_noalloc (workspace in the library's static device array) against
lgs_bin_sort with a caller workspace: identical pair order, tile ranges and pair count,
on two calls in a row, the second with a smaller input (so the array holds the first
call's contents when the second starts)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_06991_amd import lgs
    lgs.load()
    return t


def _bins(n, W, H, seed):
    rng = np.random.default_rng(seed)
    ntx, nty = (W + 15) // 16, (H + 15) // 16
    tx0 = rng.integers(0, ntx, n)
    ty0 = rng.integers(0, nty, n)
    wide = rng.random(n) < 0.005
    tx1 = np.minimum(tx0 + np.where(wide, rng.integers(1, 40, n), rng.integers(1, 4, n)), ntx)
    ty1 = np.minimum(ty0 + np.where(wide, rng.integers(1, 30, n), rng.integers(1, 4, n)), nty)
    touched = ((tx1 - tx0) * (ty1 - ty0)).astype(np.int32)
    touched[rng.random(n) < 0.2] = 0
    depth = rng.choice(rng.uniform(0.3, 9.0, max(n // 3, 1)).astype(np.float32), n)   # depth ties
    rect = np.stack([tx0, ty0, tx1, ty1], 1).astype(np.int32)
    return depth, rect, touched


def _camera(W, H):
    from paper_2602_06991_amd import lgs
    cam = lgs.lgs_camera()
    cam.width, cam.height, cam.fx, cam.fy = W, H, 1.0, 1.0
    return cam


def _with_workspace(torch, cam, n, depth, rect, touched, cap):
    from paper_2602_06991_amd import lgs
    need = lgs.lgs_bin_sort_workspace(n, cam.width, cam.height, cap)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) // 256 * 256
    ids = torch.full((cap,), -5, dtype=torch.int32, device="cuda")
    T = ((cam.width + 15) // 16) * ((cam.height + 15) // 16)
    ranges = torch.full((T, 2), -5, dtype=torch.int32, device="cuda")
    st, m = lgs.lgs_bin_sort(cam, n, depth.data_ptr(), rect.data_ptr(), touched.data_ptr(), base, need, cap,
                             ids.data_ptr(), ranges.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert st == lgs.LGS_OK
    return ids, ranges, m


def _without(torch, cam, n, depth, rect, touched, cap):
    from paper_2602_06991_amd import lgs
    ids = torch.full((cap,), -5, dtype=torch.int32, device="cuda")
    T = ((cam.width + 15) // 16) * ((cam.height + 15) // 16)
    ranges = torch.full((T, 2), -5, dtype=torch.int32, device="cuda")
    st, m = lgs.lgs_bin_sort_noalloc(cam, n, depth.data_ptr(), rect.data_ptr(), touched.data_ptr(), cap,
                                     ids.data_ptr(), ranges.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return st, ids, ranges, m


def test_no_alloc_bin_sort_matches_workspace_call(torch):
    from paper_2602_06991_amd import lgs
    for (n, W, H, seed) in [(100000, 1200, 680, 21), (20000, 640, 480, 22)]:
        depth, rect, touched = _bins(n, W, H, seed)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        d, r, t = dev(depth), dev(rect), dev(touched)
        cam = _camera(W, H)
        cap = int(touched.sum()) + 1000
        ids0, ranges0, m0 = _with_workspace(torch, cam, n, d, r, t, cap)
        st, ids1, ranges1, m1 = _without(torch, cam, n, d, r, t, cap)
        torch.cuda.synchronize()
        print(f"n={n} {W}x{H}: {m1} pairs", flush=True)
        assert st == lgs.LGS_OK and m1 == m0 == int(touched.sum())
        assert torch.equal(ids1, ids0)
        assert torch.equal(ranges1, ranges0)
    # a pair buffer that is too small: the need is reported and the outputs stay untouched
    st, ids2, ranges2, m2 = _without(torch, cam, n, d, r, t, m0 // 2)
    torch.cuda.synchronize()
    assert st == lgs.LGS_ERR_CAPACITY and m2 == m0
    assert int(ids2.ne(-5).sum()) == 0 and int(ranges2.ne(-5).sum()) == 0


def test_no_alloc_bin_sort_rejects_sizes_beyond_its_scratch():
    """Host validation only (no launch): a request whose workspace exceeds the static
    64 MiB is refused with INVALID_ARG and a message naming the limit."""
    from paper_2602_06991_amd import lgs
    cam = _camera(1200, 680)
    F = 0x100000
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_bin_sort_noalloc(cam, 3_000_000, F, F, F, 8_000_000, F, F)
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG and "scratch" in str(e.value)
    assert lgs.lgs_bin_sort_workspace(3_000_000, 1200, 680, 8_000_000) > 64 << 20
