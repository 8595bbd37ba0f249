"""The C-ABI library loads without a GPU, exports every entry point include/lgs.h
declares, and rejects bad arguments on the host before any launch."""
import ctypes
import os
import re

import pytest

from paper_2602_06991_amd import lgs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lgs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lgs_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    L = lgs.load()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
        assert n in lgs.EXPORTS, n


def test_version_and_k_set():
    assert lgs.lgs_abi_version() == 2
    assert lgs.lgs_supported_k() == [1, 2, 3, 4, 5, 8, 10, 16]


def _cam(W=64, H=48, f=50.0):
    c = lgs.lgs_camera()
    for i, v in enumerate([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]):
        c.Rt[i] = v
    c.fx = c.fy = f
    c.cx, c.cy, c.width, c.height = W / 2, H / 2, W, H
    return c


FAKE = 0x100000  # a 16-byte-aligned non-null address; never dereferenced by validation


def test_project_validation():
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_project_fwd(_cam(W=0), 4, *([FAKE] * 11))
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_project_fwd(_cam(f=-1.0), 4, *([FAKE] * 11))
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_project_fwd(_cam(), 4, FAKE, None, *([FAKE] * 9))
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    with pytest.raises(lgs.LgsError):
        lgs.lgs_project_fwd(_cam(), -1, *([FAKE] * 11))
    assert "NULL" in lgs.lgs_last_error() or "n must" in lgs.lgs_last_error()
    # n == 0 is a no-op that launches nothing
    assert lgs.lgs_project_fwd(_cam(), 0, *([None] * 11)) == lgs.LGS_OK


def test_unsupported_k_d_and_dtypes():
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_rasterize_topk_fwd(_cam(), 7, *([FAKE] * 14))
    assert e.value.status == lgs.LGS_ERR_UNSUPPORTED
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_feature_render_fwd(16, 16, 1, 4, 12, lgs.LGS_F32, FAKE, None, FAKE, FAKE, lgs.LGS_F32, FAKE)
    assert e.value.status == lgs.LGS_ERR_UNSUPPORTED
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_feature_render_fwd(16, 16, 1, 4, 16, lgs.LGS_F32, FAKE, None, FAKE, FAKE, lgs.LGS_BF16, FAKE)
    assert e.value.status == lgs.LGS_ERR_UNSUPPORTED
    with pytest.raises(lgs.LgsError) as e:   # FP8 needs a scale
        lgs.lgs_feature_render_fwd(16, 16, 1, 4, 16, lgs.LGS_FP8_E4M3, FAKE, None, FAKE, FAKE, lgs.LGS_BF16, FAKE)
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    with pytest.raises(lgs.LgsError) as e:   # misaligned map
        lgs.lgs_feature_render_fwd(16, 16, 1, 4, 16, lgs.LGS_F32, FAKE, None, FAKE, FAKE, lgs.LGS_F32, FAKE + 4)
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_feature_render_bwd(16, 16, 1, 3, 16, lgs.LGS_BF16, FAKE, None, FAKE, FAKE, lgs.LGS_BF16, FAKE,
                                   None, FAKE)
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    # the one-pass render + L1 adjoint: map and target must not overlap, nor be NULL
    fused = lambda F, T: lgs.lgs_feature_render_fwd_bwd_l1(16, 16, 1, 4, 16, lgs.LGS_BF16, FAKE, None, FAKE,
                                                           FAKE, lgs.LGS_BF16, F, T, 1.0, FAKE, FAKE)
    for F, T in ((FAKE, FAKE), (FAKE, FAKE + 16 * 16 * 16 * 2 - 16), (FAKE + 4096, FAKE), (None, FAKE),
                 (FAKE, FAKE + 8)):
        with pytest.raises(lgs.LgsError) as e:
            fused(F, T)
        assert e.value.status == lgs.LGS_ERR_INVALID_ARG, (F, T)
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_feature_render_fwd_bwd_l1(16, 16, 1, 4, 16, lgs.LGS_F32, FAKE, None, FAKE, FAKE, lgs.LGS_BF16,
                                          FAKE, FAKE + 65536, 1.0, FAKE, FAKE)
    assert e.value.status == lgs.LGS_ERR_UNSUPPORTED
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_quantize_features(10, 16, FAKE, lgs.LGS_F32, FAKE, None)
    assert e.value.status == lgs.LGS_ERR_UNSUPPORTED
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_l1_grad(10, lgs.LGS_FP8_E4M3, FAKE, FAKE, 1.0, FAKE)
    assert e.value.status == lgs.LGS_ERR_UNSUPPORTED


def test_bin_sort_workspace_and_validation():
    b0 = lgs.lgs_bin_sort_workspace(1000, 64, 48, 5000)
    b1 = lgs.lgs_bin_sort_workspace(1000, 64, 48, 50000)
    assert 0 < b0 < b1
    with pytest.raises(lgs.LgsError):
        lgs.lgs_bin_sort_workspace(-1, 64, 48, 10)
    ws = b0
    # undersized workspace and misaligned workspace are rejected before any launch
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_bin_sort(_cam(), 1000, FAKE, FAKE, FAKE, FAKE, ws - 1, 5000, FAKE, FAKE)
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_bin_sort(_cam(), 1000, FAKE, FAKE, FAKE, FAKE + 16, ws, 5000, FAKE, FAKE)
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG


def test_pose_gradient_validation():
    args = [FAKE] * 9                      # means .. dL_ddepth_g
    with pytest.raises(lgs.LgsError) as e:   # no pose output
        lgs.lgs_project_bwd_pose(_cam(), 10, *args, FAKE, FAKE, FAKE, FAKE, None)
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    with pytest.raises(lgs.LgsError) as e:   # a partial set of parameter-gradient outputs
        lgs.lgs_project_bwd_pose(_cam(), 10, *args, FAKE, None, FAKE, FAKE, FAKE)
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    assert "together" in lgs.lgs_last_error()
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_project_bwd_pose(_cam(f=0.0), 10, *args, None, None, None, None, FAKE)
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    assert lgs.lgs_project_bwd_pose(_cam(), 0, *([None] * 13), FAKE) == lgs.LGS_OK


def test_sparse_row_clearing_validation():
    # empty inputs are no-ops; bad sizes and NULL buffers are rejected before any launch
    assert lgs.lgs_mark_topk_rows(0, None, 10, 1, None) == lgs.LGS_OK
    assert lgs.lgs_zero_marked_rows(0, 8, 1, None, None) == lgs.LGS_OK
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_mark_topk_rows(-1, FAKE, 10, 1, FAKE)
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_mark_topk_rows(100, None, 10, 1, FAKE)
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_zero_marked_rows(10, 6, 1, FAKE, FAKE)      # d not a multiple of 4
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_zero_marked_rows(10, 8, 1, FAKE, FAKE + 4)  # table not 16-byte aligned
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG


def test_marked_row_quantize_validation():
    assert lgs.lgs_quantize_marked_rows(0, 8, 1, None, None, lgs.LGS_BF16, None, None) == lgs.LGS_OK
    for args, status in [((10, 12, 1, FAKE, FAKE, lgs.LGS_BF16, FAKE, None), lgs.LGS_ERR_INVALID_ARG),   # d % 8
                         ((-1, 8, 1, FAKE, FAKE, lgs.LGS_BF16, FAKE, None), lgs.LGS_ERR_INVALID_ARG),
                         ((10, 8, 1, None, FAKE, lgs.LGS_BF16, FAKE, None), lgs.LGS_ERR_INVALID_ARG),
                         ((10, 8, 1, FAKE, FAKE + 4, lgs.LGS_BF16, FAKE, None), lgs.LGS_ERR_INVALID_ARG),
                         ((10, 8, 1, FAKE, FAKE, lgs.LGS_FP8_E4M3, FAKE, None), lgs.LGS_ERR_INVALID_ARG),
                         ((10, 8, 1, FAKE, FAKE, lgs.LGS_F32, FAKE, None), lgs.LGS_ERR_UNSUPPORTED)]:
        with pytest.raises(lgs.LgsError) as e:
            lgs.lgs_quantize_marked_rows(*args)
        assert e.value.status == status, args


def test_tile_order_size_and_validation():
    # the grid (whole strips of 16 tiles over the 8 XCDs: 128 workgroups), twice
    assert lgs.lgs_tile_order_size(1200, 680, 1) == 2 * 3328   # 75 x 43 = 3225 tiles
    assert lgs.lgs_tile_order_size(640, 480, 8) == 2 * 9600    # 8 x 40 x 30
    assert lgs.lgs_tile_order_size(16, 16, 1) == 2 * 128
    assert lgs.lgs_tile_order_size(0, 480, 1) == 0
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_tile_order(_cam(), 1, None, None, FAKE)
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_tile_order(_cam(), 1, FAKE + 4, None, FAKE)    # tile_ranges not 8-byte aligned
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
    with pytest.raises(lgs.LgsError) as e:
        lgs.lgs_tile_order(_cam(f=0.0), 1, FAKE, FAKE, FAKE)
    assert e.value.status == lgs.LGS_ERR_INVALID_ARG
