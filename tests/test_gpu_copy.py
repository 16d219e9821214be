"""The streaming reference the benchmarks time beside the sweeps
(bb_copy_tiles): an exact copy, with its argument checks."""
import pytest
import torch

from paper_2107_05395_amd import BandBatchError
from paper_2107_05395_amd.solver import copy_tiles

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [0, 2, 1024, 1024 + 2, 3 * 2048 + 1026])
def test_copy_tiles_is_exact(n):
    src = torch.randn(n, dtype=torch.float64, device="cuda")
    dst = torch.full_like(src, float("nan"))
    copy_tiles(src, dst)
    assert torch.equal(dst, src)


def test_copy_tiles_rejects_bad_arguments():
    src = torch.randn(4096, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        copy_tiles(src, torch.empty(4094, dtype=torch.float64, device="cuda"))
    with pytest.raises(BandBatchError):
        copy_tiles(src[1:2049], torch.empty(2048, dtype=torch.float64, device="cuda"))   # 8-byte offset
    with pytest.raises(BandBatchError):
        copy_tiles(src[:2048], src[1024:3072])                                          # overlap


def test_copy_rows_is_a_copy_and_keeps_other_columns():
    """bb_copy_rows (the sweeps' access pattern): dst equals src bitwise on the
    n x m batch, and the columns past m of a wider array stay untouched."""
    from paper_2107_05395_amd.solver import copy_rows
    n, m, ld = 256, 96, 130
    src = torch.rand(n, ld, dtype=torch.float64, device="cuda")
    dst = torch.full((n, ld), 5.0, dtype=torch.float64, device="cuda")
    copy_rows(src[:, :m], dst[:, :m])
    torch.cuda.synchronize()
    assert torch.equal(dst[:, :m], src[:, :m]) and torch.all(dst[:, m:] == 5.0)
    from paper_2107_05395_amd import BandBatchError
    with pytest.raises(BandBatchError):
        copy_rows(src[:100, :m].contiguous(), dst[:100, :m].contiguous())   # n not a multiple of 128
