"""The ceiling-measurement kernels compute what include/tsqr_peaks.h says:
the copy is exact on sizes that leave a ragged grid-stride tail, the read's
partial sums add up to the sum of the buffer, and the FMA and MFMA loops reach
their closed-form results (integers, so exact)."""
import pytest

from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("elems16,grid", [(1, 0), (4096 * 256 * 4 + 37, 0), (1000003, 7), (5, 64), (1000003, 1 << 20)])
def test_copy_and_read(elems16, grid):
    torch = need_gpu()
    from paper_0809_2407_amd import peaks as PK

    announce(f"peaks copy/read {elems16} x 16 B, grid {grid}")
    g = torch.Generator(device="cuda")
    g.manual_seed(elems16)
    src = torch.rand(2 * elems16, generator=g, device="cuda", dtype=torch.float64)
    dst = torch.full_like(src, -7.0)
    PK.copy(src, dst, grid=grid)
    gr = grid if grid > 0 else PK.default_grid(1, 16 * elems16)
    partial = torch.full((gr,), float("nan"), dtype=torch.float64, device="cuda")
    PK.read(src, partial, grid=grid)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    assert torch.isfinite(partial).all()
    total = float(src.sum())
    assert abs(float(partial.sum()) - total) <= 1e-12 * max(1.0, total)


@pytest.mark.parametrize("grid,iters", [(1, 0), (3, 17), (0, 64)])
def test_fma_and_mfma_loops(grid, iters):
    torch = need_gpu()
    from paper_0809_2407_amd import peaks as PK

    announce(f"peaks fma/mfma grid {grid} iters {iters}")
    gr = grid if grid > 0 else PK.default_grid(2)
    out = torch.full((gr * 256,), float("nan"), dtype=torch.float64, device="cuda")
    PK.fma(out, iters, 1.0, 1.0, grid=grid)
    torch.cuda.synchronize()
    assert bool((out == 28.0 + 8.0 * iters).all())
    out.fill_(float("nan"))
    PK.mfma(out, iters, 0.5, 0.5, grid=grid)
    torch.cuda.synchronize()
    assert bool((out == 256.0 * iters).all())
    PK.mfma(out, iters, 1.5, -2.0, grid=grid)
    torch.cuda.synchronize()
    assert bool((out == 1024.0 * 1.5 * -2.0 * iters).all())


@pytest.mark.parametrize("m,n,leaf_rows,tile_rows,pad", [(20000 + 37, 32, 2048, 128, 0), (9000, 17, 1024, 128, 5),
                                                          (6000 + 3, 64, 512, 64, 0), (100, 5, 128, 16, 2),
                                                          (15, 1, 64, 16, 0)])
def test_copy_in_leaf_pattern(m, n, leaf_rows, tile_rows, pad):
    torch = need_gpu()
    from paper_0809_2407_amd import peaks as PK
    from paper_0809_2407_amd import tsqr as T

    announce(f"peaks copy_leaf {m}x{n} leaf {leaf_rows} tile {tile_rows} pad {pad}")
    g = torch.Generator(device="cuda")
    g.manual_seed(m + n)
    src = T.colmajor(m, n, ld=m + pad)
    src.copy_(torch.rand((m, n), generator=g, device="cuda", dtype=torch.float64))
    dst = T.colmajor(m, n, ld=m + 2 * pad)
    dst.fill_(-3.0)
    PK.copy_leaf(src, dst, leaf_rows, tile_rows)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
