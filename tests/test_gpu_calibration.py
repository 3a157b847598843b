"""Calibration kernels: the plain streaming copy and the copy with the y/z
sweep's memory pattern move every value exactly once and touch nothing
else (ragged grids, padded field pitch, segment lengths that do not divide
the pencil, one longer than it)."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def B(torch):
    from paper_1206_0919_amd import binding
    return binding


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("axis", [1, 2])
@pytest.mark.parametrize("seg_len", [5, 16, 64])
def test_march_copy_is_an_exact_copy(torch, B, precision, axis, seg_len):
    dims = (37, 29, 23)
    ncell = dims[0] * dims[1] * dims[2]
    pitch = ncell + 40
    dt = torch.float64 if precision == B.FP64 else torch.float32
    g = torch.Generator(device="cpu").manual_seed(7 + axis + seg_len)
    src = torch.randn(5 * pitch, generator=g, dtype=torch.float64).to(dt).cuda()
    dst = torch.full_like(src, -7.0)
    print(f"march_copy axis={axis} seg_len={seg_len} precision={precision}", flush=True)
    st = torch.cuda.current_stream()
    B.march_copy(src, dst, dims, pitch, axis, seg_len, precision, st)
    torch.cuda.synchronize()
    s = src.view(5, pitch)
    d = dst.view(5, pitch)
    assert torch.equal(d[:, :ncell], s[:, :ncell])
    assert torch.all(d[:, ncell:] == -7.0)     # the padding between fields is left alone


def test_stream_copy_is_an_exact_copy(torch, B):
    n = (3 << 20) + 48                          # bytes: not a multiple of the chunking
    src = torch.arange(n // 8, dtype=torch.float64, device="cuda")
    dst = torch.full((n // 8 + 4,), -1.0, dtype=torch.float64, device="cuda")
    B.stream_copy(src, dst, n, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert torch.equal(dst[: n // 8], src)
    assert torch.all(dst[n // 8:] == -1.0)
