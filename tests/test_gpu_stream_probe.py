"""The bandwidth calibration copy behind the bench's stream-probe leg: it moves
exactly the elements it names (arrays x n at offset shift in each array's
stride) and nothing else, and refuses what it cannot do."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,arrays,shift", [(0, 3, 0), (1, 1, 0), (1000, 19, 0), (1000, 19, 1), (4097, 9, 63)])
def test_stream_probe_copies_exactly_its_elements(gpu_lib, n, arrays, shift):
    import torch
    stride = (n + shift + 63) // 64 * 64 + 64
    src = torch.arange(arrays * stride, dtype=torch.float32, device="cuda")
    dst = torch.full_like(src, -1.0)
    gpu_lib.lbm_stream_probe(src, dst, n, stride, arrays, shift)
    torch.cuda.synchronize()
    got = dst.cpu().numpy().reshape(arrays, stride)
    want = np.full((arrays, stride), -1.0, np.float32)
    ref = np.arange(arrays * stride, dtype=np.float32).reshape(arrays, stride)
    want[:, shift:shift + n] = ref[:, shift:shift + n]
    assert np.array_equal(got, want)


def test_stream_probe_rejects_bad_arguments(gpu_lib):
    import torch
    src = torch.zeros(256, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    for n, stride, arrays, shift in ((10, 128, 2, 64), (10, 128, 0, 0), (-1, 128, 1, 0), (128, 128, 1, 1)):
        with pytest.raises(Exception):
            gpu_lib.lbm_stream_probe(src, dst, n, stride, arrays, shift)
    with pytest.raises(ValueError):                  # more than the buffers hold
        gpu_lib.lbm_stream_probe(src, dst, 10, 128, 3, 0)
