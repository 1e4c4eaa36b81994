"""GPU: the streaming-read calibration kernel reads every byte of its buffer once (its
result is the XOR of the buffer's 8-byte words)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096, (1 << 20) + 48, 64 << 20])
def test_stream_read_covers_the_buffer(nbytes):
    import torch
    from paper_2001_07158_amd import tpm
    torch.cuda.set_device(0)
    rng = np.random.default_rng(nbytes)
    host = rng.integers(0, 2**63, nbytes // 8, dtype=np.int64)
    a = torch.from_numpy(host).cuda()
    out = torch.full((1,), 12345, dtype=torch.int64, device="cuda")
    tpm.tpm_stream_read(a, nbytes, out, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert int(out.cpu()[0]) == int(np.bitwise_xor.reduce(host))
    with pytest.raises(tpm.TpmError):
        tpm.tpm_stream_read(a, 8, out)  # not a multiple of 16
