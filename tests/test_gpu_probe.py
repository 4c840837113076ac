"""The bandwidth and gather probes the benchmark measures its kernels
against: their results are exact on known data, and the binding refuses
buffers too small for the launch."""
import numpy as np
import pytest

import paper_2203_02530_amd as sp

pytestmark = pytest.mark.gpu


def test_probes_on_known_data():
    import torch
    assert torch.cuda.is_available()
    n = 1 << 20                                     # doubles
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    part = torch.zeros(4096, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    # read: every double once, one partial per block, summing to n
    sp.spmv_hbm_probe(0, src, part, n * 8, 512, stream)
    torch.cuda.synchronize()
    assert float(part[:512].sum()) == n
    # copy: dst == src
    dst = torch.zeros_like(src)
    sp.spmv_hbm_probe(1, src, dst, n * 8, 256, stream)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    # gathers of ones: each block sums exactly its gathers, in its window
    # (a window of ones for the per-XCD mode and zeros elsewhere shows that
    # block b only reads window b mod 8)
    per = sp.spmv_gathers_per_probe_block()
    w = n // 8
    marked = torch.zeros(n, dtype=torch.float64, device="cuda")
    for k in range(8):
        marked[k * w:(k + 1) * w] = float(k + 1)
    for mode in (2, 3):
        part.zero_()
        sp.spmv_hbm_probe(mode, src, part, n * 8, 64, stream)
        torch.cuda.synchronize()
        assert np.all(part[:64].cpu().numpy() == per)
    part.zero_()
    sp.spmv_hbm_probe(2, marked, part, n * 8, 64, stream)
    torch.cuda.synchronize()
    got = part[:64].cpu().numpy()
    assert np.all(got == per * (np.arange(64) % 8 + 1))
    # buffers too small for the launch are refused before it
    with pytest.raises(ValueError):
        sp.spmv_hbm_probe(0, src, part, n * 8, 8192, stream)      # part < 8192 doubles
    with pytest.raises(ValueError):
        sp.spmv_hbm_probe(1, src, part, n * 8, 64, stream)         # dst < n doubles
    with pytest.raises(TypeError):
        sp.spmv_hbm_probe(0, src.cpu(), part, n * 8, 64, stream)
