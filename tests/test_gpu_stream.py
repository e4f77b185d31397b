"""The streaming probes the bench reads its HBM ceilings from: the copy is byte-exact
(including lengths that leave a partial batch of vectors) and the read pass reads every
word: with one nonzero word in a zero buffer, exactly one lane folds to that word, so
the sink is written with it exactly when the key names it."""
import numpy as np
import pytest
import torch

import paper_2203_07673_amd as F
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

SIZES = [4, 1020, 4096 * 257 + 12]


@pytest.mark.parametrize("nwords", SIZES)
def test_stream_copy_is_exact(nwords):
    log(f"stream copy nwords={nwords}")
    data = np.random.default_rng(nwords).integers(-2**31, 2**31, size=nwords, dtype=np.int64).astype(np.int32)
    src = torch.from_numpy(data).cuda()
    dst = torch.full((nwords + 4,), 7, dtype=torch.int32, device="cuda")
    F.stream_copy(src, dst[:nwords])
    out = dst.cpu().numpy()
    assert np.array_equal(out[:nwords], data) and (out[nwords:] == 7).all()


@pytest.mark.parametrize("nwords", SIZES)
def test_stream_read_reaches_every_position(nwords):
    log(f"stream read nwords={nwords}")
    marker = 0x2545F491
    for pos in sorted({0, nwords // 2, nwords - 1}):
        buf = torch.zeros(nwords, dtype=torch.int32, device="cuda")
        buf[pos] = marker
        sink = torch.zeros(1, dtype=torch.int32, device="cuda")
        F.stream_read(buf, sink, key=marker + 1)      # no lane folds to this
        assert int(sink.item()) == 0
        F.stream_read(buf, sink, key=marker)          # the lane that read buf[pos] does
        assert int(sink.item()) == marker, pos


def test_stream_probe_errors():
    x = torch.zeros(6, dtype=torch.int8, device="cuda")
    with pytest.raises(F.FmmError):
        F.stream_copy(x, torch.zeros(6, dtype=torch.int8, device="cuda"))  # 6 bytes: not a multiple of 16
    with pytest.raises(ValueError):
        F.stream_copy(torch.zeros(8, device="cuda"), torch.zeros(4, device="cuda"))
