"""The streaming probes the bench reads its HBM ceilings from: the copy is byte-exact
(including lengths that leave a partial batch of vectors) and the read pass reads every
word: with one nonzero word in a zero buffer, exactly one lane folds to that word, so
the sink is written with it exactly when the key names it.  The gather probe reads every
word of exactly the listed rows, the same way."""
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


@pytest.mark.parametrize("row_bytes", [16, 128, 1024])
def test_stream_gather_reads_the_listed_rows(row_bytes):
    """A marker word in one row of a zero buffer reaches the sink exactly when that row is
    gathered and the key names the marker; every word position of the row is tried."""
    log(f"stream gather row_bytes={row_bytes}")
    marker = 0x2545F491
    nrows = 1000
    words = row_bytes // 4
    rng = np.random.default_rng(row_bytes)
    listed = torch.from_numpy(rng.choice(nrows, size=300, replace=False).astype(np.int32)).cuda()
    absent = int(np.setdiff1d(np.arange(nrows), listed.cpu().numpy())[0])
    present = int(listed[17])
    for row, want in ((present, marker), (absent, 0)):
        for w in sorted({0, words // 2, words - 1}):
            buf = torch.zeros(nrows * words, dtype=torch.int32, device="cuda")
            buf[row * words + w] = marker
            sink = torch.zeros(1, dtype=torch.int32, device="cuda")
            F.stream_gather(buf, row_bytes, listed, sink, key=marker + 1)  # no lane folds to this
            assert int(sink.item()) == 0
            F.stream_gather(buf, row_bytes, listed, sink, key=marker)
            assert int(sink.item()) == want, (row, w)
    with pytest.raises(ValueError):  # every index is checked against the buffer's rows first
        F.stream_gather(buf, row_bytes, torch.tensor([nrows], dtype=torch.int32, device="cuda"), sink)


def test_stream_probe_errors():
    x = torch.zeros(6, dtype=torch.int8, device="cuda")
    with pytest.raises(F.FmmError):
        F.stream_copy(x, torch.zeros(6, dtype=torch.int8, device="cuda"))  # 6 bytes: not a multiple of 16
    with pytest.raises(ValueError):
        F.stream_copy(torch.zeros(8, device="cuda"), torch.zeros(4, device="cuda"))
