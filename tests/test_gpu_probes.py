"""The measurement probes run on the GPU and do what their bandwidth and
rate figures assume: the LDS probe moves the bytes it reports, the record
probe touches uniform random records of the whole buffer, one read (and in
mode 1 one write) per access."""
import pytest
import torch

from paper_1809_11134_amd import qe

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qe.load()
    return torch.device("cuda", 0)


def test_lds_probe_bytes(dev):
    wg, iters = 64, 4
    sink = torch.zeros(wg * 256, dtype=torch.int32, device=dev)
    for mode, factor in ((0, 1), (1, 1), (2, 2)):
        nbytes = qe.probe_lds(mode, wg, iters, sink)
        torch.cuda.synchronize()
        assert nbytes == wg * 256 * iters * 8 * 16 * factor


def test_record_probe_touches_random_records(dev):
    count, n = 1 << 20, 1 << 18
    buf = torch.zeros((count, 4), dtype=torch.int32, device=dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    qe.probe_records(0, buf, n, sink, salt=7)          # reads change nothing
    torch.cuda.synchronize()
    assert int(buf.abs().sum()) == 0 and int(sink[0]) == 0
    qe.probe_records(1, buf, n, sink, salt=7)
    torch.cuda.synchronize()
    z = buf[:, 2].cpu()
    touched = int((z > 0).sum())
    # n uniform draws over count records: the expected number of distinct
    # records is count (1 - e^(-n / count)); racing increments of a record
    # drawn twice may count once, so the total lies between the two
    expect = count * (1 - (1 - 1 / count) ** n)
    assert abs(touched - expect) < 0.02 * expect
    assert touched <= int(z.sum()) <= n
    assert int(buf[:, 0].abs().sum()) == 0 and int(buf[:, 1].abs().sum()) == 0 and int(buf[:, 3].abs().sum()) == 0
    # spread over the whole buffer: every eighth of it is hit about equally
    per = (z > 0).reshape(8, -1).sum(dim=1).float()
    assert float(per.min()) > 0.9 * float(per.mean())
