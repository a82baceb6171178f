"""The memory-system probe used for the rooflines does what it reports:
the read-modify-write kind adds exactly once per access (the counts sum to
the number of accesses and the three sums to 3, 5 and 7 times it), the copy
kind copies, the compare-and-swap kind claims at most one word per access,
and every kind stays inside its buffer (a guard region after it is left
untouched)."""
import pytest
import torch

import paper_1902_05942_amd as pf

pytestmark = pytest.mark.gpu


def _buf(nbytes, guard=4096):
    whole = torch.zeros(nbytes + guard, dtype=torch.uint8, device="cuda")
    return whole, whole[:nbytes], whole[nbytes:]


def test_cell_rmw_adds_once_per_access(gpu):
    whole, buf, guard = _buf(1 << 20)
    n = pf.microbench(pf.MB_RMW, buf, 32, 3, seed=5)
    torch.cuda.synchronize()
    cells = buf.view(torch.int64).view(-1, 4)
    counts = buf.view(torch.int32).view(-1, 8)[:, 1]
    assert int(counts.sum()) == n
    assert [int(cells[:, k].sum()) for k in (1, 2, 3)] == [3 * n, 5 * n, 7 * n]
    assert int(guard.sum()) == 0


def test_copy_and_gather_scatter_cas_stay_in_bounds(gpu):
    whole, buf, guard = _buf(1 << 22)
    src = buf[: 1 << 21]
    src.copy_(torch.randint(0, 256, (1 << 21,), dtype=torch.uint8, device="cuda"))
    pf.microbench(pf.MB_COPY, buf)
    torch.cuda.synchronize()
    assert torch.equal(buf[1 << 21:], src)
    for kind, grain in ((pf.MB_GATHER, 16), (pf.MB_GATHER, 64), (pf.MB_SCATTER, 32), (pf.MB_CAS, 32)):
        pf.microbench(kind, buf, grain, 2, seed=kind)
    buf.zero_()
    n = pf.microbench(pf.MB_CAS, buf, 32, 1, seed=9)
    torch.cuda.synchronize()
    first = buf.view(torch.int32).view(-1, 8)[:, 0]
    assert 0 < int((first != 0).sum()) <= n
    assert int(guard.sum()) == 0
