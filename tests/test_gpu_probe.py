"""The random-gather probe (csc_gather_probe) reads exactly the table rows its CSR pattern
names: its per-lane XORs equal a CPU computation bit for bit, including a row heavier than
the LDS stage and empty rows."""

import numpy as np
import pytest
import torch

from helpers import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("row_bytes", [64, 128, 256, 512])
def test_gather_probe_reads_the_named_rows(csc, row_bytes):
    say(f"gather probe, {row_bytes}-byte rows")
    rng = np.random.default_rng(row_bytes)
    n_rows, n_table = 3001, 5000
    deg = rng.integers(0, 30, size=n_rows)
    deg[7] = 3000  # more entries than one block stages
    deg[8] = 0
    rowptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    colidx = rng.integers(0, n_table, size=int(rowptr[-1]))
    lanes = row_bytes // 16
    table = rng.integers(0, 2**31, size=(n_table, lanes * 4), dtype=np.int64).astype(np.uint32)
    out = csc.gather_probe(torch.from_numpy(rowptr.astype(np.int32)).cuda(),
                           torch.from_numpy(colidx.astype(np.int32)).cuda(),
                           torch.from_numpy(table.view(np.int32)).cuda(), row_bytes)
    got = out.cpu().numpy().view(np.uint32).reshape(n_rows, lanes)
    # lane q of row r: XOR over the row's entries of the four words of piece q
    pieces = np.bitwise_xor.reduce(table.reshape(n_table, lanes, 4), axis=2)  # (n_table, lanes)
    want = np.zeros((n_rows, lanes), dtype=np.uint32)
    for r in range(n_rows):
        c = colidx[rowptr[r]:rowptr[r + 1]]
        if len(c):
            want[r] = np.bitwise_xor.reduce(pieces[c], axis=0)
    assert np.array_equal(got, want)


def test_gather_probe_rejects_other_row_sizes(csc):
    rp = torch.zeros(2, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    tb = torch.zeros(64, dtype=torch.int32, device="cuda")
    with pytest.raises(csc.CscError):
        csc.gather_probe(rp, ci, tb, 96)
