"""Host-side status handling of the MD drivers: a failed evaluation on a step
that is not sampled must still raise (every step's result row, or the
run-wide folded status of the graph-launched run, is checked)."""
import ctypes

import pytest

from paper_2510_21230_amd import _lib

STRIDE = 128


def _rows(statuses, energies):
    buf = bytearray(STRIDE * len(statuses))
    for q, (st, e) in enumerate(zip(statuses, energies)):
        r = _lib.Result()
        r.e_lj = e
        r.status = st
        buf[q * STRIDE:q * STRIDE + ctypes.sizeof(_lib.Result)] = bytes(r)
    return bytes(buf)


def test_all_ok_returns_sampled_rows():
    host = _rows([0] * 6, [0.0, -1.0, -2.0, -3.0, -4.0, -5.0])
    out = _lib.rows_from_bytes(host, STRIDE, [1, 3], range(6))
    assert out.shape == (2, 4) and out[0, 0] == -1.0 and out[1, 0] == -3.0


def test_failure_on_unsampled_step_raises():
    # eager run of 5 steps sampled every 2: rows 1 and 3 are sampled, the
    # failure sits on step 3 (row 2), which is not
    host = _rows([0, 0, _lib.ATM3_EOVERFLOW, 0, 0, 0], [0.0] * 6)
    with pytest.raises(_lib.Atm3Error) as ei:
        _lib.rows_from_bytes(host, STRIDE, [1, 3], range(6))
    assert ei.value.code == _lib.ATM3_EOVERFLOW


def test_folded_status_row_of_graph_run_raises():
    # graph run: rows 0..1 sampled (both fine), row 2 holds the folded status
    host = _rows([0, 0, _lib.ATM3_ERANGE], [0.0] * 3)
    with pytest.raises(_lib.Atm3Error):
        _lib.rows_from_bytes(host, STRIDE, [0, 1], [2])
