"""Host-side argument marshalling of the Python binding (no GPU): the band table handed to
mm_plan, from a list of per-band arrays or from a BandTable already in the ABI's layout."""

import numpy as np
import pytest

from paper_2112_03370_amd import mapmaker as mm


def test_band_arrays_from_list_and_from_table():
    bands = [np.arange(3, dtype=np.float32), np.arange(5, dtype=np.float32) + 10]
    nc, off, coef, nb = mm.band_arrays(bands)
    assert nb == 2 and nc.tolist() == [3, 5] and off.tolist() == [0, 3]
    assert coef.dtype == np.float32 and coef.tolist() == [0, 1, 2, 10, 11, 12, 13, 14]
    nc2, off2, coef2, nb2 = mm.band_arrays(mm.BandTable(nc, off, coef))
    assert nb2 == 2
    assert np.array_equal(nc2, nc) and np.array_equal(off2, off) and np.array_equal(coef2, coef)
    assert nc2.dtype == np.int32 and off2.dtype == np.int64 and coef2.dtype == np.float32


def test_band_table_shared_coefficients_and_empty():
    # two bands may share coefficients (offsets need not be increasing); no bands at all is a
    # one-element placeholder the library never reads
    coef = np.arange(6, dtype=np.float32)
    nc, off, c, nb = mm.band_arrays(mm.BandTable(np.array([4, 4], np.int32),
                                                 np.array([2, 0], np.int64), coef))
    assert nb == 2 and off.tolist() == [2, 0] and c.size == 6
    assert mm.band_arrays([])[3] == 0


def test_band_table_rejects_inconsistent_tables():
    nc = np.array([3, 5], np.int32)
    off = np.array([0, 3], np.int64)
    coef = np.zeros(8, np.float32)
    with pytest.raises(ValueError):
        mm.band_arrays(mm.BandTable(nc, off[:1], coef))
    with pytest.raises(ValueError):
        mm.band_arrays(mm.BandTable(nc, off, coef[:7]))
    with pytest.raises(ValueError):
        mm.band_arrays(mm.BandTable(nc, np.array([0, -1], np.int64), coef))
