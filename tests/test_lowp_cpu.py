"""CPU checks of the low-precision reference helpers."""
import numpy as np

from tests.lowp import e4m3_decode, e4m3_encode, e4m3_table


def test_e4m3_table_landmarks():
    t = e4m3_table()
    assert t[0x7E] == 448.0 and t[0xFE] == -448.0
    assert np.isnan(t[0x7F]) and np.isnan(t[0xFF])
    assert t[0x08] == 2.0 ** -6          # smallest normal
    assert t[0x01] == 2.0 ** -9          # smallest subnormal
    assert t[0x38] == 1.0


def test_e4m3_round_trip_and_ties():
    t = e4m3_table()
    finite = np.array([c for c in range(256) if not np.isnan(t[c]) and c not in (0x80,)])
    np.testing.assert_array_equal(e4m3_encode(t[finite]), finite)
    # halfway between 1.0 (code 0x38, even) and 1.125 (0x39): ties to even
    assert e4m3_encode(np.array([1.0625]))[0] == 0x38
    # halfway between 1.125 (0x39) and 1.25 (0x3A): to 0x3A
    assert e4m3_encode(np.array([1.1875]))[0] == 0x3A
    assert e4m3_encode(np.array([1000.0]))[0] == 0x7E
    assert e4m3_decode(e4m3_encode(np.array([-3.3])))[0] == -3.25
