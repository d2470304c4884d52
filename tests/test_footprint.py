"""Footprint accounting used by serving admission (host only, no GPU)."""
from paper_1709_06924_amd import scvt


def test_footprint_grows_with_n_and_history():
    a = scvt.footprint(10000, m_hist=7)
    b = scvt.footprint(20000, m_hist=7)
    c = scvt.footprint(20000, m_hist=10)
    assert 0 < a < b < c
    # history ring: 2 (M+1) vectors of 3n doubles
    assert c - b >= 2 * 3 * 20000 * 3 * 8
    # per-generator bytes at 1M stay in the low kilobytes
    assert scvt.footprint(1 << 20, m_hist=10) / (1 << 20) < 4096
