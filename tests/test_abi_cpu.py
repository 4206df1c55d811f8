"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastid.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fid_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    import paper_1707_00516_amd as fid
    lib = ctypes.CDLL(fid.LIB_PATH)
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(fid.EXPORTS) == names


def test_status_strings_and_row_words():
    import paper_1707_00516_amd as fid
    assert fid.fid_status_str(0) == "FID_OK"
    assert "invalid" in fid.fid_status_str(fid.FID_EINVAL)
    assert fid.fid_row_words(1) == 2 and fid.fid_row_words(128) == 2
    assert fid.fid_row_words(129) == 4 and fid.fid_row_words(2048) == 32
    assert fid.fid_row_words(32768) == 512
    assert fid.fid_row_words(0) == -1 and fid.fid_row_words(65536) == -1
    assert fid.fid_version() >= 100


def test_db_bytes_and_validation():
    import paper_1707_00516_amd as fid
    # 20M x 2048 loci, padded to whole 1024-reference tiles (20,000,768 rows):
    # 256 B of words per row + four 1 KiB unit planes of slack, then 4 B of
    # popcount per row.
    padded = -(-20_000_000 // 1024) * 1024
    assert fid.fid_db_bytes(20_000_000, 2048) == padded * 256 + 4096 + padded * 4
    assert fid.fid_db_bytes(1, 1) == 1024 * 16 + 4096 + 1024 * 4
    with pytest.raises(fid.FidError) as e:
        fid.fid_db_bytes(0, 2048)
    assert e.value.status == fid.FID_EINVAL
    with pytest.raises(fid.FidError):
        fid.fid_db_bytes(10, 0)
    with pytest.raises(fid.FidError) as e:
        fid.fid_compare_full(0, 0, 0, 1, 0, 0, 1)
    assert e.value.status == fid.FID_EINVAL and "ctx" in fid.fid_last_error()


def test_no_device_is_reported():
    import torch
    import paper_1707_00516_amd as fid
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(fid.FidError) as e:
        fid.fid_ctx_create(0, 0)
    assert e.value.status == fid.FID_ENODEV


@pytest.mark.parametrize("L", [1, 7, 63, 64, 65, 127, 128, 129, 1000, 2048, 4100])
def test_pack_host_matches_numpy_packbits(L):
    """fid_pack_host: locus k -> bit k & 7 of byte k >> 3 (LSB first), rows
    padded with zero bits to 16-byte multiples; strided input rows."""
    import numpy as np
    import paper_1707_00516_amd as fid
    rng = np.random.default_rng(L)
    ld = L + 13
    b = (rng.random((23, ld)) < 0.4).astype(np.uint8)
    b[:, L:] = 7  # bytes past L are never read
    rw = fid.fid_row_words(L)
    out = np.full((23, rw), 0x5A5A5A5A5A5A5A5A, dtype=np.uint64)
    fid.fid_pack_host(b.ctypes.data, 23, L, ld, out.ctypes.data)
    want = np.packbits(b[:, :L], axis=1, bitorder="little")
    got = out.view(np.uint8)
    assert np.array_equal(got[:, :want.shape[1]], want)
    assert np.all(got[:, want.shape[1]:] == 0)


def test_pack_host_rejects_bad_input():
    import numpy as np
    import paper_1707_00516_amd as fid
    b = np.zeros((4, 100), np.uint8)
    b[2, 99] = 2
    out = np.zeros((4, fid.fid_row_words(100)), np.uint64)
    for args in ((b.ctypes.data, 4, 100, 100, out.ctypes.data),  # a byte of 2
                 (b.ctypes.data, 4, 0, 100, out.ctypes.data),    # no loci
                 (b.ctypes.data, 4, 100, 99, out.ctypes.data),   # rows overlap
                 (0, 4, 100, 100, out.ctypes.data),              # NULL input
                 (b.ctypes.data, -1, 100, 100, out.ctypes.data)):
        with pytest.raises(fid.FidError) as e:
            fid.fid_pack_host(*args)
        assert e.value.status == fid.FID_EINVAL
    fid.fid_pack_host(b.ctypes.data, 0, 100, 100, 0)  # no rows: a no-op
    fid.fid_pack_host(b.ctypes.data, 2, 100, 100, out.ctypes.data)  # rows 0-1 are fine
