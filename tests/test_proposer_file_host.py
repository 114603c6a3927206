"""Host-side checks of the network file (ltgw_proposer_save / _load) with no
context, so no device call is made: the documented layout, a bit-exact round
trip, and every refusal (missing, foreign, short, corrupt, other version,
wrong buffer size)."""
import struct

import numpy as np
import pytest


def _lib():
    from paper_2507_07816_amd import ltgw

    return ltgw


def _params(c_in, c_out, seed=3):
    ltgw = _lib()
    n = ltgw.ltgw_cnn_param_count(c_in, c_out)
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n).astype(np.float32)


def _fnv1a64(b):
    h = 0xCBF29CE484222325
    for x in b:
        h = ((h ^ x) * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def test_round_trip_and_layout(tmp_path):
    ltgw = _lib()
    p = _params(8, 24)
    path = tmp_path / "net.bin"
    ltgw.ltgw_proposer_save(None, str(path), p, 8, 24)
    raw = path.read_bytes()
    assert len(raw) == 64 + 4 * p.size
    magic, ver, ci, co, width, taps, z0, n, h = struct.unpack("<8sIiiiiiqQ", raw[:48])
    assert (magic, ver, ci, co, width, taps, z0, n) == (b"LTGWCNN\0", 1, 8, 24, 32, 5, 0, p.size)
    assert raw[48:64] == bytes(16)
    assert h == _fnv1a64(raw[64:])
    assert np.array_equal(np.frombuffer(raw[64:], "<f4"), p)
    assert ltgw.ltgw_proposer_load(None, str(path)) == (8, 24)
    q = np.zeros_like(p)
    assert ltgw.ltgw_proposer_load(None, str(path), q) == (8, 24)
    assert np.array_equal(q.view(np.uint32), p.view(np.uint32))
    assert not (tmp_path / "net.bin.tmp").exists()


def _code(fn):
    ltgw = _lib()
    with pytest.raises(ltgw.LtgwError) as e:
        fn()
    return e.value.code, str(e.value)


def test_refusals(tmp_path):
    ltgw = _lib()
    p = _params(4, 24)
    good = tmp_path / "good.bin"
    ltgw.ltgw_proposer_save(None, str(good), p, 4, 24)
    raw = good.read_bytes()
    q = np.zeros_like(p)
    code, msg = _code(lambda: ltgw.ltgw_proposer_load(None, str(tmp_path / "missing.bin"), q))
    assert code == ltgw.LTGW_E_IO and "cannot open" in msg
    bad = tmp_path / "bad.bin"
    bad.write_bytes(raw[:40])
    assert _code(lambda: ltgw.ltgw_proposer_load(None, str(bad), q))[0] == ltgw.LTGW_E_IO
    bad.write_bytes(b"NOTANET\0" + raw[8:])
    assert _code(lambda: ltgw.ltgw_proposer_load(None, str(bad), q))[0] == ltgw.LTGW_E_IO
    bad.write_bytes(raw[:8] + struct.pack("<I", 2) + raw[12:])
    assert _code(lambda: ltgw.ltgw_proposer_load(None, str(bad), q))[0] == ltgw.LTGW_E_UNSUPPORTED
    bad.write_bytes(raw[:-4])
    code, msg = _code(lambda: ltgw.ltgw_proposer_load(None, str(bad), q))
    assert code == ltgw.LTGW_E_IO and "truncated" in msg
    bad.write_bytes(raw + b"\0")
    assert _code(lambda: ltgw.ltgw_proposer_load(None, str(bad), q))[0] == ltgw.LTGW_E_IO
    flipped = bytearray(raw)
    flipped[64 + 123] ^= 0x10
    bad.write_bytes(bytes(flipped))
    code, msg = _code(lambda: ltgw.ltgw_proposer_load(None, str(bad), q))
    assert code == ltgw.LTGW_E_IO and "checksum" in msg
    bad.write_bytes(raw[:12] + struct.pack("<i", 5) + raw[16:])  # c_in no longer matches the count
    assert _code(lambda: ltgw.ltgw_proposer_load(None, str(bad), q))[0] == ltgw.LTGW_E_IO
    small = np.zeros(p.size - 1, np.float32)
    assert _code(lambda: ltgw.ltgw_proposer_load(None, str(good), small))[0] == ltgw.LTGW_E_INVALID_ARG
    # nothing is written into the buffer by a refused load
    assert not q.any()
    assert _code(lambda: ltgw.ltgw_proposer_save(None, str(tmp_path / "x.bin"), p, 0, 24))[0] == \
        ltgw.LTGW_E_INVALID_ARG
    assert _code(lambda: ltgw.ltgw_proposer_save(None, str(tmp_path / "no" / "dir.bin"), p, 4, 24))[0] == \
        ltgw.LTGW_E_IO
