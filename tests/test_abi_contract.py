"""Randomised check of the C ABI's argument validation against the contract the
header states, without a GPU: for thousands of random calls (overlapping and
touching buffers, short pitches, addresses near 2^64, empty sizes) the library
must accept exactly the calls the contract allows.  An accepted call gets as
far as device set-up and returns GF_EDEVICE here; nothing is launched."""
import numpy as np
import pytest
import torch

import paper_1909_02871_amd as gf

pytestmark = pytest.mark.skipif(torch.cuda.is_available(), reason="accepted calls would launch on a GPU")

TOP = 1 << 64
M64 = TOP - 1


def span(p, rows, ld, length):
    """(start, size) of rows x length bytes `ld` apart, or None when it does not fit in 64 bits."""
    if rows == 0 or length == 0:
        n = 0
    else:
        n = (rows - 1) * ld + length
    if n > M64 or p + n > M64:
        return None
    return (p, n)


def overlap(a, b):
    return a[1] > 0 and b[1] > 0 and a[0] < b[0] + b[1] and b[0] < a[0] + a[1]


def encode_contract(field, C, K, N, S, ld_s, Y, ld_y, length):
    if field not in (1, 2, 4, 8) or K < 0 or N < 1:
        return gf.GF_EINVAL
    if N > 256:
        return gf.GF_ERANGE
    if K == 0 or length == 0:
        return gf.GF_OK
    if not C or not S or not Y:
        return gf.GF_EINVAL
    if (N > 1 and ld_s < length) or (K > 1 and ld_y < length):
        return gf.GF_EINVAL
    ys, ss, cs = span(Y, K, ld_y, length), span(S, N, ld_s, length), span(C, K, N, N)
    if ys is None or ss is None or cs is None or overlap(ys, ss) or overlap(ys, cs):
        return gf.GF_EINVAL
    return gf.GF_EDEVICE


def region_contract(field, y, x, c, length):
    if field not in (1, 2, 4, 8) or c < 0 or c >= (1 << field):
        return gf.GF_EINVAL
    if length == 0:
        return gf.GF_OK
    if not y or not x:
        return gf.GF_EINVAL
    ys, xs = span(y, 1, 0, length), span(x, 1, 0, length)
    if ys is None or xs is None or (y != x and overlap(ys, xs)):
        return gf.GF_EINVAL
    return gf.GF_EDEVICE     # c = 0 madd also returns after device set-up


def _ptr(rng, base):
    k = rng.integers(0, 10)
    if k == 0:
        return 0
    if k == 1:
        return TOP - int(rng.integers(1, 5000))
    return base + int(rng.integers(0, 3000))


def _size(rng, small=64):
    k = rng.integers(0, 8)
    if k == 0:
        return 0
    if k == 1:
        return 1 << int(rng.integers(40, 64))
    return int(rng.integers(1, small))


def test_encode_accepts_exactly_the_contract():
    L = gf.lib()
    rng = np.random.default_rng(190902871)
    base = 0x4000_0000
    for _ in range(20000):
        field = int(rng.choice([8, 8, 8, 4, 1, 3]))
        K = int(rng.integers(-1, 6)) if rng.integers(0, 5) else int(rng.integers(250, 300))
        N = int(rng.integers(0, 6)) if rng.integers(0, 5) else int(rng.integers(250, 300))
        C, S, Y = _ptr(rng, base), _ptr(rng, base), _ptr(rng, base)
        length, ld_s, ld_y = _size(rng), _size(rng), _size(rng)
        want = encode_contract(field, C, K, N, S, ld_s, Y, ld_y, length)
        got = L.gf_encode(field, C or None, K, N, S or None, ld_s, Y or None, ld_y, length, None)
        assert got == want, (field, hex(C), K, N, hex(S), ld_s, hex(Y), ld_y, length)


def test_region_accepts_exactly_the_contract():
    L = gf.lib()
    rng = np.random.default_rng(2)
    base = 0x4000_0000
    for _ in range(20000):
        field = int(rng.choice([1, 2, 4, 8, 0]))
        c = int(rng.integers(-1, 300))
        y, x = _ptr(rng, base), _ptr(rng, base)
        length = _size(rng, 4000)
        want = region_contract(field, y, x, c, length)
        got = L.gf_region_madd(field, y or None, x or None, c, length, None)
        assert got == want, (field, hex(y), hex(x), c, length)


def decode_contract(L, field, C, N, B, ld_b, S, ld_s, length, ws, ws_bytes):
    if field not in (1, 2, 4, 8) or N < 1:
        return gf.GF_EINVAL
    if N > 256:
        return gf.GF_ERANGE
    if not C or not ws or ws_bytes < L.gf_decode_workspace(8, N, 1):
        return gf.GF_EINVAL
    if length > 0 and (not B or not S or (N > 1 and (ld_b < length or ld_s < length))):
        return gf.GF_EINVAL
    ss, bs, cs, ws_ = span(S, N, ld_s, length), span(B, N, ld_b, length), span(C, N, N, N), span(ws, 1, 0, ws_bytes)
    if ss is None or bs is None or cs is None or ws_ is None:
        return gf.GF_EINVAL
    if overlap(ss, bs) or overlap(ss, cs) or overlap(ss, ws_) or overlap(ws_, cs) or overlap(ws_, bs):
        return gf.GF_EINVAL
    return gf.GF_EDEVICE


def test_decode_accepts_exactly_the_contract():
    L = gf.lib()
    rng = np.random.default_rng(3)
    base = 0x4000_0000
    for _ in range(20000):
        field = int(rng.choice([8, 8, 2, 5]))
        N = int(rng.integers(0, 6)) if rng.integers(0, 5) else int(rng.integers(250, 300))
        C, B, S, ws = (_ptr(rng, base) for _ in range(4))
        length, ld_b, ld_s = _size(rng), _size(rng), _size(rng)
        need = int(L.gf_decode_workspace(8, max(1, min(N, 256)), 1))
        ws_bytes = int(rng.choice([0, need - 1, need, need + 100])) if need else 0
        ws_bytes = max(ws_bytes, 0)
        want = decode_contract(L, field, C, N, B, ld_b, S, ld_s, length, ws, ws_bytes)
        got = L.gf_decode(field, C or None, B or None, ld_b, N, S or None, ld_s, length, ws or None, ws_bytes, None, None)
        assert got == want, (field, hex(C), N, hex(B), ld_b, hex(S), ld_s, length, hex(ws), ws_bytes)


def _rows_bytes(p, rows, ld, width):
    return [(p + r * ld, width) for r in range(rows)] if width > 0 else []


def _any_overlap(xs, ys):
    return any(overlap(a, b) for a in xs for b in ys)


def test_accepted_recodings_never_overlap_their_outputs():
    """Recoding's checks are stricter than the per-byte rule (they compare row
    spans), so every accepted call must have outputs disjoint from each other
    and from every input, all below 2^64; and the two usual layouts (separate
    buffers; packets as rows [coefficients | payload]) must be accepted."""
    L = gf.lib()
    rng = np.random.default_rng(4)
    base = 0x4000_0000
    accepted = 0
    for _ in range(20000):
        Kout, M, N = int(rng.integers(0, 5)), int(rng.integers(1, 5)), int(rng.integers(1, 9))
        length = int(rng.integers(0, 40))
        R, Cin, Bin, Cout, Yout = (base + int(rng.integers(0, 600)) for _ in range(5))
        if rng.integers(0, 20) == 0:
            Yout = TOP - int(rng.integers(1, 300))
        ld_cin, ld_b, ld_cout, ld_y = (int(rng.integers(0, 60)) for _ in range(4))
        if rng.integers(0, 3) == 0:          # the packet-row layout, sometimes with a broken pitch
            ld = N + length + int(rng.integers(0, 8))
            Bin, Yout, ld_cin, ld_b, ld_cout, ld_y = Cin + N, Cout + N, ld, ld, ld, ld + int(rng.integers(0, 2))
        got = L.gf_recode(8, R, Kout, M, N, Cin, ld_cin, Bin, ld_b, Cout, ld_cout, Yout, ld_y, length, None)
        if got != gf.GF_EDEVICE or Kout == 0:
            continue
        accepted += 1
        outs = [_rows_bytes(Cout, Kout, ld_cout, N), _rows_bytes(Yout, Kout, ld_y, length)]
        ins = [_rows_bytes(R, Kout, M, M), _rows_bytes(Cin, M, ld_cin, N), _rows_bytes(Bin, M, ld_b, length)]
        for o in outs:
            assert all(a + n <= M64 for a, n in o)
            for i in ins:
                assert not _any_overlap(o, i), (Kout, M, N, length, R, Cin, Bin, Cout, Yout)
        assert not _any_overlap(outs[0], outs[1])
    assert accepted > 500
    # the usual layouts are accepted
    assert L.gf_recode(8, base, 3, 4, 6, base + 0x1000, 6, base + 0x2000, 100, base + 0x3000, 6,
                       base + 0x4000, 100, 100, None) == gf.GF_EDEVICE
    ld = 6 + 100 + 10
    assert L.gf_recode(8, base, 3, 4, 6, base + 0x1000, ld, base + 0x1006, ld, base + 0x3000, ld,
                       base + 0x3006, ld, 100, None) == gf.GF_EDEVICE
