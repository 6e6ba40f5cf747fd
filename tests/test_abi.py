"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_1909_02871_amd as gf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gfnc.h")

# Device pointers are never dereferenced by the argument checks; any nonzero
# value stands in for one.  Buffers of 1 MiB at distinct addresses:
P1, P2, P3, P4 = 0x10000000, 0x20000000, 0x30000000, 0x40000000


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gf_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared() == sorted(gf.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = gf.lib()
    for name in _declared():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", gf.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (gf_\w+)", out))
    assert set(_declared()) <= exported


def test_strerror():
    assert gf.strerror(0) == "success"
    assert "singular" in gf.strerror(gf.GF_ESINGULAR)
    assert gf.strerror(-99) == "unknown error"


def test_decode_workspace_sizes():
    L = gf.lib()
    assert L.gf_decode_workspace(8, 0, 1) == 0
    assert L.gf_decode_workspace(8, 257, 1) == 0
    assert L.gf_decode_workspace(3, 16, 1) == 0      # bad field
    assert L.gf_decode_workspace(8, 16, 0) == 0      # no systems
    for N in (1, 16, 100, 256):
        ws = L.gf_decode_workspace(8, N, 1)
        assert ws >= N * N + 4 and ws % 256 == 0
        for count in (2, 7, 2048):
            many = L.gf_decode_workspace(4, N, count)
            assert many >= count * (N * N + 4) and many % 256 == 0


@pytest.mark.parametrize("field", [0, 3, 5, 16, -1])
def test_bad_field(field):
    L = gf.lib()
    assert L.gf_region_madd(field, P1, P2, 1, 10, None) == gf.GF_EINVAL
    assert L.gf_region_mul(field, P1, P2, 1, 10, None) == gf.GF_EINVAL
    assert L.gf_encode(field, P1, 2, 2, P2, 10, P3, 10, 10, None) == gf.GF_EINVAL
    assert L.gf_decode(field, P1, P2, 10, 2, P3, 10, 10, P4, 1 << 16, None, None) == gf.GF_EINVAL


@pytest.mark.parametrize("field,c", [(1, 2), (2, 4), (4, 16), (8, 256), (8, -1)])
def test_coefficient_outside_field(field, c):
    assert gf.lib().gf_region_madd(field, P1, P2, c, 10, None) == gf.GF_EINVAL


def test_region_argument_checks():
    L = gf.lib()
    # zero length is a no-op even with null pointers
    assert L.gf_region_madd(8, None, None, 3, 0, None) == gf.GF_OK
    assert L.gf_region_madd(8, None, P2, 3, 10, None) == gf.GF_EINVAL
    # partial overlap is rejected
    assert L.gf_region_madd(8, P1 + 5, P1, 3, 10, None) == gf.GF_EINVAL
    assert L.gf_region_mul(8, P1, P1 + 9, 3, 10, None) == gf.GF_EINVAL


def test_encode_argument_checks():
    L = gf.lib()
    assert L.gf_encode(8, P1, 2, 0, P2, 10, P3, 10, 10, None) == gf.GF_EINVAL      # N = 0
    assert L.gf_encode(8, P1, -1, 2, P2, 10, P3, 10, 10, None) == gf.GF_EINVAL     # K < 0
    assert L.gf_encode(8, P1, 2, 257, P2, 10, P3, 10, 10, None) == gf.GF_ERANGE    # N > 256
    assert L.gf_encode(8, P1, 0, 2, P2, 10, P3, 10, 10, None) == gf.GF_OK          # K = 0: no-op
    assert L.gf_encode(8, P1, 2, 2, P2, 10, P3, 10, 0, None) == gf.GF_OK           # len = 0: no-op
    assert L.gf_encode(8, None, 2, 2, P2, 10, P3, 10, 10, None) == gf.GF_EINVAL
    assert L.gf_encode(8, P1, 2, 2, P2, 5, P3, 10, 10, None) == gf.GF_EINVAL       # ld_s < len
    assert L.gf_encode(8, P1, 2, 2, P2, 10, P2 + 5, 10, 10, None) == gf.GF_EINVAL  # Y overlaps S
    assert L.gf_encode(8, P1, 2, 2, P2, 10, P1, 10, 10, None) == gf.GF_EINVAL      # Y overlaps C


def test_decode_argument_checks():
    L = gf.lib()
    ws = L.gf_decode_workspace(8, 4, 1)
    assert L.gf_decode(8, P1, P2, 10, 0, P3, 10, 10, P4, ws, None, None) == gf.GF_EINVAL
    assert L.gf_decode(8, P1, P2, 10, 300, P3, 10, 10, P4, 1 << 20, None, None) == gf.GF_ERANGE
    assert L.gf_decode(8, P1, P2, 10, 4, P3, 10, 10, P4, ws - 1, None, None) == gf.GF_EINVAL  # small ws
    assert L.gf_decode(8, P1, P2, 10, 4, P2 + 3, 10, 10, P4, ws, None, None) == gf.GF_EINVAL  # S overlaps B
    assert L.gf_decode(8, P1, P2, 10, 4, P3, 10, 10, P3 + 8, ws, None, None) == gf.GF_EINVAL  # ws overlaps S
    # the allocation-free decode checks the same arguments (no workspace)
    assert L.gf_decode_noalloc(8, P1, P2, 10, 0, P3, 10, 10, None, None) == gf.GF_EINVAL
    assert L.gf_decode_noalloc(8, P1, P2, 10, 257, P3, 10, 10, None, None) == gf.GF_ERANGE
    assert L.gf_decode_noalloc(8, P1, P2, 10, 4, P2 + 3, 10, 10, None, None) == gf.GF_EINVAL  # S overlaps B
    assert L.gf_decode_noalloc(8, P1, P2, 10, 4, P1 + 2, 10, 10, None, None) == gf.GF_EINVAL  # S overlaps C
    assert L.gf_decode_noalloc(3, P1, P2, 10, 4, P3, 10, 10, None, None) == gf.GF_EINVAL
    assert L.gf_invert(8, P1, 4, P1 + 2, None, None) == gf.GF_EINVAL                          # Cinv overlaps C
    assert L.gf_invert(8, P1, 0, P2, None, None) == gf.GF_EINVAL


def test_plan_argument_checks():
    L = gf.lib()
    h = C.c_void_p()
    bad = (gf.gf_gen * 1)(gf.gf_gen(P1, P2, P3, 2, 0, 10, 10, 10))       # N = 0
    assert L.gf_plan_encode(8, bad, 1, None, C.byref(h)) == gf.GF_EINVAL and not h.value
    big = (gf.gf_gen * 1)(gf.gf_gen(P1, P2, P3, 2, 300, 10, 10, 10))     # N > 256
    assert L.gf_plan_encode(8, big, 1, None, C.byref(h)) == gf.GF_ERANGE
    tall = (gf.gf_gen * 1)(gf.gf_gen(P1, P2, P3, 65536, 2, 10, 10, 10))  # K > 65535 (tile row index is 16-bit)
    assert L.gf_plan_encode(8, tall, 1, None, C.byref(h)) == gf.GF_ERANGE
    assert L.gf_plan_encode(3, bad, 1, None, C.byref(h)) == gf.GF_EINVAL
    assert L.gf_plan_encode(8, bad, 1, None, None) == gf.GF_EINVAL
    sysbad = (gf.gf_sys * 1)(gf.gf_sys(P1, P2, P3, 4, 1, 10, 10, 10))    # reserved != 0
    assert L.gf_plan_decode(8, sysbad, 1, None, C.byref(h)) == gf.GF_EINVAL
    assert L.gf_encode_batched(8, P1, 1, None, None) == gf.GF_EINVAL      # no plan
    assert L.gf_plan_launch(None, None, None) == gf.GF_EINVAL
    assert L.gf_plan_launch_graph(None, None, None) == gf.GF_EINVAL
    assert L.gf_plan_errors(None, None) == gf.GF_EINVAL
    # mixed descriptors: some with pointers, some shapes only
    mixed = (gf.gf_gen * 2)(gf.gf_gen(P1, P2, P3, 2, 2, 10, 10, 10), gf.gf_gen(None, None, None, 2, 2, 10, 10, 10))
    assert L.gf_plan_encode(8, mixed, 2, None, C.byref(h)) == gf.GF_EINVAL and not h.value
    # a shape-only descriptor is still checked as a shape
    shp = (gf.gf_gen * 1)(gf.gf_gen(None, None, None, 2, 3, 10, 5, 10))  # ld_s < len
    assert L.gf_plan_encode(8, shp, 1, None, C.byref(h)) == gf.GF_EINVAL and not h.value
    L.gf_plan_destroy(None)


def test_decode_batched_argument_checks():
    """The descriptor-driven batched decode checks what the host can: field,
    count, pointers, the workspace's size and alignment, and overlaps of the
    workspace with the descriptor and rank arrays."""
    L = gf.lib()
    ws = L.gf_decode_workspace(8, 64, 10)
    assert ws > 10 * 64 * 64
    W = 0x5000_0000
    assert L.gf_decode_batched(8, P1, 0, None, None, 0, None) == gf.GF_OK        # nothing to do
    assert L.gf_decode_batched(3, P1, 10, None, W, ws, None) == gf.GF_EINVAL
    assert L.gf_decode_batched(8, P1, -1, None, W, ws, None) == gf.GF_EINVAL
    assert L.gf_decode_batched(8, None, 10, None, W, ws, None) == gf.GF_EINVAL
    assert L.gf_decode_batched(8, P1, 10, None, None, ws, None) == gf.GF_EINVAL
    assert L.gf_decode_batched(8, P1, 10, None, W + 16, ws, None) == gf.GF_EINVAL   # not 256-byte aligned
    assert L.gf_decode_batched(8, P1, 10, None, W, 1000, None) == gf.GF_EINVAL      # far too small
    assert L.gf_decode_batched(8, W + 512, 10, None, W, ws, None) == gf.GF_EINVAL   # descriptors inside ws
    assert L.gf_decode_batched(8, P1, 10, W + 512, W, ws, None) == gf.GF_EINVAL     # ranks inside ws


def test_recode_argument_checks():
    L = gf.lib()
    # R: P1 (Kout x M = 4 x 3), Cin: P2 (3 rows of N = 5, pitch 5), Bin: P3 (3 x 100), Cout/Yout in P4
    def rc(R=P1, K=4, M=3, N=5, Cin=P2, ldc=5, Bin=P3, ldb=100, Cout=P4, ldco=5, Yout=P4 + 4096, ldy=100,
           length=100):
        return L.gf_recode(8, R, K, M, N, Cin, ldc, Bin, ldb, Cout, ldco, Yout, ldy, length, None)
    assert rc(K=0) == gf.GF_OK                       # nothing to send
    assert rc(M=0) == gf.GF_EINVAL
    assert rc(N=0) == gf.GF_EINVAL
    assert rc(M=257) == gf.GF_ERANGE
    assert rc(N=257) == gf.GF_ERANGE
    assert rc(ldc=4) == gf.GF_EINVAL                 # coefficient rows narrower than N
    assert rc(ldco=4) == gf.GF_EINVAL
    assert rc(ldb=50) == gf.GF_EINVAL                # payload pitch below len
    assert rc(Cout=P2 + 1) == gf.GF_EINVAL           # Cout over Cin
    assert rc(Cout=P3 + 7) == gf.GF_EINVAL           # Cout over Bin
    assert rc(Yout=P2) == gf.GF_EINVAL               # Yout over Cin
    assert rc(Yout=P4 + 2) == gf.GF_EINVAL           # Yout over Cout
    assert rc(Yout=P1 + 1) == gf.GF_EINVAL           # Yout over R
    # packets as rows [coefficients | payload] (the accepted layout is run by the GPU tests): the
    # payload may not run into the next row's coefficients
    assert rc(Cin=P2, ldc=104, Bin=P2 + 5, ldb=104, Cout=P4, ldco=104, Yout=P4 + 5, ldy=104, length=100) == \
        gf.GF_EINVAL


def test_plan_recode_argument_checks():
    L = gf.lib()
    h = C.c_void_p()
    d = gf.gf_recode_desc(P1, P2, P3, P4, P4 + 4096, 4, 3, 5, 1, 100, 5, 100, 5, 100)   # reserved != 0
    assert L.gf_plan_recode(8, (gf.gf_recode_desc * 1)(d), 1, None, C.byref(h)) == gf.GF_EINVAL
    d.reserved, d.M = 0, 300
    assert L.gf_plan_recode(8, (gf.gf_recode_desc * 1)(d), 1, None, C.byref(h)) == gf.GF_ERANGE
    d.M, d.Kout = 3, 65536
    assert L.gf_plan_recode(8, (gf.gf_recode_desc * 1)(d), 1, None, C.byref(h)) == gf.GF_ERANGE
    d.Kout = 4
    d.M, d.Yout = 3, P2 + 1
    assert L.gf_plan_recode(8, (gf.gf_recode_desc * 1)(d), 1, None, C.byref(h)) == gf.GF_EINVAL
    assert L.gf_plan_recode(5, (gf.gf_recode_desc * 1)(d), 1, None, C.byref(h)) == gf.GF_EINVAL
    assert L.gf_plan_recode(8, None, 1, None, C.byref(h)) == gf.GF_EINVAL
    assert not h.value


def test_spans_that_do_not_fit_the_address_space_are_rejected():
    """A buffer's byte span, (rows - 1) * pitch + len, and its end address must
    fit in 64 bits; otherwise the overlap checks would see a wrapped size."""
    L = gf.lib()
    top = (1 << 64) - 8
    huge = 1 << 63
    assert L.gf_region_madd(8, top, P2, 3, 100, None) == gf.GF_EINVAL           # y runs past 2^64
    assert L.gf_region_mul(8, P1, top, 3, 100, None) == gf.GF_EINVAL            # x runs past 2^64
    assert L.gf_encode(8, P1, 3, 2, P2, 10, P3, huge, 10, None) == gf.GF_EINVAL  # 2 * 2^63 + 10 wraps
    assert L.gf_encode(8, P1, 2, 3, P2, huge, P3, 10, 10, None) == gf.GF_EINVAL
    assert L.gf_encode(8, (1 << 64) - 2, 2, 2, P2, 10, P3, 10, 10, None) == gf.GF_EINVAL   # C's 4 bytes run past 2^64
    ws = L.gf_decode_workspace(8, 4, 1)
    assert L.gf_decode(8, P1, P2, huge, 4, P3, 10, 10, P4, ws, None, None) == gf.GF_EINVAL
    assert L.gf_decode(8, P1, P2, 10, 4, P3, huge, 10, P4, ws, None, None) == gf.GF_EINVAL
    assert L.gf_decode(8, P1, P2, 10, 4, P3, 10, 10, top, ws, None, None) == gf.GF_EINVAL
    assert L.gf_invert(8, top, 4, P2, None, None) == gf.GF_EINVAL
    assert L.gf_recode(8, P1, 3, 3, 5, P2, 5, P3, 100, P4, 5, P4 + 4096, huge, 100, None) == gf.GF_EINVAL
    h = C.c_void_p()
    sysd = (gf.gf_sys * 1)(gf.gf_sys(P1, P2, P3, 4, 0, 10, huge, 10))
    assert L.gf_plan_decode(8, sysd, 1, None, C.byref(h)) == gf.GF_EINVAL and not h.value
    gens = (gf.gf_gen * 1)(gf.gf_gen(P1, P2, P3, 3, 2, 10, 10, huge))
    assert L.gf_plan_encode(8, gens, 1, None, C.byref(h)) == gf.GF_EINVAL and not h.value


def test_spans_that_fit_still_pass_validation():
    """The same calls with pitches that fit get past every argument check (and
    then report the missing device: GF_EDEVICE without a GPU)."""
    if gf.lib().gf_init() != gf.GF_EDEVICE:
        pytest.skip("a device is present: valid calls would launch")
    L = gf.lib()
    assert L.gf_region_madd(8, P1, P2, 3, 100, None) == gf.GF_EDEVICE
    assert L.gf_encode(8, P1, 3, 2, P2, 10, P3, 1 << 20, 10, None) == gf.GF_EDEVICE
    assert L.gf_encode(8, P1, 1, 2, P2, 10, P3, 1 << 63, 10, None) == gf.GF_EDEVICE   # one row: pitch unused
    ws = L.gf_decode_workspace(8, 4, 1)
    assert L.gf_decode(8, P1, P2, 10, 4, P3, 10, 10, P4, ws, None, None) == gf.GF_EDEVICE
    assert L.gf_decode_noalloc(8, P1, P2, 10, 4, P3, 10, 10, None, None) == gf.GF_EDEVICE
    assert L.gf_invert(8, P1, 4, P2, None, None) == gf.GF_EDEVICE
    assert L.gf_decode_batched(8, P1, 10, None, 0x5000_0000, L.gf_decode_workspace(8, 64, 10),
                               None) == gf.GF_EDEVICE
