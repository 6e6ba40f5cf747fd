"""The product path has no CPU fallback: without a GPU every compute call of the
binding raises before doing any work, and the library reports the missing
device rather than computing on the host."""
import numpy as np
import pytest
import torch

import paper_1909_02871_amd as gf

pytestmark = pytest.mark.skipif(torch.cuda.is_available(), reason="checks the behaviour without a GPU")


def test_binding_calls_raise_without_a_gpu():
    x = torch.zeros(16, dtype=torch.uint8)
    C = torch.zeros((2, 2), dtype=torch.uint8)
    S = torch.zeros((2, 16), dtype=torch.uint8)
    calls = [
        lambda: gf.gf_init(),
        lambda: gf.gf_region_madd(8, x, x.clone(), 3),
        lambda: gf.gf_region_mul(8, x, x.clone(), 3),
        lambda: gf.gf_encode(8, C, S, S.clone()),
        lambda: gf.gf_decode(8, C, S, S.clone()),
        lambda: gf.gf_invert(8, C, C.clone()),
        lambda: gf.gf_plan_encode(8, [(C, S, S.clone())]),
        lambda: gf.gf_recode(8, C, C, S, C.clone(), S.clone()),
        lambda: gf.Server(field=8),
    ]
    for call in calls:
        with pytest.raises((RuntimeError, TypeError)):
            call()


def test_library_reports_the_missing_device():
    L = gf.lib()
    assert L.gf_init() == gf.GF_EDEVICE
    buf = np.zeros(64, dtype=np.uint8)
    # a valid call on host memory is never computed on the host: it fails at device set-up
    p = buf.ctypes.data
    assert L.gf_region_madd(8, p, p + 32, 3, 16, None) == gf.GF_EDEVICE
    assert np.all(buf == 0)
