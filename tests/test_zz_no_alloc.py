"""GPU check of the allocation-free non-finite count (``sbim_count_nonfinite_noalloc``).

Through the C ABI, its count must equal the allocating entry point's
(``sbim_count_nonfinite``) exactly, on two calls in a row that share the static
scratch, the second with a smaller field (another handle on the same GPU), and
on finite fields.  Integer results: the bar is equality."""
import ctypes

import pytest
import torch

from paper_2102_08756_amd import SBIM, Config
from paper_2102_08756_amd.sbim import SBIM_E_INVALID

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _handle(n1, n3, planes, precision):
    pl = [dict(side=1, mu=1.0, cs=1.0, cp=3.0 ** 0.5), dict(side=-1, mu=1.0, cs=1.0, cp=3.0 ** 0.5)]
    cfg = dict(n1=n1, n3=n3, dx1=1.0, dx3=1.0, dt=0.2, planes=pl[:planes], window_cap=4,
               window_mode="fixed", eta_w=1.0, input_kind="increment")
    return SBIM(Config.from_dict(cfg, precision=precision), device=DEV)


def _planted(sb, positions, seed):
    g = torch.Generator(device=DEV).manual_seed(seed)
    u = torch.randn(sb.shape, generator=g, dtype=sb.dtype, device=DEV)
    flat = u.view(-1)
    vals = (float("nan"), float("inf"), float("-inf"))
    for k, i in enumerate(positions):
        flat[i % flat.numel()] = vals[k % 3]
    return u


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_count_equals_the_allocating_count(precision):
    big = _handle(256, 128, 2, precision)
    small = _handle(16, 8, 1, precision)
    out = torch.full((1,), -1, dtype=torch.int64, device=DEV)
    # first call: a large field with nine planted values spread over work-groups
    u1 = _planted(big, [0, 1, 5000, 77777, 123456, 160000, 196607, 3, 65536], 1)
    big.count_nonfinite_noalloc(u1, out)
    got1 = int(out.item())
    assert got1 == big.count_nonfinite(u1) == 9
    # second call in a row, a smaller field: every partial of the first is overwritten
    u2 = _planted(small, [2, 100], 2)
    small.count_nonfinite_noalloc(u2, out)
    got2 = int(out.item())
    assert got2 == small.count_nonfinite(u2) == 2
    # finite fields count zero on both handles
    z1 = torch.randn(big.shape, dtype=big.dtype, device=DEV)
    z2 = torch.randn(small.shape, dtype=small.dtype, device=DEV)
    big.count_nonfinite_noalloc(z1, out)
    assert int(out.item()) == big.count_nonfinite(z1) == 0
    small.count_nonfinite_noalloc(z2, out)
    assert int(out.item()) == small.count_nonfinite(z2) == 0
    big.close()
    small.close()


def test_noalloc_count_rejects_null_output():
    sb = _handle(16, 16, 1, "fp64")
    u = torch.randn(sb.shape, dtype=sb.dtype, device=DEV)
    rc = sb._L.sbim_count_nonfinite_noalloc(sb._h, ctypes.c_void_p(u.data_ptr()), None)
    assert rc == SBIM_E_INVALID
    with pytest.raises(ValueError):
        sb.count_nonfinite_noalloc(u, torch.zeros(1, dtype=torch.int32, device=DEV))
    sb.close()
