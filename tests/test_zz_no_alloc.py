"""bte_state_observables_noalloc (scratch in a static device array of the
library) against bte_state_observables with a caller workspace: two calls in
a row on one GPU, the second on a smaller state, so the second reads a
scratch array the first left filled; plus the size limit."""
import math

import numpy as np
import pytest

import oracle
from paper_1401_6047_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bte():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1401_6047_amd import bte as _bte
    return _bte


def device_state(torch, nx, ny, pad, seed):
    a, b = W.random_coeffs(seed, nx, ny, decay=0.05)
    b[0] = 0.0
    ta = torch.zeros((nx, ny + pad), dtype=torch.float64, device="cuda")
    tb = torch.zeros_like(ta)
    ta[:, :ny] = torch.from_numpy(a)
    tb[:, :ny] = torch.from_numpy(b)
    return a, b, ta, tb


def with_workspace(bte, torch, ta, tb, nx, ny, lo, hi, alpha, stream):
    need = bte.bte_state_observables_bytes(nx)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    wp = (ws.data_ptr() + 255) // 256 * 256
    out = torch.empty(4, dtype=torch.float64, device="cuda")
    bte.bte_state_observables(ta.data_ptr(), tb.data_ptr(), nx, ny, ta.stride(0), lo, hi, alpha,
                              wp, need, stream, out.data_ptr())
    return out


@pytest.mark.parametrize("shapes", [((512, 8193, 7), (40, 333, 0)),
                                    ((16384, 5, 3), (3, 4, 1))])
def test_noalloc_matches_workspace_entry(bte, shapes):
    import torch
    lo, hi, alpha = -7.5, 7.5, 0.9496
    stream = torch.cuda.current_stream().cuda_stream
    for i, (nx, ny, pad) in enumerate(shapes):
        a, b, ta, tb = device_state(torch, nx, ny, pad, 11 * nx + ny + i)
        ref = with_workspace(bte, torch, ta, tb, nx, ny, lo, hi, alpha, stream)
        got = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
        print(f"noalloc call {i}: nx={nx} ny={ny} ld={ny + pad}", flush=True)
        bte.bte_state_observables_noalloc(ta.data_ptr(), tb.data_ptr(), nx, ny, ta.stride(0),
                                          lo, hi, alpha, stream, got.data_ptr())
        g = got.cpu().numpy()
        r = ref.cpu().numpy()
        # the same kernels on the same values in the same order: the same bits
        assert (g == r).all(), (g, r)
        # and the Sec. 2 definitions as the oracle writes them
        pb = oracle.Problem(nx=nx, ny=ny, phiy_min=lo, phiy_max=hi, E_dc=0, E_w=0, omega=1,
                            B=0, mu=1, dt=1e-3, alpha=alpha)
        f = math.pi * math.sqrt(alpha) * (hi - lo) / (ny - 1)
        edge, top = oracle.resolution_diagnostics(pb, a, b)
        want = [2 * f * a[0].sum(), f * b[1].sum(), edge, top]
        scale = [2 * f * np.abs(a[0]).sum(), f * np.abs(b[1]).sum(), edge, top]
        for x, w_, sc in zip(g, want, scale):
            assert abs(x - w_) <= 1e-12 * sc


def test_noalloc_rejects_sizes_beyond_its_array(bte):
    import torch
    assert bte.STATE_OBS_NOALLOC_MAX_NX == 16384
    nx = bte.STATE_OBS_NOALLOC_MAX_NX + 1
    a = torch.zeros((nx, 3), dtype=torch.float64, device="cuda")
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(bte.BteError) as ei:
        bte.bte_state_observables_noalloc(a.data_ptr(), a.data_ptr(), nx, 3, 3, -1.0, 1.0, 1.0,
                                          0, out.data_ptr())
    assert ei.value.status == bte.BTE_EINVAL
    with pytest.raises(bte.BteError) as ei:
        bte.bte_state_observables_noalloc(a.data_ptr(), a.data_ptr(), 4, 2, 3, -1.0, 1.0, 1.0,
                                          0, out.data_ptr())
    assert ei.value.status == bte.BTE_EINVAL
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 0).all()
