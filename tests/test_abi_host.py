"""Host-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and validates arguments (no GPU needed for any of this)."""
import math
import subprocess

import pytest

from paper_1401_6047_amd import bte


def test_library_exports_every_header_symbol():
    names = bte.header_functions()
    assert {"bte_create", "bte_step", "bte_observables"} <= set(names)
    for n in names:
        assert hasattr(bte.lib(), n), n
    out = subprocess.run(["nm", "-D", "--defined-only", bte.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_version_and_last_error():
    assert "gfx950" in bte.bte_version()
    assert isinstance(bte.bte_last_error(), str)


def _grid(**kw):
    d = dict(n_x=128, n_y=1001, phiy_min=-10.0, phiy_max=10.0)
    d.update(kw)
    return bte.make_grid(**d)


def _params(**kw):
    d = dict(E_dc=6.0, E_w=0.1, omega=2.0, B=4.0, mu=1.0, dt=1e-4)
    d.update(kw)
    return bte.make_params(**d)


def test_workspace_bytes_scales_with_grid_and_precision():
    b64 = bte.bte_workspace_bytes(_grid(), _params())
    b32 = bte.bte_workspace_bytes(_grid(), _params(precision=bte.BTE_FP32_BULK))
    # 8 planes of (n_x + 4) x ld elements dominate
    assert b64 > 8 * 132 * 1001 * 8
    assert b32 < b64 and b32 > 8 * 132 * 1001 * 4
    big = bte.bte_workspace_bytes(_grid(n_x=512, n_y=8193, phiy_min=-20, phiy_max=20),
                                  _params(dt=2e-5, B=6.0))
    assert big > 8 * 516 * 8193 * 8


@pytest.mark.parametrize("grid_kw,param_kw,needle", [
    (dict(n_x=1), {}, "n_x"),
    (dict(n_y=2), {}, "n_y"),
    (dict(phiy_min=1.0, phiy_max=1.0), {}, "phiy"),
    (dict(phiy_max=math.inf), {}, "phiy"),
    ({}, dict(dt=0.0), "dt"),
    ({}, dict(mu=-1.0), "mu"),
    ({}, dict(alpha=0.0), "alpha"),
    ({}, dict(tau=2.0), "tau"),
    ({}, dict(omega=0.0), "omega"),
    ({}, dict(E_dc=math.nan), "finite"),
    ({}, dict(precision=7), "precision"),
    ({}, dict(B=4.0, dt=0.02), "leap-frog"),
])
def test_invalid_arguments_rejected(grid_kw, param_kw, needle):
    with pytest.raises(bte.BteError) as ei:
        bte.bte_workspace_bytes(_grid(**grid_kw), _params(**param_kw))
    assert ei.value.status == bte.BTE_EINVAL
    assert needle in str(ei.value)


def test_state_set_must_stay_below_2_gib():
    """The step kernels address a set of four state planes with 32-bit byte
    offsets: a grid whose four FP64 planes reach 2 GiB is rejected (one
    plane alone is still far below it), the same grid in FP32 bulk and a
    slightly smaller FP64 grid are accepted; the batch applies the same rule."""
    big = _grid(n_x=1024, n_y=72700)
    with pytest.raises(bte.BteError) as ei:
        bte.bte_workspace_bytes(big, _params(B=0.0))
    assert ei.value.status == bte.BTE_EINVAL and "four state planes" in str(ei.value)
    assert bte.bte_workspace_bytes(big, _params(B=0.0, precision=bte.BTE_FP32_BULK)) > 0
    assert bte.bte_workspace_bytes(_grid(n_x=1024, n_y=60000), _params(B=0.0)) > 0
    with pytest.raises(bte.BteError) as ei:
        bte.bte_batch_workspace_bytes(_cfg(n_x=1024, phiy_min=-10.0, phiy_max=10.0, dt=1e-4),
                                      [_W(ny=72700, B=0.0)])
    assert ei.value.status == bte.BTE_EINVAL and "four state planes" in str(ei.value)


def test_omega_zero_allowed_without_ac_field():
    assert bte.bte_workspace_bytes(_grid(), _params(E_w=0.0, omega=0.0)) > 0


def test_flags_must_be_zero():
    p = _params()
    p.flags = 1
    with pytest.raises(bte.BteError):
        bte.bte_workspace_bytes(_grid(), p)


def _cfg(**kw):
    d = dict(n_x=16, phiy_min=-6.0, phiy_max=6.0, dt=2e-3)
    d.update(kw)
    return bte.make_batch_config(**d)


class _W:
    def __init__(self, **kw):
        self.__dict__.update(dict(E_dc=1.0, E_w=0.1, omega=2.0, B=1.0, mu=1.0, ny=41))
        self.__dict__.update(kw)


def test_batch_workspace_bytes_and_validation():
    n1 = bte.bte_batch_workspace_bytes(_cfg(), [_W(), _W(ny=41)])
    n2 = bte.bte_batch_workspace_bytes(_cfg(), [_W(), _W(ny=401)])
    assert n2 > n1 > 0
    for cfg, inst, needle in [
        (_cfg(min_periods=1), [_W()], "min_periods"),
        (_cfg(tol=0.0), [_W()], "tol"),
        (_cfg(), [_W(omega=0.0)], "omega"),
        (_cfg(), [_W(ny=2)], "n_y"),
        (_cfg(), [_W(B=1e4)], "leap-frog"),
        (_cfg(precision=3), [_W()], "precision"),
    ]:
        with pytest.raises(bte.BteError) as ei:
            bte.bte_batch_workspace_bytes(cfg, inst)
        assert ei.value.status == bte.BTE_EINVAL and needle in str(ei.value)
    bad = bte.bte_batch_tuning(bte.BTE_KERNEL_TWO_PASS, 8, 8, 0)   # not a batch kernel form
    with pytest.raises(bte.BteError):
        bte.bte_batch_workspace_bytes(_cfg(), [_W()], bad)
    bad = bte.bte_batch_tuning(bte.BTE_KERNEL_FUSED2, 8, 8, 0, 2)    # unknown schedule
    with pytest.raises(bte.BteError) as ei:
        bte.bte_batch_workspace_bytes(_cfg(), [_W()], bad)
    assert ei.value.status == bte.BTE_EINVAL and "schedule" in str(ei.value)
    # the wide schedule holds one state slot per instance, the persistent one
    # per workgroup
    inst = [_W(ny=401)] * 4
    t = bte.bte_batch_tuning(bte.BTE_KERNEL_FUSED2, 25, 8, 16, bte.BTE_BATCH_PERSISTENT)
    w = bte.bte_batch_tuning(bte.BTE_KERNEL_FUSED2, 25, 8, 16, bte.BTE_BATCH_WIDE)
    assert bte.bte_batch_workspace_bytes(_cfg(), inst, w) < bte.bte_batch_workspace_bytes(_cfg(), inst, t)


def test_tuning_cache_key_classes():
    """The binding's JSON tuning cache keys a pick the way the library's own
    cache does: N_x, precision, the batch-size class (the smallest power of
    two at or above min(n, 4096)) and the set of N_y values."""
    cfg = _cfg()
    k12 = bte.tuning_cache_key(cfg, [_W(ny=41)] * 11 + [_W(ny=81)])
    assert k12 == f"nx16-p{cfg.precision}-n16-ny41,81"
    assert bte.tuning_cache_key(cfg, [_W()] * 16).split("-")[2] == "n16"
    assert bte.tuning_cache_key(cfg, [_W()] * 17).split("-")[2] == "n32"
    assert bte.tuning_cache_key(cfg, [_W()] * 300).split("-")[2] == "n512"
    assert bte.tuning_cache_key(cfg, [_W()] * 5000).split("-")[2] == "n4096"
    assert bte.tuning_cache_key(cfg, [_W()]).split("-")[2] == "n1"


def test_batch_tune_host_validation():
    """The sweep autotuner validates the batch before any device work."""
    for cfg, inst in [(_cfg(min_periods=1), [_W()]), (_cfg(), [_W(omega=0.0)]),
                      (_cfg(), [_W(B=1e4)])]:
        with pytest.raises(bte.BteError) as ei:
            bte.bte_batch_tune(cfg, inst)
        assert ei.value.status == bte.BTE_EINVAL
    with pytest.raises(bte.BteError) as ei:
        bte.bte_batch_tune(_cfg(), [])
    assert ei.value.status == bte.BTE_EINVAL
    assert bte.tuning_cache_key(_cfg(), [_W(ny=41), _W(ny=11), _W(ny=41)]).endswith("ny11,41")


def test_mlp_library_exports_and_host_validation():
    from paper_1401_6047_amd import mlp
    names = bte.header_functions(mlp.HEADER_PATH)
    assert "bte_mlp_train_step" in names and "bte_mlp_forward" in names
    out = subprocess.run(["nm", "-D", "--defined-only", bte.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert not [n for n in names if n not in exported]
    assert mlp.bte_mlp_param_count() == 2172672
    b16 = mlp.bte_mlp_workspace_bytes(512, mlp.BTE_MLP_BF16)
    b32 = mlp.bte_mlp_workspace_bytes(512, mlp.BTE_MLP_FP32)
    # FP32 master parameters, gradient and two moments at least
    assert b32 > b16 > 4 * 4 * 2172672
    assert mlp.bte_mlp_workspace_bytes(513, 0) > b16
    assert mlp.bte_mlp_workspace_bytes(0, 0) == 0
    assert mlp.bte_mlp_workspace_bytes(64, 7) == 0
    with pytest.raises(bte.BteError, match="workspace"):
        mlp.bte_mlp_create(64, 0, 0, 1 << 30, 0)
    with pytest.raises(bte.BteError, match="max_batch"):
        mlp.bte_mlp_create(0, 0, 256, 1 << 30, 0)
    with pytest.raises(bte.BteError, match="handle"):
        mlp.bte_mlp_forward(0, None, 4, None)


def test_reconstruct_host_validation():
    """Argument checks of the reconstruction entry points run before any
    device work (NULL pointers, sizes, alignment)."""
    from paper_1401_6047_amd import bte
    with pytest.raises(bte.BteError) as ei:
        bte.bte_reconstruct(0, 16, 4096)
    assert ei.value.status == bte.BTE_EINVAL
    for args, needle in (((0, 8, 4, 8, 8, 3, 8, 0), "NULL"),
                         ((8, 8, 4, 8, 8, 3, 0, 0), "NULL"),
                         ((8, 12, 4, 8, 8, 3, 8, 0), "aligned"),
                         ((8, 8, 4, 8, 7, 3, 8, 0), "ld >= n_y"),
                         ((8, 8, 0, 8, 8, 3, 8, 0), "n_x >= 1"),
                         ((8, 8, 4, 8, 8, 0, 8, 0), "n_phix"),
                         ((8, 8, 4, 8, 8, (1 << 20) + 1, 8, 0), "n_phix")):
        with pytest.raises(bte.BteError) as ei:
            bte.bte_reconstruct_coeffs(*args)
        assert ei.value.status == bte.BTE_EINVAL and needle in str(ei.value), (args, str(ei.value))


def test_batch_advance_host_validation():
    """bte_batch_advance rejects a NULL batch before any device work."""
    import ctypes
    left = ctypes.c_int32(0)
    rc = bte.lib().bte_batch_advance(None, 1, ctypes.byref(left))
    assert rc == bte.BTE_EINVAL
    rc = bte.lib().bte_batch_advance(None, 1, None)
    assert rc == bte.BTE_EINVAL
