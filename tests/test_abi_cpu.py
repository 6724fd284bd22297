"""Host-side checks of libmpdata that need no GPU: the library loads, exports
every entry point include/mpdata.h declares, and rejects invalid arguments
before touching the device."""
import ctypes
import re

import pytest

from paper_1507_01265_amd import _lib


def _declared():
    src = open(_lib.HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpdata_[a-z_]+)\s*\(", src)))


def test_header_declares_the_core_entry_points():
    names = _declared()
    for core in ("mpdata_create", "mpdata_step", "mpdata_destroy", "mpdata_mass",
                 "mpdata_workspace_bytes"):
        assert core in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(_declared()) <= set(_lib._SIGNATURES)


def test_abi_version_and_tiles():
    assert _lib.mpdata_abi_version() == 1
    n = _lib.mpdata_tile_count()
    assert n >= 1
    for t in range(1, n + 1):
        tx, ty, threads = _lib.mpdata_tile_info(t)
        assert tx >= 1 and ty >= 1 and 64 <= threads <= 1024
    with pytest.raises(_lib.MpdataError):
        _lib.mpdata_tile_info(n + 1)


def test_default_tile_is_a_valid_shape():
    n = _lib.mpdata_tile_count()
    for dtype in (_lib.MPDATA_FP64, _lib.MPDATA_FP32):
        for bc in (_lib.MPDATA_BC_PERIODIC, _lib.MPDATA_BC_OPEN):
            assert 1 <= _lib.mpdata_default_tile(dtype, bc) <= n
    assert _lib.mpdata_default_tile(7, 0) == 0 and _lib.mpdata_default_tile(0, 7) == 0


def _params(**kw):
    d = dict(nx=32, ny=32, nz=16, dtype=0, bc=0, iord=2, nonos=1, tile=0, eps=1e-15)
    d.update(kw)
    return _lib.mpdata_params(**d)


def test_workspace_bytes():
    b64 = _lib.mpdata_workspace_bytes(_params())
    b32 = _lib.mpdata_workspace_bytes(_params(dtype=1))
    assert b64 >= 32 * 32 * 16 * 8 and b32 >= 32 * 32 * 16 * 4 and b64 > b32
    assert b64 % 256 == 0


@pytest.mark.parametrize("bad", [dict(nx=0), dict(nz=-1), dict(dtype=2), dict(bc=5),
                                 dict(iord=0), dict(iord=17), dict(iord=1, nonos=1), dict(nonos=2),
                                 dict(eps=0.0), dict(eps=float("nan")), dict(eps=9.9e-31),
                                 dict(eps=1e-100), dict(eps=float("inf")), dict(tile=99),
                                 dict(nx=4096, ny=4096, nz=256),
                                 dict(nx=30000, ny=30000, nz=1)])
def test_invalid_params_are_rejected(bad):
    p = _params(**bad)
    assert _lib.mpdata_workspace_bytes(p) == 0
    with pytest.raises(_lib.MpdataError) as e:
        _lib.mpdata_create(p, 256, 256, 256, 256, 256, 256, 1 << 30, None)
    assert e.value.code == _lib.MPDATA_EINVAL
    assert _lib.mpdata_last_error(None)


def test_eps_floor_keeps_the_common_denominators_normal():
    """eps >= 1e-30: the FP64 pseudo-velocity divides by about h eps^3 on a
    zero background, which stays a normal double (2e-90) at the floor."""
    assert _lib.mpdata_workspace_bytes(_params(eps=1e-30)) > 0
    assert _lib.mpdata_workspace_bytes(_params(eps=0.5)) > 0
    assert _lib.mpdata_workspace_bytes(_params(eps=1e-31)) == 0
    with pytest.raises(_lib.MpdataError, match="eps"):
        _lib.mpdata_create(_params(eps=1e-40), 256, 256, 256, 256, 256, 256, 1 << 30, None)


def test_vsign_flag_needs_a_default_launch_shape():
    vs = _lib.MPDATA_FLAG_VSIGN
    assert _lib.mpdata_workspace_bytes(_params(flags=vs)) > 0
    for t in (2, 5):
        assert _lib.mpdata_workspace_bytes(_params(flags=vs, tile=t)) > 0
    for t in (1, 3, 4, 6):
        assert _lib.mpdata_workspace_bytes(_params(flags=vs, tile=t)) == 0
    assert _lib.mpdata_workspace_bytes(_params(flags=16)) == 0


def test_tvel_flag_constraints():
    """Courant numbers that change in time: iord 2, the default launch
    shape, not with the variable-sign option (with or without DIV)."""
    tv = _lib.MPDATA_FLAG_TVEL
    for dtype in (0, 1):
        for bc in (0, 1):
            for flags in (tv, tv | _lib.MPDATA_FLAG_DIV):
                assert _lib.mpdata_workspace_bytes(_params(flags=flags, dtype=dtype, bc=bc)) > 0
            default = _lib.mpdata_default_tile(dtype, bc)
            assert _lib.mpdata_workspace_bytes(_params(flags=tv, dtype=dtype, bc=bc,
                                                       tile=default)) > 0
            for t in range(1, _lib.mpdata_tile_count() + 1):
                if t != default:
                    assert _lib.mpdata_workspace_bytes(_params(flags=tv, dtype=dtype, bc=bc,
                                                               tile=t)) == 0
    assert _lib.mpdata_workspace_bytes(_params(flags=tv, iord=3)) == 0
    assert _lib.mpdata_workspace_bytes(_params(flags=tv, iord=1, nonos=0)) == 0
    assert _lib.mpdata_workspace_bytes(_params(flags=tv | _lib.MPDATA_FLAG_VSIGN)) == 0


def test_step_tv_rejects_a_null_context():
    lib = _lib.load()
    assert lib.mpdata_step_tv(None, 1, None, None, None) == _lib.MPDATA_EINVAL


def test_div_flag_needs_a_default_launch_shape():
    dv = _lib.MPDATA_FLAG_DIV
    for flags in (dv, dv | _lib.MPDATA_FLAG_VSIGN):
        assert _lib.mpdata_workspace_bytes(_params(flags=flags)) > 0
        for t in (2, 5):
            assert _lib.mpdata_workspace_bytes(_params(flags=flags, tile=t)) > 0
        for t in (1, 3, 4, 6):
            assert _lib.mpdata_workspace_bytes(_params(flags=flags, tile=t)) == 0


def test_more_corrective_passes_need_chain_buffers():
    """iord > 2: one more iterate, the three velocity face arrays and (with
    the limiter) psi1 of the head launch; from iord 4 on a second set with
    the running maximum and minimum of a middle pass, and from iord 5 on the
    minimum of the first set too; only on the default launch shape."""
    n, nf = 32 * 32 * 16, 33 * 32 * 16 + 32 * 33 * 16 + 32 * 32 * 17
    b2 = _lib.mpdata_workspace_bytes(_params())
    b3 = _lib.mpdata_workspace_bytes(_params(iord=3))
    b4 = _lib.mpdata_workspace_bytes(_params(iord=4))
    b5 = _lib.mpdata_workspace_bytes(_params(iord=5))
    b16 = _lib.mpdata_workspace_bytes(_params(iord=16))
    assert (2 * n + nf) * 8 <= b3 - b2 < (3 * n + nf) * 8
    assert b4 - b3 >= (3 * n + nf) * 8
    assert b5 - b4 >= n * 8
    assert b16 > b5
    assert _lib.mpdata_workspace_bytes(_params(iord=3, nonos=0)) <= b3 - n * 8
    assert _lib.mpdata_workspace_bytes(_params(iord=3, tile=5)) == b3
    assert _lib.mpdata_workspace_bytes(_params(iord=3, tile=1)) == 0
    assert _lib.mpdata_workspace_bytes(_params(iord=3, dtype=1, bc=1, tile=2)) > 0
    assert _lib.mpdata_workspace_bytes(_params(iord=3, dtype=1, bc=1, tile=5)) == 0


def test_plane_limit_depends_on_word_size():
    # one x-y plane is addressed with 32-bit byte offsets below 2^31 (an
    # offset of 2^31 masks a lane): 20001^2 words fit in 2 GiB as FP32, not
    # as FP64
    assert _lib.mpdata_workspace_bytes(_params(nx=20000, ny=20000, nz=1, dtype=1)) > 0
    assert _lib.mpdata_workspace_bytes(_params(nx=20000, ny=20000, nz=1, dtype=0)) == 0


def test_null_and_misaligned_pointers_are_rejected():
    p = _params()
    with pytest.raises(_lib.MpdataError, match="NULL"):
        _lib.mpdata_create(p, None, 256, 256, 256, 256, 256, 1 << 30, None)
    with pytest.raises(_lib.MpdataError, match="aligned"):
        _lib.mpdata_create(p, 258, 256, 256, 256, 256, 256, 1 << 30, None)
    with pytest.raises(_lib.MpdataError, match="workspace"):
        _lib.mpdata_create(p, 256, 256, 256, 256, 256, 256, 16, None)


def test_destroy_is_null_safe():
    _lib.mpdata_destroy(None)


def test_option_tiles_are_the_default_shapes():
    """The tuner's shapes for the variable-sign option and the divergent-flow
    term are exactly those the library accepts with those flags."""
    from paper_1507_01265_amd import autotune
    t = autotune.option_tiles()
    assert sorted(t) == [2, 5]
    for tile in range(1, _lib.mpdata_tile_count() + 1):
        ok = _lib.mpdata_workspace_bytes(_params(flags=_lib.MPDATA_FLAG_DIV, tile=tile)) > 0
        assert ok == (tile in t)


def test_batches_run_the_iord_2_step_only():
    """A batch is one launch of the fused step per step: more corrective
    passes are for single-grid contexts."""
    ok = _lib.mpdata_batch_workspace_bytes([_params(), _params(nx=20)], 0, 0)
    assert ok > 0
    assert _lib.mpdata_batch_workspace_bytes([_params(iord=3), _params(nx=20, iord=3)], 0, 0) == 0
