"""The C-ABI library loads, exports every entry point ``include/slic.h``
declares, and its pure-host logic (parameter validation, grid, workspace
sizing, error strings) behaves as documented.  No GPU needed."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slic.h")


@pytest.fixture(scope="module")
def abi():
    from paper_1509_04232_amd import _abi
    return _abi


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(slic_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(abi):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(abi.lib, n), f"{n} declared in slic.h but not exported"
    assert set(names) == set(abi.EXPORTED)


def _p(abi, **kw):
    d = dict(width=640, height=480, pitch=0, channels=3, S=16, K=0, m=10.0, flags=1, min_segment=0)
    d.update(kw)
    if d["pitch"] == 0:
        d["pitch"] = d["width"] * d["channels"]
    return abi.SlicParams(**d)


@pytest.mark.parametrize("w,h,S,K", [(640, 480, 16, 0), (1920, 1080, 8, 0), (1920, 1080, 16, 0),
                                     (640, 480, 0, 1200), (5, 3, 0, 1000), (7, 5, 100, 0),
                                     (1, 1, 1, 0), (3631, 3859, 0, 2000)])
def test_grid_matches_oracle_reading(abi, w, h, S, K):
    assert abi.slic_grid(_p(abi, width=w, height=h, S=S, K=K)) == oracle.grid(w, h, S, K)


@pytest.mark.parametrize("bad", [dict(width=0), dict(height=-1), dict(channels=2),
                                 dict(pitch=10), dict(S=-1), dict(S=0, K=0), dict(m=-1.0),
                                 dict(m=float("nan")), dict(m=float("inf")), dict(m=1e30), dict(m=2e13),
                                 dict(flags=16), dict(flags=6),
                                 dict(min_segment=-1), dict(width=1 << 25, height=1),
                                 dict(width=40000, height=40000)])
def test_invalid_params_rejected(abi, bad):
    p = _p(abi, **bad)
    assert abi.lib.slic_workspace_bytes(ctypes.byref(p)) == 0
    assert abi.lib.slic_grid(ctypes.byref(p), None, None, None) == abi.SLIC_EINVAL
    ctx = ctypes.c_void_p()
    assert abi.lib.slic_init(ctypes.byref(ctx), ctypes.byref(p), 256, None, 256, 1 << 30) == \
        abi.SLIC_EINVAL
    assert ctx.value is None


def test_workspace_size_grows_with_the_image(abi):
    small = abi.slic_workspace_bytes(_p(abi, width=320, height=240))
    big = abi.slic_workspace_bytes(_p(abi, width=1920, height=1080, S=8))
    assert 0 < small < big
    n = 1920 * 1080
    assert big >= n * (3 * 4 + 4 + 4 * 4)  # Lab, labels, connectivity scratch
    assert big % 256 == 0


def test_init_rejects_small_or_misaligned_workspace(abi):
    p = _p(abi)
    need = abi.slic_workspace_bytes(p)
    ctx = ctypes.c_void_p()
    assert abi.lib.slic_init(ctypes.byref(ctx), ctypes.byref(p), 256, None, 256, need - 1) == \
        abi.SLIC_EINVAL
    assert abi.lib.slic_init(ctypes.byref(ctx), ctypes.byref(p), 256, None, 258, need) == \
        abi.SLIC_EINVAL
    assert abi.lib.slic_init(None, ctypes.byref(p), 256, None, 256, need) == abi.SLIC_EINVAL


def test_null_context_calls(abi):
    assert abi.lib.slic_iterate(None, 1) == abi.SLIC_EINVAL
    assert abi.lib.slic_enforce_connectivity(None, None) == abi.SLIC_EINVAL
    assert abi.lib.slic_get_labels(None, 256) == abi.SLIC_EINVAL
    assert abi.lib.slic_energy(None, 256) == abi.SLIC_EINVAL
    abi.lib.slic_destroy(None)


def test_strerror(abi):
    assert abi.slic_strerror(0) == "ok"
    assert abi.slic_strerror(abi.SLIC_EINVAL) == "invalid argument"
    assert abi.slic_strerror(abi.SLIC_EHIP) == "HIP runtime error"
    assert abi.slic_strerror(99) == "unknown error"


def test_timing_read_without_launches(abi):
    abi.slic_timing_enable(True)
    assert abi.slic_timing_read("assign") == (0.0, 0)
    abi.slic_timing_enable(False)


def test_no_device_is_an_error_not_a_fallback(abi):
    """Without a GPU the library reports SLIC_EHIP (or rejects the fake
    pointers) instead of computing anything on the host."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = _p(abi)
    need = abi.slic_workspace_bytes(p)
    ctx = ctypes.c_void_p()
    rc = abi.lib.slic_init(ctypes.byref(ctx), ctypes.byref(p), 4096, None, 8192, need)
    assert rc in (abi.SLIC_EHIP, abi.SLIC_EINVAL)
    assert ctx.value is None


def test_assign_variant_table(abi):
    n = abi.slic_assign_variants()
    assert n >= 7
    shapes = [abi.slic_assign_variant_info(v) for v in range(1, n + 1)]
    for vec, rows, tw, th in shapes:
        assert vec in (1, 2, 4) and rows >= 1 and tw * th == 256 * vec * rows
    with pytest.raises(abi.SlicError):
        abi.slic_assign_variant_info(0)
    with pytest.raises(abi.SlicError):
        abi.slic_assign_variant_info(n + 1)
    # 4-wide variants need S % 4 == 0 and width % 4 == 0
    vec4 = [v for v in range(1, n + 1) if shapes[v - 1][0] == 4]
    with pytest.raises(abi.SlicError):
        abi.slic_set_assign_variant(642, 480, 16, vec4[0])
    with pytest.raises(abi.SlicError):
        abi.slic_set_assign_variant(640, 480, 6, vec4[0])
    abi.slic_set_assign_variant(640, 480, 16, vec4[0])
    assert abi.slic_get_assign_variant(640, 480, 16) == vec4[0]
    abi.slic_set_assign_variant(640, 480, 16, 0)
    assert abi.slic_get_assign_variant(640, 480, 16) != 0
    # 2-wide variants need S % 2 == 0 and width % 2 == 0
    vec2 = [v for v in range(1, n + 1) if shapes[v - 1][0] == 2]
    assert vec2
    with pytest.raises(abi.SlicError):
        abi.slic_set_assign_variant(641, 480, 16, vec2[0])
    with pytest.raises(abi.SlicError):
        abi.slic_set_assign_variant(640, 480, 7, vec2[0])
    abi.slic_set_assign_variant(640, 480, 6, vec2[0])
    abi.slic_set_assign_variant(640, 480, 6, 0)


def test_noalloc_limit_matches_header_and_is_checked_on_the_host(abi):
    text = open(HEADER).read()
    m = re.search(r"#define SLIC_NOALLOC_MAX_WORKSPACE \((\d+)u << (\d+)\)", text)
    assert m and (int(m.group(1)) << int(m.group(2))) == abi.SLIC_NOALLOC_MAX_WORKSPACE
    # 1920x1080 fits at S = 7, not at S = 6; beyond the limit the call
    # returns SLIC_EINVAL before any device call (no GPU needed)
    assert abi.slic_workspace_bytes(_p(abi, width=1920, height=1080, S=7)) <= \
        abi.SLIC_NOALLOC_MAX_WORKSPACE
    p = _p(abi, width=1920, height=1080, S=6)
    assert abi.slic_workspace_bytes(p) > abi.SLIC_NOALLOC_MAX_WORKSPACE
    assert abi.lib.slic_segment_noalloc(ctypes.byref(p), 256, 2, 1, 256, None, None, None,
                                        None) == abi.SLIC_EINVAL
    assert abi.lib.slic_segment_noalloc(ctypes.byref(_p(abi, m=-1.0)), 256, 2, 1, 256, None,
                                        None, None, None) == abi.SLIC_EINVAL


def test_compactness_bound(abi):
    """(m/S) times the diagonal (plus two cells) may reach 1e15, no more:
    every distance of Eq. 1 and of its squared form stays finite in FP32."""
    diag = (640 ** 2 + 480 ** 2) ** 0.5 + 32
    size = lambda **kw: abi.lib.slic_workspace_bytes(ctypes.byref(_p(abi, **kw)))  # noqa: E731
    assert size(m=float(1e15 * 16 / diag * 0.999)) > 0
    assert size(m=float(1e15 * 16 / diag * 1.001)) == 0
    assert size(m=0.0) > 0
