"""The C-ABI library loads and exports what include/envar.h declares (CPU only, no compute calls)."""
import os
import re

import pytest

from paper_2605_23812_amd import envar as E

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "envar.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|size_t|const char\*)\s+(envar_[a-z_]+)\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    L = E.lib()
    names = _declared()
    assert "envar_forward" in names and "envar_gradient" in names and "envar_iterate" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(E.EXPORTS) == set(names)


def test_sizes_and_control_dims():
    p = E.Problem(inv_h=32)
    assert E.control_dim(p) == 4096          # 2048 per component at h = 1/32
    assert E.cell_count(p) == 5120           # 128 x 32 + 32 x 32
    p2 = E.Problem(inv_h=128, Re=7500.0)
    assert E.control_dim(p2) == 65536        # 32768 per component at h = 1/128
    assert E.cell_count(p2) == 81920
    assert E.control_dim(E.Problem(inv_h=32, region=E.REGION_CAVITY)) == 2048
    assert E.control_dim(E.Problem(inv_h=16, region=E.REGION_BOX, box=(1.5, 1.6, -0.1, 0.0))) == 8
    # workspace grows linearly with members
    w1, w2 = E.workspace_bytes(p, 1), E.workspace_bytes(p, 2)
    w9 = E.workspace_bytes(p, 9)
    assert w1 > 0 and abs((w9 - w1) - 8 * (w2 - w1)) < 8 * 4096
    assert E.workspace_bytes(E.Problem(inv_h=32, precision=E.MIXED), 9) < w9
    # mixed precision stores the FP32 anomalies; FP64 with n <= m forms them where they are read
    assert E.gradient_bytes(8, 4096, E.MIXED) > 8 * 4096 * 4
    assert 0 < E.gradient_bytes(8, 4096) < 8 * 4096 * 8
    assert E.state_bytes(p) > 5 * 129 * 65 * 8


@pytest.mark.parametrize("bad", [dict(inv_h=24), dict(inv_h=8), dict(Re=-1.0), dict(x_cav=1.1),
                                 dict(geometry=7), dict(region=9), dict(precision=3)])
def test_invalid_problems_are_rejected(bad):
    with pytest.raises(E.EnvarError) as ei:
        E.control_dim(E.Problem(**bad))
    assert ei.value.code == E.EINVAL
    assert E.workspace_bytes(E.Problem(**bad), 4) == 0


def test_oracle_and_library_agree_on_the_control_region():
    from oracle.envar import Problem as OP

    for n, reg, oreg, box in [(32, E.REGION_COLUMN, "column", None), (32, E.REGION_CAVITY, "cavity", None),
                              (16, E.REGION_BOX, "box", (1.2, 1.9, -0.5, 0.3))]:
        kw = dict(box=box) if box else {}
        assert E.control_dim(E.Problem(inv_h=n, region=reg, **kw)) == OP(inv_h=n, region=oreg, **kw).m


def test_static_gradient_rejects_sizes_beyond_its_scratch_before_any_launch():
    """envar_gradient_static checks the workspace size against its static array on the host (no
    device call before the check, so this runs without a GPU)."""
    import ctypes

    L = E.lib()
    fake = ctypes.c_void_p(256)  # never dereferenced: the size check comes first
    for n, m, prec in [(256, 65536, E.MIXED), (1024, 65536, E.FP64), (1100, 1024, E.FP64)]:
        assert E.gradient_bytes(n, m, prec) > E.GRADIENT_STATIC_MAX_BYTES
        rc = L.envar_gradient_static(fake, fake, n, m, prec, fake, None)
        assert rc == E.ENOMEM, rc
        assert b"static array" in L.envar_last_error()
    # the benchmark's reduction fits in both precisions
    assert E.gradient_bytes(64, 65536, E.FP64) <= E.GRADIENT_STATIC_MAX_BYTES
    assert E.gradient_bytes(64, 65536, E.MIXED) <= E.GRADIENT_STATIC_MAX_BYTES


def test_gradient_flags_are_checked_before_any_launch():
    """The pseudo-inverse flag leaves the workspace size as it is; an unknown precision or flag is
    refused on the host (no device call before the check, so this runs without a GPU)."""
    import ctypes

    L = E.lib()
    for prec in (E.FP64, E.MIXED):
        assert E.gradient_bytes(40, 500, prec | E.GRADIENT_PINV) == E.gradient_bytes(40, 500, prec)
    fake = ctypes.c_void_p(256)  # never dereferenced: the precision check comes first
    for bad in (2, E.GRADIENT_PINV | 2, 32):
        rc = L.envar_gradient(fake, fake, 40, 500, bad, fake, 1 << 30, fake, None)
        assert rc == E.EINVAL, (bad, rc)
        assert b"unknown precision" in L.envar_last_error()
        rc = L.envar_gradient_static(fake, fake, 40, 500, bad, fake, None)
        assert rc == E.EINVAL, (bad, rc)
