"""The C interface on the host (no GPU needed): the library loads, exports
every function that include/fmg.h and include/fv27.h declare, and validates
parameters before any device call."""
import ctypes
import os
import re

import pytest

from paper_1406_7808_amd import fmg
from paper_1406_7808_amd import fv27

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="fmg.h", prefix="fmg_"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(%s[a-z_0-9]+)\s*\(" % prefix, src)))


def test_every_declared_symbol_is_exported():
    names = _declared() + _declared("fv27.h", "fv27_")
    assert "fmg_plan_execute" in names and "fv27_plan_execute" in names and len(names) >= 20
    lib = ctypes.CDLL(fmg._SO)
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    assert sorted(fmg.SYMBOLS) == _declared()
    assert sorted(fv27.SYMBOLS) == _declared("fv27.h", "fv27_")


FV = dict(n=(32, 16, 16), h=1 / 16, levels=5, sr_levels=2, segments=(4, 2, 2), buffers=(2, 2))


@pytest.mark.parametrize("kw,frag", [
    (dict(h=0.0), "h must be positive"),
    (dict(n=(30, 16, 16)), "divisible by 2^(levels-1)"),
    (dict(levels=2), "at most 512 cells"),
    (dict(buffers=(3, 2)), "even"),
    (dict(buffers=(8, 2)), "at least half"),
    (dict(segments=(2, 2, 2)), "cubic"),
    (dict(sr_levels=4, buffers=(2, 2, 2, 2)), "divisible by segments"),
    (dict(sr_levels=5), "sr_levels"),
    (dict(degrees=(9, 2, 1)), "Chebyshev degrees"),
])
def test_fv27_invalid_parameters_are_rejected(kw, frag):
    base = dict(FV)
    base.update(kw)
    st, msg = fv27.check_params(**base)
    assert st == fmg.FMG_EINVAL and frag in msg, msg


def test_fv27_valid_parameters():
    assert fv27.check_params(**FV)[0] == 0
    assert fv27.check_params(**dict(FV, sr_levels=0, buffers=()))[0] == 0


def _chk(N, **kw):
    base = dict(levels=5, sr_levels=2, segments=2, buffers=(2, 2))
    base.update(kw)
    return fmg.check_params(N, **base)


def test_valid_parameters():
    assert _chk(32)[0] == 0
    assert _chk(256, levels=8, sr_levels=3, segments=8, buffers=(2, 4, 6))[0] == 0
    assert _chk(512, levels=8, sr_levels=3, segments=16, buffers=(2, 4, 6))[0] == 0
    assert _chk(96, levels=6, sr_levels=2, segments=3, buffers=(2, 2))[0] == 0
    assert _chk(32, sr_levels=0, segments=1, buffers=())[0] == 0
    assert _chk(1, levels=1, sr_levels=0, segments=1, buffers=())[0] == 0


@pytest.mark.parametrize("N,kw,frag", [
    (32, dict(buffers=(3, 2)), "even"),
    (32, dict(buffers=(-2, 2)), "even"),
    (32, dict(buffers=(8, 2)), "half"),
    (32, dict(segments=3), "divisible"),
    (32, dict(segments=8, sr_levels=3, buffers=(2, 2, 2)), "divisible"),
    (32, dict(levels=2, sr_levels=0, buffers=()), "coarsest"),
    (30, dict(), "n0"),
    (32, dict(sr_levels=5, buffers=(2,) * 5), "sr_levels"),
    (32, dict(sweeps=(9, 2, 1)), "nu_pre"),
    (32, dict(segments=0), "segments_per_dim"),
    (32, dict(levels=0), "levels"),
])
def test_invalid_parameters_are_rejected(N, kw, frag):
    st, msg = _chk(N, **kw)
    assert st == fmg.FMG_EINVAL
    assert frag in msg


def test_null_buffer_schedule_rejected():
    p, keep = fmg.make_params(5, 2, 2, ())
    st = fmg.lib().fmg_check_params(32, ctypes.byref(p))
    assert st == fmg.FMG_EINVAL
    assert b"buffer_schedule" in fmg.lib().fmg_last_error()


def test_null_params_and_plan():
    L = fmg.lib()
    assert L.fmg_check_params(32, None) == fmg.FMG_EINVAL
    assert L.fmg_plan_destroy(None) == 0
    assert L.fmg_plan_execute(None, None, None, None) == fmg.FMG_EINVAL
    assert L.fmg_plan_workspace_bytes(None) == 0


# --- host-only walk of the launch schedule --------------------------------------

MODEL_CASES = [
    (2, dict(levels=1)),
    (8, dict(levels=3)),
    (40, dict(levels=4)),
    (48, dict(levels=5)),
    (32, dict(levels=5, sweeps=(0, 0, 0))),
    (32, dict(levels=5, sweeps=(3, 1, 2))),
    (32, dict(levels=5, sweeps=(8, 8, 8))),
    (32, dict(levels=5, sr_levels=2, segments=2, buffers=(2, 2))),
    (32, dict(levels=5, sr_levels=4, segments=2, buffers=(2, 2, 2, 2))),
    (32, dict(levels=5, sr_levels=1, segments=4, buffers=(0,))),
    (32, dict(levels=5, sr_levels=2, segments=1, buffers=(2, 2))),
    (96, dict(levels=6, sr_levels=2, segments=3, buffers=(2, 2))),
    (256, dict(levels=8)),
    (256, dict(levels=8, sr_levels=3, segments=8, buffers=(2, 4, 6))),
    (512, dict(levels=8, sr_levels=3, segments=16, buffers=(2, 4, 6))),
]


@pytest.mark.parametrize("N,kw", MODEL_CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_schedule_walks_without_null_pointers(N, kw, precision):
    launches, nbytes, ws = fmg.schedule_model(N, precision=precision, **kw)
    assert launches >= 1
    assert nbytes > 0
    # at least f read and u written once per cell
    assert nbytes >= 16.0 * N ** 3


def test_schedule_model_byte_counts():
    _, g, _ = fmg.schedule_model(256, levels=8)
    _, s, _ = fmg.schedule_model(256, levels=8, sr_levels=3, segments=8, buffers=(2, 4, 6))
    _, r, _ = fmg.schedule_model(256, levels=8, sr_levels=3, segments=8, buffers=(2, 4, 6),
                                 precision="fp32_refined")
    N3 = 256 ** 3
    # segmental refinement recomputes buffer cells (1.4x to 12x the genuine
    # cells on the SR levels) but its workgroup-resident segments fuse more
    # steps per pass; the refined solve runs three FP32 solves plus FP64
    # residuals
    assert 60 < g / N3 < 300
    assert 0.8 < s / g < 3.5
    assert r > s


def test_schedule_model_rejects_invalid():
    with pytest.raises(fmg.FMGError):
        fmg.schedule_model(32, levels=5, sr_levels=2, segments=2, buffers=(3, 2))
