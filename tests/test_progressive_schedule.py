"""Host-side schedules of progressive training (Sec. 3.2.4, Eq. 6, Sec. 4.2). CPU only."""
import math

import pytest

from paper_2501_14534_amd import progressive as PG
from paper_2501_14534_amd import scenes


def test_eq6_resolution_schedule():
    assert PG.resolution(0, 158, 1264, 19500) == 158
    assert PG.resolution(19500, 158, 1264, 19500) == 1264
    assert PG.resolution(40000, 158, 1264, 19500) == 1264
    assert PG.resolution(9750, 158, 1264, 19500) == 711  # 158 + 1106 / 2
    vals = [PG.resolution(i, 158, 1264, 19500) for i in range(0, 20000, 500)]
    assert vals == sorted(vals)


def test_downsample_factor_log_decay():
    assert PG.downsample_factor(0) == 8.0
    assert PG.downsample_factor(19500) == 1.0
    assert PG.downsample_factor(9750) == pytest.approx(math.sqrt(8.0))
    # the logarithm falls linearly
    a, b, c = (math.log(PG.downsample_factor(i)) for i in (1000, 2000, 3000))
    assert b - a == pytest.approx(c - b)


def test_blur_kernel_schedule():
    assert PG.blur_kernel(0) == (9, 2.4)
    assert PG.blur_kernel(99) == (9, 2.4)          # updated every 100 iterations
    k, s = PG.blur_kernel(100)
    assert k == 7 and s == pytest.approx(2.4 * (1 - 100 / 19500))
    assert PG.blur_kernel(19500) is None
    assert PG.blur_kernel(18000) is None           # below 3 taps: off
    ks = [PG.blur_kernel(i) for i in range(0, 19500, 100)]
    sizes = [k[0] for k in ks if k is not None]
    assert sizes == sorted(sizes, reverse=True) and all(k % 2 == 1 for k in sizes)
    # with 8x downsampling the kernel shrinks by the same factor (off at the start)
    assert PG.blur_kernel(0, downsample=8.0) is None
    assert PG.blur_kernel(0, downsample=2.0) == (3, 1.2)


def test_lowpass_closed_form_and_bound():
    assert PG.lowpass_s(1000, 1264, 832) == pytest.approx(1264 * 832 / (9 * math.pi * 1000))
    assert PG.lowpass_s(10 ** 7, 1264, 832) == 0.3
    assert PG.lowpass_s(0, 10, 10) == 0.3


def test_scaled_cameras_keep_the_field_of_view():
    cams = scenes.config(4, n=16).cams
    for c, d in zip(cams, PG.scaled_cameras(cams, 4.0)):
        assert d.width == round(c.width / 4) and d.height == round(c.height / 4)
        assert d.width / d.fx == pytest.approx(c.width / c.fx, rel=1e-6)
        assert d.cx / d.width == pytest.approx(c.cx / c.width, rel=1e-6)
