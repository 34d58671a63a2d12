"""Host-side helpers of the binding (no GPU): the accumulator carving and the level-resolution
progression the trainer uses for the hash fields."""
import numpy as np
import torch

import synth
from paper_2411_14847_amd.api import carve_zeroed, geometric_res


def test_carve_zeroed_layout_and_single_fill():
    specs = [((3, 10), torch.float32), ((7,), torch.int32), ((1,), torch.float32), ((4, 65), torch.float32)]
    buf, ts = carve_zeroed(specs, device="cpu")
    for (shape, dt), t in zip(specs, ts):
        assert tuple(t.shape) == shape and t.dtype == dt and t.is_contiguous()
        assert (t.data_ptr() - buf.data_ptr()) % 256 == 0  # each starts on a 256-byte boundary
    ends = sorted((t.data_ptr(), t.data_ptr() + t.numel() * 4) for t in ts)
    assert all(a[1] <= b[0] for a, b in zip(ends, ends[1:]))  # no overlap
    for t in ts:
        t.fill_(3)
    buf.zero_()
    assert all(int(t.abs().sum()) == 0 for t in ts)


def test_level_resolutions_match_the_test_generator():
    for n_min, n_max, L in ((16, 2048, 16), (16, 512, 8), (4, 64, 8), (4, 32, 8), (16, 16, 1)):
        r = geometric_res(n_min, n_max, L)
        assert r == synth.geometric_res(n_min, n_max, L)
        assert r[0] == n_min and r[-1] == n_max and all(np.diff(r) >= 0)
