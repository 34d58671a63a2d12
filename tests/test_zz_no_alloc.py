"""The allocation-free fidelity-loss call (D-SSIM maps in the library's static per-GPU scratch)
against dass_fidelity_loss_grad with caller scratch, through the C ABI: two calls in a row,
the second with fewer and smaller views, each bit-identical to the call it varies; and sizes
beyond the static scratch rejected before anything is enqueued."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import log, make_ctx

pytestmark = pytest.mark.gpu


def _images(rng, cams):
    R, T = [], []
    for c in cams:
        r = rng.uniform(size=(3, c.height, c.width)).astype(np.float32)
        t = np.clip(r + rng.normal(0, 0.1, size=r.shape), 0, 1).astype(np.float32)
        R.append(torch.from_numpy(r).cuda())
        T.append(torch.from_numpy(t).cuda())
    return R, T


def _run(ctx, cams, R, T, lam, noalloc):
    dl = [torch.full((3, c.height, c.width), 3.0, device="cuda") for c in cams]
    err = [torch.full((c.height, c.width), -1.0, device="cuda") for c in cams]
    loss = torch.full((1,), 0.25, device="cuda")
    if noalloc:
        ctx.fidelity_loss_grad_noalloc(cams, R, T, lam, dl, err, loss)
    else:
        ctx.fidelity_loss_grad(cams, R, T, lam, dl, err, loss)
    ctx.sync()
    return dl, err, loss


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_noalloc_fidelity_loss_matches_caller_scratch(lam):
    from paper_2411_14847_amd import _ffi
    rng = np.random.default_rng(77)
    first = [synth.make_camera(np.eye(3), (0, 0, 0), w, h) for w, h in ((640, 480), (300, 221), (37, 29))]
    second = [synth.make_camera(np.eye(3), (0, 0, 0), w, h) for w, h in ((150, 110), (9, 7))]
    assert sum(c.width * c.height for c in first) <= _ffi.NOALLOC_MAX_PIXELS
    ctx = make_ctx(10, first)
    for k, cams in enumerate((first, second)):
        log(f"[no-alloc] call {k}: lambda {lam}, views {[(c.width, c.height) for c in cams]}")
        R, T = _images(rng, cams)
        dl_a, err_a, loss_a = _run(ctx, cams, R, T, lam, noalloc=True)
        dl_b, err_b, loss_b = _run(ctx, cams, R, T, lam, noalloc=False)
        for v in range(len(cams)):
            assert torch.equal(dl_a[v], dl_b[v]), (k, v, (dl_a[v] - dl_b[v]).abs().max().item())
            assert torch.equal(err_a[v], err_b[v]), (k, v)
        assert torch.equal(loss_a, loss_b), (k, loss_a.item(), loss_b.item())


def test_noalloc_fidelity_loss_rejects_sizes_beyond_its_scratch():
    from paper_2411_14847_amd import _ffi
    from paper_2411_14847_amd.api import DassError
    side = int(np.ceil(np.sqrt(_ffi.NOALLOC_MAX_PIXELS))) + 1
    cams = [synth.make_camera(np.eye(3), (0, 0, 0), side, side)]
    ctx = make_ctx(10, [synth.make_camera(np.eye(3), (0, 0, 0), 64, 64)])
    x = torch.zeros(3, side, side, device="cuda")
    dl = [torch.full_like(x, 5.0)]
    with pytest.raises(DassError, match="allocation-free"):
        ctx.fidelity_loss_grad_noalloc(cams, [x], [x], 0.5, dl)
    ctx.sync()
    assert torch.all(dl[0] == 5.0)  # nothing was enqueued
