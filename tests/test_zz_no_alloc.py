"""The allocation-free residual (sf_residual_noalloc) against sf_residual.

Both run the same kernels in the same order, so the residual r = F - A U and
the per-pair norms ||r||^2 must agree bit for bit.  Two contexts in a row, the
second smaller than the first, check that what the shared static array keeps
from the previous call does not leak into the next one.
"""
import numpy as np
import pytest

from paper_1508_02977_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1508_02977_amd import api  # noqa: E402

# (W, H, B, parts_x, parts_y, overlap, seed): larger first, then smaller
CALLS = [(96, 80, 2, 3, 2, 6, 11), (40, 30, 1, 2, 2, 4, 12)]


def _context(W, H, B, px, py, d, seed):
    pairs = [synth.make_pair("plain640", seed + b, W=W, H=H) for b in range(B)]
    I0 = torch.tensor(np.stack([p.I0 for p in pairs]), dtype=torch.float64, device="cuda")
    I1 = torch.tensor(np.stack([p.I1 for p in pairs]), dtype=torch.float64, device="cuda")
    al = torch.tensor(np.stack([synth.random_alpha(W, H, seed + 7 * b) for b in range(B)]), dtype=torch.float64,
                      device="cuda")
    ctx = api.sf_create(W, H, B, px, py, d)
    api.sf_assemble(ctx, I0, I1, al)
    return ctx


def test_noalloc_residual_equals_residual_on_two_calls(gpu):
    for W, H, B, px, py, d, seed in CALLS:
        print(f"noalloc residual: {W}x{H} B={B}", flush=True)
        ctx = _context(W, H, B, px, py, d, seed)
        U = torch.tensor(np.random.default_rng(seed).normal(size=ctx.field_shape()), dtype=torch.float64,
                         device="cuda")
        r_ref = torch.full(ctx.field_shape(), np.nan, dtype=torch.float64, device="cuda")
        n_ref = api.sf_residual(ctx, U, r_ref)
        r_na = torch.full(ctx.field_shape(), np.nan, dtype=torch.float64, device="cuda")
        n_na = api.sf_residual_noalloc(ctx, U, r_na)
        assert torch.equal(r_na, r_ref)
        assert n_na == n_ref
        # the norms agree with the residual they belong to
        for b in range(B):
            assert abs(n_na[b] - float((r_ref[b] ** 2).sum())) <= 1e-12 * n_ref[b]
        # without a host output the call does not synchronise; the stream orders it
        r_async = torch.full(ctx.field_shape(), np.nan, dtype=torch.float64, device="cuda")
        assert api.sf_residual_noalloc(ctx, U, r_async, norms=False) is None
        torch.cuda.synchronize()
        assert torch.equal(r_async, r_ref)
        ctx.close()


def test_noalloc_limit_matches_header():
    import os
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    hdr = open(os.path.join(root, "include", "sfdd.h")).read()
    m = re.search(r"#define SF_NOALLOC_SCRATCH_BYTES \(1 << (\d+)\)", hdr)
    assert m and (1 << int(m.group(1))) == api.SF_NOALLOC_SCRATCH_BYTES
