"""GPU: the graph-replayed Schwarz loop (sf_schwarz_solve_graph).

The replayed chunk holds the same kernels in the same order as the ordinary
loop, so the iterate, the sweep counts and the residuals must equal those of
sf_schwarz_solve bit for bit: on small and ragged geometries, a batch with a
pair that has nothing to solve, a max_sweeps that leaves a partial chunk,
solves repeated with other work on the device in between, solves while
another stream keeps the device busy, the FP32-tile sweep form, and the
timed 640x480 workload.  One case is also held to the oracle's iterate.
"""
import numpy as np
import pytest

from oracle import fem, schwarz
from paper_1508_02977_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1508_02977_amd import api  # noqa: E402


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def planes(Uint, W, H):
    return Uint.reshape(H, W, 3).transpose(2, 0, 1).copy()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def emax(a, b):
    """Largest element-wise difference of field planes [..., 3, H, W] (or any
    array), each field relative to its own largest magnitude."""
    a, b = np.asarray(a), np.asarray(b)
    if a.ndim >= 3 and a.shape[-3] == 3:
        return max(float(np.abs(a[..., c, :, :] - b[..., c, :, :]).max() / max(np.abs(b[..., c, :, :]).max(), 1e-300))
                   for c in range(3))
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def context(kind, seed, W, H, px, py, d, batch_pairs=None):
    if batch_pairs is None:
        batch_pairs = [synth.make_pair(kind, seed, W=W, H=H)]
    B = len(batch_pairs)
    ctx = api.sf_create(W, H, B, px, py, d)
    I0 = dev(np.stack([p.I0 for p in batch_pairs]))
    I1 = dev(np.stack([p.I1 for p in batch_pairs]))
    Al = dev(np.stack([synth.random_alpha(W, H, seed + b) for b in range(B)]))
    api.sf_assemble(ctx, I0, I1, Al)
    api.sf_factor_subdomains(ctx)
    return ctx, batch_pairs


def both(ctx, rtol, max_sweeps, start=0.0):
    Ue = torch.full(ctx.field_shape(), start, dtype=torch.float64, device="cuda")
    Ug = Ue.clone()
    re = api.sf_schwarz_solve(ctx, Ue, rtol, max_sweeps)
    rg = api.sf_schwarz_solve_graph(ctx, Ug, rtol, max_sweeps)
    return (Ue, re), (Ug, rg)


@pytest.mark.parametrize("kind,seed,W,H,px,py,d", [
    ("plain64", 1, 64, 64, 2, 2, 4),
    ("plain64", 5, 37, 29, 3, 2, 5),
    ("plain640", 3, 72, 56, 3, 3, 8),
])
def test_graph_solve_equals_ordinary_solve(gpu, kind, seed, W, H, px, py, d):
    ctx, _ = context(kind, seed, W, H, px, py, d)
    (Ue, re), (Ug, rg) = both(ctx, 1e-9, 500)
    assert re[0] == api.SF_OK and rg == re
    assert torch.equal(Ug, Ue)
    ctx.close()


def test_graph_partial_chunk_and_not_converged(gpu):
    # 7 sweeps: one replayed chunk of 4, then 3 ordinary iterations
    ctx, _ = context("plain64", 2, 40, 30, 2, 2, 4)
    (Ue, re), (Ug, rg) = both(ctx, 1e-14, 7)
    assert re[0] == api.SF_NOT_CONVERGED and re[1] == [7]
    assert rg == re and torch.equal(Ug, Ue)
    # fewer sweeps than one chunk: no replay at all
    (Ue, re), (Ug, rg) = both(ctx, 1e-14, 3)
    assert rg == re and re[1] == [3] and torch.equal(Ug, Ue)
    ctx.close()


def test_graph_batch_with_a_pair_that_has_nothing_to_solve(gpu):
    W, H = 40, 30
    p = synth.make_pair("plain64", 4, W=W, H=H)
    q = synth.Pair(p.I0, p.I0.copy(), p.w, p.gain, name="identical frames")   # F = 0
    ctx, _ = context("plain64", 4, W, H, 2, 2, 4, batch_pairs=[p, q])
    (Ue, re), (Ug, rg) = both(ctx, 1e-9, 500, start=1.0)
    assert rg == re and re[1][1] == 0 and re[1][0] > 4
    assert torch.equal(Ug, Ue) and float(Ug[1].abs().max()) == 0.0
    ctx.close()


def test_graph_solves_repeat_with_other_work_in_between(gpu):
    ctx, _ = context("plain640", 7, 72, 56, 3, 3, 8)
    (Ue, re), (Ug, rg) = both(ctx, 1e-9, 500)
    assert rg == re and torch.equal(Ug, Ue)
    for start in (0.5, 0.0, -0.25):
        # ordinary launches, a residual and a host synchronisation between the graph solves
        Uo = torch.full(ctx.field_shape(), start, dtype=torch.float64, device="cuda")
        ro = api.sf_schwarz_solve(ctx, Uo, 1e-9, 500)
        r = torch.empty_like(Uo)
        api.sf_residual(ctx, Uo, r)
        torch.cuda.synchronize()
        Ug2 = torch.full(ctx.field_shape(), start, dtype=torch.float64, device="cuda")
        rg2 = api.sf_schwarz_solve_graph(ctx, Ug2, 1e-9, 500)
        assert rg2 == ro and torch.equal(Ug2, Uo)
    ctx.close()


def test_graph_iterate_matches_oracle(gpu):
    W, H, px, py, d = 64, 64, 2, 2, 4
    ctx, pairs = context("plain64", 1, W, H, px, py, d)
    U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    code, sw, _ = api.sf_schwarz_solve_graph(ctx, U, 0.0, 12)
    assert code == api.SF_NOT_CONVERGED and sw == [12]
    p = pairs[0]
    A, F = fem.assemble(p.I0, p.I1, synth.random_alpha(W, H, 1), 1.0)
    facs = schwarz.factor_subdomains(A, schwarz.decompose(W, H, px, py, d))
    Uo = schwarz.ras_solve(A, F, facs, rtol=0.0, max_sweeps=12).U
    assert emax(U[0].cpu().numpy(), planes(Uo, W, H)) <= 1e-10
    ctx.close()


def test_graph_full_size_workload(gpu):
    # the timed 640x480 pair, 4x4 subdomains, overlap 8, to 1e-8
    p = synth.make_pair("plain640", 2)
    W, H = 640, 480
    ctx = api.sf_create(W, H, 1, 4, 4, 8)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(synth.constant_alpha(W, H)[None]))
    api.sf_factor_subdomains(ctx)
    (Ue, re), (Ug, rg) = both(ctx, 1e-8, 2000)
    assert re[0] == api.SF_OK and rg == re and torch.equal(Ug, Ue)
    ctx.close()


def test_graph_solve_with_fp32_tiles_equals_ordinary_solve(gpu):
    # the FP32-tile sweep is another kernel form: replayed it must also match
    W, H, px, py, d = 72, 56, 3, 3, 8
    p = synth.make_pair("plain640", 3, W=W, H=H)
    ctx = api.sf_create(W, H, 1, px, py, d, factor_precision=api.SF_FP32)
    api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(synth.random_alpha(W, H, 3)[None]))
    api.sf_factor_subdomains(ctx)
    (Ue, re), (Ug, rg) = both(ctx, 1e-9, 500)
    assert re[0] == api.SF_OK and rg == re and torch.equal(Ug, Ue)
    ctx.close()


@pytest.mark.parametrize("W,H", [(160, 120), (640, 480)])
def test_solves_beside_a_busy_stream(gpu, W, H):
    # The sweeps are ordinary launches whose workgroups wait on each other
    # (their grid fits the co-resident capacity measured at creation); here
    # the kernels of another stream hold CUs while they start, so some
    # workgroups wait for others that are not yet resident (at 640x480 the
    # sweep takes every CU: 16 subdomains x 2 chains x 8 workgroups).  Every
    # wait is bounded; the solves (replayed and ordinary) must still end with
    # the iterate of the solve on an idle device.
    ctx, _ = context("plain640", 3, W, H, 4, 4, 8)
    Ue = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
    re = api.sf_schwarz_solve(ctx, Ue, 1e-9, 500)
    assert re[0] == api.SF_OK
    side = torch.cuda.Stream()
    a = torch.randn(2048, 2048, device="cuda")
    torch.cuda.synchronize()
    for solve in (api.sf_schwarz_solve_graph, api.sf_schwarz_solve):
        with torch.cuda.stream(side):
            for _ in range(100):
                a = torch.tanh(a @ a * 1e-3)
        U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
        r = solve(ctx, U, 1e-9, 500)
        torch.cuda.synchronize()
        assert r == re and torch.equal(U, Ue), solve.__name__
    assert torch.isfinite(a).all()
    ctx.close()


def test_contexts_solving_from_two_threads(gpu):
    # two 640x480 contexts on their own streams, solved (and one refactored
    # while the other solves) from two host threads at once (ctypes releases
    # the interpreter lock): every sweep launch takes the whole device, and
    # the per-device lock runs the calls one at a time, so both end with their
    # sequential results bit for bit
    import threading
    ctxs, refs = [], []
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for i, st in enumerate(streams):
        p = synth.make_pair("plain640", 40 + i, W=640, H=480)
        with torch.cuda.stream(st):
            ctx = api.sf_create(640, 480, 1, 4, 4, 8, stream=st)
            api.sf_assemble(ctx, dev(p.I0[None]), dev(p.I1[None]), dev(synth.random_alpha(640, 480, 40 + i)[None]))
            api.sf_factor_subdomains(ctx)
        ctxs.append(ctx)
    torch.cuda.synchronize()
    for ctx in ctxs:
        U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        refs.append((api.sf_schwarz_solve(ctx, U, 1e-9, 500), U))
    torch.cuda.synchronize()
    out = [None, None]

    def run(i, solve, U):
        out[i] = (solve(ctxs[i], U, 1e-9, 500), U)

    for solves in ((api.sf_schwarz_solve, api.sf_schwarz_solve),
                   (api.sf_schwarz_solve_graph, api.sf_schwarz_solve)):
        Us = [torch.zeros(ctx.field_shape(), dtype=torch.float64, device="cuda") for ctx in ctxs]
        torch.cuda.synchronize()
        out = [None, None]
        th = [threading.Thread(target=run, args=(i, solves[i], Us[i])) for i in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=120)
        torch.cuda.synchronize()
        for i in range(2):
            assert out[i] is not None, (i, solves[i].__name__)
            assert out[i][0] == refs[i][0] and torch.equal(out[i][1], refs[i][1]), (i, solves[i].__name__)
    # one context refactored while the other solves
    U1 = torch.zeros(ctxs[1].field_shape(), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    out = [None, None]
    ta = threading.Thread(target=lambda: out.__setitem__(0, api.sf_factor_subdomains(ctxs[0])))
    tb = threading.Thread(target=run, args=(1, api.sf_schwarz_solve, U1))
    ta.start()
    tb.start()
    ta.join(timeout=120)
    tb.join(timeout=120)
    torch.cuda.synchronize()
    assert out[1] is not None and out[1][0] == refs[1][0] and torch.equal(out[1][1], refs[1][1])
    U0 = torch.zeros(ctxs[0].field_shape(), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    assert api.sf_schwarz_solve(ctxs[0], U0, 1e-9, 500) == refs[0][0] and torch.equal(U0, refs[0][1])
    for ctx in ctxs:
        ctx.close()
