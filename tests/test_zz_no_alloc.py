"""gsf_cg_filter_noalloc, the CG filter (Algorithm 2) for callers that cannot
allocate device memory, against gsf_cg_filter on the same inputs: several
calls in a row on one device (each later one on a smaller problem than the
first, so that it runs over what the previous call left in the shared
static scratch), each bitwise equal to the workspace entry point's output
and info; and the size limit, refused on the host."""
import numpy as np
import pytest

from synth import piecewise_constant_1d, scene_2d

pytestmark = pytest.mark.gpu


def _dev(x, prec, gsf):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float32 if prec == gsf.F32 else torch.float64,
                        device="cuda")


# (shape, seed, precision, radius, steps, tol): the second call is smaller than
# the first; FP64 and a tolerance stop; a 1D signal on the one-workgroup path
CASES = [((300, 517), 1, 0, 5, 30, 0.0), ((67, 130), 2, 0, 5, 20, 0.0), ((90, 111), 3, 1, 3, 40, 1e-4),
         ((4000,), 4, 1, 4, 25, 0.0), ((20000,), 5, 0, 4, 15, 0.0)]


def test_noalloc_cg_equals_workspace_cg_in_a_row(gsf):
    for shape, seed, prec, r, k, tol in CASES:
        print(f"no-alloc CG {shape} prec={prec} r={r} k={k} tol={tol}", flush=True)
        x = piecewise_constant_1d(shape[0], 0.1, seed)[1] if len(shape) == 1 else scene_2d(*shape, 0.05, seed)[1]
        xd = _dev(x.ravel(), prec, gsf)
        op = gsf.Operator("bf", shape, xd, radius=r, sigma_d=2.0, sigma_r=0.1, prec=prec)
        ref, rinfo = op.cg_filter(xd, k, tol=tol)
        out, info = op.cg_filter_noalloc(xd, k, tol=tol)
        assert np.array_equal(out.cpu().numpy(), ref.cpu().numpy())
        assert (info.iters, info.status, info.res0, info.res) == (rinfo.iters, rinfo.status, rinfo.res0, rinfo.res)
        out2, _ = op.cg_filter_noalloc(xd, k, tol=tol, info=False)   # asynchronous form, same result
        assert np.array_equal(out2.cpu().numpy(), ref.cpu().numpy())


def test_noalloc_cg_refuses_problems_beyond_the_scratch(gsf):
    """Four FP32 vectors of 2100^2 points need 70.6 MB > 64 MiB: refused on
    the host with GSF_ESCRATCH, nothing enqueued, the output untouched."""
    import torch
    shape = (2100, 2100)
    g = torch.zeros(shape[0] * shape[1], dtype=torch.float32, device="cuda")
    op = gsf.Operator("bf", shape, g, radius=1, sigma_d=1.0, sigma_r=0.1, prec=gsf.F32)
    out = torch.full_like(g, 7.0)
    with pytest.raises(gsf.GsfError) as e:
        op.cg_filter_noalloc(g, 5, out=out)
    assert e.value.status == gsf.ESCRATCH
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
