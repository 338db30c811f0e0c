"""Batching (many uneven items, one graph launch): every item equals the same
item filtered alone through the single-item calls (bitwise: the batch runs
the same kernels), over repeated graph replays with eager work between them,
and agrees with the FP64 oracle within the FP32 bound (1e-5 relative for
every output; LOBPCG items also by their Ritz values and drop counts)."""
import numpy as np
import pytest

import oracle
from synth import batch_items, item_signal

pytestmark = pytest.mark.gpu


def _items(gsf, count=14, seed=41):
    import torch
    recipe = batch_items(seed=seed, n_images=count - 4, n_signals=4, side_range=(24, 160),
                         len_range=(300, 5000))
    out = []
    for it in recipe:
        _, noisy = item_signal(it)
        g = torch.tensor(noisy.ravel(), dtype=torch.float32, device="cuda")
        out.append(dict(kind=it["kind"], shape=it["shape"], radius=it["radius"], sigma_d=it["sigma_d"],
                        sigma_r=it["sigma_r"], eps=it["eps"], guidance=g, x0=g.clone(), method=it["method"],
                        m=it["m"], kmax=12, tol=it["tol"] if it["method"] == "cg" else 0.0, noisy=noisy))
    out[0]["method"] = "power"
    out[1]["constraint"] = out[1]["method"] == "lobpcg"
    return out


def _solo(gsf, it):
    op = gsf.Operator(it["kind"], it["shape"], it["guidance"], it["radius"], it["sigma_d"], it["sigma_r"],
                      it["eps"], gsf.F32)
    if it["method"] == "power":
        return op.power_filter(it["x0"], it["kmax"]), None
    if it["method"] == "cg":
        return op.cg_filter(it["x0"], it["kmax"], tol=it["tol"])
    return op.lobpcg_filter(it["x0"], it["m"], it["kmax"], constraint=it.get("constraint", False))


def test_batch_items_equal_single_item_calls(gsf):
    import torch
    items = _items(gsf)
    batch = gsf.Batch(items, prec=gsf.F32, autotune=True)
    graphs = gsf.Batch(items, prec=gsf.F32, autotune=False, graphs=True)
    solo = [_solo(gsf, it)[0].cpu().numpy() for it in items]
    for rep in range(4):
        for it in items:
            it["out"].fill_(float("nan"))
        torch.cuda.synchronize()
        (batch if rep % 2 == 0 else graphs).run()
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        for k, it in enumerate(items):
            got = it["out"].cpu().numpy()
            assert np.array_equal(got, solo[k]), (rep, k, it["kind"], it["method"], it["shape"])
    info = batch.info()
    assert len(info) == len(items)


def test_batch_items_match_oracle(gsf):
    import torch
    items = _items(gsf, count=8, seed=43)
    batch = gsf.Batch(items, prec=gsf.F32, autotune=False)
    batch.run()
    torch.cuda.synchronize()
    info = batch.info()
    for k, it in enumerate(items):
        x = it["noisy"].astype(np.float32).astype(np.float64)
        ref = oracle.build_operator(it["kind"], x.reshape(it["shape"]), it["radius"], it["sigma_d"], it["sigma_r"],
                                    it["eps"])
        if it["method"] == "power":
            r = oracle.power_filter(ref, x.ravel(), it["kmax"])
            tol = 1e-5
        elif it["method"] == "cg":
            r, rinfo = oracle.cg_filter(ref, x.ravel(), it["kmax"], tol=it["tol"], data_prec="f32")
            assert info[k][0] == rinfo.iters
            tol = 1e-5
        else:
            r, th, _, rinfo = oracle.lobpcg_filter(ref, x.ravel(), it["m"], it["kmax"],
                                                   constraint=it.get("constraint", False), data_prec="f32")
            assert info[k][0] == rinfo.iters
            tol = 1e-5
        got = it["out"].cpu().numpy().astype(np.float64)
        err = np.linalg.norm(got - r) / np.linalg.norm(r)
        print(f"batch item {k} {it['kind']} {it['method']} {it['shape']}: rel err {err:.2e}")
        assert err <= tol, (k, err)
