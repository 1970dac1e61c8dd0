"""Fits in a caller-supplied workspace (iht_opts.workspace, sized by iht_workspace_bytes): no device
allocation by the library, results bitwise equal to the fits whose state the genotype handle owns."""
import gc

import numpy as np
import pytest

from paper_1608_01398_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1608_01398_amd import iht  # noqa: E402


def dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def equal(x, y):
    """Bitwise-equal values, NaN (the unwritten tail of a loss trace) matching NaN."""
    return x.shape == y.shape and bool(((x == y) | (x.isnan() & y.isnan())).all())


def same(a, b):
    for key in ("support", "beta_S", "beta_cov", "loss_trace"):
        assert equal(a[key], b[key]), key
    assert np.array_equal(np.asarray(a["n_iter"]), np.asarray(b["n_iter"]))


@pytest.mark.parametrize("precision", [iht.FP64, iht.FP32, iht.MIXED_I8])
def test_fit_batch_in_workspace_allocates_nothing(precision):
    prob = synth.make_problem("c5", seed=6, n=1500, p=30_000)
    n, p = prob["n"], prob["p"]
    g = iht.Geno(prob["bed"], n)
    sub = synth.make_subset(n, 1100, 3)
    stats = [iht.Stats(g), iht.Stats(g, sub), iht.Stats(g)]
    Y = dev(np.stack([prob["y"], prob["y"], prob["y"][::-1].copy()]))
    Z = dev(prob["Z"], torch.float32)
    ks = [prob["k"], 7, 25]
    nc = Z.shape[0] + 1
    wsb = iht.workspace_bytes(n, p, max(ks), nc, precision, T=3)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    owned = iht.fit_batch(g, stats, Y, ks, Z=Z, precision=precision)
    warm = iht.fit_batch(g, stats, Y, ks, Z=Z, precision=precision, workspace=ws)  # code objects, pinned staging
    same(warm, owned)
    del warm  # its output blocks go back to torch's cache, where the next call's outputs find them
    torch.cuda.synchronize()
    ws.fill_(0xA5)  # whatever the workspace holds on entry does not matter
    # handles left by earlier tests are finalised now, not by a collection during the measured call
    gc.collect()
    gc.disable()
    try:
        free0 = torch.cuda.mem_get_info()[0]
        res = iht.fit_batch(g, stats, Y, ks, Z=Z, precision=precision, workspace=ws)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
    finally:
        gc.enable()
    assert free1 == free0, (free0, free1)
    same(res, owned)


def test_fit_in_workspace_equals_owned_and_rejects_small_or_misaligned():
    prob = synth.make_problem("c1", seed=3)
    n, p, k = prob["n"], prob["p"], prob["k"]
    g = iht.Geno(prob["bed"], n)
    s = iht.Stats(g)
    y = dev(prob["y"])
    wsb = iht.workspace_bytes(n, p, k, 1, iht.FP64)
    ws = torch.empty(wsb + 512, dtype=torch.uint8, device="cuda")
    a = iht.fit(g, s, y, k)
    b = iht.fit(g, s, y, k, workspace=ws[:wsb])
    for key in ("support", "beta_S", "beta_cov", "loss_trace"):
        assert equal(a[key], b[key]), key
    with pytest.raises(iht.IHTError, match="too small"):
        iht.fit(g, s, y, k, workspace=ws[:wsb - 256])
    with pytest.raises(iht.IHTError, match="aligned"):
        iht.fit(g, s, y, k, workspace=ws[8:wsb + 8])
    # a larger model size needs a larger workspace
    with pytest.raises(iht.IHTError, match="too small"):
        iht.fit(g, s, y, 4 * k, workspace=ws[:wsb])
