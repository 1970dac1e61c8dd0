"""iht_gradient_noalloc (scratch in a fixed device array, no allocation) through the C ABI against
iht_gradient (scratch the genotype handle allocates): bitwise the same gradient, on two calls in a
row with the second on a smaller matrix (the array keeps the first call's larger contents), with
the device's free memory unchanged across the calls; sizes past the fixed scratch are rejected
before any device work."""
import ctypes
import gc

import numpy as np
import pytest

from paper_1608_01398_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1608_01398_amd import iht  # noqa: E402


def call_noalloc(g, s, r, out, precision):
    L = iht.load()
    return L.iht_gradient_noalloc(g._h, s._h, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(out.data_ptr()), precision,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("precision", [iht.FP64, iht.FP32])
def test_noalloc_gradient_equals_gradient_twice_shrinking(precision):
    # first a matrix whose pass splits its subjects (partial sums in the scratch), then a smaller one
    cases = [(3000, 140_000, 1200), (700, 9000, None)]
    mats = []
    for n, p, sub in cases:
        prob = synth.make_problem("c1", seed=5, n=n, p=p)
        g = iht.Geno(prob["bed"], n)
        s = iht.Stats(g, None if sub is None else synth.make_subset(n, sub, 4))
        r = torch.from_numpy(np.random.default_rng(n).standard_normal(n)).cuda()
        ref = iht.gradient(g, s, r, precision)
        out = torch.full((p,), float("nan"), dtype=torch.float64, device="cuda")
        mats.append((g, s, r, ref, out))
    torch.cuda.synchronize()
    assert call_noalloc(*mats[0][:3], mats[0][4], precision) == iht.OK  # scratch address looked up here
    torch.cuda.synchronize()
    gc.collect()  # handles left by earlier tests are finalised now, not inside a measured call
    for g, s, r, ref, out in mats:
        out.fill_(float("nan"))
        gc.disable()
        try:
            free0 = torch.cuda.mem_get_info()[0]
            rc = call_noalloc(g, s, r, out, precision)
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
        finally:
            gc.enable()
        assert rc == iht.OK, iht.load().iht_last_error()
        assert free1 == free0
        assert torch.equal(out, ref)


def test_noalloc_rejects_matrices_past_the_scratch():
    L = iht.load()
    cap = L.iht_gradient_noalloc_max_bytes()
    assert cap >= 262_144 * 8
    n = cap // 8 + 100_000  # the centred residual alone (8 bytes per subject) is larger than the scratch
    prob = synth.make_problem("c1", seed=1, n=n, p=8)
    g = iht.Geno(prob["bed"], n)
    s = iht.Stats(g)
    r = torch.zeros(n, dtype=torch.float64, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    assert call_noalloc(g, s, r, out, iht.FP64) == iht.EINVAL
    assert b"scratch" in L.iht_last_error()
    assert L.iht_gradient_noalloc(None, None, None, None, 0, None) == iht.EINVAL
